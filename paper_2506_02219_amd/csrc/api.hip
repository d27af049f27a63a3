// C ABI of libsbh (declared in include/sbh.h): argument checks, error
// reporting and ownership.  Every compute step is a kernel in build.hip,
// eval.hip, brute.hip or mlp.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "sbh_internal.hpp"

struct sbh_tree {
    sbh::sbh_tree_impl impl;
};

namespace {

thread_local std::string g_last_error;

sbh_status fail(sbh_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

sbh_status hip_fail(hipError_t e, const char* where)
{
    const sbh_status s = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? SBH_ENOMEM : SBH_EHIP;
    return fail(s, "%s: %s", where, hipGetErrorString(e));
}

void free_impl(sbh::sbh_tree_impl* t)
{
    void* bufs[] = {t->pts, t->pdip, t->perm, t->codes, t->nbegin, t->ncount, t->nlevel, t->ndigit, t->nparent,
                    t->nfirst, t->nnchild, t->nagg, t->ndip, t->bagg, t->bdip, t->btopo};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
}

sbh_status check_kernel(int kernel)
{
    if (kernel != SBH_POTENTIAL && kernel != SBH_WINDING && kernel != SBH_SMOOTHDIST)
        return fail(SBH_EINVAL, "unknown kernel %d", kernel);
    return SBH_OK;
}

sbh_status check_eval_opts(const sbh_eval_opts& o)
{
    if (!(o.eps >= 0.0f) || !std::isfinite(o.eps)) return fail(SBH_EINVAL, "eps must be finite and >= 0");
    if (!(o.alpha > 0.0f) || !std::isfinite(o.alpha)) return fail(SBH_EINVAL, "alpha must be finite and > 0");
    if (o.group < 1) return fail(SBH_EINVAL, "group must be >= 1");
    if (o.rr_mode < 0 || o.rr_mode > 2) return fail(SBH_EINVAL, "rr_mode must be 0, 1 or 2");
    if (o.proposal != 0 && o.proposal != 1) return fail(SBH_EINVAL, "proposal must be 0 or 1");
    if (o.proposal == 1 && !o.mlp) return fail(SBH_EINVAL, "the learned proposal needs opts->mlp");
    return SBH_OK;
}

}  // namespace

extern "C" {

void sbh_build_opts_default(sbh_build_opts* o)
{
    if (!o) return;
    o->branching = 2;
    o->leaf_size = 8;
    o->max_level = 0;
}

void sbh_eval_opts_default(sbh_eval_opts* o)
{
    if (!o) return;
    o->eps = 1e-3f;
    o->alpha = 100.0f;
    o->group = 1;
    o->rr_mode = 0;
    o->proposal = 0;
    o->batch = 0;
    o->paths = nullptr;
    o->mlp = nullptr;
}

const char* sbh_status_string(sbh_status s)
{
    switch (s) {
    case SBH_OK: return "SBH_OK";
    case SBH_EINVAL: return "SBH_EINVAL: invalid argument";
    case SBH_ENOMEM: return "SBH_ENOMEM: device allocation failed";
    case SBH_EHIP: return "SBH_EHIP: HIP runtime error";
    case SBH_EUNSUPPORTED: return "SBH_EUNSUPPORTED: not supported";
    case SBH_ESTATE: return "SBH_ESTATE: unusable state";
    }
    return "unknown sbh_status";
}

const char* sbh_last_error(void) { return g_last_error.c_str(); }

sbh_status sbh_build(const float* sources, const float* weights, const float* normals, int64_t n,
                     const sbh_build_opts* opts, hipStream_t stream, sbh_tree** out_tree)
{
    if (!out_tree) return fail(SBH_EINVAL, "sbh_build: out_tree is NULL");
    *out_tree = nullptr;
    if (!sources || !weights) return fail(SBH_EINVAL, "sbh_build: sources and weights must not be NULL");
    if (n < 1 || n > ((int64_t)1 << 30)) return fail(SBH_EINVAL, "sbh_build: n = %lld out of range [1, 2^30]", (long long)n);
    sbh_build_opts o;
    sbh_build_opts_default(&o);
    if (opts) o = *opts;
    if (o.branching != 2 && o.branching != 4) return fail(SBH_EINVAL, "sbh_build: branching must be 2 or 4");
    if (o.leaf_size < 1 || o.leaf_size > 64) return fail(SBH_EINVAL, "sbh_build: leaf_size must be in [1, 64]");
    const int bits = o.branching == 2 ? 3 : 6;
    const int lmax = 60 / bits;
    if (o.max_level < 0 || o.max_level > lmax) return fail(SBH_EINVAL, "sbh_build: max_level must be in [0, %d]", lmax);
    if (o.max_level == 0) o.max_level = lmax;

    sbh_tree* t = new (std::nothrow) sbh_tree();
    if (!t) return fail(SBH_ENOMEM, "sbh_build: host allocation failed");
    std::memset(&t->impl, 0, sizeof(t->impl));
    (void)hipGetDevice(&t->impl.device);
    std::string msg;
    const sbh_status st =
        sbh::build_tree_impl(sources, weights, normals, n, o.branching, o.leaf_size, o.max_level, stream, &t->impl, &msg);
    if (st != SBH_OK) {
        (void)hipStreamSynchronize(stream);
        free_impl(&t->impl);
        delete t;
        return fail(st, "sbh_build: %s", msg.c_str());
    }
    *out_tree = t;
    return SBH_OK;
}

sbh_status sbh_eval(const sbh_tree* tree, const float* queries, int64_t nq, sbh_kernel kernel, float beta,
                    int32_t samples, uint64_t seed, const sbh_eval_opts* opts, hipStream_t stream, float* out)
{
    if (!tree) return fail(SBH_EINVAL, "sbh_eval: tree is NULL");
    if (nq < 0) return fail(SBH_EINVAL, "sbh_eval: nq < 0");
    if (nq > 0 && (!queries || !out)) return fail(SBH_EINVAL, "sbh_eval: queries and out must not be NULL");
    if (nq >= ((int64_t)1 << 31)) return fail(SBH_EINVAL, "sbh_eval: nq must be < 2^31");
    if (check_kernel(kernel) != SBH_OK) return SBH_EINVAL;
    if (samples < 0) return fail(SBH_EINVAL, "sbh_eval: samples < 0");
    if (samples == 0 && !(beta > 0.0f)) return fail(SBH_EINVAL, "sbh_eval: Barnes-Hut needs beta > 0");
    sbh_eval_opts o;
    sbh_eval_opts_default(&o);
    if (opts) o = *opts;
    sbh_status cs = check_eval_opts(o);
    if (cs != SBH_OK) return cs;
    const sbh::sbh_tree_impl* t = &tree->impl;
    if (kernel == SBH_WINDING && !t->has_normals)
        return fail(SBH_EINVAL, "sbh_eval: the winding kernel needs a tree built with normals");
    if (nq == 0) return SBH_OK;
    sbh::EvalLaunch e{};
    e.kernel = kernel;
    e.samples = samples;
    e.seed = seed;
    e.group = o.group;
    e.rr_mode = o.rr_mode;
    e.batch = o.batch;
    e.beta = beta;
    e.eps = o.eps;
    e.alpha = o.alpha;
    e.paths = samples > 0 ? o.paths : nullptr;
    const bool learned = samples > 0 && o.proposal == 1;
    if (learned && t->d != 2) return fail(SBH_EUNSUPPORTED, "sbh_eval: the learned proposal needs branching 2");
    const bool root_leaf = !(t->n_points > t->leaf_size && t->max_level > 0);
    hipError_t err;
    if (samples == 0) err = sbh::launch_bh_eval(t, queries, nq, e, out, stream);
    else if (learned && !root_leaf) err = sbh::launch_sbh_learned(t, queries, nq, e, o.mlp, out, stream);
    else err = sbh::launch_sbh_eval(t, queries, nq, e, out, stream);
    if (err != hipSuccess) return hip_fail(err, "sbh_eval: kernel launch");
    return SBH_OK;
}

sbh_status sbh_brute(const float* sources, const float* weights, const float* normals, int64_t n,
                     const float* queries, int64_t nq, sbh_kernel kernel, const sbh_eval_opts* opts, int32_t fp64,
                     hipStream_t stream, void* out)
{
    if (n < 1) return fail(SBH_EINVAL, "sbh_brute: n < 1");
    if (!sources || !weights) return fail(SBH_EINVAL, "sbh_brute: sources and weights must not be NULL");
    if (nq < 0) return fail(SBH_EINVAL, "sbh_brute: nq < 0");
    if (nq > 0 && (!queries || !out)) return fail(SBH_EINVAL, "sbh_brute: queries and out must not be NULL");
    if (check_kernel(kernel) != SBH_OK) return SBH_EINVAL;
    if (kernel == SBH_WINDING && !normals) return fail(SBH_EINVAL, "sbh_brute: the winding kernel needs normals");
    if (fp64 != 0 && fp64 != 1) return fail(SBH_EINVAL, "sbh_brute: fp64 must be 0 or 1");
    sbh_eval_opts o;
    sbh_eval_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.eps >= 0.0f) || !(o.alpha > 0.0f)) return fail(SBH_EINVAL, "sbh_brute: bad eps or alpha");
    if (nq == 0) return SBH_OK;
    const hipError_t err = sbh::launch_brute(sources, weights, normals, n, queries, nq, kernel, o.eps, o.alpha, fp64,
                                             out, stream);
    if (err != hipSuccess) return hip_fail(err, "sbh_brute: kernel launch");
    return SBH_OK;
}

sbh_status sbh_tree_info(const sbh_tree* tree, sbh_tree_desc* info)
{
    if (!tree || !info) return fail(SBH_EINVAL, "sbh_tree_info: NULL argument");
    const sbh::sbh_tree_impl& t = tree->impl;
    info->n_points = t.n_points;
    info->n_nodes = t.n_nodes;
    info->n_blocks = t.n_blocks;
    info->depth = t.depth;
    info->branching = t.d;
    info->leaf_size = t.leaf_size;
    info->max_level = t.max_level;
    info->has_normals = t.has_normals;
    for (int a = 0; a < 3; ++a) info->lo[a] = t.lo[a];
    info->side = t.side;
    info->inv_side = t.inv_side;
    return SBH_OK;
}

sbh_status sbh_tree_export(const sbh_tree* tree, int32_t* begin, int32_t* count, int32_t* level, int32_t* digit,
                           int32_t* parent, int32_t* first_child, int32_t* nchild, float* agg, float* dip,
                           uint32_t* perm, uint64_t* codes)
{
    if (!tree) return fail(SBH_EINVAL, "sbh_tree_export: tree is NULL");
    const sbh::sbh_tree_impl& t = tree->impl;
    const size_t nn = (size_t)t.n_nodes, np = (size_t)t.n_points;
    struct Item {
        void* dst;
        const void* src;
        size_t bytes;
    } items[] = {
        {begin, t.nbegin, nn * 4},      {count, t.ncount, nn * 4},       {level, t.nlevel, nn * 4},
        {digit, t.ndigit, nn * 4},      {parent, t.nparent, nn * 4},     {first_child, t.nfirst, nn * 4},
        {nchild, t.nnchild, nn * 4},    {agg, t.nagg, nn * 16},          {dip, t.ndip, nn * 16},
        {perm, t.perm, np * 4},         {codes, t.codes, np * 8},
    };
    for (const Item& it : items) {
        if (!it.dst) continue;
        if (!it.src) {
            std::memset(it.dst, 0, it.bytes);
            continue;
        }
        const hipError_t e = hipMemcpy(it.dst, it.src, it.bytes, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "sbh_tree_export: copy");
    }
    return SBH_OK;
}

sbh_status sbh_free(sbh_tree* tree)
{
    if (!tree) return SBH_OK;
    (void)hipDeviceSynchronize();
    free_impl(&tree->impl);
    delete tree;
    return SBH_OK;
}

// ---------------------------------------------------------------------------
// Learned child proposal
// ---------------------------------------------------------------------------
sbh_status sbh_mlp_forward(const float* params, const float* features, int64_t n, hipStream_t stream, float* logits)
{
    if (n < 0) return fail(SBH_EINVAL, "sbh_mlp_forward: n < 0");
    if (!params || (n > 0 && (!features || !logits)))
        return fail(SBH_EINVAL, "sbh_mlp_forward: NULL argument");
    if (n >= ((int64_t)1 << 31)) return fail(SBH_EINVAL, "sbh_mlp_forward: n must be < 2^31");
    const hipError_t e = sbh::launch_mlp_forward(params, features, n, logits, stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_forward: kernel launch");
    return SBH_OK;
}

sbh_status sbh_mlp_pairs(const sbh_tree* tree, const float* queries, int64_t nq, sbh_kernel kernel, uint64_t seed,
                         int32_t max_depth, const sbh_eval_opts* opts, hipStream_t stream, float* features,
                         float* targets, float* counts, int32_t* where)
{
    if (!tree) return fail(SBH_EINVAL, "sbh_mlp_pairs: tree is NULL");
    if (nq < 0) return fail(SBH_EINVAL, "sbh_mlp_pairs: nq < 0");
    const sbh::sbh_tree_impl* t = &tree->impl;
    if (t->d != 2) return fail(SBH_EUNSUPPORTED, "sbh_mlp_pairs: the learned proposal needs branching 2");
    if (max_depth < 1 || max_depth > t->max_level)
        return fail(SBH_EINVAL, "sbh_mlp_pairs: max_depth must be in [1, %d]", t->max_level);
    if (nq > 0 && (!queries || !features || !targets || !counts || !where))
        return fail(SBH_EINVAL, "sbh_mlp_pairs: NULL argument");
    if (nq * 8 * (int64_t)max_depth >= ((int64_t)1 << 31))
        return fail(SBH_EINVAL, "sbh_mlp_pairs: nq * 8 * max_depth must be < 2^31");
    if (check_kernel(kernel) != SBH_OK) return SBH_EINVAL;
    if (kernel == SBH_WINDING && !t->has_normals)
        return fail(SBH_EINVAL, "sbh_mlp_pairs: the winding kernel needs a tree built with normals");
    sbh_eval_opts o;
    sbh_eval_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.eps >= 0.0f) || !(o.alpha > 0.0f) || !std::isfinite(o.eps) || !std::isfinite(o.alpha))
        return fail(SBH_EINVAL, "sbh_mlp_pairs: bad eps or alpha");
    if (nq == 0) return SBH_OK;
    const hipError_t e = sbh::launch_mlp_pairs(t, queries, nq, max_depth, seed, kernel, o.eps, o.alpha, features,
                                               targets, counts, reinterpret_cast<int4*>(where), stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_pairs: kernel launch");
    return SBH_OK;
}

sbh_status sbh_mlp_loss_grad(const float* params, const float* features, const float* targets, const float* counts,
                             int64_t n, hipStream_t stream, float* grad)
{
    if (n < 1) return fail(SBH_EINVAL, "sbh_mlp_loss_grad: n < 1");
    if (n >= ((int64_t)1 << 31)) return fail(SBH_EINVAL, "sbh_mlp_loss_grad: n must be < 2^31");
    if (!params || !features || !targets || !counts || !grad)
        return fail(SBH_EINVAL, "sbh_mlp_loss_grad: NULL argument");
    float* partial = nullptr;
    hipError_t e = hipMallocAsync((void**)&partial, sbh::mlp_partial_floats(n) * sizeof(float), stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_loss_grad: workspace");
    e = sbh::launch_mlp_grad(params, features, targets, counts, n, 0, n, partial, grad, stream);
    const hipError_t f = hipFreeAsync(partial, stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_loss_grad: kernel launch");
    if (f != hipSuccess) return hip_fail(f, "sbh_mlp_loss_grad: workspace release");
    return SBH_OK;
}

sbh_status sbh_mlp_train(float* params, float* adam_state, const float* features, const float* targets,
                         const float* counts, int64_t n, int32_t steps, int32_t batch_rows, float lr, int32_t step0,
                         hipStream_t stream, float* losses)
{
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(SBH_EINVAL, "sbh_mlp_train: n must be in [1, 2^31)");
    if (!params || !adam_state || !features || !targets || !counts)
        return fail(SBH_EINVAL, "sbh_mlp_train: NULL argument");
    if (steps < 0 || step0 < 0) return fail(SBH_EINVAL, "sbh_mlp_train: steps and step0 must be >= 0");
    if (batch_rows < 1 || batch_rows > (1 << 24)) return fail(SBH_EINVAL, "sbh_mlp_train: batch_rows must be in [1, 2^24]");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(SBH_EINVAL, "sbh_mlp_train: lr must be finite and > 0");
    if (steps == 0) return SBH_OK;
    const int64_t b = batch_rows < n ? batch_rows : n;
    float* work = nullptr;
    const size_t pf = sbh::mlp_partial_floats(b);
    hipError_t e = hipMallocAsync((void**)&work, (pf + 1616) * sizeof(float), stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_train: workspace");
    float* grad = work + pf;
    for (int32_t s = 0; s < steps && e == hipSuccess; ++s) {
        const int64_t row_begin = ((int64_t)(step0 + s) * b) % n;
        const int64_t rows = (n - row_begin) < b ? (n - row_begin) : b;
        e = sbh::launch_mlp_grad(params, features, targets, counts, n, row_begin, rows, work, grad, stream);
        if (e == hipSuccess)
            e = sbh::launch_mlp_adam(params, adam_state, grad, lr, step0 + s, losses ? losses + s : nullptr, stream);
    }
    const hipError_t f = hipFreeAsync(work, stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_train: kernel launch");
    if (f != hipSuccess) return hip_fail(f, "sbh_mlp_train: workspace release");
    return SBH_OK;
}

}  // extern "C"
