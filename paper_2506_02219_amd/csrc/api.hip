// C ABI of libsbh (declared in include/sbh.h): argument checks, error
// reporting and ownership.  Every compute step is a kernel in build.hip,
// eval.hip, brute.hip or mlp.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

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

void free_impl(sbh::sbh_tree_impl* t, hipStream_t s)
{
    for (int i = 0; i < 3; ++i)
        if (t->slab[i]) sbh::dev_free(t->mem, t->slab[i], t->slab_bytes[i], s);
}

std::mutex g_alloc_mu;
sbh::Allocator g_alloc{nullptr, nullptr, nullptr};

// The static workspace of sbh_mlp_train_noalloc: the partial gradients of one batch (one row of
// 1616 floats per 64 rows) and the summed gradient (1616 floats).  Every GPU the library runs on
// holds its own copy until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: kernels get the per-device address that hipGetSymbolAddress returns.
constexpr size_t kScratchFloats = (size_t)(SBH_NOALLOC_MAX_BATCH_ROWS / 64 + 1) * 1616;
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up once per device (with that device current).
hipError_t scratch_ptr(float** out)
{
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
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
    if (o.rr_mode < 0 || o.rr_mode > 3) return fail(SBH_EINVAL, "rr_mode must be 0, 1, 2 or 3");
    if (o.proposal < 0 || o.proposal > 3) return fail(SBH_EINVAL, "proposal must be 0, 1, 2 or 3");
    if (o.proposal == 3 && o.group % 64 != 0)
        return fail(SBH_EINVAL, "the tile-shared score proposal needs group a multiple of 64");
    if (o.proposal == 1 && !o.mlp) return fail(SBH_EINVAL, "the learned proposal needs opts->mlp");
    if (o.subdomains < 0 || o.subdomains > 1) return fail(SBH_EINVAL, "subdomains must be 0 or 1");
    if (o.subdomains == 1 && (o.group % 64 != 0 || o.proposal != 0))
        return fail(SBH_EINVAL, "Barnes-Hut-cut subdomains need group a multiple of 64 and the uniform proposal");
    if (o.rr_mode == 3 && (o.group % 64 != 0 || o.proposal != 0 || o.subdomains != 0))
        return fail(SBH_EINVAL, "the voted roulette needs group a multiple of 64, the uniform proposal and subdomains 0");
    return SBH_OK;
}

}  // namespace

namespace sbh {

Allocator allocator_current()
{
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

hipError_t dev_alloc(const Allocator& a, void** p, size_t bytes, hipStream_t s)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (!a.alloc) return hipMallocAsync(p, bytes, s);
    *p = a.alloc(bytes, s, a.ctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_free(const Allocator& a, void* p, size_t bytes, hipStream_t s)
{
    if (!p) return;
    if (bytes == 0) bytes = 256;
    if (!a.alloc) (void)hipFreeAsync(p, s);
    else a.free(p, bytes, s, a.ctx);
}

}  // namespace sbh

extern "C" {

sbh_status sbh_set_allocator(sbh_alloc_fn alloc, sbh_free_fn free, void* ctx)
{
    if ((alloc == nullptr) != (free == nullptr))
        return fail(SBH_EINVAL, "sbh_set_allocator: give both functions or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = sbh::Allocator{alloc, free, alloc ? ctx : nullptr};
    return SBH_OK;
}

void sbh_build_opts_default(sbh_build_opts* o)
{
    if (!o) return;
    o->branching = 2;
    o->leaf_size = 8;
    o->max_level = 0;
    o->compress = 0;
    o->quadrupole = 0;
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
    o->subdomains = 0;
    o->compressed = 0;
    o->lod = 0;
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
    if (o.branching != 2 && o.branching != 4 && o.branching != 8)
        return fail(SBH_EINVAL, "sbh_build: branching must be 2, 4 or 8");
    if (o.leaf_size < 1 || o.leaf_size > 64) return fail(SBH_EINVAL, "sbh_build: leaf_size must be in [1, 64]");
    if (o.compress != 0 && o.compress != 1) return fail(SBH_EINVAL, "sbh_build: compress must be 0 or 1");
    if (o.compress && o.branching != 2)
        return fail(SBH_EUNSUPPORTED, "sbh_build: compressed aggregates need branching 2");
    if (o.quadrupole != 0 && o.quadrupole != 1) return fail(SBH_EINVAL, "sbh_build: quadrupole must be 0 or 1");
    const int bits = o.branching == 2 ? 3 : o.branching == 4 ? 6 : 9;
    const int lmax = 60 / bits;
    if (o.max_level < 0 || o.max_level > lmax) return fail(SBH_EINVAL, "sbh_build: max_level must be in [0, %d]", lmax);
    if (o.max_level == 0) o.max_level = lmax;

    sbh_tree* t = new (std::nothrow) sbh_tree();
    if (!t) return fail(SBH_ENOMEM, "sbh_build: host allocation failed");
    std::memset(&t->impl, 0, sizeof(t->impl));
    (void)hipGetDevice(&t->impl.device);
    t->impl.mem = sbh::allocator_current();
    std::string msg;
    const sbh_status st =
        sbh::build_tree_impl(sources, weights, normals, n, o.branching, o.leaf_size, o.max_level, o.compress,
                             o.quadrupole, stream, &t->impl, &msg);
    if (st != SBH_OK) {
        (void)hipStreamSynchronize(stream);
        free_impl(&t->impl, stream);
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
    const bool learned = samples > 0 && (o.proposal == 1 || o.proposal == 2);
    if (samples > 0 && o.proposal != 0 && t->d != 2)
        return fail(SBH_EUNSUPPORTED, "sbh_eval: proposals 1, 2 and 3 need branching 2");
    // branching 8 (512 children per node): the estimator's coherent walk only
    if (t->d == 8 && samples == 0)
        return fail(SBH_EUNSUPPORTED, "sbh_eval: Barnes-Hut needs branching 2 or 4");
    if (t->d == 8 && o.group % 64 != 0)
        return fail(SBH_EUNSUPPORTED, "sbh_eval: branching 8 needs group a multiple of 64");
    e.tile_score = (samples > 0 && o.proposal == 3) ? 1 : 0;
    e.cut = (samples > 0 && o.subdomains == 1) ? 1 : 0;
    if (e.cut && !(beta > 0.0f && std::isfinite(beta)))
        return fail(SBH_EINVAL, "sbh_eval: Barnes-Hut-cut subdomains need a finite beta > 0");
    if (e.cut && t->d == 8) return fail(SBH_EUNSUPPORTED, "sbh_eval: Barnes-Hut-cut subdomains need branching 2 or 4");
    if (o.compressed != 0 && o.compressed != 1) return fail(SBH_EINVAL, "sbh_eval: compressed must be 0 or 1");
    e.compressed = (samples > 0 && o.compressed == 1) ? 1 : 0;
    if (e.compressed) {
        if (!t->bq) return fail(SBH_ESTATE, "sbh_eval: compressed needs a tree built with compress = 1");
        if (o.proposal != 0 || o.subdomains != 0)
            return fail(SBH_EUNSUPPORTED, "sbh_eval: compressed needs the uniform proposal and subdomains 0");
        if (o.group % 64 != 0 && 8 * (int64_t)samples > 256)
            return fail(SBH_EUNSUPPORTED, "sbh_eval: compressed with group not a multiple of 64 needs samples <= 32");
        if (kernel != SBH_POTENTIAL && kernel != SBH_SMOOTHDIST)
            return fail(SBH_EUNSUPPORTED, "sbh_eval: compressed needs the potential or smooth-distance kernel");
    }
    if (o.lod < 0 || o.lod > 2) return fail(SBH_EINVAL, "sbh_eval: lod must be 0, 1 or 2");
    e.lod = o.lod == 2 ? 2 : 1;
    if (e.lod == 2) {
        if (!t->bquad) return fail(SBH_ESTATE, "sbh_eval: lod 2 needs a tree built with quadrupole = 1");
        if (samples == 0 || kernel != SBH_POTENTIAL || t->d != 2 || o.group % 64 != 0 || o.proposal != 0 ||
            o.subdomains != 0 || o.compressed != 0)
            return fail(SBH_EUNSUPPORTED,
                        "sbh_eval: lod 2 needs the estimator, the potential, branching 2, group a multiple of 64, "
                        "the uniform proposal, subdomains 0 and compressed 0");
    }
    const bool root_leaf = !(t->n_points > t->leaf_size && t->max_level > 0);
    hipError_t err;
    if (samples == 0) err = sbh::launch_bh_eval(t, queries, nq, e, out, stream);
    else if (learned && !root_leaf)
        err = sbh::launch_sbh_learned(t, queries, nq, e, o.proposal == 1 ? o.mlp : nullptr, out, stream);
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
                           uint32_t* perm, uint64_t* codes, float* spread2)
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
        {perm, t.perm, np * 4},         {codes, t.codes, np * 8},        {spread2, t.nspr, nn * 4},
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

sbh_status sbh_tree_export_compressed(const sbh_tree* tree, uint32_t* codes)
{
    if (!tree || !codes) return fail(SBH_EINVAL, "sbh_tree_export_compressed: NULL argument");
    const sbh::sbh_tree_impl& t = tree->impl;
    if (!t.bq) return fail(SBH_ESTATE, "sbh_tree_export_compressed: the tree was built without compress");
    const size_t bytes = (size_t)(t.n_blocks > 0 ? t.n_blocks : 1) * t.d3 * sizeof(uint2);
    const hipError_t e = hipMemcpy(codes, t.bq, bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "sbh_tree_export_compressed: copy");
    return SBH_OK;
}

sbh_status sbh_tree_export_quadrupole(const sbh_tree* tree, float* quad)
{
    if (!tree || !quad) return fail(SBH_EINVAL, "sbh_tree_export_quadrupole: NULL argument");
    const sbh::sbh_tree_impl& t = tree->impl;
    if (!t.bquad) return fail(SBH_ESTATE, "sbh_tree_export_quadrupole: the tree was built without quadrupole");
    const size_t bytes = (size_t)(t.n_blocks > 0 ? t.n_blocks : 1) * t.d3 * 2 * sizeof(float4);
    const hipError_t e = hipMemcpy(quad, t.bquad, bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "sbh_tree_export_quadrupole: copy");
    return SBH_OK;
}

sbh_status sbh_free(sbh_tree* tree)
{
    if (!tree) return SBH_OK;
    (void)hipDeviceSynchronize();
    free_impl(&tree->impl, 0);
    delete tree;
    return SBH_OK;
}

sbh_status sbh_free_async(sbh_tree* tree, hipStream_t stream)
{
    if (!tree) return SBH_OK;
    free_impl(&tree->impl, stream);
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
    const sbh::Allocator mem = sbh::allocator_current();
    const size_t wbytes = sbh::mlp_partial_floats(n) * sizeof(float);
    hipError_t e = sbh::dev_alloc(mem, (void**)&partial, wbytes, stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_loss_grad: workspace");
    e = sbh::launch_mlp_grad(params, features, targets, counts, n, 0, n, partial, grad, stream);
    sbh::dev_free(mem, partial, wbytes, stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_loss_grad: kernel launch");
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
    const sbh::Allocator mem = sbh::allocator_current();
    const size_t wbytes = (pf + 1616) * sizeof(float);
    hipError_t e = sbh::dev_alloc(mem, (void**)&work, wbytes, stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_train: workspace");
    float* grad = work + pf;
    for (int32_t s = 0; s < steps && e == hipSuccess; ++s) {
        const int64_t row_begin = ((int64_t)(step0 + s) * b) % n;
        const int64_t rows = (n - row_begin) < b ? (n - row_begin) : b;
        e = sbh::launch_mlp_grad(params, features, targets, counts, n, row_begin, rows, work, grad, stream);
        if (e == hipSuccess)
            e = sbh::launch_mlp_adam(params, adam_state, grad, lr, step0 + s, losses ? losses + s : nullptr, stream);
    }
    sbh::dev_free(mem, work, wbytes, stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_train: kernel launch");
    return SBH_OK;
}

sbh_status sbh_mlp_train_noalloc(float* params, float* adam_state, const float* features, const float* targets,
                                 const float* counts, int64_t n, int32_t steps, int32_t batch_rows, float lr,
                                 int32_t step0, hipStream_t stream, float* losses)
{
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(SBH_EINVAL, "sbh_mlp_train_noalloc: n must be in [1, 2^31)");
    if (!params || !adam_state || !features || !targets || !counts)
        return fail(SBH_EINVAL, "sbh_mlp_train_noalloc: NULL argument");
    if (steps < 0 || step0 < 0) return fail(SBH_EINVAL, "sbh_mlp_train_noalloc: steps and step0 must be >= 0");
    if (batch_rows < 1 || batch_rows > SBH_NOALLOC_MAX_BATCH_ROWS)
        return fail(SBH_EINVAL, "sbh_mlp_train_noalloc: batch_rows must be in [1, %d] (the static workspace)",
                    SBH_NOALLOC_MAX_BATCH_ROWS);
    if (!(lr > 0.0f) || !std::isfinite(lr))
        return fail(SBH_EINVAL, "sbh_mlp_train_noalloc: lr must be finite and > 0");
    if (steps == 0) return SBH_OK;
    float* work = nullptr;
    const hipError_t e0 = scratch_ptr(&work);
    if (e0 != hipSuccess) return hip_fail(e0, "sbh_mlp_train_noalloc: address of the static workspace");
    const int64_t b = batch_rows < n ? batch_rows : n;
    float* grad = work + sbh::mlp_partial_floats(b);
    hipError_t e = hipSuccess;
    for (int32_t s = 0; s < steps && e == hipSuccess; ++s) {
        const int64_t row_begin = ((int64_t)(step0 + s) * b) % n;
        const int64_t rows = (n - row_begin) < b ? (n - row_begin) : b;
        e = sbh::launch_mlp_grad(params, features, targets, counts, n, row_begin, rows, work, grad, stream);
        if (e == hipSuccess)
            e = sbh::launch_mlp_adam(params, adam_state, grad, lr, step0 + s, losses ? losses + s : nullptr, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "sbh_mlp_train_noalloc: kernel launch");
    return SBH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched evaluation
// ---------------------------------------------------------------------------
struct sbh_batch {
    int device = 0;
    sbh::Allocator mem{};                 // the allocator of the plan's tables
    int samples = 1;
    sbh_eval_opts opts{};
    std::vector<sbh::BatchItem> clouds;   // as given
    std::vector<double> cost;             // work estimate per cloud
    // groups g = 3 (d == 4) + kernel for the walk, 6 + kernel for root leaves: one launch each
    sbh::BatchItem* d_items[sbh::kBatchLaunchGroups] = {};   // the group's clouds, in launch order
    int2* d_wg[sbh::kBatchLaunchGroups] = {};                 // workgroup table: (cloud in d_items, first tile)
    int64_t tiles[sbh::kBatchLaunchGroups] = {};              // 64-query tiles of the group (table capacity)
    int n_wg[sbh::kBatchLaunchGroups] = {};
    sbh::BatchState* d_state = nullptr;   // [kBatchGroups]
    sbh_batch_config cfg{};
    size_t lds_bytes = 0;                 // per workgroup, for the occupancy cap
    size_t lds_static = 0;                // the batch kernels' own LDS per workgroup
    int lds_per_cu = 0, lds_per_wg_max = 0;
    hipStream_t cap = nullptr;
    // the groups' launches run on side streams forked from the launch stream and joined
    // back, so that in the captured graph they are parallel branches after the begin node
    // and one group's last workgroups overlap the next group's first
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSide] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t begin_node = nullptr;
};

namespace {

// (the caller has waited for the device)
void batch_release(sbh_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int i = 0; i < sbh_batch::kSide; ++i) {
        if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (int g = 0; g < sbh::kBatchLaunchGroups; ++g) {
        sbh::dev_free(b->mem, b->d_items[g], b->clouds.size() * sizeof(sbh::BatchItem), 0);
        sbh::dev_free(b->mem, b->d_wg[g], (size_t)b->tiles[g] * sizeof(int2), 0);
    }
    sbh::dev_free(b->mem, b->d_state, sbh::kBatchGroups * sizeof(sbh::BatchState), 0);
}

// Device descriptors and workgroup tables for a configuration: clouds split by
// branching factor and kernel, ordered as the configuration asks; each
// workgroup takes tile_waves consecutive tiles of one cloud (kWaveParts
// wavefronts each).  The occupancy cap reserves LDS so that at most
// 4 waves_per_simd / (tile_waves kWaveParts) workgroups fit on a compute unit
// (4 SIMDs); 8 waves per SIMD is the hardware's own limit.
// the launch group of a cloud: the walk by (branching factor, kernel), or the exact sum of a root leaf
int batch_group(const sbh::BatchItem& it)
{
    return it.root_leaf ? sbh::kBatchGroups + it.kernel : (it.d == 4 ? 3 : 0) + it.kernel;
}

hipError_t batch_upload(sbh_batch* b, const sbh_batch_config& c)
{
    std::vector<int> order(b->clouds.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    if (c.heavy_first)
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->cost[x] > b->cost[y]; });
    b->lds_bytes = 0;
    if (c.waves_per_simd < 8) {
        // a workgroup's LDS (its own arrays plus the reservation) is the unit's share
        // for per_cu workgroups, so that one more does not fit
        const int per_cu = std::max(1, 4 * c.waves_per_simd / (c.tile_waves * sbh::kWaveParts));
        const size_t total = std::min((size_t)(b->lds_per_cu / per_cu), (size_t)b->lds_per_wg_max) & ~(size_t)511;
        b->lds_bytes = total > b->lds_static ? total - b->lds_static : 0;
    }
    for (int g = 0; g < sbh::kBatchLaunchGroups; ++g) {
        std::vector<sbh::BatchItem> v;
        std::vector<int2> wg;
        for (int idx : order) {
            const sbh::BatchItem& it = b->clouds[idx];
            if (batch_group(it) != g) continue;
            const int64_t tiles = (it.nq + 63) / 64;
            for (int64_t t = 0; t < tiles; t += c.tile_waves) wg.push_back(make_int2((int)v.size(), (int)t));
            v.push_back(it);
        }
        b->n_wg[g] = (int)wg.size();
        if (!v.empty()) {
            hipError_t e = hipMemcpy(b->d_items[g], v.data(), v.size() * sizeof(sbh::BatchItem), hipMemcpyHostToDevice);
            if (e == hipSuccess && !wg.empty())
                e = hipMemcpy(b->d_wg[g], wg.data(), wg.size() * sizeof(int2), hipMemcpyHostToDevice);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// the launch state, then every group's launch on the side streams (group i of those with
// work on side stream i mod kSide), which s waits for
hipError_t batch_enqueue(sbh_batch* b, uint64_t seed, uint32_t batch, hipStream_t s)
{
    hipError_t e = sbh::launch_batch_begin(b->d_state, seed, batch, s);
    if (e == hipSuccess) e = hipEventRecord(b->fork, s);
    int used = 0;
    for (int g = 0; g < sbh::kBatchLaunchGroups && e == hipSuccess; ++g) {
        if (b->n_wg[g] == 0) continue;
        hipStream_t sg = b->side[used % sbh_batch::kSide];
        if (used < sbh_batch::kSide) e = hipStreamWaitEvent(sg, b->fork, 0);
        ++used;
        if (e != hipSuccess) break;
        if (g < sbh::kBatchGroups)
            e = sbh::launch_sbh_batch(g < 3 ? 2 : 4, g % 3, b->d_items[g], b->d_wg[g], b->n_wg[g], b->cfg.tile_waves,
                                      b->lds_bytes, b->d_state + g, b->samples, b->opts.group, b->opts.rr_mode,
                                      b->opts.eps, b->opts.alpha, sg);
        else
            e = sbh::launch_leaf_batch(g - sbh::kBatchGroups, b->d_items[g], b->d_wg[g], b->n_wg[g], b->cfg.tile_waves,
                                       b->opts.eps, b->opts.alpha, sg);
    }
    for (int i = 0; i < std::min(used, sbh_batch::kSide) && e == hipSuccess; ++i) {
        e = hipEventRecord(b->join[i], b->side[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[i], 0);
    }
    return e;
}

}  // namespace

extern "C" {

sbh_status sbh_batch_create(const sbh_batch_item* items, int32_t count, int32_t samples, const sbh_eval_opts* opts,
                            const sbh_batch_config* config, hipStream_t stream, sbh_batch** out)
{
    if (!items || !out) return fail(SBH_EINVAL, "sbh_batch_create: NULL argument");
    if (count < 1 || count > (1 << 20)) return fail(SBH_EINVAL, "sbh_batch_create: count must be in [1, 2^20]");
    if (samples < 1) return fail(SBH_EINVAL, "sbh_batch_create: samples must be >= 1");
    sbh_eval_opts o;
    sbh_eval_opts_default(&o);
    o.group = 64;
    if (opts) o = *opts;
    if (check_eval_opts(o) != SBH_OK) return SBH_EINVAL;
    if (o.subdomains != 0) return fail(SBH_EUNSUPPORTED, "sbh_batch_create: batches take the root's children as subdomains");
    if (o.compressed != 0 || o.lod == 2)
        return fail(SBH_EUNSUPPORTED, "sbh_batch_create: batches walk the float32 point-mass aggregates");
    if (o.group % 64 != 0) return fail(SBH_EINVAL, "sbh_batch_create: group must be a multiple of 64");
    if (o.proposal != 0) return fail(SBH_EUNSUPPORTED, "sbh_batch_create: only the uniform proposal is batched");
    if (o.paths) return fail(SBH_EINVAL, "sbh_batch_create: path records are not available in a batch");
    if (config) {
        if (config->tile_waves < 1 || config->tile_waves > sbh::kBatchMaxTileWaves)
            return fail(SBH_EINVAL, "sbh_batch_create: tile_waves must be 1 or 2");
        if (config->waves_per_simd < 1 || config->waves_per_simd > 8)
            return fail(SBH_EINVAL, "sbh_batch_create: waves_per_simd must be in [1, 8]");
        if (config->heavy_first != 0 && config->heavy_first != 1)
            return fail(SBH_EINVAL, "sbh_batch_create: heavy_first must be 0 or 1");
    }
    int64_t tiles_total = 0;
    for (int32_t i = 0; i < count; ++i) {
        const sbh_batch_item& it = items[i];
        if (!it.tree) return fail(SBH_EINVAL, "sbh_batch_create: item %d has no tree", i);
        if (it.nq < 0 || it.nq >= ((int64_t)1 << 31)) return fail(SBH_EINVAL, "sbh_batch_create: item %d: bad nq", i);
        if (it.nq > 0 && (!it.queries || !it.out))
            return fail(SBH_EINVAL, "sbh_batch_create: item %d: queries and out must not be NULL", i);
        if (check_kernel(it.kernel) != SBH_OK) return SBH_EINVAL;
        if (it.kernel == SBH_WINDING && !it.tree->impl.has_normals)
            return fail(SBH_EINVAL, "sbh_batch_create: item %d: the winding kernel needs normals", i);
        tiles_total += (it.nq + 63) / 64;
    }
    if (tiles_total >= ((int64_t)1 << 31)) return fail(SBH_EINVAL, "sbh_batch_create: too many queries");
    sbh_batch* b = new (std::nothrow) sbh_batch();
    if (!b) return fail(SBH_ENOMEM, "sbh_batch_create: host allocation");
    b->samples = samples;
    b->opts = o;
    b->mem = sbh::allocator_current();
    (void)hipGetDevice(&b->device);
    for (int32_t i = 0; i < count; ++i) {
        const sbh::sbh_tree_impl* t = &items[i].tree->impl;
        sbh::BatchItem it{};
        it.tv = sbh::make_view(t);
        it.queries = items[i].queries;
        it.out = items[i].out;
        it.nq = items[i].nq;
        it.kernel = items[i].kernel;
        it.d = t->d;
        it.root_leaf = it.tv.root_internal ? 0 : 1;
        b->clouds.push_back(it);
        b->cost.push_back((double)it.nq * (double)(t->depth + 1) * (it.kernel == SBH_WINDING ? 1.5 : 1.0) * samples);
        b->tiles[batch_group(it)] += (it.nq + 63) / 64;
    }
    hipError_t e = hipDeviceGetAttribute(&b->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                         b->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&b->lds_per_wg_max, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device);
    if (e == hipSuccess) e = sbh::batch_static_lds(&b->lds_static);
    for (int g = 0; g < sbh::kBatchLaunchGroups && e == hipSuccess; ++g) {
        e = sbh::dev_alloc(b->mem, (void**)&b->d_items[g], (size_t)count * sizeof(sbh::BatchItem), stream);
        if (e == hipSuccess && b->tiles[g] > 0)
            e = sbh::dev_alloc(b->mem, (void**)&b->d_wg[g], (size_t)b->tiles[g] * sizeof(int2), stream);
    }
    if (e == hipSuccess)
        e = sbh::dev_alloc(b->mem, (void**)&b->d_state, sbh::kBatchGroups * sizeof(sbh::BatchState), stream);
    // the tables are written by synchronous copies and read on other streams (graph replays)
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    for (int i = 0; i < sbh_batch::kSide && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipDeviceSynchronize();
        batch_release(b);
        delete b;
        return hip_fail(e, "sbh_batch_create: allocation");
    }
    if (config) {
        b->cfg = *config;
        b->cfg.ms = 0.0f;
    } else {
        // autotune: time every candidate on the batch itself (outputs are written)
        hipEvent_t e0 = nullptr, e1 = nullptr;
        e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        float best = INFINITY;
        sbh_batch_config best_cfg{1, 8, 1, 0.0f};
        const int tws[] = {1, 2};
        const int wpss[] = {4, 8};
        for (int heavy = 0; heavy < 2 && e == hipSuccess; ++heavy)
            for (int tw : tws)
                for (int wps : wpss) {
                    if (e != hipSuccess) break;
                    sbh_batch_config c{tw, wps, heavy, 0.0f};
                    b->cfg = c;
                    e = batch_upload(b, c);
                    if (e == hipSuccess) e = batch_enqueue(b, 0, 0, stream);   // warm-up
                    if (e == hipSuccess) e = hipEventRecord(e0, stream);
                    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = batch_enqueue(b, 0, 0, stream);
                    if (e == hipSuccess) e = hipEventRecord(e1, stream);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.0f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e == hipSuccess && ms / 3.0f < best) {
                        best = ms / 3.0f;
                        best_cfg = c;
                        best_cfg.ms = best;
                    }
                }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        b->cfg = best_cfg;
    }
    if (e == hipSuccess) e = batch_upload(b, b->cfg);
    // capture the launch sequence once; sbh_batch_launch replays it
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t le = batch_enqueue(b, 0, 0, b->cap);
        e = hipStreamEndCapture(b->cap, &b->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e == hipSuccess) {
        size_t n = 0;
        e = hipGraphGetNodes(b->graph, nullptr, &n);
        std::vector<hipGraphNode_t> nodes(n);
        if (e == hipSuccess && n > 0) e = hipGraphGetNodes(b->graph, nodes.data(), &n);
        for (size_t i = 0; i < n && e == hipSuccess; ++i) {
            hipGraphNodeType ty;
            if (hipGraphNodeGetType(nodes[i], &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
            hipKernelNodeParams kp{};
            if (hipGraphKernelNodeGetParams(nodes[i], &kp) == hipSuccess && kp.func == sbh::batch_begin_kernel())
                b->begin_node = nodes[i];
        }
        if (e == hipSuccess && !b->begin_node) e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) {
        (void)hipDeviceSynchronize();
        batch_release(b);
        delete b;
        return hip_fail(e, "sbh_batch_create: tuning or graph capture");
    }
    *out = b;
    return SBH_OK;
}

sbh_status sbh_batch_launch(sbh_batch* b, uint64_t seed, uint32_t batch, hipStream_t stream)
{
    if (!b) return fail(SBH_EINVAL, "sbh_batch_launch: NULL plan");
    sbh::BatchState* st = b->d_state;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32), bw = batch;
    void* args[] = {&st, &k0, &k1, &bw};
    hipKernelNodeParams kp{};
    kp.func = sbh::batch_begin_kernel();
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipError_t e = hipGraphExecKernelNodeSetParams(b->exec, b->begin_node, &kp);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, stream);
    if (e != hipSuccess) return hip_fail(e, "sbh_batch_launch");
    return SBH_OK;
}

sbh_status sbh_batch_get_config(const sbh_batch* b, sbh_batch_config* cfg)
{
    if (!b || !cfg) return fail(SBH_EINVAL, "sbh_batch_get_config: NULL argument");
    *cfg = b->cfg;
    return SBH_OK;
}

sbh_status sbh_batch_free(sbh_batch* b)
{
    if (!b) return SBH_OK;
    (void)hipDeviceSynchronize();
    batch_release(b);
    delete b;
    return SBH_OK;
}

}  // extern "C"
