// Internal declarations shared by the HIP translation units of libsbh.
//
// Device data layout of a tree (all in HBM, built by build.hip):
//   pts    float4[M]         sorted points (x, y, z, w)
//   pdip   float4[M]         sorted w*n (winding only)
//   Nodes, breadth-first, Morton order within a level (for export/build):
//     nbegin/ncount/nlevel/ndigit/nparent/nfirst/nnchild int32[n_nodes]
//     nagg float4[n_nodes] (centre of mass, weight), ndip float4[n_nodes],
//     nspr float[n_nodes] (second moment sum w |p - com|^2 / weight)
//   Child blocks, one per internal node, in breadth-first order of the
//   internal nodes (the root's block is block 0):
//     bagg   float4[n_blocks][d^3]   aggregate of the child in digit slot s
//                                    (zero for an empty slot)
//     bdip   float4[n_blocks][d^3]   summed w*n per slot (winding only)
//     bspr   float[n_blocks][d^3]    second moment per slot (zero for an empty slot)
//     btopo  uint32[n_blocks][TS]    point count per slot, then at [d^3] the
//                                    block id of the first internal child;
//                                    the internal children of one node hold
//                                    consecutive block ids in slot order.
//   A node is internal iff count > leaf_size and level < max_level, so the
//   counts alone tell which slots own blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/sbh.h"

namespace sbh {

constexpr int kMaxLevels = 64;

__host__ __device__ constexpr int topo_stride(int d3) { return ((d3 + 1 + 15) / 16) * 16; }

struct TreeView {
    const float4* pts;
    const float4* pdip;
    const float4* bagg;
    const float4* bdip;
    const float* bspr;
    const uint32_t* btopo;
    const float4* nagg;   // nagg[0] = root aggregate
    const float4* ndip;
    const uint2* bq;      // compressed child aggregates, or NULL
    const float4* bquad;  // scaled second-moment tensors (two float4 per child slot), or NULL
    int32_t n_points;
    int32_t leaf_size;
    int32_t max_level;
    int32_t root_internal;
    int32_t wide;         // an array of the tree reaches 4 GiB: the walks take 64-bit offsets
    float lo[3];
    float side;
    float diam0;          // root cell diagonal; level l has diam0 / d^l
};

// Loads and stores through the global address space.  Kernels that read
// their tree pointers from memory (batched descriptors) would otherwise see
// generic addresses and use flat vector loads where scalar loads serve; for
// pointers passed as kernel arguments these are the loads the compiler emits
// anyway.
#define SBH_GLOBAL __attribute__((address_space(1)))
typedef float sbh_f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 gld4(const float4* p)
{
    const sbh_f32x4 v = *(const SBH_GLOBAL sbh_f32x4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float gld(const float* p) { return *(const SBH_GLOBAL float*)p; }
__device__ __forceinline__ uint32_t gld(const uint32_t* p) { return *(const SBH_GLOBAL uint32_t*)p; }
__device__ __forceinline__ void gst(float* p, float v) { *(SBH_GLOBAL float*)p = v; }

// Device memory of the library: one allocator pair (sbh_set_allocator), or
// the default, the stream-ordered hipMallocAsync / hipFreeAsync.  Objects keep
// the pair they were allocated with and release through it.
struct Allocator {
    sbh_alloc_fn alloc;   // nullptr: the default
    sbh_free_fn free;
    void* ctx;
};
Allocator allocator_current();
hipError_t dev_alloc(const Allocator& a, void** p, size_t bytes, hipStream_t s);
void dev_free(const Allocator& a, void* p, size_t bytes, hipStream_t s);

struct sbh_tree_impl {
    int device;
    Allocator mem;    // the allocator the tree's slabs came from
    int d, d3, bits, leaf_size, max_level, depth, has_normals;
    int64_t n_points, n_nodes, n_blocks;
    float lo[3], side, inv_side;
    float diam[kMaxLevels];
    float4 *pts, *pdip;
    uint32_t* perm;
    uint64_t* codes;
    int32_t *nbegin, *ncount, *nlevel, *ndigit, *nparent, *nfirst, *nnchild;
    float4 *nagg, *ndip;
    float* nspr;
    float4 *bagg, *bdip;
    float* bspr;
    uint32_t* btopo;
    // compressed aggregates (built on request): per child slot two words, binary16
    // {offset x | offset y << 16, offset z | mass fraction << 16}; NULL when absent
    uint2* bq;
    // second-order LOD (built on request): per child slot two float4, the second-moment
    // tensor Q about the child's centre of mass, scaled for the term's evaluation:
    // {1.5 Qxx, 1.5 Qyy, 1.5 Qzz, 3 Qxy}, {3 Qxz, 3 Qyz, tr(Q) / 2, 0}; NULL when absent
    float4* bquad;
    void* slab[3];   // the allocations the arrays above are carved from: points, nodes, blocks
    size_t slab_bytes[3];
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32
// S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and key increments
// 0x9E3779B9 / 0xBB67AE85.
// ---------------------------------------------------------------------------
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // full 64-bit products: one multiply-add instruction gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// Kernel terms f in float32.  `a` = (centre or position, weight), `dp` = w*n.
// ---------------------------------------------------------------------------
struct KParams {
    float eps2;      // eps^2 (potential)
    float alpha;     // smooth distance
    float wscale;    // 1 / mean weight (smooth distance)
};

constexpr float kInv4Pi = 0.0795774715459476679f;

// Single-instruction square root and reciprocal (v_sqrt_f32 / v_rcp_f32,
// about 1 ulp).  Used in the roulette probability, the estimator weights and
// the far-field tests, where the parity tests' near-tie margins (1e-5)
// cover a few ulps.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// The evaluation code is compiled with floating-point contraction off and
// explicit fmaf where a fused multiply-add is wanted, so that a value is the
// same in every kernel that inlines it (single-tree and batched launches
// give bit-identical results).
__device__ __forceinline__ float norm2(float dx, float dy, float dz) { return fmaf(dz, dz, fmaf(dx, dx, dy * dy)); }

template <int K>
__device__ __forceinline__ float term_r2(float4 a, float4 dp, float dx, float dy, float dz, float r2,
                                         const KParams& kp, float r0)
{
#pragma clang fp contract(off)
    if constexpr (K == SBH_POTENTIAL) {
        return a.w * __builtin_amdgcn_rsqf(r2 + kp.eps2);
    } else if constexpr (K == SBH_WINDING) {
        const float inv = __builtin_amdgcn_rsqf(r2);
        const float v = fmaf(dp.z, dz, fmaf(dp.x, dx, dp.y * dy)) * (inv * inv * inv) * kInv4Pi;
        return r2 > 0.0f ? v : 0.0f;
    } else {
        const float r = fsqrt(r2);
        return a.w * kp.wscale * __expf(-kp.alpha * (r - r0));
    }
}

template <int K>
__device__ __forceinline__ float term(float4 a, float4 dp, float qx, float qy, float qz, const KParams& kp,
                                      float r0)
{
#pragma clang fp contract(off)
    const float dx = a.x - qx, dy = a.y - qy, dz = a.z - qz;
    return term_r2<K>(a, dp, dx, dy, dz, norm2(dx, dy, dz), kp, r0);
}

// acc + term_r2<K>(...), with the final add fused into a multiply-add.
template <int K>
__device__ __forceinline__ float term_r2_acc(float4 a, float4 dp, float dx, float dy, float dz, float r2,
                                             const KParams& kp, float r0, float acc)
{
#pragma clang fp contract(off)
    if constexpr (K == SBH_POTENTIAL) {
        return fmaf(a.w, __builtin_amdgcn_rsqf(r2 + kp.eps2), acc);
    } else if constexpr (K == SBH_WINDING) {
        const float inv = __builtin_amdgcn_rsqf(r2);
        const float s = r2 > 0.0f ? (inv * inv * inv) * kInv4Pi : 0.0f;   // 0 at r = 0, where the dot is 0 too
        return fmaf(fmaf(dp.z, dz, fmaf(dp.x, dx, dp.y * dy)), s, acc);
    } else {
        const float r = fsqrt(r2);
        return fmaf(a.w * kp.wscale, __expf(-kp.alpha * (r - r0)), acc);
    }
}

// acc + term<K>(...): the sums of the walks.  For the potential the softening
// enters the first multiply-add of the squared distance and the weight the
// accumulating one (the value differs from term() by rounding only).
template <int K>
__device__ __forceinline__ float term_acc(float4 a, float4 dp, float qx, float qy, float qz, const KParams& kp,
                                          float r0, float acc)
{
#pragma clang fp contract(off)
    const float dx = a.x - qx, dy = a.y - qy, dz = a.z - qz;
    if constexpr (K == SBH_POTENTIAL) {
        const float r2e = fmaf(dz, dz, fmaf(dx, dx, fmaf(dy, dy, kp.eps2)));
        return fmaf(a.w, __builtin_amdgcn_rsqf(r2e), acc);
    } else {
        return term_r2_acc<K>(a, dp, dx, dy, dz, norm2(dx, dy, dz), kp, r0, acc);
    }
}

// Lower bound on the distance from q to any source: its distance to the
// root cube.
__device__ __forceinline__ float cube_distance(const TreeView& tv, float qx, float qy, float qz)
{
    const float ex = fmaxf(fmaxf(tv.lo[0] - qx, qx - (tv.lo[0] + tv.side)), 0.0f);
    const float ey = fmaxf(fmaxf(tv.lo[1] - qy, qy - (tv.lo[1] + tv.side)), 0.0f);
    const float ez = fmaxf(fmaxf(tv.lo[2] - qz, qz - (tv.lo[2] + tv.side)), 0.0f);
    return __builtin_sqrtf(norm2(ex, ey, ez));
}

// Margin of the smooth-distance shift: the shift lies this many 1/alpha below
// the distance to the source that the descent below finds, so that source's
// term is at least e^-30 of its weight share (far from float32 underflow).
constexpr float kSmoothShiftMargin = 30.0f;

// Shift r0 of the smooth-distance sum for query q.  Float32 cannot hold
// w exp(-alpha r) once alpha r exceeds about 87, so the kernels evaluate
// (w / wbar) exp(-alpha (r - r0)) and report r0 - (log F + log wbar) / alpha.
// r0 comes from a greedy descent: from the root, into the non-empty child
// whose cell is nearest to q, down to a leaf; r_up is the distance from q to
// the nearest point of that leaf (an upper bound on the distance to the
// nearest source), and
//   r0 = max(r_up - kSmoothShiftMargin / alpha, distance to the root cube),
// so the sum is at least e^-30 times that point's weight share and no term
// of a point nearer than r0 can exceed the float32 range unless the descent
// missed the nearest source by more than about 100 / alpha.  The shift is a
// common factor of every term: the estimate of the scaled sum stays
// unbiased.  Cells follow the tree's quantisation (a level-l cell of side
// side / d^l); d = 4 digits hold two octree digits, the higher one in bits
// 3..5.
// The cell index along axis a (0 = x) of the child in slot c: a slot of a
// d = 2^g tree holds g octree digits (3 bits each, the coarser ones higher),
// whose bit a is that axis' bit at that level.
__device__ __forceinline__ int digit_axis(int c, int a)
{
    return ((c >> a) & 1) | ((c >> (a + 2)) & 2) | ((c >> (a + 4)) & 4);
}

template <int D>
__device__ __forceinline__ float smooth_shift(const TreeView& tv, float qx, float qy, float qz, float alpha)
{
#pragma clang fp contract(off)
    constexpr int D3 = D * D * D;
    constexpr int TS = topo_stride(D3);
    const float q[3] = {qx, qy, qz};
    float cl[3] = {tv.lo[0], tv.lo[1], tv.lo[2]};
    float cs = tv.side;
    uint32_t n = (uint32_t)tv.n_points, begin = 0u;
    uint32_t blk = 0u;
    for (int level = 0; (int)n > tv.leaf_size && level < tv.max_level; ++level) {
        const float hs = cs * (1.0f / (float)D);
        float dd[3][D];   // squared distance from q to each slab of the cell along each axis
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const float lo = cl[a] + (float)i * hs, hi = lo + hs;
                const float e = fmaxf(fmaxf(lo - q[a], q[a] - hi), 0.0f);
                dd[a][i] = e * e;
            }
        const uint32_t* bt = tv.btopo + (uint64_t)blk * TS;
        float best = INFINITY;
        uint32_t pre = 0u, pre_b = 0u, n_b = 0u;
        int c_b = 0, nint = 0, nint_b = 0;
        for (int c = 0; c < D3; ++c) {
            const uint32_t cnt = gld(bt + c);
            const int ix = digit_axis(c, 0), iy = digit_axis(c, 1), iz = digit_axis(c, 2);
            const float d2 = dd[0][ix] + dd[1][iy] + dd[2][iz];
            if (cnt != 0u && d2 < best) {
                best = d2;
                c_b = c;
                pre_b = pre;
                n_b = cnt;
                nint_b = nint;
            }
            nint += ((int)cnt > tv.leaf_size && level + 1 < tv.max_level) ? 1 : 0;
            pre += cnt;
        }
        const int ix = digit_axis(c_b, 0), iy = digit_axis(c_b, 1), iz = digit_axis(c_b, 2);
        cl[0] += (float)ix * hs;
        cl[1] += (float)iy * hs;
        cl[2] += (float)iz * hs;
        cs = hs;
        blk = gld(bt + D3) + (uint32_t)nint_b;
        begin += pre_b;
        n = n_b;
    }
    float r2 = INFINITY;
    for (uint32_t i = 0; i < n; ++i) {
        const float4 p = gld4(tv.pts + (uint64_t)(begin + i));
        r2 = fminf(r2, norm2(p.x - qx, p.y - qy, p.z - qz));
    }
    return fmaxf(__builtin_sqrtf(r2) - kSmoothShiftMargin / alpha, cube_distance(tv, qx, qy, qz));
}

// A query with a non-finite coordinate has no defined value: NaN.
__device__ __forceinline__ float nan_unless_finite(float v, float qx, float qy, float qz)
{
    return (__builtin_isfinite(qx) && __builtin_isfinite(qy) && __builtin_isfinite(qz)) ? v : __builtin_nanf("");
}

// The value written for query q from the estimated (or summed) F: the smooth
// distance r0 - (log F + log wbar) / alpha, or F itself.
template <int K>
__device__ __forceinline__ float query_value(float F, float r0, float logwbar, float alpha, float qx, float qy,
                                             float qz)
{
    const float v = (K == SBH_SMOOTHDIST) ? r0 - (logf(F) + logwbar) / alpha : F;
    return nan_unless_finite(v, qx, qy, qz);
}

// ---------------------------------------------------------------------------
// Host-side launchers (defined in the .hip files).  All return hipError_t.
// ---------------------------------------------------------------------------
struct BuildScratch;

hipError_t launch_bbox(const float* src, const float* w, const float* nrm, int64_t n, float* params_dev,
                       float* partial_dev, int nblocks, hipStream_t s);
hipError_t launch_morton(const float* src, int64_t n, const float* params_dev, uint64_t* keys, uint32_t* vals,
                         hipStream_t s);
hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n,
                            int begin_bit, int end_bit, uint32_t* hist, uint32_t* scan_tmp, hipStream_t s);
size_t radix_sort_hist_size(int64_t n);
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, uint32_t* tmp,
                              hipStream_t s);
size_t scan_tmp_size(int64_t n);

struct EvalLaunch {
    int kernel;
    int samples;
    uint64_t seed;
    int group;
    int rr_mode;
    uint32_t batch;
    float beta;
    float eps, alpha;
    int32_t* paths;
    int tile_score;     // coherent walk with the tile-shared score proposal (d = 2, group % 64 == 0)
    int cut;            // subdomains: the Barnes-Hut cut at beta (group % 64 == 0, d = 2 or 4)
    int compressed;     // the coherent walk on the compressed aggregates (d = 2, potential or smooth distance)
    int lod;            // 2: second-order node terms (potential, d = 2, coherent walk)
};

hipError_t launch_sbh_eval(const sbh_tree_impl* t, const float* queries, int64_t nq, const EvalLaunch& e,
                           float* out, hipStream_t s);
hipError_t launch_bh_eval(const sbh_tree_impl* t, const float* queries, int64_t nq, const EvalLaunch& e,
                          float* out, hipStream_t s);
hipError_t launch_brute(const float* src, const float* w, const float* nrm, int64_t n, const float* queries,
                        int64_t nq, int kernel, float eps, float alpha, int fp64, void* out, hipStream_t s);
sbh_status build_tree_impl(const float* src, const float* w, const float* nrm, int64_t n, int d, int leaf_size,
                           int max_level, int compress, int quadrupole, hipStream_t s, sbh_tree_impl* t,
                           std::string* msg);

TreeView make_view(const sbh_tree_impl* t);

// batched persistent evaluation (eval.hip)
struct BatchItem {          // one cloud of a batch (device copy)
    TreeView tv;
    const float* queries;
    float* out;
    int64_t nq;
    int32_t kernel, d, root_leaf, pad;
};
struct BatchState {         // per-launch Philox key and batch word
    uint32_t key0, key1, batch, pad;
};
constexpr int kBatchGroups = 6;   // (branching factor 2 or 4) x (kernel)
constexpr int kBatchLaunchGroups = kBatchGroups + 3;   // and one exact-sum group per kernel (root leaves)
constexpr int kBatchMaxTileWaves = 2;   // tiles per batch workgroup
// Wavefronts that share one 64-query tile in the coherent kernels (single-tree
// and batched), each walking an equal share of the root slots.
constexpr int kWaveParts = 2;
hipError_t launch_batch_begin(BatchState* st, uint64_t seed, uint32_t batch, hipStream_t s);
// One launch of a group: workgroup b (of `blocks`, each of `tile_waves` wavefronts) evaluates tiles
// wg[b].y, wg[b].y + 1, ... of cloud items[wg[b].x]; `lds_bytes` of dynamic LDS per workgroup (not
// touched) cap the number of workgroups resident on a compute unit.
hipError_t launch_sbh_batch(int d, int kernel, const BatchItem* items, const int2* wg, int blocks, int tile_waves,
                            size_t lds_bytes, const BatchState* st, int samples, int group, int rr_mode, float eps,
                            float alpha, hipStream_t s);
void* batch_begin_kernel();
hipError_t batch_static_lds(size_t* bytes);   // the batch kernels' own LDS per workgroup
hipError_t launch_leaf_batch(int kernel, const BatchItem* items, const int2* wg, int blocks, int tile_waves, float eps,
                             float alpha, hipStream_t s);

// learned proposal (mlp.hip)
constexpr int kMlpParams = 1608;
hipError_t launch_sbh_learned(const sbh_tree_impl* t, const float* queries, int64_t nq, const EvalLaunch& e,
                              const float* prm, float* out, hipStream_t s);
hipError_t launch_mlp_forward(const float* prm, const float* x, int64_t n, float* z, hipStream_t s);
size_t mlp_partial_floats(int64_t rows);
hipError_t launch_mlp_grad(const float* prm, const float* X, const float* Tg, const float* Cn, int64_t n,
                           int64_t row_begin, int64_t rows, float* partial, float* grad, hipStream_t s);
hipError_t launch_mlp_adam(float* prm, float* state, const float* grad, float lr, int step, float* loss_out,
                           hipStream_t s);
hipError_t launch_mlp_pairs(const sbh_tree_impl* t, const float* queries, int64_t nq, int lmax, uint64_t seed,
                            int kernel, float eps, float alpha, float* X, float* Tg, float* Cn, int4* loc,
                            hipStream_t s);

}  // namespace sbh
