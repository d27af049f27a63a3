// Tree construction on the GPU (Section 3.1: an octree-like tree over the
// sources with per-node aggregate weight and centre of mass; the summed
// dipole w*n is added for the winding kernel).
//
// Pipeline, every step a kernel on the caller's stream:
//   1. root cube: per-axis min/max, side = largest extent, inv_side =
//      fl32(1/side) (correctly rounded), plus an input validity flag;
//   2. Morton code: cell_a = min(2^20-1, (u32) fl32(fl32(x_a - lo_a) *
//      inv_side) * 2^20), bits of x/y/z interleaved into 60 bits;
//   3. stable LSD radix sort of (code, index), 8-bit digits;
//   4. levels top-down: a node at level l is a maximal run of equal
//      (bits*l)-bit prefix; it is split iff count > leaf_size and l < max;
//      its children are found by binary search for each digit and compacted
//      in (parent, digit) order, which is breadth-first order;
//   5. aggregates bottom-up (leaves from points, internal nodes from
//      children) and packing into the per-node child blocks.
// Levels need their node counts on the host, so the build synchronises twice
// per level (its internal nodes, then their children); it is not part of the
// timed evaluation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sbh_internal.hpp"

namespace sbh {

// ---------------------------------------------------------------------------
// 1. Root cube and validation
// ---------------------------------------------------------------------------
constexpr int kBboxThreads = 256;

__global__ void __launch_bounds__(kBboxThreads) k_bbox_partial(const float* __restrict__ src,
                                                               const float* __restrict__ w,
                                                               const float* __restrict__ nrm, int64_t n,
                                                               float* __restrict__ partial)
{
    float mn0 = INFINITY, mn1 = INFINITY, mn2 = INFINITY;
    float mx0 = -INFINITY, mx1 = -INFINITY, mx2 = -INFINITY;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = src[3 * i], y = src[3 * i + 1], z = src[3 * i + 2];
        const float wi = w[i];
        bad |= !(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z));
        bad |= !(wi > 0.0f && __builtin_isfinite(wi));
        if (nrm) {
            const float a = nrm[3 * i], b = nrm[3 * i + 1], c = nrm[3 * i + 2];
            bad |= !(__builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c));
        }
        mn0 = fminf(mn0, x); mn1 = fminf(mn1, y); mn2 = fminf(mn2, z);
        mx0 = fmaxf(mx0, x); mx1 = fmaxf(mx1, y); mx2 = fmaxf(mx2, z);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mn0 = fminf(mn0, __shfl_xor(mn0, o)); mn1 = fminf(mn1, __shfl_xor(mn1, o)); mn2 = fminf(mn2, __shfl_xor(mn2, o));
        mx0 = fmaxf(mx0, __shfl_xor(mx0, o)); mx1 = fmaxf(mx1, __shfl_xor(mx1, o)); mx2 = fmaxf(mx2, __shfl_xor(mx2, o));
        bad |= __shfl_xor(bad, o);
    }
    __shared__ float sh[kBboxThreads / 64][7];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        sh[wv][0] = mn0; sh[wv][1] = mn1; sh[wv][2] = mn2;
        sh[wv][3] = mx0; sh[wv][4] = mx1; sh[wv][5] = mx2; sh[wv][6] = (float)bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBboxThreads / 64; ++k) {
            for (int a = 0; a < 3; ++a) {
                sh[0][a] = fminf(sh[0][a], sh[k][a]);
                sh[0][3 + a] = fmaxf(sh[0][3 + a], sh[k][3 + a]);
            }
            sh[0][6] = fmaxf(sh[0][6], sh[k][6]);
        }
        for (int a = 0; a < 7; ++a) partial[blockIdx.x * 8 + a] = sh[0][a];
    }
}

// params: lo[3], side, inv_side, bad.  One workgroup: each thread folds a
// stride of the partials, then the wavefronts and the workgroup combine
// (min and max are exact, so the order does not change the result).
__global__ void __launch_bounds__(kBboxThreads) k_bbox_final(const float* __restrict__ partial, int nb,
                                                             float* __restrict__ params)
{
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    float bad = 0.0f;
    for (int b = threadIdx.x; b < nb; b += kBboxThreads) {
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], partial[b * 8 + a]);
            mx[a] = fmaxf(mx[a], partial[b * 8 + 3 + a]);
        }
        bad = fmaxf(bad, partial[b * 8 + 6]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], __shfl_xor(mn[a], o));
            mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o));
        }
        bad = fmaxf(bad, __shfl_xor(bad, o));
    }
    __shared__ float sh[kBboxThreads / 64][7];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        for (int a = 0; a < 3; ++a) {
            sh[wv][a] = mn[a];
            sh[wv][3 + a] = mx[a];
        }
        sh[wv][6] = bad;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int k = 1; k < kBboxThreads / 64; ++k) {
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], sh[k][a]);
            mx[a] = fmaxf(mx[a], sh[k][3 + a]);
        }
        bad = fmaxf(bad, sh[k][6]);
    }
    float side = 0.0f;
    for (int a = 0; a < 3; ++a) {
        const float e = __fsub_rn(mx[a], mn[a]);
        side = e > side ? e : side;
    }
    if (side == 0.0f) side = 1.0f;
    params[0] = mn[0]; params[1] = mn[1]; params[2] = mn[2];
    params[3] = side;
    params[4] = __fdiv_rn(1.0f, side);
    params[5] = bad;
}

hipError_t launch_bbox(const float* src, const float* w, const float* nrm, int64_t n, float* params_dev,
                       float* partial_dev, int nblocks, hipStream_t s)
{
    k_bbox_partial<<<nblocks, kBboxThreads, 0, s>>>(src, w, nrm, n, partial_dev);
    k_bbox_final<<<1, kBboxThreads, 0, s>>>(partial_dev, nblocks, params_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 2. Morton codes
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread_bits3(uint32_t v)
{
    // bit k of v (k < 21) moves to bit 3k
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t quantize(float x, float lo, float inv_side)
{
    float u = __fsub_rn(x, lo);
    u = __fmul_rn(u, inv_side);
    u = __fmul_rn(u, 1048576.0f);
    uint32_t c = (uint32_t)u;  // truncation; u >= 0
    return c > 1048575u ? 1048575u : c;
}

__global__ void k_morton(const float* __restrict__ src, int64_t n, const float* __restrict__ params,
                         uint64_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float inv = params[4];
    const uint32_t cx = quantize(src[3 * i], params[0], inv);
    const uint32_t cy = quantize(src[3 * i + 1], params[1], inv);
    const uint32_t cz = quantize(src[3 * i + 2], params[2], inv);
    keys[i] = spread_bits3(cx) | (spread_bits3(cy) << 1) | (spread_bits3(cz) << 2);
    vals[i] = (uint32_t)i;
}

hipError_t launch_morton(const float* src, int64_t n, const float* params_dev, uint64_t* keys, uint32_t* vals,
                         hipStream_t s)
{
    const int64_t nb = (n + 255) / 256;
    k_morton<<<(unsigned)nb, 256, 0, s>>>(src, n, params_dev, keys, vals);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 (tile scan + recursive scan of tile sums)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane)
{
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tile(const uint32_t* in, uint32_t* out, int64_t n,
                                                            uint32_t* __restrict__ tile_sums)
{
    __shared__ uint32_t tile[kScanTile];
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t idx = base + k * kScanThreads + threadIdx.x;
        tile[k * kScanThreads + threadIdx.x] = idx < n ? in[idx] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanItems], tsum = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = tile[threadIdx.x * kScanItems + k];
        tsum += v[k];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t incl = wave_inclusive_scan(tsum, lane);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t woff = 0, total = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) {
        if (k < wv) woff += wsum[k];
        total += wsum[k];
    }
    uint32_t run = woff + incl - tsum;
    for (int k = 0; k < kScanItems; ++k) {
        tile[threadIdx.x * kScanItems + k] = run;
        run += v[k];
    }
    __syncthreads();
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t idx = base + k * kScanThreads + threadIdx.x;
        if (idx < n) out[idx] = tile[k * kScanThreads + threadIdx.x];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(uint32_t* out, int64_t n, const uint32_t* __restrict__ offs)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] += offs[idx / kScanTile];
}

size_t scan_tmp_size(int64_t n)
{
    size_t total = 1;  // room for the final total
    while (n > 1) {
        const int64_t nb = (n + kScanTile - 1) / kScanTile;
        total += (size_t)nb + 64;
        n = nb;
    }
    return total + 64;
}

// out may alias in.  *total_dev receives the sum of all inputs.
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, uint32_t* tmp,
                              hipStream_t s)
{
    if (n <= 0) return hipMemsetAsync(total_dev, 0, sizeof(uint32_t), s);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        k_scan_tile<<<1, kScanThreads, 0, s>>>(in, out, n, total_dev);
        return hipGetLastError();
    }
    uint32_t* sums = tmp;
    k_scan_tile<<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive_u32(sums, sums, nb, total_dev, tmp + nb + 64, s);
    if (e != hipSuccess) return e;
    k_scan_add<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, n, sums);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3. Stable LSD radix sort of (uint64 key, uint32 value), 8-bit digits.
// Each block owns a tile of 4096 keys; wave w of the block owns the w-th
// quarter and walks it in 16 chunks of 64 in order, so ranks computed as
// (digit offset of the tile) + (earlier waves) + (earlier chunks of this
// wave) + (earlier lanes of this chunk) preserve the input order of equal
// digits.
// ---------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsChunks = 16;
constexpr int kRsTile = kRsThreads * kRsChunks;

__global__ void __launch_bounds__(kRsThreads) k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                        uint32_t* __restrict__ hist, int nb)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int k = 0; k < kRsChunks; ++k) {
        const int64_t idx = base + k * kRsThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const uint64_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ vals, int64_t n, int shift,
                                                           const uint32_t* __restrict__ offs, int nb,
                                                           uint64_t* __restrict__ kout, uint32_t* __restrict__ vout)
{
    __shared__ uint32_t wcnt[kRsWaves][256];
    __shared__ uint32_t gbase[256];
    for (int w = 0; w < kRsWaves; ++w) wcnt[w][threadIdx.x] = 0;
    gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t kk[kRsChunks];
    uint32_t vv[kRsChunks], rank[kRsChunks], dig[kRsChunks];
    const int64_t wbase = (int64_t)blockIdx.x * kRsTile + (int64_t)wv * (kRsChunks * 64);
    for (int c = 0; c < kRsChunks; ++c) {
        const int64_t idx = wbase + c * 64 + lane;
        const bool valid = idx < n;
        const uint64_t key = valid ? keys[idx] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t below = __popcll(m & lt_mask);
        const uint32_t cnt = __popcll(m);
        const uint32_t base = wcnt[wv][d];
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) wcnt[wv][d] = base + cnt;
        __builtin_amdgcn_wave_barrier();
        kk[c] = key;
        vv[c] = valid ? vals[idx] : 0u;
        rank[c] = base + below;
        dig[c] = valid ? d : 256u;
    }
    __syncthreads();
    {
        uint32_t run = 0;
        for (int w = 0; w < kRsWaves; ++w) {
            const uint32_t t = wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = run;
            run += t;
        }
    }
    __syncthreads();
    for (int c = 0; c < kRsChunks; ++c) {
        if (dig[c] < 256u) {
            const uint32_t pos = gbase[dig[c]] + wcnt[wv][dig[c]] + rank[c];
            kout[pos] = kk[c];
            vout[pos] = vv[c];
        }
    }
}

size_t radix_sort_hist_size(int64_t n)
{
    const int64_t nb = (n + kRsTile - 1) / kRsTile;
    return (size_t)nb * 256;
}

hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n,
                            int begin_bit, int end_bit, uint32_t* hist, uint32_t* scan_tmp, hipStream_t s)
{
    const int nb = (int)((n + kRsTile - 1) / kRsTile);
    uint64_t *ks = keys, *kd = keys_tmp;
    uint32_t *vs = vals, *vd = vals_tmp;
    int passes = 0;
    for (int shift = begin_bit; shift < end_bit; shift += 8, ++passes) {
        k_rs_hist<<<nb, kRsThreads, 0, s>>>(ks, n, shift, hist, nb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = scan_exclusive_u32(hist, hist, (int64_t)nb * 256, scan_tmp, scan_tmp + 1, s);
        if (e != hipSuccess) return e;
        k_rs_scatter<<<nb, kRsThreads, 0, s>>>(ks, vs, n, shift, hist, nb, kd, vd);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* tk = ks; ks = kd; kd = tk;
        uint32_t* tv = vs; vs = vd; vd = tv;
    }
    if (passes & 1) {
        hipError_t e = hipMemcpyAsync(keys, ks, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(vals, vs, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// 4. Levels
// ---------------------------------------------------------------------------
struct float3v {
    float x, y, z;
};

__global__ void k_gather_points(const float* __restrict__ src, const float* __restrict__ w,
                                const float* __restrict__ nrm, const uint32_t* __restrict__ perm, int64_t n,
                                float4* __restrict__ pts, float4* __restrict__ pdip)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t i = perm[s];
    const float wi = w[i];
    // a point's three floats in one 12-byte load: the reads are random, so each
    // separate load would be another cache-line request
    float3v x;
    __builtin_memcpy(&x, src + 3 * (int64_t)i, sizeof(x));
    pts[s] = make_float4(x.x, x.y, x.z, wi);
    if (pdip) {
        float3v m;
        __builtin_memcpy(&m, nrm + 3 * (int64_t)i, sizeof(m));
        pdip[s] = make_float4(wi * m.x, wi * m.y, wi * m.z, 0.0f);
    }
}

// flags[i] = node i of this level is internal; also resets first/nchild
__global__ void k_level_flags(const int32_t* __restrict__ lc, int n, int level, int leaf, int maxlev,
                              uint32_t* __restrict__ flags, int32_t* __restrict__ lfirst,
                              int32_t* __restrict__ lnch)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = (lc[i] > leaf && level < maxlev) ? 1u : 0u;
    lfirst[i] = -1;
    lnch[i] = 0;
}

__global__ void k_internal_map(const uint32_t* __restrict__ flags, const uint32_t* __restrict__ iscan, int n,
                               int32_t* __restrict__ imap)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flags[i]) imap[iscan[i]] = i;
}

__device__ __forceinline__ int32_t lower_bound_prefix(const uint64_t* __restrict__ codes, int32_t b, int32_t e,
                                                      int shift, uint64_t key)
{
    while (b < e) {
        const int32_t mid = b + ((e - b) >> 1);
        if ((codes[mid] >> shift) < key) b = mid + 1;
        else e = mid;
    }
    return b;
}

// one thread per (internal node k of this level, digit slot)
__global__ void k_children(const int32_t* __restrict__ lb, const int32_t* __restrict__ lc,
                           const int32_t* __restrict__ imap, int n_int, int level, int bits, int d3,
                           const uint64_t* __restrict__ codes, uint32_t blk_off, uint32_t* __restrict__ btopo, int ts,
                           uint32_t* __restrict__ ccount, int32_t* __restrict__ cbegin, uint32_t* __restrict__ cflag)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_int * d3) return;
    const int k = (int)(t / d3), dg = (int)(t % d3);
    const int i = imap[k];
    const int32_t b = lb[i], e = lb[i] + lc[i];
    const int shift = 60 - bits * (level + 1);
    const uint64_t prefix = codes[b] >> (shift + bits);
    const uint64_t key = (prefix << bits) | (uint64_t)dg;
    const int32_t lo = lower_bound_prefix(codes, b, e, shift, key);
    const int32_t hi = lower_bound_prefix(codes, lo, e, shift, key + 1);
    const uint32_t cnt = (uint32_t)(hi - lo);
    btopo[(int64_t)(blk_off + k) * ts + dg] = cnt;
    ccount[t] = cnt;
    cbegin[t] = lo;
    cflag[t] = cnt > 0 ? 1u : 0u;
}

// one thread per (internal node k, slot): emit the non-empty children into the next level
__global__ void k_emit(const uint32_t* __restrict__ ccount, const int32_t* __restrict__ cbegin,
                       const uint32_t* __restrict__ cscan, const int32_t* __restrict__ imap, int n_int, int d3,
                       int32_t off_cur, int32_t off_next, uint32_t blk_off, int32_t* __restrict__ nb_next,
                       int32_t* __restrict__ nc_next, int32_t* __restrict__ npar_next, int32_t* __restrict__ ndig_next,
                       int32_t* __restrict__ npblk_next, int32_t* __restrict__ lfirst, int32_t* __restrict__ lnch)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_int * d3) return;
    const int k = (int)(t / d3), dg = (int)(t % d3);
    const int i = imap[k];
    const uint32_t cnt = ccount[t];
    if (cnt > 0) {
        const uint32_t c = cscan[t];
        nb_next[c] = cbegin[t];
        nc_next[c] = (int32_t)cnt;
        npar_next[c] = off_cur + i;
        ndig_next[c] = dg;
        npblk_next[c] = (int32_t)(blk_off + k);
    }
    if (dg == 0) {
        int nch = 0;
        for (int q = 0; q < d3; ++q) nch += ccount[(int64_t)k * d3 + q] > 0;
        lfirst[i] = off_next + (int32_t)cscan[t];
        lnch[i] = nch;
    }
}

// block of internal node k (level l) gets the block id of its first internal child
__global__ void k_set_base(const uint32_t* __restrict__ cscan_prev, int n_int_prev, int d3, uint32_t blk_off_prev,
                           const uint32_t* __restrict__ iscan_next, uint32_t blk_off_next, uint32_t* __restrict__ btopo,
                           int ts)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_int_prev) return;
    const uint32_t fc = cscan_prev[(int64_t)k * d3];
    btopo[(int64_t)(blk_off_prev + k) * ts + d3] = blk_off_next + iscan_next[fc];
}

// ---------------------------------------------------------------------------
// 5. Aggregates and packing
// ---------------------------------------------------------------------------
// Aggregates of one level's nodes (offset off, n of them), in float64: from
// the points of a leaf, from the children's float64 aggregates for an
// internal node (mass, w-weighted centre of mass, summed w n, and the second
// moment about the centre of mass by the parallel-axis rule, a sum of
// non-negative terms).  The tree stores each as the float32 nearest to its
// float64 value: one rounding, so a one-point leaf's centre of mass is its
// point and its second moment exactly 0, as the definitions give.
__global__ void k_aggregate(int32_t off, int32_t n, const int32_t* __restrict__ nbegin,
                            const int32_t* __restrict__ ncount, const int32_t* __restrict__ nfirst,
                            const int32_t* __restrict__ nnchild, const float4* __restrict__ pts,
                            const float4* __restrict__ pdip, double4* __restrict__ agg64, double4* __restrict__ dip64,
                            double* __restrict__ spr64, float4* __restrict__ nagg, float4* __restrict__ ndip,
                            float* __restrict__ nspr, double* __restrict__ quad64)
{
#pragma clang fp contract(off)
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t g = off + i;
    double m = 0.0, sx = 0.0, sy = 0.0, sz = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
    const int32_t f = nfirst[g];
    if (f < 0) {
        const int32_t b = nbegin[g], e = b + ncount[g];
        for (int32_t s = b; s < e; ++s) {
            const float4 p = pts[s];
            const double w = p.w;
            m += w; sx += w * (double)p.x; sy += w * (double)p.y; sz += w * (double)p.z;
            if (pdip) { const float4 q = pdip[s]; dx += q.x; dy += q.y; dz += q.z; }
        }
    } else {
        const int32_t e = f + nnchild[g];
        for (int32_t c = f; c < e; ++c) {
            const double4 a = agg64[c];
            m += a.w; sx += a.w * a.x; sy += a.w * a.y; sz += a.w * a.z;
            if (pdip) { const double4 q = dip64[c]; dx += q.x; dy += q.y; dz += q.z; }
        }
    }
    const double cx = sx / m, cy = sy / m, cz = sz / m;
    double s2 = 0.0;
    if (f < 0) {
        const int32_t b = nbegin[g], e = b + ncount[g];
        for (int32_t s = b; s < e; ++s) {
            const float4 p = pts[s];
            const double ex = (double)p.x - cx, ey = (double)p.y - cy, ez = (double)p.z - cz;
            s2 += (double)p.w * (ex * ex + ey * ey + ez * ez);
        }
    } else {
        const int32_t e = f + nnchild[g];
        for (int32_t c = f; c < e; ++c) {
            const double4 a = agg64[c];
            const double ex = a.x - cx, ey = a.y - cy, ez = a.z - cz;
            s2 += a.w * (spr64[c] + (ex * ex + ey * ey + ez * ez));
        }
    }
    s2 /= m;
    if (quad64) {
        // second-moment tensor about the centre of mass, Q = sum w (p - c)(p - c)^T: over the
        // points of a leaf; over the children of a node by the parallel-axis rule,
        // Q = sum_c (Q_c + m_c (c_c - c)(c_c - c)^T)
        double Q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (f < 0) {
            const int32_t b = nbegin[g], e = b + ncount[g];
            for (int32_t s = b; s < e; ++s) {
                const float4 p = pts[s];
                const double ww = p.w, ex = (double)p.x - cx, ey = (double)p.y - cy, ez = (double)p.z - cz;
                Q[0] += ww * ex * ex; Q[1] += ww * ey * ey; Q[2] += ww * ez * ez;
                Q[3] += ww * ex * ey; Q[4] += ww * ex * ez; Q[5] += ww * ey * ez;
            }
        } else {
            const int32_t e = f + nnchild[g];
            for (int32_t c = f; c < e; ++c) {
                const double4 a = agg64[c];
                const double* qc = quad64 + 6 * (int64_t)c;
                const double ex = a.x - cx, ey = a.y - cy, ez = a.z - cz;
                Q[0] += qc[0] + a.w * ex * ex; Q[1] += qc[1] + a.w * ey * ey; Q[2] += qc[2] + a.w * ez * ez;
                Q[3] += qc[3] + a.w * ex * ey; Q[4] += qc[4] + a.w * ex * ez; Q[5] += qc[5] + a.w * ey * ez;
            }
        }
        for (int k = 0; k < 6; ++k) quad64[6 * (int64_t)g + k] = Q[k];
    }
    agg64[g] = make_double4(cx, cy, cz, m);
    spr64[g] = s2;
    nagg[g] = make_float4((float)cx, (float)cy, (float)cz, (float)m);
    nspr[g] = (float)s2;
    if (pdip) {
        dip64[g] = make_double4(dx, dy, dz, 0.0);
        ndip[g] = make_float4((float)dx, (float)dy, (float)dz, 0.0f);
    }
}

// binary16 value nearest to x (round to nearest even) as a double: the rounding
// is done on x itself (no float32 rounding first); |x| beyond binary16's range
// gives +-infinity, x below it the nearest subnormal.
__device__ __forceinline__ double f16_round_d(double x)
{
    if (!(x == x) || x == 0.0 || __builtin_isinf(x)) return x;
    int e;
    (void)frexp(x, &e);
    int ex = e - 1;
    if (ex < -14) ex = -14;
    const double quantum = ldexp(1.0, ex - 10);
    const double r = rint(x / quantum) * quantum;
    if (fabs(r) > 65504.0) return x > 0.0 ? __builtin_inf() : -__builtin_inf();
    return r;
}

__device__ __forceinline__ uint32_t f16_bits(double exact16)
{
    const _Float16 h = (_Float16)(float)exact16;   // exact: the value is a binary16 number
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}

// Compressed aggregates of one level's nodes (offset off, n of them; level
// >= 1), top-down: each node's binary16 offset from its decoded parent in
// units of its cell side sl, and its binary16 fraction of the decoded parent's
// mass, decoded again in float64 for its own children.  agg64 holds the exact
// aggregates (float64 sums, k_aggregate); qagg the decoded ones (com, mass).
__global__ void k_compress(int32_t off, int32_t n, double sl, const int32_t* __restrict__ nparent,
                           const int32_t* __restrict__ npblk, const int32_t* __restrict__ ndig,
                           const double4* __restrict__ agg64, double4* __restrict__ qagg, uint2* __restrict__ bq,
                           int d3)
{
#pragma clang fp contract(off)
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t g = off + i;
    const double4 a = agg64[g];
    const double4 pq = qagg[nparent[g]];
    const double ox = f16_round_d((a.x - pq.x) / sl);
    const double oy = f16_round_d((a.y - pq.y) / sl);
    const double oz = f16_round_d((a.z - pq.z) / sl);
    const double fm = f16_round_d(a.w / pq.w);
    qagg[g] = make_double4(pq.x + ox * sl, pq.y + oy * sl, pq.z + oz * sl, pq.w * fm);
    bq[(int64_t)npblk[g] * d3 + ndig[g]] = make_uint2(f16_bits(ox) | (f16_bits(oy) << 16), f16_bits(oz) | (f16_bits(fm) << 16));
}

// the root's decoded aggregate: its float32 centre of mass and mass
__global__ void k_compress_root(const double4* __restrict__ agg64, double4* __restrict__ qagg)
{
    const double4 a = agg64[0];
    qagg[0] = make_double4((double)(float)a.x, (double)(float)a.y, (double)(float)a.z, (double)(float)a.w);
}

// The children's second-moment tensors into their block slots, scaled for the
// second-order term (rounded once from float64).
__global__ void k_pack_quad(int32_t n_nodes, const int32_t* __restrict__ npblk, const int32_t* __restrict__ ndig,
                            const double* __restrict__ quad64, float4* __restrict__ bquad, int d3)
{
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (g >= n_nodes) return;
    const int64_t slot = (int64_t)npblk[g] * d3 + ndig[g];
    const double* Q = quad64 + 6 * (int64_t)g;
    bquad[2 * slot] = make_float4((float)(1.5 * Q[0]), (float)(1.5 * Q[1]), (float)(1.5 * Q[2]), (float)(3.0 * Q[3]));
    bquad[2 * slot + 1] = make_float4((float)(3.0 * Q[4]), (float)(3.0 * Q[5]), (float)(0.5 * (Q[0] + Q[1] + Q[2])), 0.0f);
}

__global__ void k_pack(int32_t n_nodes, const int32_t* __restrict__ npblk, const int32_t* __restrict__ ndig,
                       const float4* __restrict__ nagg, const float4* __restrict__ ndip,
                       const float* __restrict__ nspr, float4* __restrict__ bagg, float4* __restrict__ bdip,
                       float* __restrict__ bspr, int d3)
{
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (g >= n_nodes) return;
    const int64_t slot = (int64_t)npblk[g] * d3 + ndig[g];
    bagg[slot] = nagg[g];
    bspr[slot] = nspr[g];
    if (bdip) bdip[slot] = ndip[g];
}

// the root's level arrays: first point 0, all n points, no parent, digit 0, no parent block
__global__ void k_root_init(int32_t n, int32_t* b, int32_t* c, int32_t* par, int32_t* dig, int32_t* pblk)
{
    if (threadIdx.x != 0) return;
    b[0] = 0;
    c[0] = n;
    par[0] = -1;
    dig[0] = 0;
    pblk[0] = -1;
}

// The per-level arrays concatenated into the node and block arrays, each
// family in one launch (the tables travel as kernel arguments).
constexpr int kLevelTab = 24;   // levels of a tree: at most 60 / 3 + 1 = 21
struct LevelTab {
    int64_t off[kLevelTab + 1];          // first node of each level
    const int32_t* src[7][kLevelTab];    // begin, count, digit, parent, first child, child count, parent block
};
struct NodeDst {
    int32_t* p[8];                       // the same seven node arrays, then the level
};
struct TopoTab {
    int64_t off[kLevelTab + 1];          // first topology word of each level's blocks
    const uint32_t* src[kLevelTab];
};

__global__ void k_concat_levels(LevelTab tab, int n_levels, NodeDst dst)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= tab.off[n_levels]) return;
    int l = 0;
    while (g >= tab.off[l + 1]) ++l;
    const int64_t i = g - tab.off[l];
#pragma unroll
    for (int a = 0; a < 7; ++a) dst.p[a][g] = tab.src[a][l][i];
    dst.p[7][g] = l;
}

__global__ void k_concat_topo(TopoTab tab, int n_levels, uint32_t* __restrict__ btopo)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= tab.off[n_levels]) return;
    int l = 0;
    while (g >= tab.off[l + 1]) ++l;
    btopo[g] = tab.src[l][g - tab.off[l]];
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------
namespace {

// The tree's own arrays are carved, at 256-B boundaries, out of three
// allocations (points, nodes, blocks) that the tree frees when it is released.
template <class T>
size_t carve_bytes(int64_t count)
{
    return ((size_t)count * sizeof(T) + 255) & ~(size_t)255;
}

struct Carver {
    char* p;
    template <class T> T* take(int64_t count)
    {
        T* r = (T*)p;
        p += carve_bytes<T>(count);
        return r;
    }
};

// Temporaries of one build: a bump allocator over a few large chunks.  A
// build takes some two hundred temporaries, and one allocation each cost
// several times the build's kernels.  Chunks come from the library's
// allocator on the build's stream and go back to it, in stream order, when
// the build ends.
struct DevPool {
    static constexpr size_t kChunk = (size_t)64 << 20;
    Allocator mem;
    hipStream_t s;
    std::vector<std::pair<void*, size_t>> chunks;
    char* cur = nullptr;
    size_t left = 0;
    hipError_t err = hipSuccess;
    DevPool(const Allocator& a, hipStream_t st) : mem(a), s(st) {}
    template <class T>
    T* alloc(int64_t count)
    {
        if (err != hipSuccess) return nullptr;
        const size_t bytes = (((size_t)(count > 0 ? count : 1) * sizeof(T)) + 255) & ~(size_t)255;
        if (bytes > left) {
            void* p = nullptr;
            const size_t sz = bytes > kChunk ? bytes : kChunk;
            err = dev_alloc(mem, &p, sz, s);
            if (err != hipSuccess) return nullptr;
            chunks.push_back({p, sz});
            cur = (char*)p;
            left = sz;
        }
        T* r = (T*)cur;
        cur += bytes;
        left -= bytes;
        return r;
    }
    ~DevPool()
    {
        for (auto& c : chunks) dev_free(mem, c.first, c.second, s);
    }
};

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

struct LevelBufs {
    int32_t n = 0;
    int32_t *b = nullptr, *c = nullptr, *par = nullptr, *dig = nullptr, *pblk = nullptr, *first = nullptr,
            *nch = nullptr;
};

}  // namespace

// Builds the tree into *t.  Returns SBH_OK or an error code with *msg set.
sbh_status build_tree_impl(const float* src, const float* w, const float* nrm, int64_t n, int d, int leaf_size,
                           int max_level, int compress, int quadrupole, hipStream_t s, sbh_tree_impl* t,
                           std::string* msg)
{
    DevPool tmp(t->mem, s);
    auto fail_hip = [&](hipError_t e, const char* where) {
        *msg = std::string(where) + ": " + hipGetErrorString(e);
        return e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? SBH_ENOMEM : SBH_EHIP;
    };
#define SBH_TRY(expr, where)                        \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return fail_hip(e_, where); \
    } while (0)
#define SBH_ALLOC_OK(where)                                    \
    do {                                                       \
        if (tmp.err != hipSuccess) return fail_hip(tmp.err, where); \
    } while (0)

    const int lg = d == 2 ? 1 : d == 4 ? 2 : 3;
    const int bits = 3 * lg;
    const int d3 = d * d * d;
    const int ts = topo_stride(d3);
    t->d = d; t->d3 = d3; t->bits = bits; t->leaf_size = leaf_size; t->max_level = max_level;
    t->n_points = n; t->has_normals = nrm != nullptr;

    // 1. root cube + validation
    const int nbb = (int)std::min<int64_t>(1024, (n + 2047) / 2048 > 0 ? (n + 2047) / 2048 : 1);
    float* params = tmp.alloc<float>(8);
    float* partial = tmp.alloc<float>((int64_t)nbb * 8);
    SBH_ALLOC_OK("allocating bbox buffers");
    SBH_TRY(launch_bbox(src, w, nrm, n, params, partial, nbb, s), "bbox kernel");
    float hp[8];
    SBH_TRY(hipMemcpyAsync(hp, params, 6 * sizeof(float), hipMemcpyDeviceToHost, s), "bbox copy");
    SBH_TRY(hipStreamSynchronize(s), "bbox sync");
    if (hp[5] != 0.0f) {
        *msg = "sbh_build: non-finite coordinate or normal, or weight not finite and > 0";
        return SBH_EINVAL;
    }
    t->lo[0] = hp[0]; t->lo[1] = hp[1]; t->lo[2] = hp[2];
    t->side = hp[3]; t->inv_side = hp[4];
    for (int l = 0; l < kMaxLevels; ++l) t->diam[l] = (float)(std::sqrt(3.0) * (double)t->side / std::pow((double)d, l));

    // 2-3. codes and sort
    uint64_t* keys = tmp.alloc<uint64_t>(n);
    uint32_t* vals = tmp.alloc<uint32_t>(n);
    uint64_t* keys2 = tmp.alloc<uint64_t>(n);
    uint32_t* vals2 = tmp.alloc<uint32_t>(n);
    uint32_t* hist = tmp.alloc<uint32_t>((int64_t)radix_sort_hist_size(n));
    const int64_t scan_cap = std::max<int64_t>((int64_t)radix_sort_hist_size(n), n * (int64_t)d3 / 2 + d3 * 4);
    uint32_t* stmp = tmp.alloc<uint32_t>((int64_t)scan_tmp_size(std::max<int64_t>(scan_cap, n)) + 8);
    SBH_ALLOC_OK("allocating sort buffers");
    SBH_TRY(launch_morton(src, n, params, keys, vals, s), "morton kernel");
    SBH_TRY(radix_sort_pairs(keys, vals, keys2, vals2, n, 0, 64, hist, stmp, s), "radix sort");

    // sorted points (owned by the tree)
    t->slab_bytes[0] = carve_bytes<float4>(n) * (nrm ? 2 : 1) + carve_bytes<uint32_t>(n) + carve_bytes<uint64_t>(n);
    SBH_TRY(dev_alloc(t->mem, &t->slab[0], t->slab_bytes[0], s), "allocating points");
    {
        Carver c{(char*)t->slab[0]};
        t->pts = c.take<float4>(n);
        if (nrm) t->pdip = c.take<float4>(n);
        t->perm = c.take<uint32_t>(n);
        t->codes = c.take<uint64_t>(n);
    }
    k_gather_points<<<nblk(n), 256, 0, s>>>(src, w, nrm, vals, n, t->pts, t->pdip);
    SBH_TRY(hipGetLastError(), "gather kernel");
    SBH_TRY(hipMemcpyAsync(t->perm, vals, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s), "perm copy");
    SBH_TRY(hipMemcpyAsync(t->codes, keys, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s), "codes copy");
    const uint64_t* codes = t->codes;

    // 4. levels
    std::vector<LevelBufs> lv;
    std::vector<uint32_t> blk_off;   // first block id of each level's internal nodes
    std::vector<int32_t> n_int_lv;
    LevelBufs root;
    root.n = 1;
    root.b = tmp.alloc<int32_t>(1); root.c = tmp.alloc<int32_t>(1); root.par = tmp.alloc<int32_t>(1);
    root.dig = tmp.alloc<int32_t>(1); root.pblk = tmp.alloc<int32_t>(1);
    root.first = tmp.alloc<int32_t>(1); root.nch = tmp.alloc<int32_t>(1);
    SBH_ALLOC_OK("allocating root");
    k_root_init<<<1, 64, 0, s>>>((int32_t)n, root.b, root.c, root.par, root.dig, root.pblk);
    SBH_TRY(hipGetLastError(), "root init kernel");
    lv.push_back(root);
    uint32_t* total = stmp;  // scan totals land here; scans use stmp+1.. as scratch
    uint32_t* scan_scratch = stmp + 1;
    std::vector<uint32_t*> cscan_lv;
    std::vector<uint32_t*> iscan_lv;
    int64_t n_blocks = 0;
    // btopo is built in per-level pieces, then concatenated
    std::vector<uint32_t*> btopo_lv;

    for (int level = 0;; ++level) {
        LevelBufs& L = lv[level];
        uint32_t* flags = tmp.alloc<uint32_t>(L.n);
        uint32_t* iscan = tmp.alloc<uint32_t>(L.n);
        SBH_ALLOC_OK("allocating level flags");
        k_level_flags<<<nblk(L.n), 256, 0, s>>>(L.c, L.n, level, leaf_size, max_level, flags, L.first, L.nch);
        SBH_TRY(hipGetLastError(), "level flags kernel");
        SBH_TRY(scan_exclusive_u32(flags, iscan, L.n, total, scan_scratch, s), "internal scan");
        uint32_t n_int = 0;
        SBH_TRY(hipMemcpyAsync(&n_int, total, 4, hipMemcpyDeviceToHost, s), "internal count copy");
        SBH_TRY(hipStreamSynchronize(s), "level sync");
        iscan_lv.push_back(iscan);
        blk_off.push_back((uint32_t)n_blocks);
        n_int_lv.push_back((int32_t)n_int);
        // base pointers of the previous level's blocks
        if (level > 0 && n_int_lv[level - 1] > 0) {
            // btopo_lv[level-1] is that level's own piece, indexed from 0
            k_set_base<<<nblk(n_int_lv[level - 1]), 256, 0, s>>>(cscan_lv[level - 1], n_int_lv[level - 1], d3, 0u,
                                                                 iscan, (uint32_t)n_blocks, btopo_lv[level - 1], ts);
            SBH_TRY(hipGetLastError(), "set base kernel");
        }
        if (n_int == 0) {
            btopo_lv.push_back(nullptr);
            cscan_lv.push_back(nullptr);
            break;
        }
        int32_t* imap = tmp.alloc<int32_t>(n_int);
        uint32_t* bt = tmp.alloc<uint32_t>((int64_t)n_int * ts);
        uint32_t* ccount = tmp.alloc<uint32_t>((int64_t)n_int * d3);
        int32_t* cbegin = tmp.alloc<int32_t>((int64_t)n_int * d3);
        uint32_t* cflag = tmp.alloc<uint32_t>((int64_t)n_int * d3);
        uint32_t* cscan = tmp.alloc<uint32_t>((int64_t)n_int * d3);
        SBH_ALLOC_OK("allocating level children");
        SBH_TRY(hipMemsetAsync(bt, 0, (size_t)n_int * ts * sizeof(uint32_t), s), "topo clear");
        k_internal_map<<<nblk(L.n), 256, 0, s>>>(flags, iscan, L.n, imap);
        SBH_TRY(hipGetLastError(), "internal map kernel");
        // each level writes its own piece of the topology array (block ids
        // relative to the level); the pieces are concatenated at the end
        k_children<<<nblk((int64_t)n_int * d3), 256, 0, s>>>(L.b, L.c, imap, (int)n_int, level, bits, d3, codes, 0u,
                                                             bt, ts, ccount, cbegin, cflag);
        SBH_TRY(hipGetLastError(), "children kernel");
        SBH_TRY(scan_exclusive_u32(cflag, cscan, (int64_t)n_int * d3, total, scan_scratch, s), "children scan");
        uint32_t n_next = 0;
        SBH_TRY(hipMemcpyAsync(&n_next, total, 4, hipMemcpyDeviceToHost, s), "children count copy");
        SBH_TRY(hipStreamSynchronize(s), "children sync");
        int32_t off_cur = 0;
        for (int l = 0; l < level; ++l) off_cur += lv[l].n;
        const int32_t off_next = off_cur + L.n;
        LevelBufs N;
        N.n = (int32_t)n_next;
        N.b = tmp.alloc<int32_t>(N.n); N.c = tmp.alloc<int32_t>(N.n); N.par = tmp.alloc<int32_t>(N.n);
        N.dig = tmp.alloc<int32_t>(N.n); N.pblk = tmp.alloc<int32_t>(N.n);
        N.first = tmp.alloc<int32_t>(N.n); N.nch = tmp.alloc<int32_t>(N.n);
        SBH_ALLOC_OK("allocating next level");
        k_emit<<<nblk((int64_t)n_int * d3), 256, 0, s>>>(ccount, cbegin, cscan, imap, (int)n_int, d3, off_cur,
                                                         off_next, (uint32_t)n_blocks, N.b, N.c, N.par, N.dig, N.pblk,
                                                         L.first, L.nch);
        SBH_TRY(hipGetLastError(), "emit kernel");
        btopo_lv.push_back(bt);
        cscan_lv.push_back(cscan);
        n_blocks += n_int;
        lv.push_back(N);
    }
    // a level whose nodes are all leaves ends the loop; trailing empty levels cannot occur
    const int n_levels = (int)lv.size();
    int64_t n_nodes = 0;
    for (auto& L : lv) n_nodes += L.n;
    t->n_nodes = n_nodes;
    t->n_blocks = n_blocks;
    t->depth = n_levels - 1;
    if (n_nodes >= (int64_t)1 << 31) {
        *msg = "sbh_build: tree too large";
        return SBH_EINVAL;
    }

    // concatenate level arrays into node arrays
    t->slab_bytes[1] =
        carve_bytes<int32_t>(n_nodes) * 7 + carve_bytes<float4>(n_nodes) * (nrm ? 2 : 1) + carve_bytes<float>(n_nodes);
    SBH_TRY(dev_alloc(t->mem, &t->slab[1], t->slab_bytes[1], s), "allocating nodes");
    {
        Carver c{(char*)t->slab[1]};
        t->nbegin = c.take<int32_t>(n_nodes);
        t->ncount = c.take<int32_t>(n_nodes);
        t->nlevel = c.take<int32_t>(n_nodes);
        t->ndigit = c.take<int32_t>(n_nodes);
        t->nparent = c.take<int32_t>(n_nodes);
        t->nfirst = c.take<int32_t>(n_nodes);
        t->nnchild = c.take<int32_t>(n_nodes);
        t->nagg = c.take<float4>(n_nodes);
        if (nrm) t->ndip = c.take<float4>(n_nodes);
        t->nspr = c.take<float>(n_nodes);
    }
    int32_t* npblk = tmp.alloc<int32_t>(n_nodes);
    SBH_ALLOC_OK("allocating parent blocks");
    if (n_levels > kLevelTab) {
        *msg = "sbh_build: too many levels";
        return SBH_EINVAL;
    }
    {
        LevelTab tab{};
        for (int l = 0; l < n_levels; ++l) {
            const LevelBufs& L = lv[l];
            tab.off[l + 1] = tab.off[l] + L.n;
            const int32_t* src[7] = {L.b, L.c, L.dig, L.par, L.first, L.nch, L.pblk};
            for (int a = 0; a < 7; ++a) tab.src[a][l] = src[a];
        }
        const NodeDst dst{{t->nbegin, t->ncount, t->ndigit, t->nparent, t->nfirst, t->nnchild, npblk, t->nlevel}};
        k_concat_levels<<<nblk(n_nodes), 256, 0, s>>>(tab, n_levels, dst);
        SBH_TRY(hipGetLastError(), "node concatenation kernel");
    }
    // block arrays
    const int64_t nbk = n_blocks > 0 ? n_blocks : 1;
    {
        const size_t bytes = carve_bytes<uint32_t>(nbk * ts) + carve_bytes<float4>(nbk * d3) * (nrm ? 2 : 1) +
                             carve_bytes<float>(nbk * d3) + (compress ? carve_bytes<uint2>(nbk * d3) : 0) +
                             (quadrupole ? carve_bytes<float4>(2 * nbk * d3) : 0);
        t->slab_bytes[2] = bytes;
        SBH_TRY(dev_alloc(t->mem, &t->slab[2], bytes, s), "allocating blocks");
        SBH_TRY(hipMemsetAsync(t->slab[2], 0, bytes, s), "blocks clear");
        Carver c{(char*)t->slab[2]};
        t->btopo = c.take<uint32_t>(nbk * ts);
        t->bagg = c.take<float4>(nbk * d3);
        t->bspr = c.take<float>(nbk * d3);
        if (nrm) t->bdip = c.take<float4>(nbk * d3);
        if (compress) t->bq = c.take<uint2>(nbk * d3);
        if (quadrupole) t->bquad = c.take<float4>(2 * nbk * d3);
    }
    if (n_blocks > 0) {   // a level's blocks follow the previous level's (blk_off)
        TopoTab tt{};
        for (int l = 0; l < n_levels; ++l) {
            const bool has = n_int_lv[l] > 0 && btopo_lv[l];
            tt.off[l + 1] = tt.off[l] + (has ? (int64_t)n_int_lv[l] * ts : 0);
            tt.src[l] = btopo_lv[l];
        }
        k_concat_topo<<<nblk(tt.off[n_levels]), 256, 0, s>>>(tt, n_levels, t->btopo);
        SBH_TRY(hipGetLastError(), "topology concatenation kernel");
    }
    // 5. aggregates bottom-up, then pack into the child blocks
    {
        std::vector<int64_t> off(n_levels + 1, 0);
        for (int l = 0; l < n_levels; ++l) off[l + 1] = off[l] + lv[l].n;
        double4* agg64 = tmp.alloc<double4>(n_nodes);
        double4* dip64 = nrm ? tmp.alloc<double4>(n_nodes) : nullptr;
        double* spr64 = tmp.alloc<double>(n_nodes);
        double* quad64 = quadrupole ? tmp.alloc<double>(6 * n_nodes) : nullptr;
        SBH_ALLOC_OK("allocating float64 aggregates");
        for (int l = n_levels - 1; l >= 0; --l) {
            k_aggregate<<<nblk(lv[l].n), 256, 0, s>>>((int32_t)off[l], lv[l].n, t->nbegin, t->ncount, t->nfirst,
                                                      t->nnchild, t->pts, t->pdip, agg64, dip64, spr64, t->nagg,
                                                      t->ndip, t->nspr, quad64);
            SBH_TRY(hipGetLastError(), "aggregate kernel");
        }
        if (quadrupole && n_nodes > 1) {
            k_pack_quad<<<nblk(n_nodes - 1), 256, 0, s>>>((int32_t)n_nodes, npblk, t->ndigit, quad64, t->bquad, d3);
            SBH_TRY(hipGetLastError(), "quadrupole pack kernel");
        }
        if (compress && n_nodes > 1) {   // compressed aggregates, top-down from the root's
            double4* qagg = tmp.alloc<double4>(n_nodes);
            SBH_ALLOC_OK("allocating decoded aggregates");
            k_compress_root<<<1, 1, 0, s>>>(agg64, qagg);
            SBH_TRY(hipGetLastError(), "compress kernel");
            for (int l = 1; l < n_levels; ++l) {
                const double sl = (double)t->side / std::pow((double)d, (double)l);
                k_compress<<<nblk(lv[l].n), 256, 0, s>>>((int32_t)off[l], lv[l].n, sl, t->nparent, npblk, t->ndigit,
                                                         agg64, qagg, t->bq, d3);
                SBH_TRY(hipGetLastError(), "compress kernel");
            }
        }
    }
    if (n_nodes > 1) {
        k_pack<<<nblk(n_nodes - 1), 256, 0, s>>>((int32_t)n_nodes, npblk, t->ndigit, t->nagg, t->ndip, t->nspr,
                                                 t->bagg, t->bdip, t->bspr, d3);
        SBH_TRY(hipGetLastError(), "pack kernel");
    }
    SBH_TRY(hipStreamSynchronize(s), "build sync");
    return SBH_OK;
#undef SBH_TRY
#undef SBH_ALLOC_OK
}

}  // namespace sbh
