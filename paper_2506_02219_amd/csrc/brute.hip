// Exact evaluation of Eq. (1), F(q_j) = sum_i m_i f(p_i, q_j), by tiling the
// sources through LDS (each workgroup stages a tile of sources once and every
// lane reuses it for its own queries).  The float64 variant computes every
// term and the sum in double and provides the reference values; the float32
// variants are the GPU brute-force comparator.
//
// The smooth-distance sum is accumulated relative to the nearest source seen
// so far (s = sum w exp(-alpha (r - rmin))), rescaling s when rmin drops, so
// that it neither underflows nor overflows; the result is
// rmin - log(s) / alpha.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sbh_internal.hpp"

namespace sbh {

constexpr int kBruteThreads = 256;

template <int K, typename R>
__device__ __forceinline__ void brute_accumulate(R px, R py, R pz, R w, R nx, R ny, R nz, R qx, R qy, R qz, R eps2,
                                                 R alpha, R& acc, R& rmin)
{
    const R dx = px - qx, dy = py - qy, dz = pz - qz;
    const R r2 = dx * dx + dy * dy + dz * dz;
    if constexpr (K == SBH_POTENTIAL) {
        acc += w / sqrt(r2 + eps2);
    } else if constexpr (K == SBH_WINDING) {
        if (r2 > R(0)) {
            const R r = sqrt(r2);
            acc += (nx * dx + ny * dy + nz * dz) / (R(4.0 * M_PI) * r2 * r);
        }
    } else {
        const R r = sqrt(r2);
        if (r < rmin) {
            acc = acc * exp(-alpha * (rmin - r)) + w;
            rmin = r;
        } else {
            acc += w * exp(-alpha * (r - rmin));
        }
    }
}

template <int K, typename R>
__global__ void __launch_bounds__(kBruteThreads) k_brute(const float* __restrict__ src, const float* __restrict__ w,
                                                         const float* __restrict__ nrm, int64_t n,
                                                         const float* __restrict__ queries, int64_t nq, R eps2,
                                                         R alpha, R* __restrict__ out)
{
    constexpr int NW = (K == SBH_WINDING) ? kBruteThreads : 1;
    __shared__ R sx[kBruteThreads], sy[kBruteThreads], sz[kBruteThreads], sw[kBruteThreads];
    __shared__ R snx[NW], sny[NW], snz[NW];
    const int64_t j = (int64_t)blockIdx.x * kBruteThreads + threadIdx.x;
    const bool valid = j < nq;
    R qx = 0, qy = 0, qz = 0;
    if (valid) {
        qx = queries[3 * j];
        qy = queries[3 * j + 1];
        qz = queries[3 * j + 2];
    }
    R total = 0, rmin = R(INFINITY);
    for (int64_t t0 = 0; t0 < n; t0 += kBruteThreads) {
        const int64_t i = t0 + threadIdx.x;
        if (i < n) {
            sx[threadIdx.x] = (R)src[3 * i];
            sy[threadIdx.x] = (R)src[3 * i + 1];
            sz[threadIdx.x] = (R)src[3 * i + 2];
            sw[threadIdx.x] = (R)w[i];
            if constexpr (K == SBH_WINDING) {
                snx[threadIdx.x] = (R)w[i] * (R)nrm[3 * i];
                sny[threadIdx.x] = (R)w[i] * (R)nrm[3 * i + 1];
                snz[threadIdx.x] = (R)w[i] * (R)nrm[3 * i + 2];
            }
        }
        __syncthreads();
        const int cnt = (int)((n - t0) < kBruteThreads ? (n - t0) : kBruteThreads);
        R acc = (K == SBH_SMOOTHDIST) ? total : R(0);
        for (int k = 0; k < cnt; ++k) {
            R nx = 0, ny = 0, nz = 0;
            if constexpr (K == SBH_WINDING) {
                nx = snx[k];
                ny = sny[k];
                nz = snz[k];
            }
            brute_accumulate<K, R>(sx[k], sy[k], sz[k], sw[k], nx, ny, nz, qx, qy, qz, eps2, alpha, acc, rmin);
        }
        if constexpr (K == SBH_SMOOTHDIST) total = acc;
        else total += acc;  // per-tile partial sums
        __syncthreads();
    }
    if (valid) {
        R v = total;
        if constexpr (K == SBH_SMOOTHDIST) v = rmin - log(total) / alpha;
        // a query with a non-finite coordinate has no defined value
        const bool fin = __builtin_isfinite(qx) && __builtin_isfinite(qy) && __builtin_isfinite(qz);
        out[j] = fin ? v : R(NAN);
    }
}

// The float32 comparator for the potential and the winding number: a tile of
// 256 sources staged in LDS as (x, y, z, w) (and w n for the dipoles), read
// back as one broadcast 16-byte load per source, and kQPL queries per lane, so
// that a workgroup streams the sources once for 256 kQPL queries and every LDS
// read feeds kQPL terms.  A term is three differences, the squared distance
// with eps^2 folded in (three fused multiply-adds), the hardware reciprocal
// square root and the weighted accumulation.
constexpr int kQPL = 4;

template <int K>
__global__ void __launch_bounds__(kBruteThreads) k_brute32(const float* __restrict__ src, const float* __restrict__ w,
                                                           const float* __restrict__ nrm, int64_t n,
                                                           const float* __restrict__ queries, int64_t nq, float eps2,
                                                           float* __restrict__ out)
{
    static_assert(K == SBH_POTENTIAL || K == SBH_WINDING, "the smooth distance keeps its rescaling kernel");
    __shared__ float4 sp[kBruteThreads];
    __shared__ float4 sd[K == SBH_WINDING ? kBruteThreads : 1];
    const int64_t j0 = (int64_t)blockIdx.x * (kBruteThreads * kQPL) + threadIdx.x;
    float qx[kQPL], qy[kQPL], qz[kQPL], total[kQPL];
#pragma unroll
    for (int u = 0; u < kQPL; ++u) {
        const int64_t j = j0 + (int64_t)u * kBruteThreads;
        const bool valid = j < nq;
        qx[u] = valid ? queries[3 * j] : 0.0f;
        qy[u] = valid ? queries[3 * j + 1] : 0.0f;
        qz[u] = valid ? queries[3 * j + 2] : 0.0f;
        total[u] = 0.0f;
    }
    for (int64_t t0 = 0; t0 < n; t0 += kBruteThreads) {
        const int64_t i = t0 + threadIdx.x;
        if (i < n) {
            const float wi = w[i];
            sp[threadIdx.x] = make_float4(src[3 * i], src[3 * i + 1], src[3 * i + 2], wi);
            if constexpr (K == SBH_WINDING)
                sd[threadIdx.x] = make_float4(wi * nrm[3 * i], wi * nrm[3 * i + 1], wi * nrm[3 * i + 2], 0.0f);
        }
        __syncthreads();
        const int cnt = (int)((n - t0) < kBruteThreads ? (n - t0) : kBruteThreads);
        float acc[kQPL];   // the tile's partial sums, added to the totals after the tile
#pragma unroll
        for (int u = 0; u < kQPL; ++u) acc[u] = 0.0f;
        for (int k = 0; k < cnt; ++k) {
            const float4 p = sp[k];
            float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
            if constexpr (K == SBH_WINDING) m = sd[k];
#pragma unroll
            for (int u = 0; u < kQPL; ++u) {
                const float dx = p.x - qx[u], dy = p.y - qy[u], dz = p.z - qz[u];
                if constexpr (K == SBH_POTENTIAL) {
                    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
                    acc[u] = fmaf(p.w, __builtin_amdgcn_rsqf(r2), acc[u]);
                } else {
                    // (n . d) / (4 pi |d|^3); a source at the query itself adds nothing
                    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    const float ir = __builtin_amdgcn_rsqf(r2);
                    const float v = fmaf(m.z, dz, fmaf(m.y, dy, m.x * dx)) * (ir * ir * ir);
                    acc[u] += r2 > 0.0f ? v : 0.0f;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kQPL; ++u) total[u] += acc[u];
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kQPL; ++u) {
        const int64_t j = j0 + (int64_t)u * kBruteThreads;
        if (j >= nq) continue;
        float v = total[u];
        if constexpr (K == SBH_WINDING) v *= (float)(1.0 / (4.0 * M_PI));
        // a query with a non-finite coordinate has no defined value
        const bool fin = __builtin_isfinite(qx[u]) && __builtin_isfinite(qy[u]) && __builtin_isfinite(qz[u]);
        out[j] = fin ? v : NAN;
    }
}

template <int K>
static hipError_t launch_brute_k(const float* src, const float* w, const float* nrm, int64_t n, const float* q,
                                 int64_t nq, float eps, float alpha, int fp64, void* out, hipStream_t s)
{
    const unsigned blocks = (unsigned)((nq + kBruteThreads - 1) / kBruteThreads);
    if (fp64) {
        k_brute<K, double><<<blocks, kBruteThreads, 0, s>>>(src, w, nrm, n, q, nq, (double)eps * (double)eps,
                                                            (double)alpha, (double*)out);
    } else if constexpr (K == SBH_SMOOTHDIST) {
        k_brute<K, float><<<blocks, kBruteThreads, 0, s>>>(src, w, nrm, n, q, nq, eps * eps, alpha, (float*)out);
    } else {
        const unsigned b32 = (unsigned)((nq + kBruteThreads * kQPL - 1) / (kBruteThreads * kQPL));
        k_brute32<K><<<b32, kBruteThreads, 0, s>>>(src, w, nrm, n, q, nq, eps * eps, (float*)out);
    }
    return hipGetLastError();
}

hipError_t launch_brute(const float* src, const float* w, const float* nrm, int64_t n, const float* queries,
                        int64_t nq, int kernel, float eps, float alpha, int fp64, void* out, hipStream_t s)
{
    if (kernel == SBH_POTENTIAL) return launch_brute_k<SBH_POTENTIAL>(src, w, nrm, n, queries, nq, eps, alpha, fp64, out, s);
    if (kernel == SBH_WINDING) return launch_brute_k<SBH_WINDING>(src, w, nrm, n, queries, nq, eps, alpha, fp64, out, s);
    return launch_brute_k<SBH_SMOOTHDIST>(src, w, nrm, n, queries, nq, eps, alpha, fp64, out, s);
}

}  // namespace sbh
