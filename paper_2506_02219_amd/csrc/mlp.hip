// Learned child proposal: an 8 -> 32 -> 32 -> 8 ReLU network on MFMA
// (v_mfma_f32_16x16x16f16: binary16 operands, float32 accumulation).
//
// The paper draws the path index uniformly and leaves importance sampling
// open (Section 3.3); Theorem 1 holds for any child distribution with
// q_c > 0.  At an internal node the network sees one feature per child slot,
// the log of the child's quadrupole score relative to its siblings,
//   score_c = m_c s_c^2 / (|p_c - q|^2 + s_c^2)^(3/2),  f_c = max(-1, ln(score_c / max score) / 16)
// (m_c weight, p_c centre of mass, s_c^2 second moment; f = -1 for an empty
// slot), and returns logits z = W3 h2 + b3 + 16 f.  The proposal is
//   pi_c = exp(z_c) / sum_c' exp(z_c')   over non-empty slots,
//   q_c  = (1 - 1/8) pi_c + (1/8) n_c / n_T,
// so an all-zero network samples in proportion to the scores (the "score"
// proposal, which also runs without the network) and every non-empty child
// keeps q_c >= n_c / (8 n_T).
//
// Parameters: float32 [1608] = W1[32][8] b1[32] W2[32][32] b2[32] W3[8][32]
// b3[8]; the kernels round the weight matrices to binary16 (nearest even).
//
// MFMA fragment layout (16x16x16, wave64): lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] (j = 0..3) and D[4(l/16)+i][l%16] (i = 0..3).  The
// network is evaluated transposed (weights as A, activations as B), so a
// layer's D fragment, after bias and ReLU, is already the next layer's B
// fragment: inference needs no LDS.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sbh_internal.hpp"

namespace sbh {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kOffW1 = 0, kOffB1 = 256, kOffW2 = 288, kOffB2 = 1312, kOffW3 = 1344, kOffB3 = 1600;
constexpr float kLambda = 0.125f;

__device__ __forceinline__ f4 mfma(h4 a, h4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }

// A-operand fragments of the three weight matrices and this lane's biases
struct MlpRegs {
    h4 w1[2];       // [t]: W1[16t + l%16][4(l/16) + j] (inputs >= 8 are 0)
    h4 w2[2][2];    // [t][kc]: W2[16t + l%16][16kc + 4(l/16) + j]
    h4 w3[2];       // [kc]: W3[l%16][16kc + 4(l/16) + j] (outputs >= 8 are 0)
    float b1[2][4], b2[2][4], b3[4];
};

// ---------------------------------------------------------------------------
// Per-lane weight fragments for inference
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mlp_load_regs(MlpRegs& R, const float* __restrict__ prm, int lane)
{
    const int r = lane & 15, q = (lane >> 4) * 4;
    for (int t = 0; t < 2; ++t) {
        h4 w;
        for (int j = 0; j < 4; ++j) w[j] = (q + j < 8) ? (_Float16)prm[kOffW1 + (16 * t + r) * 8 + q + j] : (_Float16)0.0f;
        R.w1[t] = w;
        for (int kc = 0; kc < 2; ++kc) {
            h4 v;
            for (int j = 0; j < 4; ++j) v[j] = (_Float16)prm[kOffW2 + (16 * t + r) * 32 + 16 * kc + q + j];
            R.w2[t][kc] = v;
        }
        h4 u;
        for (int j = 0; j < 4; ++j) u[j] = (r < 8) ? (_Float16)prm[kOffW3 + r * 32 + 16 * t + q + j] : (_Float16)0.0f;
        R.w3[t] = u;
        for (int i = 0; i < 4; ++i) {
            R.b1[t][i] = prm[kOffB1 + 16 * t + q + i];
            R.b2[t][i] = prm[kOffB2 + 16 * t + q + i];
        }
    }
    for (int i = 0; i < 4; ++i) R.b3[i] = (q + i < 8) ? prm[kOffB3 + q + i] : 0.0f;
}

__device__ __forceinline__ h4 bias_relu_h(f4 d, const float* b)
{
    h4 h;
    for (int i = 0; i < 4; ++i) {
        const float v = d[i] + b[i];
        h[i] = v > 0.0f ? (_Float16)v : (_Float16)0.0f;
    }
    return h;
}

// Logits z = W3 h2 + b3 + 16 f of every lane's own sample (features f[8]) for
// the whole wavefront: four groups of 16 samples, eight MFMAs each.  All 64
// lanes must be active.
__device__ __forceinline__ void mlp_forward_wave(const MlpRegs& R, const float f[8], float z[8], int lane)
{
    const int r = lane & 15, hi = lane >> 4;
    for (int g = 0; g < 4; ++g) {
        const int src = 16 * g + r;
        float v[8];
        for (int k = 0; k < 8; ++k) v[k] = __shfl(f[k], src, 64);
        h4 xb;
        for (int j = 0; j < 4; ++j) xb[j] = hi == 0 ? (_Float16)v[j] : hi == 1 ? (_Float16)v[4 + j] : (_Float16)0.0f;
        const f4 zero = {0.f, 0.f, 0.f, 0.f};
        const h4 h1a = bias_relu_h(mfma(R.w1[0], xb, zero), R.b1[0]);
        const h4 h1b = bias_relu_h(mfma(R.w1[1], xb, zero), R.b1[1]);
        const h4 h2a = bias_relu_h(mfma(R.w2[0][1], h1b, mfma(R.w2[0][0], h1a, zero)), R.b2[0]);
        const h4 h2b = bias_relu_h(mfma(R.w2[1][1], h1b, mfma(R.w2[1][0], h1a, zero)), R.b2[1]);
        f4 o = mfma(R.w3[1], h2b, mfma(R.w3[0], h2a, zero));
        for (int i = 0; i < 4; ++i) o[i] += R.b3[i];
        // lane r holds logits 0..3 and lane 16 + r logits 4..7 of sample 16 g + r
        float zl[4], zh[4];
        for (int i = 0; i < 4; ++i) {
            zl[i] = __shfl(o[i], r, 64);
            zh[i] = __shfl(o[i], 16 + r, 64);
        }
        if (hi == g) {
            for (int i = 0; i < 4; ++i) {
                z[i] = zl[i];
                z[4 + i] = zh[i];
            }
        }
    }
    for (int k = 0; k < 8; ++k) z[k] += 16.0f * f[k];   // the features pass straight to the logits
}

// Features of (internal node, query q) from the node's child block: the
// relative log quadrupole score of each slot, -1 for empty slots (and for
// every slot when all scores are 0).
__device__ __forceinline__ void score_features(const float4* __restrict__ ba, const float* __restrict__ bs,
                                               const uint32_t cnt[8], float qx, float qy, float qz, float f[8])
{
#pragma clang fp contract(off)
    float sc[8];
    float smax = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float4 a = ba[c];
        const float s2 = bs[c];
        const float dx = a.x - qx, dy = a.y - qy, dz = a.z - qz;
        const float x = norm2(dx, dy, dz) + s2;
        const float r = x > 0.0f ? __frsqrt_rn(x) : 0.0f;
        const float v = cnt[c] ? a.w * s2 * (r * r * r) : 0.0f;
        sc[c] = v;
        smax = fmaxf(smax, v);
    }
    const float inv = smax > 0.0f ? 1.0f / smax : 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        f[c] = sc[c] >= smax && smax > 0.0f ? 0.0f
             : sc[c] > 0.0f                 ? fmaxf(-1.0f, __logf(sc[c] * inv) * 0.0625f)
                                            : -1.0f;
}

// Proposal without the network (z = 16 f): softmax(16 f)_c is
// max(score_c / max score, e^-16) normalised over the non-empty slots, so no
// logarithm or exponential is needed.
__device__ __forceinline__ void score_probs(const float4* __restrict__ ba, const float* __restrict__ bs,
                                            const uint32_t cnt[8], uint32_t nT, float qx, float qy, float qz,
                                            float qv[8])
{
#pragma clang fp contract(off)
    float sc[8];
    float smax = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float4 a = ba[c];
        const float s2 = bs[c];
        const float dx = a.x - qx, dy = a.y - qy, dz = a.z - qz;
        const float x = norm2(dx, dy, dz) + s2;
        const float r = x > 0.0f ? __frsqrt_rn(x) : 0.0f;
        const float v = cnt[c] ? a.w * s2 * (r * r * r) : 0.0f;
        sc[c] = v;
        smax = fmaxf(smax, v);
    }
    const float inv = smax > 0.0f ? frcp(smax) : 0.0f;
    float tot = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        // a slot whose score is 0 has feature -1, i.e. the floor e^-16 (all slots when every score is 0)
        sc[c] = cnt[c] ? (smax > 0.0f ? fmaxf(sc[c] * inv, 1.12535175e-7f) : 1.0f) : 0.0f;
        tot += sc[c];
    }
    const float w = (1.0f - kLambda) * frcp(tot), fn = kLambda * frcp((float)nT);
#pragma unroll
    for (int c = 0; c < 8; ++c) qv[c] = cnt[c] ? sc[c] * w + (float)cnt[c] * fn : 0.0f;
}

// q_c for the eight slots from the logits and the slot counts; empty slots 0.
__device__ __forceinline__ void learned_probs(const float z[8], const uint32_t cnt[8], uint32_t nT, float qv[8])
{
    float zmax = -INFINITY;
    for (int c = 0; c < 8; ++c)
        if (cnt[c]) zmax = fmaxf(zmax, z[c]);
    float e[8], s = 0.0f;
    for (int c = 0; c < 8; ++c) {
        e[c] = cnt[c] ? __expf(z[c] - zmax) : 0.0f;
        s += e[c];
    }
    const float inv = 1.0f / s, fn = 1.0f / (float)nT;
    for (int c = 0; c < 8; ++c) qv[c] = cnt[c] ? (1.0f - kLambda) * e[c] * inv + kLambda * (float)cnt[c] * fn : 0.0f;
}

// ---------------------------------------------------------------------------
// Forward over rows of features (verification entry point)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ prm, const float* __restrict__ x,
                                                     int64_t n, float* __restrict__ z)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w0 = i - lane;
    if (w0 >= n) return;   // whole wavefront past the end
    MlpRegs R;
    mlp_load_regs(R, prm, lane);
    float f[8], o[8];
    for (int k = 0; k < 8; ++k) f[k] = i < n ? x[8 * i + k] : 0.0f;
    mlp_forward_wave(R, f, o, lane);
    if (i < n)
        for (int k = 0; k < 8; ++k) z[8 * i + k] = o[k];
}

// ---------------------------------------------------------------------------
// Training: forward + backward for 64 rows per wavefront (one wavefront per
// block), operand fragments staged through LDS.  Per-wave partial gradients
// are summed in a fixed order by k_mlp_reduce (deterministic).
// ---------------------------------------------------------------------------
// D(16x16) = A(16x16) * B(16x16) + C; A(m, k) at a[m*am + k*ak], B(k, n) at b[k*bk + n*bn]
__device__ __forceinline__ f4 mfma_lds(const _Float16* a, int am, int ak, const _Float16* b, int bk, int bn, f4 c)
{
    const int l = threadIdx.x & 63, r = l & 15, q = (l >> 4) * 4;
    h4 av, bv;
    for (int j = 0; j < 4; ++j) {
        av[j] = a[r * am + (q + j) * ak];
        bv[j] = b[(q + j) * bk + r * bn];
    }
    return mfma(av, bv, c);
}

struct TrainLds {
    _Float16 w1[32 * 16];   // W1 padded to 16 inputs
    _Float16 w2[32 * 32];
    _Float16 w3[16 * 32];   // W3 padded to 16 outputs
    _Float16 x[64 * 16], h1[64 * 32], h2[64 * 32], dz[64 * 16], dh2[64 * 32], dh1[64 * 32];
    float zf[64 * 16], dh2f[64 * 32], dh1f[64 * 32];
    float xf[64 * 8];   // float32 features (skip term)
};

constexpr int kGradStride = 1608 + 8;   // partial-gradient row: 1608 parameters, then the loss

// Rows [row_begin + 64 b, row_begin + 64 b + 64) for block b; rows >= n or
// with all counts 0 contribute nothing.  Sums (not means) over the rows:
// the deltas stay O(1) in binary16; k_mlp_reduce divides by the row count.
__global__ void __launch_bounds__(64) k_mlp_grad(const float* __restrict__ prm, const float* __restrict__ X,
                                                 const float* __restrict__ Tg, const float* __restrict__ Cn, int64_t n,
                                                 int64_t row_begin, int64_t rows, float* __restrict__ partial)
{
    __shared__ TrainLds S;
    const int l = threadIdx.x, r = l & 15, hi = l >> 4, q = hi * 4;
    for (int i = l; i < 32 * 16; i += 64) S.w1[i] = (i % 16) < 8 ? (_Float16)prm[kOffW1 + (i / 16) * 8 + (i % 16)] : (_Float16)0.0f;
    for (int i = l; i < 32 * 32; i += 64) S.w2[i] = (_Float16)prm[kOffW2 + i];
    for (int i = l; i < 16 * 32; i += 64) S.w3[i] = (i / 32) < 8 ? (_Float16)prm[kOffW3 + i] : (_Float16)0.0f;
    // this lane's row
    const int64_t rel = (int64_t)blockIdx.x * 64 + l;
    const int64_t row = row_begin + rel;
    bool valid = rel < rows && row < n;
    float tg[8], cn[8];
    float csum = 0.0f;
    for (int k = 0; k < 8; ++k) {
        tg[k] = valid ? Tg[8 * row + k] : 0.0f;
        cn[k] = valid ? Cn[8 * row + k] : 0.0f;
        csum += cn[k];
        const float xv = valid ? X[8 * row + k] : 0.0f;
        S.xf[l * 8 + k] = xv;
        S.x[l * 16 + k] = (_Float16)xv;
        S.x[l * 16 + 8 + k] = (_Float16)0.0f;
    }
    valid = valid && csum > 0.0f;
    __syncthreads();
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    // forward, group by group (same operands and accumulation order as inference)
    for (int g = 0; g < 4; ++g) {
        const int s0 = 16 * g;
        for (int t = 0; t < 2; ++t) {
            const f4 d = mfma_lds(S.w1 + 16 * t * 16, 16, 1, S.x + s0 * 16, 1, 16, zero);
            for (int i = 0; i < 4; ++i) {
                const float v = d[i] + prm[kOffB1 + 16 * t + q + i];
                S.h1[(s0 + r) * 32 + 16 * t + q + i] = v > 0.0f ? (_Float16)v : (_Float16)0.0f;
            }
        }
        __syncthreads();
        for (int t = 0; t < 2; ++t) {
            f4 d = mfma_lds(S.w2 + 16 * t * 32, 32, 1, S.h1 + s0 * 32, 1, 32, zero);
            d = mfma_lds(S.w2 + 16 * t * 32 + 16, 32, 1, S.h1 + s0 * 32 + 16, 1, 32, d);
            for (int i = 0; i < 4; ++i) {
                const float v = d[i] + prm[kOffB2 + 16 * t + q + i];
                S.h2[(s0 + r) * 32 + 16 * t + q + i] = v > 0.0f ? (_Float16)v : (_Float16)0.0f;
            }
        }
        __syncthreads();
        f4 o = mfma_lds(S.w3, 32, 1, S.h2 + s0 * 32, 1, 32, zero);
        o = mfma_lds(S.w3 + 16, 32, 1, S.h2 + s0 * 32 + 16, 1, 32, o);
        for (int i = 0; i < 4; ++i) {
            float v = 0.0f;
            if (q + i < 8) {
                v = o[i] + prm[kOffB3 + q + i];
                v = v + 16.0f * S.xf[(s0 + r) * 8 + q + i];
            }
            S.zf[(s0 + r) * 16 + q + i] = v;
        }
        __syncthreads();
    }
    // loss and dL/dz for this lane's row: soft cross-entropy against the softmax over non-empty slots
    float loss = 0.0f;
    {
        float zmax = -INFINITY;
        for (int c = 0; c < 8; ++c)
            if (cn[c] > 0.0f) zmax = fmaxf(zmax, S.zf[l * 16 + c]);
        float e[8], s = 0.0f;
        for (int c = 0; c < 8; ++c) {
            e[c] = cn[c] > 0.0f ? expf(S.zf[l * 16 + c] - zmax) : 0.0f;
            s += e[c];
        }
        for (int c = 0; c < 16; ++c) {
            float dz = 0.0f;
            if (c < 8 && valid && cn[c] > 0.0f) {
                const float pi = e[c] / s;
                if (tg[c] > 0.0f) loss -= tg[c] * logf(pi);
                dz = pi - tg[c];
            }
            S.zf[l * 16 + c] = dz;
            S.dz[l * 16 + c] = (_Float16)dz;
        }
    }
    __syncthreads();
    // back-propagate deltas, group by group
    for (int g = 0; g < 4; ++g) {
        const int s0 = 16 * g;
        for (int kt = 0; kt < 2; ++kt) {   // dH2^T = W3^T dZ^T, masked by H2 > 0
            const f4 d = mfma_lds(S.w3 + 16 * kt, 1, 32, S.dz + s0 * 16, 1, 16, zero);
            for (int i = 0; i < 4; ++i) {
                const int idx = (s0 + r) * 32 + 16 * kt + q + i;
                const float v = (float)S.h2[idx] > 0.0f ? d[i] : 0.0f;
                S.dh2f[idx] = v;
                S.dh2[idx] = (_Float16)v;
            }
        }
        __syncthreads();
        for (int kt = 0; kt < 2; ++kt) {   // dH1^T = W2^T dH2^T, masked by H1 > 0
            f4 d = mfma_lds(S.w2 + 16 * kt, 1, 32, S.dh2 + s0 * 32, 1, 32, zero);
            d = mfma_lds(S.w2 + 16 * 32 + 16 * kt, 1, 32, S.dh2 + s0 * 32 + 16, 1, 32, d);
            for (int i = 0; i < 4; ++i) {
                const int idx = (s0 + r) * 32 + 16 * kt + q + i;
                const float v = (float)S.h1[idx] > 0.0f ? d[i] : 0.0f;
                S.dh1f[idx] = v;
                S.dh1[idx] = (_Float16)v;
            }
        }
        __syncthreads();
    }
    // weight gradients: sums over the 64 rows (K = rows, 16 at a time)
    float* out = partial + (int64_t)blockIdx.x * kGradStride;
    for (int kt = 0; kt < 2; ++kt) {   // dW3[c][k] = sum_s dz[s][c] h2[s][k]
        f4 d = zero;
        for (int g = 0; g < 4; ++g) d = mfma_lds(S.dz + 16 * g * 16, 1, 16, S.h2 + 16 * g * 32 + 16 * kt, 32, 1, d);
        for (int i = 0; i < 4; ++i)
            if (q + i < 8) out[kOffW3 + (q + i) * 32 + 16 * kt + r] = d[i];
    }
    for (int nt = 0; nt < 2; ++nt)
        for (int kt = 0; kt < 2; ++kt) {   // dW2[n][k] = sum_s dh2[s][n] h1[s][k]
            f4 d = zero;
            for (int g = 0; g < 4; ++g)
                d = mfma_lds(S.dh2 + 16 * g * 32 + 16 * nt, 1, 32, S.h1 + 16 * g * 32 + 16 * kt, 32, 1, d);
            for (int i = 0; i < 4; ++i) out[kOffW2 + (16 * nt + q + i) * 32 + 16 * kt + r] = d[i];
        }
    for (int nt = 0; nt < 2; ++nt) {   // dW1[n][k] = sum_s dh1[s][n] x[s][k]
        f4 d = zero;
        for (int g = 0; g < 4; ++g) d = mfma_lds(S.dh1 + 16 * g * 32 + 16 * nt, 1, 32, S.x + 16 * g * 16, 16, 1, d);
        for (int i = 0; i < 4; ++i)
            if (r < 8) out[kOffW1 + (16 * nt + q + i) * 8 + r] = d[i];
    }
    // bias gradients from the float32 deltas, fixed order over rows
    if (l < 32) {
        float a1 = 0.0f, a2 = 0.0f;
        for (int s = 0; s < 64; ++s) {
            a1 += S.dh1f[s * 32 + l];
            a2 += S.dh2f[s * 32 + l];
        }
        out[kOffB1 + l] = a1;
        out[kOffB2 + l] = a2;
    } else if (l < 40) {
        float a3 = 0.0f;
        for (int s = 0; s < 64; ++s) a3 += S.zf[s * 16 + (l - 32)];
        out[kOffB3 + l - 32] = a3;
    }
    // loss of the block (fixed-order wave reduction)
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    const float nvalid = (float)__popcll(__ballot(valid));
    if (l == 0) {
        out[1608] = loss;
        out[1609] = nvalid;
    }
}

// Means over the rows that count, sums over blocks in a fixed order:
// grad[0..1607] gradient, grad[1608] loss, grad[1609] number of rows.  A
// workgroup takes 64 consecutive entries; its kReduceParts wavefronts each sum
// one run of consecutive blocks in block order, and the runs' sums are added
// in run order (independent loads in flight instead of one serial chain).
constexpr int kReduceParts = 8;
__global__ void __launch_bounds__(64 * kReduceParts) k_mlp_reduce(const float* __restrict__ partial, int nblocks,
                                                                  float* __restrict__ grad)
{
    __shared__ float ps[kReduceParts][64];
    __shared__ float pc[kReduceParts];
    const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + l;
    const int per = (nblocks + kReduceParts - 1) / kReduceParts;
    const int b0 = g * per, b1 = min(nblocks, b0 + per);
    float s = 0.0f, cnt = 0.0f;
    for (int b = b0; b < b1; ++b) {
        if (p <= 1609) s += partial[(int64_t)b * kGradStride + p];
        cnt += partial[(int64_t)b * kGradStride + 1609];
    }
    ps[g][l] = s;
    if (l == 0) pc[g] = cnt;
    __syncthreads();
    if (g == 0 && p <= 1609) {
        float t = ps[0][l], c = pc[0];
        for (int k = 1; k < kReduceParts; ++k) {
            t += ps[k][l];
            c += pc[k];
        }
        grad[p] = p == 1609 ? c : t / fmaxf(c, 1.0f);
    }
}

// Adam (Kingma and Ba): state m[1608], v[1608]
__global__ void k_mlp_adam(float* __restrict__ prm, float* __restrict__ state, const float* __restrict__ grad,
                           float lr, float bc1, float bc2, float* __restrict__ loss_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss_out) *loss_out = grad[1608];
    if (p >= 1608) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = grad[p];
    const float m = b1 * state[p] + (1.0f - b1) * g;
    const float v = b2 * state[1608 + p] + (1.0f - b2) * g * g;
    state[p] = m;
    state[1608 + p] = v;
    prm[p] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

// ---------------------------------------------------------------------------
// Training pairs: uniform paths from every subdomain on the Philox stream
// (query, slot, step/2, 0xFFFFFFFF); each internal node on a path is a row
// [query][slot][depth] with its features, child counts and the location of
// its children block for the target kernel.
// ---------------------------------------------------------------------------
__global__ void k_mlp_pairs(TreeView tv, const float* __restrict__ queries, int64_t nq, int lmax, uint32_t key0,
                            uint32_t key1, float* __restrict__ X, float* __restrict__ Cn, int4* __restrict__ loc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq * 8) return;
    const int64_t j = t / 8;
    const int slot = (int)(t % 8);
    const float qx = queries[3 * j], qy = queries[3 * j + 1], qz = queries[3 * j + 2];
    const uint32_t* rt = tv.btopo;
    const uint32_t n_a = tv.root_internal ? rt[slot] : 0u;
    uint32_t beginT = 0u;
    int32_t nint = 0;
    for (int c = 0; c < slot; ++c) {
        beginT += rt[c];
        nint += ((int)rt[c] > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
    }
    int32_t blk = (int32_t)rt[8] + nint;
    uint32_t nT = n_a;
    int level = 1;
    u32x4 rnd = {0u, 0u, 0u, 0u};
    for (int k = 0; k < lmax; ++k) {
        const int64_t row = (j * 8 + slot) * lmax + k;
        const bool internal = n_a > 0u && (int)nT > tv.leaf_size && level < tv.max_level;
        if (!internal) {
            for (int c = 0; c < 8; ++c) {
                X[8 * row + c] = 0.0f;
                Cn[8 * row + c] = 0.0f;
            }
            loc[row] = make_int4(-1, 0, 0, 0);
            nT = 0u;
            continue;
        }
        const uint32_t* bt = tv.btopo + (int64_t)blk * topo_stride(8);
        uint32_t cnt[8];
        for (int c = 0; c < 8; ++c) cnt[c] = bt[c];
        float f[8];
        score_features(tv.bagg + (int64_t)blk * 8, tv.bspr + (int64_t)blk * 8, cnt, qx, qy, qz, f);
        for (int c = 0; c < 8; ++c) {
            X[8 * row + c] = f[c];
            Cn[8 * row + c] = (float)cnt[c];
        }
        loc[row] = make_int4(blk, (int32_t)beginT, (int32_t)nT, level);
        if ((k & 1) == 0) rnd = philox4x32_10((uint32_t)j, (uint32_t)slot, (uint32_t)(k >> 1), 0xFFFFFFFFu, key0, key1);
        const uint32_t r = __umulhi((k & 1) ? rnd.z : rnd.x, nT);
        uint32_t pre = 0u, preC = 0u, nC = 0u;
        int32_t ni = 0, niC = 0;
        for (int c = 0; c < 8; ++c) {
            const bool hit = (r - pre) < cnt[c];
            preC = hit ? pre : preC;
            niC = hit ? ni : niC;
            nC = hit ? cnt[c] : nC;
            ni += ((int)cnt[c] > tv.leaf_size && level + 1 < tv.max_level) ? 1 : 0;
            pre += cnt[c];
        }
        beginT += preC;
        nT = nC;
        blk = (int32_t)bt[8] + niC;
        ++level;
    }
}

// float64 term of one source for the targets (no smooth-distance shift)
template <int K>
__device__ __forceinline__ double term64(float4 p, float4 dp, double qx, double qy, double qz, double eps2,
                                         double alpha)
{
    const double dx = (double)p.x - qx, dy = (double)p.y - qy, dz = (double)p.z - qz;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if constexpr (K == SBH_POTENTIAL) {
        return (double)p.w / sqrt(r2 + eps2);
    } else if constexpr (K == SBH_WINDING) {
        if (r2 == 0.0) return 0.0;
        return ((double)dp.x * dx + (double)dp.y * dy + (double)dp.z * dz) / (4.0 * M_PI * r2 * sqrt(r2));
    } else {
        return (double)p.w * exp(-alpha * sqrt(r2));
    }
}

// one block per row: per-slot exact sums over the node's points (float64),
// residual against the child's aggregate term, normalised
template <int K>
__global__ void __launch_bounds__(256) k_mlp_targets(TreeView tv, const float* __restrict__ queries, int lmax,
                                                     const int4* __restrict__ loc, double eps2, double alpha,
                                                     float* __restrict__ Tg)
{
    const int64_t row = blockIdx.x;
    const int4 L = loc[row];
    if (L.x < 0) {
        if (threadIdx.x < 8) Tg[8 * row + threadIdx.x] = 0.0f;
        return;
    }
    const int64_t j = row / (8 * lmax);
    const double qx = queries[3 * j], qy = queries[3 * j + 1], qz = queries[3 * j + 2];
    const uint32_t* bt = tv.btopo + (int64_t)L.x * topo_stride(8);
    uint32_t bound[9];
    bound[0] = 0u;
    for (int c = 0; c < 8; ++c) bound[c + 1] = bound[c] + bt[c];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    for (uint32_t i = threadIdx.x; i < (uint32_t)L.z; i += blockDim.x) {
        const float4 p = tv.pts[L.y + i];
        const float4 dp = (K == SBH_WINDING) ? tv.pdip[L.y + i] : zero4;
        const double v = term64<K>(p, dp, qx, qy, qz, eps2, alpha);
        for (int c = 0; c < 8; ++c)
            if (i >= bound[c] && i < bound[c + 1]) acc[c] += v;
    }
    __shared__ double red[8][256];
    for (int c = 0; c < 8; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < 8; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double rr[8], rs = 0.0;
        for (int c = 0; c < 8; ++c) {
            rr[c] = 0.0;
            if (bt[c] == 0u) continue;
            const float4 a = tv.bagg[(int64_t)L.x * 8 + c];
            const float4 d = (K == SBH_WINDING) ? tv.bdip[(int64_t)L.x * 8 + c] : zero4;
            rr[c] = fabs(red[c][0] - term64<K>(a, d, qx, qy, qz, eps2, alpha));
            rs += rr[c];
        }
        for (int c = 0; c < 8; ++c)
            Tg[8 * row + c] = rs > 0.0 ? (float)(rr[c] / rs) : (float)bt[c] / (float)L.z;
    }
}

// ---------------------------------------------------------------------------
// Estimator with the learned (NET) or score proposal (d = 2).  Lanes as in
// the per-query kernel (8 queries x 8 subdomain slots per wavefront, every
// lane its own path); the walk is a wavefront-uniform loop so that the
// network runs on MFMA for all 64 lanes at once, every step at which some
// lane stands on an internal node.  At an internal node the child block is
// scanned first (its terms give the swap, its aggregates the features), then
// a slot is drawn by inverse CDF from q_c with a 24-bit uniform, then the
// roulette of Eq. (5); at a leaf a point is drawn uniformly.  The swap of a
// step is weighted by 1 / (prod q * prod p) (Eq. (7) with p(I in T) the
// product of the selection probabilities).
// ---------------------------------------------------------------------------
struct LearnArgs {
    int32_t samples;
    int32_t group;
    int32_t rr_mode;
    uint32_t batch;
    uint32_t key0, key1;
    float eps2, alpha;
    int32_t* paths;
    const float* prm;
};

template <int K, bool TRACE, bool NET>
__global__ void __launch_bounds__(256) k_sbh_learned(TreeView tv, const float* __restrict__ queries, int64_t nq,
                                                     LearnArgs a, float* __restrict__ out)
{
#pragma clang fp contract(off)
    constexpr int D3 = 8;
    constexpr int TS = topo_stride(D3);
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int lane = threadIdx.x & 63;
    const int slot = lane & 7;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t j = wave * 8 + (lane >> 3);
    if (wave * 8 >= nq) return;   // whole wavefront past the end
    const bool valid = j < nq;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (valid) {
        qx = queries[3 * j];
        qy = queries[3 * j + 1];
        qz = queries[3 * j + 2];
    }
    MlpRegs R;
    bool net = NET;
    if constexpr (NET) {
        // parameters that are not all finite are ignored (the zero network: the score proposal)
        bool bad = false;
        for (int i = lane; i < kMlpParams; i += 64) bad |= !__builtin_isfinite(a.prm[i]);
        net = __ballot(bad) == 0ull;
        mlp_load_regs(R, a.prm, lane);
    }
    KParams kp{a.eps2, a.alpha, 1.0f};
    float logwbar = 0.f, r0 = 0.f;
    if constexpr (K == SBH_SMOOTHDIST) {
        const float wbar = tv.nagg[0].w / (float)tv.n_points;
        kp.wscale = 1.0f / wbar;
        logwbar = logf(wbar);
        r0 = smooth_shift<2>(tv, qx, qy, qz, a.alpha);
    }
    const uint32_t* __restrict__ rt = tv.btopo;
    const uint32_t n_a = valid ? rt[slot] : 0u;
    uint32_t begin_a = 0u;
    int32_t nint_a = 0;
    for (int c = 0; c < slot; ++c) {
        begin_a += rt[c];
        nint_a += ((int)rt[c] > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
    }
    const int32_t blk_a = (int32_t)rt[D3] + nint_a;
    const float4 agg_a = tv.bagg[slot];
    float4 dip_a = zero4;
    if (tv.bdip) dip_a = tv.bdip[slot];
    const float cv = n_a ? term<K>(agg_a, (K == SBH_WINDING) ? dip_a : zero4, qx, qy, qz, kp, r0) : 0.0f;
    const uint32_t stream = (uint32_t)(a.group == 1 ? j : j / a.group);
    float fa = 0.0f;
    u32x4 rnd = {0u, 0u, 0u, 0u};
    for (int s = 0; s < a.samples; ++s) {
        bool act = n_a > 0u;
        uint32_t nT = n_a, beginT = begin_a;
        int32_t blk = blk_a;
        int level = 1;
        float diamT = tv.diam0 * 0.5f;
        float4 aggT = agg_a;
        float dT = fsqrt(norm2(agg_a.x - qx, agg_a.y - qy, agg_a.z - qz));   // |com_T - q|, carried step to step
        float tT = cv, prr = 1.0f, psel = 1.0f, acc = 0.0f;
        int steps = 0, flag = 0;
        int32_t end_b = (int32_t)beginT, end_l = level;
        const uint32_t ctr1 = (uint32_t)(slot * a.samples + s);
        for (int k = 0;; ++k) {
            if (act && nT == 1u) {
                flag = 1;
                end_b = (int32_t)beginT;
                end_l = level;
                act = false;
            }
            if (__ballot(act) == 0ull) break;
            if (act && (k & 1) == 0) rnd = philox4x32_10(stream, ctr1, (uint32_t)(k >> 1), a.batch, a.key0, a.key1);
            const uint32_t xsel = (k & 1) ? rnd.z : rnd.x;
            const uint32_t xrr = (k & 1) ? rnd.w : rnd.y;
            const bool internal = act && (int)nT > tv.leaf_size && level < tv.max_level;
            const float4* __restrict__ ba = tv.bagg + (int64_t)blk * D3;
            const uint32_t* __restrict__ bt = tv.btopo + (int64_t)blk * TS;
            uint32_t cnt[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
            float tv8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float sumc = 0.0f;
            if (internal) {
                // the child block: terms for the swap, scores for the proposal
                const float4* __restrict__ bd = tv.bdip + (int64_t)blk * D3;
#pragma unroll
                for (int c = 0; c < D3; ++c) {
                    cnt[c] = bt[c];
                    const float4 gd = (K == SBH_WINDING) ? bd[c] : zero4;
                    const float v = term<K>(ba[c], gd, qx, qy, qz, kp, r0);
                    tv8[c] = cnt[c] ? v : 0.0f;
                    sumc += tv8[c];
                }
                if constexpr (NET) score_features(ba, tv.bspr + (int64_t)blk * D3, cnt, qx, qy, qz, f);
            }
            float z[8];
            if constexpr (NET) {
                if (net) {
                    if (__ballot(internal) != 0ull) mlp_forward_wave(R, f, z, lane);
                } else {
#pragma unroll
                    for (int c = 0; c < 8; ++c) z[c] = 16.0f * f[c];
                }
            }
            if (!act) continue;
            float4 aggC;
            uint32_t nC = 1u, beginC;
            int32_t blkC = 0;
            int csel = 0;
            float qsel, tC = 0.0f;
            if (internal) {
                float qv[8];
                if constexpr (NET) learned_probs(z, cnt, nT, qv);
                else score_probs(ba, tv.bspr + (int64_t)blk * D3, cnt, nT, qx, qy, qz, qv);
                const float u_sel = (float)(xsel >> 8) * 5.9604644775390625e-8f;
                // first slot whose running sum exceeds u; rounding can leave the
                // total just below u, then the last non-empty slot is taken
                float cum = 0.0f;
                uint32_t pre = 0u, preC = 0u, preL = 0u, nL = 0u;
                int32_t ni = 0, niC = 0, niL = 0;
                int last = 0;
                float qL = 0.0f, tL = 0.0f;
                bool found = false;
                nC = 0u;
                qsel = 0.0f;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const bool ne = cnt[c] != 0u;
                    last = ne ? c : last;
                    preL = ne ? pre : preL;
                    niL = ne ? ni : niL;
                    nL = ne ? cnt[c] : nL;
                    qL = ne ? qv[c] : qL;
                    tL = ne ? tv8[c] : tL;
                    cum += qv[c];
                    const bool hit = !found && ne && u_sel < cum;
                    csel = hit ? c : csel;
                    preC = hit ? pre : preC;
                    niC = hit ? ni : niC;
                    nC = hit ? cnt[c] : nC;
                    qsel = hit ? qv[c] : qsel;
                    tC = hit ? tv8[c] : tC;
                    found = found || hit;
                    ni += ((int)cnt[c] > tv.leaf_size && level + 1 < tv.max_level) ? 1 : 0;
                    pre += cnt[c];
                }
                if (!found) {
                    csel = last;
                    preC = preL;
                    niC = niL;
                    nC = nL;
                    qsel = qL;
                    tC = tL;
                }
                aggC = ba[csel];
                beginC = beginT + preC;
                blkC = (int32_t)bt[D3] + niC;
            } else {
                const uint32_t r = __umulhi(xsel, nT);
                aggC = tv.pts[beginT + r];
                beginC = beginT + r;
                csel = (int)r;
                qsel = 1.0f / (float)nT;
            }
            float p, dC = 0.0f;
            if (a.rr_mode == 0) {
                const float cx = aggC.x - qx, cy = aggC.y - qy, cz = aggC.z - qz;
                dC = fsqrt(norm2(cx, cy, cz));
                p = fminf(1.0f, fmaxf(diamT, dT) * frcp(2.0f * dC));
            } else {
                p = a.rr_mode == 1 ? 1.0f : 0.5f;
            }
            const float u = (float)(xrr >> 8) * 5.9604644775390625e-8f;
            if (u >= p) {
                flag = 0;
                end_b = (int32_t)beginT;
                end_l = level;
                act = false;
                continue;
            }
            if (!internal) {   // leaf: its points are the virtual children
                for (uint32_t i = 0; i < nT; ++i) {
                    const float4 g = tv.pts[beginT + i];
                    const float4 gd = (K == SBH_WINDING) ? tv.pdip[beginT + i] : zero4;
                    sumc = term_acc<K>(g, gd, qx, qy, qz, kp, r0, sumc);
                }
            }
            prr *= p;
            acc += (sumc - tT) * frcp(psel * prr);
            psel *= qsel;
            ++steps;
            if (!internal) {
                flag = 2;
                end_b = (int32_t)beginC;
                end_l = level + 1;
                act = false;
                continue;
            }
            aggT = aggC;
            dT = dC;
            tT = tC;
            nT = nC;
            beginT = beginC;
            blk = blkC;
            ++level;
            diamT *= 0.5f;
        }
        if constexpr (TRACE) {
            if (valid)
                reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)a.samples + s] =
                    n_a ? make_int4(end_b, end_l, steps, flag) : make_int4(-1, 0, 0, 0);
        }
        fa += acc;
    }
    float val = n_a ? cv + fa / (float)a.samples : 0.0f;
#pragma unroll
    for (int o = 1; o < D3; o <<= 1) val += __shfl_xor(val, o);
    if (valid && slot == 0) out[j] = query_value<K>(val, r0, logwbar, a.alpha, qx, qy, qz);
}

// The same estimator with lane refill: a wavefront owns a pool of kLearnPool
// paths (Q queries x 8 subdomains x S samples); a lane whose path has ended
// takes the next one, handed out in lane order, so lanes do not idle while
// the wavefront's longest path finishes.  The network still runs once per
// step for all 64 lanes.  Every path's sum is stored at its own place in LDS,
// and each query adds CV_a + F_a / S over its subdomains in slot order at the
// end.  The step is the one above, operation for operation.
constexpr int kLearnPool = 256;

template <int K, bool TRACE, bool NET>
__global__ void __launch_bounds__(256) k_sbh_learned_pool(TreeView tv, const float* __restrict__ queries, int64_t nq,
                                                          LearnArgs a, float* __restrict__ out)
{
#pragma clang fp contract(off)
    constexpr int D3 = 8;
    constexpr int TS = topo_stride(D3);
    __shared__ float res[4][kLearnPool];
    __shared__ float cvs[4][kLearnPool];
    __shared__ uint32_t tab[4][D3][3];
    __shared__ float4 root_agg[D3];
    __shared__ float4 root_dip[K == SBH_WINDING ? D3 : 1];
    __shared__ float qpos[4][kLearnPool / D3 * 3];
    __shared__ float qr0[K == SBH_SMOOTHDIST ? 4 : 1][kLearnPool / D3];   // the queries' smooth-distance shifts
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int S = a.samples;
    const int Q = kLearnPool / (D3 * S);   // the launcher keeps 8 S <= kLearnPool
    const int NP = Q * D3 * S;
    const int64_t q0 = ((int64_t)blockIdx.x * 4 + wv) * Q;
    for (int c = threadIdx.x; c < D3; c += 256) {   // before the block's waves part: all reach the barrier
        root_agg[c] = tv.bagg[c];
        if constexpr (K == SBH_WINDING) root_dip[c] = tv.bdip[c];
    }
    __syncthreads();
    if (q0 >= nq) return;
    MlpRegs R;
    bool net = NET;
    if constexpr (NET) {
        // parameters that are not all finite are ignored (the zero network: the score proposal)
        bool bad = false;
        for (int i = lane; i < kMlpParams; i += 64) bad |= !__builtin_isfinite(a.prm[i]);
        net = __ballot(bad) == 0ull;
        mlp_load_regs(R, a.prm, lane);
    }
    KParams kp{a.eps2, a.alpha, 1.0f};
    float logwbar = 0.f;
    if constexpr (K == SBH_SMOOTHDIST) {
        const float wbar = tv.nagg[0].w / (float)tv.n_points;
        kp.wscale = 1.0f / wbar;
        logwbar = logf(wbar);
    }
    {   // the root block's subdomains and the wavefront's queries, once per wavefront
        const uint32_t* __restrict__ rt = tv.btopo;
        const int32_t base = (int32_t)rt[D3];
        uint32_t begin = 0u;
        int32_t nint = 0;
        for (int c = 0; c < D3; ++c) {
            const uint32_t n = rt[c];
            if (lane == 0) {
                tab[wv][c][0] = n;
                tab[wv][c][1] = begin;
                tab[wv][c][2] = (uint32_t)(base + nint);
            }
            begin += n;
            nint += ((int)n > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
        }
        for (int i = lane; i < 3 * Q; i += 64) qpos[wv][i] = q0 * 3 + i < 3 * nq ? queries[3 * q0 + i] : 0.0f;
        if constexpr (K == SBH_SMOOTHDIST) {
            if (lane < Q) {
                const int64_t jq = q0 + lane;
                qr0[wv][lane] = jq < nq ? smooth_shift<2>(tv, queries[3 * jq], queries[3 * jq + 1], queries[3 * jq + 2],
                                                          a.alpha)
                                        : 0.0f;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    int p = lane, slot = 0, smp = 0, k = 0, level = 1, steps = 0, flag = 0;
    int64_t j = 0;
    float qx = 0.f, qy = 0.f, qz = 0.f, r0 = 0.f;
    uint32_t nT = 0u, beginT = 0u, stream = 0u, ctr1 = 0u;
    int32_t blk = 0, end_b = 0, end_l = 1;
    float diamT = 0.f, dT = 0.f, tT = 0.f, prr = 1.f, psel = 1.f, acc = 0.f;
    u32x4 rnd = {0u, 0u, 0u, 0u};
    bool open = false;   // a path with points is being walked
    auto start = [&](int np) {
        p = np;
        open = false;
        if (p >= NP) {
            p = -1;
            return;
        }
        const int qi = p / (D3 * S), rem = p % (D3 * S);
        slot = rem / S;
        smp = rem % S;
        j = q0 + qi;
        acc = 0.0f;
        if (j >= nq) return;   // past the end of the query set: an empty path
        qx = qpos[wv][3 * qi];
        qy = qpos[wv][3 * qi + 1];
        qz = qpos[wv][3 * qi + 2];
        if constexpr (K == SBH_SMOOTHDIST) r0 = qr0[wv][qi];
        const uint32_t n_a = tab[wv][slot][0];
        if (n_a == 0u) {   // empty subdomain
            if constexpr (TRACE) reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)S + smp] = make_int4(-1, 0, 0, 0);
            return;
        }
        const float4 agg_a = root_agg[slot];
        const float cv = term<K>(agg_a, (K == SBH_WINDING) ? root_dip[slot] : zero4, qx, qy, qz, kp, r0);
        if (smp == 0) cvs[wv][p / S] = cv;
        nT = n_a;
        beginT = tab[wv][slot][1];
        blk = (int32_t)tab[wv][slot][2];
        level = 1;
        diamT = tv.diam0 * 0.5f;
        dT = fsqrt(norm2(agg_a.x - qx, agg_a.y - qy, agg_a.z - qz));
        tT = cv;
        prr = 1.0f;
        psel = 1.0f;
        steps = 0;
        flag = 0;
        k = 0;
        stream = (uint32_t)(a.group == 1 ? j : j / a.group);
        ctr1 = (uint32_t)(slot * S + smp);
        end_b = (int32_t)beginT;
        end_l = level;
        open = true;
    };
    start(lane);
    int next = 64;   // the next path of the pool to hand out
    while (__ballot(p >= 0) != 0ull) {
        bool done = p >= 0 && !open;   // an empty path ends at once
        bool internal = false;
        uint32_t xsel = 0u, xrr = 0u;
        const float4* __restrict__ ba = tv.bagg + (int64_t)blk * D3;
        const uint32_t* __restrict__ bt = tv.btopo + (int64_t)blk * TS;
        uint32_t cnt[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        float tv8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float sumc = 0.0f;
        if (open) {
            if (nT == 1u) {
                flag = 1;
                end_b = (int32_t)beginT;
                end_l = level;
                done = true;
            } else {
                if ((k & 1) == 0) rnd = philox4x32_10(stream, ctr1, (uint32_t)(k >> 1), a.batch, a.key0, a.key1);
                xsel = (k & 1) ? rnd.z : rnd.x;
                xrr = (k & 1) ? rnd.w : rnd.y;
                internal = (int)nT > tv.leaf_size && level < tv.max_level;
                if (internal) {
                    // the child block: terms for the swap, scores for the proposal
                    const float4* __restrict__ bd = tv.bdip + (int64_t)blk * D3;
#pragma unroll
                    for (int c = 0; c < D3; ++c) {
                        cnt[c] = bt[c];
                        const float4 gd = (K == SBH_WINDING) ? bd[c] : zero4;
                        const float v = term<K>(ba[c], gd, qx, qy, qz, kp, r0);
                        tv8[c] = cnt[c] ? v : 0.0f;
                        sumc += tv8[c];
                    }
                    if constexpr (NET) score_features(ba, tv.bspr + (int64_t)blk * D3, cnt, qx, qy, qz, f);
                }
            }
        }
        float z[8];
        if constexpr (NET) {
            if (net) {
                if (__ballot(internal) != 0ull) mlp_forward_wave(R, f, z, lane);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) z[c] = 16.0f * f[c];
            }
        }
        if (open && !done) {
            float4 aggC;
            uint32_t nC = 1u, beginC;
            int32_t blkC = 0;
            int csel = 0;
            float qsel, tC = 0.0f;
            if (internal) {
                float qv[8];
                if constexpr (NET) learned_probs(z, cnt, nT, qv);
                else score_probs(ba, tv.bspr + (int64_t)blk * D3, cnt, nT, qx, qy, qz, qv);
                const float u_sel = (float)(xsel >> 8) * 5.9604644775390625e-8f;
                // first slot whose running sum exceeds u; rounding can leave the
                // total just below u, then the last non-empty slot is taken
                float cum = 0.0f;
                uint32_t pre = 0u, preC = 0u, preL = 0u, nL = 0u;
                int32_t ni = 0, niC = 0, niL = 0;
                int last = 0;
                float qL = 0.0f, tL = 0.0f;
                bool found = false;
                nC = 0u;
                qsel = 0.0f;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const bool ne = cnt[c] != 0u;
                    last = ne ? c : last;
                    preL = ne ? pre : preL;
                    niL = ne ? ni : niL;
                    nL = ne ? cnt[c] : nL;
                    qL = ne ? qv[c] : qL;
                    tL = ne ? tv8[c] : tL;
                    cum += qv[c];
                    const bool hit = !found && ne && u_sel < cum;
                    csel = hit ? c : csel;
                    preC = hit ? pre : preC;
                    niC = hit ? ni : niC;
                    nC = hit ? cnt[c] : nC;
                    qsel = hit ? qv[c] : qsel;
                    tC = hit ? tv8[c] : tC;
                    found = found || hit;
                    ni += ((int)cnt[c] > tv.leaf_size && level + 1 < tv.max_level) ? 1 : 0;
                    pre += cnt[c];
                }
                if (!found) {
                    csel = last;
                    preC = preL;
                    niC = niL;
                    nC = nL;
                    qsel = qL;
                    tC = tL;
                }
                aggC = ba[csel];
                beginC = beginT + preC;
                blkC = (int32_t)bt[D3] + niC;
            } else {
                const uint32_t r = __umulhi(xsel, nT);
                aggC = tv.pts[beginT + r];
                beginC = beginT + r;
                qsel = 1.0f / (float)nT;
            }
            float pr, dC = 0.0f;
            if (a.rr_mode == 0) {
                const float cx = aggC.x - qx, cy = aggC.y - qy, cz = aggC.z - qz;
                dC = fsqrt(norm2(cx, cy, cz));
                pr = fminf(1.0f, fmaxf(diamT, dT) * frcp(2.0f * dC));
            } else {
                pr = a.rr_mode == 1 ? 1.0f : 0.5f;
            }
            const float u = (float)(xrr >> 8) * 5.9604644775390625e-8f;
            if (u >= pr) {
                flag = 0;
                end_b = (int32_t)beginT;
                end_l = level;
                done = true;
            } else {
                if (!internal) {   // leaf: its points are the virtual children
                    for (uint32_t i = 0; i < nT; ++i) {
                        const float4 g = tv.pts[beginT + i];
                        const float4 gd = (K == SBH_WINDING) ? tv.pdip[beginT + i] : zero4;
                        sumc = term_acc<K>(g, gd, qx, qy, qz, kp, r0, sumc);
                    }
                }
                prr *= pr;
                acc += (sumc - tT) * frcp(psel * prr);
                psel *= qsel;
                ++steps;
                if (!internal) {
                    flag = 2;
                    end_b = (int32_t)beginC;
                    end_l = level + 1;
                    done = true;
                } else {
                    dT = dC;
                    tT = tC;
                    nT = nC;
                    beginT = beginC;
                    blk = blkC;
                    ++level;
                    diamT *= 0.5f;
                    ++k;
                }
            }
        }
        if (done && open) {
            if constexpr (TRACE) reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)S + smp] = make_int4(end_b, end_l, steps, flag);
        }
        if (done) res[wv][p] = acc;
        // hand the next paths of the pool to the lanes that finished, in lane order
        const uint64_t fin = __ballot(done);
        if (fin != 0ull) {
            if (done) start(next + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(fin >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fin, 0u)));
            next += __popcll(fin);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // per query: the subdomain totals CV_a + F_a / S in slot order
    const int64_t jq = q0 + lane;
    if (lane < Q && jq < nq) {
        float val = 0.0f;
        for (int c = 0; c < D3; ++c) {
            if (tab[wv][c][0] == 0u) continue;
            float fa = 0.0f;
            for (int t = 0; t < S; ++t) fa += res[wv][(lane * D3 + c) * S + t];
            val += cvs[wv][lane * D3 + c] + fa / (float)S;
        }
        const float rq = (K == SBH_SMOOTHDIST) ? qr0[wv][lane] : 0.0f;
        out[jq] = query_value<K>(val, rq, logwbar, a.alpha, queries[3 * jq], queries[3 * jq + 1], queries[3 * jq + 2]);
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_mlp_forward(const float* prm, const float* x, int64_t n, float* z, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_mlp_forward<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(prm, x, n, z);
    return hipGetLastError();
}

size_t mlp_partial_floats(int64_t rows) { return (size_t)((rows + 63) / 64) * kGradStride; }

hipError_t launch_mlp_grad(const float* prm, const float* X, const float* Tg, const float* Cn, int64_t n,
                           int64_t row_begin, int64_t rows, float* partial, float* grad, hipStream_t s)
{
    const int nb = (int)((rows + 63) / 64);
    k_mlp_grad<<<nb, 64, 0, s>>>(prm, X, Tg, Cn, n, row_begin, rows, partial);
    k_mlp_reduce<<<(1610 + 63) / 64, 64 * kReduceParts, 0, s>>>(partial, nb, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* prm, float* state, const float* grad, float lr, int step, float* loss_out,
                           hipStream_t s)
{
    const float bc1 = 1.0f - powf(0.9f, (float)(step + 1));
    const float bc2 = 1.0f - powf(0.999f, (float)(step + 1));
    k_mlp_adam<<<(1608 + 255) / 256, 256, 0, s>>>(prm, state, grad, lr, bc1, bc2, loss_out);
    return hipGetLastError();
}

hipError_t launch_mlp_pairs(const sbh_tree_impl* t, const float* queries, int64_t nq, int lmax, uint64_t seed,
                            int kernel, float eps, float alpha, float* X, float* Tg, float* Cn, int4* loc,
                            hipStream_t s)
{
    const TreeView tv = make_view(t);
    k_mlp_pairs<<<(unsigned)((nq * 8 + 127) / 128), 128, 0, s>>>(tv, queries, nq, lmax, (uint32_t)seed,
                                                                   (uint32_t)(seed >> 32), X, Cn, loc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned rows = (unsigned)(nq * 8 * lmax);
    const double eps2 = (double)eps * (double)eps;
    if (kernel == SBH_POTENTIAL) k_mlp_targets<SBH_POTENTIAL><<<rows, 256, 0, s>>>(tv, queries, lmax, loc, eps2, alpha, Tg);
    else if (kernel == SBH_WINDING) k_mlp_targets<SBH_WINDING><<<rows, 256, 0, s>>>(tv, queries, lmax, loc, eps2, alpha, Tg);
    else k_mlp_targets<SBH_SMOOTHDIST><<<rows, 256, 0, s>>>(tv, queries, lmax, loc, eps2, alpha, Tg);
    return hipGetLastError();
}

}  // namespace sbh

namespace sbh {
hipError_t launch_sbh_learned(const sbh_tree_impl* t, const float* queries, int64_t nq, const EvalLaunch& e,
                              const float* prm, float* out, hipStream_t s)
{
    const TreeView tv = make_view(t);
    LearnArgs a{e.samples, e.group, e.rr_mode, e.batch, (uint32_t)e.seed, (uint32_t)(e.seed >> 32),
                e.eps * e.eps, e.alpha, e.paths, prm};
    // lane refill from a pool of paths per wavefront while 8 S <= kLearnPool (one path per lane beyond)
    const bool pool = 8 * (int64_t)e.samples <= kLearnPool;
    const int64_t qpw = pool ? kLearnPool / (8 * e.samples) : 8;
    const int64_t waves = (nq + qpw - 1) / qpw;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
#define SBH_LAUNCH_L(KK, NN)                                                                               \
    do {                                                                                                   \
        if (pool) {                                                                                        \
            if (e.paths) k_sbh_learned_pool<KK, true, NN><<<blocks, 256, 0, s>>>(tv, queries, nq, a, out);   \
            else k_sbh_learned_pool<KK, false, NN><<<blocks, 256, 0, s>>>(tv, queries, nq, a, out);          \
        } else {                                                                                           \
            if (e.paths) k_sbh_learned<KK, true, NN><<<blocks, 256, 0, s>>>(tv, queries, nq, a, out);        \
            else k_sbh_learned<KK, false, NN><<<blocks, 256, 0, s>>>(tv, queries, nq, a, out);               \
        }                                                                                                  \
    } while (0)
#define SBH_LAUNCH_K(NN)                                        \
    do {                                                        \
        if (e.kernel == SBH_POTENTIAL) SBH_LAUNCH_L(SBH_POTENTIAL, NN);    \
        else if (e.kernel == SBH_WINDING) SBH_LAUNCH_L(SBH_WINDING, NN);   \
        else SBH_LAUNCH_L(SBH_SMOOTHDIST, NN);                  \
    } while (0)
    if (prm) SBH_LAUNCH_K(true);
    else SBH_LAUNCH_K(false);
#undef SBH_LAUNCH_K
#undef SBH_LAUNCH_L
    return hipGetLastError();
}
}  // namespace sbh
