// Evaluation kernels on a built tree.
//
// k_sbh: the stratified path-sample estimator (Section 3.3, Eqs. (5)-(7),
// Section 3.3.1, Algorithm 2).  One lane owns one (query, subdomain) pair:
// with d = 2 a wavefront holds 8 queries x the 8 root-child slots, with d = 4
// one query x 64 slots.  A lane evaluates its control variate CV_a and its S
// path samples; the d^3 lanes of a query then add their subdomain totals in
// a fixed butterfly order, so the result does not depend on the launch.
//
// Per path step at node T (children block `blk`):
//   random words  Philox4x32-10(key = seed, ctr = (stream, slot*S+s, k/2,
//                 batch)); words (x, y) drive step k even, (z, w) step k odd;
//   selection     r = umulhi(word, n_T) in [0, n_T): the child whose point
//                 range holds offset r (probability n_c / n_T), i.e. the
//                 uniform path index of the paper drawn one level at a time;
//   roulette      p = min(1, max(1, b_T) / b_c) with b = |q - com| / |B| (Eq.
//                 (5)); since |B_c| = |B_T| / d this is
//                 min(1, max(|B_T|, |q - com_T|) / (d |q - com_c|));
//                 stop iff u >= p, u = (word >> 8) * 2^-24;
//   swap          Delta = sum_c f_c - f_T over the whole block (Eq. (6)),
//                 added with weight n_a / (n_T * prod p) (Eq. (7));
//   leaf          a leaf with several points uses its points as virtual
//                 children (|B| / d) and ends the path after one step.
//
// k_bh: Barnes-Hut (Eq. (2), Algorithm 1) with wavefront voting: a
// wavefront walks one depth-first traversal for its 64 queries; a child is
// opened when any lane's far-field test fails; leaves that are opened are
// summed exactly.  The traversal stack is wavefront-uniform and lives in LDS.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <type_traits>

#include <algorithm>

#include "sbh_internal.hpp"

namespace sbh {

struct SbhArgs {
    int32_t samples;
    int32_t group;
    int32_t rr_mode;
    uint32_t batch;
    uint32_t key0, key1;
    float eps2, alpha;
    int32_t* paths;
};

TreeView make_view(const sbh_tree_impl* t)
{
    TreeView v{};
    v.pts = t->pts;
    v.pdip = t->pdip;
    v.bagg = t->bagg;
    v.bdip = t->bdip;
    v.bspr = t->bspr;
    v.btopo = t->btopo;
    v.nagg = t->nagg;
    v.ndip = t->ndip;
    v.bq = t->bq;
    v.bquad = t->bquad;
    v.n_points = (int32_t)t->n_points;
    v.leaf_size = t->leaf_size;
    v.max_level = t->max_level;
    v.root_internal = (t->n_points > t->leaf_size && t->max_level > 0) ? 1 : 0;
    const uint64_t nbk = (uint64_t)(t->n_blocks > 0 ? t->n_blocks : 1);
    const uint64_t big = std::max({nbk * (uint64_t)t->d3 * (t->bquad ? 32u : 16u),
                                   nbk * (uint64_t)topo_stride(t->d3) * 4u, (uint64_t)t->n_points * 16u});
    // SBH_FORCE_WIDE_OFFSETS=1 takes the 64-bit offsets for any tree (a diagnostic:
    // both forms give the same values bit for bit)
    const char* force = std::getenv("SBH_FORCE_WIDE_OFFSETS");
    v.wide = (big >= ((uint64_t)1 << 32) || (force && force[0] == '1')) ? 1 : 0;
    v.lo[0] = t->lo[0]; v.lo[1] = t->lo[1]; v.lo[2] = t->lo[2];
    v.side = t->side;
    v.diam0 = t->diam[0];
    return v;
}

// Component-wise select (a select of whole float4 values can be lowered
// through private memory).
__device__ __forceinline__ float4 sel4(bool c, float4 a, float4 b)
{
    return make_float4(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z, c ? a.w : b.w);
}

// Smooth-distance scaling: terms are (w / wbar) exp(-alpha (r - r0)); the
// reported distance is r0 - (log(sum) + log(wbar)) / alpha.
__device__ __forceinline__ void smooth_setup(const TreeView& tv, float& wscale, float& logwbar)
{
    const float wbar = gld4(tv.nagg).w / (float)tv.n_points;
    wscale = 1.0f / wbar;
    logwbar = logf(wbar);
}

template <int D, int K, bool TRACE>
__device__ __forceinline__ float sample_path(const TreeView& tv, float qx, float qy, float qz, float r0,
                                             const KParams& kp, uint32_t n_a, uint32_t begin_a, int32_t blk_a,
                                             float4 agg_a, float t_a, uint32_t ctr0, uint32_t ctr1, uint32_t ctr3,
                                             uint32_t key0, uint32_t key1, int rr_mode, int4* rec)
{
#pragma clang fp contract(off)
    constexpr int D3 = D * D * D;
    constexpr int TS = topo_stride(D3);
    constexpr float kInvD = 1.0f / (float)D;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t nT = n_a, beginT = begin_a;
    int32_t blk = blk_a;
    int level = 1;
    float diamT = tv.diam0 * kInvD;
    float4 aggT = agg_a;
    float dT = fsqrt(norm2(agg_a.x - qx, agg_a.y - qy, agg_a.z - qz));   // |com_T - q|, carried step to step
    float tT = t_a;
    float prr = 1.0f;
    float acc = 0.0f;
    const float fna = (float)n_a;
    int steps = 0, flag = 0;
    int32_t end_b = (int32_t)beginT, end_l = level;
    u32x4 rnd = {0u, 0u, 0u, 0u};
    for (int k = 0;; ++k) {
        end_b = (int32_t)beginT;
        end_l = level;
        if (nT == 1u) {
            flag = 1;
            break;
        }
        if ((k & 1) == 0) rnd = philox4x32_10(ctr0, ctr1, (uint32_t)(k >> 1), ctr3, key0, key1);
        const uint32_t xsel = (k & 1) ? rnd.z : rnd.x;
        const uint32_t xrr = (k & 1) ? rnd.w : rnd.y;
        const uint32_t r = __umulhi(xsel, nT);
        const bool internal = (int)nT > tv.leaf_size && level < tv.max_level;
        const float4* __restrict__ ba = tv.bagg + (int64_t)blk * D3;
        const float4* __restrict__ bd = tv.bdip + (int64_t)blk * D3;
        const uint32_t* __restrict__ bt = tv.btopo + (int64_t)blk * TS;
        float4 aggC;
        uint32_t nC = 1u, beginC;
        int32_t blkC = 0;
        int csel = 0;
        if (internal) {
            // child selection from the point counts alone
            uint32_t pre = 0u, preC = 0u;
            int32_t nint = 0, nintC = 0;
#pragma unroll
            for (int c = 0; c < D3; ++c) {
                const uint32_t cnt = bt[c];
                const bool hit = (r - pre) < cnt;
                csel = hit ? c : csel;
                preC = hit ? pre : preC;
                nintC = hit ? nint : nintC;
                nC = hit ? cnt : nC;
                nint += ((int)cnt > tv.leaf_size && level + 1 < tv.max_level) ? 1 : 0;
                pre += cnt;
            }
            aggC = ba[csel];
            beginC = beginT + preC;
            blkC = (int32_t)bt[D3] + nintC;
        } else {
            aggC = tv.pts[beginT + r];
            beginC = beginT + r;
        }
        // roulette first (Eq. (5)); a lane that stops never reads the rest of the block
        float p;
        float dC = 0.0f;
        if (rr_mode == 0) {
            const float cx = aggC.x - qx, cy = aggC.y - qy, cz = aggC.z - qz;
            dC = fsqrt(norm2(cx, cy, cz));
            p = fminf(1.0f, fmaxf(diamT, dT) * frcp((float)D * dC));
        } else {
            p = rr_mode == 1 ? 1.0f : 0.5f;
        }
        const float u = (float)(xrr >> 8) * 5.9604644775390625e-8f;
        if (u >= p) {
            flag = 0;
            break;
        }
        // contribution swap, Eq. (6)
        float sumc = 0.0f, tC = 0.0f;
        if (internal) {
#pragma unroll
            for (int c = 0; c < D3; ++c) {
                const uint32_t cnt = bt[c];
                const float4 g = ba[c];
                const float4 gd = (K == SBH_WINDING) ? bd[c] : zero4;
                const float v = term<K>(g, gd, qx, qy, qz, kp, r0);
                const float vv = cnt ? v : 0.0f;
                sumc += vv;
                tC = (c == csel) ? vv : tC;
            }
        } else {
            for (uint32_t i = 0; i < nT; ++i) {
                const float4 g = tv.pts[beginT + i];
                const float4 gd = (K == SBH_WINDING) ? tv.pdip[beginT + i] : zero4;
                const float v = term<K>(g, gd, qx, qy, qz, kp, r0);
                sumc += v;
                tC = (i == r) ? v : tC;
            }
        }
        prr *= p;
        acc += (sumc - tT) * (fna * frcp((float)nT * prr));
        ++steps;
        if (!internal) {
            end_b = (int32_t)beginC;
            end_l = level + 1;
            flag = 2;
            break;
        }
        aggT = aggC;
        dT = dC;
        tT = tC;
        nT = nC;
        beginT = beginC;
        blk = blkC;
        ++level;
        diamT *= kInvD;
    }
    if constexpr (TRACE) *rec = make_int4(end_b, end_l, steps, flag);
    return acc;
}

template <int D, int K, bool TRACE>
__global__ void __launch_bounds__(256) k_sbh(TreeView tv, const float* __restrict__ queries, int64_t nq,
                                             SbhArgs a, float* __restrict__ out)
{
#pragma clang fp contract(off)
    constexpr int D3 = D * D * D;
    constexpr int QPW = 64 / D3;
    const int lane = threadIdx.x & 63;
    const int slot = lane % D3;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t j = wave * QPW + lane / D3;
    if (wave * QPW >= nq) return;  // whole wavefront past the end
    const bool valid = j < nq;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (valid) {
        qx = queries[3 * j];
        qy = queries[3 * j + 1];
        qz = queries[3 * j + 2];
    }
    KParams kp{a.eps2, a.alpha, 1.0f};
    float logwbar = 0.f, r0 = 0.f;
    if constexpr (K == SBH_SMOOTHDIST) {
        smooth_setup(tv, kp.wscale, logwbar);
        r0 = smooth_shift<D>(tv, qx, qy, qz, a.alpha);
    }
    const uint32_t* __restrict__ rt = tv.btopo;  // root block
    const uint32_t n_a = valid ? rt[slot] : 0u;
    float val = 0.0f;
    if (n_a > 0u) {
        uint32_t begin_a = 0u;
        int32_t nint = 0;
        for (int c = 0; c < slot; ++c) {
            const uint32_t cnt = rt[c];
            begin_a += cnt;
            nint += ((int)cnt > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
        }
        const int32_t blk_a = (int32_t)rt[D3] + nint;
        const float4 agg_a = tv.bagg[slot];
        const float4 dip_a = (K == SBH_WINDING) ? tv.bdip[slot] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float cv = term<K>(agg_a, dip_a, qx, qy, qz, kp, r0);  // control variate CV_a
        const uint32_t stream = (uint32_t)(a.group == 1 ? j : j / a.group);
        float fa = 0.0f;
        for (int s = 0; s < a.samples; ++s) {
            int4 rec;
            fa += sample_path<D, K, TRACE>(tv, qx, qy, qz, r0, kp, n_a, begin_a, blk_a, agg_a, cv, stream,
                                           (uint32_t)(slot * a.samples + s), a.batch, a.key0, a.key1, a.rr_mode,
                                           &rec);
            if constexpr (TRACE) {
                reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)a.samples + s] = rec;
            }
        }
        val = cv + fa / (float)a.samples;
    } else if (TRACE && valid) {
        for (int s = 0; s < a.samples; ++s)
            reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)a.samples + s] = make_int4(-1, 0, 0, 0);
    }
    // fixed-order butterfly over the d^3 lanes of this query (every lane ends
    // with the same bits because float addition is commutative)
#pragma unroll
    for (int o = 1; o < D3; o <<= 1) val += __shfl_xor(val, o);
    if (valid && slot == 0) out[j] = query_value<K>(val, r0, logwbar, a.alpha, qx, qy, qz);
}

// ---------------------------------------------------------------------------
// Per-lane estimator with lane refill.  Each lane walks its own path, so the
// paths of a wavefront end at different steps; instead of idling, a lane
// whose path has ended takes the next path of the wavefront's pool
// (kPoolPaths paths: Q queries x d^3 subdomains x S samples, handed out in
// lane order).  Every path's sum is stored at its own place in LDS, and once
// the pool is drained each query adds CV_a + F_a / S over its subdomains in
// slot order, so the result does not depend on which lane walked what.  The
// step is the one of sample_path, operation for operation.
// CMP (d = 2, potential and smooth distance): the walk on the compressed
// aggregates, each child decoded from its 8-byte code as in the coherent
// compressed walk (the lane carries its node's decoded offset from the query,
// its decoded mass and its children's cell side); a node of one point takes
// the leaf step.
// ---------------------------------------------------------------------------
constexpr int kPoolPaths = 256;

// The uniform variate of a 32-bit random word: its top 24 bits times 2^-24
// (exactly representable, in [0, 1)).
__device__ __forceinline__ float unit24(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-8f; }

// A compressed aggregate's field: the binary16 number in the low 16 bits, as a float.
__device__ __forceinline__ float h16(uint32_t bits) { return (float)__builtin_bit_cast(_Float16, (uint16_t)bits); }
typedef uint32_t sbh_u32x4v __attribute__((ext_vector_type(4)));
// 16 bytes (16-byte aligned): adjacent loads of a block merge into one wide scalar load
__device__ __forceinline__ sbh_u32x4v gld4u(const uint32_t* p) { return *(const SBH_GLOBAL sbh_u32x4v*)p; }

template <int D, int K, bool TRACE, bool CMP = false>
__global__ void __launch_bounds__(256) k_sbh_pool(TreeView tv, const float* __restrict__ queries, int64_t nq,
                                                  SbhArgs a, float* __restrict__ out)
{
#pragma clang fp contract(off)
    static_assert(!CMP || (D == 2 && K != SBH_WINDING), "compressed aggregates: d = 2, no dipoles");
    constexpr int D3 = D * D * D;
    constexpr bool KEEPN = D == 2;   // the block's counts are kept in registers (eight of them)
    constexpr int TS = topo_stride(D3);
    constexpr float kInvD = 1.0f / (float)D;
    __shared__ float res[4][kPoolPaths];   // per path: its sum F (before the division by S)
    __shared__ float cvs[4][kPoolPaths];   // per (query, subdomain): the control variate CV_a
    __shared__ uint32_t tab[4][D3][3];     // per subdomain: point count, first point, block id
    __shared__ float4 root_agg[D3];        // the subdomains' aggregates (and dipoles), for every path start
    __shared__ float4 root_dip[K == SBH_WINDING ? D3 : 1];
    __shared__ float qpos[4][kPoolPaths / 8 * 3];   // the wavefront's query positions (Q <= kPoolPaths / d^3)
    __shared__ float qr0[K == SBH_SMOOTHDIST ? 4 : 1][kPoolPaths / 8];   // their smooth-distance shifts
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int S = a.samples;
    const int Q = kPoolPaths / (D3 * S);   // queries per wavefront (the launcher keeps D^3 S <= kPoolPaths)
    const int NP = Q * D3 * S;
    const int64_t q0 = ((int64_t)blockIdx.x * 4 + wv) * Q;
    for (int c = threadIdx.x; c < D3; c += 256) {   // before the block's waves part: all reach the barrier
        if constexpr (CMP) {
            // a subdomain's decoded aggregate is q-independent except for its offset: keep the
            // root's float32 centre of mass with the slot's offset code (x, y, z: cell sides of
            // level 1) and its decoded mass
            const float4 g0 = gld4(tv.nagg);
            const uint32_t w0 = gld(reinterpret_cast<const uint32_t*>(tv.bq) + 2 * c);
            const uint32_t w1 = gld(reinterpret_cast<const uint32_t*>(tv.bq) + 2 * c + 1);
            root_agg[c] = make_float4(h16(w0 & 0xFFFFu), h16(w0 >> 16), h16(w1 & 0xFFFFu), g0.w * h16(w1 >> 16));
        } else {
            root_agg[c] = gld4(tv.bagg + c);
        }
        if constexpr (K == SBH_WINDING) root_dip[c] = gld4(tv.bdip + c);
    }
    __syncthreads();
    if (q0 >= nq) return;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    KParams kp{a.eps2, a.alpha, 1.0f};
    float logwbar = 0.f;
    if constexpr (K == SBH_SMOOTHDIST) smooth_setup(tv, kp.wscale, logwbar);
    {   // the root block's subdomains, once per wavefront
        const uint32_t* __restrict__ rt = tv.btopo;
        const int32_t base = (int32_t)gld(rt + D3);
        uint32_t begin = 0u;
        int32_t nint = 0;
        for (int c = 0; c < D3; ++c) {
            const uint32_t n = gld(rt + c);
            if (lane == 0) {
                tab[wv][c][0] = n;
                tab[wv][c][1] = begin;
                tab[wv][c][2] = (uint32_t)(base + nint);
            }
            begin += n;
            nint += ((int)n > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
        }
        for (int i = lane; i < 3 * Q; i += 64)   // the wavefront's queries (past the end: zero)
            qpos[wv][i] = q0 * 3 + i < 3 * nq ? gld(queries + 3 * q0 + i) : 0.0f;
        if constexpr (K == SBH_SMOOTHDIST) {
            if (lane < Q) {
                const int64_t jq = q0 + lane;
                qr0[wv][lane] = jq < nq ? smooth_shift<D>(tv, gld(queries + 3 * jq), gld(queries + 3 * jq + 1),
                                                          gld(queries + 3 * jq + 2), a.alpha)
                                        : 0.0f;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // lane state: the path (p < 0: none left) and its walk
    int p = lane, slot = 0, smp = 0, k = 0, level = 1, steps = 0, flag = 0;
    int64_t j = 0;
    float qx = 0.f, qy = 0.f, qz = 0.f, r0 = 0.f;
    uint32_t nT = 0u, beginT = 0u, ctr0 = 0u, ctr1 = 0u;
    int32_t blk = 0, end_b = 0, end_l = 1;
    float diamT = 0.f, dT = 0.f, tT = 0.f, prr = 1.f, acc = 0.f, fna = 0.f;
    float dTx = 0.f, dTy = 0.f, dTz = 0.f, mT = 0.f, sideC = 0.f;   // CMP: the node's decoded aggregate
    const float4 g0 = CMP ? gld4(tv.nagg) : zero4;                   // CMP: the root's
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
        const float4 dip_a = (K == SBH_WINDING) ? root_dip[slot] : zero4;
        float cv;
        if constexpr (CMP) {
            const float s1 = tv.side * 0.5f;
            dTx = fmaf(agg_a.x, s1, g0.x - qx);
            dTy = fmaf(agg_a.y, s1, g0.y - qy);
            dTz = fmaf(agg_a.z, s1, g0.z - qz);
            mT = agg_a.w;
            sideC = tv.side * 0.25f;
            cv = term_r2<K>(make_float4(0.f, 0.f, 0.f, mT), zero4, dTx, dTy, dTz, norm2(dTx, dTy, dTz), kp, r0);
        } else {
            cv = term<K>(agg_a, dip_a, qx, qy, qz, kp, r0);   // control variate CV_a
        }
        if (smp == 0) cvs[wv][p / S] = cv;
        nT = n_a;
        beginT = tab[wv][slot][1];
        blk = (int32_t)tab[wv][slot][2];
        level = 1;
        diamT = tv.diam0 * kInvD;
        dT = CMP ? fsqrt(norm2(dTx, dTy, dTz)) : fsqrt(norm2(agg_a.x - qx, agg_a.y - qy, agg_a.z - qz));
        tT = cv;
        prr = 1.0f;
        fna = (float)n_a;
        steps = 0;
        flag = 0;
        k = 0;
        ctr0 = (uint32_t)(a.group == 1 ? j : j / a.group);
        ctr1 = (uint32_t)(slot * S + smp);
        end_b = (int32_t)beginT;
        end_l = level;
        open = true;
    };
    start(lane);
    int next = 64;   // the next path of the pool to hand out
    while (__ballot(p >= 0) != 0ull) {
        bool done = p >= 0 && !open;   // an empty path ends at once
        if (open) {
            end_b = (int32_t)beginT;
            end_l = level;
            if (nT == 1u && !CMP) {
                flag = 1;
                done = true;
            } else {
                if ((k & 1) == 0) rnd = philox4x32_10(ctr0, ctr1, (uint32_t)(k >> 1), a.batch, a.key0, a.key1);
                const uint32_t xsel = (k & 1) ? rnd.z : rnd.x;
                const uint32_t xrr = (k & 1) ? rnd.w : rnd.y;
                const uint32_t r = __umulhi(xsel, nT);
                const bool internal = (int)nT > tv.leaf_size && level < tv.max_level;
                const float4* __restrict__ ba = tv.bagg + (int64_t)blk * D3;
                const float4* __restrict__ bd = tv.bdip + (int64_t)blk * D3;
                const uint32_t* __restrict__ bt = tv.btopo + (int64_t)blk * TS;
                float4 aggC, dpC = zero4;
                uint32_t nC = 1u, beginC;
                int32_t blkC = 0;
                // d = 2: the block's eight counts stay in registers from the selection to the swap
                // (a reload is another gather per lane), and a compressed block's codes arrive with
                // them, so decoding the selected child waits on no further load
                uint32_t cn[KEEPN ? D3 : 1];
                sbh_u32x4v cb[CMP ? D3 / 2 : 1];
                auto count = [&](int c) -> uint32_t {
                    if constexpr (KEEPN) return cn[c];
                    else return gld(bt + c);
                };
                if (internal) {
                    if constexpr (KEEPN) {
#pragma unroll
                        for (int c = 0; c < D3; ++c) cn[c] = gld(bt + c);
                    }
                    if constexpr (CMP) {
                        const uint32_t* __restrict__ qb = reinterpret_cast<const uint32_t*>(tv.bq) + (int64_t)blk * 16;
#pragma unroll
                        for (int i = 0; i < D3 / 2; ++i) cb[i] = gld4u(qb + 4 * i);
                    }
                    // child selection from the point counts alone
                    uint32_t pre = 0u, preC = 0u;
                    int32_t nint = 0, nintC = 0;
                    int csel = 0;
                    uint32_t w0 = 0u, w1 = 0u;
#pragma unroll
                    for (int c = 0; c < D3; ++c) {
                        const uint32_t cnt = count(c);
                        const bool hit = (r - pre) < cnt;
                        csel = hit ? c : csel;
                        preC = hit ? pre : preC;
                        nintC = hit ? nint : nintC;
                        nC = hit ? cnt : nC;
                        if constexpr (CMP) {
                            w0 = hit ? ((c & 1) ? cb[c >> 1].z : cb[c >> 1].x) : w0;
                            w1 = hit ? ((c & 1) ? cb[c >> 1].w : cb[c >> 1].y) : w1;
                        }
                        nint += ((int)cnt > tv.leaf_size && level + 1 < tv.max_level) ? 1 : 0;
                        pre += cnt;
                    }
                    if constexpr (CMP) {
                        // the selected child decoded: offset o s_c + (com^q_T - q), mass m^q_T f
                        aggC = make_float4(fmaf(h16(w0 & 0xFFFFu), sideC, dTx), fmaf(h16(w0 >> 16), sideC, dTy),
                                           fmaf(h16(w1 & 0xFFFFu), sideC, dTz), fmaf(h16(w1 >> 16), mT, 0.0f));
                    } else {
                        aggC = gld4(ba + csel);
                    }
                    if constexpr (K == SBH_WINDING) dpC = gld4(bd + csel);
                    beginC = beginT + preC;
                    blkC = (int32_t)gld(bt + D3) + nintC;
                } else {
                    aggC = gld4(tv.pts + beginT + r);
                    if constexpr (CMP) aggC = make_float4(aggC.x - qx, aggC.y - qy, aggC.z - qz, aggC.w);
                    if constexpr (K == SBH_WINDING) dpC = gld4(tv.pdip + beginT + r);
                    beginC = beginT + r;
                }
                // roulette first (Eq. (5)); its offset and squared distance also give the
                // selected child's own term, bit for bit the value the swap's sum takes for it
                // (CMP: aggC holds the offset itself)
                float pr;
                float dC = 0.0f;
                const float cx = CMP ? aggC.x : aggC.x - qx;
                const float cy = CMP ? aggC.y : aggC.y - qy;
                const float cz = CMP ? aggC.z : aggC.z - qz;
                const float r2C = norm2(cx, cy, cz);
                if (a.rr_mode == 0) {
                    dC = fsqrt(r2C);
                    pr = fminf(1.0f, fmaxf(diamT, dT) * frcp((float)D * dC));
                } else {
                    pr = a.rr_mode == 1 ? 1.0f : 0.5f;
                }
                if (unit24(xrr) >= pr) {
                    flag = 0;
                    done = true;
                } else {
                    // contribution swap, Eq. (6)
                    float sumc = 0.0f;
                    const float tC = term_r2<K>(aggC, dpC, cx, cy, cz, r2C, kp, r0);
                    if (internal && CMP) {
#pragma unroll
                        for (int c = 0; c < D3; ++c) {
                            const uint32_t cnt = count(c);
                            const uint32_t c0 = (c & 1) ? cb[c >> 1].z : cb[c >> 1].x;
                            const uint32_t c1 = (c & 1) ? cb[c >> 1].w : cb[c >> 1].y;
                            const float ex = fmaf(h16(c0 & 0xFFFFu), sideC, dTx);
                            const float ey = fmaf(h16(c0 >> 16), sideC, dTy);
                            const float ez = fmaf(h16(c1 & 0xFFFFu), sideC, dTz);
                            const float mc = fmaf(h16(c1 >> 16), mT, 0.0f);
                            const float v = term_r2_acc<K>(make_float4(0.f, 0.f, 0.f, mc), zero4, ex, ey, ez,
                                                           norm2(ex, ey, ez), kp, r0, sumc);
                            sumc = cnt ? v : sumc;
                        }
                    } else if (internal) {
#pragma unroll
                        for (int c = 0; c < D3; ++c) {
                            const uint32_t cnt = count(c);
                            const float4 gd = (K == SBH_WINDING) ? gld4(bd + c) : zero4;
                            const float v = term_acc<K>(gld4(ba + c), gd, qx, qy, qz, kp, r0, sumc);
                            sumc = cnt ? v : sumc;
                        }
                    } else {
                        for (uint32_t i = 0; i < nT; ++i) {
                            const float4 gd = (K == SBH_WINDING) ? gld4(tv.pdip + beginT + i) : zero4;
                            sumc = term_acc<K>(gld4(tv.pts + beginT + i), gd, qx, qy, qz, kp, r0, sumc);
                        }
                    }
                    prr *= pr;
                    acc += (sumc - tT) * (fna * frcp((float)nT * prr));
                    ++steps;
                    if (!internal) {
                        end_b = (int32_t)beginC;
                        end_l = level + 1;
                        flag = 2;
                        done = true;
                    } else {
                        dT = dC;
                        tT = tC;
                        nT = nC;
                        beginT = beginC;
                        blk = blkC;
                        ++level;
                        diamT *= kInvD;
                        ++k;
                        if constexpr (CMP) {
                            dTx = cx;
                            dTy = cy;
                            dTz = cz;
                            mT = aggC.w;
                            sideC *= kInvD;
                        }
                    }
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
        gst(out + jq, query_value<K>(val, rq, logwbar, a.alpha, qpos[wv][3 * lane], qpos[wv][3 * lane + 1],
                                     qpos[wv][3 * lane + 2]));
    }
}

// ---------------------------------------------------------------------------
// Coherent estimator: one lane per query, one random stream per wavefront.
// When G is a multiple of 64 the 64 queries of a wavefront share their
// Philox stream, so under the uniform proposal the selected child at every
// step is the same for all of them (selection does not depend on q): the
// wavefront walks one path per (subdomain, sample), reading each child block
// once for all its lanes, and only the Russian-roulette test (p depends on q)
// retires lanes individually.  This is the shared-seed design of the paper's
// implementation section on 64-wide wavefronts.  Per query the subdomain
// totals CV_a + F_a / S are added in slot order within each part of the
// slots that one wavefront walks (kWaveParts parts), then the parts' sums in
// part order.
// ---------------------------------------------------------------------------
// The largest of the 64 lanes' values (non-negative floats order as their bit
// patterns): an inclusive max-scan by DPP row shifts and row broadcasts, read
// from lane 63.  Needs every lane active.
__device__ __forceinline__ float wave_max_nonneg(float v)
{
    uint32_t x = __float_as_uint(v);
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false));   // row_shr:1
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false));   // row_shr:2
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false));   // row_shr:4
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false));   // row_shr:8
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false));   // row_bcast:15
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false));   // row_bcast:31
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)x, 63));
}

// max(a, b) of two non-negative finite floats as one instruction (fmaxf quiets
// NaN inputs first, two more instructions that the walk does not need)
// Byte offsets into the tree's arrays: 32-bit while every array of the tree is
// below 4 GiB (scalar loads then take the offset as a register operand, with no
// 64-bit address arithmetic), 64-bit otherwise.
template <bool O64>
struct TreeOff {
    using T = uint32_t;
};
template <>
struct TreeOff<true> {
    using T = uint64_t;
};
template <class T, class O>
__device__ __forceinline__ const T* at_off(const T* base, O byte_off)
{
    return (const T*)((const char*)base + byte_off);
}

// the value lane c holds, as a wavefront-uniform scalar
__device__ __forceinline__ float rdlane(float v, int c)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), c));
}

__device__ __forceinline__ float vmax(float a, float b)
{
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Random words of the coherent walk.  They do not depend on the query, so one
// vector Philox evaluation serves eight paths of a wavefront: lane l holds the
// block (counter word 2 = step pair) of step pair l & 7 of path 8m + (l >> 3).
// Step k of path p reads its two words from lane 8 (p & 7) + k / 2, the
// roulette word already as its uniform variate u = (x >> 8) 2^-24.  Steps
// past the sixteenth (rare: the roulette ends most paths within a few steps,
// and trees are seldom that deep) compute their block again on the vector
// unit (lane 0 holds it).  Counters are those of the per-query walk.
struct PathWords {
    u32x4 vr;
    int chunk = -1;   // m of the eight paths held, -1 before the first
    __device__ __forceinline__ void need(uint32_t path, uint32_t ctr0, uint32_t ctr3, uint32_t key0, uint32_t key1)
    {
        if ((int)(path >> 3) != chunk) {
            chunk = (int)(path >> 3);
            const uint32_t l = threadIdx.x & 63;
            vr = philox4x32_10(ctr0, (path & ~7u) + (l >> 3), l & 7u, ctr3, key0, key1);
            vr.y = __float_as_uint(unit24(vr.y));
            vr.w = __float_as_uint(unit24(vr.w));
        }
    }
    // the selection word and the roulette variate of step k of `path`
    __device__ __forceinline__ void step(int k, uint32_t path, uint32_t ctr0, uint32_t ctr3, uint32_t key0,
                                         uint32_t key1, uint32_t& xsel, float& u) const
    {
        if (k < 16) {
            const int src = (int)((path & 7u) << 3) + (k >> 1);
            xsel = __builtin_amdgcn_readlane((k & 1) ? vr.z : vr.x, src);
            u = __uint_as_float(__builtin_amdgcn_readlane((k & 1) ? vr.w : vr.y, src));
        } else {
            const u32x4 e = philox4x32_10(ctr0, path, (uint32_t)(k >> 1) + (threadIdx.x & 7u), ctr3, key0, key1);
            xsel = __builtin_amdgcn_readlane((k & 1) ? e.z : e.x, 0);
            u = unit24(__builtin_amdgcn_readlane((k & 1) ? e.w : e.y, 0));
        }
    }
    // the same for a step k < 16 whose parity is known at compile time (ODD: k odd)
    template <bool ODD>
    __device__ __forceinline__ void step_held(int k, uint32_t path, uint32_t& xsel, float& u) const
    {
        const int src = (int)((path & 7u) << 3) + (k >> 1);
        xsel = __builtin_amdgcn_readlane(ODD ? vr.z : vr.x, src);
        u = __uint_as_float(__builtin_amdgcn_readlane(ODD ? vr.w : vr.y, src));
    }
    // and for a step k >= 16 (the variate as a wavefront-uniform scalar)
    __device__ __forceinline__ void step_late(int k, uint32_t path, uint32_t ctr0, uint32_t ctr3, uint32_t key0,
                                              uint32_t key1, uint32_t& xsel, float& u) const
    {
        const u32x4 e = philox4x32_10(ctr0, path, (uint32_t)(k >> 1) + (threadIdx.x & 7u), ctr3, key0, key1);
        xsel = __builtin_amdgcn_readlane((k & 1) ? e.z : e.x, 0);
        u = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(unit24((k & 1) ? e.w : e.y))));
    }
};

// The words of one path only (the Barnes-Hut-cut subdomains, which are found
// one at a time): lane l holds the block of step pair l, for steps 0..127
// (deeper than any tree), its roulette words converted.
struct PathWordsOne {
    u32x4 vr;
    __device__ __forceinline__ void compute(uint32_t ctr0, uint32_t ctr1, uint32_t ctr2_base, uint32_t ctr3,
                                            uint32_t key0, uint32_t key1)
    {
        vr = philox4x32_10(ctr0, ctr1, ctr2_base + (threadIdx.x & 63u), ctr3, key0, key1);
        vr.y = __float_as_uint(unit24(vr.y));
        vr.w = __float_as_uint(unit24(vr.w));
    }
    __device__ __forceinline__ void step(int k, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t& xsel,
                                         float& u) const
    {
        xsel = __builtin_amdgcn_readlane((k & 1) ? vr.z : vr.x, k >> 1);
        u = __uint_as_float(__builtin_amdgcn_readlane((k & 1) ? vr.w : vr.y, k >> 1));
    }
    template <bool ODD>
    __device__ __forceinline__ void step_held(int k, uint32_t, uint32_t& xsel, float& u) const
    {
        xsel = __builtin_amdgcn_readlane(ODD ? vr.z : vr.x, k >> 1);
        u = __uint_as_float(__builtin_amdgcn_readlane(ODD ? vr.w : vr.y, k >> 1));
    }
    __device__ __forceinline__ void step_late(int k, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t& xsel,
                                              float& u) const
    {
        step(k, 0u, 0u, 0u, 0u, 0u, xsel, u);
    }
};

// One path of the coherent walk from subdomain node a (n_a points from begin_a, at
// level level_a; blk_a its child block when internal), for the wavefront's 64 queries.
// VM: the roulette compiled in: 0 Eq. (5) (rr_mode 0), 1 Eq. (5) voted over
// the wavefront (rr_mode 3), 2 chosen at run time among rr_mode 0, 1 and 2.
template <int D, int K, bool TRACE, bool O64, class PW = PathWords, int VM = 2>
__device__ __forceinline__ float wave_path(const TreeView& tv, float qx, float qy, float qz, float r0,
                                           const KParams& kp, bool valid, uint32_t n_a, uint32_t begin_a,
                                           int32_t blk_a, float4 agg_a, float t_a, const PW& pw,
                                           uint32_t ctr0, uint32_t ctr1, uint32_t ctr3, uint32_t key0,
                                           uint32_t key1, int rr_mode, int4* rec, int level_a = 1)
{
#pragma clang fp contract(off)
    constexpr int D3 = D * D * D;
    constexpr int TS = topo_stride(D3);
    constexpr float kInvD = 1.0f / (float)D;
    using Off = typename TreeOff<O64>::T;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    // d = 4: each wavefront's row for the child block of the step; every kernel that walks
    // paths runs at most four wavefronts per workgroup (256 threads), one row each
    __shared__ float4 sblk[D == 4 ? 4 : 1][64];
    __shared__ float4 sblkd[D == 4 && K == SBH_WINDING ? 4 : 1][64];
    // wavefront-uniform walk state
    uint32_t nT = n_a, beginT = begin_a;
    int32_t blk = blk_a;
    int level = level_a;
    float diamT = ldexpf(tv.diam0, -level_a * (D == 2 ? 1 : D == 4 ? 2 : 3));
    const float fna = (float)n_a;
    // per-lane state; actm holds the lanes still walking (wavefront-uniform): a lane's own
    // flag is its bit, so that the votes below are single compares and no per-lane flag is
    // carried from step to step
    uint64_t actm = __ballot(valid);
    float dT = fsqrt(norm2(agg_a.x - qx, agg_a.y - qy, agg_a.z - qz));   // |com_T - q|, carried step to step
    float tT = t_a, prr = 1.0f, acc = 0.0f;
    int steps = 0, flag = 0;
    int32_t end_b = (int32_t)beginT, end_l = level;
    // the roulette (Eq. (5)); the offset and squared distance it takes also give the
    // selected child's own term, which opens the swap's sum and is the next step's control
    // variate (the two agree bit for bit and the child is not evaluated twice)
    // (Eq. (5) is evaluated in every mode and replaced by the mode's constant, a select
    // rather than a branch)
    const bool rr_eq5 = VM != 2 || rr_mode == 0;
    const float rr_fixed = rr_mode == 1 ? 1.0f : 0.5f;
    // rr_mode 3: Eq. (5) voted over the wavefront (the largest p of its queries with finite
    // coordinates, the same for every lane, so the wavefront stops or continues as one)
    constexpr bool rr_vote = VM == 1;
    const bool voter = valid && __builtin_isfinite(qx) && __builtin_isfinite(qy) && __builtin_isfinite(qz);
    // One reciprocal square root gives both |c - q| and 1 / (D |c - q|).  At |c - q| = 0
    // the distance is NaN, which the next step's max ignores (v_max returns the other
    // operand), and p = min(1, inf) = 1 as Eq. (5)'s limit.
    auto roulette = [&](float r2C, float& dC) -> float {
        const float ic = __builtin_amdgcn_rsqf(r2C);
        dC = r2C * ic;
        const float p5 = fminf(1.0f, vmax(diamT, dT) * (kInvD * ic));
        float p = rr_eq5 ? p5 : rr_fixed;
        if (rr_vote) p = wave_max_nonneg(voter ? p : 0.0f);
        return p;
    };
    int k = 0;
    // internal nodes: the walk leaves the loops below at a leaf, or when the roulette
    // has stopped every lane (actm then 0); each loop's only exit is its condition
    // (leaf_size >= 1, so an internal node holds at least two points)
    bool go = actm != 0ull && (int)nT > tv.leaf_size && level < tv.max_level;
    const int lvl_int = tv.max_level - 1;   // a child below this level can be internal
    // one internal step.  mode 0 / 1: an even / odd step k < 16, whose random words the
    // wavefront holds (the first loop below takes them in pairs, so that each knows where
    // its words are); mode 2: a step k >= 16, which computes them again
    auto internal_step = [&](auto mode) {
        constexpr int M = decltype(mode)::value;
        uint32_t xsel;
        float u;
        if constexpr (M == 2) pw.step_late(k, ctr1, ctr0, ctr3, key0, key1, xsel, u);
        else pw.template step_held<M == 1>(k, ctr1, xsel, u);
        const uint32_t r = __umulhi(xsel, nT);
        const Off boff = (Off)(uint32_t)blk * (Off)(D3 * 16);   // the block's aggregates and dipoles
        const Off toff = (Off)(uint32_t)blk * (Off)(TS * 4);    // its topology row
        const uint32_t* __restrict__ bt = at_off(tv.btopo, toff);
        float4 aggC, dpC = zero4;   // the selected child's aggregate (and dipole)
        uint32_t nC = 1u, beginC;
        int32_t blkC = 0;
        int csel = 0;
        uint32_t nonempty = 0u;   // d = 2: slots with points (wavefront-uniform)
        uint64_t nonempty64 = 0ull;   // d = 4
        uint32_t nonempty8 = 0u;      // d = 8: this lane's eight slots with points
        if constexpr (D == 2) {
            // child selection across lanes 0..7 (one slot each): an exclusive scan of the
            // counts by DPP row shifts, then ballots give the slot whose range holds r, the
            // internal slots before it and the non-empty slots
            // (lanes 8..63 load the row's last word, padding that the build leaves zero: they
            // hold a zero count and none of them votes)
            static_assert(TS - 1 > D3, "the topology row needs a padding word");
            const int ln = threadIdx.x & 63;
            const uint32_t cl = gld(bt + (ln < D3 ? ln : TS - 1));
            uint32_t inc = cl;
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x111, 0xF, 0xF, false);   // row_shr:1
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x112, 0xF, 0xF, false);   // row_shr:2
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x114, 0xF, 0xF, false);   // row_shr:4
            const uint32_t excl = inc - cl;
            // (r < n_T, so exactly one slot holds it)
            const uint32_t hm = (uint32_t)__ballot((r - excl) < cl);
            const uint32_t im = level < lvl_int ? (uint32_t)__ballot((int)cl > tv.leaf_size) : 0u;
            nonempty = (uint32_t)__ballot(cl != 0u);
            csel = __builtin_ctz(hm);
            const uint32_t preC = (uint32_t)__builtin_amdgcn_readlane((int)excl, csel);
            nC = (uint32_t)__builtin_amdgcn_readlane((int)cl, csel);
            const int32_t nintC = __popc(im & ((1u << csel) - 1u));
            aggC = gld4(at_off(tv.bagg, boff + (Off)(csel * 16)));
            if constexpr (K == SBH_WINDING) dpC = gld4(at_off(tv.bdip, boff + (Off)(csel * 16)));
            beginC = beginT + preC;
            blkC = (int32_t)gld(bt + D3) + nintC;
        } else if constexpr (D == 4) {
            // 64 slots, one per lane: an inclusive scan of the counts across the wavefront
            // (row shifts within rows of 16 lanes, then the row broadcasts of lanes 15 and 31),
            // and ballots give the slot whose range holds r, the internal slots before it and
            // the non-empty slots
            const int ln = threadIdx.x & 63;
            const uint32_t cl = gld(bt + ln);
            uint32_t inc = cl;
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x111, 0xF, 0xF, false);   // row_shr:1
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x112, 0xF, 0xF, false);   // row_shr:2
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x114, 0xF, 0xF, false);   // row_shr:4
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x118, 0xF, 0xF, false);   // row_shr:8
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x142, 0xA, 0xF, false);   // row_bcast:15
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x143, 0xC, 0xF, false);   // row_bcast:31
            const uint32_t excl = inc - cl;
            const uint64_t hm = __ballot((r - excl) < cl);
            const uint64_t im = level < lvl_int ? __ballot((int)cl > tv.leaf_size) : 0ull;
            nonempty64 = __ballot(cl != 0u);
            csel = (int)__builtin_ctzll(hm);
            const uint32_t preC = (uint32_t)__builtin_amdgcn_readlane((int)excl, csel);
            nC = (uint32_t)__builtin_amdgcn_readlane((int)cl, csel);
            const int32_t nintC = (int32_t)__popcll(im & ((1ull << csel) - 1ull));
            aggC = gld4(at_off(tv.bagg, boff + (Off)(csel * 16)));
            if constexpr (K == SBH_WINDING) dpC = gld4(at_off(tv.bdip, boff + (Off)(csel * 16)));
            beginC = beginT + preC;
            blkC = (int32_t)gld(bt + D3) + nintC;
        } else {
            // d = 8: 512 slots, eight per lane (lane l holds slots 8l .. 8l + 7, two 16-byte
            // loads); each lane's point total and internal-slot count are scanned across the
            // wavefront as the d = 4 counts are, a ballot finds the lane whose range holds r,
            // and that lane's eight slots give the child; each lane keeps its non-empty slots
            // as eight bits for the swap
            static_assert(D3 == 512, "eight slots per lane");
            const int ln = threadIdx.x & 63;
            const sbh_u32x4v c0 = gld4u(bt + 8 * ln), c1 = gld4u(bt + 8 * ln + 4);
            const uint32_t cl[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
            const bool deeper = level < lvl_int;
            uint32_t tot = 0u, nin = 0u;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                tot += cl[i];
                nin += (deeper && (int)cl[i] > tv.leaf_size) ? 1u : 0u;
                nonempty8 |= cl[i] != 0u ? 1u << i : 0u;
            }
            uint32_t inc = tot, inci = nin;
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x111, 0xF, 0xF, false);    // row_shr:1
            inci += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inci, 0x111, 0xF, 0xF, false);
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x112, 0xF, 0xF, false);    // row_shr:2
            inci += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inci, 0x112, 0xF, 0xF, false);
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x114, 0xF, 0xF, false);    // row_shr:4
            inci += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inci, 0x114, 0xF, 0xF, false);
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x118, 0xF, 0xF, false);    // row_shr:8
            inci += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inci, 0x118, 0xF, 0xF, false);
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x142, 0xA, 0xF, false);    // row_bcast:15
            inci += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inci, 0x142, 0xA, 0xF, false);
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x143, 0xC, 0xF, false);    // row_bcast:31
            inci += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inci, 0x143, 0xC, 0xF, false);
            const uint32_t excl = inc - tot;
            // (r < n_T, so exactly one lane's range holds it; in the other lanes no slot hits)
            const int L = (int)__builtin_ctzll(__ballot((r - excl) < tot));
            uint32_t pre = excl, preS = 0u, nS = 0u, niS = 0u, ni = inci - nin;
            int sl = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const bool hit = (r - pre) < cl[i];
                sl = hit ? i : sl;
                preS = hit ? pre : preS;
                nS = hit ? cl[i] : nS;
                niS = hit ? ni : niS;
                ni += (deeper && (int)cl[i] > tv.leaf_size) ? 1u : 0u;
                pre += cl[i];
            }
            csel = 8 * L + __builtin_amdgcn_readlane(sl, L);
            const uint32_t preC = (uint32_t)__builtin_amdgcn_readlane((int)preS, L);
            nC = (uint32_t)__builtin_amdgcn_readlane((int)nS, L);
            const int32_t nintC = __builtin_amdgcn_readlane((int)niS, L);
            aggC = gld4(at_off(tv.bagg, boff + (Off)(csel * 16)));
            if constexpr (K == SBH_WINDING) dpC = gld4(at_off(tv.bdip, boff + (Off)(csel * 16)));
            beginC = beginT + preC;
            blkC = (int32_t)gld(bt + D3) + nintC;
        }
        // roulette first: the swap is only needed by lanes that continue
        float dC;
        const float cx = aggC.x - qx, cy = aggC.y - qy, cz = aggC.z - qz;
        const float r2C = norm2(cx, cy, cz);
        const float p = roulette(r2C, dC);
        const uint64_t contm = __ballot(u < p) & actm;
        if (__builtin_amdgcn_inverse_ballot_w64(actm & ~contm)) {   // lanes this roulette stops
            flag = 0;
            end_b = (int32_t)beginT;
            end_l = level;
        }
        actm = contm;
        if (contm != 0ull) {
            // contribution swap, Eq. (6)
            const float tC = term_r2<K>(aggC, dpC, cx, cy, cz, r2C, kp, r0);
            float sumc = tC;
            const float4* __restrict__ ba = at_off(tv.bagg, boff);
            const float4* __restrict__ bd = at_off(tv.bdip, boff);
            if constexpr (D == 2) {
                // the block in one batch of scalar loads; only the other non-empty slots (about
                // half of them on a surface) are evaluated, behind wavefront-uniform branches
                const uint32_t rest = nonempty & ~(1u << csel);
                float4 g8[D3];
#pragma unroll
                for (int c = 0; c < D3; ++c) g8[c] = gld4(ba + c);
#pragma unroll
                for (int c = 0; c < D3; ++c) {
                    if (!((rest >> c) & 1u)) continue;
                    const float4 gd = (K == SBH_WINDING) ? gld4(bd + c) : zero4;
                    sumc = term_acc<K>(g8[c], gd, qx, qy, qz, kp, r0, sumc);
                }
            } else if constexpr (D == 4) {
                // the block in one coalesced load (lane c holds slot c), staged in the wavefront's
                // LDS row, then the other non-empty slots (a surface fills a few of the 64) in
                // turn, each read back by every lane as one broadcast LDS load
                const int ln = threadIdx.x & 63;
                const int wv = (threadIdx.x >> 6) & 3;
                sblk[wv][ln] = gld4(ba + ln);
                if constexpr (K == SBH_WINDING) sblkd[wv][ln] = gld4(bd + ln);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                uint64_t rest = nonempty64 & ~(1ull << csel);
                while (rest) {
                    const int c = (int)__builtin_ctzll(rest);
                    rest &= rest - 1ull;
                    const float4 g = sblk[wv][c];
                    float4 gd = zero4;
                    if constexpr (K == SBH_WINDING) gd = make_float4(sblkd[wv][c].x, sblkd[wv][c].y, sblkd[wv][c].z, 0.0f);
                    sumc = term_acc<K>(g, gd, qx, qy, qz, kp, r0, sumc);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // the row is reused next step
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else {
                // only the other non-empty slots (a surface fills a few of a node's 512), in slot
                // order: the lanes in order, each lane's eight bits in order
                const int ln = threadIdx.x & 63;
                const uint32_t mine = ln == (csel >> 3) ? nonempty8 & ~(1u << (csel & 7)) : nonempty8;
                uint64_t lanes = __ballot(mine != 0u);
                while (lanes) {
                    const int l = (int)__builtin_ctzll(lanes);
                    lanes &= lanes - 1ull;
                    uint32_t ml = (uint32_t)__builtin_amdgcn_readlane((int)mine, l);
                    while (ml) {
                        const int c = 8 * l + (int)__builtin_ctz(ml);
                        ml &= ml - 1u;
                        const float4 gd = (K == SBH_WINDING) ? gld4(bd + c) : zero4;
                        sumc = term_acc<K>(gld4(ba + c), gd, qx, qy, qz, kp, r0, sumc);
                    }
                }
            }
            // the lanes the roulette keeps take the step (selects, not a branch)
            const bool cont = __builtin_amdgcn_inverse_ballot_w64(contm);
            const float prr2 = prr * p;
            const float acc2 = acc + (sumc - tT) * (fna * frcp((float)nT * prr2));
            prr = cont ? prr2 : prr;
            acc = cont ? acc2 : acc;
            tT = cont ? tC : tT;
            steps += cont ? 1 : 0;
            dT = dC;
            nT = nC;
            beginT = beginC;
            blk = blkC;
            ++level;
            diamT *= kInvD;
            ++k;
        }
        go = actm != 0ull && (int)nT > tv.leaf_size && level < tv.max_level;
    };
    while (go && k < 16) {   // k is even here, so both steps are below 16
        internal_step(std::integral_constant<int, 0>{});
        if (go) internal_step(std::integral_constant<int, 1>{});
    }
    while (go) internal_step(std::integral_constant<int, 2>{});
    if (actm != 0ull) {
        if (nT == 1u) {   // a single point: the walk is exact from here
            if (__builtin_amdgcn_inverse_ballot_w64(actm)) { flag = 1; end_b = (int32_t)beginT; end_l = level; }
        } else {          // a leaf: its points are the virtual children, one drawn uniformly
            uint32_t xsel;
            float u;
            pw.step(k, ctr1, ctr0, ctr3, key0, key1, xsel, u);
            const uint32_t r = __umulhi(xsel, nT);
            const float4 aggC = gld4(at_off(tv.pts, (Off)(beginT + r) * (Off)16));
            const float4 dpC = (K == SBH_WINDING) ? gld4(at_off(tv.pdip, (Off)(beginT + r) * (Off)16)) : zero4;
            float dC;
            const float cx = aggC.x - qx, cy = aggC.y - qy, cz = aggC.z - qz;
            const float r2C = norm2(cx, cy, cz);
            const float p = roulette(r2C, dC);
            const uint64_t contm = __ballot(u < p) & actm;
            if (__builtin_amdgcn_inverse_ballot_w64(actm & ~contm)) {
                flag = 0;
                end_b = (int32_t)beginT;
                end_l = level;
            }
            if (contm != 0ull) {
                float sumc = term_r2<K>(aggC, dpC, cx, cy, cz, r2C, kp, r0);
                for (uint32_t i = 0; i < nT; ++i) {
                    if (i == r) continue;   // the selected point: its term opened the sum
                    const Off po = (Off)(beginT + i) * (Off)16;
                    const float4 gd = (K == SBH_WINDING) ? gld4(at_off(tv.pdip, po)) : zero4;
                    sumc = term_acc<K>(gld4(at_off(tv.pts, po)), gd, qx, qy, qz, kp, r0, sumc);
                }
                if (__builtin_amdgcn_inverse_ballot_w64(contm)) {
                    prr *= p;
                    acc += (sumc - tT) * (fna * frcp((float)nT * prr));
                    ++steps;
                    flag = 2;
                    end_b = (int32_t)(beginT + r);
                    end_l = level + 1;
                }
            }
        }
    }
    if constexpr (TRACE) *rec = make_int4(end_b, end_l, steps, flag);
    return acc;
}

// ---------------------------------------------------------------------------
// The coherent walk on compressed aggregates (d = 2; potential and smooth
// distance; uniform path index).  A child block is eight 8-byte codes: the
// child's centre of mass as a binary16 offset from its decoded parent in units
// of its cell side, and its mass as a binary16 fraction of the decoded
// parent's.  Each lane carries the decoded parent's offset from its query
// (dT, float32) and the wavefront the decoded parent mass mT, so a child's
// offset is one multiply-add per axis: com^q_c - q = o_c s_c + (com^q_T - q).
// The decoded values are those the oracle defines, up to float32 rounding.
// A node holding one point is not exact under compression, so it takes the
// leaf step too (its point is a virtual child).  Random words, selection and
// roulette are those of wave_path.
// ---------------------------------------------------------------------------

template <int K, bool TRACE, bool O64, int VM>
__device__ __forceinline__ float wave_path_q(const TreeView& tv, float qx, float qy, float qz, float r0,
                                             const KParams& kp, bool valid, uint32_t n_a, uint32_t begin_a,
                                             int32_t blk_a, float dax, float day, float daz, float m_a, float t_a,
                                             const PathWords& pw, uint32_t ctr0, uint32_t ctr1, uint32_t ctr3,
                                             uint32_t key0, uint32_t key1, int rr_mode, int4* rec)
{
#pragma clang fp contract(off)
    constexpr int D3 = 8;
    constexpr int TS = topo_stride(D3);
    constexpr float kInvD = 0.5f;
    using Off = typename TreeOff<O64>::T;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t nT = n_a, beginT = begin_a;
    int32_t blk = blk_a;
    int level = 1;
    float diamT = tv.diam0 * kInvD;
    float sideC = tv.side * 0.25f;   // the cell side of the children of a level-1 node
    float mT = m_a;
    const float fna = (float)n_a;
    uint64_t actm = __ballot(valid);
    float dTx = dax, dTy = day, dTz = daz;
    float dT = fsqrt(norm2(dax, day, daz));
    float tT = t_a, prr = 1.0f, acc = 0.0f;
    int steps = 0, flag = 0;
    int32_t end_b = (int32_t)beginT, end_l = level;
    const bool rr_eq5 = VM != 2 || rr_mode == 0;   // VM: the roulette, as in wave_path
    const float rr_fixed = rr_mode == 1 ? 1.0f : 0.5f;
    // rr_mode 3: Eq. (5) voted over the wavefront (the largest p of its queries with finite
    // coordinates, the same for every lane, so the wavefront stops or continues as one)
    constexpr bool rr_vote = VM == 1;
    const bool voter = valid && __builtin_isfinite(qx) && __builtin_isfinite(qy) && __builtin_isfinite(qz);
    auto roulette = [&](float r2C, float& dC) -> float {
        const float ic = __builtin_amdgcn_rsqf(r2C);
        dC = r2C * ic;
        const float p5 = fminf(1.0f, vmax(diamT, dT) * (kInvD * ic));
        float p = rr_eq5 ? p5 : rr_fixed;
        if (rr_vote) p = wave_max_nonneg(voter ? p : 0.0f);
        return p;
    };
    int k = 0;
    bool go = actm != 0ull && (int)nT > tv.leaf_size && level < tv.max_level;
    const int lvl_int = tv.max_level - 1;
    auto internal_step = [&](auto mode) {
        constexpr int M = decltype(mode)::value;
        uint32_t xsel;
        float u;
        if constexpr (M == 2) pw.step_late(k, ctr1, ctr0, ctr3, key0, key1, xsel, u);
        else pw.template step_held<M == 1>(k, ctr1, xsel, u);
        const uint32_t r = __umulhi(xsel, nT);
        const Off qoff = (Off)(uint32_t)blk * (Off)(D3 * 8);    // the block's codes
        const Off toff = (Off)(uint32_t)blk * (Off)(TS * 4);
        const uint32_t* __restrict__ bt = at_off(tv.btopo, toff);
        const uint32_t* __restrict__ bqw = at_off(reinterpret_cast<const uint32_t*>(tv.bq), qoff);
        // child selection across lanes 0..7, as wave_path
        const int ln = threadIdx.x & 63;
        const uint32_t cl = gld(bt + (ln < D3 ? ln : TS - 1));
        uint32_t inc = cl;
        inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x111, 0xF, 0xF, false);   // row_shr:1
        inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x112, 0xF, 0xF, false);   // row_shr:2
        inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x114, 0xF, 0xF, false);   // row_shr:4
        const uint32_t excl = inc - cl;
        const uint32_t hm = (uint32_t)__ballot((r - excl) < cl);
        const uint32_t im = level < lvl_int ? (uint32_t)__ballot((int)cl > tv.leaf_size) : 0u;
        const uint32_t nonempty = (uint32_t)__ballot(cl != 0u);
        const int csel = __builtin_ctz(hm);
        const uint32_t preC = (uint32_t)__builtin_amdgcn_readlane((int)excl, csel);
        const uint32_t nC = (uint32_t)__builtin_amdgcn_readlane((int)cl, csel);
        const int32_t nintC = __popc(im & ((1u << csel) - 1u));
        const uint32_t w0 = gld(bqw + 2 * csel), w1 = gld(bqw + 2 * csel + 1);
        const uint32_t beginC = beginT + preC;
        const int32_t blkC = (int32_t)gld(bt + D3) + nintC;
        // the selected child's offset and the roulette (Eq. (5))
        const float cx = fmaf(h16(w0 & 0xFFFFu), sideC, dTx);
        const float cy = fmaf(h16(w0 >> 16), sideC, dTy);
        const float cz = fmaf(h16(w1 & 0xFFFFu), sideC, dTz);
        const float r2C = norm2(cx, cy, cz);
        float dC;
        const float p = roulette(r2C, dC);
        const float mC = fmaf(h16(w1 >> 16), mT, 0.0f);
        const uint64_t contm = __ballot(u < p) & actm;
        if (__builtin_amdgcn_inverse_ballot_w64(actm & ~contm)) {
            flag = 0;
            end_b = (int32_t)beginT;
            end_l = level;
        }
        actm = contm;
        if (contm != 0ull) {
            // contribution swap, Eq. (6): the selected child's term opens the sum
            const float tC = term_r2<K>(make_float4(0.f, 0.f, 0.f, mC), zero4, cx, cy, cz, r2C, kp, r0);
            float sumc = tC;
            sbh_u32x4v cb[D3 / 2];   // the block's codes: slot c in words 2c, 2c + 1
#pragma unroll
            for (int i = 0; i < D3 / 2; ++i) cb[i] = gld4u(bqw + 4 * i);
            const uint32_t rest = nonempty & ~(1u << csel);
#pragma unroll
            for (int c = 0; c < D3; ++c) {
                if (!((rest >> c) & 1u)) continue;
                const uint32_t c0 = (c & 1) ? cb[c >> 1].z : cb[c >> 1].x;
                const uint32_t c1 = (c & 1) ? cb[c >> 1].w : cb[c >> 1].y;
                const float ex = fmaf(h16(c0 & 0xFFFFu), sideC, dTx);
                const float ey = fmaf(h16(c0 >> 16), sideC, dTy);
                const float ez = fmaf(h16(c1 & 0xFFFFu), sideC, dTz);
                const float mc = fmaf(h16(c1 >> 16), mT, 0.0f);   // = mT f (masses are not negative)
                sumc = term_r2_acc<K>(make_float4(0.f, 0.f, 0.f, mc), zero4, ex, ey, ez, norm2(ex, ey, ez), kp, r0,
                                      sumc);
            }
            const bool cont = __builtin_amdgcn_inverse_ballot_w64(contm);
            const float prr2 = prr * p;
            const float acc2 = acc + (sumc - tT) * (fna * frcp((float)nT * prr2));
            prr = cont ? prr2 : prr;
            acc = cont ? acc2 : acc;
            tT = cont ? tC : tT;
            steps += cont ? 1 : 0;
            dT = dC;
            dTx = cx;
            dTy = cy;
            dTz = cz;
            mT = mC;
            nT = nC;
            beginT = beginC;
            blk = blkC;
            ++level;
            diamT *= kInvD;
            sideC *= kInvD;
            ++k;
        }
        go = actm != 0ull && (int)nT > tv.leaf_size && level < tv.max_level;
    };
    while (go && k < 16) {
        internal_step(std::integral_constant<int, 0>{});
        if (go) internal_step(std::integral_constant<int, 1>{});
    }
    while (go) internal_step(std::integral_constant<int, 2>{});
    if (actm != 0ull) {
        // a leaf (one point included): its points are the virtual children, one drawn uniformly
        uint32_t xsel;
        float u;
        pw.step(k, ctr1, ctr0, ctr3, key0, key1, xsel, u);
        const uint32_t r = __umulhi(xsel, nT);
        const float4 aggC = gld4(at_off(tv.pts, (Off)(beginT + r) * (Off)16));
        float dC;
        const float cx = aggC.x - qx, cy = aggC.y - qy, cz = aggC.z - qz;
        const float r2C = norm2(cx, cy, cz);
        const float p = roulette(r2C, dC);
        const uint64_t contm = __ballot(u < p) & actm;
        if (__builtin_amdgcn_inverse_ballot_w64(actm & ~contm)) {
            flag = 0;
            end_b = (int32_t)beginT;
            end_l = level;
        }
        if (contm != 0ull) {
            float sumc = term_r2<K>(aggC, zero4, cx, cy, cz, r2C, kp, r0);
            for (uint32_t i = 0; i < nT; ++i) {
                if (i == r) continue;
                const Off po = (Off)(beginT + i) * (Off)16;
                sumc = term_acc<K>(gld4(at_off(tv.pts, po)), zero4, qx, qy, qz, kp, r0, sumc);
            }
            if (__builtin_amdgcn_inverse_ballot_w64(contm)) {
                prr *= p;
                acc += (sumc - tT) * (fna * frcp((float)nT * prr));
                ++steps;
                flag = 2;
                end_b = (int32_t)(beginT + r);
                end_l = level + 1;
            }
        }
    }
    if constexpr (TRACE) *rec = make_int4(end_b, end_l, steps, flag);
    return acc;
}

// One tile (64 consecutive queries) of the compressed walk: the root's
// subdomains decoded from the root block's codes (com^q_a - q = o_a s_1 +
// (com_0 - q), m^q_a = m_0 f_a, with com_0 and m_0 the root's float32
// aggregate), then wave_path_q per (subdomain, sample).  Two wavefronts per
// tile share the slots as k_sbh_wave's do.
template <int K, bool TRACE, int P, bool O64, int VM>
__device__ __forceinline__ void sbh_wave_tile_q(const TreeView& tv, const float* __restrict__ queries, int64_t nq,
                                                const SbhArgs& a, float* __restrict__ out, int64_t wave, int part,
                                                int w, float (*part_f)[64], uint32_t* done)
{
#pragma clang fp contract(off)
    constexpr int D3 = 8;
    const int lane = threadIdx.x & 63;
    const int64_t j0 = wave * 64;
    if (j0 >= nq) return;
    const int64_t j = j0 + lane;
    const bool valid = j < nq;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (valid) {
        qx = gld(queries + 3 * j);
        qy = gld(queries + 3 * j + 1);
        qz = gld(queries + 3 * j + 2);
    }
    KParams kp{a.eps2, a.alpha, 1.0f};
    float logwbar = 0.f, r0 = 0.f;
    if constexpr (K == SBH_SMOOTHDIST) {
        smooth_setup(tv, kp.wscale, logwbar);
        r0 = smooth_shift<2>(tv, qx, qy, qz, a.alpha);
    }
    const uint32_t stream = (uint32_t)(j0 / a.group);
    const uint32_t* __restrict__ rt = tv.btopo;
    const uint32_t* __restrict__ rq = reinterpret_cast<const uint32_t*>(tv.bq);
    const int32_t base_root = (int32_t)gld(rt + D3);
    const float4 g0 = gld4(tv.nagg);
    const float s1 = tv.side * 0.5f;   // the cell side of level 1
    const float ox0 = g0.x - qx, oy0 = g0.y - qy, oz0 = g0.z - qz;
    const int slot_lo = part * (D3 / P), slot_hi = slot_lo + D3 / P;
    uint32_t begin_a = 0u;
    int32_t nint = 0;
    for (int slot = 0; slot < slot_lo; ++slot) {
        const uint32_t n_a = gld(rt + slot);
        begin_a += n_a;
        nint += ((int)n_a > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
    }
    float F = 0.0f;
    PathWords pw;
    for (int slot = slot_lo; slot < slot_hi; ++slot) {
        const uint32_t n_a = gld(rt + slot);
        if (n_a == 0u) {
            if constexpr (TRACE) {
                if (valid)
                    for (int s = 0; s < a.samples; ++s)
                        reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)a.samples + s] = make_int4(-1, 0, 0, 0);
            }
            continue;
        }
        const int32_t blk_a = base_root + nint;
        const uint32_t w0 = gld(rq + 2 * slot), w1 = gld(rq + 2 * slot + 1);
        const float dax = fmaf(h16(w0 & 0xFFFFu), s1, ox0);
        const float day = fmaf(h16(w0 >> 16), s1, oy0);
        const float daz = fmaf(h16(w1 & 0xFFFFu), s1, oz0);
        const float m_a = g0.w * h16(w1 >> 16);
        const float cv = term_r2<K>(make_float4(0.f, 0.f, 0.f, m_a), make_float4(0.f, 0.f, 0.f, 0.f), dax, day, daz,
                                    norm2(dax, day, daz), kp, r0);   // control variate CV_a
        float fa = 0.0f;
        for (int s = 0; s < a.samples; ++s) {
            int4 rec;
            const uint32_t path = (uint32_t)(slot * a.samples + s);
            pw.need(path, stream, a.batch, a.key0, a.key1);
            fa += wave_path_q<K, TRACE, O64, VM>(tv, qx, qy, qz, r0, kp, valid, n_a, begin_a, blk_a, dax, day, daz, m_a,
                                             cv, pw, stream, path, a.batch, a.key0, a.key1, a.rr_mode, &rec);
            if constexpr (TRACE) {
                if (valid) reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)a.samples + s] = rec;
            }
        }
        F += cv + fa / (float)a.samples;
        begin_a += n_a;
        nint += ((int)n_a > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
    }
    if constexpr (P > 1) {
        const int tl = w / P;
        part_f[w][lane] = F;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        uint32_t prev = 0u;
        if (lane == 0) prev = __hip_atomic_fetch_add(&done[tl], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (__builtin_amdgcn_readfirstlane(prev) != (uint32_t)(P - 1)) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        F = part_f[tl * P][lane];
#pragma unroll
        for (int q = 1; q < P; ++q) F += part_f[tl * P + q][lane];
    }
    if (valid) gst(out + j, query_value<K>(F, r0, logwbar, a.alpha, qx, qy, qz));
}

template <int K, bool TRACE, bool O64, int VM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_sbh_wave_q(TreeView tv, const float* __restrict__ queries, int64_t nq, SbhArgs a, float* __restrict__ out)
{
    constexpr int P = kWaveParts, TPB = 4 / P;
    __shared__ float part_f[4][64];
    __shared__ uint32_t done[TPB];
    if constexpr (P > 1) {
        if (threadIdx.x < TPB) done[threadIdx.x] = 0u;
        __syncthreads();
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tile = (int64_t)blockIdx.x * TPB + w / P;
    sbh_wave_tile_q<K, TRACE, P, O64, VM>(tv, queries, nq, a, out, tile, w % P, w, part_f, done);
}

// ---------------------------------------------------------------------------
// The coherent walk with second-order node terms (d = 2, potential, uniform
// path index).  A node's term is its point-mass term plus, where the query
// sees it as far (|x| >= |B|, x = com - q), the next term of its Taylor
// expansion about the centre of mass:
//   m u + 1/2 u^5 (3 x^T Q x - tr(Q) (|x|^2 + eps^2)),  u = (|x|^2 + eps^2)^(-1/2),
// with Q the node's second-moment tensor, stored per child slot scaled as
// A = {1.5 Qxx, 1.5 Qyy, 1.5 Qzz, 3 Qxy}, {3 Qxz, 3 Qyz, tr(Q) / 2}, so that
// the term is m u + u^5 (x^T A x - h (|x|^2 + eps^2)).  Points stay exact
// (their tensor is zero), so a one-point node ends the walk as in wave_path.
// Selection, random words and roulette are those of wave_path.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float term_l2(float m, float4 qa, float4 qb, float dx, float dy, float dz, float r2,
                                         float diam2, float eps2)
{
#pragma clang fp contract(off)
    const float s2 = r2 + eps2;
    const float u = __builtin_amdgcn_rsqf(s2);
    const float xa = fmaf(qa.x, dx, fmaf(qa.w, dy, qb.x * dz));
    const float ya = fmaf(qa.y, dy, qb.y * dz);
    const float xax = fmaf(dx, xa, fmaf(dy, ya, qa.z * (dz * dz)));
    const float u2 = u * u;
    const float c = (u2 * u2 * u) * fmaf(-qb.z, s2, xax);
    return fmaf(m, u, r2 >= diam2 ? c : 0.0f);
}

template <bool TRACE, bool O64, int VM>
__device__ __forceinline__ float wave_path_l2(const TreeView& tv, float qx, float qy, float qz, const KParams& kp,
                                              bool valid, uint32_t n_a, uint32_t begin_a, int32_t blk_a, float4 agg_a,
                                              float t_a, const PathWords& pw, uint32_t ctr0, uint32_t ctr1,
                                              uint32_t ctr3, uint32_t key0, uint32_t key1, int rr_mode, int4* rec)
{
#pragma clang fp contract(off)
    constexpr int D3 = 8;
    constexpr int TS = topo_stride(D3);
    constexpr float kInvD = 0.5f;
    using Off = typename TreeOff<O64>::T;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t nT = n_a, beginT = begin_a;
    int32_t blk = blk_a;
    int level = 1;
    float diamT = tv.diam0 * kInvD;
    const float fna = (float)n_a;
    uint64_t actm = __ballot(valid);
    float dT = fsqrt(norm2(agg_a.x - qx, agg_a.y - qy, agg_a.z - qz));
    float tT = t_a, prr = 1.0f, acc = 0.0f;
    int steps = 0, flag = 0;
    int32_t end_b = (int32_t)beginT, end_l = level;
    const bool rr_eq5 = VM != 2 || rr_mode == 0;   // VM: the roulette, as in wave_path
    const float rr_fixed = rr_mode == 1 ? 1.0f : 0.5f;
    // rr_mode 3: Eq. (5) voted over the wavefront (the largest p of its queries with finite
    // coordinates, the same for every lane, so the wavefront stops or continues as one)
    constexpr bool rr_vote = VM == 1;
    const bool voter = valid && __builtin_isfinite(qx) && __builtin_isfinite(qy) && __builtin_isfinite(qz);
    auto roulette = [&](float r2C, float& dC) -> float {
        const float ic = __builtin_amdgcn_rsqf(r2C);
        dC = r2C * ic;
        const float p5 = fminf(1.0f, vmax(diamT, dT) * (kInvD * ic));
        float p = rr_eq5 ? p5 : rr_fixed;
        if (rr_vote) p = wave_max_nonneg(voter ? p : 0.0f);
        return p;
    };
    int k = 0;
    bool go = actm != 0ull && (int)nT > tv.leaf_size && level < tv.max_level;
    const int lvl_int = tv.max_level - 1;
    auto internal_step = [&](auto mode) {
        constexpr int M = decltype(mode)::value;
        uint32_t xsel;
        float u;
        if constexpr (M == 2) pw.step_late(k, ctr1, ctr0, ctr3, key0, key1, xsel, u);
        else pw.template step_held<M == 1>(k, ctr1, xsel, u);
        const uint32_t r = __umulhi(xsel, nT);
        const Off boff = (Off)(uint32_t)blk * (Off)(D3 * 16);   // the block's aggregates
        const Off qoff = (Off)(uint32_t)blk * (Off)(D3 * 32);   // and its tensors
        const Off toff = (Off)(uint32_t)blk * (Off)(TS * 4);
        const uint32_t* __restrict__ bt = at_off(tv.btopo, toff);
        const int ln = threadIdx.x & 63;
        const uint32_t cl = gld(bt + (ln < D3 ? ln : TS - 1));
        uint32_t inc = cl;
        inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x111, 0xF, 0xF, false);   // row_shr:1
        inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x112, 0xF, 0xF, false);   // row_shr:2
        inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x114, 0xF, 0xF, false);   // row_shr:4
        const uint32_t excl = inc - cl;
        const uint32_t hm = (uint32_t)__ballot((r - excl) < cl);
        const uint32_t im = level < lvl_int ? (uint32_t)__ballot((int)cl > tv.leaf_size) : 0u;
        const uint32_t nonempty = (uint32_t)__ballot(cl != 0u);
        const int csel = __builtin_ctz(hm);
        const uint32_t preC = (uint32_t)__builtin_amdgcn_readlane((int)excl, csel);
        const uint32_t nC = (uint32_t)__builtin_amdgcn_readlane((int)cl, csel);
        const int32_t nintC = __popc(im & ((1u << csel) - 1u));
        const float4 aggC = gld4(at_off(tv.bagg, boff + (Off)(csel * 16)));
        const uint32_t beginC = beginT + preC;
        const int32_t blkC = (int32_t)gld(bt + D3) + nintC;
        float dC;
        const float cx = aggC.x - qx, cy = aggC.y - qy, cz = aggC.z - qz;
        const float r2C = norm2(cx, cy, cz);
        const float p = roulette(r2C, dC);
        const uint64_t contm = __ballot(u < p) & actm;
        if (__builtin_amdgcn_inverse_ballot_w64(actm & ~contm)) {
            flag = 0;
            end_b = (int32_t)beginT;
            end_l = level;
        }
        actm = contm;
        if (contm != 0ull) {
            // contribution swap, Eq. (6), with second-order terms
            const float diamC = diamT * kInvD, d2C = diamC * diamC;
            const float4* __restrict__ bqd = at_off(tv.bquad, qoff);
            const float tC = term_l2(aggC.w, gld4(bqd + 2 * csel), gld4(bqd + 2 * csel + 1), cx, cy, cz, r2C, d2C,
                                     kp.eps2);
            float sumc = tC;
            const float4* __restrict__ ba = at_off(tv.bagg, boff);
            float4 g8[D3];
#pragma unroll
            for (int c = 0; c < D3; ++c) g8[c] = gld4(ba + c);
            const uint32_t rest = nonempty & ~(1u << csel);
#pragma unroll
            for (int c = 0; c < D3; ++c) {
                if (!((rest >> c) & 1u)) continue;
                const float ex = g8[c].x - qx, ey = g8[c].y - qy, ez = g8[c].z - qz;
                sumc += term_l2(g8[c].w, gld4(bqd + 2 * c), gld4(bqd + 2 * c + 1), ex, ey, ez, norm2(ex, ey, ez), d2C,
                                kp.eps2);
            }
            const bool cont = __builtin_amdgcn_inverse_ballot_w64(contm);
            const float prr2 = prr * p;
            const float acc2 = acc + (sumc - tT) * (fna * frcp((float)nT * prr2));
            prr = cont ? prr2 : prr;
            acc = cont ? acc2 : acc;
            tT = cont ? tC : tT;
            steps += cont ? 1 : 0;
            dT = dC;
            nT = nC;
            beginT = beginC;
            blk = blkC;
            ++level;
            diamT *= kInvD;
            ++k;
        }
        go = actm != 0ull && (int)nT > tv.leaf_size && level < tv.max_level;
    };
    while (go && k < 16) {
        internal_step(std::integral_constant<int, 0>{});
        if (go) internal_step(std::integral_constant<int, 1>{});
    }
    while (go) internal_step(std::integral_constant<int, 2>{});
    if (actm != 0ull) {
        if (nT == 1u) {   // a single point: its node term is exact (a zero tensor)
            if (__builtin_amdgcn_inverse_ballot_w64(actm)) { flag = 1; end_b = (int32_t)beginT; end_l = level; }
        } else {          // a leaf: its points are the virtual children, one drawn uniformly
            uint32_t xsel;
            float u;
            pw.step(k, ctr1, ctr0, ctr3, key0, key1, xsel, u);
            const uint32_t r = __umulhi(xsel, nT);
            const float4 aggC = gld4(at_off(tv.pts, (Off)(beginT + r) * (Off)16));
            float dC;
            const float cx = aggC.x - qx, cy = aggC.y - qy, cz = aggC.z - qz;
            const float r2C = norm2(cx, cy, cz);
            const float p = roulette(r2C, dC);
            const uint64_t contm = __ballot(u < p) & actm;
            if (__builtin_amdgcn_inverse_ballot_w64(actm & ~contm)) {
                flag = 0;
                end_b = (int32_t)beginT;
                end_l = level;
            }
            if (contm != 0ull) {
                float sumc = term_r2<SBH_POTENTIAL>(aggC, zero4, cx, cy, cz, r2C, kp, 0.0f);
                for (uint32_t i = 0; i < nT; ++i) {
                    if (i == r) continue;
                    const Off po = (Off)(beginT + i) * (Off)16;
                    sumc = term_acc<SBH_POTENTIAL>(gld4(at_off(tv.pts, po)), zero4, qx, qy, qz, kp, 0.0f, sumc);
                }
                if (__builtin_amdgcn_inverse_ballot_w64(contm)) {
                    prr *= p;
                    acc += (sumc - tT) * (fna * frcp((float)nT * prr));
                    ++steps;
                    flag = 2;
                    end_b = (int32_t)(beginT + r);
                    end_l = level + 1;
                }
            }
        }
    }
    if constexpr (TRACE) *rec = make_int4(end_b, end_l, steps, flag);
    return acc;
}

// One tile of 64 consecutive queries of the second-order walk (two wavefronts
// per tile share the slots as k_sbh_wave's do).
template <bool TRACE, int P, bool O64, int VM>
__device__ __forceinline__ void sbh_wave_tile_l2(const TreeView& tv, const float* __restrict__ queries, int64_t nq,
                                                 const SbhArgs& a, float* __restrict__ out, int64_t wave, int part,
                                                 int w, float (*part_f)[64], uint32_t* done)
{
#pragma clang fp contract(off)
    constexpr int D3 = 8;
    const int lane = threadIdx.x & 63;
    const int64_t j0 = wave * 64;
    if (j0 >= nq) return;
    const int64_t j = j0 + lane;
    const bool valid = j < nq;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (valid) {
        qx = gld(queries + 3 * j);
        qy = gld(queries + 3 * j + 1);
        qz = gld(queries + 3 * j + 2);
    }
    KParams kp{a.eps2, a.alpha, 1.0f};
    const uint32_t stream = (uint32_t)(j0 / a.group);
    const uint32_t* __restrict__ rt = tv.btopo;
    const int32_t base_root = (int32_t)gld(rt + D3);
    const float diam1 = tv.diam0 * 0.5f, d21 = diam1 * diam1;
    const int slot_lo = part * (D3 / P), slot_hi = slot_lo + D3 / P;
    uint32_t begin_a = 0u;
    int32_t nint = 0;
    for (int slot = 0; slot < slot_lo; ++slot) {
        const uint32_t n_a = gld(rt + slot);
        begin_a += n_a;
        nint += ((int)n_a > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
    }
    float F = 0.0f;
    PathWords pw;
    for (int slot = slot_lo; slot < slot_hi; ++slot) {
        const uint32_t n_a = gld(rt + slot);
        if (n_a == 0u) {
            if constexpr (TRACE) {
                if (valid)
                    for (int s = 0; s < a.samples; ++s)
                        reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)a.samples + s] = make_int4(-1, 0, 0, 0);
            }
            continue;
        }
        const int32_t blk_a = base_root + nint;
        const float4 agg_a = gld4(tv.bagg + slot);
        const float dx = agg_a.x - qx, dy = agg_a.y - qy, dz = agg_a.z - qz;
        const float cv = term_l2(agg_a.w, gld4(tv.bquad + 2 * slot), gld4(tv.bquad + 2 * slot + 1), dx, dy, dz,
                                 norm2(dx, dy, dz), d21, kp.eps2);   // control variate CV_a
        float fa = 0.0f;
        for (int s = 0; s < a.samples; ++s) {
            int4 rec;
            const uint32_t path = (uint32_t)(slot * a.samples + s);
            pw.need(path, stream, a.batch, a.key0, a.key1);
            fa += wave_path_l2<TRACE, O64, VM>(tv, qx, qy, qz, kp, valid, n_a, begin_a, blk_a, agg_a, cv, pw, stream, path,
                                           a.batch, a.key0, a.key1, a.rr_mode, &rec);
            if constexpr (TRACE) {
                if (valid) reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)a.samples + s] = rec;
            }
        }
        F += cv + fa / (float)a.samples;
        begin_a += n_a;
        nint += ((int)n_a > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
    }
    if constexpr (P > 1) {
        const int tl = w / P;
        part_f[w][lane] = F;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        uint32_t prev = 0u;
        if (lane == 0) prev = __hip_atomic_fetch_add(&done[tl], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (__builtin_amdgcn_readfirstlane(prev) != (uint32_t)(P - 1)) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        F = part_f[tl * P][lane];
#pragma unroll
        for (int q = 1; q < P; ++q) F += part_f[tl * P + q][lane];
    }
    if (valid) gst(out + j, query_value<SBH_POTENTIAL>(F, 0.0f, 0.0f, a.alpha, qx, qy, qz));
}

template <bool TRACE, bool O64, int VM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_sbh_wave_l2(TreeView tv, const float* __restrict__ queries, int64_t nq, SbhArgs a, float* __restrict__ out)
{
    constexpr int P = kWaveParts, TPB = 4 / P;
    __shared__ float part_f[4][64];
    __shared__ uint32_t done[TPB];
    if constexpr (P > 1) {
        if (threadIdx.x < TPB) done[threadIdx.x] = 0u;
        __syncthreads();
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tile = (int64_t)blockIdx.x * TPB + w / P;
    sbh_wave_tile_l2<TRACE, P, O64, VM>(tv, queries, nq, a, out, tile, w % P, w, part_f, done);
}

// Sum over the 64 lanes of eight values per lane, in a fixed order, on the
// vector unit (no LDS): a swap between the wavefront's halves and one between
// row pairs (gfx950 lane-swap instructions) each halve the values a lane
// holds, a row rotation by 8 leaves lanes 8c .. 8c + 7 with value c, and a
// segmented shift-add scan leaves its total in lane 8c + 7.
__device__ __forceinline__ float wave_sum8(const float v[8])
{
    const int l = threadIdx.x & 63;
    float w4[4], w2[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {   // lanes 0..31 keep values 0..3, lanes 32..63 values 4..7
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[4 + i]), false, false);
        w4[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {   // rows 0..3 keep values (0, 1), (2, 3), (4, 5), (6, 7)
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w4[i]), __float_as_uint(w4[2 + i]), false, false);
        w2[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool b3 = (l >> 3) & 1;
    const float keep = b3 ? w2[1] : w2[0], send = b3 ? w2[0] : w2[1];
    float w = keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), 0x128, 0xF, 0xF, false));  // row_ror:8
    w += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(w), 0x111, 0xF, 0xF, true));   // row_shr:1
    w += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(w), 0x112, 0xF, 0xF, true));   // row_shr:2
    w += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(w), 0x114, 0xF, 0xF, true));   // row_shr:4
    return w;
}

// The coherent walk with the tile-shared score proposal (d = 2): at an
// internal node every lane computes its own score proposal pi_c (the
// relative quadrupole scores of the children, floored at e^-16), the
// wavefront averages them over its valid lanes (the tile of 64 consecutive
// queries), and the shared path draws the child from
//   q_c = (1 - 1/8) mean pi_c + (1/8) n_c / n_T,
// so that the walk stays shared; each lane's swap is divided by the product
// of the q's drawn (Eq. (7) with p(I in T) = prod q).  The child block is
// scanned before the selection (its distances feed the scores).
template <int K, bool TRACE, bool O64>
__device__ __forceinline__ float wave_path_tile(const TreeView& tv, float qx, float qy, float qz, float r0,
                                                const KParams& kp, bool valid, float inv_valid, uint32_t n_a,
                                                uint32_t begin_a, int32_t blk_a, float4 agg_a, float t_a,
                                                const PathWords& pw, uint32_t ctr0, uint32_t ctr1, uint32_t ctr3,
                                                uint32_t key0, uint32_t key1, int rr_mode, int4* rec)
{
#pragma clang fp contract(off)
    constexpr int D3 = 8;
    constexpr int TS = topo_stride(D3);
    constexpr float kLam = 0.125f;
    using Off = typename TreeOff<O64>::T;   // byte offsets into the tree's arrays, as in wave_path
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int ln = threadIdx.x & 63;
    uint32_t nT = n_a, beginT = begin_a;
    int32_t blk = blk_a;
    int level = 1;
    float diamT = tv.diam0 * 0.5f;
    uint64_t actm = __ballot(valid);   // lanes still walking, as a lane mask (a lane's flag is its bit)
    const bool rr_eq5 = rr_mode == 0;
    const float rr_fixed = rr_mode == 1 ? 1.0f : 0.5f;
    float dT = fsqrt(norm2(agg_a.x - qx, agg_a.y - qy, agg_a.z - qz));
    float tT = t_a, prr = 1.0f, psel = 1.0f, acc = 0.0f;
    int steps = 0, flag = 0;
    int32_t end_b = (int32_t)beginT, end_l = level;
    for (int k = 0; actm != 0ull; ++k) {   // later steps leave by the roulette's vote
        if (nT == 1u) {
            if (__builtin_amdgcn_inverse_ballot_w64(actm)) { flag = 1; end_b = (int32_t)beginT; end_l = level; }
            break;
        }
        uint32_t xsel;
        float u;
        pw.step(k, ctr1, ctr0, ctr3, key0, key1, xsel, u);
        const bool internal = (int)nT > tv.leaf_size && level < tv.max_level;
        float4 aggC, dpC = zero4;
        uint32_t nC = 1u, beginC;
        int32_t blkC = 0;
        float qsel;
        uint32_t rleaf = 0u;
        uint32_t nonempty = 0u;   // slots with points (wavefront-uniform)
        int csel = 0;
        float4 g8[D3];            // the block's aggregates, kept for the swap
        float r2[D3];             // this lane's squared distances to them, shared by score and term
        if (internal) {
            const Off boff = (Off)(uint32_t)blk * (Off)(D3 * 16);
            const float4* __restrict__ ba = at_off(tv.bagg, boff);
            const float* __restrict__ bs = at_off(tv.bspr, (Off)(uint32_t)blk * (Off)(D3 * 4));
            const uint32_t* __restrict__ bt = at_off(tv.btopo, (Off)(uint32_t)blk * (Off)(TS * 4));
            // counts in lanes 0..7 (lanes 8..63 read the row's zero padding word)
            const uint32_t cl = gld(bt + (ln < D3 ? ln : TS - 1));
            uint32_t inc = cl;
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x111, 0xF, 0xF, false);
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x112, 0xF, 0xF, false);
            inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x114, 0xF, 0xF, false);
            const uint32_t excl = inc - cl;
            const uint32_t im = level + 1 < tv.max_level ? (uint32_t)__ballot((int)cl > tv.leaf_size) : 0u;
            nonempty = (uint32_t)__ballot(cl != 0u);
            // this lane's scores from the block (one batch of scalar loads); the terms of the
            // swap wait until the roulette has kept some lane
            float s8[D3], pi[D3];
#pragma unroll
            for (int c = 0; c < D3; ++c) {
                g8[c] = gld4(ba + c);
                s8[c] = gld(bs + c);
            }
            float smax = 0.0f;
#pragma unroll
            for (int c = 0; c < D3; ++c) {
                pi[c] = 0.0f;
                r2[c] = 0.0f;
                if (!((nonempty >> c) & 1u)) continue;
                r2[c] = norm2(g8[c].x - qx, g8[c].y - qy, g8[c].z - qz);
                const float x = r2[c] + s8[c];
                const float rs = x > 0.0f ? __builtin_amdgcn_rsqf(x) : 0.0f;
                pi[c] = g8[c].w * s8[c] * (rs * rs * rs);
                smax = fmaxf(smax, pi[c]);
            }
            // every slot takes the same instructions, with no branch: an empty slot's score is 0
            // and its floor 0; a lane whose scores are all 0 gets 1 for every non-empty slot
            constexpr float kFloor = 1.12535175e-7f;   // e^-16
            const bool pos = smax > 0.0f;
            const float inv = pos ? frcp(smax) : 0.0f;
            const float fl = pos ? kFloor : 1.0f;
            float tot = 0.0f;
#pragma unroll
            for (int c = 0; c < D3; ++c) {
                pi[c] = fmaxf(pi[c] * inv, ((nonempty >> c) & 1u) ? fl : 0.0f);
                tot += pi[c];
            }
            const float invt = valid ? frcp(tot) : 0.0f;   // lanes past the end of the query set add nothing
#pragma unroll
            for (int c = 0; c < D3; ++c) pi[c] *= invt;
            const float msum = wave_sum8(pi);                 // lane 8c + 7 holds the sum of pi_c
            // q and the inverse-CDF selection across lanes 0..7, one slot each: lane c takes its
            // slot's tile sum from lane 8c + 7 and forms q_c (zero for an empty slot); an
            // inclusive scan gives the running totals, and the first lane whose total exceeds
            // u is the selected slot (the last non-empty one if rounding left the total below u)
            const float u_sel = unit24(xsel);
            const float fnT = frcp((float)nT);
            const float mc = __int_as_float(__builtin_amdgcn_ds_bpermute(((8 * ln + 7) & 63) << 2, __float_as_int(msum)));
            const float qc = ln < D3 ? (1.0f - kLam) * (mc * inv_valid) + kLam * ((float)cl * fnT) : 0.0f;
            float cum = qc;
            cum += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(cum), 0x111, 0xF, 0xF, true));   // row_shr:1
            cum += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(cum), 0x112, 0xF, 0xF, true));   // row_shr:2
            cum += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(cum), 0x114, 0xF, 0xF, true));   // row_shr:4
            const uint64_t hit = __ballot(u_sel < cum) & ((1ull << D3) - 1ull);
            csel = hit ? __ffsll((unsigned long long)hit) - 1 : 31 - __builtin_clz(nonempty);
            qsel = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qc), csel));
            const uint32_t preC = (uint32_t)__builtin_amdgcn_readlane((int)excl, csel);
            nC = (uint32_t)__builtin_amdgcn_readlane((int)cl, csel);
            aggC = gld4(at_off(tv.bagg, boff + (Off)(csel * 16)));
            if constexpr (K == SBH_WINDING) dpC = gld4(at_off(tv.bdip, boff + (Off)(csel * 16)));
            beginC = beginT + preC;
            blkC = (int32_t)gld(bt + D3) + __popc(im & ((1u << csel) - 1u));
        } else {
            rleaf = __umulhi(xsel, nT);
            aggC = gld4(at_off(tv.pts, (Off)(beginT + rleaf) * (Off)16));
            if constexpr (K == SBH_WINDING) dpC = gld4(at_off(tv.pdip, (Off)(beginT + rleaf) * (Off)16));
            beginC = beginT + rleaf;
            qsel = frcp((float)nT);
        }
        // roulette (Eq. (5)); its offset and squared distance also give the selected child's
        // own term, bit for bit the value the swap's sum takes for it
        const float cx = aggC.x - qx, cy = aggC.y - qy, cz = aggC.z - qz;
        const float r2C = norm2(cx, cy, cz);
        const float ic = __builtin_amdgcn_rsqf(r2C);   // |c - q| and 1 / (2 |c - q|) from one rsq, as in wave_path
        const float dC = r2C * ic;
        const float p5 = fminf(1.0f, vmax(diamT, dT) * (0.5f * ic));
        const float p = rr_eq5 ? p5 : rr_fixed;   // the roulette mode as a select
        const uint64_t contm = __ballot(u < p) & actm;
        const bool cont = __builtin_amdgcn_inverse_ballot_w64(contm);
        if (__builtin_amdgcn_inverse_ballot_w64(actm & ~contm)) {
            flag = 0;
            end_b = (int32_t)beginT;
            end_l = level;
        }
        if (contm == 0ull) break;
        // the selected child's own term opens the swap's sum (and is the next step's
        // control variate), the other non-empty children follow
        const float tC = term_r2<K>(aggC, dpC, cx, cy, cz, r2C, kp, r0);
        float sumc = tC;
        if (internal) {   // contribution swap over the non-empty children, Eq. (6)
            const float4* __restrict__ bd = at_off(tv.bdip, (Off)(uint32_t)blk * (Off)(D3 * 16));
            const uint32_t rest = nonempty & ~(1u << csel);
#pragma unroll
            for (int c = 0; c < D3; ++c) {
                if (!((rest >> c) & 1u)) continue;
                const float4 gd = (K == SBH_WINDING) ? gld4(bd + c) : zero4;
                sumc = term_r2_acc<K>(g8[c], gd, g8[c].x - qx, g8[c].y - qy, g8[c].z - qz, r2[c], kp, r0, sumc);
            }
        } else {   // leaf: its points are the virtual children
            for (uint32_t i = 0; i < nT; ++i) {
                if (i == rleaf) continue;   // the selected point: its term opened the sum
                const Off po = (Off)(beginT + i) * (Off)16;
                const float4 g = gld4(at_off(tv.pts, po));
                const float4 gd = (K == SBH_WINDING) ? gld4(at_off(tv.pdip, po)) : zero4;
                sumc = term_acc<K>(g, gd, qx, qy, qz, kp, r0, sumc);
            }
        }
        {   // the lanes the roulette keeps take the step (selects, not a branch)
            const float prr2 = prr * p;
            const float acc2 = acc + (sumc - tT) * frcp(psel * prr2);
            prr = cont ? prr2 : prr;
            acc = cont ? acc2 : acc;
            tT = cont ? tC : tT;
            steps += cont ? 1 : 0;
        }
        psel *= qsel;
        if (!internal) {
            if (cont) {
                flag = 2;
                end_b = (int32_t)beginC;
                end_l = level + 1;
            }
            break;
        }
        actm = contm;
        dT = dC;
        nT = nC;
        beginT = beginC;
        blk = blkC;
        ++level;
        diamT *= 0.5f;
    }
    if constexpr (TRACE) *rec = make_int4(end_b, end_l, steps, flag);
    return acc;
}

// One wavefront-tile of 64 consecutive queries (j = 64 wave + lane) with the
// shared walk; used by the single-tree kernel and by the batched kernel.
// TILE: the tile-shared score proposal (d = 2) instead of the uniform path index.
// A tile's root slots may be split over P wavefronts of one workgroup: part p
// takes slots [p D^3 / P, (p + 1) D^3 / P) and keeps its own sum; the last
// part of the tile to finish adds the P sums in part order and writes the
// output.  This shortens the chain of dependent steps one wavefront walks
// (the launch's floor on its duration) at the price of one more Philox
// evaluation per part.  LDS: part_f [wavefronts of the block][64] and one
// counter per tile of the block in `done`, zeroed before the block's first
// barrier.  four (P = 2, d = 2: the last tiles of a launch): the tile is
// split over four wavefronts of two slots each, which store each slot's
// total in part_f [slot][64]; the last of them adds the totals in the
// association of two parts (slots 0-3 in order, slots 4-7 in order, then
// the two sums), so a query's value does not depend on how its tile was
// split.  (A run-time choice: one inlined walk serves both splits.)
template <int D, int K, bool TRACE, bool TILE = false, int P = 1, bool O64 = false, int VM = 2, bool SPLIT = false>
__device__ __forceinline__ void sbh_wave_tile(const TreeView& tv, const float* __restrict__ queries, int64_t nq,
                                              const SbhArgs& a, float* __restrict__ out, int64_t wave, int part = 0,
                                              int w = 0, float (*part_f)[64] = nullptr, uint32_t* done = nullptr,
                                              bool four = false)
{
#pragma clang fp contract(off)
    constexpr int D3 = D * D * D;
    static_assert(D3 % P == 0, "parts must split the root slots evenly");
    constexpr bool kFour = SPLIT && D == 2 && P == 2;   // the four-way split is compiled in
    if constexpr (!kFour) four = false;
    const int lane = threadIdx.x & 63;
    const int64_t j0 = wave * 64;
    if (j0 >= nq) return;
    const int64_t j = j0 + lane;
    const bool valid = j < nq;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (valid) {
        qx = gld(queries + 3 * j);
        qy = gld(queries + 3 * j + 1);
        qz = gld(queries + 3 * j + 2);
    }
    KParams kp{a.eps2, a.alpha, 1.0f};
    float logwbar = 0.f, r0 = 0.f;
    if constexpr (K == SBH_SMOOTHDIST) {
        smooth_setup(tv, kp.wscale, logwbar);
        r0 = smooth_shift<D>(tv, qx, qy, qz, a.alpha);
    }
    const uint32_t stream = (uint32_t)(j0 / a.group);   // a.group is a multiple of 64
    const float inv_valid = 1.0f / (float)__popcll(__ballot(valid));
    (void)inv_valid;
    const uint32_t* __restrict__ rt = tv.btopo;
    const int32_t base_root = (int32_t)gld(rt + D3);
    const int nslots = four ? 2 : D3 / P;
    const int slot_lo = part * nslots, slot_hi = slot_lo + nslots;
    uint32_t begin_a = 0u;
    int32_t nint = 0;
    for (int slot = 0; slot < slot_lo; ++slot) {   // points and internal blocks of the slots before the part
        const uint32_t n_a = gld(rt + slot);
        begin_a += n_a;
        nint += ((int)n_a > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
    }
    float F = 0.0f;
    PathWords pw;
    for (int slot = slot_lo; slot < slot_hi; ++slot) {
        const uint32_t n_a = gld(rt + slot);
        if (n_a == 0u) {
            if constexpr (TRACE) {
                if (valid)
                    for (int s = 0; s < a.samples; ++s)
                        reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)a.samples + s] = make_int4(-1, 0, 0, 0);
            }
            continue;
        }
        const int32_t blk_a = base_root + nint;
        const float4 agg_a = gld4(tv.bagg + slot);
        const float4 dip_a = (K == SBH_WINDING) ? gld4(tv.bdip + slot) : make_float4(0.f, 0.f, 0.f, 0.f);
        const float cv = term<K>(agg_a, dip_a, qx, qy, qz, kp, r0);  // control variate CV_a
        float fa = 0.0f;
        for (int s = 0; s < a.samples; ++s) {
            int4 rec;
            const uint32_t path = (uint32_t)(slot * a.samples + s);
            pw.need(path, stream, a.batch, a.key0, a.key1);
            if constexpr (TILE && D == 2)
                fa += wave_path_tile<K, TRACE, O64>(tv, qx, qy, qz, r0, kp, valid, inv_valid, n_a, begin_a, blk_a,
                                                    agg_a, cv, pw, stream, path, a.batch, a.key0, a.key1, a.rr_mode,
                                                    &rec);
            else
                fa += wave_path<D, K, TRACE, O64, PathWords, VM>(tv, qx, qy, qz, r0, kp, valid, n_a, begin_a, blk_a,
                                                                 agg_a, cv, pw,
                                                  stream, path, a.batch, a.key0, a.key1, a.rr_mode, &rec);
            if constexpr (TRACE) {
                if (valid) reinterpret_cast<int4*>(a.paths)[(j * D3 + slot) * (int64_t)a.samples + s] = rec;
            }
        }
        const float vs = cv + fa / (float)a.samples;
        if (kFour && four) part_f[slot][lane] = vs;
        else F += vs;
        begin_a += n_a;
        nint += ((int)n_a > tv.leaf_size && 1 < tv.max_level) ? 1 : 0;
    }
    if (kFour && four) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        uint32_t prev = 0u;
        if (lane == 0) prev = __hip_atomic_fetch_add(&done[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (__builtin_amdgcn_readfirstlane(prev) != 3u) return;   // another part finishes the tile
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        float fa_lo = 0.0f, fa_hi = 0.0f;
#pragma unroll
        for (int slot = 0; slot < 4; ++slot)
            if (gld(rt + slot) != 0u) fa_lo += part_f[slot][lane];
#pragma unroll
        for (int slot = 4; slot < 8; ++slot)
            if (gld(rt + slot) != 0u) fa_hi += part_f[slot][lane];
        F = fa_lo + fa_hi;
    } else if constexpr (P > 1) {
        const int tl = w / P;   // the tile's index within the block
        part_f[w][lane] = F;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        uint32_t prev = 0u;
        if (lane == 0) prev = __hip_atomic_fetch_add(&done[tl], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (__builtin_amdgcn_readfirstlane(prev) != (uint32_t)(P - 1)) return;   // another part finishes the tile
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        F = part_f[tl * P][lane];
#pragma unroll
        for (int q = 1; q < P; ++q) F += part_f[tl * P + q][lane];
    }
    if (valid) gst(out + j, query_value<K>(F, r0, logwbar, a.alpha, qx, qy, qz));
}

// Tiles below split_tile: TPB tiles per block, each over kWaveParts wavefronts;
// from split_tile on (d = 2, the end of the launch, where the last wavefronts
// run on a partly idle chip): one tile per block over all four wavefronts,
// which halves the chain of steps each of them walks.
template <int D, int K, bool TRACE, bool O64, int VM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_sbh_wave(TreeView tv, const float* __restrict__ queries, int64_t nq, SbhArgs a, float* __restrict__ out,
           int64_t split_tile)
{
    constexpr int P = kWaveParts, TPB = 4 / P;   // 4 wavefronts per block, TPB tiles
    static_assert(P == 2, "the tail split assumes two parts per tile");
    __shared__ float part_f[D == 2 ? 8 : 4][64];
    __shared__ uint32_t done[TPB];
    if (threadIdx.x < TPB) done[threadIdx.x] = 0u;
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nb2 = split_tile / TPB;
    const bool four = D == 2 && (int64_t)blockIdx.x >= nb2;
    const int64_t tile = four ? split_tile + ((int64_t)blockIdx.x - nb2) : (int64_t)blockIdx.x * TPB + w / P;
    sbh_wave_tile<D, K, TRACE, false, P, O64, VM, true>(tv, queries, nq, a, out, tile, four ? w : w % P, w, part_f,
                                                        done, four);
}

// Tiles of the launch's four-part tail (d = 2): kTailTiles, or SBH_TAIL_TILES
// from the environment (a tuning override; values are the same for any split).
constexpr int64_t kTailTiles = 1024;
static int64_t tail_tiles()
{
    const char* e = std::getenv("SBH_TAIL_TILES");
    if (e && e[0]) {
        const long long v = std::atoll(e);
        return v < 0 ? 0 : (int64_t)v;
    }
    return kTailTiles;
}

// the coherent walk with the tile-shared score proposal (d = 2)
template <int K, bool TRACE, bool O64>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_sbh_wave_tile(TreeView tv, const float* __restrict__ queries, int64_t nq, SbhArgs a, float* __restrict__ out)
{
    constexpr int P = kWaveParts, TPB = 4 / P;   // as k_sbh_wave
    __shared__ float part_f[4][64];
    __shared__ uint32_t done[TPB];
    if constexpr (P > 1) {
        if (threadIdx.x < TPB) done[threadIdx.x] = 0u;
        __syncthreads();
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tile = (int64_t)blockIdx.x * TPB + w / P;
    sbh_wave_tile<2, K, TRACE, true, P, O64>(tv, queries, nq, a, out, tile, w % P, w, part_f, done);
}

// ---------------------------------------------------------------------------
// Barnes-Hut with wavefront voting
// ---------------------------------------------------------------------------
struct BhArgs {
    float beta;
    float eps2, alpha;
};

template <int D>
constexpr int bh_stack_depth()
{
    return D == 2 ? (8 - 1) * 20 + 2 : (64 - 1) * 10 + 2;
}

template <int D, int K, bool O64>
__global__ void __launch_bounds__(256) k_bh(TreeView tv, const float* __restrict__ queries, int64_t nq, BhArgs a,
                                            float* __restrict__ out)
{
#pragma clang fp contract(off)
    constexpr int D3 = D * D * D;
    constexpr int TS = topo_stride(D3);
    using Off = typename TreeOff<O64>::T;   // byte offsets into the tree's arrays, as in the walks
    constexpr int MAXS = bh_stack_depth<D>();
    // an entry is a child block to open: {block id, first point} and, apart, the level of its
    // node (block ids take all 32 bits; levels are below 64)
    __shared__ int2 stack[256 / 64][MAXS];
    __shared__ uint8_t stack_lvl[256 / 64][MAXS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (((int64_t)blockIdx.x * blockDim.x + wv * 64) >= nq) return;
    const bool valid = j < nq;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (valid) {
        qx = queries[3 * j];
        qy = queries[3 * j + 1];
        qz = queries[3 * j + 2];
    }
    // a query with a non-finite coordinate has no value (NaN) and takes no part in the vote, so
    // the cut its wavefront neighbours get is the one they would get without it
    const bool votes = valid && __builtin_isfinite(qx) && __builtin_isfinite(qy) && __builtin_isfinite(qz);
    KParams kp{a.eps2, a.alpha, 1.0f};
    float logwbar = 0.f, r0 = 0.f;
    if constexpr (K == SBH_SMOOTHDIST) {
        smooth_setup(tv, kp.wscale, logwbar);
        r0 = smooth_shift<D>(tv, qx, qy, qz, a.alpha);
    }
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    float acc = 0.0f;
    int sp = 0;
    // root: accepted when every lane passes the far-field test
    {
        const float4 g = tv.nagg[0];
        const float dx = g.x - qx, dy = g.y - qy, dz = g.z - qz;
        const float lim = a.beta * tv.diam0;   // |q - com| / |B| >= beta, squared
        const bool near = votes && !(norm2(dx, dy, dz) >= lim * lim);
        if (__ballot(near) == 0ull) {
            acc = term<K>(g, (K == SBH_WINDING) ? tv.ndip[0] : zero4, qx, qy, qz, kp, r0);
        } else if (!tv.root_internal) {
            for (int i = 0; i < tv.n_points; ++i)
                acc = term_acc<K>(tv.pts[i], (K == SBH_WINDING) ? tv.pdip[i] : zero4, qx, qy, qz, kp, r0, acc);
        } else {
            if (lane == 0) {
                stack[wv][0] = make_int2(0, 0);   // block 0, first point 0
                stack_lvl[wv][0] = 0;             // the root's level
            }
            sp = 1;
        }
    }
    __builtin_amdgcn_wave_barrier();
    while (sp > 0) {
        --sp;
        const int2 e = stack[wv][sp];
        const int32_t blk = __builtin_amdgcn_readfirstlane(e.x);
        const int level = __builtin_amdgcn_readfirstlane((int)stack_lvl[wv][sp]);
        uint32_t pre = (uint32_t)__builtin_amdgcn_readfirstlane(e.y);
        __builtin_amdgcn_wave_barrier();
        const float diamC = ldexpf(tv.diam0, -(level + 1) * (D == 2 ? 1 : 2));
        const float limC = a.beta * diamC;
        const Off boff = (Off)(uint32_t)blk * (Off)(D3 * 16);
        const float4* __restrict__ ba = at_off(tv.bagg, boff);
        const float4* __restrict__ bd = at_off(tv.bdip, boff);
        const uint32_t* __restrict__ bt = at_off(tv.btopo, (Off)(uint32_t)blk * (Off)(TS * 4));
        const int32_t base = (int32_t)bt[D3];
        int32_t nint = 0;
        for (int c = 0; c < D3; ++c) {
            const uint32_t cnt = bt[c];
            if (cnt == 0u) continue;
            const bool internal_c = (int)cnt > tv.leaf_size && level + 1 < tv.max_level;
            const float4 g = ba[c];
            const float dx = g.x - qx, dy = g.y - qy, dz = g.z - qz;
            const float r2 = norm2(dx, dy, dz);
            const bool near = votes && !(r2 >= limC * limC);
            if (__ballot(near) == 0ull) {
                acc = term_r2_acc<K>(g, (K == SBH_WINDING) ? bd[c] : zero4, dx, dy, dz, r2, kp, r0, acc);
            } else if (internal_c) {
                if (lane == 0) {
                    stack[wv][sp] = make_int2(base + nint, (int32_t)pre);
                    stack_lvl[wv][sp] = (uint8_t)(level + 1);
                }
                ++sp;
            } else {
                for (uint32_t i = pre; i < pre + cnt; ++i) {
                    const Off po = (Off)i * (Off)16;
                    acc = term_acc<K>(*at_off(tv.pts, po), (K == SBH_WINDING) ? *at_off(tv.pdip, po) : zero4, qx, qy,
                                      qz, kp, r0, acc);
                }
            }
            nint += internal_c ? 1 : 0;
            pre += cnt;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (valid) out[j] = query_value<K>(acc, r0, logwbar, a.alpha, qx, qy, qz);
}

// Stratification by a Barnes-Hut cut (Section 3.3.1 names the contribution
// nodes D(q, beta) of a low beta as path roots in place of the root's
// children).  One wavefront per 64 consecutive queries walks the tree
// depth-first as Barnes-Hut does (uniform LDS stack, scalar block loads): a
// child that every valid query of the wavefront sees as far (far-field ratio
// >= beta_low) is a subdomain, whose control variate and S coherent path
// samples (wave_path from that node) are added at once; a child that is not
// far is opened when internal and summed exactly when a leaf.  Random words of
// the path from subdomain a (first point b_a, level l_a), sample s: the Philox
// blocks with counter (stream id, b_a, l_a 2^24 + s 2^16 + step pair, batch).
// With TRACE, paths[j] receives {subdomains, leaves summed exactly, accepted
// steps, sum of end levels} of query j.
template <int D, int K, bool TRACE, bool O64>
__global__ void __launch_bounds__(256) k_sbh_cut(TreeView tv, const float* __restrict__ queries, int64_t nq,
                                                 SbhArgs a, float beta_low, float* __restrict__ out)
{
#pragma clang fp contract(off)
    constexpr int D3 = D * D * D;
    constexpr int TS = topo_stride(D3);
    constexpr int LG = D == 2 ? 1 : D == 4 ? 2 : 3;
    using Off = typename TreeOff<O64>::T;
    constexpr int MAXS = bh_stack_depth<D>();
    __shared__ int2 stack[256 / 64][MAXS];
    __shared__ uint8_t stack_lvl[256 / 64][MAXS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t j0 = ((int64_t)blockIdx.x * 4 + wv) * 64;
    if (j0 >= nq) return;
    const int64_t j = j0 + lane;
    const bool valid = j < nq;
    float qx = 0.f, qy = 0.f, qz = 0.f;
    if (valid) {
        qx = gld(queries + 3 * j);
        qy = gld(queries + 3 * j + 1);
        qz = gld(queries + 3 * j + 2);
    }
    // a query with a non-finite coordinate has no value and takes no part in the vote
    const bool votes = valid && __builtin_isfinite(qx) && __builtin_isfinite(qy) && __builtin_isfinite(qz);
    KParams kp{a.eps2, a.alpha, 1.0f};
    float logwbar = 0.f, r0 = 0.f;
    if constexpr (K == SBH_SMOOTHDIST) {
        smooth_setup(tv, kp.wscale, logwbar);
        r0 = smooth_shift<D>(tv, qx, qy, qz, a.alpha);
    }
    const uint32_t stream = (uint32_t)(j0 / a.group);   // a.group is a multiple of 64
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    float F = 0.0f;
    int n_sub = 0, n_leaf = 0, steps = 0, end_levels = 0;
    int sp = 0;
    if (lane == 0) {
        stack[wv][0] = make_int2(0, 0);   // the root's children: block 0, first point 0
        stack_lvl[wv][0] = 0;
    }
    sp = 1;
    __builtin_amdgcn_wave_barrier();
    while (sp > 0) {
        --sp;
        const int2 e = stack[wv][sp];
        const int32_t blk = __builtin_amdgcn_readfirstlane(e.x);
        const int level = __builtin_amdgcn_readfirstlane((int)stack_lvl[wv][sp]);
        uint32_t pre = (uint32_t)__builtin_amdgcn_readfirstlane(e.y);
        __builtin_amdgcn_wave_barrier();
        const float diamC = ldexpf(tv.diam0, -(level + 1) * LG);
        const float lim = beta_low * diamC;
        const Off boff = (Off)(uint32_t)blk * (Off)(D3 * 16);
        const float4* __restrict__ ba = at_off(tv.bagg, boff);
        const float4* __restrict__ bd = at_off(tv.bdip, boff);
        const uint32_t* __restrict__ bt = at_off(tv.btopo, (Off)(uint32_t)blk * (Off)(TS * 4));
        const int32_t base = (int32_t)gld(bt + D3);
        int32_t nint = 0;
        for (int c = 0; c < D3; ++c) {
            const uint32_t cnt = gld(bt + c);
            if (cnt == 0u) continue;
            const bool internal_c = (int)cnt > tv.leaf_size && level + 1 < tv.max_level;
            const float4 g = gld4(ba + c);
            const float4 gd = (K == SBH_WINDING) ? gld4(bd + c) : zero4;
            const float dx = g.x - qx, dy = g.y - qy, dz = g.z - qz;
            const float r2 = norm2(dx, dy, dz);
            const bool near = votes && !(r2 >= lim * lim);
            if (__ballot(near) == 0ull) {
                // a subdomain: its control variate and S paths rooted at it
                const float cv = term_r2<K>(g, gd, dx, dy, dz, r2, kp, r0);
                const int32_t blk_c = internal_c ? base + nint : 0;
                float fa = 0.0f;
                for (int s2 = 0; s2 < a.samples; ++s2) {
                    PathWordsOne pw;
                    pw.compute(stream, pre, ((uint32_t)(level + 1) << 24) | ((uint32_t)s2 << 16), a.batch, a.key0,
                               a.key1);
                    int4 rec;
                    fa += wave_path<D, K, TRACE, O64, PathWordsOne, 2>(tv, qx, qy, qz, r0, kp, valid, cnt, pre, blk_c, g,
                                                                    cv, pw, stream, 0u, a.batch, a.key0, a.key1,
                                                                    a.rr_mode, &rec, level + 1);
                    if constexpr (TRACE) {
                        steps += rec.z;
                        end_levels += rec.y;
                    }
                }
                F += cv + fa / (float)a.samples;
                ++n_sub;
            } else if (internal_c) {
                if (lane == 0) {
                    stack[wv][sp] = make_int2(base + nint, (int32_t)pre);
                    stack_lvl[wv][sp] = (uint8_t)(level + 1);
                }
                ++sp;
            } else {
                for (uint32_t i = pre; i < pre + cnt; ++i) {
                    const Off po = (Off)i * (Off)16;
                    F = term_acc<K>(*at_off(tv.pts, po), (K == SBH_WINDING) ? *at_off(tv.pdip, po) : zero4, qx, qy, qz,
                                    kp, r0, F);
                }
                ++n_leaf;
            }
            nint += internal_c ? 1 : 0;
            pre += cnt;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (valid) {
        gst(out + j, query_value<K>(F, r0, logwbar, a.alpha, qx, qy, qz));
        if constexpr (TRACE) reinterpret_cast<int4*>(a.paths)[j] = make_int4(n_sub, n_leaf, steps, end_levels);
    }
}

// A tree whose root is a leaf: every query is summed exactly over its points.
template <int K>
__device__ __forceinline__ void leaf_exact_query(const TreeView& tv, const float* __restrict__ queries, int64_t j,
                                                 float eps2, float alpha, float* __restrict__ out)
{
#pragma clang fp contract(off)
    const float qx = gld(queries + 3 * j), qy = gld(queries + 3 * j + 1), qz = gld(queries + 3 * j + 2);
    KParams kp{eps2, alpha, 1.0f};
    float logwbar = 0.f, r0 = 0.f;
    if constexpr (K == SBH_SMOOTHDIST) {
        smooth_setup(tv, kp.wscale, logwbar);
        r0 = smooth_shift<2>(tv, qx, qy, qz, alpha);   // the root is a leaf: every point is examined
    }
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    float acc = 0.0f;
    for (int i = 0; i < tv.n_points; ++i)
        acc = term_acc<K>(gld4(tv.pts + i), (K == SBH_WINDING) ? gld4(tv.pdip + i) : zero4, qx, qy, qz, kp, r0, acc);
    gst(out + j, query_value<K>(acc, r0, logwbar, alpha, qx, qy, qz));
}

template <int K>
__global__ void __launch_bounds__(256) k_leaf_exact(TreeView tv, const float* __restrict__ queries, int64_t nq,
                                                    float eps2, float alpha, float* __restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nq) return;
    leaf_exact_query<K>(tv, queries, j, eps2, alpha, out);
}

// ---------------------------------------------------------------------------
// Batched evaluation: many trees and query sets in one launch per group.
// A work item is one workgroup: a run of wavefront-tiles (64 queries each)
// of one cloud, so that small clouds fill the machine together and large
// ones are split.  Each tile runs exactly the code of the single-tree
// kernels, so a cloud's results do not depend on the batch around it.
// ---------------------------------------------------------------------------
// key, batch word and a cleared work counter for every group of the batch
__global__ void k_batch_begin(BatchState* st, uint32_t key0, uint32_t key1, uint32_t batch)
{
    if (blockIdx.x == 0 && threadIdx.x < kBatchGroups) {
        st[threadIdx.x].key0 = key0;
        st[threadIdx.x].key1 = key1;
        st[threadIdx.x].batch = batch;
        st[threadIdx.x].pad = 0u;
    }
}

// One launch per (branching factor, kernel) group present in the batch, so
// that each instance keeps the registers of the single-tree kernel.  A
// workgroup is one work item: consecutive tiles of one cloud, one per
// wavefront, looked up in the workgroup table; the hardware dispatcher
// starts workgroups as earlier ones finish, which balances clouds of uneven
// cost without a shared work counter.
template <int D, int K, int VM = 2>
__global__ void __launch_bounds__(64 * kBatchMaxTileWaves * kWaveParts) __attribute__((amdgpu_waves_per_eu(8)))
k_sbh_batch(const BatchItem* __restrict__ items, const int2* __restrict__ wg, const BatchState* __restrict__ st,
            SbhArgs base)
{
    constexpr int P = kWaveParts;
    static_assert(kBatchMaxTileWaves * P <= 4, "the walk keeps one LDS row per wavefront, four per workgroup");
    __shared__ float part_f[kBatchMaxTileWaves * P][64];
    __shared__ uint32_t done[kBatchMaxTileWaves];
    if constexpr (P > 1) {
        if (threadIdx.x < kBatchMaxTileWaves) done[threadIdx.x] = 0u;
        __syncthreads();
    }
    const int2 g = wg[blockIdx.x];
    const BatchItem* __restrict__ it = items + __builtin_amdgcn_readfirstlane(g.x);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wave = (int64_t)__builtin_amdgcn_readfirstlane(g.y) + w / P;   // the tile
    const int64_t nq = it->nq;
    if (wave * 64 >= nq) return;
    SbhArgs a = base;
    a.key0 = st->key0;
    a.key1 = st->key1;
    a.batch = st->batch;
    // the descriptor stays in memory and its fields are read where they are used
    // (scalar loads), as kernel arguments are
    if (it->tv.wide)
        sbh_wave_tile<D, K, false, false, P, true, VM>(it->tv, it->queries, nq, a, it->out, wave, w % P, w, part_f,
                                                       done);
    else
        sbh_wave_tile<D, K, false, false, P, false, VM>(it->tv, it->queries, nq, a, it->out, wave, w % P, w, part_f,
                                                        done);
}

// Clouds whose root is a leaf are summed exactly, as sbh_eval does, in launches
// of their own (one per kernel): kept out of k_sbh_batch, the branch would
// cost the walk its registers.
template <int K>
__global__ void __launch_bounds__(64 * kBatchMaxTileWaves)
k_leaf_batch(const BatchItem* __restrict__ items, const int2* __restrict__ wg, float eps2, float alpha)
{
    const int2 g = wg[blockIdx.x];
    const BatchItem* __restrict__ it = items + __builtin_amdgcn_readfirstlane(g.x);
    const int64_t j = ((int64_t)__builtin_amdgcn_readfirstlane(g.y) + (threadIdx.x >> 6)) * 64 + (threadIdx.x & 63);
    if (j < it->nq) leaf_exact_query<K>(it->tv, it->queries, j, eps2, alpha, it->out);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int K>
static hipError_t launch_leaf(const TreeView& tv, const float* q, int64_t nq, const EvalLaunch& e, float* out,
                              hipStream_t s)
{
    k_leaf_exact<K><<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(tv, q, nq, e.eps * e.eps, e.alpha, out);
    return hipGetLastError();
}

template <int D, int K>
static hipError_t launch_sbh_dk(const TreeView& tv, const float* q, int64_t nq, const EvalLaunch& e, float* out,
                                hipStream_t s)
{
    constexpr int QPW = D == 8 ? 1 : 64 / (D * D * D);
    SbhArgs a{e.samples, e.group, e.rr_mode, e.batch, (uint32_t)e.seed, (uint32_t)(e.seed >> 32),
              e.eps * e.eps, e.alpha, e.paths};
    if (e.group % 64 == 0) {
        const int64_t tiles = (nq + 63) / 64;
        const unsigned wblocks = (unsigned)((tiles + (4 / kWaveParts) - 1) / (4 / kWaveParts));
        if (e.tile_score) {
            if constexpr (D == 2) {
                if (tv.wide) {
                    if (e.paths) k_sbh_wave_tile<K, true, true><<<wblocks, 256, 0, s>>>(tv, q, nq, a, out);
                    else k_sbh_wave_tile<K, false, true><<<wblocks, 256, 0, s>>>(tv, q, nq, a, out);
                } else {
                    if (e.paths) k_sbh_wave_tile<K, true, false><<<wblocks, 256, 0, s>>>(tv, q, nq, a, out);
                    else k_sbh_wave_tile<K, false, false><<<wblocks, 256, 0, s>>>(tv, q, nq, a, out);
                }
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        }
        // d = 2: the last tiles over four wavefronts each (split_tile a multiple of the two
        // tiles a block takes before it)
        constexpr int64_t TPB = 4 / kWaveParts;
        int64_t split = (tiles + TPB - 1) / TPB * TPB;
        unsigned blocks = wblocks;
        if constexpr (D == 2) {
            split = std::max<int64_t>(0, tiles - std::min(tail_tiles(), tiles)) / TPB * TPB;
            blocks = (unsigned)(split / TPB + (tiles - split));
        }
        // each roulette is a kernel of its own (Eq. (5), voted, and the run-time ablation modes),
        // so that the default walk carries no test of rr_mode
#define SBH_WAVE(VV)                                                                                        \
    do {                                                                                                    \
        if (tv.wide) {                                                                                      \
            if (e.paths) k_sbh_wave<D, K, true, true, VV><<<blocks, 256, 0, s>>>(tv, q, nq, a, out, split);  \
            else k_sbh_wave<D, K, false, true, VV><<<blocks, 256, 0, s>>>(tv, q, nq, a, out, split);         \
        } else {                                                                                            \
            if (e.paths) k_sbh_wave<D, K, true, false, VV><<<blocks, 256, 0, s>>>(tv, q, nq, a, out, split); \
            else k_sbh_wave<D, K, false, false, VV><<<blocks, 256, 0, s>>>(tv, q, nq, a, out, split);        \
        }                                                                                                   \
    } while (0)
        if (e.rr_mode == 0) SBH_WAVE(0);
        else if (e.rr_mode == 3) SBH_WAVE(1);
        else SBH_WAVE(2);
#undef SBH_WAVE
        return hipGetLastError();
    }
    if constexpr (D == 8) {
        return hipErrorInvalidValue;   // branching 8: the coherent walk only (the API checks G)
    } else if ((int64_t)D * D * D * e.samples <= kPoolPaths) {
        // per-lane walks with lane refill: Q queries per wavefront, four wavefronts per block
        const int64_t qpw = kPoolPaths / (D * D * D * e.samples);
        const int64_t waves = (nq + qpw - 1) / qpw;
        const unsigned blocks = (unsigned)((waves + 3) / 4);
        if (e.paths) k_sbh_pool<D, K, true><<<blocks, 256, 0, s>>>(tv, q, nq, a, out);
        else k_sbh_pool<D, K, false><<<blocks, 256, 0, s>>>(tv, q, nq, a, out);
        return hipGetLastError();
    } else {
        const int64_t waves = (nq + QPW - 1) / QPW;
        const unsigned blocks = (unsigned)((waves + 3) / 4);
        if (e.paths) k_sbh<D, K, true><<<blocks, 256, 0, s>>>(tv, q, nq, a, out);
        else k_sbh<D, K, false><<<blocks, 256, 0, s>>>(tv, q, nq, a, out);
        return hipGetLastError();
    }
}

template <int D, int K>
static hipError_t launch_cut_dk(const TreeView& tv, const float* q, int64_t nq, const EvalLaunch& e, float* out,
                                hipStream_t s)
{
    SbhArgs a{e.samples, e.group, e.rr_mode, e.batch, (uint32_t)e.seed, (uint32_t)(e.seed >> 32),
              e.eps * e.eps, e.alpha, e.paths};
    const unsigned blocks = (unsigned)(((nq + 63) / 64 + 3) / 4);
    if (tv.wide) {
        if (e.paths) k_sbh_cut<D, K, true, true><<<blocks, 256, 0, s>>>(tv, q, nq, a, e.beta, out);
        else k_sbh_cut<D, K, false, true><<<blocks, 256, 0, s>>>(tv, q, nq, a, e.beta, out);
    } else {
        if (e.paths) k_sbh_cut<D, K, true, false><<<blocks, 256, 0, s>>>(tv, q, nq, a, e.beta, out);
        else k_sbh_cut<D, K, false, false><<<blocks, 256, 0, s>>>(tv, q, nq, a, e.beta, out);
    }
    return hipGetLastError();
}

template <int D, int K>
static hipError_t launch_bh_dk(const TreeView& tv, const float* q, int64_t nq, const EvalLaunch& e, float* out,
                               hipStream_t s)
{
    BhArgs a{e.beta, e.eps * e.eps, e.alpha};
    if (tv.wide) k_bh<D, K, true><<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(tv, q, nq, a, out);
    else k_bh<D, K, false><<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(tv, q, nq, a, out);
    return hipGetLastError();
}

#define SBH_DISPATCH(FN, t, ...)                                              \
    do {                                                                      \
        if ((t)->d == 2) {                                                    \
            if (e.kernel == SBH_POTENTIAL) return FN<2, SBH_POTENTIAL>(__VA_ARGS__);   \
            if (e.kernel == SBH_WINDING) return FN<2, SBH_WINDING>(__VA_ARGS__);       \
            return FN<2, SBH_SMOOTHDIST>(__VA_ARGS__);                        \
        } else {                                                              \
            if (e.kernel == SBH_POTENTIAL) return FN<4, SBH_POTENTIAL>(__VA_ARGS__);   \
            if (e.kernel == SBH_WINDING) return FN<4, SBH_WINDING>(__VA_ARGS__);       \
            return FN<4, SBH_SMOOTHDIST>(__VA_ARGS__);                        \
        }                                                                     \
    } while (0)

hipError_t launch_sbh_eval(const sbh_tree_impl* t, const float* queries, int64_t nq, const EvalLaunch& e,
                           float* out, hipStream_t s)
{
    const TreeView tv = make_view(t);
    if (!tv.root_internal) {
        if (e.kernel == SBH_POTENTIAL) return launch_leaf<SBH_POTENTIAL>(tv, queries, nq, e, out, s);
        if (e.kernel == SBH_WINDING) return launch_leaf<SBH_WINDING>(tv, queries, nq, e, out, s);
        return launch_leaf<SBH_SMOOTHDIST>(tv, queries, nq, e, out, s);
    }
    if (e.lod == 2) {   // second-order node terms (d = 2, potential, G a multiple of 64)
        SbhArgs a{e.samples, e.group, e.rr_mode, e.batch, (uint32_t)e.seed, (uint32_t)(e.seed >> 32),
                  e.eps * e.eps, e.alpha, e.paths};
        const unsigned wblocks = (unsigned)(((nq + 63) / 64 + (4 / kWaveParts) - 1) / (4 / kWaveParts));
#define SBH_L2(VV)                                                                                          \
    do {                                                                                                    \
        if (tv.wide) {                                                                                      \
            if (e.paths) k_sbh_wave_l2<true, true, VV><<<wblocks, 256, 0, s>>>(tv, queries, nq, a, out);     \
            else k_sbh_wave_l2<false, true, VV><<<wblocks, 256, 0, s>>>(tv, queries, nq, a, out);            \
        } else {                                                                                            \
            if (e.paths) k_sbh_wave_l2<true, false, VV><<<wblocks, 256, 0, s>>>(tv, queries, nq, a, out);    \
            else k_sbh_wave_l2<false, false, VV><<<wblocks, 256, 0, s>>>(tv, queries, nq, a, out);           \
        }                                                                                                   \
    } while (0)
        if (e.rr_mode == 0) SBH_L2(0);
        else if (e.rr_mode == 3) SBH_L2(1);
        else SBH_L2(2);
#undef SBH_L2
        return hipGetLastError();
    }
    if (e.compressed) {   // the coherent walk on compressed aggregates (d = 2, potential or smooth distance)
        SbhArgs a{e.samples, e.group, e.rr_mode, e.batch, (uint32_t)e.seed, (uint32_t)(e.seed >> 32),
                  e.eps * e.eps, e.alpha, e.paths};
        if (e.group % 64 != 0) {   // per-query streams: the per-lane walk with lane refill
            if (8 * e.samples > kPoolPaths) return hipErrorInvalidValue;   // the API checks S
            const int64_t qpw = kPoolPaths / (8 * e.samples);
            const unsigned blocks = (unsigned)(((nq + qpw - 1) / qpw + 3) / 4);
            if (e.kernel == SBH_POTENTIAL) {
                if (e.paths) k_sbh_pool<2, SBH_POTENTIAL, true, true><<<blocks, 256, 0, s>>>(tv, queries, nq, a, out);
                else k_sbh_pool<2, SBH_POTENTIAL, false, true><<<blocks, 256, 0, s>>>(tv, queries, nq, a, out);
            } else {
                if (e.paths) k_sbh_pool<2, SBH_SMOOTHDIST, true, true><<<blocks, 256, 0, s>>>(tv, queries, nq, a, out);
                else k_sbh_pool<2, SBH_SMOOTHDIST, false, true><<<blocks, 256, 0, s>>>(tv, queries, nq, a, out);
            }
            return hipGetLastError();
        }
        const unsigned wblocks = (unsigned)(((nq + 63) / 64 + (4 / kWaveParts) - 1) / (4 / kWaveParts));
#define SBH_QV(KK, VV)                                                                                      \
    do {                                                                                                    \
        if (tv.wide) {                                                                                      \
            if (e.paths) k_sbh_wave_q<KK, true, true, VV><<<wblocks, 256, 0, s>>>(tv, queries, nq, a, out);  \
            else k_sbh_wave_q<KK, false, true, VV><<<wblocks, 256, 0, s>>>(tv, queries, nq, a, out);         \
        } else {                                                                                            \
            if (e.paths) k_sbh_wave_q<KK, true, false, VV><<<wblocks, 256, 0, s>>>(tv, queries, nq, a, out); \
            else k_sbh_wave_q<KK, false, false, VV><<<wblocks, 256, 0, s>>>(tv, queries, nq, a, out);        \
        }                                                                                                   \
    } while (0)
#define SBH_Q(KK)                                                                                           \
    do {                                                                                                    \
        if (e.rr_mode == 0) SBH_QV(KK, 0);                                                                  \
        else if (e.rr_mode == 3) SBH_QV(KK, 1);                                                             \
        else SBH_QV(KK, 2);                                                                                 \
    } while (0)
        if (e.kernel == SBH_POTENTIAL) SBH_Q(SBH_POTENTIAL);
        else SBH_Q(SBH_SMOOTHDIST);
#undef SBH_Q
#undef SBH_QV
        return hipGetLastError();
    }
    if (e.cut) {   // subdomains: the Barnes-Hut cut (branching 2 and 4)
        SBH_DISPATCH(launch_cut_dk, t, tv, queries, nq, e, out, s);
    }
    if (t->d == 8) {
        if (e.kernel == SBH_POTENTIAL) return launch_sbh_dk<8, SBH_POTENTIAL>(tv, queries, nq, e, out, s);
        if (e.kernel == SBH_WINDING) return launch_sbh_dk<8, SBH_WINDING>(tv, queries, nq, e, out, s);
        return launch_sbh_dk<8, SBH_SMOOTHDIST>(tv, queries, nq, e, out, s);
    }
    SBH_DISPATCH(launch_sbh_dk, t, tv, queries, nq, e, out, s);
}

hipError_t launch_bh_eval(const sbh_tree_impl* t, const float* queries, int64_t nq, const EvalLaunch& e,
                          float* out, hipStream_t s)
{
    const TreeView tv = make_view(t);
    SBH_DISPATCH(launch_bh_dk, t, tv, queries, nq, e, out, s);
}

hipError_t launch_batch_begin(BatchState* st, uint64_t seed, uint32_t batch, hipStream_t s)
{
    k_batch_begin<<<1, 64, 0, s>>>(st, (uint32_t)seed, (uint32_t)(seed >> 32), batch);
    return hipGetLastError();
}

hipError_t launch_sbh_batch(int d, int kernel, const BatchItem* items, const int2* wg, int blocks, int tile_waves,
                            size_t lds_bytes, const BatchState* st, int samples, int group, int rr_mode, float eps,
                            float alpha, hipStream_t s)
{
    SbhArgs a{samples, group, rr_mode, 0u, 0u, 0u, eps * eps, alpha, nullptr};
    const dim3 block(64 * tile_waves * kWaveParts);
    // a kernel per roulette (Eq. (5), voted, the ablation modes), as in the single-tree launch
#define SBH_LAUNCH_B(DD, KK)                                                                      \
    do {                                                                                          \
        if (rr_mode == 0) k_sbh_batch<DD, KK, 0><<<blocks, block, lds_bytes, s>>>(items, wg, st, a); \
        else if (rr_mode == 3) k_sbh_batch<DD, KK, 1><<<blocks, block, lds_bytes, s>>>(items, wg, st, a); \
        else k_sbh_batch<DD, KK, 2><<<blocks, block, lds_bytes, s>>>(items, wg, st, a);            \
    } while (0)
    if (d == 2) {
        if (kernel == SBH_POTENTIAL) SBH_LAUNCH_B(2, SBH_POTENTIAL);
        else if (kernel == SBH_WINDING) SBH_LAUNCH_B(2, SBH_WINDING);
        else SBH_LAUNCH_B(2, SBH_SMOOTHDIST);
    } else {
        if (kernel == SBH_POTENTIAL) SBH_LAUNCH_B(4, SBH_POTENTIAL);
        else if (kernel == SBH_WINDING) SBH_LAUNCH_B(4, SBH_WINDING);
        else SBH_LAUNCH_B(4, SBH_SMOOTHDIST);
    }
#undef SBH_LAUNCH_B
    return hipGetLastError();
}

hipError_t launch_leaf_batch(int kernel, const BatchItem* items, const int2* wg, int blocks, int tile_waves, float eps,
                             float alpha, hipStream_t s)
{
    const dim3 block(64 * tile_waves);
    if (kernel == SBH_POTENTIAL) k_leaf_batch<SBH_POTENTIAL><<<blocks, block, 0, s>>>(items, wg, eps * eps, alpha);
    else if (kernel == SBH_WINDING) k_leaf_batch<SBH_WINDING><<<blocks, block, 0, s>>>(items, wg, eps * eps, alpha);
    else k_leaf_batch<SBH_SMOOTHDIST><<<blocks, block, 0, s>>>(items, wg, eps * eps, alpha);
    return hipGetLastError();
}

void* batch_begin_kernel() { return reinterpret_cast<void*>(&k_batch_begin); }

hipError_t batch_static_lds(size_t* bytes)
{
    size_t m = 0;
    const void* fns[] = {reinterpret_cast<const void*>(&k_sbh_batch<2, SBH_POTENTIAL>),
                         reinterpret_cast<const void*>(&k_sbh_batch<2, SBH_WINDING>),
                         reinterpret_cast<const void*>(&k_sbh_batch<2, SBH_SMOOTHDIST>),
                         reinterpret_cast<const void*>(&k_sbh_batch<4, SBH_POTENTIAL>),
                         reinterpret_cast<const void*>(&k_sbh_batch<4, SBH_WINDING>),
                         reinterpret_cast<const void*>(&k_sbh_batch<4, SBH_SMOOTHDIST>)};
    for (const void* f : fns) {
        hipFuncAttributes fa{};
        const hipError_t e = hipFuncGetAttributes(&fa, f);
        if (e != hipSuccess) return e;
        m = std::max(m, (size_t)fa.sharedSizeBytes);
    }
    *bytes = m;
    return hipSuccess;
}

}  // namespace sbh
