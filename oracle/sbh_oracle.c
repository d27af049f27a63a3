/*
 * FP64 CPU oracle for the stochastic Barnes-Hut estimator
 * (Madan, Sharp, Williams, Museth, Levin: "Stochastic Barnes-Hut
 * Approximation for Fast Summation on the GPU", SIGGRAPH 2025).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load it; the product path never does.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * What each part follows:
 *   kernel sum ............ Section 3, Eq. (1)   (the index under the sum is i)
 *   tree and aggregates ... Section 3.1 (octree-like tree, per-node box,
 *                           aggregate mass, centre of mass)
 *   Barnes-Hut ............ Section 3.1, Eq. (2), Algorithm 1
 *   path estimator ........ Section 3.3, Eqs. (5)-(7), Section 3.3.1
 *                           (domain stratification), Algorithm 2
 *   unbiasedness .......... Theorem 1 and its proof (Appendix A), via the
 *                           exact-expectation enumerator below
 *   Philox4x32-10 ......... Salmon, Moraes, Dror, Shaw, "Parallel random
 *                           numbers: as easy as 1, 2, 3", SC'11
 *
 * Readings where the paper is silent (kept identical on the HIP side):
 *   - |B| is the octree CELL diagonal sqrt(3)*side/d^level, so a child's box
 *     is exactly 1/d of its parent's (Section 3.3, far-field ratio argument).
 *   - The tree is built from a 60-bit Morton code of fp32-quantised
 *     coordinates; a node is split iff count > leaf_size and level < max.
 *   - A leaf holding several points treats them as virtual children with box
 *     diameter |B_leaf|/d (the paper assumes one point per leaf).
 *   - The path index is drawn one level at a time: child c of T with
 *     probability n_c/n_T, which composes to the uniform path index.
 *   - Random numbers: Philox4x32-10, key = seed, counter = (stream, a*S+s,
 *     step/2, batch); words (0,1) drive step 2k, words (2,3) step 2k+1; the
 *     first word of a pair selects, the second (top 24 bits) drives the
 *     Russian roulette test "stop iff u >= p".
 *   - Barnes-Hut opens a leaf that is not far by summing its points exactly.
 *
 * Build: gcc -O2 -std=c99 -fopenmp -ffp-contract=off -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_POTENTIAL 0
#define ORC_WINDING 1
#define ORC_SMOOTHDIST 2
#define ORC_LINEAR 99 /* test kernel: first-order LOD is exact for it */

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 S-box with    */
/* multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments               */
/* 0x9E3779B9 / 0xBB67AE85.                                                   */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        uint32_t n0 = hi_b ^ c1 ^ k0;
        uint32_t n1 = lo_b;
        uint32_t n2 = hi_a ^ c3 ^ k1;
        uint32_t n3 = lo_a;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Kernels f: the term of one source (or one node aggregate) at query q.     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kernel;
    double eps;   /* potential softening */
    double alpha; /* smooth-distance sharpness */
} kparams;

/* m: mass (weight) of the source/aggregate, p: position (or centre of mass),
 * dip: summed w*n (winding only). */
static double term(const kparams* kp, const double p[3], double m, const double dip[3], const double q[3])
{
    double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    switch (kp->kernel) {
    case ORC_POTENTIAL:
        return m / sqrt(r2 + kp->eps * kp->eps);
    case ORC_WINDING: {
        if (r2 == 0.0) return 0.0;
        double r = sqrt(r2);
        return (dip[0] * dx + dip[1] * dy + dip[2] * dz) / (4.0 * ORC_PI * r2 * r);
    }
    case ORC_SMOOTHDIST:
        return m * exp(-kp->alpha * sqrt(r2));
    case ORC_LINEAR:
        /* m * (1 + g.(p - q)) with g = (0.3, -0.2, 0.1) */
        return m * (1.0 + 0.3 * dx - 0.2 * dy + 0.1 * dz);
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Brute force, Eq. (1): F(q) = sum_i m_i f(p_i, q), index order, Neumaier   */
/* compensated summation.                                                     */
/* ------------------------------------------------------------------------ */
void orc_brute(const float* src, const float* w, const float* nrm, int64_t m,
               const float* qry, int64_t n, int kernel, double eps, double alpha,
               double* out, int nthreads)
{
    kparams kp = {kernel, eps, alpha};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t j = 0; j < n; ++j) {
        double q[3] = {qry[3 * j], qry[3 * j + 1], qry[3 * j + 2]};
        double s = 0.0, c = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            double p[3] = {src[3 * i], src[3 * i + 1], src[3 * i + 2]};
            double wi = w[i];
            double d[3] = {0, 0, 0};
            if (nrm) {
                d[0] = wi * (double)nrm[3 * i];
                d[1] = wi * (double)nrm[3 * i + 1];
                d[2] = wi * (double)nrm[3 * i + 2];
            }
            double t = term(&kp, p, wi, d, q);
            double y = s + t;
            if (fabs(s) >= fabs(t)) c += (s - y) + t;
            else c += (t - y) + s;
            s = y;
        }
        out[j] = s + c;
    }
}

/* ------------------------------------------------------------------------ */
/* Tree (Section 3.1): octree-like, per-dimension branching d, built from    */
/* Morton codes of fp32-quantised coordinates.                                */
/* ------------------------------------------------------------------------ */
typedef struct orc_tree {
    int64_t m;
    int d, bits, leaf_size, max_level, depth;
    float lo[3], side, inv_side;
    /* points in sorted (Morton) order, in double */
    double* pxyz;  /* [m][3] */
    double* pw;    /* [m] */
    double* pdip;  /* [m][3]  w*n, zeros without normals */
    int has_normals;
    int64_t* perm;   /* sorted position -> input index */
    uint64_t* codes; /* sorted codes */
    /* nodes in BFS order; within a level, Morton order */
    int64_t n_nodes, cap;
    int64_t *begin, *count, *first_child, *parent;
    int32_t *level, *nchild, *digit;
    double *mass, *com, *dip; /* com, dip: [n][3] */
    double* spr;              /* second moment sum w |p - com|^2 / mass */
    double diam[64];          /* |B| per level */
    /* The reading of |B| (a study of the paper's wording; 0 is the one both
     * sides implement): 0 the cell diagonal, 1 the cell side, 2 the diagonal
     * of the axis-aligned box of the node's own points (bdiag), under which
     * a point (a one-point node, or a leaf's virtual child) has |B| = 0. */
    int diam_mode;
    double* bdiag;            /* [n] tight-box diagonals, mode 2 only */
    /* Compressed interior aggregates (the conclusion's quantisation of the
     * node-aggregate buffer): when cmp is set, every node term and far-field
     * ratio uses the decoded aggregates qcom / qmass below instead of the
     * exact ones; leaves' points stay exact. */
    int cmp;
    double *qcom, *qmass;     /* [n][3], [n] decoded centres of mass and masses */
    float* qcode;             /* [n][4] the stored binary16 values: offset x, y, z, mass fraction */
    /* Second-order level of detail (Section 3.1 allows higher-order node
     * approximations): lod 2 adds, for the potential, the quadrupole term of
     * the node's Taylor expansion about its centre of mass wherever the query
     * sees the node as far (|q - com| >= |B|). */
    int lod;
    double* quad;             /* [n][6] Q = sum w (p - com)(p - com)^T: xx, yy, zz, xy, xz, yz */
} orc_tree;

static uint64_t spread3(uint32_t v)
{
    /* bit k of v -> bit 3k of the result (k < 20) */
    uint64_t r = 0;
    for (int k = 0; k < 20; ++k)
        if (v & (1u << k)) r |= (uint64_t)1 << (3 * k);
    return r;
}

static const uint64_t* g_sort_codes;
static int cmp_code_index(const void* a, const void* b)
{
    int64_t ia = *(const int64_t*)a, ib = *(const int64_t*)b;
    uint64_t ca = g_sort_codes[ia], cb = g_sort_codes[ib];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return (ia < ib) ? -1 : (ia > ib);
}

static void push_node(orc_tree* t, int64_t b, int64_t c, int32_t lev, int64_t par, int32_t dig)
{
    if (t->n_nodes == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 1024;
        t->begin = realloc(t->begin, t->cap * sizeof(int64_t));
        t->count = realloc(t->count, t->cap * sizeof(int64_t));
        t->first_child = realloc(t->first_child, t->cap * sizeof(int64_t));
        t->parent = realloc(t->parent, t->cap * sizeof(int64_t));
        t->level = realloc(t->level, t->cap * sizeof(int32_t));
        t->nchild = realloc(t->nchild, t->cap * sizeof(int32_t));
        t->digit = realloc(t->digit, t->cap * sizeof(int32_t));
    }
    int64_t i = t->n_nodes++;
    t->begin[i] = b;
    t->count[i] = c;
    t->first_child[i] = -1;
    t->parent[i] = par;
    t->level[i] = lev;
    t->nchild[i] = 0;
    t->digit[i] = dig;
}

static int is_internal(const orc_tree* t, int64_t i)
{
    return t->count[i] > t->leaf_size && t->level[i] < t->max_level;
}

void orc_tree_free(orc_tree* t)
{
    if (!t) return;
    free(t->pxyz); free(t->pw); free(t->pdip); free(t->perm); free(t->codes);
    free(t->begin); free(t->count); free(t->first_child); free(t->parent);
    free(t->level); free(t->nchild); free(t->digit);
    free(t->mass); free(t->com); free(t->dip); free(t->spr); free(t->bdiag);
    free(t->qcom); free(t->qmass); free(t->qcode); free(t->quad);
    free(t);
}

/* d in {2,4,8}; max_level <= 60 / (3 log2 d); leaf_size >= 1. */
orc_tree* orc_tree_build(const float* src, const float* w, const float* nrm, int64_t m,
                         int d, int leaf_size, int max_level)
{
    if (m <= 0 || leaf_size < 1) return NULL;
    int lg = (d == 2) ? 1 : (d == 4) ? 2 : (d == 8) ? 3 : 0;
    if (!lg) return NULL;
    int bits = 3 * lg;
    if (max_level <= 0 || max_level > 60 / bits) max_level = 60 / bits;
    orc_tree* t = calloc(1, sizeof(orc_tree));
    t->m = m; t->d = d; t->bits = bits; t->leaf_size = leaf_size; t->max_level = max_level;

    /* root cube, in fp32 exactly as specified */
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = src[a]; hi[a] = src[a]; }
    for (int64_t i = 1; i < m; ++i)
        for (int a = 0; a < 3; ++a) {
            float x = src[3 * i + a];
            if (x < lo[a]) lo[a] = x;
            if (x > hi[a]) hi[a] = x;
        }
    float side = 0.0f;
    for (int a = 0; a < 3; ++a) {
        float e = hi[a] - lo[a];
        if (e > side) side = e;
    }
    if (side == 0.0f) side = 1.0f;
    float inv_side = 1.0f / side;
    for (int a = 0; a < 3; ++a) t->lo[a] = lo[a];
    t->side = side; t->inv_side = inv_side;

    /* quantise (fp32, no contraction) and Morton-encode: bit 3k+a = bit k of axis a */
    uint64_t* code = malloc(m * sizeof(uint64_t));
    for (int64_t i = 0; i < m; ++i) {
        uint32_t cell[3];
        for (int a = 0; a < 3; ++a) {
            float u = src[3 * i + a] - lo[a];
            u = u * inv_side;
            u = u * 1048576.0f;
            uint32_t c = (uint32_t)u;
            if (c > 1048575u) c = 1048575u;
            cell[a] = c;
        }
        code[i] = spread3(cell[0]) | (spread3(cell[1]) << 1) | (spread3(cell[2]) << 2);
    }
    /* stable sort by code (ties by input index) */
    int64_t* perm = malloc(m * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) perm[i] = i;
    g_sort_codes = code;
    qsort(perm, (size_t)m, sizeof(int64_t), cmp_code_index);
    t->perm = perm;
    t->codes = malloc(m * sizeof(uint64_t));
    t->pxyz = malloc(3 * m * sizeof(double));
    t->pw = malloc(m * sizeof(double));
    t->pdip = calloc(3 * m, sizeof(double));
    t->has_normals = nrm != NULL;
    for (int64_t s = 0; s < m; ++s) {
        int64_t i = perm[s];
        t->codes[s] = code[i];
        for (int a = 0; a < 3; ++a) t->pxyz[3 * s + a] = src[3 * i + a];
        t->pw[s] = w[i];
        if (nrm)
            for (int a = 0; a < 3; ++a) t->pdip[3 * s + a] = (double)w[i] * (double)nrm[3 * i + a];
    }
    free(code);

    /* breadth-first construction: a node is its maximal run of equal prefix;
     * its children are the non-empty runs of the next digit, in digit order */
    push_node(t, 0, m, 0, -1, 0);
    uint64_t dmask = ((uint64_t)1 << bits) - 1;
    for (int64_t i = 0; i < t->n_nodes; ++i) {
        if (!is_internal(t, i)) continue;
        int shift = 60 - bits * (t->level[i] + 1);
        int64_t b = t->begin[i], e = t->begin[i] + t->count[i];
        t->first_child[i] = t->n_nodes;
        int64_t j = b;
        while (j < e) {
            uint64_t dig = (t->codes[j] >> shift) & dmask;
            int64_t k = j;
            while (k < e && ((t->codes[k] >> shift) & dmask) == dig) ++k;
            push_node(t, j, k - j, t->level[i] + 1, i, (int32_t)dig);
            t->nchild[i] += 1;
            j = k;
        }
    }
    int depth = 0;
    for (int64_t i = 0; i < t->n_nodes; ++i)
        if (t->level[i] > depth) depth = t->level[i];
    t->depth = depth;

    /* aggregates straight from their definition: mass = sum w, centre of
     * mass = sum w p / mass, dipole = sum w n */
    int64_t nn = t->n_nodes;
    t->mass = malloc(nn * sizeof(double));
    t->com = malloc(3 * nn * sizeof(double));
    t->dip = malloc(3 * nn * sizeof(double));
    t->spr = malloc(nn * sizeof(double));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < nn; ++i) {
        double ms = 0, cx = 0, cy = 0, cz = 0, dx = 0, dy = 0, dz = 0;
        for (int64_t s = t->begin[i]; s < t->begin[i] + t->count[i]; ++s) {
            double wi = t->pw[s];
            ms += wi;
            cx += wi * t->pxyz[3 * s];
            cy += wi * t->pxyz[3 * s + 1];
            cz += wi * t->pxyz[3 * s + 2];
            dx += t->pdip[3 * s];
            dy += t->pdip[3 * s + 1];
            dz += t->pdip[3 * s + 2];
        }
        t->mass[i] = ms;
        t->com[3 * i] = cx / ms;
        t->com[3 * i + 1] = cy / ms;
        t->com[3 * i + 2] = cz / ms;
        t->dip[3 * i] = dx;
        t->dip[3 * i + 1] = dy;
        t->dip[3 * i + 2] = dz;
        double s2 = 0.0;
        for (int64_t s = t->begin[i]; s < t->begin[i] + t->count[i]; ++s) {
            double ex = t->pxyz[3 * s] - t->com[3 * i], ey = t->pxyz[3 * s + 1] - t->com[3 * i + 1],
                   ez = t->pxyz[3 * s + 2] - t->com[3 * i + 2];
            s2 += t->pw[s] * (ex * ex + ey * ey + ez * ez);
        }
        t->spr[i] = s2 / ms;
    }
    /* cell diagonal per level */
    double dl = 1.0;
    for (int l = 0; l < 64; ++l) {
        t->diam[l] = sqrt(3.0) * (double)side / dl;
        dl *= (double)d;
    }
    return t;
}

int64_t orc_tree_num_nodes(const orc_tree* t) { return t->n_nodes; }

/* meta: lo[3], side, inv_side, d, leaf_size, max_level, depth, m */
void orc_tree_meta(const orc_tree* t, double* meta)
{
    meta[0] = t->lo[0]; meta[1] = t->lo[1]; meta[2] = t->lo[2];
    meta[3] = t->side; meta[4] = t->inv_side;
    meta[5] = t->d; meta[6] = t->leaf_size; meta[7] = t->max_level; meta[8] = t->depth;
    meta[9] = (double)t->m;
}

/* agg: [n][8] = com xyz, mass, dip xyz, |B|; spread2: [n] second moments */
void orc_tree_export(const orc_tree* t, int64_t* begin, int64_t* count, int32_t* level,
                     int64_t* first_child, int32_t* nchild, int32_t* digit, int64_t* parent,
                     double* agg, int64_t* perm, uint64_t* codes, double* spread2)
{
    for (int64_t i = 0; i < t->n_nodes; ++i) {
        if (begin) begin[i] = t->begin[i];
        if (count) count[i] = t->count[i];
        if (level) level[i] = t->level[i];
        if (first_child) first_child[i] = t->first_child[i];
        if (nchild) nchild[i] = t->nchild[i];
        if (digit) digit[i] = t->digit[i];
        if (parent) parent[i] = t->parent[i];
        if (agg) {
            agg[8 * i + 0] = t->com[3 * i];
            agg[8 * i + 1] = t->com[3 * i + 1];
            agg[8 * i + 2] = t->com[3 * i + 2];
            agg[8 * i + 3] = t->mass[i];
            agg[8 * i + 4] = t->dip[3 * i];
            agg[8 * i + 5] = t->dip[3 * i + 1];
            agg[8 * i + 6] = t->dip[3 * i + 2];
            agg[8 * i + 7] = t->diam[t->level[i]];
        }
        if (spread2) spread2[i] = t->spr[i];
    }
    for (int64_t s = 0; s < t->m; ++s) {
        if (perm) perm[s] = t->perm[s];
        if (codes) codes[s] = t->codes[s];
    }
}

static const double* node_com(const orc_tree* t, int64_t i) { return t->cmp ? &t->qcom[3 * i] : &t->com[3 * i]; }
static double node_mass(const orc_tree* t, int64_t i) { return t->cmp ? t->qmass[i] : t->mass[i]; }

/* binary16 value nearest to x (round to nearest even), as a double: the
 * rounding is done on x itself, not on a float32 rounding of it. */
static double f16_round_d(double x)
{
    if (!(x == x) || x == 0.0 || isinf(x)) return x;
    int e;
    (void)frexp(x, &e);
    int ex = e - 1;
    if (ex < -14) ex = -14;
    double quantum = ldexp(1.0, ex - 10);
    double r = nearbyint(x / quantum) * quantum;
    if (fabs(r) > 65504.0) return x > 0 ? INFINITY : -INFINITY;
    return r;
}

/* Compressed aggregates.  The root keeps its centre of mass and mass as
 * float32 values.  A node v at level L >= 1 with parent P (already decoded)
 * stores, in binary16,
 *   o_v = (com_v - com^q_P) / s_L   (per axis; s_L = side / d^L, v's cell side)
 *   f_v = m_v / m^q_P
 * and decodes to com^q_v = com^q_P + o_v s_L, m^q_v = m^q_P f_v (float64
 * arithmetic, in that order).  Offsets are relative to the decoded parent, so
 * the error of a centre of mass is one binary16 rounding of its cell side and
 * does not accumulate down the tree; the estimator stays unbiased for any
 * aggregate values (Theorem 1). */
int orc_tree_set_compressed(orc_tree* t, int on)
{
    if (on && t->lod == 2) return -1;
    if (on && !t->qcom) {
        int64_t n = t->n_nodes;
        /* the exact aggregates the codes round, in a fixed float64 summation order: a leaf sums its
         * points in sorted order (m = sum w, s = sum w p), an internal node its children in slot
         * order (m = sum m_c, s = sum m_c com_c); com = s / m.  (The centre-of-mass definition
         * above sums every node's points directly; the two agree to float64 rounding, and the
         * codes need one order that the GPU build follows too.) */
        double* bm = malloc(n * sizeof(double));
        double* bc = malloc(3 * n * sizeof(double));
        for (int64_t v = n - 1; v >= 0; --v) {   /* children follow their parents */
            double m = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
            if (is_internal(t, v)) {
                for (int64_t c = t->first_child[v]; c < t->first_child[v] + t->nchild[v]; ++c) {
                    m += bm[c];
                    sx += bm[c] * bc[3 * c];
                    sy += bm[c] * bc[3 * c + 1];
                    sz += bm[c] * bc[3 * c + 2];
                }
            } else {
                for (int64_t q = t->begin[v]; q < t->begin[v] + t->count[v]; ++q) {
                    double w = t->pw[q];
                    m += w;
                    sx += w * t->pxyz[3 * q];
                    sy += w * t->pxyz[3 * q + 1];
                    sz += w * t->pxyz[3 * q + 2];
                }
            }
            bm[v] = m;
            bc[3 * v] = sx / m;
            bc[3 * v + 1] = sy / m;
            bc[3 * v + 2] = sz / m;
        }
        t->qcom = malloc(3 * n * sizeof(double));
        t->qmass = malloc(n * sizeof(double));
        t->qcode = calloc(4 * n, sizeof(float));
        for (int a = 0; a < 3; ++a) t->qcom[a] = (double)(float)bc[a];
        t->qmass[0] = (double)(float)bm[0];
        for (int64_t v = 1; v < n; ++v) {   /* breadth-first: every parent precedes its children */
            int64_t P = t->parent[v];
            double sl = (double)t->side / pow((double)t->d, (double)t->level[v]);
            for (int a = 0; a < 3; ++a) {
                double o = f16_round_d((bc[3 * v + a] - t->qcom[3 * P + a]) / sl);
                t->qcode[4 * v + a] = (float)o;
                t->qcom[3 * v + a] = t->qcom[3 * P + a] + o * sl;
            }
            double f = f16_round_d(bm[v] / t->qmass[P]);
            t->qcode[4 * v + 3] = (float)f;
            t->qmass[v] = t->qmass[P] * f;
        }
        free(bm);
        free(bc);
    }
    t->cmp = on ? 1 : 0;
    return 0;
}

/* The decoded aggregates and the stored codes, for tests: qagg [n][4] = com^q xyz, m^q;
 * code [n][4] = o_x, o_y, o_z, f (the root's row is zero). */
void orc_tree_compressed(const orc_tree* t, double* qagg, float* code)
{
    for (int64_t i = 0; i < t->n_nodes; ++i) {
        for (int a = 0; a < 3; ++a) qagg[4 * i + a] = t->qcom[3 * i + a];
        qagg[4 * i + 3] = t->qmass[i];
        for (int a = 0; a < 4; ++a) code[4 * i + a] = t->qcode[4 * i + a];
    }
}

static double node_term(const orc_tree* t, const kparams* kp, int64_t i, const double q[3]);
static double node_term_m(const orc_tree* t, const kparams* kp, int64_t i, const double q[3], double* margin);

static double point_term(const orc_tree* t, const kparams* kp, int64_t s, const double q[3])
{
    return term(kp, &t->pxyz[3 * s], t->pw[s], &t->pdip[3 * s], q);
}

/* Sensitivity of a term to its centre: |grad_p f(p, q)| * |p|, where the
 * gradient is taken with respect to the term's position p (a source point or
 * a node's centre of mass).  A float32 tree stores every centre with an error
 * of a few 2^-24 |p|, so this bounds how far a float32 evaluation of the same
 * estimate can move for reasons other than rounding in the evaluation
 * itself.  Potential and smooth distance: the exact gradient norm
 * (m r / (r^2 + eps^2)^(3/2) and alpha m e^(-alpha r)).  Winding number: the
 * gradient of dip.(p - q) / (4 pi r^3) is (dip - 3 (dip.u) u) / (4 pi r^3)
 * with u the unit offset, whose norm lies between |dip| / (4 pi r^3) and
 * 2 |dip| / (4 pi r^3); the bound 4 |dip| / (4 pi r^3) is used.
 * Diagnostic only; it never enters an estimate. */
static double sens_at(const kparams* kp, const double p[3], double m, const double dip[3], const double q[3])
{
    double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
    double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
    double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    switch (kp->kernel) {
    case ORC_POTENTIAL: {
        double s2 = r2 + kp->eps * kp->eps;
        return m * r / (s2 * sqrt(s2)) * pn;
    }
    case ORC_WINDING: {
        if (r2 == 0.0) return 0.0;
        double dn = sqrt(dip[0] * dip[0] + dip[1] * dip[1] + dip[2] * dip[2]);
        return dn / (ORC_PI * r2 * r) * pn;
    }
    case ORC_SMOOTHDIST:
        return kp->alpha * m * exp(-kp->alpha * r) * pn;
    default:
        return 0.0;
    }
}

static double node_sens(const orc_tree* t, const kparams* kp, int64_t i, const double q[3])
{
    return sens_at(kp, node_com(t, i), node_mass(t, i), &t->dip[3 * i], q);
}

/* One term and its sensitivity at an arbitrary (p, m, dip, q): out = {f, sens}
 * (for the tests that pin the sensitivity against finite differences of f). */
void orc_term_sens(int kernel, double eps, double alpha, const double p[3], double m, const double dip[3],
                   const double q[3], double out[2])
{
    kparams kp = {kernel, eps, alpha};
    out[0] = term(&kp, p, m, dip, q);
    out[1] = sens_at(&kp, p, m, dip, q);
}

static double dist2(const double a[3], const double q[3])
{
    double dx = a[0] - q[0], dy = a[1] - q[1], dz = a[2] - q[2];
    return dx * dx + dy * dy + dz * dz;
}

static double dist3(const double a[3], const double q[3]) { return sqrt(dist2(a, q)); }

/* |B| of node i, and of a virtual child (one point) of leaf i, under the
 * tree's diameter reading. */
static double node_diam(const orc_tree* t, int64_t i)
{
    if (t->diam_mode == 2) return t->bdiag[i];
    double c = t->diam[t->level[i]];
    return t->diam_mode == 1 ? c / sqrt(3.0) : c;
}

/* The second-order term of node i for the potential f = (r^2 + eps^2)^(-1/2):
 * expanding f(p) about the centre of mass c, the first-order terms cancel
 * (c is the weighted mean) and the second-order one is 1/2 sum_ij Q_ij
 * d_i d_j f with d_i d_j f = 3 u^5 x_i x_j - u^3 delta_ij (x = c - q,
 * u = (|x|^2 + eps^2)^(-1/2)): 1/2 u^5 (3 x^T Q x - tr(Q) (|x|^2 + eps^2)).
 * It is added where the node is far (|x| >= |B|, the threshold under which
 * Eq. (5) never stops a path), since the expansion diverges inside the node.
 * margin, if given, takes the relative distance of |x| / |B| from 1 (the
 * decision a float32 evaluation may take the other way). */
static double quad_term(const orc_tree* t, const kparams* kp, int64_t i, const double q[3], double* margin)
{
    const double* c = &t->com[3 * i];
    const double* Q = &t->quad[6 * i];
    double x = c[0] - q[0], y = c[1] - q[1], z = c[2] - q[2];
    double r2 = x * x + y * y + z * z, B = node_diam(t, i);
    if (margin) {
        double g = fabs(sqrt(r2) / B - 1.0);
        if (g < *margin) *margin = g;
    }
    if (!(r2 >= B * B)) return 0.0;
    double s2 = r2 + kp->eps * kp->eps, u = 1.0 / sqrt(s2), u2 = u * u;
    double xQx = Q[0] * x * x + Q[1] * y * y + Q[2] * z * z + 2.0 * (Q[3] * x * y + Q[4] * x * z + Q[5] * y * z);
    return 0.5 * u * u2 * u2 * (3.0 * xQx - (Q[0] + Q[1] + Q[2]) * s2);
}

static double node_term_m(const orc_tree* t, const kparams* kp, int64_t i, const double q[3], double* margin)
{
    double v = term(kp, node_com(t, i), node_mass(t, i), &t->dip[3 * i], q);
    if (t->lod == 2 && kp->kernel == ORC_POTENTIAL) v += quad_term(t, kp, i, q, margin);
    return v;
}

static double node_term(const orc_tree* t, const kparams* kp, int64_t i, const double q[3])
{
    return node_term_m(t, kp, i, q, NULL);
}

/* lod 1: point-mass node terms (the paper's); lod 2: plus the quadrupole term
 * (potential only).  The second-moment tensors are computed on first use,
 * from each node's own points about its centre of mass (float64).  The
 * compressed aggregates and lod 2 exclude each other (returns -1). */
int orc_tree_set_lod(orc_tree* t, int lod)
{
    if (lod != 1 && lod != 2) return -1;
    if (lod == 2 && t->cmp) return -1;
    if (lod == 2 && !t->quad) {
        t->quad = calloc(6 * (size_t)t->n_nodes, sizeof(double));
        for (int64_t v = 0; v < t->n_nodes; ++v) {
            const double* c = &t->com[3 * v];
            double* Q = &t->quad[6 * v];
            for (int64_t s = t->begin[v]; s < t->begin[v] + t->count[v]; ++s) {
                double w = t->pw[s];
                double x = t->pxyz[3 * s] - c[0], y = t->pxyz[3 * s + 1] - c[1], z = t->pxyz[3 * s + 2] - c[2];
                Q[0] += w * x * x; Q[1] += w * y * y; Q[2] += w * z * z;
                Q[3] += w * x * y; Q[4] += w * x * z; Q[5] += w * y * z;
            }
        }
    }
    t->lod = lod;
    return 0;
}

/* The second-moment tensors, for tests: quad [n][6] (lod 2 computes them). */
void orc_tree_quad(const orc_tree* t, double* quad)
{
    for (int64_t i = 0; i < 6 * t->n_nodes; ++i) quad[i] = t->quad ? t->quad[i] : 0.0;
}

/* A node's term at an arbitrary query under the tree's lod (tests). */
double orc_node_term(const orc_tree* t, int kernel, double eps, double alpha, int64_t i, const double q[3])
{
    kparams kp = {kernel, eps, alpha};
    return node_term(t, &kp, i, q);
}

static double point_diam(const orc_tree* t, int64_t leaf)
{
    if (t->diam_mode == 2) return 0.0;
    double c = t->diam[t->level[leaf] + 1];
    return t->diam_mode == 1 ? c / sqrt(3.0) : c;
}

/* Switch the tree's reading of |B| (mode as in orc_tree); returns 0 on success. */
int orc_tree_set_diam_mode(orc_tree* t, int mode)
{
    if (mode < 0 || mode > 2) return -1;
    if (mode == 2 && !t->bdiag) {
        t->bdiag = malloc(t->n_nodes * sizeof(double));
        for (int64_t i = 0; i < t->n_nodes; ++i) {
            double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int64_t s = t->begin[i]; s < t->begin[i] + t->count[i]; ++s)
                for (int a = 0; a < 3; ++a) {
                    double x = t->pxyz[3 * s + a];
                    if (x < lo[a]) lo[a] = x;
                    if (x > hi[a]) hi[a] = x;
                }
            double e2 = 0.0;
            for (int a = 0; a < 3; ++a) e2 += (hi[a] - lo[a]) * (hi[a] - lo[a]);
            t->bdiag[i] = sqrt(e2);
        }
    }
    t->diam_mode = mode;
    return 0;
}

static double leaf_exact(const orc_tree* t, const kparams* kp, int64_t i, const double q[3])
{
    double s = 0.0;
    for (int64_t k = t->begin[i]; k < t->begin[i] + t->count[i]; ++k) s += point_term(t, kp, k, q);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Barnes-Hut, Algorithm 1 / Eq. (2).  The far-field test is                  */
/* ||q - com|| / |B| >= beta.  A leaf that is not far is summed exactly.      */
/* Vote mode (group > 1): for each group of `group` consecutive queries a     */
/* node is opened iff some query of the group fails the far-field test; all   */
/* queries of the group then share the same cut.  group = 1 is per query.    */
/* ------------------------------------------------------------------------ */
static void bh_group(const orc_tree* t, const kparams* kp, int64_t node, const double* qs, int gn,
                     double beta, double* acc, double* margin, int64_t* visited)
{
    int open = 0;
    *visited += 1;
    for (int g = 0; g < gn; ++g) {
        double bt = dist3(node_com(t, node), &qs[3 * g]) / node_diam(t, node);
        double mg = fabs(bt - beta) / beta;
        if (mg < margin[g]) margin[g] = mg;
        if (!(bt >= beta)) open = 1;
    }
    if (!open) {
        for (int g = 0; g < gn; ++g) acc[g] += node_term(t, kp, node, &qs[3 * g]);
        return;
    }
    if (!is_internal(t, node)) {
        for (int g = 0; g < gn; ++g) acc[g] += leaf_exact(t, kp, node, &qs[3 * g]);
        return;
    }
    for (int c = 0; c < t->nchild[node]; ++c)
        bh_group(t, kp, t->first_child[node] + c, qs, gn, beta, acc, margin, visited);
}

void orc_bh(const orc_tree* t, const float* qry, int64_t n, int kernel, double eps, double alpha,
            double beta, int group, double* out, double* min_margin, int64_t* visited, int nthreads)
{
    kparams kp = {kernel, eps, alpha};
    if (group < 1) group = 1;
    int64_t ng = (n + group - 1) / group;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t gi = 0; gi < ng; ++gi) {
        int64_t j0 = gi * group;
        int gn = (int)((n - j0 < group) ? (n - j0) : group);
        double* qs = malloc(3 * gn * sizeof(double));
        double* acc = calloc(gn, sizeof(double));
        double* mg = malloc(gn * sizeof(double));
        for (int g = 0; g < gn; ++g) {
            for (int a = 0; a < 3; ++a) qs[3 * g + a] = qry[3 * (j0 + g) + a];
            mg[g] = INFINITY;
        }
        int64_t vis = 0;
        bh_group(t, &kp, 0, qs, gn, beta, acc, mg, &vis);
        for (int g = 0; g < gn; ++g) {
            out[j0 + g] = acc[g];
            if (min_margin) min_margin[j0 + g] = mg[g];
            if (visited) visited[j0 + g] = vis;
        }
        free(qs); free(acc); free(mg);
    }
}

/* ======================================================================== */
/* Learned child proposal (importance sampling of the path index, which     */
/* Section 3.3 leaves open).  A node-level MLP 8 -> 32 -> 32 -> 8 (ReLU)     */
/* maps one feature per child slot (d = 2) -- the log of the child's         */
/* quadrupole score relative to its siblings -- to one logit per slot, with  */
/* the features also added to the logits (times 16), so that a zero network */
/* samples in proportion to the scores.                                      */
/* Proposal: pi_c = exp(z_c) / sum exp(z) over non-empty slots, mixed        */
/* defensively with the uniform path index:                                  */
/*   q_c = (1 - LAMBDA) pi_c + LAMBDA n_c / n_T,                             */
/* so every non-empty child keeps q_c > 0 and Theorem 1 still applies.      */
/* Parameters (float32, 1608): W1[32][8] b1[32] W2[32][32] b2[32]            */
/* W3[8][32] b3[8].  Inference uses the weight matrices rounded to binary16  */
/* and binary16 inputs and hidden activations with float32 sums, which this */
/* oracle emulates (mode 1); mode 0 is plain float64 for gradient checks.   */
/* ======================================================================== */
#define MLP_IN 8
#define MLP_H 32
#define MLP_OUT 8
#define MLP_OFF_W1 0
#define MLP_OFF_B1 (MLP_OFF_W1 + MLP_H * MLP_IN)
#define MLP_OFF_W2 (MLP_OFF_B1 + MLP_H)
#define MLP_OFF_B2 (MLP_OFF_W2 + MLP_H * MLP_H)
#define MLP_OFF_W3 (MLP_OFF_B2 + MLP_H)
#define MLP_OFF_B3 (MLP_OFF_W3 + MLP_OUT * MLP_H)
#define MLP_NPARAM (MLP_OFF_B3 + MLP_OUT)
#define MLP_LAMBDA 0.125

int orc_mlp_nparam(void) { return MLP_NPARAM; }

/* nearest IEEE binary16 value of x (ties to even), as a float; overflow to inf */
static float f16_round(float x)
{
    if (!(x == x) || x == 0.0f || isinf(x)) return x;
    int e;
    double m = frexp((double)x, &e);   /* x = m 2^e, 0.5 <= |m| < 1 */
    (void)m;
    int ex = e - 1;                    /* x = m' 2^ex, 1 <= |m'| < 2 */
    if (ex < -14) ex = -14;            /* subnormal range: fixed quantum 2^-24 */
    double quantum = ldexp(1.0, ex - 10);
    double r = nearbyint((double)x / quantum) * quantum;   /* default rounding: to nearest even */
    if (fabs(r) > 65504.0) return x > 0 ? INFINITY : -INFINITY;
    return (float)r;
}

float orc_f16_round(float x) { return f16_round(x); }

/* Features of (internal node T, query q): one per child slot k.  For child c
 * in slot k, with mass m_c, centre of mass p_c and second moment
 * s_c^2 = sum w |p - p_c|^2 / m_c,
 *   score_c = m_c s_c^2 / (|p_c - q|^2 + s_c^2)^(3/2)
 * is the size of the quadrupole term of c's residual under the 1/r kernel
 * (softened inside c's spread), and
 *   f_k = max(-1, ln(score_c / max_c' score_c') / 16),
 * -1 for an empty slot (and for every slot when all scores are 0). */
static void mlp_features(const orc_tree* t, int64_t T, const double q[3], double f[8])
{
    double sc[8];
    double smax = 0.0;
    for (int k = 0; k < 8; ++k) { sc[k] = -1.0; f[k] = -1.0; }
    for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch) {
        double r2 = dist2(&t->com[3 * ch], q);
        double s2 = t->spr[ch];
        double v = t->mass[ch] * s2 / pow(r2 + s2, 1.5);
        if (!(r2 + s2 > 0.0)) v = 0.0;
        sc[t->digit[ch]] = v;
        if (v > smax) smax = v;
    }
    if (smax > 0.0)
        for (int k = 0; k < 8; ++k)
            if (sc[k] > 0.0) {
                double l = log(sc[k] / smax) / 16.0;
                f[k] = l > -1.0 ? l : -1.0;
            }
}

/* Logits z = W3 h2 + b3 + 16 x (the features pass straight to the logits, so
 * an all-zero network proposes in proportion to the children's scores).
 * mode 1: binary16 weights / inputs / hidden activations, each dot product
 * summed exactly and rounded once to float32, bias and skip term added in
 * float32; mode 0: float64 throughout.  Optional outputs keep the
 * activations. */
static void mlp_forward(const float* prm, const float x[8], int mode, double z[8], double h1o[32], double h2o[32])
{
    double xin[MLP_IN], h1[MLP_H], h2[MLP_H];
    for (int k = 0; k < MLP_IN; ++k) xin[k] = mode ? f16_round(x[k]) : (double)x[k];
    for (int n = 0; n < MLP_H; ++n) {
        double s = 0.0;
        for (int k = 0; k < MLP_IN; ++k) {
            double w = mode ? f16_round(prm[MLP_OFF_W1 + n * MLP_IN + k]) : prm[MLP_OFF_W1 + n * MLP_IN + k];
            s += w * xin[k];
        }
        double a;
        if (mode) { float af = (float)s; af = af + prm[MLP_OFF_B1 + n]; a = af > 0.0f ? f16_round(af) : 0.0; }
        else { a = s + prm[MLP_OFF_B1 + n]; a = a > 0.0 ? a : 0.0; }
        h1[n] = a;
    }
    for (int n = 0; n < MLP_H; ++n) {
        double s = 0.0;
        for (int k = 0; k < MLP_H; ++k) {
            double w = mode ? f16_round(prm[MLP_OFF_W2 + n * MLP_H + k]) : prm[MLP_OFF_W2 + n * MLP_H + k];
            s += w * h1[k];
        }
        double a;
        if (mode) { float af = (float)s; af = af + prm[MLP_OFF_B2 + n]; a = af > 0.0f ? f16_round(af) : 0.0; }
        else { a = s + prm[MLP_OFF_B2 + n]; a = a > 0.0 ? a : 0.0; }
        h2[n] = a;
    }
    for (int c = 0; c < MLP_OUT; ++c) {
        double s = 0.0;
        for (int k = 0; k < MLP_H; ++k) {
            double w = mode ? f16_round(prm[MLP_OFF_W3 + c * MLP_H + k]) : prm[MLP_OFF_W3 + c * MLP_H + k];
            s += w * h2[k];
        }
        if (mode) { float af = (float)s; af = af + prm[MLP_OFF_B3 + c]; af = af + 16.0f * x[c]; z[c] = af; }
        else z[c] = s + prm[MLP_OFF_B3 + c] + 16.0 * (double)x[c];
    }
    if (h1o) for (int n = 0; n < MLP_H; ++n) h1o[n] = h1[n];
    if (h2o) for (int n = 0; n < MLP_H; ++n) h2o[n] = h2[n];
}

/* softmax over the non-empty slots (cnt > 0) */
static void masked_softmax(const double z[8], const double cnt[8], double pi[8])
{
    double zmax = -INFINITY, s = 0.0;
    for (int c = 0; c < MLP_OUT; ++c) if (cnt[c] > 0 && z[c] > zmax) zmax = z[c];
    for (int c = 0; c < MLP_OUT; ++c) { pi[c] = cnt[c] > 0 ? exp(z[c] - zmax) : 0.0; s += pi[c]; }
    for (int c = 0; c < MLP_OUT; ++c) pi[c] /= s;
}

/* q_c for the (up to 8) children of internal node T: the network's softmax
 * mixed with the uniform path index, q = (1 - lambda) pi + lambda n_c / n_T.
 * The features enter the network as float32 values. */
static void learned_q(const orc_tree* t, const float* prm, int64_t T, const double q[3], double qc[8],
                      int slot_of_child[8], int* nk)
{
    double f[8];
    float xf[8];
    double z[8], cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0}, pi[8];
    mlp_features(t, T, q, f);
    for (int k = 0; k < 8; ++k) xf[k] = (float)f[k];
    mlp_forward(prm, xf, 1, z, NULL, NULL);
    *nk = t->nchild[T];
    for (int i = 0; i < t->nchild[T]; ++i) {
        int64_t ch = t->first_child[T] + i;
        slot_of_child[i] = t->digit[ch];
        cnt[t->digit[ch]] = (double)t->count[ch];
    }
    masked_softmax(z, cnt, pi);
    for (int i = 0; i < t->nchild[T]; ++i) {
        int s = slot_of_child[i];
        qc[i] = (1.0 - MLP_LAMBDA) * pi[s] + MLP_LAMBDA * cnt[s] / (double)t->count[T];
    }
}

/* Score proposal of one query: pi_c = max(score_c / max score, e^-16)
 * normalised over the non-empty slots (uniform over them when every score is
 * 0), i.e. the softmax of 16 f with the features above; by slot. */
static void score_pi(const orc_tree* t, int64_t T, const double q[3], double pi[8])
{
    double sc[8], smax = 0.0, tot = 0.0;
    int ne[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 8; ++k) { sc[k] = 0.0; pi[k] = 0.0; }
    for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch) {
        double r2 = dist2(&t->com[3 * ch], q), s2 = t->spr[ch];
        double v = (r2 + s2 > 0.0) ? t->mass[ch] * s2 / pow(r2 + s2, 1.5) : 0.0;
        sc[t->digit[ch]] = v;
        ne[t->digit[ch]] = 1;
        if (v > smax) smax = v;
    }
    for (int k = 0; k < 8; ++k) {
        if (!ne[k]) continue;
        double r = smax > 0.0 ? sc[k] / smax : 1.0;
        pi[k] = r > exp(-16.0) ? r : exp(-16.0);
        tot += pi[k];
    }
    for (int k = 0; k < 8; ++k) pi[k] /= tot;
}

/* Which child distribution the estimator uses at internal nodes:
 *   prm != NULL: the learned proposal of each query (learned_q);
 *   tile != NULL: the tile-shared score proposal: queries are grouped in tiles
 *     of 64 consecutive indices, and every query of a tile uses
 *     q_c = (1 - LAMBDA) mean over the tile of score_pi_c + LAMBDA n_c / n_T
 *     (tile = the tile's query positions, ntile of them);
 *   neither: the uniform path index. */
typedef struct {
    const float* prm;
    const float* tile;
    int64_t ntile;
} proposal;

/* q_c per child of internal node T (children order); returns 0 for the uniform path index */
static int proposal_q(const orc_tree* t, const proposal* pr, int64_t T, const double q[3], double qc[8],
                      int slots[8], int* nk)
{
    if (pr && pr->prm) {
        learned_q(t, pr->prm, T, q, qc, slots, nk);
        return 1;
    }
    if (pr && pr->tile) {
        double mean[8] = {0, 0, 0, 0, 0, 0, 0, 0}, pi[8];
        for (int64_t i = 0; i < pr->ntile; ++i) {
            double qi[3] = {pr->tile[3 * i], pr->tile[3 * i + 1], pr->tile[3 * i + 2]};
            score_pi(t, T, qi, pi);
            for (int k = 0; k < 8; ++k) mean[k] += pi[k];
        }
        *nk = t->nchild[T];
        for (int i = 0; i < t->nchild[T]; ++i) {
            int64_t ch = t->first_child[T] + i;
            slots[i] = t->digit[ch];
            qc[i] = (1.0 - MLP_LAMBDA) * mean[slots[i]] / (double)pr->ntile +
                    MLP_LAMBDA * (double)t->count[ch] / (double)t->count[T];
        }
        return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Stochastic path estimator: Eqs. (5)-(7), Section 3.3.1, Algorithm 2.       */
/* ------------------------------------------------------------------------ */

/* Russian-roulette probability of moving from a node (far-field ratio bT) to
 * its chosen child (far-field ratio bc): Eq. (5), or the ablations
 * rr_mode 1 (p = 1, no roulette) and 2 (p = 1/2). */
static double rr_prob(int rr_mode, double bT, double bc)
{
    if (rr_mode == 1) return 1.0;
    if (rr_mode == 2) return 0.5;
    if (bc == 0.0) return 1.0;
    double r = (bT > 1.0 ? bT : 1.0) / bc;
    return r < 1.0 ? r : 1.0;
}

typedef struct {
    double value;    /* estimate of this path's residual sum */
    double absum;    /* sum of |terms| that entered it, weighted like the value */
    double sens;     /* sum of node-term sensitivities (node_sens), weighted like the value */
    double margin;   /* min |u - p| over its roulette decisions */
    int32_t end_begin, end_level, steps, flags;
} path_out;

/* One path sample rooted at subdomain node `a` (Algorithm 2, inner loop).
 * counter = (sigma, a_slot*S + s, step/2, batch), key = (seed lo, seed hi). */
static path_out sample_path(const orc_tree* t, const kparams* kp, const double q[3], int64_t a,
                            uint32_t sigma, uint32_t stream2, uint32_t ctr2_base, uint32_t batch, uint64_t seed,
                            int rr_mode, const proposal* prop)
{
    path_out po = {0.0, 0.0, 0.0, INFINITY, 0, 0, 0, 0};
    int64_t T = a;                  /* current node (a real node) */
    double tT = node_term_m(t, kp, a, q, &po.margin);
    double p_sel = 1.0;             /* probability that the path index lies in T */
    double p_rr = 1.0;              /* running product of roulette probabilities */
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int k = 0;; ++k) {
        int64_t nT = t->count[T];
        po.end_begin = (int32_t)t->begin[T];
        po.end_level = t->level[T];
        /* a one-point node: nothing left to refine (with compressed aggregates its term is not
         * its point's, so it takes one more step, onto the point as a virtual child) */
        if (nT == 1 && !t->cmp) { po.flags = 1; break; }
        uint32_t ctr[4] = {sigma, stream2, ctr2_base + (uint32_t)(k >> 1), batch}, rnd[4];
        orc_philox4x32_10(ctr, key, rnd);
        uint32_t x_sel = rnd[2 * (k & 1)], x_rr = rnd[2 * (k & 1) + 1];
        double u_rr = (double)(x_rr >> 8) * (1.0 / 16777216.0);
        /* uniform path index inside T: offset r in [0, nT) */
        int64_t r = (int64_t)(((uint64_t)x_sel * (uint64_t)nT) >> 32);
        int64_t target = t->begin[T] + r;
        double bT = dist3(node_com(t, T), q) / node_diam(t, T);
        double sum_children = 0.0, abs_children = 0.0, sens_step = node_sens(t, kp, T, q);
        double bc, tc, q_c;
        int64_t c_node = -1;
        if (is_internal(t, T)) {
            int64_t c = -1;
            for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch) {
                double v = node_term_m(t, kp, ch, q, &po.margin);
                sum_children += v;
                abs_children += fabs(v);
                sens_step += node_sens(t, kp, ch, q);
                if (target >= t->begin[ch] && target < t->begin[ch] + t->count[ch]) c = ch;
            }
            q_c = (double)t->count[c] / (double)nT;
            double qv[8];
            int slots[8], nk;
            if (proposal_q(t, prop, T, q, qv, slots, &nk)) {
                /* learned or score proposal: inverse-CDF selection over the slots with a 24-bit uniform */
                double u_sel = (double)(x_sel >> 8) * (1.0 / 16777216.0), cum = 0.0;
                int ci = nk - 1;
                for (int i = 0; i < nk; ++i) {
                    cum += qv[i];
                    double mg = fabs(u_sel - cum);
                    if (i < nk - 1 && mg < po.margin) po.margin = mg;
                    if (u_sel < cum) { ci = i; break; }
                }
                c = t->first_child[T] + ci;
                q_c = qv[ci];
            }
            c_node = c;
            bc = dist3(node_com(t, c), q) / node_diam(t, c);
            tc = node_term(t, kp, c, q);
        } else {
            /* leaf with several points: the points are virtual children */
            for (int64_t s = t->begin[T]; s < t->begin[T] + nT; ++s) {
                double v = point_term(t, kp, s, q);
                sum_children += v;
                abs_children += fabs(v);
            }
            bc = dist3(&t->pxyz[3 * target], q) / point_diam(t, T);
            tc = point_term(t, kp, target, q);
            q_c = 1.0 / (double)nT;
        }
        double p = rr_prob(rr_mode, bT, bc);
        double mg = fabs(u_rr - p);
        if (rr_mode == 0 && mg < po.margin) po.margin = mg;
        if (u_rr >= p) { po.flags = 0; break; }
        p_rr *= p;
        double delta = sum_children - tT;          /* contribution swap, Eq. (6) */
        double wgt = 1.0 / (p_sel * p_rr);          /* 1 / (p(I in T) p(K >= k+1)), Eq. (7) */
        po.value += delta * wgt;
        po.absum += (abs_children + fabs(tT)) * wgt;
        po.sens += sens_step * wgt;
        po.steps += 1;
        p_sel *= q_c;
        if (c_node < 0) {                           /* moved onto a virtual point */
            po.end_begin = (int32_t)target;
            po.end_level = t->level[T] + 1;
            po.flags = 2;
            break;
        }
        T = c_node;
        tT = tc;
    }
    return po;
}

/* Subdomains are the root's children (slot = digit); a root that is a leaf
 * is summed exactly.  The random stream of query j is its index (qindex[j]
 * when given, so that a subset can be evaluated as part of a larger set).
 * Output per query: F estimate; optional: minimal
 * roulette margin, conditioning sum, and per-path records laid out
 * [n][d^3][S] x int32{begin, level, steps, flags} (absent slots: begin -1). */
void orc_sbh(const orc_tree* t, const float* qry, int64_t n, int kernel, double eps, double alpha,
             int S, uint64_t seed, int G, uint32_t batch, int rr_mode, const int64_t* qindex, const float* prm,
             const float* tile_all, int64_t n_all, double* out, double* min_margin, double* absum, double* sens,
             int32_t* paths, int nthreads)
{
    kparams kp = {kernel, eps, alpha};
    int d3 = t->d * t->d * t->d;
    if (G < 1) G = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t j = 0; j < n; ++j) {
        double q[3] = {qry[3 * j], qry[3 * j + 1], qry[3 * j + 2]};
        int64_t jj = qindex ? qindex[j] : j;   /* the query's index in the full query set */
        uint32_t sigma = (uint32_t)(G == 1 ? jj : jj / G);
        proposal prop = {prm, NULL, 0};
        if (tile_all) {   /* the tile of 64 consecutive indices holding jj, within the full query set */
            int64_t t0 = (jj / 64) * 64, t1 = t0 + 64 < n_all ? t0 + 64 : n_all;
            prop.tile = &tile_all[3 * t0];
            prop.ntile = t1 - t0;
        }
        double F = 0.0, A = 0.0, SN = 0.0, mg = INFINITY;
        if (paths)
            for (int k = 0; k < d3 * S; ++k) {
                int32_t* rec = &paths[((int64_t)j * d3 * S + k) * 4];
                rec[0] = -1; rec[1] = 0; rec[2] = 0; rec[3] = 0;
            }
        if (!is_internal(t, 0)) {
            F = leaf_exact(t, &kp, 0, q);
            A = fabs(F);
        } else {
            for (int ci = 0; ci < t->nchild[0]; ++ci) {
                int64_t a = t->first_child[0] + ci;
                int slot = t->digit[a];
                double cv = node_term_m(t, &kp, a, q, &mg);     /* control variate CV_a */
                double Fa = 0.0, Aa = 0.0, Sa = 0.0;
                for (int s = 0; s < S; ++s) {
                    path_out po = sample_path(t, &kp, q, a, sigma, (uint32_t)(slot * S + s), 0u, batch, seed, rr_mode,
                                              &prop);
                    Fa += po.value;
                    Aa += po.absum;
                    Sa += po.sens;
                    if (po.margin < mg) mg = po.margin;
                    if (paths) {
                        int32_t* rec = &paths[((int64_t)j * d3 * S + (int64_t)slot * S + s) * 4];
                        rec[0] = po.end_begin; rec[1] = po.end_level; rec[2] = po.steps; rec[3] = po.flags;
                    }
                }
                F += cv + Fa / S;
                A += fabs(cv) + Aa / S;
                SN += node_sens(t, &kp, a, q) + Sa / S;
            }
        }
        out[j] = F;
        if (min_margin) min_margin[j] = mg;
        if (absum) absum[j] = A;
        if (sens) sens[j] = SN;
    }
}

/* ------------------------------------------------------------------------ */
/* The roulette voted over a tile (rr_mode 3).  The queries of a tile of 64  */
/* consecutive indices share one random stream (G a multiple of 64), so     */
/* under the uniform path index they walk the same node sequence and test   */
/* the same variate u.  Here the tile also shares the roulette probability: */
/* at each step every query of the tile continues with p = the largest      */
/* Eq. (5) probability among the tile's queries with finite coordinates (a  */
/* probability fixed before u is drawn, so each query's estimate stays      */
/* unbiased, as for any roulette in (0, 1]; Theorem 1).  The tile stops or  */
/* continues together.  Counters, selection and the estimate are those of   */
/* sample_path.  Per query: value, margin (|u - p| of its tile's            */
/* decisions), absum, sens and path records as orc_sbh's.                   */
/* ------------------------------------------------------------------------ */
static int finite3(const double* q) { return isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]); }

/* the voted probability of the step from T onto child c (c < 0: onto point `target` of leaf T) */
static double vote_prob(const orc_tree* t, const double* qs, int gn, int64_t T, int64_t c, int64_t target)
{
    double pw = 0.0;
    for (int g = 0; g < gn; ++g) {
        const double* q = &qs[3 * g];
        if (!finite3(q)) continue;
        double bT = dist3(node_com(t, T), q) / node_diam(t, T);
        double bc = c >= 0 ? dist3(node_com(t, c), q) / node_diam(t, c)
                           : dist3(&t->pxyz[3 * target], q) / point_diam(t, T);
        double p = rr_prob(0, bT, bc);
        if (p > pw) pw = p;
    }
    return pw;
}
static void vote_group(const orc_tree* t, const kparams* kp, const double* qs, int gn, uint32_t sigma, int S,
                       uint64_t seed, uint32_t batch, int d3, double* F, double* A, double* SN, double* mg,
                       int32_t* paths)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double* tT = malloc(sizeof(double) * gn);
    double* acc = malloc(sizeof(double) * gn);
    double* ab = malloc(sizeof(double) * gn);
    double* sn = malloc(sizeof(double) * gn);
    double* sum = malloc(sizeof(double) * gn);
    double* abc = malloc(sizeof(double) * gn);
    double* snc = malloc(sizeof(double) * gn);
    double* tc = malloc(sizeof(double) * gn);
    double* Fa = malloc(sizeof(double) * gn);
    double* Aa = malloc(sizeof(double) * gn);
    double* Sa = malloc(sizeof(double) * gn);
    for (int ci = 0; ci < t->nchild[0]; ++ci) {
        int64_t a = t->first_child[0] + ci;
        int slot = t->digit[a];
        for (int g = 0; g < gn; ++g) { Fa[g] = 0.0; Aa[g] = 0.0; Sa[g] = 0.0; }
        for (int s = 0; s < S; ++s) {
            int64_t T = a;
            double p_sel = 1.0, p_rr = 1.0;
            int32_t end_b = (int32_t)t->begin[a], end_l = t->level[a], steps = 0, flags = 0;
            for (int g = 0; g < gn; ++g) {
                tT[g] = node_term_m(t, kp, a, &qs[3 * g], &mg[g]);
                acc[g] = 0.0; ab[g] = 0.0; sn[g] = 0.0;
            }
            for (int k = 0;; ++k) {
                int64_t nT = t->count[T];
                end_b = (int32_t)t->begin[T];
                end_l = t->level[T];
                if (nT == 1 && !t->cmp) { flags = 1; break; }
                uint32_t ctr[4] = {sigma, (uint32_t)(slot * S + s), (uint32_t)(k >> 1), batch}, rnd[4];
                orc_philox4x32_10(ctr, key, rnd);
                uint32_t x_sel = rnd[2 * (k & 1)], x_rr = rnd[2 * (k & 1) + 1];
                double u = (double)(x_rr >> 8) * (1.0 / 16777216.0);
                int64_t r = (int64_t)(((uint64_t)x_sel * (uint64_t)nT) >> 32);
                int64_t target = t->begin[T] + r, c = -1;
                double q_c;
                int internal = is_internal(t, T);
                if (internal) {
                    for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch)
                        if (target >= t->begin[ch] && target < t->begin[ch] + t->count[ch]) c = ch;
                    q_c = (double)t->count[c] / (double)nT;
                } else {
                    q_c = 1.0 / (double)nT;
                }
                /* every query's Eq. (5) probability at this step; the tile takes the largest */
                double pw = vote_prob(t, qs, gn, T, internal ? c : -1, target);
                for (int g = 0; g < gn; ++g) {
                    double m = fabs(u - pw);
                    if (m < mg[g]) mg[g] = m;
                }
                if (u >= pw) { flags = 0; break; }
                p_rr *= pw;
                double wgt = 1.0 / (p_sel * p_rr);
                for (int g = 0; g < gn; ++g) {
                    const double* q = &qs[3 * g];
                    sum[g] = 0.0; abc[g] = 0.0; snc[g] = node_sens(t, kp, T, q);
                    if (internal) {
                        for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch) {
                            double v = node_term_m(t, kp, ch, q, &mg[g]);
                            sum[g] += v;
                            abc[g] += fabs(v);
                            snc[g] += node_sens(t, kp, ch, q);
                        }
                        tc[g] = node_term(t, kp, c, q);
                    } else {
                        for (int64_t p = t->begin[T]; p < t->begin[T] + nT; ++p) {
                            double v = point_term(t, kp, p, q);
                            sum[g] += v;
                            abc[g] += fabs(v);
                        }
                    }
                    acc[g] += (sum[g] - tT[g]) * wgt;
                    ab[g] += (abc[g] + fabs(tT[g])) * wgt;
                    sn[g] += snc[g] * wgt;
                }
                steps += 1;
                p_sel *= q_c;
                if (!internal) {
                    end_b = (int32_t)target;
                    end_l = t->level[T] + 1;
                    flags = 2;
                    break;
                }
                T = c;
                for (int g = 0; g < gn; ++g) tT[g] = tc[g];
            }
            for (int g = 0; g < gn; ++g) { Fa[g] += acc[g]; Aa[g] += ab[g]; Sa[g] += sn[g]; }
            if (paths)
                for (int g = 0; g < gn; ++g) {
                    int32_t* rec = &paths[((int64_t)g * d3 * S + (int64_t)slot * S + s) * 4];
                    rec[0] = end_b; rec[1] = end_l; rec[2] = steps; rec[3] = flags;
                }
        }
        for (int g = 0; g < gn; ++g) {
            const double* q = &qs[3 * g];
            double cv = node_term_m(t, kp, a, q, &mg[g]);
            F[g] += cv + Fa[g] / S;
            A[g] += fabs(cv) + Aa[g] / S;
            SN[g] += node_sens(t, kp, a, q) + Sa[g] / S;
        }
    }
    free(tT); free(acc); free(ab); free(sn); free(sum); free(abc); free(snc); free(tc);
    free(Fa); free(Aa); free(Sa);
}

/* The voted roulette for n queries; stream id floor(qindex[j] / G) (qindex
 * NULL: j), G a multiple of 64; the queries vote in tiles of 64 consecutive
 * indices: a tile is a run of consecutive entries with equal floor(index /
 * 64) (a subset must hold whole tiles). */
void orc_sbh_vote(const orc_tree* t, const float* qry, int64_t n, int kernel, double eps, double alpha, int S,
                  uint64_t seed, int G, uint32_t batch, const int64_t* qindex, double* out, double* min_margin,
                  double* absum, double* sens, int32_t* paths, int nthreads)
{
    kparams kp = {kernel, eps, alpha};
    int d3 = t->d * t->d * t->d;
    if (G < 1) G = 1;
    /* group starts: a new group wherever the stream id changes */
    int64_t* start = malloc(sizeof(int64_t) * (n + 1));
    int64_t ng = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t jj = qindex ? qindex[j] : j;
        if (j == 0 || jj / 64 != (qindex ? qindex[j - 1] : j - 1) / 64) start[ng++] = j;
    }
    start[ng] = n;
    if (paths)
        for (int64_t k = 0; k < n * d3 * S; ++k) {
            int32_t* rec = &paths[k * 4];
            rec[0] = -1; rec[1] = 0; rec[2] = 0; rec[3] = 0;
        }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t gi = 0; gi < ng; ++gi) {
        int64_t j0 = start[gi], j1 = start[gi + 1];
        int gn = (int)(j1 - j0);
        double* qs = malloc(sizeof(double) * 3 * gn);
        double* F = calloc(gn, sizeof(double));
        double* A = calloc(gn, sizeof(double));
        double* SN = calloc(gn, sizeof(double));
        double* mg = malloc(sizeof(double) * gn);
        for (int g = 0; g < gn; ++g) {
            for (int c = 0; c < 3; ++c) qs[3 * g + c] = qry[3 * (j0 + g) + c];
            mg[g] = INFINITY;
        }
        int64_t jj = qindex ? qindex[j0] : j0;
        if (!is_internal(t, 0)) {
            for (int g = 0; g < gn; ++g) { F[g] = leaf_exact(t, &kp, 0, &qs[3 * g]); A[g] = fabs(F[g]); }
        } else {
            vote_group(t, &kp, qs, gn, (uint32_t)(jj / G), S, seed, batch, d3, F, A, SN, mg,
                       paths ? &paths[j0 * d3 * S * 4] : NULL);
        }
        for (int g = 0; g < gn; ++g) {
            out[j0 + g] = F[g];
            if (min_margin) min_margin[j0 + g] = mg[g];
            if (absum) absum[j0 + g] = A[g];
            if (sens) sens[j0 + g] = SN[g];
        }
        free(qs); free(F); free(A); free(SN); free(mg);
    }
    free(start);
}

/* ------------------------------------------------------------------------ */
/* Stratification by a Barnes-Hut cut (Section 3.3.1 names the contribution */
/* nodes D(q, beta) of a low beta as an alternative to the root's children   */
/* as path roots).  The cut is voted over groups of `vote` consecutive       */
/* queries, as Barnes-Hut's is: walking from the root, a node is a subdomain */
/* when every query of the group has far-field ratio >= beta_low; otherwise  */
/* an internal node is opened and a leaf is summed exactly.  Each subdomain a */
/* contributes its control variate m_a f(p_a, q) plus the mean of S path     */
/* samples rooted at a (Algorithm 2's inner loop).  The subdomains cover     */
/* every point once, so Theorem 1 applies to each and the sum is unbiased.   */
/* Random numbers: the path from subdomain a (first point b_a, level l_a),   */
/* sample s, step k draws from the Philox block with counter                 */
/* (stream id, b_a, l_a 2^24 + s 2^16 + floor(k/2), batch).                  */
/* Digest per query: {subdomains, leaves summed exactly, accepted steps over */
/* all paths, sum of the paths' end levels}.                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    double F, A, SN, mg;
    int32_t dig[4];
} cut_acc;

static double expect_rec(const orc_tree* t, const kparams* kp, const double q[3], int64_t T, double tT,
                         double ps, double pr, int rr_mode, const proposal* prop);

static void cut_group(const orc_tree* t, const kparams* kp, int64_t node, const double* qs, const uint32_t* sig,
                      int gn, double beta_low, int S, uint64_t seed, uint32_t batch, int rr_mode, int expect,
                      cut_acc* acc)
{
    int open = 0;
    for (int g = 0; g < gn; ++g) {
        double bt = dist3(node_com(t, node), &qs[3 * g]) / node_diam(t, node);
        if (!(bt >= beta_low)) open = 1;
    }
    if (!open) {
        for (int g = 0; g < gn; ++g) {
            const double* q = &qs[3 * g];
            double cv = node_term(t, kp, node, q);
            cut_acc* A = &acc[g];
            A->dig[0] += 1;
            if (expect) {   /* the exact expectation of the subdomain's paths (Theorem 1) */
                A->F += cv + (t->count[node] > 1 ? expect_rec(t, kp, q, node, cv, 1.0, 1.0, rr_mode, NULL) : 0.0);
                continue;
            }
            double Fa = 0.0, Aa = 0.0, Sa = 0.0;
            for (int s = 0; s < S; ++s) {
                uint32_t c2 = ((uint32_t)t->level[node] << 24) | ((uint32_t)s << 16);
                path_out po = sample_path(t, kp, q, node, sig[g], (uint32_t)t->begin[node], c2, batch, seed, rr_mode,
                                          NULL);
                Fa += po.value;
                Aa += po.absum;
                Sa += po.sens;
                if (po.margin < A->mg) A->mg = po.margin;
                A->dig[2] += po.steps;
                A->dig[3] += po.end_level;
            }
            A->F += cv + Fa / S;
            A->A += fabs(cv) + Aa / S;
            A->SN += node_sens(t, kp, node, q) + Sa / S;
        }
        return;
    }
    if (!is_internal(t, node)) {
        for (int g = 0; g < gn; ++g) {
            double v = leaf_exact(t, kp, node, &qs[3 * g]);
            acc[g].F += v;
            acc[g].A += fabs(v);
            acc[g].dig[1] += 1;
        }
        return;
    }
    for (int c = 0; c < t->nchild[node]; ++c)
        cut_group(t, kp, t->first_child[node] + c, qs, sig, gn, beta_low, S, seed, batch, rr_mode, expect, acc);
}

/* The cut-stratified estimator for n queries; stream id of query j is
 * floor(qindex[j] / G) (qindex NULL: j); votes over groups of `vote`
 * consecutive queries of the given set.  expect != 0: the exact expectation
 * instead of a sample. */
void orc_sbh_cut(const orc_tree* t, const float* qry, int64_t n, int kernel, double eps, double alpha, int S,
                 uint64_t seed, int G, int vote, uint32_t batch, int rr_mode, double beta_low, const int64_t* qindex,
                 int expect, double* out, double* min_margin, double* absum, double* sens, int32_t* digest,
                 int nthreads)
{
    kparams kp = {kernel, eps, alpha};
    if (G < 1) G = 1;
    if (vote < 1) vote = 1;
    int64_t ng = (n + vote - 1) / vote;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t gi = 0; gi < ng; ++gi) {
        int64_t j0 = gi * vote;
        int gn = (int)((n - j0 < vote) ? (n - j0) : vote);
        double* qs = malloc(3 * gn * sizeof(double));
        uint32_t* sig = malloc(gn * sizeof(uint32_t));
        cut_acc* acc = calloc(gn, sizeof(cut_acc));
        for (int g = 0; g < gn; ++g) {
            for (int a = 0; a < 3; ++a) qs[3 * g + a] = qry[3 * (j0 + g) + a];
            int64_t jj = qindex ? qindex[j0 + g] : j0 + g;
            sig[g] = (uint32_t)(jj / G);
            acc[g].mg = INFINITY;
        }
        if (!is_internal(t, 0)) {
            for (int g = 0; g < gn; ++g) {
                acc[g].F = leaf_exact(t, &kp, 0, &qs[3 * g]);
                acc[g].A = fabs(acc[g].F);
                acc[g].dig[1] = 1;
            }
        } else {
            for (int c = 0; c < t->nchild[0]; ++c)
                cut_group(t, &kp, t->first_child[0] + c, qs, sig, gn, beta_low, S, seed, batch, rr_mode, expect, acc);
        }
        for (int g = 0; g < gn; ++g) {
            out[j0 + g] = acc[g].F;
            if (min_margin) min_margin[j0 + g] = acc[g].mg;
            if (absum) absum[j0 + g] = acc[g].A;
            if (sens) sens[j0 + g] = acc[g].SN;
            if (digest)
                for (int k = 0; k < 4; ++k) digest[4 * (j0 + g) + k] = acc[g].dig[k];
        }
        free(qs); free(sig); free(acc);
    }
}

/* ------------------------------------------------------------------------ */
/* Exact expectation of the estimator (Theorem 1, Appendix A).  For a path   */
/* at node T, reached with selection probability ps and roulette product pr, */
/* the expected remaining contribution is                                    */
/*   V(T) = sum_c q_c p_c [ Delta_T / (ps pr p_c) + V(c) ],                  */
/* with V = 0 at one-point leaves and virtual points; E[F_1] = sum_a CV_a +  */
/* V(a).  Exponential in nothing: one visit per node per query.             */
/* ------------------------------------------------------------------------ */
static double expect_rec(const orc_tree* t, const kparams* kp, const double q[3], int64_t T, double tT,
                         double ps, double pr, int rr_mode, const proposal* prop)
{
    int64_t nT = t->count[T];
    if (nT == 1 && !t->cmp) return 0.0;
    double bT = dist3(node_com(t, T), q) / node_diam(t, T);
    double total = 0.0;
    if (is_internal(t, T)) {
        double sum = 0.0;
        for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch)
            sum += node_term(t, kp, ch, q);
        double delta = sum - tT;
        double qv[8];
        int slots[8], nk;
        int nonuni = proposal_q(t, prop, T, q, qv, slots, &nk);
        for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch) {
            double qc = nonuni ? qv[ch - t->first_child[T]] : (double)t->count[ch] / (double)nT;
            double pc = rr_prob(rr_mode, bT, dist3(node_com(t, ch), q) / node_diam(t, ch));
            double tc = node_term(t, kp, ch, q);
            total += qc * pc * (delta / (ps * pr * pc) + expect_rec(t, kp, q, ch, tc, ps * qc, pr * pc, rr_mode, prop));
        }
    } else {
        double sum = 0.0;
        for (int64_t s = t->begin[T]; s < t->begin[T] + nT; ++s) sum += point_term(t, kp, s, q);
        double delta = sum - tT;
        for (int64_t s = t->begin[T]; s < t->begin[T] + nT; ++s) {
            double qc = 1.0 / (double)nT;
            double pc = rr_prob(rr_mode, bT, dist3(&t->pxyz[3 * s], q) / point_diam(t, T));
            total += qc * pc * (delta / (ps * pr * pc));
        }
    }
    return total;
}

/* The exact expectation (Theorem 1) of query g's one-sample estimate under
 * the roulette voted over its tile (queries qs, gn of them). */
static double expect_vote_rec(const orc_tree* t, const kparams* kp, const double* qs, int gn, int g, int64_t T,
                              double tT, double ps, double pr)
{
    const double* q = &qs[3 * g];
    int64_t nT = t->count[T];
    if (nT == 1 && !t->cmp) return 0.0;
    double total = 0.0;
    if (is_internal(t, T)) {
        double sum = 0.0;
        for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch)
            sum += node_term(t, kp, ch, q);
        double delta = sum - tT;
        for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch) {
            double qc = (double)t->count[ch] / (double)nT;
            double pc = vote_prob(t, qs, gn, T, ch, -1);
            if (pc == 0.0) continue;
            double tc = node_term(t, kp, ch, q);
            total += qc * pc * (delta / (ps * pr * pc) + expect_vote_rec(t, kp, qs, gn, g, ch, tc, ps * qc, pr * pc));
        }
    } else {
        double sum = 0.0;
        for (int64_t s = t->begin[T]; s < t->begin[T] + nT; ++s) sum += point_term(t, kp, s, q);
        double delta = sum - tT;
        for (int64_t s = t->begin[T]; s < t->begin[T] + nT; ++s) {
            double pc = vote_prob(t, qs, gn, T, -1, s);
            if (pc == 0.0) continue;
            total += (1.0 / (double)nT) * pc * (delta / (ps * pr * pc));
        }
    }
    return total;
}

void orc_sbh_vote_expect(const orc_tree* t, const float* qry, int64_t n, int kernel, double eps, double alpha,
                         double* out, int nthreads)
{
    kparams kp = {kernel, eps, alpha};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t j = 0; j < n; ++j) {
        int64_t t0 = (j / 64) * 64, t1 = t0 + 64 < n ? t0 + 64 : n;
        int gn = (int)(t1 - t0);
        double qs[64 * 3];
        for (int k = 0; k < 3 * gn; ++k) qs[k] = qry[3 * t0 + k];
        const double* q = &qs[3 * (j - t0)];
        if (!is_internal(t, 0)) { out[j] = leaf_exact(t, &kp, 0, q); continue; }
        double F = 0.0;
        for (int ci = 0; ci < t->nchild[0]; ++ci) {
            int64_t a = t->first_child[0] + ci;
            double cv = node_term(t, &kp, a, q);
            F += cv + expect_vote_rec(t, &kp, qs, gn, (int)(j - t0), a, cv, 1.0, 1.0);
        }
        out[j] = F;
    }
}

void orc_sbh_expect(const orc_tree* t, const float* qry, int64_t n, int kernel, double eps, double alpha,
                    int rr_mode, const float* prm, int tiles, double* out, int nthreads)
{
    kparams kp = {kernel, eps, alpha};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t j = 0; j < n; ++j) {
        double q[3] = {qry[3 * j], qry[3 * j + 1], qry[3 * j + 2]};
        if (!is_internal(t, 0)) { out[j] = leaf_exact(t, &kp, 0, q); continue; }
        proposal prop = {prm, NULL, 0};
        if (tiles) {   /* tile-shared score proposal over the tiles of 64 consecutive queries */
            int64_t t0 = (j / 64) * 64, t1 = t0 + 64 < n ? t0 + 64 : n;
            prop.tile = &qry[3 * t0];
            prop.ntile = t1 - t0;
        }
        double F = 0.0;
        for (int ci = 0; ci < t->nchild[0]; ++ci) {
            int64_t a = t->first_child[0] + ci;
            double cv = node_term(t, &kp, a, q);
            F += cv + expect_rec(t, &kp, q, a, cv, 1.0, 1.0, rr_mode, &prop);
        }
        out[j] = F;
    }
}

/* ------------------------------------------------------------------------ */
/* Refine-every-node telescoping sum (Section 3.2, Eqs. (3)-(4)):            */
/*   sum_a CV_a + sum over every node T below the subdomains of Delta_T,     */
/* with leaves refined into their points.  Equals Eq. (1).                   */
/* ------------------------------------------------------------------------ */
void orc_refine_all(const orc_tree* t, const float* qry, int64_t n, int kernel, double eps, double alpha,
                    double* out)
{
    kparams kp = {kernel, eps, alpha};
    for (int64_t j = 0; j < n; ++j) {
        double q[3] = {qry[3 * j], qry[3 * j + 1], qry[3 * j + 2]};
        if (!is_internal(t, 0)) { out[j] = leaf_exact(t, &kp, 0, q); continue; }
        double F = 0.0;
        for (int ci = 0; ci < t->nchild[0]; ++ci) F += node_term(t, &kp, t->first_child[0] + ci, q);
        for (int64_t T = 1; T < t->n_nodes; ++T) {
            if (t->count[T] == 1) continue;
            double sum = 0.0;
            if (is_internal(t, T)) {
                for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch)
                    sum += node_term(t, &kp, ch, q);
            } else {
                sum = leaf_exact(t, &kp, T, q);
            }
            F += sum - node_term(t, &kp, T, q);
        }
        out[j] = F;
    }
}


/* ------------------------------------------------------------------------ */
/* Learned-proposal training support (batch entry points).                  */
/* ------------------------------------------------------------------------ */

/* Features (float64) for (internal node, query) pairs. */
void orc_mlp_features(const orc_tree* t, const int64_t* node, const float* qry, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; ++i) {
        double q[3] = {qry[3 * i], qry[3 * i + 1], qry[3 * i + 2]};
        mlp_features(t, node[i], q, &out[8 * i]);
    }
}

/* Logits for a batch of feature rows (mode 1 binary16 emulation, 0 float64). */
void orc_mlp_forward(const float* prm, const float* x, int64_t n, int mode, double* z)
{
    for (int64_t i = 0; i < n; ++i) mlp_forward(prm, &x[8 * i], mode, &z[8 * i], NULL, NULL);
}

/* Mean soft cross-entropy  L = -(1/n) sum_i sum_c t_ic log pi_ic,  pi the
 * softmax of the logits over the non-empty slots (cnt > 0), and its gradient
 * with respect to the float32 parameters (float64 back-propagation through
 * the forward of `mode`; the skip term has no parameters). */
double orc_mlp_loss_grad(const float* prm, const float* x, const float* tgt, const float* cnt, int64_t n, int mode,
                         double* grad)
{
    for (int k = 0; k < MLP_NPARAM; ++k) grad[k] = 0.0;
    double loss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double z[8], h1[32], h2[32], pi[8], c8[8], dz[8], dh2[32], dh1[32], xin[8];
        mlp_forward(prm, &x[8 * i], mode, z, h1, h2);
        for (int c = 0; c < 8; ++c) c8[c] = cnt[8 * i + c];
        masked_softmax(z, c8, pi);
        for (int c = 0; c < 8; ++c) {
            double tc = tgt[8 * i + c];
            if (c8[c] > 0) {
                if (tc > 0) loss -= tc * log(pi[c]);
                dz[c] = (pi[c] - tc) / (double)n;
            } else {
                dz[c] = 0.0;
            }
        }
        for (int k = 0; k < 8; ++k) xin[k] = mode ? f16_round(x[8 * i + k]) : (double)x[8 * i + k];
#define WV(off) (mode ? (double)f16_round(prm[off]) : (double)prm[off])
        for (int k = 0; k < 32; ++k) {
            double sacc = 0.0;
            for (int c = 0; c < 8; ++c) {
                grad[MLP_OFF_W3 + c * 32 + k] += dz[c] * h2[k];
                sacc += dz[c] * WV(MLP_OFF_W3 + c * 32 + k);
            }
            dh2[k] = h2[k] > 0 ? sacc : 0.0;
        }
        for (int c = 0; c < 8; ++c) grad[MLP_OFF_B3 + c] += dz[c];
        for (int k = 0; k < 32; ++k) {
            double sacc = 0.0;
            for (int m = 0; m < 32; ++m) {
                grad[MLP_OFF_W2 + m * 32 + k] += dh2[m] * h1[k];
                sacc += dh2[m] * WV(MLP_OFF_W2 + m * 32 + k);
            }
            dh1[k] = h1[k] > 0 ? sacc : 0.0;
        }
        for (int m = 0; m < 32; ++m) grad[MLP_OFF_B2 + m] += dh2[m];
        for (int m = 0; m < 32; ++m) {
            for (int k = 0; k < 8; ++k) grad[MLP_OFF_W1 + m * 8 + k] += dh1[m] * xin[k];
            grad[MLP_OFF_B1 + m] += dh1[m];
        }
#undef WV
    }
    return loss / (double)n;
}

/* Training targets: for internal node `node[i]` and query i, the residual of
 * every child slot, r_c = |sum_{j in c} f(p_j, q) - f_LOD(c, q)| (brute force
 * over the child's points), normalised to sum 1 (n_c / n_T when all are 0);
 * cnt receives the child point counts per slot. */
void orc_child_targets(const orc_tree* t, const int64_t* node, const float* qry, int64_t n, int kernel, double eps,
                       double alpha, float* tgt, float* cnt)
{
    kparams kp = {kernel, eps, alpha};
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double q[3] = {qry[3 * i], qry[3 * i + 1], qry[3 * i + 2]};
        int64_t T = node[i];
        double r[8] = {0, 0, 0, 0, 0, 0, 0, 0}, rs = 0.0;
        for (int c = 0; c < 8; ++c) cnt[8 * i + c] = 0.0f;
        for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch) {
            int s = t->digit[ch];
            double ex = leaf_exact(t, &kp, ch, q);
            r[s] = fabs(ex - node_term(t, &kp, ch, q));
            rs += r[s];
            cnt[8 * i + s] = (float)t->count[ch];
        }
        for (int c = 0; c < 8; ++c)
            tgt[8 * i + c] = rs > 0 ? (float)(r[c] / rs) : cnt[8 * i + c] / (float)t->count[T];
    }
}

/* Training pairs for the proposal network.  For every training query j and
 * non-empty root child (slot a) a path is walked from a with the uniform
 * path index, using the Philox stream (j, a, step/2, 0xFFFFFFFF) (the batch
 * word all ones keeps it apart from estimation streams; word 2*(step&1) of
 * the block selects), down to a leaf; every internal node on the way is one
 * (query, node) pair.  Layout [nq][d^3][lmax] with node = -1 for an unused
 * row. */
void orc_mlp_pairs(const orc_tree* t, int64_t nq, uint64_t seed, int lmax, int64_t* node_out)
{
    int d3 = t->d * t->d * t->d;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < nq * d3 * lmax; ++i) node_out[i] = -1;
    if (!is_internal(t, 0)) return;
    for (int64_t j = 0; j < nq; ++j) {
        for (int ci = 0; ci < t->nchild[0]; ++ci) {
            int64_t a = t->first_child[0] + ci;
            int slot = t->digit[a];
            int64_t T = a;
            for (int k = 0; k < lmax && is_internal(t, T); ++k) {
                int64_t row = (j * d3 + slot) * lmax + k;
                node_out[row] = T;
                uint32_t ctr[4] = {(uint32_t)j, (uint32_t)slot, (uint32_t)(k >> 1), 0xFFFFFFFFu}, rnd[4];
                orc_philox4x32_10(ctr, key, rnd);
                int64_t r = (int64_t)(((uint64_t)rnd[2 * (k & 1)] * (uint64_t)t->count[T]) >> 32);
                int64_t target = t->begin[T] + r, c = -1;
                for (int64_t ch = t->first_child[T]; ch < t->first_child[T] + t->nchild[T]; ++ch)
                    if (target >= t->begin[ch] && target < t->begin[ch] + t->count[ch]) c = ch;
                T = c;
            }
        }
    }
}
