/*
 * sbh.h - C ABI of the stochastic Barnes-Hut library for AMD Instinct MI355X
 * (gfx950).  Madan, Sharp, Williams, Museth, Levin, "Stochastic Barnes-Hut
 * Approximation for Fast Summation on the GPU" (SIGGRAPH 2025).
 *
 * Problem (Section 3, Eq. (1)): given sources p_i with weights m_i and query
 * points q_j, evaluate F(q_j) = sum_i m_i f(p_i, q_j) for every query.
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless marked (host).  Arrays are dense,
 *     row-major, float32 unless stated: points are [n][3] (x, y, z).
 *   - Every call enqueues its work on `stream` (0 = the null stream) and
 *     returns without waiting for it, except where a call says it
 *     synchronises.  Build and export synchronise `stream`.
 *   - Arguments are checked on the host before anything is enqueued; on an
 *     error nothing is written to any output and a negative status is
 *     returned.  sbh_last_error() then holds a message for this thread.
 *   - The library never frees memory it did not allocate.  Output buffers
 *     are owned by the caller and overwritten.
 *   - Results are a deterministic function of the inputs and the documented
 *     arguments only (never of launch geometry).
 */
#ifndef SBH_H
#define SBH_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sbh_status {
    SBH_OK = 0,
    SBH_EINVAL = -1,        /* invalid argument (null pointer, bad size, NaN input, bad enum) */
    SBH_ENOMEM = -2,        /* device allocation failed */
    SBH_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    SBH_EUNSUPPORTED = -4,  /* valid request that the library does not implement */
    SBH_ESTATE = -5         /* object in an unusable state */
} sbh_status;

/* Kernels f(p, q) (results section: potential, winding numbers, smooth
 * distances).  For one source p with weight w (and unit normal n):
 *   SBH_POTENTIAL   w / sqrt(|p-q|^2 + eps^2)                 (softened 1/r)
 *   SBH_WINDING     w n.(p-q) / (4 pi |p-q|^3), 0 at p = q     (dipole)
 *   SBH_SMOOTHDIST  w exp(-alpha |p-q|); the reported value is the smooth
 *                   distance -log(F)/alpha of the (estimated) sum F.
 * A tree node uses its aggregate in place of one source: total weight and
 * weighted centre of mass; the winding kernel uses the summed w n. */
typedef enum sbh_kernel {
    SBH_POTENTIAL = 0,
    SBH_WINDING = 1,
    SBH_SMOOTHDIST = 2
} sbh_kernel;

/* Child-selection distributions of the estimator (sbh_eval_opts.proposal). */
typedef enum sbh_proposal {
    SBH_PROPOSAL_UNIFORM = 0,     /* the uniform path index (Section 3.3) */
    SBH_PROPOSAL_LEARNED = 1,     /* the learned proposal (network parameters in opts->mlp) */
    SBH_PROPOSAL_SCORE = 2,       /* per-query quadrupole-score proposal (the learned one with a zero network) */
    SBH_PROPOSAL_TILE_SCORE = 3   /* the score proposal averaged over tiles of 64 consecutive queries */
} sbh_proposal;

typedef struct sbh_build_opts {
    int32_t branching;   /* per-dimension branching d: 2 (octree), 4 (64-way) or 8 (512-way); default 2 */
    int32_t leaf_size;   /* a node is split iff it holds more points than this; 1..64, default 8 */
    int32_t max_level;   /* deepest level; 0 = 60/(3 log2 d): 20 for d=2, 10 for d=4, 6 for d=8 */
    int32_t compress;    /* 1: also store the compressed interior aggregates (the conclusion's
                            quantised node buffer; branching 2): for each child c of an internal
                            node P, binary16 o_c = (com_c - com^q_P) / s_c per axis (s_c the
                            side of c's cell) and f_c = m_c / m^q_P, where com^q, m^q are the
                            decoded values com^q_c = com^q_P + o_c s_c, m^q_c = m^q_P f_c
                            (float64; the root's are its float32 centre of mass and mass; the
                            exact aggregates summed in float64, a leaf over its points in order,
                            an internal node over its children in slot order); 8 bytes per
                            child instead of 16.  Default 0. */
    int32_t quadrupole;  /* 1: also store each child's second-moment tensor about its centre of
                            mass, Q = sum w (p - com)(p - com)^T (float64 sums, rounded once),
                            for second-order node terms (sbh_eval_opts.lod = 2; Section 3.1's
                            higher-order approximations); 32 bytes per child.  Default 0. */
} sbh_build_opts;

typedef struct sbh_eval_opts {
    float eps;           /* potential softening, >= 0; default 1e-3 */
    float alpha;         /* smooth-distance sharpness, > 0; default 100 */
    int32_t group;       /* G >= 1: queries j with equal floor(j/G) share one random
                            stream (G = 1: every query has its own); default 1 */
    int32_t rr_mode;     /* Russian roulette: 0 = Eq. (5) (default), 1 = p = 1 (none),
                            2 = p = 1/2 (the two comparisons of the supplement), 3 = Eq. (5)
                            voted over each tile of 64 consecutive queries: every query of
                            the tile continues with the largest Eq. (5) p among the tile's
                            queries with finite coordinates (still unbiased, Theorem 1); needs
                            group a multiple of 64, the uniform proposal and subdomains 0 */
    int32_t proposal;    /* child-selection distribution: 0 = uniform path index
                            (the paper's, default); 1 = the learned proposal with
                            network parameters opts->mlp; 2 = the score proposal
                            (the learned one with an all-zero network, evaluated
                            without it); 3 = the tile-shared score proposal
                            (group a multiple of 64).  1, 2 and 3: branching 2 only. */
    uint32_t batch;      /* fourth Philox counter word, for independent batches; default 0 */
    int32_t* paths;      /* optional DEVICE [nq][d^3][samples][4] int32 records of every
                            sampled path: {end begin, end level, accepted steps, stop
                            reason (0 roulette, 1 one-point node, 2 virtual point)};
                            subdomain slots that are empty hold begin = -1.  NULL = off. */
    const float* mlp;    /* DEVICE [SBH_MLP_NPARAM] network parameters for proposal 1; default NULL.
                            Parameters that are not all finite are ignored: the kernel then
                            uses the score proposal (the zero network). */
    int32_t subdomains;  /* path roots (Section 3.3.1): 0 = the root's children (default);
                            1 = the Barnes-Hut cut D(q, beta) with beta = sbh_eval's beta:
                            walking from the root, a node that every query of the wavefront
                            (64 consecutive queries) sees as far (|q - com| / |B| >= beta) is
                            a subdomain; a node that is not far is opened, a leaf summed
                            exactly.  1 needs group a multiple of 64, the uniform proposal and
                            branching 2 or 4; paths, if given, is then [nq][4] int32: {subdomains,
                            leaves summed exactly, accepted steps of all paths, sum of their
                            end levels}. */
    int32_t compressed;  /* 1: walk on the tree's compressed interior aggregates (built with
                            sbh_build_opts.compress = 1; the conclusion's compressed LOD
                            representation): each node's centre of mass and mass are the
                            binary16-coded values decoded down from the root, and a node of one
                            point takes the leaf step.  Needs the uniform proposal, subdomains
                            0, the potential or smooth-distance kernel, and samples <= 32 when
                            group is not a multiple of 64.  Default 0. */
    int32_t lod;         /* order of the node terms: 1 (or 0, the default) the point mass
                            m f(com, q) of Section 3.1; 2 adds, for the potential, the next term
                            of the Taylor expansion about the centre of mass wherever the query
                            sees the node as far (|q - com| >= |B|):
                            1/2 u^5 (3 x^T Q x - tr(Q) (|x|^2 + eps^2)), x = com - q,
                            u = (|x|^2 + eps^2)^(-1/2).  2 needs a tree built with quadrupole =
                            1, branching 2, the potential, samples >= 1, group a multiple of 64,
                            the uniform proposal, subdomains 0 and compressed 0.  The estimator
                            stays unbiased (Theorem 1 holds for any node terms). */
} sbh_eval_opts;

typedef struct sbh_tree sbh_tree;   /* opaque; immutable after sbh_build */

typedef struct sbh_tree_desc {      /* host copy of a tree's sizes */
    int64_t n_points, n_nodes, n_blocks;
    int32_t depth, branching, leaf_size, max_level, has_normals;
    float lo[3], side, inv_side;    /* root cube [lo, lo + side]^3 and fl32(1/side) */
} sbh_tree_desc;

/* Learned proposal network: 8 features -> 32 -> 32 -> 8 logits with ReLU.
 * Parameters are float32 [SBH_MLP_NPARAM] = W1[32][8] b1[32] W2[32][32] b2[32]
 * W3[8][32] b3[8] (row-major, out x in); the kernels evaluate it with binary16
 * weights, inputs and hidden activations and float32 accumulation (MFMA).
 * Gradient buffers hold SBH_MLP_GRAD_SIZE floats: the gradient, then the
 * mean loss, then the number of rows that entered the mean. */
#define SBH_MLP_NPARAM 1608
#define SBH_MLP_GRAD_SIZE 1610

/*
 * Device memory.  Every device allocation of the library goes through one
 * allocator pair: a tree's arrays and the temporaries of its build, the
 * proposal network's workspaces and a batch plan's tables.
 *   alloc(bytes, stream, ctx) returns device memory of at least `bytes`
 *     bytes, 256-byte aligned, usable by work enqueued on `stream` from the
 *     moment of the call on (stream order), or NULL when it cannot; the
 *     library then releases what the failed call had taken, enqueues nothing
 *     more and returns SBH_ENOMEM.
 *   free(ptr, bytes, stream, ctx) returns an allocation; work that reads it
 *     has been enqueued on `stream` before the call (or has completed when
 *     `stream` is 0 and the library has waited for the device first).
 * The default (both NULL) is hipMallocAsync / hipFreeAsync on the call's
 * stream.  A PyTorch caller can pass its caching allocator here.
 */
typedef void* (*sbh_alloc_fn)(size_t bytes, hipStream_t stream, void* ctx);
typedef void (*sbh_free_fn)(void* ptr, size_t bytes, hipStream_t stream, void* ctx);

/*
 * sbh_set_allocator - set the allocator of later allocations (process-wide).
 * Objects keep the allocator they were created with and release through it,
 * so a change does not affect trees or plans that exist.  Both NULL restores
 * the default.  Call it while no other thread is inside the library.
 * Errors: SBH_EINVAL (exactly one of alloc and free NULL).
 */
sbh_status sbh_set_allocator(sbh_alloc_fn alloc, sbh_free_fn free, void* ctx);

/* Fill option structs with the defaults documented above. */
void sbh_build_opts_default(sbh_build_opts* opts /*host*/);
void sbh_eval_opts_default(sbh_eval_opts* opts /*host*/);

/*
 * sbh_build - the spatial tree of Section 3.1 (octree-like, per-dimension
 * branching d) with per-node aggregate weight, centre of mass and summed
 * dipole, built on the GPU; each node also keeps the second moment of its
 * points about the centre of mass (for the learned proposal's features).
 *   sources  [n][3]   source positions p_i (finite)
 *   weights  [n]      source weights m_i (finite, > 0)
 *   normals  [n][3]   unit normals (needed for SBH_WINDING) or NULL
 *   n        1 <= n <= 2^30
 *   opts     (host) or NULL for defaults
 *   out_tree (host) receives the tree; the caller releases it with sbh_free.
 * The tree copies what it needs; the inputs may be freed when the call
 * returns.  Synchronises `stream`.  Errors: SBH_EINVAL (null pointer, n out
 * of range, bad option, non-finite coordinate or normal, weight <= 0),
 * SBH_ENOMEM, SBH_EHIP.
 */
sbh_status sbh_build(const float* sources, const float* weights, const float* normals, int64_t n,
                     const sbh_build_opts* opts, hipStream_t stream, sbh_tree** out_tree);

/*
 * sbh_eval - evaluate every query on a tree.
 *   samples >= 1: the stratified path-sample estimator (Section 3.3, Eqs.
 *     (5)-(7), Algorithm 2) with S = samples paths per subdomain; the
 *     subdomains are the root's children (Section 3.3.1).  Random numbers:
 *     Philox4x32-10 with key = seed and counter = (stream id, slot*S + s,
 *     step/2, opts->batch), stream id = j (G = 1) or floor(j/G).  beta is
 *     ignored.  Unbiased for F (Theorem 1) for the potential and winding
 *     kernels.
 *   samples == 0: Barnes-Hut (Eq. (2), Algorithm 1) with opening parameter
 *     beta > 0 (INFINITY = exact): a node is accepted iff |q - com| / |B| >=
 *     beta, where |B| is the diagonal of the node's cell; a leaf that is not
 *     accepted is summed exactly.  Queries are voted on in groups of 64
 *     consecutive indices: a node is opened for the whole group if any of
 *     its queries needs it.
 *   queries [nq][3]; out [nq] float32 (smooth distance for SBH_SMOOTHDIST).
 *   nq = 0 is a no-op.  Errors: SBH_EINVAL (null pointers, nq < 0, bad
 *   kernel, samples < 0, beta <= 0 or NaN with samples == 0, group < 1,
 *   eps < 0, alpha <= 0, SBH_WINDING on a tree without normals, proposal
 *   not 0..3, proposal 1 without opts->mlp, proposal 3 with a group that is
 *   not a multiple of 64), SBH_EUNSUPPORTED (proposals 1-3 on a tree with
 *   branching 4 or 8; on a tree with branching 8, Barnes-Hut and groups
 *   that are not a multiple of 64), SBH_EHIP.
 *
 *   Learned and score proposals (opts->proposal = 1, 2).  Section 3.3 draws
 *   the path index uniformly and leaves importance sampling open; Theorem 1
 *   needs only that every point can be reached, so any child distribution
 *   q_c > 0 over the non-empty children keeps the estimator unbiased when
 *   the swap of each step is divided by the product of the q's chosen so far
 *   (in place of n_T / n_a, Eq. (7)).  At an internal node T each child c
 *   has the quadrupole score m_c s_c^2 / (|p_c - q|^2 + s_c^2)^(3/2) (weight,
 *   centre of mass, second moment) -- a bound on the size of c's residual
 *   under the 1/r kernel -- and the feature f_c = max(-1, ln(score_c / max
 *   score) / 16) (-1 for empty slots).  The network (proposal 1) maps f to
 *   logits z = NN(f) + 16 f; proposal 2 uses z = 16 f.  Then
 *     q_c = (7/8) exp(z_c) / sum_c' exp(z_c') + (1/8) n_c / n_T
 *   over the non-empty slots; the child is the first non-empty slot whose
 *   running sum of q exceeds u = (x >> 8) 2^-24 of the selection word x (the
 *   last non-empty slot if rounding leaves the total below u).  Leaves choose
 *   a point uniformly.
 *
 *   Tile-shared score proposal (opts->proposal = 3).  Queries are taken in
 *   tiles of 64 consecutive indices (the wavefronts of the shared-stream
 *   walk); at each internal node every query of a tile uses the same
 *     q_c = (7/8) mean over the tile's queries of pi_c(q) + (1/8) n_c / n_T,
 *   pi_c(q) = max(score_c(q) / max score(q), e^-16) normalised over the
 *   non-empty slots (proposal 2's softmax), so that the tile keeps one
 *   shared path; q depends only on the node and the tile's queries, and the
 *   estimator stays unbiased for every query.  It pays when a tile's queries
 *   are close to one another (e.g. a grid in its own order).
 *
 *   The shared-stream walk and Barnes-Hut address a tree with 32-bit byte
 *   offsets while each of its arrays is below 4 GiB, with 64-bit ones beyond
 *   (the values are the same).  Setting the environment variable
 *   SBH_FORCE_WIDE_OFFSETS=1 takes the 64-bit form for every tree; it is
 *   read when sbh_eval runs and when a batch plan is created.
 */
sbh_status sbh_eval(const sbh_tree* tree, const float* queries, int64_t nq, sbh_kernel kernel,
                    float beta, int32_t samples, uint64_t seed, const sbh_eval_opts* opts,
                    hipStream_t stream, float* out);

/*
 * sbh_brute - Eq. (1) evaluated exactly by tiling the sources through LDS.
 *   fp64 = 0: float32 arithmetic, out is float[nq];
 *   fp64 = 1: float64 arithmetic, out is double[nq] (the reference values).
 * Kernels, eps and alpha as for sbh_eval (opts may be NULL).  Sources are in
 * the caller's order; no tree is needed.  Errors: SBH_EINVAL, SBH_EHIP.
 */
sbh_status sbh_brute(const float* sources, const float* weights, const float* normals, int64_t n,
                     const float* queries, int64_t nq, sbh_kernel kernel, const sbh_eval_opts* opts,
                     int32_t fp64, hipStream_t stream, void* out);

/*
 * sbh_mlp_forward - logits of the proposal network.
 *   params [SBH_MLP_NPARAM], features [n][8], logits [n][8] (float32).
 *   n = 0 is a no-op.  Errors: SBH_EINVAL (NULL argument, n < 0 or >= 2^31),
 *   SBH_EHIP.
 */
sbh_status sbh_mlp_forward(const float* params, const float* features, int64_t n, hipStream_t stream,
                           float* logits);

/*
 * sbh_mlp_pairs - training rows for the proposal.  For query j and subdomain
 * slot a (the root's children, Section 3.3.1) a path is walked from a with
 * the uniform path index, drawing from Philox4x32-10 with key = seed and
 * counter = (j, a, step/2, 0xFFFFFFFF) (word 2 (step & 1) selects); every
 * internal node T on it down to depth max_depth is one row
 * r = (j * 8 + a) * max_depth + step:
 *   features [rows][8]  the network inputs of (T, q_j): per child slot the
 *                       relative log quadrupole score (see sbh_eval)
 *   targets  [rows][8]  per child slot c: |sum over c's points of f - f of c's
 *                       aggregate| (float64), normalised to sum 1 (n_c / n_T
 *                       when every residual is 0): the share of T's refinement
 *                       error that c carries (Eqs. (3)-(4))
 *   counts   [rows][8]  n_c per slot (0 = empty slot)
 *   where    [rows][4]  int32 {children block, first point, n_T, level} of T
 * Rows past the end of a path are all zero with where = {-1, 0, 0, 0}.
 * rows = nq * 8 * max_depth; 1 <= max_depth <= the tree's max_level.
 * Kernels and eps / alpha (opts, may be NULL) as for sbh_eval.  Errors:
 * SBH_EINVAL, SBH_EUNSUPPORTED (branching 4), SBH_EHIP.
 */
sbh_status sbh_mlp_pairs(const sbh_tree* tree, const float* queries, int64_t nq, sbh_kernel kernel, uint64_t seed,
                         int32_t max_depth, const sbh_eval_opts* opts, hipStream_t stream, float* features,
                         float* targets, float* counts, int32_t* where);

/*
 * sbh_mlp_loss_grad - mean over the rows with some non-zero count of the soft
 * cross-entropy -sum_c t_c log pi_c, pi_c = n_c exp(z_c) / sum n_c' exp(z_c'),
 * and its gradient with respect to params (back-propagation through the
 * binary16 forward; deltas in binary16, sums in float32).
 *   features, targets, counts [n][8] as written by sbh_mlp_pairs;
 *   grad [SBH_MLP_GRAD_SIZE].  Allocates a stream-ordered workspace of
 *   about 6.3 KiB per 64 rows.  Errors: SBH_EINVAL (NULL argument, n < 1
 *   or >= 2^31), SBH_ENOMEM, SBH_EHIP.
 */
sbh_status sbh_mlp_loss_grad(const float* params, const float* features, const float* targets, const float* counts,
                             int64_t n, hipStream_t stream, float* grad);

/*
 * sbh_mlp_train - `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8,
 * learning rate lr) on params in place.  Step s (counted from step0, which
 * sets the bias correction, so that training can be continued) uses the
 * rows [b (step0 + s) mod n, ...) up to b = min(batch_rows, n) rows or the
 * end of the set; shuffle the rows beforehand.  adam_state [2][1608]
 * (first and second moments, zero before the first step); losses [steps]
 * (optional) receives each step's mean loss.  Allocates a stream-ordered
 * workspace like sbh_mlp_loss_grad.  Errors: SBH_EINVAL (NULL argument, n
 * out of range, steps or step0 < 0, batch_rows outside [1, 2^24], lr not
 * finite and > 0), SBH_ENOMEM, SBH_EHIP.
 */
sbh_status sbh_mlp_train(float* params, float* adam_state, const float* features, const float* targets,
                         const float* counts, int64_t n, int32_t steps, int32_t batch_rows, float lr, int32_t step0,
                         hipStream_t stream, float* losses);

/*
 * sbh_mlp_train_noalloc - sbh_mlp_train without any device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * or training loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results (bit for bit) as sbh_mlp_train.  The workspace is a
 * static array in device memory of (SBH_NOALLOC_MAX_BATCH_ROWS / 64 + 1)
 * * 1616 floats (about 3.2 MiB), one copy per GPU, held until the process
 * ends; its address is looked up on the first call on each device.  The
 * workspace holds no state between calls (every word a call reads it has
 * written first), but it is shared: calls that overlap in time on one GPU
 * (on different streams, or from different threads) race and give wrong
 * results.  Errors: as sbh_mlp_train, and SBH_EINVAL for batch_rows above
 * SBH_NOALLOC_MAX_BATCH_ROWS; never SBH_ENOMEM.
 */
#define SBH_NOALLOC_MAX_BATCH_ROWS 32768
sbh_status sbh_mlp_train_noalloc(float* params, float* adam_state, const float* features, const float* targets,
                                 const float* counts, int64_t n, int32_t steps, int32_t batch_rows, float lr,
                                 int32_t step0, hipStream_t stream, float* losses);

/* ------------------------------------------------------------------------
 * Batched evaluation: many trees and query sets (of uneven sizes) evaluated
 * by one launch per (branching factor, kernel) group present, replayed from
 * a HIP graph.  A work item is one workgroup that evaluates tile_waves tiles
 * (64 consecutive queries each) of the same cloud; the hardware
 * dispatcher starts workgroups as earlier ones finish, so clouds of uneven
 * cost balance without a shared work counter.  Each tile runs the same code
 * as sbh_eval with samples >= 1 and opts->group a multiple of 64, so every
 * cloud's output is bit-identical to its own sbh_eval call with the same
 * seed, batch word and options.
 * ------------------------------------------------------------------------ */
typedef struct sbh_batch sbh_batch;   /* opaque plan */

typedef struct sbh_batch_item {
    const sbh_tree* tree;
    const float* queries;   /* DEVICE [nq][3] */
    float* out;             /* DEVICE [nq] */
    int64_t nq;             /* 0 <= nq < 2^31 */
    int32_t kernel;         /* sbh_kernel */
    int32_t reserved;       /* 0 */
} sbh_batch_item;

typedef struct sbh_batch_config {
    int32_t tile_waves;      /* 64-query tiles per workgroup: 1 or 2 */
    int32_t waves_per_simd;  /* 1..8: resident wavefronts per SIMD to aim for (8 = the hardware's own
                                limit; below it, LDS is reserved per workgroup to cap residency, as far
                                as the per-workgroup LDS limit allows) */
    int32_t heavy_first;     /* 1: workgroups of the costliest clouds (queries x depth) first */
    float ms;                /* autotuned plans: measured time of one batch; else 0 */
} sbh_batch_config;

/*
 * sbh_batch_create - validate the items, copy their descriptors to the
 * device and capture the launch sequence in a HIP graph.
 *   items (host) [count], 1 <= count <= 2^20; samples >= 1; opts as for
 *   sbh_eval with group a multiple of 64, proposal 0 and no path records
 *   (NULL: the defaults with group 64).
 *   config (host): the launch configuration, or NULL to autotune: every
 *   candidate (tile_waves 1, 2; waves_per_simd 4, 8; heavy_first 0, 1)
 *   is timed on the batch itself (seed 0) and the fastest kept; this writes
 *   the outputs and synchronises `stream`.
 * The plan keeps pointers to the trees, queries and outputs, which must
 * stay valid (and the trees alive) until sbh_batch_free.  It allocates
 * 6 x 16 bytes of launch state, the descriptors and the workgroup tables
 * (8 bytes per tile) on the current device, and owns four streams (default
 * priority) and four events: the graph's launch groups (one per branching
 * factor and kernel, and the exact sums of root-leaf clouds) are forked
 * from its first node onto three of them and joined back, so that they
 * run as parallel branches.
 * Errors: SBH_EINVAL, SBH_EUNSUPPORTED (proposal != 0), SBH_ENOMEM, SBH_EHIP.
 */
sbh_status sbh_batch_create(const sbh_batch_item* items, int32_t count, int32_t samples, const sbh_eval_opts* opts,
                            const sbh_batch_config* config, hipStream_t stream, sbh_batch** out);

/*
 * sbh_batch_launch - evaluate every item with Philox key `seed` and fourth
 * counter word `batch` (as opts->batch of sbh_eval): sets the key in the
 * graph's first node and replays the graph on `stream`.  Allocates nothing.
 * Launches of one plan that overlap (several streams) race on its launch
 * state.  Errors: SBH_EINVAL (NULL plan), SBH_EHIP.
 */
sbh_status sbh_batch_launch(sbh_batch* batch_plan, uint64_t seed, uint32_t batch, hipStream_t stream);

/* sbh_batch_get_config - the plan's launch configuration into *cfg (host). */
sbh_status sbh_batch_get_config(const sbh_batch* batch_plan, sbh_batch_config* cfg);

/* sbh_batch_free - release a plan (waits for the device). NULL is a no-op. */
sbh_status sbh_batch_free(sbh_batch* batch_plan);

/* sbh_tree_info - sizes and root cube of a tree into *info (host). */
sbh_status sbh_tree_info(const sbh_tree* tree, sbh_tree_desc* info);

/*
 * sbh_tree_export - copy the tree to host arrays (for verification).  Every
 * pointer is (host) and may be NULL to skip that array.  Node arrays have
 * n_nodes entries in breadth-first order (Morton order within a level):
 *   begin, count      range of the node in sorted point order
 *   level, digit      depth (root 0) and child digit within the parent
 *   parent            parent node id (-1 for the root)
 *   first_child, nchild  children are ids first_child .. first_child+nchild-1
 *                     (first_child = -1 for a leaf)
 *   agg  [n_nodes][4] centre of mass (x, y, z) and total weight
 *   dip  [n_nodes][4] summed w n (x, y, z), 0
 *   spread2 [n_nodes] second moment sum w |p - com|^2 / total weight
 * Point arrays have n_points entries: perm (sorted position -> input index)
 * and codes (the 60-bit Morton codes, sorted).  Synchronises the null stream.
 */
sbh_status sbh_tree_export(const sbh_tree* tree, int32_t* begin, int32_t* count, int32_t* level,
                           int32_t* digit, int32_t* parent, int32_t* first_child, int32_t* nchild,
                           float* agg, float* dip, uint32_t* perm, uint64_t* codes, float* spread2);

/*
 * sbh_tree_export_compressed - copy a tree's compressed aggregates (built with
 * opts->compress = 1) to the host: codes [n_blocks][d^3][2] uint32, the child
 * block of the b-th internal node (breadth-first order) in row b, slot s the
 * child with digit s: {offset x | offset y << 16, offset z | mass fraction
 * << 16}, binary16 bit patterns (zero for empty slots).  Synchronises the null
 * stream.  Errors: SBH_EINVAL (NULL), SBH_ESTATE (no compressed aggregates),
 * SBH_EHIP.
 */
sbh_status sbh_tree_export_compressed(const sbh_tree* tree, uint32_t* codes);

/*
 * sbh_tree_export_quadrupole - copy a tree's scaled second-moment tensors
 * (built with opts->quadrupole = 1) to the host: quad [n_blocks][d^3][8]
 * float, laid out as the child blocks of sbh_tree_export_compressed: {1.5
 * Qxx, 1.5 Qyy, 1.5 Qzz, 3 Qxy, 3 Qxz, 3 Qyz, tr(Q) / 2, 0} of the child in
 * each slot (zero for empty slots).  Synchronises the null stream.  Errors:
 * SBH_EINVAL (NULL), SBH_ESTATE (no tensors), SBH_EHIP.
 */
sbh_status sbh_tree_export_quadrupole(const sbh_tree* tree, float* quad);

/* sbh_free - release a tree (waits for the device to finish using it). NULL is a no-op. */
sbh_status sbh_free(sbh_tree* tree);

/*
 * sbh_free_async - release a tree in stream order, without waiting: its
 * memory is handed back to its allocator on `stream`.  Every use of the tree
 * must have been enqueued on `stream`, or ordered before it by the caller
 * (events), before this call.  NULL is a no-op.
 */
sbh_status sbh_free_async(sbh_tree* tree, hipStream_t stream);

/* Static text for a status code. */
const char* sbh_status_string(sbh_status status);

/* Message of the last failed call on this thread ("" if none). */
const char* sbh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SBH_H */
