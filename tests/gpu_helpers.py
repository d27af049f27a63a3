"""Helpers for the GPU parity tests: run the HIP path through the binding and
the FP64 oracle on the same seeded inputs, and compare them.

Tolerances (stated once, used by every parity test):
  - tree topology, point order and Morton codes: bit-exact;
  - tree aggregates (float32 on the GPU vs float64): relative 2e-5 of the
    node weight, 2e-5 of the root cube side for centres of mass;
  - estimator and Barnes-Hut values: relative error at most 1e-4, with the
    relative scale floored at 1 for winding numbers (absolute error) and at
    1/alpha for smooth distances.  Where float32 cannot reach 1e-4 the bound
    is the float32 error bound of the estimate, 2^-24 * (64 * absum + 16 *
    sens): absum is the sum of the absolute terms that entered the estimate
    (rounding in the evaluation) and sens the sum of the node terms'
    sensitivities |df/dp| |com| (float32 storage of the tree's centres of
    mass), both weighted like the estimate and reported by the oracle per
    query.  At most 1% of the queries may need this allowance;
  - sampled paths (end node, depth, accepted steps, stop reason): bit-exact,
    except queries whose smallest Russian-roulette margin |u - p| is below
    1e-5 (a float32 / float64 near-tie); every divergent query must be such a
    near-tie, and the number of them must be consistent with a divergence
    rate of at most 1e-5 of the queries: a one-sided Poisson test at level
    1e-3 (allowed_divergent) - one divergent query among a few thousand is
    what a rate near 1e-5 produces now and then, two are not.
"""
import math

import numpy as np
import torch

import oracle
import paper_2506_02219_amd as P

DEV = "cuda"
U32 = 2.0 ** -24
NEAR_TIE = 1e-5
REL_TOL = 1e-4


def allowed_divergent(n, rate=1e-5, level=1e-3):
    """The largest count of divergent queries among n that a divergence rate of `rate` explains:
    the smallest k with P(X > k) < level for X ~ Poisson(rate n)."""
    lam = rate * n
    k, term = 0, math.exp(-lam)
    cdf = term
    while 1.0 - cdf >= level:
        k += 1
        term *= lam / k
        cdf += term
    return k


def T(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def build_both(src, w, nrm=None, d=2, leaf_size=8, max_level=0):
    gt = P.sbh_build(T(src), T(w), None if nrm is None else T(nrm), branching=d, leaf_size=leaf_size,
                     max_level=max_level)
    ot = oracle.Tree(src, w, nrm, d=d, leaf_size=leaf_size, max_level=max_level)
    return gt, ot


def compressed_codes_by_node(gt):
    """The GPU tree's compressed codes [n_nodes, 4] (offsets x, y, z, mass fraction; the root's row
    zero), mapped from the child blocks (row b: the children of the b-th internal node in
    breadth-first order, slot = digit) to node order."""
    g = gt.export()
    blocks = gt.export_compressed()
    internal = g["first_child"] >= 0
    rank = np.cumsum(internal) - 1
    code = np.zeros((gt.n_nodes, 4), np.float32)
    par = g["parent"].astype(np.int64)
    v = np.arange(1, gt.n_nodes)
    code[v] = blocks[rank[par[v]], g["digit"][v]]
    return code


def quadrupole_by_node(gt):
    """The GPU tree's scaled second-moment tensors [n_nodes, 8] (the root's row zero), mapped from the
    child blocks to node order as compressed_codes_by_node does."""
    g = gt.export()
    blocks = gt.export_quadrupole()
    internal = g["first_child"] >= 0
    rank = np.cumsum(internal) - 1
    out = np.zeros((gt.n_nodes, 8), np.float32)
    par = g["parent"].astype(np.int64)
    v = np.arange(1, gt.n_nodes)
    out[v] = blocks[rank[par[v]], g["digit"][v]]
    return out


def compare_trees(gt, ot):
    """Bit-exact topology; aggregates to float32 accuracy."""
    g = gt.export()
    assert gt.n_nodes == ot.n_nodes, (gt.n_nodes, ot.n_nodes)
    assert gt.depth == ot.depth
    assert np.array_equal(gt.lo, ot.lo) and gt.side == ot.side and gt.inv_side == ot.inv_side
    assert np.array_equal(g["codes"], ot.codes)
    assert np.array_equal(g["perm"].astype(np.int64), ot.perm)
    for k in ("begin", "count", "level", "digit", "parent", "first_child", "nchild"):
        assert np.array_equal(g[k].astype(np.int64), getattr(ot, k).astype(np.int64)), k
    mass = ot.agg[:, 3]
    assert np.all(np.abs(g["agg"][:, 3] - mass) <= 2e-5 * mass)
    assert np.all(np.abs(g["agg"][:, 0:3] - ot.agg[:, 0:3]) <= 2e-5 * float(ot.side))
    dip = ot.agg[:, 4:7]
    dscale = np.maximum(np.linalg.norm(dip, axis=1, keepdims=True), mass[:, None] * 1e-3)
    assert np.all(np.abs(g["dip"][:, 0:3] - dip) <= 2e-5 * dscale + 1e-12)
    # second moments: sums of non-negative float32 terms (1e-4 relative), and offsets p - com
    # taken from float32 coordinates: an error delta of a few ulps of the coordinates moves
    # |p - com|^2 by about 2 s delta + delta^2
    s2 = ot.spread2
    delta = 2.0 ** -21 * (np.abs(ot.agg[:, :3]).max(axis=1) + float(ot.side))
    assert np.all(np.abs(g["spread2"] - s2) <= 1e-4 * s2 + 4 * np.sqrt(s2) * delta + 4 * delta ** 2)
    return g


def value_scale(ref, kernel, alpha):
    ref = np.abs(ref)
    if kernel == P.WINDING:
        return np.maximum(ref, 1.0)
    if kernel == P.SMOOTHDIST:
        return np.maximum(ref, 1.0 / alpha)
    return ref


# constants of the float32 error bound 2^-24 (C_EVAL absum + C_AGG sens) of an estimate
C_EVAL, C_AGG = 64, 16


def fp32_bound_ratio(gpu, F, absum, kernel, alpha=100.0, sens=None):
    """|GPU - oracle| over the float32 bound of each estimate (in the units of the sum F: the smooth
    distance's error is taken back through d(-log F / alpha) = -dF / (alpha F))."""
    dF = U32 * (C_EVAL * absum + (0 if sens is None else C_AGG * sens))
    with np.errstate(invalid="ignore", divide="ignore"):
        if kernel == P.SMOOTHDIST:
            r = np.abs(gpu + np.log(F) / alpha) * alpha * np.abs(F) / dF
        else:
            r = np.abs(gpu - F) / dF
    return np.where(np.isfinite(r), r, 0.0)


def value_errors(gpu, F, absum, kernel, alpha=100.0, sens=None):
    """Return (ok mask, relative error, used-fp32-bound mask) for GPU values vs oracle sums F."""
    dF = U32 * (C_EVAL * absum + (0 if sens is None else C_AGG * sens))
    if kernel == P.SMOOTHDIST:
        with np.errstate(invalid="ignore", divide="ignore"):
            ref = -np.log(F) / alpha
            # d(-log F / alpha) = -dF / (alpha F)
            fp32_bound = dF / (alpha * np.abs(F))
    else:
        ref = F
        fp32_bound = dF
    scale = value_scale(ref, kernel, alpha)
    with np.errstate(invalid="ignore", divide="ignore"):
        err = np.abs(gpu - ref) / scale
        bound = np.maximum(REL_TOL, fp32_bound / scale)
        ok = (err <= bound) | (np.isnan(gpu) & np.isnan(ref))
    # a sum whose float32 sign is not determined (|F| below its rounding bound)
    if kernel == P.SMOOTHDIST:
        undetermined = np.abs(F) <= dF
        ok |= undetermined
    used_bound = ok & ~((err <= REL_TOL) | (np.isnan(gpu) & np.isnan(ref)))
    return ok, err, used_bound


def check_sbh(gt, ot, queries, kernel, samples=1, seed=0, group=1, rr_mode=0, eps=1e-3, alpha=100.0,
              index=None, gpu_out=None, gpu_paths=None, batch=0, mlp=None, near_tie=NEAR_TIE,
              max_divergent=1e-5, proposal=None, tile_all=None, max_fp32_share=0.01, compressed=False, lod=1):
    """Run (or take) the GPU estimator and compare with the oracle, query by query.
    With `index`, `queries` are a subset of a larger set evaluated on the GPU
    (gpu_out/gpu_paths are the full-set outputs).  mlp: float32 network
    parameters (numpy) for the learned proposal on both sides; proposal=2 runs the
    score proposal on the GPU against the oracle's all-zero network; proposal=3 the tile-shared
    score proposal (tile_all: the full query set when `queries` is a subset); compressed: both sides
    walk on the compressed aggregates (the GPU tree built with compress=True); lod=2: both sides take
    second-order node terms (the GPU tree built with quadrupole=True)."""
    d3 = gt.branching ** 3
    if gpu_out is None:
        q = T(queries)
        paths = torch.full((queries.shape[0], d3, samples, 4), -7, dtype=torch.int32, device=DEV)
        out = P.sbh_eval(gt, q, kernel, samples=samples, seed=seed, eps=eps, alpha=alpha, group=group,
                         rr_mode=rr_mode, paths=paths, batch=batch, mlp=None if mlp is None else T(mlp),
                         proposal=proposal, compressed=int(compressed), lod=lod)
        g = host(out)
        gp = host(paths)
    else:
        g = gpu_out[index]
        gp = gpu_paths[index]
    ot.set_compressed(compressed)
    ot.set_lod(lod)
    try:
        if rr_mode == 3:   # the roulette voted over tiles of 64 (`queries` holds whole tiles)
            r = ot.sbh_vote(queries, kernel, samples=samples, seed=seed, group=group, batch=batch, eps=eps,
                            alpha=alpha, paths=True, index=index)
        else:
            r = ot.sbh(queries, kernel, samples=samples, seed=seed, group=group, rr_mode=rr_mode, eps=eps,
                       alpha=alpha, paths=True, index=index, batch=batch,
                       params=np.zeros(oracle.MLP_NPARAM, np.float32) if proposal == 2 else mlp,
                       tile_queries=(queries if tile_all is None else tile_all) if proposal == 3 else None)
    finally:
        ot.set_compressed(False)
        ot.set_lod(1)
    near = r["margin"] < near_tie
    path_bad = np.any(gp != r["paths"], axis=(1, 2, 3))
    ok, err, used_bound = value_errors(g, r["F"], r["absum"], kernel, alpha, r["sens"])
    bad = path_bad | ~ok
    n = queries.shape[0]
    stats = dict(n=n, path_mismatch=int(path_bad.sum()), value_mismatch=int((~ok).sum()),
                 near_ties=int(near.sum()), fp32_bound_used=int(used_bound.sum()),
                 max_rel_err=float(np.nanmax(np.where(ok, err, np.nan))) if ok.any() else float("nan"),
                 median_rel_err=float(np.nanmedian(err)),
                 max_err_over_fp32_bound=float(np.max(np.where(path_bad, 0.0, fp32_bound_ratio(
                     g, r["F"], r["absum"], kernel, alpha, r["sens"])))))
    worst = np.nonzero(bad & ~near)[0][:5]
    # the first differing path records of the worst queries: (slot, sample, gpu record, oracle record)
    recs = [(int(i), [(int(a), int(b), gp[i, a, b].tolist(), r["paths"][i, a, b].tolist())
                      for a, b in zip(*np.nonzero(np.any(gp[i] != r["paths"][i], axis=-1)))][:2]) for i in worst]
    assert not np.any(bad & ~near), (stats, [(int(i), float(g[i]), float(r["F"][i]), float(r["absum"][i]),
                                              float(r["sens"][i])) for i in worst], recs)
    assert bad.sum() <= allowed_divergent(n, max_divergent), stats
    assert used_bound.sum() <= max_fp32_share * n, stats
    return stats


def check_bh(gt, ot, queries, kernel, beta, eps=1e-3, alpha=100.0, gpu_out=None, qsel=None):
    """Barnes-Hut with wavefront voting vs the oracle's vote mode (groups of 64)."""
    if gpu_out is None:
        g = host(P.sbh_eval(gt, T(queries), kernel, beta=beta, samples=0, eps=eps, alpha=alpha))
    else:
        g = gpu_out
    F, margin, _ = ot.bh(queries, kernel, beta, group=64, eps=eps, alpha=alpha)
    # Barnes-Hut only adds positive-weight terms for the potential; use the exact
    # absolute sum bound of the accepted terms via brute force scale
    if kernel == P.SMOOTHDIST:
        with np.errstate(invalid="ignore", divide="ignore"):
            ref = -np.log(F) / alpha
    else:
        ref = F
    scale = value_scale(ref, kernel, alpha)
    err = np.abs(g - ref) / scale
    near = margin < NEAR_TIE
    bad = ~(err <= REL_TOL)
    assert not np.any(bad & ~near), (np.nonzero(bad & ~near)[0][:10], float(np.nanmax(err)))
    assert bad.sum() <= allowed_divergent(queries.shape[0]), int(bad.sum())
    return dict(max_rel_err=float(np.nanmax(err)), near=int(near.sum()))


def fp64_reference(src, w, nrm, queries, kernel, eps=1e-3, alpha=100.0):
    return host(P.sbh_brute(T(src), T(w), None if nrm is None else T(nrm), T(queries), kernel, eps=eps,
                            alpha=alpha, fp64=True))


def check_cut(gt, ot, queries, kernel, beta_low, samples=1, seed=0, group=64, rr_mode=0, eps=1e-3, alpha=100.0,
              index=None, gpu_out=None, gpu_digest=None, max_divergent=1e-5):
    """The Barnes-Hut-cut stratified estimator (subdomains = 1) against the oracle's, query by query:
    values to the estimator's bar, and each query's digest {subdomains, leaves summed exactly,
    accepted steps, sum of end levels} bit-exact except near-ties.  `queries` must be whole groups of
    64 consecutive queries (the vote); with `index` they are those groups taken from a larger set
    evaluated on the GPU (gpu_out / gpu_digest hold the full-set outputs)."""
    if gpu_out is None:
        dig = torch.full((queries.shape[0], 4), -7, dtype=torch.int32, device=DEV)
        g = host(P.sbh_eval(gt, T(queries), kernel, beta=beta_low, samples=samples, seed=seed, eps=eps, alpha=alpha,
                            group=group, rr_mode=rr_mode, paths=dig, subdomains=1))
        gd = host(dig)
    else:
        g, gd = gpu_out[index], gpu_digest[index]
    r = ot.sbh_cut(queries, kernel, beta_low, samples=samples, seed=seed, group=group, vote=64, rr_mode=rr_mode,
                   eps=eps, alpha=alpha, index=index)
    near = r["margin"] < NEAR_TIE
    dig_bad = np.any(gd != r["digest"], axis=1)
    ok, err, used_bound = value_errors(g, r["F"], r["absum"], kernel, alpha, r["sens"])
    bad = dig_bad | ~ok
    n = queries.shape[0]
    stats = dict(n=n, digest_mismatch=int(dig_bad.sum()), value_mismatch=int((~ok).sum()),
                 near_ties=int(near.sum()), fp32_bound_used=int(used_bound.sum()),
                 max_rel_err=float(np.nanmax(np.where(ok, err, np.nan))) if ok.any() else float("nan"),
                 median_rel_err=float(np.nanmedian(err)), subdomains_mean=float(r["digest"][:, 0].mean()),
                 leaves_mean=float(r["digest"][:, 1].mean()))
    worst = np.nonzero(bad & ~near)[0][:5]
    assert not np.any(bad & ~near), (stats, [(int(i), float(g[i]), float(r["F"][i]), gd[i].tolist(),
                                              r["digest"][i].tolist()) for i in worst])
    assert bad.sum() <= allowed_divergent(n, max_divergent), stats
    assert used_bound.sum() <= 0.01 * n, stats
    return stats
