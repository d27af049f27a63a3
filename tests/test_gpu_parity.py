"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Small cases span several tiles and ragged tails; the full-size workloads are
checked on sampled queries in the launch configuration the benchmark times.
Tolerances are stated in gpu_helpers.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_2506_02219_amd as P
from gpu_helpers import (check_cut, DEV, T, host, build_both, compare_trees, check_sbh, check_bh, fp64_reference,
                         value_scale)

pytestmark = pytest.mark.gpu


def surface(m, seed=21, level=4):
    pts, nrm, w, _ = W.star_surface(m, seed, level=level)
    return pts.astype(np.float32), nrm.astype(np.float32), w.astype(np.float32)


def box_queries(n, seed, lo=-1.5, hi=1.5):
    return np.random.Generator(np.random.PCG64(seed)).uniform(lo, hi, (n, 3)).astype(np.float32)


# ----------------------------------------------------------------------------- brute force
@pytest.mark.parametrize("kernel", [P.POTENTIAL, P.WINDING, P.SMOOTHDIST])
def test_brute_matches_oracle(kernel):
    src, nrm, w = surface(3001)
    q = box_queries(1000, 3)
    F = oracle.brute(src, w, nrm, q, kernel)
    ref = oracle.smooth_distance(F) if kernel == P.SMOOTHDIST else F
    g64 = fp64_reference(src, w, nrm, q, kernel)
    assert np.all(np.abs(g64 - ref) <= 1e-11 * value_scale(ref, kernel, 100.0))
    g32 = host(P.sbh_brute(T(src), T(w), T(nrm), T(q), kernel))
    assert np.all(np.abs(g32 - ref) <= 1e-4 * value_scale(ref, kernel, 100.0))


# ----------------------------------------------------------------------------- tree
@pytest.mark.parametrize("d", [2, 4, 8])
def test_tree_bit_exact_c1(d):
    c = W.c1()
    gt, ot = build_both(c.sources, c.weights, d=d)
    compare_trees(gt, ot)


@pytest.mark.parametrize("d,leaf", [(2, 8), (4, 8), (2, 1), (8, 8)])
def test_tree_bit_exact_surface(d, leaf):
    src, nrm, w = surface(50000, 5)
    gt, ot = build_both(src, w, nrm, d=d, leaf_size=leaf)
    compare_trees(gt, ot)


def test_tree_duplicates_and_max_level():
    src = np.array([[0.3, 0.3, 0.3]] * 40 + [[0, 0, 0], [1, 1, 1]] + [[0.7, 0.2, 0.9]] * 3, np.float32)
    w = np.linspace(0.5, 1.5, len(src)).astype(np.float32)
    for d, ml in ((2, 0), (2, 5), (4, 3), (8, 0), (8, 2)):
        gt, ot = build_both(src, w, d=d, leaf_size=4, max_level=ml)
        compare_trees(gt, ot)


@pytest.mark.parametrize("m", [1, 2, 5, 8, 9, 4097])
def test_tree_small_and_ragged(m):
    c = W.uniform_cube(m, 1, 77)
    gt, ot = build_both(c.sources, c.weights)
    compare_trees(gt, ot)


# ----------------------------------------------------------------------------- stochastic estimator
@pytest.mark.parametrize("d,S,G,rr", [(2, 1, 1, 0), (2, 4, 1, 0), (4, 1, 1, 0), (4, 2, 1, 0),
                                      (2, 2, 1, 1), (2, 2, 1, 2), (2, 1, 8, 0),
                                      # d^3 S above the per-wavefront path pool: one path per lane, no refill
                                      (4, 8, 1, 0), (2, 40, 1, 0),
                                      # the pool at its limit (one query per wavefront); a group that is
                                      # not a multiple of 64
                                      (2, 32, 1, 0), (2, 1, 100, 0),
                                      # G a multiple of 64: one shared stream per wavefront (coherent kernel)
                                      (2, 1, 64, 0), (2, 3, 128, 0), (4, 1, 64, 0), (2, 2, 64, 2)])
def test_sbh_parity_c1(d, S, G, rr):
    c = W.c1()
    gt, ot = build_both(c.sources, c.weights, d=d)
    st = check_sbh(gt, ot, c.queries, P.POTENTIAL, samples=S, seed=0, group=G, rr_mode=rr)
    print(st)


@pytest.mark.parametrize("kernel", [P.WINDING, P.SMOOTHDIST, P.POTENTIAL])
@pytest.mark.parametrize("d", [2, 4])
@pytest.mark.parametrize("G", [1, 64])
def test_sbh_parity_surface_kernels(kernel, d, G):
    src, nrm, w = surface(30000, 9)
    q = box_queries(3000, 4)  # ragged: 3000 = 46 * 64 + 56
    gt, ot = build_both(src, w, nrm, d=d)
    st = check_sbh(gt, ot, q, kernel, samples=2, seed=123, alpha=100.0, group=G)
    print(st)


def test_sbh_seeds_and_batch_words_change_streams():
    c = W.c1()
    gt, ot = build_both(c.sources, c.weights)
    outs = []
    for seed, batch in ((1, 0), (2**40 + 5, 0), (7, 3), (7, 0)):
        check_sbh(gt, ot, c.queries[:512], P.POTENTIAL, samples=1, seed=seed, batch=batch)
        outs.append(host(P.sbh_eval(gt, T(c.queries[:512]), P.POTENTIAL, samples=1, seed=seed, batch=batch)))
    assert not np.array_equal(outs[2], outs[3])


@pytest.mark.parametrize("G", [1, 64])
def test_sbh_deterministic_and_launch_independent(G):
    c = W.c1()
    gt, _ = build_both(c.sources, c.weights)
    q = T(c.queries)
    a = host(P.sbh_eval(gt, q, P.POTENTIAL, samples=3, seed=9, group=G))
    b = host(P.sbh_eval(gt, q, P.POTENTIAL, samples=3, seed=9, group=G))
    assert np.array_equal(a, b)
    # a query's value depends only on its index, not on how many queries share the launch
    part = host(P.sbh_eval(gt, q[:1000], P.POTENTIAL, samples=3, seed=9, group=G))
    assert np.array_equal(part, a[:1000])


@pytest.mark.parametrize("kernel", [P.POTENTIAL, P.WINDING, P.SMOOTHDIST])
@pytest.mark.parametrize("S", [1, 3])
def test_sbh_tail_split_gives_the_same_values(kernel, S, monkeypatch):
    """The coherent walk (d = 2) walks the last tiles of a launch over four wavefronts instead of
    two and adds the slot totals in the two-part association: every value and path must be the
    same bit for bit whatever the number of four-part tiles (none, some, all), on a ragged count."""
    src, nrm, w = surface(20000, seed=35)
    nq = 64 * 37 + 21
    q = T(box_queries(nq, 36))
    gt = P.sbh_build(T(src), T(w), T(nrm) if kernel == P.WINDING else None)

    def run():
        paths = torch.full((nq, 8, S, 4), -7, dtype=torch.int32, device=DEV)
        out = P.sbh_eval(gt, q, kernel, samples=S, seed=5, group=64, paths=paths, alpha=100.0)
        plain = P.sbh_eval(gt, q, kernel, samples=S, seed=5, group=64, alpha=100.0)
        return [host(out), host(paths), host(plain)]

    res = []
    for tail in ("0", "7", "20", "100000"):
        monkeypatch.setenv("SBH_TAIL_TILES", tail)
        res.append(run())
    for r in res[1:]:
        for x, y in zip(res[0], r):
            assert np.array_equal(x, y, equal_nan=True)


@pytest.mark.parametrize("kernel,branching", [(P.POTENTIAL, 2), (P.WINDING, 2), (P.SMOOTHDIST, 4)])
def test_sbh_wide_offsets_give_the_same_walk(kernel, branching, monkeypatch):
    """The coherent walks and Barnes-Hut take 32-bit byte offsets into trees below 4 GiB and
    64-bit ones beyond; forcing the 64-bit form on a small tree must change no value and no
    path."""
    src, nrm, w = surface(20000, seed=33)
    q = T(box_queries(3001, 34))
    gt = P.sbh_build(T(src), T(w), T(nrm) if kernel == P.WINDING else None, branching=branching)
    d3 = branching ** 3

    def run():
        paths = torch.full((3001, d3, 2, 4), -7, dtype=torch.int32, device=DEV)
        out = P.sbh_eval(gt, q, kernel, samples=2, seed=5, group=64, paths=paths, alpha=100.0)
        plain = P.sbh_eval(gt, q, kernel, samples=2, seed=5, group=64, alpha=100.0)
        bh = P.sbh_eval(gt, q, kernel, beta=0.7, samples=0, alpha=100.0)   # Barnes-Hut takes the same offsets
        res = [host(out), host(paths), host(plain), host(bh)]
        if branching == 2:   # and the tile-shared score proposal's walk
            res.append(host(P.sbh_eval(gt, q, kernel, samples=1, seed=5, group=64, alpha=100.0, proposal=3)))
        return res

    a = run()
    monkeypatch.setenv("SBH_FORCE_WIDE_OFFSETS", "1")
    b = run()
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True)


def test_sbh_root_leaf_is_exact():
    for m in (1, 5, 8):
        c = W.uniform_cube(m, 100, 31)
        gt, ot = build_both(c.sources, c.weights)
        g = host(P.sbh_eval(gt, T(c.queries), P.POTENTIAL, samples=1))
        F = oracle.brute(c.sources, c.weights, None, c.queries, P.POTENTIAL)
        assert np.allclose(g, F, rtol=2e-6)
        b = host(P.sbh_eval(gt, T(c.queries), P.POTENTIAL, beta=2.0, samples=0))
        assert np.allclose(b, F, rtol=2e-6)


def test_sbh_empty_and_tiny_query_sets():
    c = W.c1()
    gt, ot = build_both(c.sources, c.weights)
    out = torch.full((4,), 123.0, device=DEV)
    P.sbh_eval(gt, T(c.queries[:0]), P.POTENTIAL, out=out[:0])
    assert np.all(host(out) == 123.0)
    for n in (1, 7, 63, 65):
        check_sbh(gt, ot, c.queries[:n], P.POTENTIAL, samples=1)


def test_duplicate_points_estimator():
    src = np.array([[0.3, 0.3, 0.3]] * 40 + [[0, 0, 0], [1, 1, 1]] + [[0.7, 0.2, 0.9]] * 30, np.float32)
    w = np.linspace(0.5, 1.5, len(src)).astype(np.float32)
    q = box_queries(500, 8, -0.5, 1.5)
    gt, ot = build_both(src, w, d=2, leaf_size=4, max_level=6)
    check_sbh(gt, ot, q, P.POTENTIAL, samples=2)


# ----------------------------------------------------------------------------- Barnes-Hut-cut subdomains
@pytest.mark.parametrize("d,S,G,rr,beta_low", [(2, 1, 64, 0, 0.4), (2, 2, 64, 0, 1.0), (2, 1, 128, 1, 0.6),
                                               (2, 1, 64, 2, 2.0), (4, 1, 64, 0, 0.5), (4, 2, 64, 0, 1.2)])
def test_sbh_cut_parity_c1(d, S, G, rr, beta_low):
    c = W.c1()
    gt, ot = build_both(c.sources, c.weights, d=d)
    print(check_cut(gt, ot, c.queries[:2000], P.POTENTIAL, beta_low, samples=S, seed=2, group=G, rr_mode=rr))


@pytest.mark.parametrize("kernel", [P.WINDING, P.SMOOTHDIST, P.POTENTIAL])
def test_sbh_cut_parity_surface(kernel):
    src, nrm, w = surface(30000, 9)
    q = box_queries(1000, 4)   # ragged: 15 full groups and 40 queries
    gt, ot = build_both(src, w, nrm)
    print(check_cut(gt, ot, q, kernel, 0.5, samples=1, seed=7, alpha=100.0))


def test_sbh_cut_limits_and_errors():
    c = W.c1()
    gt = P.sbh_build(T(c.sources), T(c.weights))
    q = T(c.queries[:640])
    F = oracle.brute(c.sources, c.weights, None, c.queries[:640], P.POTENTIAL)
    # no node far: every leaf summed exactly
    v = host(P.sbh_eval(gt, q, P.POTENTIAL, beta=1e9, samples=1, group=64, subdomains=1))
    assert np.max(np.abs(v - F) / np.abs(F)) < 1e-5
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_eval(gt, q, P.POTENTIAL, beta=0.5, samples=1, group=1, subdomains=1)     # needs G % 64 == 0
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_eval(gt, q, P.POTENTIAL, beta=float("inf"), samples=1, group=64, subdomains=1)
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_eval(gt, q, P.POTENTIAL, beta=0.5, samples=1, group=64, subdomains=1, proposal=3)


# ----------------------------------------------------------------------------- branching 8
@pytest.mark.parametrize("S,rr", [(1, 0), (2, 0), (1, 1), (1, 2)])
def test_sbh_parity_branching8_c1(S, rr):
    """Branching 8 (512 children per node, the largest factor of the paper's branching study): the
    coherent walk (G a multiple of 64) against the oracle."""
    c = W.c1()
    gt, ot = build_both(c.sources, c.weights, d=8)
    print(check_sbh(gt, ot, c.queries[:2000], P.POTENTIAL, samples=S, seed=3, group=64, rr_mode=rr))


@pytest.mark.parametrize("kernel", [P.WINDING, P.SMOOTHDIST])
def test_sbh_parity_branching8_surface(kernel):
    src, nrm, w = surface(30000, 9)
    q = box_queries(1000, 4)
    gt, ot = build_both(src, w, nrm, d=8)
    print(check_sbh(gt, ot, q, kernel, samples=1, seed=123, alpha=100.0, group=128))


def test_branching8_limits():
    c = W.c1()
    gt = P.sbh_build(T(c.sources), T(c.weights), branching=8)
    q = T(c.queries[:100])
    with pytest.raises(P.SbhError, match="EUNSUPPORTED"):
        P.sbh_eval(gt, q, P.POTENTIAL, samples=1, group=1)         # per-query streams: branching 2 and 4
    with pytest.raises(P.SbhError, match="EUNSUPPORTED"):
        P.sbh_eval(gt, q, P.POTENTIAL, samples=0, beta=2.0)       # Barnes-Hut: branching 2 and 4
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_build(T(c.sources), T(c.weights), branching=3)


def test_argument_errors():
    c = W.c1()
    gt, _ = build_both(c.sources[:100], c.weights[:100])
    q = T(c.queries[:10])
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_eval(gt, q, P.WINDING)          # no normals
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_eval(gt, q, P.POTENTIAL, samples=0, beta=0.0)
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_eval(gt, q, 7)
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_eval(gt, q, P.POTENTIAL, group=0)
    bad = c.sources[:100].copy(); bad[5, 1] = np.nan
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_build(T(bad), T(c.weights[:100]))
    wneg = c.weights[:100].copy(); wneg[3] = -1
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_build(T(c.sources[:100]), T(wneg))
    with pytest.raises(P.SbhError, match="EINVAL"):
        P.sbh_build(T(c.sources[:100]), T(c.weights[:100]), branching=3)


# ----------------------------------------------------------------------------- Barnes-Hut
@pytest.mark.parametrize("d,beta", [(2, 2.0), (2, 0.7), (4, 2.0), (2, 6.0)])
def test_bh_parity_c1(d, beta):
    c = W.c1()
    gt, ot = build_both(c.sources, c.weights, d=d)
    print(check_bh(gt, ot, c.queries, P.POTENTIAL, beta))


@pytest.mark.parametrize("kernel", [P.WINDING, P.SMOOTHDIST])
def test_bh_parity_surface_kernels(kernel):
    src, nrm, w = surface(30000, 9)
    q = box_queries(3000, 4)
    gt, ot = build_both(src, w, nrm)
    print(check_bh(gt, ot, q, kernel, 2.0, alpha=100.0))


def test_bh_infinite_beta_is_exact():
    src, nrm, w = surface(20000, 2)
    q = box_queries(700, 1)
    gt, _ = build_both(src, w, nrm)
    for kernel in (P.POTENTIAL, P.WINDING):
        g = host(P.sbh_eval(gt, T(q), kernel, beta=math.inf, samples=0))
        ref = fp64_reference(src, w, nrm, q, kernel)
        assert np.all(np.abs(g - ref) <= 1e-4 * value_scale(ref, kernel, 100.0))


# ----------------------------------------------------------------------------- deep trees
def geometric_cluster(n, seed=12):
    """Half of the points uniform in the cube [-1/2, 1/2]^3, half at distances 2^-u (u uniform in
    [2, 19]) from its centre, the origin: the tree reaches level 18 and more there.  Around the
    origin float32 resolves offsets of 2^-19 to full precision (around 1/2 it would keep only about
    six bits of them, and the centres of mass and second moments of the deepest nodes would be
    noise on both sides of the comparison)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = n // 2
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    c = np.zeros(3)
    cl = c + d * (2.0 ** -rng.uniform(2, 19, m))[:, None]
    src = np.concatenate([rng.uniform(-0.5, 0.5, (n - m, 3)), cl]).astype(np.float32)
    w = rng.uniform(0.5, 1.5, n).astype(np.float32)
    q = (c + rng.normal(size=(1024, 3)) * (2.0 ** -rng.uniform(3, 14, 1024))[:, None]).astype(np.float32)
    return src, w, q


@pytest.mark.parametrize("G,rr,proposal", [(64, 1, None), (64, 2, None), (1, 1, None), (1, 2, None),
                                            (64, 0, None), (64, 1, 3), (1, 1, 2)])
def test_deep_tree_paths_beyond_sixteen_steps(G, rr, proposal):
    """Leaf size 1 on a geometric cluster: paths without roulette (rr = 1) and with p = 1/2 run
    past step 16, where the coherent walk computes its random words again instead of taking the
    ones it holds; every path record must still match the oracle bit for bit."""
    src, w, q = geometric_cluster(6000)
    gt, ot = build_both(src, w, leaf_size=1)
    assert gt.depth >= 18, gt.depth
    paths = torch.full((q.shape[0], 8, 1, 4), -7, dtype=torch.int32, device=DEV)
    out = host(P.sbh_eval(gt, T(q), P.POTENTIAL, samples=1, seed=4, group=G, rr_mode=rr, paths=paths,
                          proposal=proposal))
    pth = host(paths)
    st = check_sbh(gt, ot, q, P.POTENTIAL, samples=1, seed=4, group=G, rr_mode=rr, gpu_out=out, gpu_paths=pth,
                   index=np.arange(q.shape[0]), proposal=proposal)
    deep = int((pth[..., 2] >= 17).sum())
    print(st, "paths with >= 17 accepted steps:", deep)
    if rr == 1:   # no roulette: every path into the cluster runs to a one-point leaf
        assert deep > 0
