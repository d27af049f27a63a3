"""Parity of the roulette voted over a wavefront (rr_mode 3: the 64 queries of
a tile share their stream, and with it the node sequence and the variate u;
they also share p, the largest Eq. (5) probability among the tile's queries
with finite coordinates, and stop or continue together) with the FP64
oracle's voted estimator, to the tolerances stated in gpu_helpers.

Covered: the branching factors of the coherent walk (2, 4 and 8), every
kernel at alpha = 100, S = 1 and 3, G = 64 and 128, ragged tails, the
four-part tail tiles, a deep tree whose paths pass step 16, the compressed
and second-order walks, a query with non-finite coordinates (which does not
vote), the batched kernel (bit-identical to single calls), the 2^22 potential
workload on sampled whole tiles, and the option's limits."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_2506_02219_amd as P
from gpu_helpers import DEV, T, host, build_both, compare_trees, check_sbh

pytestmark = pytest.mark.gpu


def surface(m, seed=21, level=4):
    pts, nrm, w, _ = W.star_surface(m, seed, level=level)
    return pts.astype(np.float32), nrm.astype(np.float32), w.astype(np.float32)


def box_queries(n, seed, lo=-1.5, hi=1.5):
    return np.random.Generator(np.random.PCG64(seed)).uniform(lo, hi, (n, 3)).astype(np.float32)


@pytest.mark.parametrize("d", [2, 4, 8])
@pytest.mark.parametrize("S", [1, 3])
@pytest.mark.parametrize("G", [64, 128])
def test_vote_parity_c1(d, S, G):
    c = W.c1()
    gt, ot = build_both(c.sources, c.weights, d=d)
    print(check_sbh(gt, ot, c.queries, P.POTENTIAL, samples=S, seed=3, group=G, rr_mode=3))


@pytest.mark.parametrize("kernel", [P.WINDING, P.SMOOTHDIST, P.POTENTIAL])
def test_vote_parity_surface_kernels(kernel):
    src, nrm, w = surface(30000, 9)
    q = box_queries(3000, 4)   # ragged: 3000 = 46 * 64 + 56
    gt, ot = build_both(src, w, nrm)
    print(check_sbh(gt, ot, q, kernel, samples=2, seed=123, alpha=100.0, group=64, rr_mode=3))


def test_vote_deep_tree():
    rng = np.random.Generator(np.random.PCG64(3))
    m = 3000
    dd = rng.normal(size=(m, 3))
    dd /= np.linalg.norm(dd, axis=1, keepdims=True)
    src = np.concatenate([rng.uniform(-0.5, 0.5, (m, 3)), dd * (2.0 ** -rng.uniform(2, 19, m))[:, None]])
    src = src.astype(np.float32)
    w = rng.uniform(0.5, 1.5, 2 * m).astype(np.float32)
    q = (rng.normal(size=(1024, 3)) * (2.0 ** -rng.uniform(3, 14, 1024))[:, None]).astype(np.float32)
    gt, ot = build_both(src, w, leaf_size=1)
    assert gt.depth >= 18
    paths = torch.full((q.shape[0], 8, 1, 4), -7, dtype=torch.int32, device=DEV)
    out = host(P.sbh_eval(gt, T(q), P.POTENTIAL, samples=1, seed=4, group=64, rr_mode=3, paths=paths))
    pth = host(paths)
    st = check_sbh(gt, ot, q, P.POTENTIAL, samples=1, seed=4, group=64, rr_mode=3, gpu_out=out, gpu_paths=pth,
                   index=np.arange(q.shape[0]))
    print(st, "paths with >= 17 accepted steps:", int((pth[..., 2] >= 17).sum()))
    # every lane of a tile has its tile's records
    pt = pth.reshape(16, 64, 8, 1, 4)
    assert np.all(pt == pt[:, :1])


def test_vote_with_compressed_and_second_order_terms():
    cl = W.uniform_cube(30000, 2000 + 45, 8)
    for kw, okw in ((dict(compress=True), dict(compressed=True)), (dict(quadrupole=True), dict(lod=2))):
        gt = P.sbh_build(T(cl.sources), T(cl.weights), **kw)
        ot = oracle.Tree(cl.sources, cl.weights, None, d=2, leaf_size=8)
        compare_trees(gt, ot)
        print(kw, check_sbh(gt, ot, cl.queries, P.POTENTIAL, samples=2, seed=6, group=64, rr_mode=3, **okw))


def test_non_finite_query_does_not_vote():
    cl = W.uniform_cube(20000, 640, 10)
    q = cl.queries.copy()
    q[70] = np.nan   # in the second tile
    gt, ot = build_both(cl.sources, cl.weights)
    out = host(P.sbh_eval(gt, T(q), P.POTENTIAL, samples=1, seed=2, group=64, rr_mode=3))
    assert np.isnan(out[70]) and np.all(np.isfinite(np.delete(out, 70)))
    print(check_sbh(gt, ot, q, P.POTENTIAL, samples=1, seed=2, group=64, rr_mode=3))


def test_vote_tail_split_and_launch_independence(monkeypatch):
    cl = W.uniform_cube(20000, 64 * 30 + 7, 12)
    gt, _ = build_both(cl.sources, cl.weights)
    q = T(cl.queries)
    res = []
    for tail in ("0", "5", "1000"):
        monkeypatch.setenv("SBH_TAIL_TILES", tail)
        res.append(host(P.sbh_eval(gt, q, P.POTENTIAL, samples=2, seed=7, group=64, rr_mode=3)))
    for r in res[1:]:
        assert np.array_equal(r, res[0])
    part = host(P.sbh_eval(gt, q[:640], P.POTENTIAL, samples=2, seed=7, group=64, rr_mode=3))
    assert np.array_equal(part, res[0][:640])


def test_vote_batch_equals_single_calls():
    specs = [(3000, 2500, 0, 11, 2), (700, 64, 1, 12, 2), (20000, 4097, 2, 14, 2), (9000, 1000, 1, 16, 4)]
    trees, qs, kernels = [], [], []
    for m, n, k, seed, d in specs:
        cl = W.c4_cloud(dict(index=seed, m=m, n=n, kernel=k, seed=seed))
        trees.append(P.sbh_build(T(cl.sources), T(cl.weights), None if cl.normals is None else T(cl.normals),
                                 branching=d))
        qs.append(T(np.ascontiguousarray(cl.queries[:n])))
        kernels.append(k)
    b = P.Batch(trees, qs, kernels, samples=2, alpha=100.0, rr_mode=3)
    outs = [host(o) for o in b.launch(5, 2)]
    for t, q, k, o in zip(trees, qs, kernels, outs):
        r = host(P.sbh_eval(t, q, k, samples=2, seed=5, group=64, alpha=100.0, batch=2, rr_mode=3))
        assert np.array_equal(o, r, equal_nan=True)
    b.free()


def test_vote_fullsize_c5():
    """The 2^22-source potential workload (the shuffled plane, G = 64): every query evaluated, 24
    sampled whole tiles recomputed by the oracle."""
    c5 = W.c5()
    q, _ = W.shuffle_queries(c5.queries, 4242)
    gt = P.sbh_build(T(c5.sources), T(c5.weights))
    ot = oracle.Tree(c5.sources, c5.weights, None, d=2, leaf_size=8)
    compare_trees(gt, ot)
    paths = torch.empty((q.shape[0], 8, 1, 4), dtype=torch.int32, device=DEV)
    out = host(P.sbh_eval(gt, T(q), P.POTENTIAL, samples=1, seed=0, group=64, rr_mode=3, paths=paths))
    pth = host(paths)
    g = np.sort(np.random.Generator(np.random.PCG64(5)).choice(q.shape[0] // 64, 24, replace=False))
    idx = (g[:, None] * 64 + np.arange(64)[None, :]).ravel()
    print(check_sbh(gt, ot, q[idx], P.POTENTIAL, samples=1, seed=0, group=64, rr_mode=3, index=idx, gpu_out=out,
                    gpu_paths=pth))


def test_vote_limits():
    cl = W.uniform_cube(3000, 128, 2)
    gt = P.sbh_build(T(cl.sources), T(cl.weights))
    q = T(cl.queries)
    for kw in (dict(group=1), dict(group=32), dict(proposal=3), dict(proposal=2, group=1),
               dict(subdomains=1, beta=0.5)):
        with pytest.raises(P.SbhError):
            P.sbh_eval(gt, q, P.POTENTIAL, rr_mode=3, **{"samples": 1, "group": 64, **kw})
    with pytest.raises(P.SbhError):
        P.sbh_eval(gt, q, P.POTENTIAL, samples=1, group=64, rr_mode=4)
    # Barnes-Hut takes no roulette
    a = host(P.sbh_eval(gt, q, P.POTENTIAL, beta=1.0, samples=0, group=64, rr_mode=3))
    b = host(P.sbh_eval(gt, q, P.POTENTIAL, beta=1.0, samples=0))
    assert np.array_equal(a, b)
