"""Parity of the compressed-aggregate walk (the conclusion's compressed
level-of-detail representation under the estimator of Section 3.3) with the
FP64 oracle on the same compressed aggregates.

  - the binary16 codes the GPU build stores are bit-identical to the
    oracle's, node by node (the float64 aggregates they round are summed in
    the same order on both sides);
  - estimates and path records of the coherent walk (G = 64) and of the
    per-lane walk (per-query streams, G = 1 and G = 7) match the oracle's walk
    on the decoded aggregates, to the tolerances stated in
    gpu_helpers, on ragged query counts, several samples, every roulette
    mode, a deep tree whose paths pass step 16, and the full-size 2^22-source
    potential workload on sampled queries;
  - the option's limits are errors, not fallbacks."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_2506_02219_amd as P
from gpu_helpers import DEV, T, host, compare_trees, check_sbh, compressed_codes_by_node

pytestmark = pytest.mark.gpu


def build_cmp(src, w, leaf_size=8):
    gt = P.sbh_build(T(src), T(w), branching=2, leaf_size=leaf_size, compress=True)
    ot = oracle.Tree(src, w, None, d=2, leaf_size=leaf_size)
    compare_trees(gt, ot)
    return gt, ot


def geometric_cluster(n, seed=3):
    """Half the points uniform in [-1/2, 1/2]^3, half at distances 2^-u (u uniform in [2, 19]) from
    the origin: a tree of level 18 and more, queries near the cluster."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = n // 2
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    cl = d * (2.0 ** -rng.uniform(2, 19, m))[:, None]
    src = np.concatenate([rng.uniform(-0.5, 0.5, (n - m, 3)), cl]).astype(np.float32)
    w = rng.uniform(0.5, 1.5, n).astype(np.float32)
    q = (rng.normal(size=(1024, 3)) * (2.0 ** -rng.uniform(3, 14, 1024))[:, None]).astype(np.float32)
    return src, w, q


@pytest.mark.parametrize("case", ["uniform", "cluster"])
def test_codes_bit_exact(case):
    if case == "uniform":
        cl = W.uniform_cube(50000, 64, 31)
        src, w = cl.sources, cl.weights
    else:
        src, w, _ = geometric_cluster(20000)
    gt, ot = build_cmp(src, w, leaf_size=8 if case == "uniform" else 1)
    g = compressed_codes_by_node(gt)
    _, o = ot.compressed()
    assert np.array_equal(g.view(np.uint32), o.view(np.uint32)), int((g != o).any(axis=1).sum())


@pytest.mark.parametrize("kernel", [P.POTENTIAL, P.SMOOTHDIST])
@pytest.mark.parametrize("S", [1, 3])
@pytest.mark.parametrize("rr", [0, 1])
@pytest.mark.parametrize("G", [64, 1])
def test_compressed_walk_parity(kernel, S, rr, G):
    cl = W.uniform_cube(40000, 3000 + 37, 7)   # ragged: 3037 = 47 * 64 + 29
    gt, ot = build_cmp(cl.sources, cl.weights)
    st = check_sbh(gt, ot, cl.queries, kernel, samples=S, seed=11, group=G, rr_mode=rr, alpha=100.0,
                   compressed=True)
    print(st)


@pytest.mark.parametrize("rr", [0, 1, 2])
@pytest.mark.parametrize("G", [64, 1])
def test_compressed_deep_tree(rr, G):
    """Leaf size 1 on the geometric cluster: one-point nodes take the leaf step, and paths without
    roulette run past step 16."""
    src, w, q = geometric_cluster(6000)
    gt, ot = build_cmp(src, w, leaf_size=1)
    assert gt.depth >= 18, gt.depth
    paths = torch.full((q.shape[0], 8, 1, 4), -7, dtype=torch.int32, device=DEV)
    out = host(P.sbh_eval(gt, T(q), P.POTENTIAL, samples=1, seed=4, group=G, rr_mode=rr, paths=paths,
                          compressed=1))
    pth = host(paths)
    st = check_sbh(gt, ot, q, P.POTENTIAL, samples=1, seed=4, group=G, rr_mode=rr, gpu_out=out, gpu_paths=pth,
                   index=np.arange(q.shape[0]), compressed=True)
    print(st, "paths with >= 17 accepted steps:", int((pth[..., 2] >= 17).sum()))
    assert not np.any(pth[..., 3] == 1)   # no one-point stop under compression


@pytest.mark.parametrize("G,S", [(128, 2), (7, 2), (1, 32)])
def test_compressed_group_and_batch_words(G, S):
    """G = 128 (two wavefronts share a stream), G = 7 (streams across lanes of the per-lane walk),
    S = 32 (the per-lane walk's largest pool share) and a nonzero batch word reach the same streams
    on both sides."""
    cl = W.uniform_cube(20000, 1000, 9)
    gt, ot = build_cmp(cl.sources, cl.weights)
    print(check_sbh(gt, ot, cl.queries, P.POTENTIAL, samples=S, seed=5, group=G, batch=7, compressed=True))


def test_compressed_fullsize_c5():
    """The 2^22-source potential workload (the shuffled plane, G = 64 and G = 1): codes compared on
    every node, every query evaluated, 1500 sampled queries recomputed by the oracle at their
    indices."""
    c5 = W.c5()
    q, _ = W.shuffle_queries(c5.queries, 4242)
    gt, ot = build_cmp(c5.sources, c5.weights)
    _, o = ot.compressed()
    assert np.array_equal(compressed_codes_by_node(gt).view(np.uint32), o.view(np.uint32))
    idx = np.sort(np.random.Generator(np.random.PCG64(17)).choice(q.shape[0], 1500, replace=False))
    for G in (64, 1):
        paths = torch.empty((q.shape[0], 8, 1, 4), dtype=torch.int32, device=DEV)
        out = host(P.sbh_eval(gt, T(q), P.POTENTIAL, samples=1, seed=0, group=G, paths=paths, compressed=1))
        pth = host(paths)
        print(G, check_sbh(gt, ot, q[idx], P.POTENTIAL, samples=1, seed=0, group=G, index=idx, gpu_out=out,
                           gpu_paths=pth, compressed=True))


def test_compressed_limits():
    cl = W.uniform_cube(5000, 128, 2)
    q = T(cl.queries)
    plain = P.sbh_build(T(cl.sources), T(cl.weights))
    with pytest.raises(P.SbhError) as e:
        P.sbh_eval(plain, q, P.POTENTIAL, samples=1, group=64, compressed=1)
    assert "compress" in str(e.value)
    gt = P.sbh_build(T(cl.sources), T(cl.weights), compress=True)
    for kw in (dict(group=1, samples=33), dict(group=64, proposal=3), dict(group=1, proposal=2),
               dict(group=64, subdomains=1, beta=0.5)):
        with pytest.raises(P.SbhError):
            P.sbh_eval(gt, q, P.POTENTIAL, compressed=1, **{"samples": 1, **kw})
    nrm = np.zeros_like(cl.sources)
    nrm[:, 2] = 1.0
    gw = P.sbh_build(T(cl.sources), T(cl.weights), T(nrm), compress=True)
    with pytest.raises(P.SbhError):
        P.sbh_eval(gw, q, P.WINDING, samples=1, group=64, compressed=1)
    with pytest.raises(P.SbhError):
        P.sbh_build(T(cl.sources), T(cl.weights), branching=4, compress=True)
    with pytest.raises(P.SbhError):
        P.sbh_eval(gt, q, P.POTENTIAL, samples=1, group=64, compressed=2)
    # Barnes-Hut ignores the option; the uncompressed walk on a compressed tree is unchanged
    a = host(P.sbh_eval(gt, q, P.POTENTIAL, samples=1, seed=3, group=64))
    b = host(P.sbh_eval(plain, q, P.POTENTIAL, samples=1, seed=3, group=64))
    assert np.array_equal(a, b)
    # an empty query set is a no-op
    P.sbh_eval(gt, T(np.zeros((0, 3), np.float32)), P.POTENTIAL, samples=1, group=64, compressed=1)
