"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times (d = 2, G = 64 coherent wavefronts and G = 1 per-query
streams; the score, tile and network proposals; d = 4): the whole tree is compared bit-exactly, every query is evaluated on
the GPU, and a seeded sample of queries is recomputed one by one by the
oracle (at their original indices, so they use the same random streams).
Barnes-Hut is checked on sampled groups of 64 consecutive queries."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_2506_02219_amd as P
from gpu_helpers import DEV, T, host, compare_trees, check_sbh, check_bh, check_cut

pytestmark = pytest.mark.gpu

NSAMPLE = 1500


def run_full(cl, group, samples, alpha=100.0, d=2, proposal=None, trees=None, mlp=None):
    if trees is None:
        gt = P.sbh_build(T(cl.sources), T(cl.weights), None if cl.normals is None else T(cl.normals), branching=d)
        ot = oracle.Tree(cl.sources, cl.weights, cl.normals, d=d, leaf_size=8)
        compare_trees(gt, ot)
    else:
        gt, ot = trees
    q = T(cl.queries)
    paths = torch.empty((cl.n, d ** 3, samples, 4), dtype=torch.int32, device=DEV)
    out = host(P.sbh_eval(gt, q, cl.kernel, samples=samples, seed=0, group=group, alpha=alpha, paths=paths,
                          proposal=proposal, mlp=None if mlp is None else T(mlp)))
    pth = host(paths)
    idx = np.sort(np.random.Generator(np.random.PCG64(17)).choice(cl.n, NSAMPLE, replace=False))
    st = check_sbh(gt, ot, cl.queries[idx], cl.kernel, samples=samples, seed=0, group=group, alpha=alpha,
                   index=idx, gpu_out=out, gpu_paths=pth, proposal=proposal, mlp=mlp,
                   tile_all=cl.queries if proposal == 3 else None)
    return gt, ot, st


def bh_sampled(gt, ot, cl, beta=2.0, ngroups=24):
    out = host(P.sbh_eval(gt, T(cl.queries), cl.kernel, beta=beta, samples=0))
    g = np.random.Generator(np.random.PCG64(5)).choice(cl.n // 64, ngroups, replace=False)
    idx = (g[:, None] * 64 + np.arange(64)[None, :]).ravel()
    return check_bh(gt, ot, cl.queries[idx], cl.kernel, beta, gpu_out=out[idx])


@pytest.fixture(scope="module")
def c2():
    return W.c2()


@pytest.fixture(scope="module")
def c5():
    return W.c5()


@pytest.fixture(scope="module")
def c3():
    return W.c3()


@pytest.mark.parametrize("group", [64, 1])
def test_c2_winding_fullsize(c2, group):
    q, _ = W.shuffle_queries(c2.queries, 4242) if group > 1 else (c2.queries, None)
    cl = W.Cloud(c2.sources, c2.weights, c2.normals, q, c2.kernel)
    gt, ot, st = run_full(cl, group, 1)
    print(st)
    if group == 1:
        print(bh_sampled(gt, ot, cl))


def test_c5_potential_fullsize(c5):
    q, _ = W.shuffle_queries(c5.queries, 4242)
    cl = W.Cloud(c5.sources, c5.weights, None, q, c5.kernel)
    gt, ot, st = run_full(cl, 64, 1)
    print(st)
    print(bh_sampled(gt, ot, cl))
    # the plane in its own order with the tile-shared score proposal (same trees)
    grid = W.Cloud(c5.sources, c5.weights, None, c5.queries, c5.kernel)
    print(run_full(grid, 64, 1, proposal=3, trees=(gt, ot))[2])
    # the per-query proposals the benchmark times on this tree (G = 1, the shuffled plane): the score
    # proposal, and a network (exact in binary16, so that both sides see the same logits)
    print(run_full(cl, 1, 1, proposal=2, trees=(gt, ot))[2])
    print(run_full(cl, 1, 1, mlp=dyadic_network(47), trees=(gt, ot))[2])


def dyadic_network(seed):
    """Network parameters whose hidden values and logits are exact in binary16 and float32 (W1 = W2 = 0,
    every other value a multiple of 2^-6): the GPU and the oracle see identical logits."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(oracle.MLP_NPARAM, np.float32)
    p[256:288] = rng.integers(-64, 65, 32) / 64.0
    p[1312:1344] = rng.integers(0, 65, 32) / 64.0
    p[1344:1600] = rng.integers(-64, 65, 256) / 64.0
    p[1600:1608] = rng.integers(-64, 65, 8) / 64.0
    return p


def test_c5_potential_fullsize_branching4(c5):
    """The 2^22-source tree at d = 4 (the paper's branching factor for the estimator), both stream modes."""
    q, _ = W.shuffle_queries(c5.queries, 4242)
    cl = W.Cloud(c5.sources, c5.weights, None, q, c5.kernel)
    gt, ot, st = run_full(cl, 64, 1, d=4)
    print(st)
    print(run_full(cl, 1, 1, d=4, trees=(gt, ot))[2])


@pytest.mark.parametrize("samples", [1, 4])
def test_c3_smooth_fullsize(c3, samples):
    cl = W.Cloud(c3.sources, c3.weights, c3.normals, c3.queries, c3.kernel)
    gt, ot, st = run_full(cl, 64, samples)
    print(st)


def test_c5_potential_fullsize_cut_subdomains(c5):
    """Subdomains from the Barnes-Hut cut at beta = 0.5 on the 2^22-source potential workload (the
    shuffled plane, G = 64): 24 sampled groups of 64 queries (whole groups, for the vote)."""
    q, _ = W.shuffle_queries(c5.queries, 4242)
    gt = P.sbh_build(T(c5.sources), T(c5.weights))
    ot = oracle.Tree(c5.sources, c5.weights, None, d=2, leaf_size=8)
    dig = torch.empty((q.shape[0], 4), dtype=torch.int32, device=DEV)
    out = host(P.sbh_eval(gt, T(q), P.POTENTIAL, beta=0.5, samples=1, seed=0, group=64, paths=dig, subdomains=1))
    g = np.random.Generator(np.random.PCG64(5)).choice(q.shape[0] // 64, 24, replace=False)
    idx = (np.sort(g)[:, None] * 64 + np.arange(64)[None, :]).ravel()
    print(check_cut(gt, ot, q[idx], P.POTENTIAL, 0.5, index=idx, gpu_out=out, gpu_digest=host(dig)))
