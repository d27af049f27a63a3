"""CPU pins of the oracle's Barnes-Hut-cut stratification (Section 3.3.1: the
contribution nodes D(q, beta) of a low beta as path roots in place of the
root's children), independent of the GPU.

  - Theorem 1 per subdomain: the exact expectation (every subdomain's control
    variate plus the exact expectation of its paths, leaves summed exactly)
    equals the float64 brute-force sum, for every kernel, both branching
    factors and every roulette mode;
  - the cut partitions the points: subdomains and exactly summed leaves
    together hold every point once;
  - beta_low so large that no node is far: every leaf is summed exactly, so
    the estimate is the brute-force sum for every seed (no subdomain);
  - beta_low so small that every root child is far: the subdomains are the
    root's children;
  - the vote: the cut (subdomains, leaves summed exactly) is the same for
    every query of a group;
  - the sampled mean over many seeds is within a CLT bound of the sum."""
import numpy as np
import pytest
from scipy.stats import norm

import workloads as W

POT, WIND, SMOOTH = 0, 1, 2


def _cloud(kernel, m=500, n=40, seed=3):
    if kernel == POT:
        cl = W.uniform_cube(m, n, seed)
        return cl.sources, cl.weights, None, cl.queries
    pts, nrm, w, _ = W.star_surface(m, seed, level=3)
    q = np.random.Generator(np.random.PCG64(seed)).uniform(-1.4, 1.4, (n, 3)).astype(np.float32)
    return pts.astype(np.float32), w.astype(np.float32), nrm.astype(np.float32), q


@pytest.mark.parametrize("d", [2, 4])
@pytest.mark.parametrize("rr_mode", [0, 1, 2])
@pytest.mark.parametrize("kernel", [POT, WIND, SMOOTH])
@pytest.mark.parametrize("beta_low", [0.3, 1.0, 3.0])
def test_cut_expectation_equals_brute_force(orc, d, rr_mode, kernel, beta_low):
    src, w, nrm, q = _cloud(kernel)
    t = orc.Tree(src, w, nrm, d=d, leaf_size=4)
    F = orc.brute(src, w, nrm, q, kernel, alpha=20.0)
    e = t.sbh_cut(q, kernel, beta_low, rr_mode=rr_mode, alpha=20.0, expect=True)["F"]
    scale = np.maximum(np.abs(F), 1.0 if kernel == WIND else 1e-300)
    assert np.max(np.abs(e - F) / scale) < 1e-11


def _cut_points(t, q, beta_low, vote=64):
    """Points covered by the cut's subdomains and by its exactly summed leaves, recomputed from the
    exported tree with NumPy (the voted walk, written out a second time)."""
    internal = t.internal
    kids = {}
    for i in range(1, t.n_nodes):
        kids.setdefault(int(t.parent[i]), []).append(i)
    diam = np.sqrt(3.0) * float(t.side) / float(t.d) ** t.level.astype(np.float64)
    covered = np.zeros(t.m, np.int64)
    n_sub = n_leaf = 0
    stack = list(kids[0])[::-1]
    while stack:
        v = stack.pop()
        far = np.all(np.linalg.norm(q.astype(np.float64) - t.agg[v, :3], axis=1) / diam[v] >= beta_low)
        if far or not internal[v]:
            covered[t.begin[v]:t.begin[v] + t.count[v]] += 1
            n_sub += int(far)
            n_leaf += int(not far)
        else:
            stack.extend(kids[v][::-1])
    return covered, n_sub, n_leaf


@pytest.mark.parametrize("beta_low", [0.4, 1.5])
def test_cut_partitions_the_points_and_is_voted(orc, beta_low):
    src, w, nrm, q = _cloud(POT, m=3000, n=64)
    t = orc.Tree(src, w, d=2, leaf_size=4)
    r = t.sbh_cut(q, POT, beta_low, samples=2)
    dg = r["digest"]
    assert np.all(dg[:, 0] == dg[0, 0]) and np.all(dg[:, 1] == dg[0, 1])   # one cut per group
    covered, n_sub, n_leaf = _cut_points(t, q, beta_low)
    assert np.all(covered == 1)
    assert (dg[0, 0], dg[0, 1]) == (n_sub, n_leaf)


def test_cut_limits(orc):
    src, w, nrm, q = _cloud(POT, m=800, n=64)
    t = orc.Tree(src, w, d=2, leaf_size=4)
    F = orc.brute(src, w, None, q, POT)
    # no node far: every leaf summed exactly, whatever the seed
    for seed in (0, 5):
        r = t.sbh_cut(q, POT, 1e9, seed=seed)
        assert np.all(r["digest"][:, 0] == 0)
        assert np.max(np.abs(r["F"] - F) / np.abs(F)) < 1e-12
    # every root child far: the subdomains are the root's children
    r = t.sbh_cut(q, POT, 1e-9)
    assert np.all(r["digest"][:, 0] == t.nchild[0]) and np.all(r["digest"][:, 1] == 0)


@pytest.mark.parametrize("beta_low", [0.3, 0.8])
def test_cut_sampled_mean_converges_to_brute_force(orc, beta_low):
    src, w, nrm, q = _cloud(POT, m=400, n=16, seed=8)
    t = orc.Tree(src, w, d=2, leaf_size=4)
    F = orc.brute(src, w, None, q, POT)
    K = 3000
    acc = np.array([t.sbh_cut(q, POT, beta_low, seed=s, vote=16)["F"] for s in range(K)])
    mean, se = acc.mean(0), acc.std(0, ddof=1) / np.sqrt(K)
    z = norm.isf(1e-3 / (2 * q.shape[0]))
    assert np.all(np.abs(mean - F) <= z * se + 1e-12 * np.abs(F)), np.max(np.abs(mean - F) / se)
    assert np.all(acc.std(0) > 0)
