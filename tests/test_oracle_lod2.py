"""CPU pins of the oracle's second-order level of detail (Section 3.1 allows
higher-order node approximations in place of the point mass; the estimator of
Section 3.3 and Theorem 1 on top of it), independent of the GPU.

  - the second-moment tensor of a node is the weighted sum of its points'
    outer products about its centre of mass (recomputed with NumPy);
  - the quadrupole term is the next order of the Taylor expansion: far from a
    cluster the point-mass error falls as r^-3 and the second-order error as
    r^-4 (halving the distance multiplies them by about 8 and 16), and at
    each distance the second-order error is far below the point mass's;
    both a wrong sign and a wrong factor of the tensor or trace break this;
  - the term is added only where the node is far (|q - com| >= |B|);
  - Theorem 1: the exact expectation with second-order node terms equals the
    float64 brute-force sum for every roulette mode and d in {2, 4};
  - the sampled mean over many seeds is within a CLT bound of the sum;
  - the estimator's median error falls on far queries (the control variates
    absorb more of the sum)."""
import numpy as np
import pytest
from scipy.stats import norm

import workloads as W

POT = 0


def _cluster(m=60, seed=2, a=0.1):
    rng = np.random.Generator(np.random.PCG64(seed))
    src = (a * rng.uniform(-0.5, 0.5, (m, 3)) + np.array([0.3, -0.2, 0.1])).astype(np.float32)
    w = rng.uniform(0.2, 2.0, m).astype(np.float32)
    return src, w


def test_second_moments_from_the_points(orc):
    cl = W.uniform_cube(3000, 4, 21)
    t = orc.Tree(cl.sources, cl.weights, d=2, leaf_size=4)
    t.set_lod(2)
    Q = t.quad()
    pts = cl.sources[t.perm].astype(np.float64)
    pw = cl.weights[t.perm].astype(np.float64)
    for i in np.random.Generator(np.random.PCG64(0)).choice(t.n_nodes, 200, replace=False):
        sl = slice(t.begin[i], t.begin[i] + t.count[i])
        x = pts[sl] - t.agg[i, :3]
        M = (pw[sl, None, None] * x[:, :, None] * x[:, None, :]).sum(0)
        want = np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])
        assert np.allclose(Q[i], want, rtol=1e-10, atol=1e-14 * max(1.0, np.abs(want).max()))
    # a one-point node has a zero tensor
    one = np.nonzero(t.count == 1)[0]
    assert one.size > 0 and np.all(Q[one] == 0.0)


def test_quadrupole_is_the_next_taylor_order(orc):
    src, w = _cluster()
    t = orc.Tree(src, w, d=2, leaf_size=100)   # one node: the root, a leaf holding the cluster
    com = t.agg[0, :3]
    rng = np.random.Generator(np.random.PCG64(3))
    dirs = rng.normal(size=(20, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    B = float(t.agg[0, 7])
    e1, e2 = [], []
    for r in (2.0 * B, 4.0 * B, 8.0 * B):
        q = com + r * dirs
        exact = orc.brute(src, w, None, q.astype(np.float32), POT)
        qf = q.astype(np.float32).astype(np.float64)
        t.set_lod(1)
        v1 = np.array([t.node_term(0, x) for x in qf])
        t.set_lod(2)
        v2 = np.array([t.node_term(0, x) for x in qf])
        e1.append(np.abs(v1 - exact))
        e2.append(np.abs(v2 - exact))
    e1, e2 = np.array(e1), np.array(e2)
    r1 = np.median(e1[1:] / e1[:-1], axis=1)
    r2 = np.median(e2[1:] / e2[:-1], axis=1)
    assert np.all((r1 > 1 / 11) & (r1 < 1 / 6)), r1      # ~ r^-3
    assert np.all((r2 > 1 / 22) & (r2 < 1 / 12)), r2      # ~ r^-4
    assert np.all(np.median(e2 / e1, axis=1) < 0.35)


def test_quadrupole_only_where_far(orc):
    src, w = _cluster()
    t = orc.Tree(src, w, d=2, leaf_size=100)
    com = t.agg[0, :3]
    B = float(t.agg[0, 7])
    t.set_lod(1)
    near = com + np.array([0.99 * B, 0.0, 0.0])
    far = com + np.array([1.01 * B, 0.0, 0.0])
    m1 = [t.node_term(0, x) for x in (near, far)]
    t.set_lod(2)
    m2 = [t.node_term(0, x) for x in (near, far)]
    assert m2[0] == m1[0] and m2[1] != m1[1]


@pytest.mark.parametrize("d", [2, 4])
@pytest.mark.parametrize("rr_mode", [0, 1, 2])
def test_lod2_expectation_equals_brute_force(orc, d, rr_mode):
    cl = W.uniform_cube(600, 40, 3)
    t = orc.Tree(cl.sources, cl.weights, d=d, leaf_size=4)
    t.set_lod(2)
    F = orc.brute(cl.sources, cl.weights, None, cl.queries, POT)
    e = t.expect(cl.queries, POT, rr_mode=rr_mode)
    assert np.max(np.abs(e - F) / np.abs(F)) < 1e-11


def test_lod2_sampled_mean_converges_to_brute_force(orc):
    cl = W.uniform_cube(400, 16, 8)
    t = orc.Tree(cl.sources, cl.weights, d=2, leaf_size=2)
    t.set_lod(2)
    F = orc.brute(cl.sources, cl.weights, None, cl.queries, POT)
    K = 3000
    acc = np.array([t.sbh(cl.queries, POT, seed=s, group=16)["F"] for s in range(K)])
    mean, se = acc.mean(0), acc.std(0, ddof=1) / np.sqrt(K)
    z = norm.isf(1e-3 / (2 * cl.queries.shape[0]))
    assert np.all(np.abs(mean - F) <= z * se + 1e-12 * np.abs(F)), np.max(np.abs(mean - F) / se)


def test_lod2_lowers_the_far_field_error(orc):
    cl = W.uniform_cube(4000, 1, 5)
    rng = np.random.Generator(np.random.PCG64(1))
    u = rng.normal(size=(1000, 3))
    q = (0.5 + 3.0 * u / np.linalg.norm(u, axis=1, keepdims=True)).astype(np.float32)
    t = orc.Tree(cl.sources, cl.weights, d=2, leaf_size=8)
    F = orc.brute(cl.sources, cl.weights, None, q, POT)
    med = {}
    for lod in (1, 2):
        t.set_lod(lod)
        med[lod] = np.median(np.abs(np.array([t.sbh(q, POT, seed=s, group=64)["F"] for s in range(4)]) - F) / F)
    assert med[2] < 0.2 * med[1], med


def test_lod2_and_compression_exclude_each_other(orc):
    cl = W.uniform_cube(300, 4, 1)
    t = orc.Tree(cl.sources, cl.weights, d=2, leaf_size=4)
    t.set_lod(2)
    with pytest.raises(ValueError):
        t.set_compressed(True)
    t.set_lod(1)
    t.set_compressed(True)
    with pytest.raises(ValueError):
        t.set_lod(2)
    with pytest.raises(ValueError):
        t.set_lod(3)
