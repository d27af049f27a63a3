"""Pins for the oracle's learned-proposal parts (importance sampling of the path
index, which Section 3.3 leaves open).

- binary16 rounding: against NumPy's float16 conversion (an independent
  implementation of IEEE round-to-nearest-even);
- loss gradient: against central finite differences in float64;
- an all-zero network reduces the proposal to the uniform path index, and the
  exact expectation with ANY network still equals Eq. (1) (Theorem 1 holds
  for every child distribution with q_c > 0);
- the sampled mean with a random network converges to Eq. (1);
- training targets: recomputed by brute force with NumPy.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

POT, WIND = 0, 1


def random_params(seed, scale=0.4):
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.uniform(-scale, scale, oracle.MLP_NPARAM)).astype(np.float32)


def test_f16_round_matches_numpy_float16():
    rng = np.random.Generator(np.random.PCG64(1))
    xs = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-8, 5, 20000).astype(np.float32),
        np.array([0.0, -0.0, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 65504.0, 65519.99, 65520.0, -65520.0,
                  2.0 ** -25, 3 * 2.0 ** -25, 2.0 ** -24, 6.1e-5, 2.0 ** -14 - 2.0 ** -26], np.float32)])
    ours = np.array([oracle.f16_round(float(x)) for x in xs])
    ref = xs.astype(np.float16).astype(np.float64)
    assert np.array_equal(ours, ref) or np.all((ours == ref) | (np.isnan(ours) & np.isnan(ref)))


def test_mlp_zero_network_gives_bias_logits():
    prm = np.zeros(oracle.MLP_NPARAM, np.float32)
    prm[-8:] = np.arange(8) * 0.25
    x = np.random.Generator(np.random.PCG64(2)).uniform(-1, 1, (5, 8)).astype(np.float32)
    for mode in (0, 1):
        assert np.array_equal(oracle.mlp_forward(prm, x, mode), np.tile(np.arange(8) * 0.25, (5, 1)))


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.Generator(np.random.PCG64(3))
    prm = random_params(4)
    n = 40
    x = rng.uniform(-1, 1, (n, 8)).astype(np.float32)
    cnt = rng.integers(0, 20, (n, 8)).astype(np.float32)
    cnt[:, 0] += 1
    tgt = rng.random((n, 8)) * (cnt > 0)
    tgt = (tgt / tgt.sum(1, keepdims=True)).astype(np.float32)
    loss, g = oracle.mlp_loss_grad(prm, x, tgt, cnt, mode=0)
    h = 2.0 ** -16   # exact perturbation of |p| < 0.5 in float32; small enough to miss ReLU kinks
    idx = rng.choice(oracle.MLP_NPARAM, 300, replace=False)
    fd = []
    for i in idx:
        p1 = prm.copy(); p1[i] += h
        p0 = prm.copy(); p0[i] -= h
        fd.append((oracle.mlp_loss_grad(p1, x, tgt, cnt, 0)[0] - oracle.mlp_loss_grad(p0, x, tgt, cnt, 0)[0]) / (2 * h))
    fd = np.array(fd)
    rel = np.linalg.norm(fd - g[idx]) / np.linalg.norm(g[idx])
    assert rel < 1e-5, rel
    assert loss > 0


def _surface_tree(m=180, seed=21, d=2, leaf=3):
    pts, nrm, w, _ = W.star_surface(m, seed, level=2)
    pts, nrm, w = pts.astype(np.float32), nrm.astype(np.float32), w.astype(np.float32)
    return pts, nrm, w, oracle.Tree(pts, w, nrm, d=d, leaf_size=leaf)


def test_zero_network_is_the_uniform_proposal():
    pts, nrm, w, t = _surface_tree()
    q = np.random.Generator(np.random.PCG64(5)).uniform(-1.4, 1.4, (25, 3)).astype(np.float32)
    zero = np.zeros(oracle.MLP_NPARAM, np.float32)
    for kernel in (POT, WIND):
        a = t.expect(q, kernel)
        b = t.expect(q, kernel, params=zero)
        assert np.allclose(a, b, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kernel", [POT, WIND])
@pytest.mark.parametrize("rr_mode", [0, 2])
def test_learned_proposal_expectation_equals_brute_force(kernel, rr_mode):
    pts, nrm, w, t = _surface_tree()
    q = np.random.Generator(np.random.PCG64(6)).uniform(-1.4, 1.4, (25, 3)).astype(np.float32)
    F = oracle.brute(pts, w, nrm, q, kernel)
    for seed in (7, 8):
        E = t.expect(q, kernel, rr_mode=rr_mode, params=random_params(seed, 1.0))
        scale = np.maximum(np.abs(F), 1e-3 * np.abs(F).max())
        assert np.all(np.abs(E - F) / scale < 1e-11)


def test_learned_sampler_mean_converges():
    cl = W.uniform_cube(400, 12, 8)
    t = oracle.Tree(cl.sources, cl.weights, d=2, leaf_size=4)
    F = oracle.brute(cl.sources, cl.weights, None, cl.queries, POT)
    prm = random_params(9, 1.0)
    K = 3000
    acc = np.array([t.sbh(cl.queries, POT, seed=100 + s, params=prm)["F"] for s in range(K)])
    from scipy.stats import norm
    z = norm.isf(1e-3 / (2 * len(F)))
    se = acc.std(0, ddof=1) / math.sqrt(K)
    assert np.all(np.abs(acc.mean(0) - F) <= z * se)
    # the learned proposal really changes the paths
    plain = t.sbh(cl.queries, POT, seed=100, paths=True)["paths"]
    learned = t.sbh(cl.queries, POT, seed=100, params=prm, paths=True)["paths"]
    assert not np.array_equal(plain, learned)


def test_child_targets_match_numpy_brute_force():
    cl = W.c1()
    t = oracle.Tree(cl.sources, cl.weights, d=2, leaf_size=8)
    internal = np.nonzero(t.internal)[0][:12]
    q = cl.queries[:12]
    tg, cn = t.child_targets(internal, q, POT)
    P = cl.sources[t.perm].astype(np.float64); Wt = cl.weights[t.perm].astype(np.float64)
    for i, T in enumerate(internal):
        r = np.zeros(8)
        for ch in range(t.first_child[T], t.first_child[T] + t.nchild[T]):
            b, n = t.begin[ch], t.count[ch]
            qq = q[i].astype(np.float64)
            exact = np.sum(Wt[b:b + n] / np.sqrt(np.sum((P[b:b + n] - qq) ** 2, 1) + 1e-6))
            lod = t.agg[ch, 3] / math.sqrt(np.sum((t.agg[ch, :3] - qq) ** 2) + 1e-6)
            r[t.digit[ch]] = abs(exact - lod)
            assert cn[i, t.digit[ch]] == n
        assert np.allclose(tg[i], r / r.sum(), rtol=1e-5, atol=1e-7)


def test_training_pairs_follow_uniform_paths():
    cl = W.c1()
    t = oracle.Tree(cl.sources, cl.weights)
    nd, na = t.mlp_pairs(20, seed=3)
    for j in range(20):
        for a in range(8):
            row = nd[j, a]
            row = row[row >= 0]
            assert len(row) >= 1 and t.level[row[0]] == 1 and t.digit[row[0]] == a
            assert np.all(t.parent[row[1:]] == row[:-1])           # a root-to-leaf chain
            assert np.all(t.internal[row])
            assert np.all(na[j, a][: len(row)] == t.count[row[0]])
    # different seeds give different paths
    nd2, _ = t.mlp_pairs(20, seed=4)
    assert not np.array_equal(nd, nd2)
