"""Pins for the oracle's learned-proposal parts (importance sampling of the path
index, which Section 3.3 leaves open).

- binary16 rounding: against NumPy's float16 conversion (an independent
  implementation of IEEE round-to-nearest-even);
- loss gradient: against central finite differences in float64;
- the child score m s^2 / (r^2 + s^2)^(3/2) behind the features: second
  moments recomputed from the points, and the score bounds the true residual
  of a far child (the quadrupole term of the 1/r multipole expansion about
  the centre of mass, whose dipole term vanishes);
- the exact expectation with ANY network still equals Eq. (1) (Theorem 1
  holds for every child distribution with q_c > 0), and the sampled mean
  with a random network converges to it;
- the zero network (proposal in proportion to the scores) lowers the
  estimator's variance on a surface against the uniform path index;
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


def test_mlp_zero_network_gives_bias_plus_skip_logits():
    prm = np.zeros(oracle.MLP_NPARAM, np.float32)
    prm[-8:] = np.arange(8) * 0.25
    x = np.random.Generator(np.random.PCG64(2)).uniform(-1, 1, (5, 8)).astype(np.float32)
    b = np.tile(np.arange(8, dtype=np.float32) * np.float32(0.25), (5, 1))
    assert np.array_equal(oracle.mlp_forward(prm, x, 1), (b + np.float32(16) * x).astype(np.float64))
    assert np.array_equal(oracle.mlp_forward(prm, x, 0), b.astype(np.float64) + 16.0 * x.astype(np.float64))


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


def test_second_moments_match_numpy():
    pts, nrm, w, t = _surface_tree()
    P = pts[t.perm].astype(np.float64); Wt = w[t.perm].astype(np.float64)
    for i in range(t.n_nodes):
        b, n = t.begin[i], t.count[i]
        com = (Wt[b:b + n, None] * P[b:b + n]).sum(0) / Wt[b:b + n].sum()
        s2 = (Wt[b:b + n] * ((P[b:b + n] - com) ** 2).sum(1)).sum() / Wt[b:b + n].sum()
        assert abs(t.spread2[i] - s2) <= 1e-12 * max(s2, 1e-300) + 1e-300


def _scores(t, T, q):
    """score of each child slot from the exported aggregates (nan for empty slots)"""
    sc = np.full(8, np.nan)
    for ch in range(t.first_child[T], t.first_child[T] + t.nchild[T]):
        r2 = np.sum((t.agg[ch, :3] - q) ** 2)
        s2 = t.spread2[ch]
        sc[t.digit[ch]] = t.agg[ch, 3] * s2 / (r2 + s2) ** 1.5
    return sc


def test_score_bounds_the_residual_of_far_children():
    """|sum_c f - f(LOD_c)| <= m s^2 / r^3 (1 + O(R/r)) for the 1/r kernel: the quadrupole
    term of the expansion about the centre of mass is at most m s^2 / r^3, and R/r < 1/8 keeps
    the higher orders under a 1.5 factor.  The bound is also not loose by orders of magnitude."""
    cl = W.uniform_cube(3000, 0, 17)
    t = oracle.Tree(cl.sources, cl.weights, d=2, leaf_size=8)
    P = cl.sources[t.perm].astype(np.float64); Wt = cl.weights[t.perm].astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(18))
    ratios = []
    for T in np.nonzero(t.internal)[0][:40]:
        for _ in range(3):
            q = t.agg[T, :3] + rng.normal(size=3) * 0 + rng.choice([-1, 1], 3) * rng.uniform(2, 6, 3)
            sc = _scores(t, T, q)
            for ch in range(t.first_child[T], t.first_child[T] + t.nchild[T]):
                b, n = t.begin[ch], t.count[ch]
                rad = np.sqrt(((P[b:b + n] - t.agg[ch, :3]) ** 2).sum(1)).max()
                r = np.sqrt(((t.agg[ch, :3] - q) ** 2).sum())
                if n < 2 or r < 8 * rad:
                    continue
                ex = np.sum(Wt[b:b + n] / np.sqrt(((P[b:b + n] - q) ** 2).sum(1) + 1e-6))
                lod = t.agg[ch, 3] / np.sqrt(r * r + 1e-6)
                res = abs(ex - lod)
                assert res <= 1.5 * sc[t.digit[ch]] + 1e-12 * lod
                ratios.append(res / sc[t.digit[ch]])
    assert len(ratios) > 100 and np.median(ratios) > 0.05


def test_features_are_relative_log_scores():
    pts, nrm, w, t = _surface_tree()
    q = np.random.Generator(np.random.PCG64(5)).uniform(-1.4, 1.4, (30, 3)).astype(np.float32)
    nodes = np.nonzero(t.internal)[0][:30]
    f = t.mlp_features(nodes, q)
    for i, T in enumerate(nodes):
        sc = _scores(t, T, q[i].astype(np.float64))
        ne = ~np.isnan(sc)
        want = np.full(8, -1.0)
        if np.nanmax(sc) > 0:
            with np.errstate(divide="ignore"):
                want[ne] = np.maximum(-1.0, np.log(sc[ne] / np.nanmax(sc)) / 16)
        assert np.allclose(f[i], want, rtol=0, atol=1e-12)
        assert f[i].max() == 0.0 or np.all(f[i] == -1.0)


def test_score_proposal_lowers_the_variance_on_a_surface():
    """The zero network samples in proportion to the scores: on a surface its per-query
    spread over seeds is clearly below the uniform path index's."""
    pts, nrm, w, _ = W.star_surface(4000, 33, level=4)
    t = oracle.Tree(pts.astype(np.float32), w.astype(np.float32), d=2, leaf_size=8)
    q = np.random.Generator(np.random.PCG64(34)).uniform(-1.4, 1.4, (60, 3)).astype(np.float32)
    F = oracle.brute(pts.astype(np.float32), w.astype(np.float32), None, q, POT)
    zero = np.zeros(oracle.MLP_NPARAM, np.float32)
    K = 300
    uni = np.array([t.sbh(q, POT, seed=500 + s)["F"] for s in range(K)])
    sco = np.array([t.sbh(q, POT, seed=500 + s, params=zero)["F"] for s in range(K)])
    ru = np.median(np.sqrt(np.mean((uni - F) ** 2, 0)) / F)
    rs = np.median(np.sqrt(np.mean((sco - F) ** 2, 0)) / F)
    assert rs < 0.85 * ru, (rs, ru)


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
    nd = t.mlp_pairs(20, seed=3)
    for j in range(20):
        for a in range(8):
            row = nd[j, a]
            row = row[row >= 0]
            assert len(row) >= 1 and t.level[row[0]] == 1 and t.digit[row[0]] == a
            assert np.all(t.parent[row[1:]] == row[:-1])           # a root-to-leaf chain
            assert np.all(t.internal[row])
    # different seeds give different paths
    nd2 = t.mlp_pairs(20, seed=4)
    assert not np.array_equal(nd, nd2)


# ----------------------------------------------------------------------------- tile-shared score proposal
def _tile_case():
    pts, nrm, w, _ = W.star_surface(3000, 41, level=3)
    pts, w = pts.astype(np.float32), w.astype(np.float32)
    t = oracle.Tree(pts, w, d=2, leaf_size=6)
    # rows of 64 neighbouring pixels (as consecutive queries of a grid) and a partial last tile
    xs = (np.arange(64) + 0.5) * (3.0 / 1000) - 0.6
    q = np.concatenate([np.stack([xs, np.full(64, y), np.zeros(64)], 1) for y in (-0.9, 0.1, 1.25)])[:170]
    return pts, w, t, q.astype(np.float32)


@pytest.mark.parametrize("rr_mode", [0, 2])
def test_tile_proposal_expectation_equals_brute_force(rr_mode):
    """Theorem 1 with the tile-shared proposal: q depends on the node and the tile only."""
    pts, w, t, q = _tile_case()
    F = oracle.brute(pts, w, None, q, POT)
    E = t.expect(q, POT, rr_mode=rr_mode, tiles=True)
    assert np.all(np.abs(E - F) / np.abs(F) < 1e-11)


def test_tile_of_one_query_is_that_querys_score_proposal():
    """A tile holding a single query proposes exactly that query's score proposal (the zero
    network), computed by another route (float32 features and the network's softmax)."""
    pts, w, t, q = _tile_case()
    zero = np.zeros(oracle.MLP_NPARAM, np.float32)
    for j in (0, 77, 169):
        a = t.sbh(q[j:j + 1], POT, samples=3, seed=5, paths=True, tile_queries=q[j:j + 1])
        b = t.sbh(q[j:j + 1], POT, samples=3, seed=5, paths=True, params=zero)
        assert np.array_equal(a["paths"], b["paths"]) or min(a["margin"][0], b["margin"][0]) < 1e-6
        assert abs(a["F"][0] - b["F"][0]) <= 1e-6 * abs(b["F"][0])


def test_tile_sampler_mean_converges_and_lowers_the_spread():
    pts, w, t, q = _tile_case()
    F = oracle.brute(pts, w, None, q, POT)
    K = 1500
    tile = np.array([t.sbh(q, POT, seed=900 + s, group=64, tile_queries=q)["F"] for s in range(K)])
    uni = np.array([t.sbh(q, POT, seed=900 + s, group=64)["F"] for s in range(K)])
    from scipy.stats import norm
    z = norm.isf(1e-3 / (2 * len(F)))
    se = tile.std(0, ddof=1) / math.sqrt(K)
    assert np.all(np.abs(tile.mean(0) - F) <= z * se)
    rt = np.median(np.sqrt(np.mean((tile - F) ** 2, 0)) / F)
    ru = np.median(np.sqrt(np.mean((uni - F) ** 2, 0)) / F)
    assert rt < 0.85 * ru, (rt, ru)
