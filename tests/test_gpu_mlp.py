"""GPU parity of the learned child proposal: MFMA network, training rows,
loss gradient, Adam training and the estimators that use it (learned and
score proposals).

Section 3.3 draws the path index uniformly; the learned proposal replaces
that draw by q_c > 0 (Theorem 1 still holds).  Tolerances:
  - counts, row locations and the valid mask: bit-exact;
  - features (relative log scores in [-1, 0]): 2e-6 absolute (float32 scores
    from float32 aggregates against float64);
  - targets: the residual |exact - LOD| of a child is a difference of nearly
    equal sums when the child is far away, and the GPU takes the child's
    aggregate from float32 storage (the oracle's is float64).  Rounding the
    oracle's aggregates to float32 on the CPU moves its targets on the cube
    case by 1.2e-5 (median), 3.6e-4 (99th percentile), 1.5e-3 (max); bars
    per row (largest slot error): median 5e-5, 99% of rows 1e-3, all 4e-3;
  - logits: both sides round weights, inputs and hidden values to binary16;
    the oracle sums each dot product exactly and rounds once, MFMA does not,
    so a pre-activation can differ by an ulp of float32 and then round to the
    neighbouring binary16 hidden value.  Bound per logit: 2^-9 times the
    magnitudes that such a flip can move (sum |W3| |h2| + sum |W3| |W2| |h1|),
    plus float32 rounding; 99% of rows within 1e-5 (1 + |z|);
  - gradient: deltas in binary16 (relative 2^-11 each): relative L2 error
    below 5e-3, loss to 1e-4;
  - estimator with the score proposal or an exactly representable network
    (logits that differ only by the float32 rounding of the features, about
    1e-6): values to the uniform estimator's bar; a query may take another
    child only where the oracle's smallest margin (roulette or selection,
    |u - sum q|) is below 1e-5.  A query makes about 40 selections with up to
    7 boundaries each, so such near-ties are more frequent than for the
    uniform estimator: at most 0.3% of queries may diverge;
  - with a general network: at most 1% of queries may take a different child
    where the margin is below 5e-3 (a logit flip as above).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2506_02219_amd as P
import workloads as W
from gpu_helpers import DEV, NEAR_TIE, T, build_both, check_sbh, compare_trees, fp64_reference, host

pytestmark = pytest.mark.gpu


def random_params(seed, scale=0.4):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, oracle.MLP_NPARAM).astype(np.float32)


def dyadic_constant_params(seed):
    """W1 = W2 = 0 and every other value a multiple of 2^-6 in [-1, 1]: the
    hidden values are binary16-exact and every logit is an exact float32 sum,
    so both sides see identical logits (constant over nodes and queries)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(oracle.MLP_NPARAM, np.float32)
    p[256:288] = rng.integers(-64, 65, 32) / 64.0           # b1 (inactive: W2 = 0)
    p[1312:1344] = rng.integers(0, 65, 32) / 64.0           # b2 >= 0: h2 = b2
    p[1344:1600] = rng.integers(-64, 65, 256) / 64.0        # W3
    p[1600:1608] = rng.integers(-64, 65, 8) / 64.0          # b3
    return p


def surface_cloud(m=6000, seed=31):
    pts, nrm, w, _ = W.star_surface(m, seed, level=5)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    q = rng.uniform(-1.3, 1.3, (2000, 3)).astype(np.float32)
    return pts.astype(np.float32), nrm.astype(np.float32), w.astype(np.float32), q


def logit_bound(prm, x, z):
    """2^-9 (sum |W3||h2| + sum |W3| |W2| |h1|) + 2^-20 (1 + |z|) per logit (float64 forward)."""
    W1 = prm[0:256].reshape(32, 8).astype(np.float64); b1 = prm[256:288].astype(np.float64)
    W2 = prm[288:1312].reshape(32, 32).astype(np.float64); b2 = prm[1312:1344].astype(np.float64)
    W3 = prm[1344:1600].reshape(8, 32).astype(np.float64)
    h1 = np.maximum(x.astype(np.float64) @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    a3 = np.abs(W3)
    return 2.0 ** -9 * (np.abs(h2) @ a3.T + (np.abs(h1) @ np.abs(W2).T) @ a3.T) + 2.0 ** -20 * (1 + np.abs(z))


@pytest.mark.parametrize("n", [1, 63, 1000 + 37])
@pytest.mark.parametrize("pseed,scale", [(11, 0.4), (12, 1.5)])
def test_forward_matches_oracle(n, pseed, scale):
    prm = random_params(pseed, scale)
    x = np.random.Generator(np.random.PCG64(n)).uniform(-1, 1, (n, 8)).astype(np.float32)
    zg = host(P.sbh_mlp_forward(T(prm), T(x)))
    zo = oracle.mlp_forward(prm, x, mode=1)
    err = np.abs(zg - zo)
    assert np.all(err <= logit_bound(prm, x, zo)), float(err.max())
    close = np.all(err <= 1e-5 * (1 + np.abs(zo)), axis=1)
    assert (~close).sum() <= max(1, 0.01 * n), (close.mean(), float(err.max()))


def test_forward_zero_and_dyadic_networks_are_exact():
    x = np.random.Generator(np.random.PCG64(3)).uniform(-1, 1, (500, 8)).astype(np.float32)
    for prm in (np.zeros(oracle.MLP_NPARAM, np.float32), dyadic_constant_params(4)):
        zg = host(P.sbh_mlp_forward(T(prm), T(x)))
        assert np.array_equal(zg.astype(np.float64), oracle.mlp_forward(prm, x, mode=1))


def _pairs_case(kind):
    if kind == "cube":
        cl = W.c1()
        return cl.sources, cl.weights, None, cl.queries[:48], P.POTENTIAL
    pts, nrm, w, q = surface_cloud()
    return pts, w, nrm, q[:48], P.WINDING


@pytest.mark.parametrize("kind", ["cube", "surface"])
def test_training_rows_match_oracle(kind):
    src, w, nrm, q, kernel = _pairs_case(kind)
    gt, ot = build_both(src, w, nrm)
    compare_trees(gt, ot)
    seed = 77
    X, Tg, Cn, where = P.sbh_mlp_pairs(gt, T(q), kernel, seed=seed)
    X, Tg, Cn, where = host(X), host(Tg), host(Cn), host(where)
    Xo, Tgo, Cno, valid = ot.training_set(q, kernel, seed=seed)
    assert np.array_equal(where[:, 0] >= 0, valid)
    nd = ot.mlp_pairs(q.shape[0], seed)
    node = nd.reshape(-1)[valid]
    assert np.array_equal(where[valid, 1], ot.begin[node])
    assert np.array_equal(where[valid, 2], ot.count[node])
    assert np.array_equal(where[valid, 3], ot.level[node])
    assert np.array_equal(Cn, Cno)
    assert np.all(np.abs(X - Xo) <= 2e-6), float(np.abs(X - Xo).max())
    assert np.all(X[valid] >= -1) and np.all(X[valid].max(axis=1) == 0)
    assert np.all(X[~valid] == 0) and np.all(Tg[~valid] == 0)
    terr = np.abs(Tg - Tgo).max(axis=1)[valid]
    assert np.all(terr <= 4e-3), float(terr.max())
    assert np.median(terr) <= 5e-5 and np.mean(terr <= 1e-3) >= 0.99, np.quantile(terr, [0.5, 0.99])
    assert valid.sum() > 8 * q.shape[0]


def test_training_rows_on_a_root_leaf_are_empty():
    src = np.random.Generator(np.random.PCG64(5)).uniform(0, 1, (6, 3)).astype(np.float32)
    gt = P.sbh_build(T(src), T(np.ones(6, np.float32)))
    X, Tg, Cn, where = P.sbh_mlp_pairs(gt, T(src), P.POTENTIAL, max_depth=3)
    assert np.all(host(where)[:, 0] == -1) and np.all(host(X) == 0) and np.all(host(Cn) == 0)


def _random_rows(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, (n, 8)).astype(np.float32)
    cnt = rng.integers(0, 20, (n, 8)).astype(np.float32) * (rng.random((n, 8)) < 0.7)
    cnt[:, 3] += 1
    tg = rng.random((n, 8)) * (cnt > 0)
    tg = (tg / tg.sum(1, keepdims=True)).astype(np.float32)
    return x, tg, cnt


@pytest.mark.parametrize("n", [1, 64, 4096 + 45])
def test_loss_gradient_matches_oracle(n):
    prm = random_params(21, 0.5)
    x, tg, cnt = _random_rows(n, 22)
    g = host(P.sbh_mlp_loss_grad(T(prm), T(x), T(tg), T(cnt)))
    loss, go = oracle.mlp_loss_grad(prm, x, tg, cnt, mode=1)
    assert g[1609] == n
    assert abs(g[1608] - loss) <= 1e-4 * abs(loss), (g[1608], loss)
    rel = np.linalg.norm(g[:1608] - go) / np.linalg.norm(go)
    assert rel < 5e-3, rel


def test_loss_gradient_ignores_rows_without_children():
    prm = random_params(23, 0.5)
    x, tg, cnt = _random_rows(300, 24)
    cnt[::3] = 0
    tg[::3] = 0
    g = host(P.sbh_mlp_loss_grad(T(prm), T(x), T(tg), T(cnt)))
    keep = np.ones(300, bool); keep[::3] = False
    loss, go = oracle.mlp_loss_grad(prm, x[keep], tg[keep], cnt[keep], mode=1)
    assert g[1609] == keep.sum()
    assert abs(g[1608] - loss) <= 1e-4 * abs(loss)
    assert np.linalg.norm(g[:1608] - go) / np.linalg.norm(go) < 5e-3


def test_one_adam_step_moves_each_parameter_by_lr():
    """First Adam step from zero moments: m_hat = g, v_hat = g^2, so the update is lr * g / (|g| + 1e-8)."""
    prm = random_params(25, 0.5)
    x, tg, cnt = _random_rows(2048, 26)
    _, go = oracle.mlp_loss_grad(prm, x, tg, cnt, mode=1)
    p = T(prm.copy()); st = torch.zeros(2 * P.MLP_NPARAM, device=DEV)
    losses = torch.zeros(1, device=DEV)
    lr = 1e-3
    P.sbh_mlp_train(p, st, T(x), T(tg), T(cnt), steps=1, batch_rows=4096, lr=lr, losses=losses)
    step = prm.astype(np.float64) - host(p)
    big = np.abs(go) > 2e-2 * np.abs(go).max()
    assert np.all(np.abs(step[big] - lr * np.sign(go[big])) <= 1e-3 * lr + 1e-7)
    assert np.all(np.abs(step) <= lr * (1 + 1e-3) + 1e-7)
    assert host(losses)[0] > 0


def test_training_lowers_the_loss_on_real_rows():
    src, w, nrm, q, kernel = _pairs_case("surface")
    gt = P.sbh_build(T(src), T(w), T(nrm))
    qq = np.random.Generator(np.random.PCG64(8)).uniform(-1.3, 1.3, (512, 3)).astype(np.float32)
    X, Tg, Cn, where = P.sbh_mlp_pairs(gt, T(qq), kernel, seed=9)
    keep = torch.nonzero(where[:, 0] >= 0).squeeze(1)
    perm = keep[torch.randperm(keep.numel(), generator=torch.Generator().manual_seed(0)).to(DEV)]
    X, Tg, Cn = X[perm].contiguous(), Tg[perm].contiguous(), Cn[perm].contiguous()
    p = torch.zeros(P.MLP_NPARAM, device=DEV)
    p[:256] = T(random_params(27, 0.3)[:256]); p[288:1312] = T(random_params(28, 0.15)[288:1312])
    st = torch.zeros(2 * P.MLP_NPARAM, device=DEV)
    before = float(host(P.sbh_mlp_loss_grad(p, X, Tg, Cn))[1608])
    losses = torch.zeros(300, device=DEV)
    P.sbh_mlp_train(p, st, X, Tg, Cn, steps=300, batch_rows=1024, lr=3e-3, losses=losses)
    after = float(host(P.sbh_mlp_loss_grad(p, X, Tg, Cn))[1608])
    # the start is the score proposal (zero output layer); training must improve on it
    print(dict(before=before, after=after))
    assert after < before - 1e-3, (before, after)
    assert np.all(np.isfinite(host(losses)))


@pytest.fixture(scope="module")
def trained_vs_score():
    """A network trained on rows from three surfaces, kept at the chunk with the lowest validation
    error on a fourth (the untrained network, which is the score proposal, included), and the median
    errors of the uniform path index, the score proposal and that network on a fifth."""
    import paper_2506_02219_amd.learned as L

    def surface_case(seed):
        pts, nrm, w, _ = W.star_surface(1 << 14, seed, level=5)
        q = np.random.Generator(np.random.PCG64(seed + 1000)).uniform(-1.3, 1.3, (2048, 3)).astype(np.float32)
        q[:, 2] *= 0.25   # a slab around the surface's equator
        gt = P.sbh_build(T(pts.astype(np.float32)), T(w.astype(np.float32)))
        ref = fp64_reference(pts.astype(np.float32), w.astype(np.float32), None, q, P.POTENTIAL)
        return gt, T(q), ref

    def med_err(gt, q, ref, proposal, params=None, seeds=(1, 2, 3)):
        errs = []
        for s in seeds:
            v = host(P.sbh_eval(gt, q, P.POTENTIAL, samples=1, seed=s, proposal=proposal, mlp=params))
            errs.append(np.median(np.abs(v - ref) / np.abs(ref)))
        return float(np.mean(errs))

    rows = []
    for seed in (61, 62, 63):
        gt, q, _ = surface_case(seed)
        rows.append(L.training_rows(gt, q, P.POTENTIAL, seed=seed))
    X = torch.cat([r[0] for r in rows]); Tg = torch.cat([r[1] for r in rows]); Cn = torch.cat([r[2] for r in rows])
    gv, qv, rv = surface_case(64)
    gh, qh, rh = surface_case(65)
    p0 = L.init_params(0)
    best, hist = L.train_selected(p0.clone(), X, Tg, Cn, steps=400, chunks=4, batch_rows=2048, lr=2e-3,
                                  validate=lambda prm: med_err(gv, qv, rv, 1, prm, seeds=(7,)))
    r = dict(hist=hist, best_validation=med_err(gv, qv, rv, 1, best, seeds=(7,)), uniform=med_err(gh, qh, rh, 0),
             score=med_err(gh, qh, rh, 2), trained=med_err(gh, qh, rh, 1, best))
    print(r)
    return r


def test_trained_network_selection_and_importance(trained_vs_score):
    """Model selection never returns a network that validates worse than the untrained one (the score
    proposal), and both importance proposals beat the uniform path index on a held-out surface."""
    r = trained_vs_score
    assert r["hist"][0][1] >= min(v for _, v in r["hist"])        # selection keeps the best
    assert r["best_validation"] <= r["hist"][0][1]                 # never worse than untrained
    assert r["score"] < r["uniform"] and r["trained"] < r["uniform"], r


@pytest.mark.xfail(reason="measured: training lowers the cross-entropy but not the estimator's error; on the "
                          "held-out surface the selected network is the score proposal or within a few per cent of "
                          "it (GPU: score 9.3e-3, trained 9.3e-3 to 9.6e-3; CPU study with a variance objective: "
                          "score 9.35e-3, cross-entropy 9.55e-3, variance 9.43e-3)", strict=False)
def test_trained_network_beats_the_score_proposal(trained_vs_score):
    """What the trained network gains over the method without it: a strictly lower held-out error than
    the score proposal it starts from."""
    r = trained_vs_score
    assert r["trained"] < 0.97 * r["score"], r


@pytest.mark.parametrize("samples,group", [(1, 1), (4, 1), (2, 7)])
def test_estimator_exact_network_strict_parity(samples, group):
    cl = W.c1()
    gt, ot = build_both(cl.sources, cl.weights)
    prm = dyadic_constant_params(41)
    print(check_sbh(gt, ot, cl.queries[:1500], P.POTENTIAL, samples=samples, seed=5, group=group, mlp=prm))


@pytest.mark.parametrize("kernel", [P.WINDING, P.SMOOTHDIST])
def test_estimator_exact_network_surface_kernels(kernel):
    pts, nrm, w, q = surface_cloud()
    gt, ot = build_both(pts, w, nrm)
    print(check_sbh(gt, ot, q[:1000], kernel, samples=2, seed=6, alpha=100.0, mlp=dyadic_constant_params(42)))


@pytest.mark.parametrize("rr_mode", [1, 2])
def test_estimator_exact_network_roulette_ablations(rr_mode):
    cl = W.c1()
    gt, ot = build_both(cl.sources, cl.weights)
    check_sbh(gt, ot, cl.queries[:800], P.POTENTIAL, samples=1, seed=7, rr_mode=rr_mode,
              mlp=dyadic_constant_params(43))


@pytest.mark.parametrize("kernel", [P.POTENTIAL, P.WINDING])
@pytest.mark.parametrize("samples,group", [(1, 1), (3, 5)])
def test_score_proposal_parity(kernel, samples, group):
    """Proposal 2 (no network) against the oracle's all-zero network."""
    if kernel == P.POTENTIAL:
        cl = W.c1()
        src, w, nrm, q = cl.sources, cl.weights, None, cl.queries[:2000]
    else:
        src, nrm, w, q = surface_cloud()
    gt, ot = build_both(src, w, nrm)
    print(check_sbh(gt, ot, q, kernel, samples=samples, seed=9, group=group, proposal=2, ))


@pytest.mark.parametrize("kind", ["cube", "surface"])
def test_estimator_general_network(kind):
    if kind == "cube":
        cl = W.c1()
        src, w, nrm, q, kernel = cl.sources, cl.weights, None, cl.queries[:1500], P.POTENTIAL
    else:
        src, nrm, w, q = surface_cloud()
        kernel = P.WINDING
        q = q[:1500]
    gt, ot = build_both(src, w, nrm)
    st = check_sbh(gt, ot, q, kernel, samples=2, seed=8, mlp=random_params(44, 1.0), near_tie=5e-3,
                   max_divergent=0.01)
    print(st)


def test_learned_estimator_is_unbiased_on_the_gpu():
    """Mean of many independent batches against the float64 brute-force sum (z-test)."""
    cl = W.uniform_cube(400, 16, 8)
    gt = P.sbh_build(T(cl.sources), T(cl.weights), leaf_size=4)
    F = host(P.sbh_brute(T(cl.sources), T(cl.weights), None, T(cl.queries), P.POTENTIAL, fp64=True))
    prm = T(random_params(45, 1.0))
    q = T(cl.queries)
    K = 4000
    acc = torch.stack([P.sbh_eval(gt, q, P.POTENTIAL, samples=1, seed=3, batch=b, mlp=prm) for b in range(K)])
    acc = host(acc).astype(np.float64)
    from scipy.stats import norm
    z = norm.isf(1e-3 / (2 * len(F)))
    se = acc.std(0, ddof=1) / math.sqrt(K)
    assert np.all(np.abs(acc.mean(0) - F) <= z * se + 1e-6 * np.abs(F))


def test_learned_root_leaf_is_exact_and_branching_four_is_refused():
    src = np.random.Generator(np.random.PCG64(9)).uniform(0, 1, (5, 3)).astype(np.float32)
    w = np.ones(5, np.float32)
    gt = P.sbh_build(T(src), T(w))
    q = np.random.Generator(np.random.PCG64(10)).uniform(-1, 2, (70, 3)).astype(np.float32)
    out = host(P.sbh_eval(gt, T(q), P.POTENTIAL, samples=2, mlp=T(random_params(46))))
    F = oracle.brute(src, w, None, q, P.POTENTIAL)
    assert np.all(np.abs(out - F) <= 1e-5 * np.abs(F))
    g4 = P.sbh_build(T(W.c1().sources), T(W.c1().weights), branching=4)
    with pytest.raises(P.SbhError) as e:
        P.sbh_eval(g4, T(q), P.POTENTIAL, samples=1, mlp=T(random_params(46)))
    assert "SBH_EUNSUPPORTED" in str(e.value)


# ----------------------------------------------------------------------------- tile-shared score proposal
def grid_rows(n, y0=-0.9, dy=0.2):
    """rows of 64 neighbouring pixels (a grid in its own order), n queries"""
    xs = (np.arange(64) + 0.5) * (3.0 / 1000) - 0.4
    rows = [np.stack([xs, np.full(64, y0 + dy * i), np.zeros(64)], 1) for i in range((n + 63) // 64)]
    return np.concatenate(rows)[:n].astype(np.float32)


@pytest.mark.parametrize("kernel", [P.POTENTIAL, P.WINDING, P.SMOOTHDIST])
@pytest.mark.parametrize("samples,group", [(1, 64), (2, 128)])
def test_tile_proposal_parity(kernel, samples, group):
    pts, nrm, w, _ = surface_cloud()
    q = grid_rows(1000)   # 15 full tiles and a ragged one
    gt, ot = build_both(pts, w, nrm)
    print(check_sbh(gt, ot, q, kernel, samples=samples, seed=11, group=group, alpha=100.0, proposal=3))


def test_tile_proposal_random_queries_and_roulette_modes():
    cl = W.c1()
    gt, ot = build_both(cl.sources, cl.weights)
    for rr in (0, 1, 2):
        check_sbh(gt, ot, cl.queries[:1300], P.POTENTIAL, samples=1, seed=12, group=64, rr_mode=rr, proposal=3)


def test_tile_proposal_argument_errors():
    cl = W.c1()
    gt = P.sbh_build(T(cl.sources), T(cl.weights))
    with pytest.raises(P.SbhError):
        P.sbh_eval(gt, T(cl.queries[:100]), P.POTENTIAL, samples=1, group=1, proposal=3)
    g4 = P.sbh_build(T(cl.sources), T(cl.weights), branching=4)
    with pytest.raises(P.SbhError):
        P.sbh_eval(g4, T(cl.queries[:100]), P.POTENTIAL, samples=1, group=64, proposal=3)


def test_non_finite_network_falls_back_to_the_score_proposal():
    cl = W.c1()
    gt = P.sbh_build(T(cl.sources), T(cl.weights))
    q = T(cl.queries[:700])
    bad = random_params(50, 1.0)
    bad[123] = np.nan
    bad[1500] = np.inf
    a = host(P.sbh_eval(gt, q, P.POTENTIAL, samples=2, seed=3, mlp=T(bad)))
    zero = host(P.sbh_eval(gt, q, P.POTENTIAL, samples=2, seed=3, mlp=T(np.zeros(P.MLP_NPARAM, np.float32))))
    assert np.all(np.isfinite(a))
    assert np.array_equal(a, zero)
