"""CPU pins of the oracle's roulette voted over a tile (rr_mode 3: the 64
queries of a tile share their random stream, and with it the node sequence
and the variate u; here they also share p, the largest Eq. (5) probability
among them, and stop or continue together), independent of the GPU.

  - Theorem 1: the exact expectation under the voted roulette equals the
    float64 brute-force sum, every kernel, d in {2, 4}, a ragged last tile;
  - the sampled mean over many seeds is within a CLT bound of the sum;
  - a tile of one query is the per-query Eq. (5) estimator, bit for bit;
  - a tile's p is at least each of its queries' own Eq. (5) p: on the same
    streams no query accepts fewer steps than under Eq. (5) (a minimum in
    place of the maximum fails this);
  - every query of a tile has the same path records;
  - a query with a non-finite coordinate does not vote: the other queries of
    its tile get what the tile without it gives;
  - the vote lowers the error at nearly the same number of wavefront steps."""
import numpy as np
import pytest
from scipy.stats import norm

import workloads as W

POT, WIND, SMOOTH = 0, 1, 2


def _cloud(kernel, m=500, n=100, seed=3):
    if kernel == POT:
        cl = W.uniform_cube(m, n, seed)
        return cl.sources, cl.weights, None, cl.queries
    pts, nrm, w, _ = W.star_surface(m, seed, level=3)
    q = np.random.Generator(np.random.PCG64(seed)).uniform(-1.4, 1.4, (n, 3)).astype(np.float32)
    return pts.astype(np.float32), w.astype(np.float32), nrm.astype(np.float32), q


@pytest.mark.parametrize("d", [2, 4])
@pytest.mark.parametrize("kernel", [POT, WIND, SMOOTH])
def test_vote_expectation_equals_brute_force(orc, d, kernel):
    src, w, nrm, q = _cloud(kernel)   # 100 queries: a tile of 64 and one of 36
    t = orc.Tree(src, w, nrm, d=d, leaf_size=4)
    F = orc.brute(src, w, nrm, q, kernel, alpha=20.0)
    e = t.vote_expect(q, kernel, alpha=20.0)
    scale = np.maximum(np.abs(F), 1.0 if kernel == WIND else 1e-300)
    assert np.max(np.abs(e - F) / scale) < 1e-11


def test_vote_sampled_mean_converges_to_brute_force(orc):
    cl = W.uniform_cube(400, 70, 8)
    t = orc.Tree(cl.sources, cl.weights, d=2, leaf_size=2)
    F = orc.brute(cl.sources, cl.weights, None, cl.queries, POT)
    K = 3000
    acc = np.array([t.sbh_vote(cl.queries, POT, seed=s, group=64)["F"] for s in range(K)])
    mean, se = acc.mean(0), acc.std(0, ddof=1) / np.sqrt(K)
    z = norm.isf(1e-3 / (2 * cl.queries.shape[0]))
    assert np.all(np.abs(mean - F) <= z * se + 1e-12 * np.abs(F)), np.max(np.abs(mean - F) / se)


def test_one_query_tiles_are_the_per_query_estimator(orc):
    cl = W.uniform_cube(3000, 200, 5)
    t = orc.Tree(cl.sources, cl.weights, d=2, leaf_size=8)
    idx = np.arange(200, dtype=np.int64) * 64   # every query alone in its tile
    for S in (1, 3):
        v = t.sbh_vote(cl.queries, POT, samples=S, seed=4, group=64, index=idx, paths=True)
        r = t.sbh(cl.queries, POT, samples=S, seed=4, group=64, index=idx, paths=True)
        assert np.array_equal(v["F"], r["F"])
        assert np.array_equal(v["paths"], r["paths"])


def test_vote_never_accepts_fewer_steps_than_eq5(orc):
    cl = W.uniform_cube(20000, 640, 6)
    t = orc.Tree(cl.sources, cl.weights, d=2, leaf_size=8)
    v = t.sbh_vote(cl.queries, POT, seed=2, group=64, paths=True)["paths"]
    r = t.sbh(cl.queries, POT, seed=2, group=64, paths=True)["paths"]
    present = v[..., 0] >= 0
    assert np.all(v[..., 2][present] >= r[..., 2][present])
    assert np.any(v[..., 2][present] > r[..., 2][present])
    # every query of a tile has its tile's records
    vt = v.reshape(10, 64, 8, 1, 4)
    assert np.all(vt == vt[:, :1])


def test_non_finite_queries_do_not_vote(orc):
    cl = W.uniform_cube(5000, 64, 7)
    t = orc.Tree(cl.sources, cl.weights, d=2, leaf_size=8)
    q = cl.queries.copy()
    q[17] = np.nan
    full = t.sbh_vote(q, POT, seed=9, group=64)["F"]
    keep = np.delete(np.arange(64), 17)
    sub = t.sbh_vote(cl.queries[keep], POT, seed=9, group=64, index=keep)["F"]
    assert np.isnan(full[17])
    assert np.array_equal(full[keep], sub)


def test_vote_lowers_the_error_at_nearly_the_same_wavefront_steps(orc):
    c5 = W.c5(m=1 << 16, res=128)
    qs, _ = W.shuffle_queries(c5.queries, 4242)
    q = qs[:64 * 40]
    t = orc.Tree(c5.sources, c5.weights, d=2, leaf_size=8)
    ref = orc.brute(c5.sources, c5.weights, None, q, POT)
    med, steps = {}, {}
    for mode in ("eq5", "vote"):
        errs, ws = [], []
        for seed in range(4):
            r = (t.sbh(q, POT, seed=seed, group=64, paths=True) if mode == "eq5"
                 else t.sbh_vote(q, POT, seed=seed, group=64, paths=True))
            errs.append(np.abs(r["F"] - ref) / np.abs(ref))
            p = r["paths"]
            att = np.where(p[..., 0] >= 0, p[..., 2] + (p[..., 3] == 0), 0).reshape(40, 64, 8)
            ws.append(att.max(axis=1).mean())
        med[mode], steps[mode] = np.median(np.concatenate(errs)), np.mean(ws)
    assert med["vote"] < 0.9 * med["eq5"], med
    assert steps["vote"] < 1.1 * steps["eq5"], steps
