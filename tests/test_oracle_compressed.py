"""CPU pins of the oracle's compressed interior aggregates (the conclusion's
compressed level-of-detail representation; estimator of Section 3.3 and
Theorem 1 on top of it), independent of the GPU.

  - every stored code is a binary16 number;
  - every decoded centre of mass is within one binary16 rounding (in units of
    the node's cell side) of the exact one, and every decoded mass within one
    binary16 rounding (relative) of the exact one, at every depth: the offsets
    are taken from the decoded parent, so errors do not pile up down the tree;
  - the decoded values follow from the codes alone, top-down from the root's
    float32 aggregate;
  - Theorem 1 holds for any aggregate values: the exact expectation of the
    estimator on the compressed aggregates equals the float64 brute-force
    sum, every kernel and roulette mode (this fails if a one-point node
    stopped the walk with its inexact decoded term);
  - the sampled mean over many seeds is within a CLT bound of the sum, and no
    path stops at a one-point node (it takes the leaf step instead)."""
import numpy as np
import pytest
from scipy.stats import norm

import workloads as W

POT, WIND, SMOOTH = 0, 1, 2


def _cloud(kernel, m=600, n=40, seed=3):
    if kernel == POT:
        cl = W.uniform_cube(m, n, seed)
        return cl.sources, cl.weights, None, cl.queries
    pts, nrm, w, _ = W.star_surface(m, seed, level=3)
    q = np.random.Generator(np.random.PCG64(seed)).uniform(-1.4, 1.4, (n, 3)).astype(np.float32)
    return pts.astype(np.float32), w.astype(np.float32), nrm.astype(np.float32), q


def _clustered(m=3000, seed=11):
    """A deep tree: a tight Gaussian cluster inside a uniform cube (levels well past 10)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.0, 1.0, (m // 2, 3))
    b = 0.5 + 1e-4 * rng.standard_normal((m - m // 2, 3))
    src = np.concatenate([a, b]).astype(np.float32)
    w = rng.uniform(0.5, 2.0, m).astype(np.float32)
    return src, w


@pytest.mark.parametrize("d", [2, 4])
@pytest.mark.parametrize("which", ["uniform", "clustered"])
def test_codes_are_binary16_and_decode_within_one_rounding(orc, d, which):
    if which == "uniform":
        src, w, _, _ = _cloud(POT)
    else:
        src, w = _clustered()
    t = orc.Tree(src, w, d=d, leaf_size=4)
    qa, code = t.compressed()
    assert np.all(code[0] == 0)
    assert np.array_equal(code.astype(np.float16).astype(np.float32), code)
    com, mass = t.agg[:, :3], t.agg[:, 3]
    v = np.arange(1, t.n_nodes)
    par = t.parent[v]
    sl = float(t.side) / float(d) ** t.level[v].astype(np.float64)
    # one binary16 rounding of x = (com_v - com^q_P) / s_L: |error| <= 2^-11 |x| (normal), 2^-25 (subnormal)
    x = (com[v] - qa[par, :3]) / sl[:, None]
    slack = 1e-12 * (np.abs(com[v]) + float(t.side))   # the exact centre of mass summed in another order
    err = np.abs(qa[v, :3] - com[v])
    assert np.all(err <= sl[:, None] * np.maximum(2.0 ** -11 * np.abs(x), 2.0 ** -25) + slack)
    merr = np.abs(qa[v, 3] - mass[v])
    assert np.all(merr <= np.maximum(2.0 ** -11 * mass[v], 2.0 ** -25 * qa[par, 3]) + 1e-12 * mass[v])
    # the root: its float32 aggregate
    assert np.array_equal(qa[0, :3], com[0].astype(np.float32).astype(np.float64))
    if which == "clustered":
        assert t.depth * int(np.log2(d)) >= 12


def test_decoded_values_follow_from_the_codes(orc):
    src, w = _clustered(2000, seed=4)
    t = orc.Tree(src, w, d=2, leaf_size=4)
    qa, code = t.compressed()
    dec = np.zeros_like(qa)
    dec[0] = qa[0]
    for v in range(1, t.n_nodes):   # parents precede children
        P = t.parent[v]
        sl = float(t.side) / 2.0 ** int(t.level[v])
        dec[v, :3] = dec[P, :3] + code[v, :3].astype(np.float64) * sl
        dec[v, 3] = dec[P, 3] * float(code[v, 3])
    assert np.array_equal(dec, qa)


@pytest.mark.parametrize("d", [2, 4])
@pytest.mark.parametrize("rr_mode", [0, 1, 2])
@pytest.mark.parametrize("kernel", [POT, WIND, SMOOTH])
def test_compressed_expectation_equals_brute_force(orc, d, rr_mode, kernel):
    src, w, nrm, q = _cloud(kernel)
    t = orc.Tree(src, w, nrm, d=d, leaf_size=4)
    F = orc.brute(src, w, nrm, q, kernel, alpha=20.0)
    t.set_compressed(True)
    e = t.expect(q, kernel, rr_mode=rr_mode, alpha=20.0)
    t.set_compressed(False)
    scale = np.maximum(np.abs(F), 1.0 if kernel == WIND else 1e-300)
    assert np.max(np.abs(e - F) / scale) < 1e-11
    # the same holds on the exact aggregates, which the compressed ones differ from
    e0 = t.expect(q, kernel, rr_mode=rr_mode, alpha=20.0)
    assert np.max(np.abs(e0 - F) / scale) < 1e-11
    qa, _ = t.compressed()
    assert np.any(qa[1:, :3] != t.agg[1:, :3]) and np.any(qa[1:, 3] != t.agg[1:, 3])


def test_compressed_sampled_mean_converges_to_brute_force(orc):
    src, w, _, q = _cloud(POT, m=400, n=16, seed=8)
    t = orc.Tree(src, w, d=2, leaf_size=1)   # one-point leaves everywhere
    F = orc.brute(src, w, None, q, POT)
    t.set_compressed(True)
    K = 3000
    runs = [t.sbh(q, POT, seed=s, group=16, paths=True) for s in range(K)]
    t.set_compressed(False)
    acc = np.array([r["F"] for r in runs])
    mean, se = acc.mean(0), acc.std(0, ddof=1) / np.sqrt(K)
    z = norm.isf(1e-3 / (2 * q.shape[0]))
    assert np.all(np.abs(mean - F) <= z * se + 1e-12 * np.abs(F)), np.max(np.abs(mean - F) / se)
    flags = np.concatenate([r["paths"][..., 3].ravel() for r in runs])
    begins = np.concatenate([r["paths"][..., 0].ravel() for r in runs])
    assert not np.any(flags[begins >= 0] == 1)    # no one-point stop
    assert np.any(flags == 2)                      # leaf steps onto points do happen
    # without compression the same tree stops at one-point nodes
    r0 = t.sbh(q, POT, seed=0, group=16, paths=True)
    assert np.any(r0["paths"][..., 3] == 1)
