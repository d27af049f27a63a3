"""Pins of the oracle's per-query diagnostics, which set how the GPU parity
tests treat float32 conditioning and near-tie roulette decisions:

  - the centre sensitivity |grad_p f| |p| of a term, against central finite
    differences of the oracle's own term (exact for the potential and the
    smooth distance; for the winding number the oracle uses the bound
    4 |dip| / (4 pi r^3) of the gradient norm, which lies within [2, 4] times it);
  - the estimate, its absolute-term sum, its sensitivity sum, its smallest
    roulette margin and its path records, against an independent NumPy walk
    of Algorithm 2 / Eqs. (5)-(7) over the exported tree, driven by the same
    Philox4x32-10 counters (the generator itself is pinned by its published
    known-answer vectors in test_oracle_pins).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

KERNELS = (oracle.POTENTIAL, oracle.WINDING, oracle.SMOOTHDIST)


@pytest.mark.parametrize("kernel", KERNELS)
def test_sensitivity_against_finite_differences(kernel):
    rng = np.random.Generator(np.random.PCG64(404))
    for _ in range(200):
        p = rng.uniform(-1.5, 1.5, 3)
        q = p + rng.normal(size=3) * rng.choice([0.01, 0.1, 0.5])
        m = rng.uniform(0.2, 3.0)
        dip = rng.normal(size=3)
        f0, sens = oracle.term_sens(kernel, p, m, dip, q, eps=1e-3, alpha=20.0)
        r = np.linalg.norm(p - q)
        h = 1e-6 * r
        g = np.zeros(3)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            g[a] = (oracle.term_sens(kernel, p + e, m, dip, q, eps=1e-3, alpha=20.0)[0] -
                    oracle.term_sens(kernel, p - e, m, dip, q, eps=1e-3, alpha=20.0)[0]) / (2 * h)
        fd = np.linalg.norm(g) * np.linalg.norm(p)
        if kernel == oracle.WINDING:
            # bound of the gradient norm: between 2 and 4 times the finite-difference value
            assert 2.0 * (1 - 1e-5) * fd <= sens <= 4.0 * (1 + 1e-5) * fd, (sens, fd)
        else:
            assert abs(sens - fd) <= 1e-6 * fd, (sens, fd)


def _term(kernel, p, m, dip, q, eps, alpha):
    d = p - q
    r2 = float(d @ d)
    if kernel == oracle.POTENTIAL:
        return m / math.sqrt(r2 + eps * eps)
    if kernel == oracle.WINDING:
        return 0.0 if r2 == 0.0 else float(dip @ d) / (4 * math.pi * r2 * math.sqrt(r2))
    return m * math.exp(-alpha * math.sqrt(r2))


def _walk_all(ot, src, w, nrm, queries, kernel, S, seed, G, rr_mode, eps, alpha):
    """Algorithm 2 written out over the exported tree: subdomains are the root's
    children; at node T a Philox block (stream, slot S + s, k / 2, 0) gives the
    selection word (first of the step's pair) and the roulette variate (second,
    top 24 bits); the child holding offset floor(x n_T / 2^32) of T's sorted
    range is taken; Eq. (5) gives p (cell diagonals); the swap of Eq. (6) is
    weighted by n_a / (n_T prod p) (Eq. (7)).  Leaves with several points use
    their points as children of diameter |B_T| / d and end the path."""
    perm = ot.perm
    P = src[perm].astype(np.float64)
    Wt = w[perm].astype(np.float64)
    D = (w[perm, None].astype(np.float64) * nrm[perm].astype(np.float64)) if nrm is not None else np.zeros((len(w), 3))
    com, mass, dip = ot.agg[:, 0:3], ot.agg[:, 3], ot.agg[:, 4:7]
    diam = [math.sqrt(3.0) * float(ot.side) / ot.d ** l for l in range(ot.max_level + 2)]
    internal = ot.internal
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)

    def node_f(i, q):
        return _term(kernel, com[i], mass[i], dip[i], q, eps, alpha)

    def node_s(i, q):
        return oracle.term_sens(kernel, com[i], mass[i], dip[i], q, eps, alpha)[1]

    def pt_f(s, q):
        return _term(kernel, P[s], Wt[s], D[s], q, eps, alpha)

    def rr(bT, bc):
        if rr_mode == 1:
            return 1.0
        if rr_mode == 2:
            return 0.5
        if bc == 0.0:
            return 1.0
        return min(1.0, max(1.0, bT) / bc)

    def path(q, a, sigma, stream2):
        T, tT, psel, prr = a, node_f(a, q), 1.0, 1.0
        val = ab = sn = 0.0
        margin = math.inf
        rec = [0, 0, 0, 0]
        k = 0
        while True:
            nT = int(ot.count[T])
            rec[0], rec[1] = int(ot.begin[T]), int(ot.level[T])
            if nT == 1:
                rec[3] = 1
                break
            rnd = oracle.philox4x32_10([sigma, stream2, k >> 1, 0], key)
            xs, xr = int(rnd[2 * (k & 1)]), int(rnd[2 * (k & 1) + 1])
            u = (xr >> 8) / 2.0 ** 24
            target = int(ot.begin[T]) + ((xs * nT) >> 32)
            bT = np.linalg.norm(q - com[T]) / diam[ot.level[T]]
            dc = diam[ot.level[T] + 1]
            step_s = node_s(T, q)
            if internal[T]:
                kids = range(int(ot.first_child[T]), int(ot.first_child[T]) + int(ot.nchild[T]))
                vals = [node_f(c, q) for c in kids]
                step_s += sum(node_s(c, q) for c in kids)
                c = next(c for c in kids if ot.begin[c] <= target < ot.begin[c] + ot.count[c])
                qc = ot.count[c] / nT
                bc = np.linalg.norm(q - com[c]) / dc
                tc = node_f(c, q)
            else:
                vals = [pt_f(s, q) for s in range(int(ot.begin[T]), int(ot.begin[T]) + nT)]
                c = None
                qc = 1.0 / nT
                bc = np.linalg.norm(q - P[target]) / dc
                tc = None
            p = rr(bT, bc)
            if rr_mode == 0:
                margin = min(margin, abs(u - p))
            if u >= p:
                rec[3] = 0
                break
            prr *= p
            wgt = 1.0 / (psel * prr)
            val += (sum(vals) - tT) * wgt
            ab += (sum(abs(v) for v in vals) + abs(tT)) * wgt
            sn += step_s * wgt
            rec[2] += 1
            psel *= qc
            if c is None:
                rec[0], rec[1], rec[3] = target, int(ot.level[T]) + 1, 2
                break
            T, tT = c, tc
            k += 1
        return val, ab, sn, margin, rec

    n, d3 = queries.shape[0], ot.d ** 3
    F, A, SN, MG = np.zeros(n), np.zeros(n), np.zeros(n), np.full(n, math.inf)
    recs = np.zeros((n, d3, S, 4), np.int32)
    recs[:, :, :, 0] = -1
    root_kids = range(int(ot.first_child[0]), int(ot.first_child[0]) + int(ot.nchild[0]))
    for j in range(n):
        q = queries[j].astype(np.float64)
        sigma = j if G == 1 else j // G
        for a in root_kids:
            slot = int(ot.digit[a])
            cv = node_f(a, q)
            fa = aa = sa = 0.0
            for s in range(S):
                v, ab_, sn_, mg, rec = path(q, a, sigma, slot * S + s)
                fa += v; aa += ab_; sa += sn_
                MG[j] = min(MG[j], mg)
                recs[j, slot, s] = rec
            F[j] += cv + fa / S
            A[j] += abs(cv) + aa / S
            SN[j] += node_s(a, q) + sa / S
    return F, A, SN, MG, recs


@pytest.mark.parametrize("kernel,d,S,G,rr_mode", [(oracle.POTENTIAL, 2, 2, 1, 0), (oracle.WINDING, 2, 1, 8, 0),
                                                  (oracle.SMOOTHDIST, 2, 1, 1, 0), (oracle.POTENTIAL, 4, 1, 1, 0),
                                                  (oracle.POTENTIAL, 2, 1, 1, 1), (oracle.WINDING, 2, 2, 1, 2)])
def test_walk_diagnostics_against_numpy_walk(kernel, d, S, G, rr_mode):
    pts, nrm, w, _ = W.star_surface(600, 31, level=3)
    pts, nrm, w = pts.astype(np.float32), nrm.astype(np.float32), w.astype(np.float32)
    q = np.random.Generator(np.random.PCG64(8)).uniform(-1.3, 1.3, (24, 3)).astype(np.float32)
    ot = oracle.Tree(pts, w, nrm, d=d, leaf_size=4)
    seed = (3 << 32) + 11
    alpha = 5.0
    r = ot.sbh(q, kernel, samples=S, seed=seed, group=G, rr_mode=rr_mode, eps=1e-3, alpha=alpha, paths=True)
    F, A, SN, MG, recs = _walk_all(ot, pts, w, nrm, q, kernel, S, seed, G, rr_mode, 1e-3, alpha)
    assert np.array_equal(r["paths"], recs)
    assert (recs[..., 2] > 0).any()
    np.testing.assert_allclose(r["F"], F, rtol=1e-11, atol=1e-13 * np.abs(A).max())
    np.testing.assert_allclose(r["absum"], A, rtol=1e-11)
    np.testing.assert_allclose(r["sens"], SN, rtol=1e-11)
    if rr_mode == 0:
        np.testing.assert_allclose(r["margin"], MG, rtol=1e-9, atol=1e-15)
    else:
        assert np.all(np.isinf(r["margin"]))
