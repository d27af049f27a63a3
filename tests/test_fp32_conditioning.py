"""What float32 can reach: the estimator evaluated with every operation
rounded to float32 (NumPy float32 arithmetic, correctly rounded), on the
oracle's own paths and with the oracle's aggregates rounded once to float32
(the storage the GPU tree uses), against the float64 oracle.

This pins the parity bar of the GPU tests from both sides, independently of
the GPU: the float32 error bound 2^-24 (C_EVAL absum + C_AGG sens) that the
parity tests allow must cover every error of this evaluation, and the bound
is needed at all (the 1e-4 relative bar alone is not reachable in float32)
where this evaluation misses 1e-4 too - which happens for a share of the
smooth-distance queries well above 1e-5 (sums that cancel below their
float32 rounding bound, whose sign float32 cannot determine), and for no
potential query of the plane workload.

The estimator is Algorithm 2 with Eqs. (5)-(7); each path's nodes are the
ancestors of the end node the oracle records, so the emulation follows the
same path.  Its roulette products are taken in float64 (a path decision,
not an error term)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import C_EVAL, C_AGG, U32

F32 = np.float32
ALPHA = 100.0


def _term(kernel, p, w, dp, q, r0, wbar):
    d = (p - q).astype(F32)
    r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]).astype(F32)
    if kernel == oracle.POTENTIAL:
        return (w / np.sqrt((r2 + F32(1e-6)).astype(F32))).astype(F32)
    if kernel == oracle.SMOOTHDIST:
        r = np.sqrt(r2).astype(F32)
        return ((w / wbar).astype(F32) * np.exp((F32(-ALPHA) * (r - r0)).astype(F32))).astype(F32)
    num = (dp[..., 0] * d[..., 0] + dp[..., 1] * d[..., 1] + dp[..., 2] * d[..., 2]).astype(F32)
    den = (F32(4 * math.pi) * r2 * np.sqrt(r2)).astype(F32)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(r2 > 0, (num / den).astype(F32), F32(0)).astype(F32)


def emulate_f32(cl, ot, q, rec, kernel, samples, r0=None):
    """Float32 estimates of queries q along the path records rec [n, 8, S, 4] of the oracle."""
    key = ot.level.astype(np.int64) * (1 << 32) + ot.begin
    order = np.argsort(key)
    ks = key[order]
    com64 = ot.agg[:, 0:3]
    com, m, dip = com64.astype(F32), ot.agg[:, 3].astype(F32), ot.agg[:, 4:7].astype(F32)
    pts, pw = cl.sources[ot.perm].astype(F32), cl.weights[ot.perm].astype(F32)
    pdp = None if cl.normals is None else (cl.normals[ot.perm].astype(np.float64) *
                                           cl.weights[ot.perm][:, None]).astype(F32)
    diam = math.sqrt(3.0) * float(ot.side) / 2.0 ** np.arange(64)
    wbar = F32(np.mean(cl.weights.astype(np.float64)))
    internal = ot.internal
    out = np.zeros(len(q))
    for j in range(len(q)):
        qq = q[j].astype(F32)
        shift = F32(0) if r0 is None else F32(r0[j])
        t = lambda p, w, dp: _term(kernel, p, w, dp, qq, shift, wbar)
        acc = F32(0)
        for slot in range(8):
            if rec[j, slot, 0, 0] < 0:
                continue
            Fa = F32(0)
            for s in range(samples):
                eb, el, _, flag = (int(v) for v in rec[j, slot, s])
                if flag == 2:   # moved onto a point of a leaf: the path ends at that leaf
                    end = order[np.searchsorted(ks, (el - 1) * (1 << 32) + eb, side="right") - 1]
                else:
                    end = order[np.searchsorted(ks, el * (1 << 32) + eb)]
                chain = [end]
                while ot.level[chain[-1]] > 1:
                    chain.append(ot.parent[chain[-1]])
                chain = chain[::-1]
                a = chain[0]
                tT = t(com[a], m[a], dip[a])
                psel, prr = 1.0, 1.0
                for k, T in enumerate(chain if flag == 2 else chain[:-1]):
                    if k + 1 < len(chain):
                        c = chain[k + 1]
                        bc, nc = np.linalg.norm(com64[c] - q[j]) / diam[ot.level[T] + 1], ot.count[c]
                    else:
                        bc, nc = np.linalg.norm(cl.sources[ot.perm[eb]] - q[j]) / diam[ot.level[T] + 1], 1
                    bT = np.linalg.norm(com64[T] - q[j]) / diam[ot.level[T]]
                    prr *= 1.0 if bc == 0 else min(1.0, max(1.0, bT) / bc)      # Eq. (5)
                    if internal[T]:
                        ch = np.arange(ot.first_child[T], ot.first_child[T] + ot.nchild[T])
                        tc = t(com[ch], m[ch], dip[ch])
                        tnext = tc[int(np.nonzero(ch == chain[k + 1])[0][0])] if k + 1 < len(chain) else None
                    else:
                        sl = slice(ot.begin[T], ot.begin[T] + ot.count[T])
                        tc, tnext = t(pts[sl], pw[sl], None if pdp is None else pdp[sl]), None
                    delta = F32(tc.sum(dtype=F32) - tT)                            # Eq. (6)
                    Fa = F32(Fa + delta * F32(1.0 / (psel * prr)))                  # Eq. (7)
                    psel *= nc / ot.count[T]
                    tT = tnext
            acc = F32(acc + F32(t(com[a], m[a], dip[a]) + F32(Fa / F32(samples))))
        if kernel == oracle.SMOOTHDIST:
            with np.errstate(divide="ignore", invalid="ignore"):
                out[j] = float(shift) - (math.log(acc) if acc > 0 else math.nan) / ALPHA - math.log(float(wbar)) / ALPHA
        else:
            out[j] = float(acc)
    return out


def _compare(cl, kernel, n, group=64, samples=1, seed=17):
    ot = oracle.Tree(cl.sources, cl.weights, cl.normals, d=2, leaf_size=8)
    idx = np.sort(np.random.Generator(np.random.PCG64(seed)).choice(cl.n, n, replace=False))
    q = cl.queries[idx]
    r = ot.sbh(q, kernel, samples=samples, seed=0, group=group, paths=True, index=idx, alpha=ALPHA)
    r0 = None
    if kernel == oracle.SMOOTHDIST:
        # the shift of the float32 sum: a bit nearer than the nearest source (brute force in float64)
        d2 = np.full(n, np.inf)
        src = cl.sources.astype(np.float64)
        for i0 in range(0, n, 256):
            qq = q[i0:i0 + 256].astype(np.float64)
            d2[i0:i0 + 256] = np.min(((src[None, :, :] - qq[:, None, :]) ** 2).sum(-1), axis=1)
        r0 = np.maximum(np.sqrt(d2) - 30.0 / ALPHA, 0.0)
    v = emulate_f32(cl, ot, q, r["paths"], kernel, samples, r0)
    F = r["F"]
    dF = U32 * (C_EVAL * r["absum"] + C_AGG * r["sens"])
    with np.errstate(divide="ignore", invalid="ignore"):
        if kernel == oracle.SMOOTHDIST:
            ref = -np.log(F) / ALPHA
            rel = np.abs(v - ref) / np.maximum(np.abs(ref), 1.0 / ALPHA)
            over = np.abs(v - ref) * ALPHA * np.abs(F) / dF
            determined = np.abs(F) > dF
        else:
            ref = F
            rel = np.abs(v - ref) / (np.maximum(np.abs(ref), 1.0) if kernel == oracle.WINDING else np.abs(ref))
            over = np.abs(v - ref) / dF
            determined = np.ones(n, bool)
    both_nan = np.isnan(v) & np.isnan(ref)
    return np.where(both_nan, 0.0, rel), np.where(both_nan | ~determined, 0.0, over), determined


def test_float32_reaches_the_bar_on_the_potential_plane():
    """2^18 star-surface samples, the shuffled plane: every query within 1e-4 in float32, and the
    errors sit well inside the bound."""
    c = W.c5(m=1 << 18, res=200)
    qs, _ = W.shuffle_queries(c.queries, 4242)
    cl = W.Cloud(c.sources, c.weights, None, qs, c.kernel)
    rel, over, _ = _compare(cl, oracle.POTENTIAL, 1500)
    print("potential: max rel", rel.max(), "max err / bound", over.max())
    assert rel.max() <= 1e-4
    assert over.max() <= 1.0


def test_float32_misses_the_bar_on_some_smooth_distances_and_the_bound_covers_them():
    """30,000 samples of a star surface, box queries in [-1.5, 1.5]^3, alpha = 100, two samples per
    subdomain: a careful float32 evaluation misses 1e-4 on a share of queries above 1e-5 (one-sample
    sums that cancel to a small fraction of their terms); the float32 bound of the parity tests
    covers every error."""
    pts, nrm, w, _ = W.star_surface(30000, 9, level=4)
    q = np.random.Generator(np.random.PCG64(4)).uniform(-1.5, 1.5, (3000, 3))
    c = W.Cloud(pts.astype(np.float32), w.astype(np.float32), nrm.astype(np.float32), q.astype(np.float32),
                oracle.SMOOTHDIST)
    rel, over, det = _compare(c, oracle.SMOOTHDIST, 3000, samples=2)
    miss = int((~(rel <= 1e-4)).sum())
    print("smooth distance: queries above 1e-4:", miss, "of", len(rel), "sign not determined in float32:",
          int((~det).sum()), "max err / bound", over.max())
    # a share of at least 3/3000, far above 1e-5: mostly sums whose float32 rounding bound exceeds
    # their size (their sign, hence -log F, is not determined in float32)
    assert miss >= 3
    assert over.max() <= 1.0


def test_float32_bound_covers_the_winding_number():
    c = W.c2(m=1 << 16, res=120)
    rel, over, _ = _compare(c, oracle.WINDING, 1500)
    print("winding: max rel", rel.max(), "max err / bound", over.max())
    assert over.max() <= 1.0
