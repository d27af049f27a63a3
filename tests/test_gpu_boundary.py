"""The C-ABI boundary on the GPU: the allocator hook (a caller's allocator
gives the same tree; an injected failure at every allocation of a build is
reported as SBH_ENOMEM and leaks nothing), stream-ordered release, queries
with non-finite coordinates, and the smooth distance of queries far from
every source (the shifted float32 sum of the smooth-distance kernel)."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_2506_02219_amd as P
from gpu_helpers import DEV, T, host, build_both, compare_trees, check_sbh, value_errors

pytestmark = pytest.mark.gpu


class CountingAllocator:
    """PyTorch's caching allocator behind a counter; refuses the fail_at-th request (1-based)."""

    def __init__(self, fail_at=0):
        self.fail_at, self.calls, self.live = fail_at, 0, {}

    def alloc(self, nbytes, stream):
        self.calls += 1
        if self.calls == self.fail_at:
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, stream=stream or None)
        self.live[p] = nbytes
        return p

    def free(self, ptr, nbytes, stream):
        assert self.live.pop(ptr) == nbytes
        torch.cuda.caching_allocator_delete(ptr)


def _surface(m=20000, seed=3):
    pts, nrm, w, _ = W.star_surface(m, seed, level=4)
    return pts.astype(np.float32), nrm.astype(np.float32), w.astype(np.float32)


def test_caller_allocator_same_tree_and_every_failure_reported():
    src, nrm, w = _surface()
    ref = P.sbh_build(T(src), T(w), T(nrm))
    g_ref = ref.export()
    q = T(np.random.Generator(np.random.PCG64(2)).uniform(-1.5, 1.5, (5000, 3)).astype(np.float32))
    v_ref = host(P.sbh_eval(ref, q, P.WINDING, samples=1, seed=3, group=64))
    ca = CountingAllocator()
    P.sbh_set_allocator(ca.alloc, ca.free)
    try:
        t = P.sbh_build(T(src), T(w), T(nrm))
        n_calls = ca.calls
        assert n_calls >= 4 and len(ca.live) == 3   # the tree keeps its three slabs
        g = t.export()
        for k in g:
            assert np.array_equal(g[k], g_ref[k]), k
        assert np.array_equal(host(P.sbh_eval(t, q, P.WINDING, samples=1, seed=3, group=64)), v_ref)
        t.free_async()
        assert not ca.live
        # refuse each allocation of a build in turn
        for k in range(1, n_calls + 1):
            ca.fail_at, ca.calls = k, 0
            with pytest.raises(P.SbhError) as ei:
                P.sbh_build(T(src), T(w), T(nrm))
            assert ei.value.status.startswith("SBH_ENOMEM"), (k, str(ei.value))
            torch.cuda.synchronize()
            assert not ca.live, (k, ca.live)
        # the training workspace goes through the allocator too
        ca.fail_at, ca.calls = 1, 0
        prm = torch.zeros(P.MLP_NPARAM, device=DEV)
        x = torch.zeros((64, 8), device=DEV)
        with pytest.raises(P.SbhError):
            P.sbh_mlp_loss_grad(prm, x, x, x + 1)
        assert not ca.live
    finally:
        P.sbh_set_allocator()
    # a tree built before keeps working after the allocator changed
    assert np.array_equal(host(P.sbh_eval(ref, q, P.WINDING, samples=1, seed=3, group=64)), v_ref)
    ref.free()


def test_non_finite_queries_give_nan():
    c = W.c1()
    gt = P.sbh_build(T(c.sources), T(c.weights))
    q = c.queries[:200].copy()
    bad = np.array([3, 64, 65, 130, 199])
    q[bad[0], 0] = np.nan
    q[bad[1], 1] = np.inf
    q[bad[2], 2] = -np.inf
    q[bad[3]] = np.nan
    q[bad[4], 1] = np.nan
    good = np.setdiff1d(np.arange(200), bad)
    qt = T(q)
    for kernel in (P.POTENTIAL, P.SMOOTHDIST):
        for kw in (dict(samples=1, group=1), dict(samples=1, group=64), dict(samples=2, group=5),
                   dict(samples=0, beta=2.0)):
            v = host(P.sbh_eval(gt, qt, kernel, seed=1, **kw))
            qr = c.queries[:200].copy()
            if kw["samples"] == 0:
                # Barnes-Hut's cut is voted by the wavefront: a query without a value must not vote,
                # and a query far from every node (accepted at the root) does not either
                qr[bad] = 1e6
            ref = host(P.sbh_eval(gt, T(qr), kernel, seed=1, **kw))
            assert np.all(np.isnan(v[bad])), (kernel, kw)
            # the other queries of the same launch are untouched
            assert np.array_equal(v[good], ref[good]), (kernel, kw)
        vb = host(P.sbh_brute(T(c.sources), T(c.weights), None, qt, kernel))
        assert np.all(np.isnan(vb[bad])) and np.all(np.isfinite(vb[good]))


def _sphere(m, radius, seed=4):
    """Fibonacci points on a sphere of the given radius around (0.5, 0.5, 0.5), equal weights."""
    i = np.arange(m) + 0.5
    phi = np.arccos(1 - 2 * i / m)
    th = math.pi * (1 + 5 ** 0.5) * i
    p = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    return (0.5 + radius * p).astype(np.float32), np.full(m, 4 * math.pi * radius ** 2 / m, np.float32)


@pytest.mark.parametrize("G", [1, 64])
def test_smooth_distance_far_from_every_source(G):
    """alpha = 100 and queries inside a hollow sphere of radius 1: at the centre every source is at
    distance 1 and exp(-alpha r) = e^-100 is below float32's range.  The shifted sum stays finite;
    the values agree with the float64 oracle within the float32 conditioning of each estimate."""
    src, w = _sphere(30000, 1.0)
    gt, ot = build_both(src, w)
    rng = np.random.Generator(np.random.PCG64(6))
    q = (0.5 + rng.uniform(-0.6, 0.6, (640, 3))).astype(np.float32)
    q[0] = 0.5   # the centre
    out = host(P.sbh_eval(gt, T(q), P.SMOOTHDIST, samples=1, seed=2, group=G, alpha=100.0))
    r = ot.sbh(q, P.SMOOTHDIST, samples=1, seed=2, group=G, alpha=100.0)
    # no underflow: never +inf; the value is finite exactly where the estimated sum is positive (a
    # one-sample estimate of the sum can be negative, and then -log F / alpha is NaN on both sides),
    # except sums whose float32 sign is not determined
    assert not np.any(np.isinf(out))
    sure = np.abs(r["F"]) > 2.0 ** -24 * (64 * r["absum"] + 16 * r["sens"])
    assert np.array_equal(np.isfinite(out)[sure], (r["F"] > 0)[sure])
    assert np.isfinite(out[0]) and (r["F"] > 0).sum() > 0.8 * q.shape[0]
    ok, err, used = value_errors(out, r["F"], r["absum"], P.SMOOTHDIST, 100.0, r["sens"])
    assert ok.all(), (np.nonzero(~ok)[0][:5], float(np.nanmax(err)))
    # Barnes-Hut and brute force on the same queries
    bh = host(P.sbh_eval(gt, T(q), P.SMOOTHDIST, beta=2.0, samples=0, alpha=100.0))
    assert np.all(np.isfinite(bh))
    br = host(P.sbh_brute(T(src), T(w), None, T(q), P.SMOOTHDIST, alpha=100.0))
    ex = oracle.smooth_distance(oracle.brute(src, w, None, q, P.SMOOTHDIST, alpha=100.0))
    assert np.all(np.abs(br - ex) <= 1e-4 * np.maximum(np.abs(ex), 0.01))
