"""Batched evaluation (sbh_batch_*): many clouds of uneven size in one launch
per group, replayed from a HIP graph.

Bar: every cloud's output is bit-identical to its own sbh_eval call (same
seed, batch word and options), for the autotuned and for fixed launch
configurations, on every replay; one cloud is also compared with the oracle
directly (values to the estimator's bar, near-ties as in gpu_helpers).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_02219_amd as P
import workloads as W
from gpu_helpers import DEV, NEAR_TIE, T, host, value_errors

pytestmark = pytest.mark.gpu

SPECS = [  # (m, n, kernel, seed, branching): uneven sizes, every kernel, both branchings,
    (3000, 2500, 0, 11, 2),        # a root leaf and an empty query set
    (700, 64, 1, 12, 2),
    (5, 130, 0, 13, 2),
    (20000, 4097, 2, 14, 2),
    (1500, 0, 0, 15, 2),
    (9000, 1000, 1, 16, 4),
    (256, 63, 0, 17, 2),
    (40000, 9000, 0, 18, 2),
    (2500, 777, 2, 19, 4),
    (6000, 3001, 1, 20, 2),
]
ALPHA = 100.0


def make_batch(specs=SPECS):
    clouds, trees, qs = [], [], []
    for m, n, k, seed, d in specs:
        cl = W.c4_cloud(dict(index=seed, m=m, n=max(n, 1), kernel=k, seed=seed))
        q = cl.queries[:n]
        gt = P.sbh_build(T(cl.sources), T(cl.weights), None if cl.normals is None else T(cl.normals), branching=d)
        clouds.append(cl); trees.append(gt); qs.append(T(np.ascontiguousarray(q).reshape(-1, 3)))
    return clouds, trees, qs


def single(trees, qs, kernels, samples, seed, batch):
    return [host(P.sbh_eval(t, q, k, samples=samples, seed=seed, group=64, alpha=ALPHA, batch=batch))
            for t, q, k in zip(trees, qs, kernels)]


@pytest.mark.parametrize("config", [None, (1, 8, 0), (2, 4, 1), (2, 1, 0), (1, 3, 1)])
def test_batch_equals_single_calls(config):
    clouds, trees, qs = make_batch()
    kernels = [s[2] for s in SPECS]
    b = P.Batch(trees, qs, kernels, samples=2, alpha=ALPHA, config=config)
    print(b.config)
    for seed, bw in ((5, 0), (6, 3)):
        outs = [host(o) for o in b.launch(seed, bw)]
        ref = single(trees, qs, kernels, 2, seed, bw)
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert o.shape == r.shape
            assert np.array_equal(o, r, equal_nan=True), (i, np.abs(o - r).max() if o.size else 0)
    b.free()


def test_batch_with_wide_offsets_equals_single_calls(monkeypatch):
    """A plan made while 64-bit tree offsets are forced (see the parity tests) gives the
    values of the ordinary 32-bit single calls."""
    clouds, trees, qs = make_batch(SPECS[:8])
    kernels = [s[2] for s in SPECS[:8]]
    ref = single(trees, qs, kernels, 1, 9, 2)
    monkeypatch.setenv("SBH_FORCE_WIDE_OFFSETS", "1")
    b = P.Batch(trees, qs, kernels, samples=1, alpha=ALPHA, config=(2, 8, 1))
    outs = [host(o) for o in b.launch(9, 2)]
    for o, r in zip(outs, ref):
        assert np.array_equal(o, r, equal_nan=True)
    b.free()


def test_graph_replays_with_eager_work_between():
    clouds, trees, qs = make_batch(SPECS[:6])
    kernels = [s[2] for s in SPECS[:6]]
    b = P.Batch(trees, qs, kernels, samples=1, alpha=ALPHA, config=(2, 8, 1))
    junk = torch.zeros(1 << 20, device=DEV)
    for r in range(5):
        outs = [host(o) for o in b.launch(100 + r, r)]
        junk.add_(1.0)                       # eager work and a synchronisation between replays
        torch.cuda.synchronize()
        ref = single(trees, qs, kernels, 1, 100 + r, r)
        for o, e in zip(outs, ref):
            assert np.array_equal(o, e, equal_nan=True)
    b.free()


def test_batch_cloud_against_the_oracle():
    spec = (20000, 3000, 0, 21, 2)
    clouds, trees, qs = make_batch([spec, (3000, 2000, 1, 22, 2)])
    b = P.Batch(trees, qs, [0, 1], samples=1, alpha=ALPHA)
    outs = [host(o) for o in b.launch(9, 0)]
    for cl, o, k, d in ((clouds[0], outs[0], 0, 2), (clouds[1], outs[1], 1, 2)):
        n = o.shape[0]
        ot = oracle.Tree(cl.sources, cl.weights, cl.normals, d=d)
        r = ot.sbh(cl.queries[:n], k, samples=1, seed=9, group=64, alpha=ALPHA)
        ok, err, used = value_errors(o, r["F"], r["absum"], k, ALPHA, r["sens"])
        near = r["margin"] < NEAR_TIE
        assert np.all(ok | near), (np.nonzero(~ok & ~near)[0][:5], float(np.nanmax(err)))
        assert (~ok).sum() <= max(1, 1e-5 * n)
    b.free()


def test_batch_argument_errors():
    clouds, trees, qs = make_batch(SPECS[:2])
    with pytest.raises(P.SbhError):
        P.Batch(trees, qs, [0, 1], group=32)            # not a multiple of 64
    with pytest.raises(P.SbhError):
        P.Batch(trees, qs, [0, 1], config=(0, 8, 0))   # tile_waves not 1 or 2
    with pytest.raises(P.SbhError):
        P.Batch(trees, qs, [0, 1], config=(3, 8, 0))
    with pytest.raises(P.SbhError):
        P.Batch(trees, qs, [0, 1], config=(2, 9, 0))   # waves_per_simd > 8
    with pytest.raises(P.SbhError):
        P.Batch(trees[:1], qs[:1], [1])                 # winding on a tree without normals
