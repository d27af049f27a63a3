"""sbh_mlp_train_noalloc (the training entry point that allocates nothing and
uses the library's static device workspace) against sbh_mlp_train: same
parameters, Adam state and losses, bit for bit, on two calls in a row, the
second with fewer rows and a smaller batch than the first; sizes beyond the
workspace are refused."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_2506_02219_amd as P
from paper_2506_02219_amd import learned as L
from gpu_helpers import DEV, T

pytestmark = pytest.mark.gpu


def _rows():
    c = W.c1()
    tree = P.sbh_build(T(c.sources), T(c.weights))
    X, Tg, Cn = L.training_rows(tree, T(c.queries[:1024]), P.POTENTIAL, seed=3)
    tree.free()
    return X, Tg, Cn


def _train(fn, X, Tg, Cn, steps, batch_rows, step0, prm0, state0):
    prm, state = prm0.clone(), state0.clone()
    losses = torch.full((steps,), -1.0, device=DEV)
    fn(prm, state, X, Tg, Cn, steps, batch_rows=batch_rows, lr=2e-3, step0=step0, losses=losses)
    torch.cuda.synchronize()
    return prm.cpu().numpy(), state.cpu().numpy(), losses.cpu().numpy()


def test_noalloc_training_matches_the_allocating_call():
    X, Tg, Cn = _rows()
    n = X.shape[0]
    assert n > 5000, n
    prm0 = L.init_params(5)
    state0 = torch.zeros(2 * P.MLP_NPARAM, device=DEV)
    # first call: every row, batches up to the workspace's limit; second: a prefix of the rows, a
    # smaller batch, continuing from step 7 (the workspace still holds the first call's partials)
    cases = [(n, P.MLP_NOALLOC_MAX_BATCH_ROWS, 5, 0), (n // 3, 1000, 9, 7)]
    prm_a, state_a = prm0, state0
    for rows, batch, steps, step0 in cases:
        args = (X[:rows], Tg[:rows], Cn[:rows], steps, batch, step0)
        ref = _train(P.sbh_mlp_train, *args, prm_a, state_a)
        got = _train(P.sbh_mlp_train_noalloc, *args, prm_a, state_a)
        for a, b, what in zip(ref, got, ("params", "adam state", "losses")):
            assert np.array_equal(a, b), (rows, batch, what, float(np.abs(a - b).max()))
        assert np.all(np.isfinite(got[2])) and np.all(got[2] > 0)
        prm_a, state_a = torch.from_numpy(got[0]).to(DEV), torch.from_numpy(got[1]).to(DEV)


def test_noalloc_training_refuses_batches_beyond_the_workspace():
    prm = L.init_params(1)
    state = torch.zeros(2 * P.MLP_NPARAM, device=DEV)
    x = torch.zeros((64, 8), device=DEV)
    with pytest.raises(P.SbhError) as ei:
        P.sbh_mlp_train_noalloc(prm, state, x, x, x + 1, 1, batch_rows=P.MLP_NOALLOC_MAX_BATCH_ROWS + 1)
    assert ei.value.status.startswith("SBH_EINVAL")
    # nothing was written
    assert torch.equal(state, torch.zeros_like(state))
