"""Training of the learned child proposal on the GPU (sbh_mlp_* entry points).

Section 3.3 samples the path index uniformly; Theorem 1 only needs every
child to keep a positive probability, so the estimator stays unbiased under
any proposal that is divided out.  The network (8 features -> 32 -> 32 -> 8
logits, ReLU, plus 16 times the features) takes each child's relative log
quadrupole score and is trained to put the probability of each child in
proportion to the share of the node's refinement error (Eqs. (3)-(4)) that
the child carries: targets are the per-child residuals |sum over the child's
points - the child's aggregate term|, computed exactly on the GPU along
uniform paths.  The loss is the soft cross-entropy between those shares and
the softmax of the logits over the non-empty children; the optimiser is
Adam.  With a zero output layer the network is the score proposal.

Argument marshalling and row bookkeeping only: features, targets, forward,
backward and the Adam step all run in libsbh's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import MLP_NPARAM, sbh_mlp_loss_grad, sbh_mlp_pairs, sbh_mlp_train

OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 256, 288, 1312, 1344, 1600


def init_params(seed: int, device="cuda") -> torch.Tensor:
    """Uniform fan-in initialisation of the two hidden layers; output layer zero,
    so that the untrained network is exactly the score proposal (logits 16 f)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(MLP_NPARAM, np.float32)
    p[OFF_W1:OFF_B1] = rng.uniform(-1, 1, 256) / np.sqrt(8.0)
    p[OFF_W2:OFF_B2] = rng.uniform(-1, 1, 1024) / np.sqrt(32.0)
    return torch.from_numpy(p).to(device)


def training_rows(tree, queries: torch.Tensor, kernel: int, seed: int, max_depth=None, eps=1e-3, alpha=100.0):
    """Features, targets and child counts of every internal node on uniform paths
    from each subdomain of each query (rows past the end of a path removed)."""
    X, Tg, Cn, where = sbh_mlp_pairs(tree, queries, kernel, seed=seed, max_depth=max_depth, eps=eps, alpha=alpha)
    keep = torch.nonzero(where[:, 0] >= 0).squeeze(1)
    return X[keep], Tg[keep], Cn[keep]


def _shuffle(n: int, seed: int, index: int, device) -> torch.Tensor:
    """The row permutation of shuffle `index` of a training run: a function of (seed, index) only."""
    g = torch.Generator().manual_seed(int(seed) * 1000003 + int(index))
    return torch.randperm(n, generator=g).to(device)


def train(params: torch.Tensor, X: torch.Tensor, Tg: torch.Tensor, Cn: torch.Tensor, steps: int,
          batch_rows: int = 8192, lr: float = 2e-3, seed: int = 0, epochs_per_shuffle: int = 1, state=None,
          step0: int = 0):
    """`steps` Adam steps on `params` in place, the run's steps step0 .. step0 + steps - 1.  The rows
    are shuffled at the start of every `epochs_per_shuffle` epochs by a permutation that depends on
    (seed, shuffle index) only, and each step's batch on the step's index (sbh_mlp_train), so that a
    run continued from a checkpoint (params, Adam state and step0 saved by save_checkpoint) takes the
    same batches, and ends with the same parameters bit for bit, as one that was not interrupted.
    state: the Adam moments [2 * MLP_NPARAM] (None: zero, a fresh run).  Returns the per-step losses
    (device tensor) and the Adam state."""
    n = X.shape[0]
    if state is None:
        state = torch.zeros(2 * MLP_NPARAM, dtype=torch.float32, device=params.device)
    losses = torch.zeros(max(steps, 1), dtype=torch.float32, device=params.device)
    per = max(1, (n + batch_rows - 1) // batch_rows) * max(1, epochs_per_shuffle)   # steps per shuffle
    done, end = int(step0), int(step0) + int(steps)
    while done < end:
        e = done // per
        perm = _shuffle(n, seed, e, params.device)
        Xs, Ts, Cs = X[perm].contiguous(), Tg[perm].contiguous(), Cn[perm].contiguous()
        k = min(end, (e + 1) * per) - done
        sbh_mlp_train(params, state, Xs, Ts, Cs, steps=k, batch_rows=batch_rows, lr=lr, step0=done,
                      losses=losses[done - step0:done - step0 + k])
        done += k
    return losses[:steps], state


def save_checkpoint(path, params: torch.Tensor, state: torch.Tensor, step: int):
    """Parameters, Adam state and the number of steps taken, as a .npz of plain arrays (no pickles)."""
    np.savez(path, params=params.detach().cpu().numpy().astype(np.float32),
             adam_state=state.detach().cpu().numpy().astype(np.float32), step=np.int64(step))


def load_checkpoint(path, device="cuda"):
    """(params, Adam state, step) saved by save_checkpoint."""
    with np.load(path, allow_pickle=False) as z:
        p, st, k = z["params"], z["adam_state"], int(z["step"])
    if p.shape != (MLP_NPARAM,) or st.shape != (2 * MLP_NPARAM,):
        raise ValueError("not a checkpoint of the proposal network")
    return torch.from_numpy(p).to(device), torch.from_numpy(st).to(device), k


def train_selected(params: torch.Tensor, X, Tg, Cn, steps: int, validate, chunks: int = 8, batch_rows: int = 8192,
                   lr: float = 2e-3, seed: int = 0):
    """Train in `chunks` equal parts and keep the parameters with the lowest `validate(params)` (a
    validation error of the estimator), the untrained parameters included.  Returns (best params,
    history of (steps done, validation value))."""
    best = params.clone()
    best_v = validate(params)
    hist = [(0, best_v)]
    state = torch.zeros(2 * MLP_NPARAM, dtype=torch.float32, device=params.device)
    n = X.shape[0]
    gen = torch.Generator().manual_seed(seed)
    per = max(1, steps // max(chunks, 1))
    done = 0
    while done < steps:
        perm = torch.randperm(n, generator=gen).to(params.device)
        Xs, Ts, Cs = X[perm].contiguous(), Tg[perm].contiguous(), Cn[perm].contiguous()
        k = min(per, steps - done)
        sbh_mlp_train(params, state, Xs, Ts, Cs, steps=k, batch_rows=batch_rows, lr=lr, step0=done)
        done += k
        v = validate(params)
        hist.append((done, v))
        if v < best_v:
            best_v = v
            best = params.clone()
    return best, hist


def mean_loss(params, X, Tg, Cn) -> float:
    return float(sbh_mlp_loss_grad(params, X, Tg, Cn)[MLP_NPARAM].item())
