"""Can a trained proposal network beat the score proposal it starts from?  A
float64 CPU study on the oracle, independent of the GPU.

Rows (features, residual-share targets, child counts) from uniform paths on
three 2^14-sample star surfaces, queries in a slab around the equator; the
network 8 -> 32 -> 32 -> 8 (ReLU) with the score features added to the
logits (16 f) and the defensive mixture q = (7/8) softmax + (1/8) n_c / n_T,
as the library's learned proposal; trained with Adam (PyTorch CPU autograd)
on either
  - the soft cross-entropy -sum t log softmax(z) (what the GPU trains), or
  - the one-step variance objective sum_c t_c^2 / q_c (minimised, like the
    cross-entropy, by q proportional to the residual shares t);
kept at the checkpoint with the lowest validation error of the estimator on a
fourth surface and evaluated on a fifth, against the score proposal (the
untrained network).  Errors: median relative error of the oracle's
estimator with that proposal (S = 1, three seeds) against brute force.

Run: python oracle/learned_study.py"""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle            # noqa: E402
import workloads as W    # noqa: E402

LAM = oracle.MLP_LAMBDA


def case(seed, nq=2048):
    pts, _, w, _ = W.star_surface(1 << 14, seed, level=5)
    q = np.random.Generator(np.random.PCG64(seed + 1000)).uniform(-1.3, 1.3, (nq, 3)).astype(np.float32)
    q[:, 2] *= 0.25
    ot = oracle.Tree(pts.astype(np.float32), w.astype(np.float32))
    ref = oracle.brute(pts.astype(np.float32), w.astype(np.float32), None, q, oracle.POTENTIAL)
    return ot, q, ref


def median_error(ot, q, ref, params, seeds=(1, 2, 3)):
    e = [np.median(np.abs(ot.sbh(q, oracle.POTENTIAL, samples=1, seed=s, params=params)["F"] - ref) / np.abs(ref))
         for s in seeds]
    return float(np.mean(e))


def forward(p, X):
    W1 = p[0:256].view(32, 8); b1 = p[256:288]; W2 = p[288:1312].view(32, 32); b2 = p[1312:1344]
    W3 = p[1344:1600].view(8, 32); b3 = p[1600:1608]
    h1 = torch.relu(X @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    return h2 @ W3.T + b3 + 16 * X


def proposal(z, Cn):
    pi = torch.softmax(z.masked_fill(Cn <= 0, -1e30), 1)
    return (1 - LAM) * pi + LAM * Cn / Cn.sum(1, keepdim=True), pi


def loss_cross_entropy(p, X, Tg, Cn):
    _, pi = proposal(forward(p, X), Cn)
    return -(Tg * torch.log(pi.clamp_min(1e-300))).sum(1).mean()


def loss_variance(p, X, Tg, Cn):
    q, _ = proposal(forward(p, X), Cn)
    return ((Tg ** 2) / q.clamp_min(1e-300)).masked_fill(Cn <= 0, 0).sum(1).mean()


def init(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(oracle.MLP_NPARAM)
    p[0:256] = rng.uniform(-1, 1, 256) / np.sqrt(8.0)
    p[288:1312] = rng.uniform(-1, 1, 1024) / np.sqrt(32.0)
    return torch.tensor(p, requires_grad=True)


def run(steps=2000, batch=2048, lr=2e-3):
    torch.manual_seed(0)
    rows = []
    for seed in (61, 62, 63):
        ot, q, _ = case(seed)
        X, Tg, Cn, valid = ot.training_set(q, oracle.POTENTIAL, seed=seed)
        rows.append((X[valid], Tg[valid], Cn[valid]))
    X = torch.tensor(np.concatenate([r[0] for r in rows]), dtype=torch.float64)
    Tg = torch.tensor(np.concatenate([r[1] for r in rows]), dtype=torch.float64)
    Cn = torch.tensor(np.concatenate([r[2] for r in rows]), dtype=torch.float64)
    keep = Cn.sum(1) > 0
    X, Tg, Cn = X[keep], Tg[keep], Cn[keep]
    val, held = case(64), case(65)
    zero = np.zeros(oracle.MLP_NPARAM, np.float32)
    out = dict(rows=int(X.shape[0]), score=dict(validation=median_error(*val, zero), held_out=median_error(*held, zero)))
    for name, lf in (("cross_entropy", loss_cross_entropy), ("variance", loss_variance)):
        p = init(0)
        opt = torch.optim.Adam([p], lr=lr)
        best_v, best_p = median_error(*val, p.detach().numpy().astype(np.float32), seeds=(7,)), p.detach().clone()
        hist = []
        for step in range(1, steps + 1):
            idx = torch.randint(0, X.shape[0], (batch,))
            opt.zero_grad()
            lf(p, X[idx], Tg[idx], Cn[idx]).backward()
            opt.step()
            if step % 250 == 0:
                v = median_error(*val, p.detach().numpy().astype(np.float32), seeds=(7,))
                with torch.no_grad():
                    hist.append((step, float(lf(p, X, Tg, Cn)), v))
                if v < best_v:
                    best_v, best_p = v, p.detach().clone()
        out[name] = dict(history=hist, best_validation=best_v,
                         held_out=median_error(*held, best_p.numpy().astype(np.float32)))
        print(name, out[name], flush=True)
    return out


if __name__ == "__main__":
    r = run()
    print("score proposal:", r["score"])
    for k in ("cross_entropy", "variance"):
        print(f"{k}: best validation {r[k]['best_validation']:.4e}, held-out {r[k]['held_out']:.4e}")
