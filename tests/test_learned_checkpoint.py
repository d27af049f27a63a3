"""Checkpoint and resume of the proposal network's training
(paper_2506_02219_amd.learned): a checkpoint holds the parameters, the Adam
moments and the step count as plain arrays (.npz, loaded without pickles),
and a run continued from one takes the same batches as a run that was not
interrupted (shuffles depend on (seed, shuffle index), batches on the step
index), so both end with the same parameters bit for bit."""
import numpy as np
import pytest
import torch

import paper_2506_02219_amd as P
from paper_2506_02219_amd import learned as L


def test_checkpoint_round_trip_on_the_host(tmp_path):
    rng = np.random.Generator(np.random.PCG64(3))
    p = torch.from_numpy(rng.standard_normal(P.MLP_NPARAM).astype(np.float32))
    st = torch.from_numpy(rng.standard_normal(2 * P.MLP_NPARAM).astype(np.float32))
    path = tmp_path / "ckpt.npz"
    L.save_checkpoint(path, p, st, 1234)
    p2, st2, k = L.load_checkpoint(path, device="cpu")
    assert k == 1234 and torch.equal(p, p2) and torch.equal(st, st2)
    np.savez(tmp_path / "bad.npz", params=np.zeros(5, np.float32), adam_state=np.zeros(3, np.float32),
             step=np.int64(0))
    with pytest.raises(ValueError):
        L.load_checkpoint(tmp_path / "bad.npz", device="cpu")


def test_shuffles_depend_on_seed_and_index_only():
    a = L._shuffle(1000, 5, 3, "cpu")
    b = L._shuffle(1000, 5, 3, "cpu")
    c = L._shuffle(1000, 5, 4, "cpu")
    assert torch.equal(a, b) and not torch.equal(a, c)
    assert torch.equal(torch.sort(a).values, torch.arange(1000))


@pytest.mark.gpu
def test_resumed_training_equals_uninterrupted_training(tmp_path):
    import workloads as W
    dev = "cuda"
    pts, nrm, w, _ = W.star_surface(20000, 31, level=4)
    gt = P.sbh_build(torch.from_numpy(pts.astype(np.float32)).to(dev), torch.from_numpy(w.astype(np.float32)).to(dev))
    q = np.random.Generator(np.random.PCG64(8)).uniform(-1.3, 1.3, (512, 3)).astype(np.float32)
    X, Tg, Cn = L.training_rows(gt, torch.from_numpy(q).to(dev), P.POTENTIAL, seed=9)
    assert X.shape[0] > 3000
    p0 = L.init_params(4)
    # uninterrupted: 300 steps over several shuffles (batches of 1024 rows)
    pa = p0.clone()
    la, sa = L.train(pa, X, Tg, Cn, steps=300, batch_rows=1024, lr=3e-3, seed=7)
    # interrupted after 130 steps (mid-shuffle), saved, loaded, continued to 300
    pb = p0.clone()
    lb1, sb = L.train(pb, X, Tg, Cn, steps=130, batch_rows=1024, lr=3e-3, seed=7)
    L.save_checkpoint(tmp_path / "ckpt.npz", pb, sb, 130)
    del pb, sb
    pc, sc, k = L.load_checkpoint(tmp_path / "ckpt.npz", device=dev)
    lb2, sc = L.train(pc, X, Tg, Cn, steps=300 - k, batch_rows=1024, lr=3e-3, seed=7, state=sc, step0=k)
    torch.cuda.synchronize()
    assert torch.equal(pa, pc) and torch.equal(sa, sc)
    assert torch.equal(la, torch.cat([lb1, lb2]))
    assert float(la[-20:].mean()) < float(la[:20].mean())
