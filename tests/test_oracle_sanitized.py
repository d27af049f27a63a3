"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle is the parity authority, so a memory or undefined-behaviour bug in
it would corrupt every pin and parity test silently.  This test compiles
oracle/sbh_oracle.c with -fsanitize=address,undefined (every error fatal) and
drives each of its entry points on small inputs, through the same Python
wrapper the tests use, in a subprocess that preloads the ASan runtime:
brute force, trees of every branching factor and leaf size (duplicates and
a depth cap included), the export, Barnes-Hut, the estimator (every roulette
mode, several samples and stream groups, the network, score and tile
proposals, every diameter reading), the exact expectations, every-node
refinement, the Barnes-Hut-cut and voted estimators, compressed aggregates,
second-order terms, and the proposal network's functions."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
import sys
sys.path.insert(0, ROOT)
import numpy as np
import oracle
oracle._build.LIB = LIB
import workloads as W

rng = np.random.Generator(np.random.PCG64(7))
for kernel in (0, 1, 2):
    pts, nrm, w, _ = W.star_surface(300, 3, level=2)
    pts, nrm, w = pts.astype(np.float32), nrm.astype(np.float32), w.astype(np.float32)
    q = rng.uniform(-1.3, 1.3, (70, 3)).astype(np.float32)
    oracle.brute(pts, w, nrm, q, kernel)
    for d, leaf, lmax in ((2, 4, 0), (4, 2, 0), (8, 8, 0), (2, 1, 5)):
        t = oracle.Tree(pts, w, nrm, d=d, leaf_size=leaf, max_level=lmax)
        t.bh(q, kernel, 0.7, group=64)
        t.refine_all(q, kernel)
        for rr in (0, 1, 2):
            t.sbh(q, kernel, samples=2, seed=1, group=1, rr_mode=rr, paths=True, batch=3)
            t.expect(q[:8], kernel, rr_mode=rr)
        t.sbh(q, kernel, samples=1, seed=2, group=64, paths=True, index=np.arange(70) + 5)
        t.sbh_vote(q, kernel, samples=2, seed=3, group=64, paths=True)
        t.vote_expect(q[:10], kernel)
        t.sbh_cut(q, kernel, 0.6, samples=1, seed=4)
        t.sbh_cut(q[:8], kernel, 0.6, expect=True)
        if d == 2:
            prm = (rng.standard_normal(oracle.MLP_NPARAM) * 0.1).astype(np.float32)
            t.sbh(q, kernel, samples=1, seed=5, group=1, paths=True, params=prm)
            t.sbh(q, kernel, samples=1, seed=5, group=64, paths=True,
                  params=np.zeros(oracle.MLP_NPARAM, np.float32), tile_queries=q)
            t.expect(q[:6], kernel, params=prm)
            t.expect(q[:6], kernel, tiles=True)
            X, Tg, Cn, valid = t.training_set(q[:20], kernel, seed=6)
            oracle.mlp_forward(prm, X[valid][:50])
            oracle.mlp_loss_grad(prm, X[valid][:50], Tg[valid][:50], Cn[valid][:50])
            for mode in (1, 2):
                t.set_diam_mode(mode)
                t.sbh(q, kernel, samples=1, seed=7, group=64, paths=True)
            t.set_diam_mode(0)
        if kernel == 0:
            t.set_compressed(True)
            t.compressed()
            t.sbh(q, kernel, samples=2, seed=8, group=64, paths=True)
            t.expect(q[:6], kernel)
            t.set_compressed(False)
            t.set_lod(2)
            t.quad()
            t.node_term(0, q[0].astype(np.float64))
            t.sbh(q, kernel, samples=2, seed=9, group=64, paths=True)
            t.sbh_vote(q, kernel, samples=1, seed=9, group=64, paths=True)
            t.expect(q[:6], kernel)
            t.set_lod(1)
        t.export() if hasattr(t, "export") else None
    oracle.term_sens(kernel, np.array([0.1, 0.2, 0.3]), 1.5, np.array([0.0, 0.0, 1.0]), np.array([1.0, -1.0, 0.5]))
dup = np.repeat(rng.uniform(0, 1, (5, 3)), 40, axis=0).astype(np.float32)
td = oracle.Tree(dup, np.ones(200, np.float32), d=2, leaf_size=8)
td.sbh(dup[:64], 0, samples=1, seed=1, group=64, paths=True)
oracle.f16_round(0.1)
oracle.philox4x32_10(np.array([1, 2, 3, 4], np.uint32), np.array([5, 6], np.uint32))
print("sanitized oracle ok")
'''


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("the ASan runtime is not available")
    lib = str(tmp_path / "liboracle_sanitized.so")
    subprocess.run([gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-std=c99", "-ffp-contract=off", "-shared", "-fPIC", "-o", lib,
                    os.path.join(ROOT, "oracle", "sbh_oracle.c"), "-lm"], check=True)
    script = tmp_path / "drive.py"
    script.write_text(f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + DRIVER)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.returncode, r.stdout[-2000:],
                                                                    r.stderr[-4000:])
