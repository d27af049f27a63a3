"""Readings study on a setup shaped like the paper's mesh-dataset comparison
(Table 1; results section): which reading of the paper's wording changes the
ordering of the estimator and Barnes-Hut?

Setup: 2^15 area-uniform samples of a random star-shaped surface (the
stand-in for the paper's meshes), isotropically rescaled to fit [-1, 1]^3,
equal masses 1/M, the unsoftened 1/r potential, queries on a regular grid in
[-1, 1]^3; the estimator with one sample per subdomain on a tree of
per-dimension branching 4 (the paper's choice for its method), Barnes-Hut at
beta = 2 on branching 2 (the paper's choice for it), per query.  Errors are
absolute, against the float64 brute force.  Readings varied: |B| as the cell
diagonal (the one both sides of this repository implement), the cell side,
or the diagonal of the box of the node's own points (Section 3.1's
wording); leaves of 8 points (virtual children) or of one point (the
paper's assumption).  Also the roulette of Eq. (5) against none (p = 1,
Appendix C).

Oracle only (float64); run as a script: python oracle/readings_study.py [grid]"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle            # noqa: E402
import workloads as W    # noqa: E402

READINGS = [("cell diagonal", 0, 8), ("cell diagonal", 0, 1), ("cell side", 1, 8),
            ("box of the points", 2, 8), ("box of the points", 2, 1)]


def setup(m=1 << 15, grid=50, seed=77):
    pts, _, _, _ = W.star_surface(m, seed)
    c = (pts.max(0) + pts.min(0)) / 2
    s = (pts.max(0) - pts.min(0)).max() / 2
    src = ((pts - c) / s).astype(np.float32)
    w = np.full(m, 1.0 / m, np.float32)
    g = (np.arange(grid) + 0.5) / grid * 2 - 1
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    return src, w, q


def run(grid=50, threads=0):
    src, w, q = setup(grid=grid)
    ref = oracle.brute(src, w, None, q, oracle.POTENTIAL, eps=0.0, threads=threads)
    rows = []
    for name, mode, leaf in READINGS:
        t0 = time.time()
        t4 = oracle.Tree(src, w, d=4, leaf_size=leaf)
        t2 = oracle.Tree(src, w, d=2, leaf_size=leaf)
        t4.set_diam_mode(mode)
        t2.set_diam_mode(mode)
        row = dict(reading=name, leaf_size=leaf)
        for rr, key in ((0, "eq5"), (1, "p1")):
            F = t4.sbh(q, oracle.POTENTIAL, samples=1, seed=0, group=1, rr_mode=rr, eps=0.0, threads=threads)["F"]
            e = np.abs(F - ref)
            row[key] = (float(np.median(e)), float(np.mean(e)))
        F, _, _ = t2.bh(q, oracle.POTENTIAL, 2.0, group=1, eps=0.0, threads=threads)
        e = np.abs(F - ref)
        row["bh2"] = (float(np.median(e)), float(np.mean(e)))
        row["seconds"] = round(time.time() - t0, 1)
        rows.append(row)
        print(row, flush=True)
    return rows


if __name__ == "__main__":
    grid = int(sys.argv[1]) if len(sys.argv) > 1 else 50
    rows = run(grid)
    print("| |B| | leaf | estimator, Eq. (5): median / mean | estimator, p = 1 | Barnes-Hut beta = 2 |")
    print("|---|---|---|---|---|")
    for r in rows:
        f = lambda v: f"{v[0]:.2e} / {v[1]:.2e}"
        print(f"| {r['reading']} | {r['leaf_size']} | {f(r['eq5'])} | {f(r['p1'])} | {f(r['bh2'])} |")
