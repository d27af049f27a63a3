"""Benchmark: queries/s of the stochastic Barnes-Hut estimator at its own
median relative error, against deterministic Barnes-Hut at the same error,
on one MI355X.

Default workload: the learned-vs-plain potential workload, 2^22 area-weighted
samples of a random star-shaped surface (radius 1 + 0.15 g, g a random
spherical-harmonic field of degrees 1..6), softened potential (eps = 1e-3),
queries = the 1000 x 1000 pixel centres of the z=0 plane over [-1.5,1.5]^2,
S = 1 sample per subdomain, Philox seed 0.  --config c2 (winding numbers,
2^20 sources) and c3 (smooth distances, 2^22 sources) run the other
workloads.

A step is one evaluation of every query (sbh_eval) on a tree built once
before the timed region (the tree build is timed separately and reported as
build_ms).  The error of a method is the median over a fixed sample of
queries of |F - F_ref| / max(|F_ref|, floor) against float64 GPU brute force
(floor 1 for winding numbers, 1/alpha for smooth distances, 0 for the
potential).  Deterministic Barnes-Hut is swept over beta and its time at the
stochastic method's error is interpolated in log(time)-log(error).

Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    "c1": dict(gen="c1", kernel=0, samples=1, beta=2.0),
    "c2": dict(gen="c2", kernel=1, samples=1, beta=2.0),
    "c3": dict(gen="c3", kernel=2, samples=1, beta=2.0),
    "c5": dict(gen="c5", kernel=0, samples=1, beta=2.0),
}
BETAS = [0.2, 0.25, 0.3, 0.35, 0.4, 0.5, 0.6, 0.75, 1, 1.5, 2, 3, 4, 6, 8, 12, 16, 24, 32, 40]
S_SWEEP = [1, 2, 4, 8, 16, 32]
FP32_PEAK_TFLOPS = 157.3
# flops of one brute-force interaction: three differences, the squared distance (three products,
# two sums) and eps^2, the reciprocal square root, the weight and the sum (potential); the
# winding number adds r^-3 (two products) and the dot product with the dipole (five); the smooth
# distance has the distance, the exponent (two) and the rescaled sum (two) instead
BRUTE_FLOPS = {0: 12, 1: 17, 2: 14}
# float32 operations per kernel term: differences, squared distance, the
# kernel itself, the weight; transcendental calls counted as one operation
TERM_FLOPS = {0: 11, 1: 17, 2: 14}
# the roulette of one attempted step: offset and squared distance to the selected child (6), one
# reciprocal square root, the max, two products and the min of Eq. (5)
ROULETTE_FLOPS = 11
# the weight update of one accepted step: the swap's difference, p product, 1 / (n_T prod p) and
# the accumulation
STEP_FLOPS = 6
HBM_PEAK_GBS = 8000.0
# L2 of MI355X: 8 XCDs x 16 channels x 128 bytes per clock x 2.4 GHz (the per-query-stream walk's
# gathers are served from L2 and the Infinity Cache, not from HBM)
L2_PEAK_GBS = 8 * 16 * 128 * 2.4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # a few hundred steps: the GPU's clocks take some milliseconds of load to ramp up, and a step of
    # the headline is about 0.1 ms
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="c5", choices=sorted(CONFIGS))
    ap.add_argument("--branching", type=int, default=2, help="tree of the stochastic estimator")
    ap.add_argument("--bh-branching", type=int, default=2, help="tree of the Barnes-Hut comparator")
    ap.add_argument("--group", type=int, default=64, help="queries per shared random stream (64: one per wavefront)")
    ap.add_argument("--samples", type=int, default=None)
    ap.add_argument("--err-sample", type=int, default=16384)
    ap.add_argument("--no-bh", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-cloud batched evaluation")
    ap.add_argument("--no-grid", action="store_true", help="skip the estimator on the plane's original order")
    ap.add_argument("--no-cut", action="store_true", help="skip the Barnes-Hut-cut subdomains")
    ap.add_argument("--no-compressed", action="store_true", help="skip the compressed-aggregate walk")
    ap.add_argument("--no-lod2", action="store_true", help="skip the second-order (quadrupole) walk")
    ap.add_argument("--no-vote", action="store_true", help="skip the roulette voted over the wavefront")
    ap.add_argument("--no-brute", action="store_true", help="skip the float32 brute-force timing of every query")
    ap.add_argument("--train-seeds", type=int, default=16, help="training surfaces (seeds 5001...)")
    ap.add_argument("--train-queries", type=int, default=2048, help="training queries per surface")
    ap.add_argument("--train-steps", type=int, default=4000)
    ap.add_argument("--train-batch", type=int, default=8192)
    ap.add_argument("--train-lr", type=float, default=2e-3)
    ap.add_argument("--ablation", action="store_true",
                    help="only the roulette / branching ablation on c1-c3 (one JSON line of its own)")
    return ap.parse_args()


def _training_surface(seed):
    import workloads as W
    pts, _, w, _ = W.star_surface(1 << 22, seed)
    return np.ascontiguousarray(pts, np.float32), np.ascontiguousarray(w, np.float32)


def _batch_cloud(spec):
    import workloads as W
    cl = W.c4_cloud(spec)
    return cl.sources, cl.weights, cl.normals, cl.queries, int(spec["kernel"])


def batch_clouds():
    """The 64 clouds of the batched workload, generated in forked CPU workers."""
    import multiprocessing as mp
    import workloads as W
    specs = W.c4_specs()
    with mp.get_context("fork").Pool(max(1, min(16, os.cpu_count() or 1))) as pool:
        return pool.map(_batch_cloud, specs)


def training_surfaces(seeds):
    """The held-out training clouds, generated in forked CPU workers (before the GPU is touched)."""
    import multiprocessing as mp
    procs = max(1, min(len(seeds), 16, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(_training_surface, seeds)


def log_interp(xs, ys, x):
    """y at x on the piecewise log-log curve through (xs, ys) (xs in any order); None outside."""
    pts = sorted(zip(xs, ys))
    for (x0, y0), (x1, y1) in zip(pts, pts[1:]):
        if x0 <= x <= x1 and x0 > 0 and x1 > x0 and y0 > 0 and y1 > 0:
            f = (math.log(x) - math.log(x0)) / (math.log(x1) - math.log(x0))
            return math.exp(math.log(y0) + f * (math.log(y1) - math.log(y0)))
    return None


def rel_errors(v, ref, kernel, alpha=100.0):
    ref = np.asarray(ref, np.float64)
    v = np.asarray(v, np.float64)
    if kernel == 1:
        scale = np.maximum(np.abs(ref), 1.0)
    elif kernel == 2:
        scale = np.maximum(np.abs(ref), 1.0 / alpha)
    else:
        scale = np.abs(ref)
    e = np.abs(v - ref) / scale
    return np.where(np.isnan(e), np.inf, e)


def git_sha():
    """HEAD of the repository when it is a git checkout; on a copy without .git (the benchmark box),
    the revision the library was built from (written by the build, +dirty when its sources differed)."""
    import subprocess
    try:
        sha = subprocess.run(["git", "rev-parse", "HEAD"], cwd=ROOT, capture_output=True, text=True,
                             timeout=10).stdout.strip()
        if sha:
            return sha
    except Exception:
        pass
    try:
        with open(os.path.join(ROOT, "paper_2506_02219_amd", "_build", "source_revision.txt")) as f:
            return "built-from:" + f.read().strip()
    except OSError:
        return None


def csrc_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2506_02219_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


ABLATION_RR = {0: "eq5", 1: "p=1", 2: "p=1/2", 3: "eq5 voted over the wavefront"}


def ablation(args):
    """The paper's roulette study (Appendix C) and the branching factor (Section 3.3): the estimator
    with Eq. (5), with p = 1 (no roulette), with p = 1/2 and with Eq. (5) voted over each wavefront's
    64 queries, on trees of branching 2, 4 and 8, on the
    potential (c1), winding (c2, shuffled plane) and smooth-distance (c3) workloads; one sample per
    subdomain, G = 64 (the coherent walk).  Time per evaluation of every query (HIP events, median
    of rounds of K launches) and median relative error against float64 brute force on a fixed
    sample; accepted steps per path from the kernel's own path records."""
    import torch
    import workloads as W
    import paper_2506_02219_amd as P
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for name in ("c1", "c2", "c3"):
        cl = getattr(W, name)()
        kernel = CONFIGS[name]["kernel"]
        q_np = W.shuffle_queries(cl.queries, 4242)[0] if name == "c2" else cl.queries
        src = torch.from_numpy(cl.sources).to(dev)
        wts = torch.from_numpy(cl.weights).to(dev)
        nrm = None if cl.normals is None else torch.from_numpy(cl.normals).to(dev)
        qry = torch.from_numpy(q_np).to(dev)
        N = qry.shape[0]
        ns = min(N, 8192)
        sidx = np.sort(np.random.Generator(np.random.PCG64(99)).choice(N, size=ns, replace=False))
        sidx_t = torch.from_numpy(sidx).to(dev)
        ref = P.sbh_brute(src, wts, nrm, qry[sidx_t].contiguous(), kernel, fp64=True).cpu().numpy()
        out = torch.empty(N, dtype=torch.float32, device=dev)
        for d in (2, 4, 8):
            tree = P.sbh_build(src, wts, nrm, branching=d, leaf_size=8)
            for rr in (0, 1, 2, 3):
                def run(rr=rr):
                    P.sbh_eval(tree, qry, kernel, samples=1, seed=0, group=64, rr_mode=rr, out=out)
                for _ in range(2):
                    run()
                times = []
                for _ in range(5):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(args.steps):
                        run()
                    e1.record(stream)
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1) / args.steps)
                run()
                torch.cuda.synchronize()
                err = float(np.median(rel_errors(out[sidx_t].cpu().numpy(), ref, kernel)))
                paths = torch.empty((N, d ** 3, 1, 4), dtype=torch.int32, device=dev)
                P.sbh_eval(tree, qry, kernel, samples=1, seed=0, group=64, rr_mode=rr, out=out, paths=paths)
                rec = paths.view(-1, 4)
                acc_steps = float(rec[rec[:, 0] >= 0][:, 2].double().mean())   # on the GPU: d = 8 records are GBs
                del paths, rec
                rows.append(dict(workload=cl.name, kernel=["potential", "winding", "smoothdist"][kernel], queries=N,
                                 branching=d, roulette=ABLATION_RR[rr], ms=float(np.median(times)),
                                 median_rel_err=err, accepted_steps_per_path=acc_steps,
                                 # time x error^2: the cost of reaching a fixed error (variance ~ 1/S)
                                 work_at_unit_variance=float(np.median(times)) * err * err))
                print(f"[ablation] {cl.name} d={d} {ABLATION_RR[rr]}: {rows[-1]['ms']:.4f} ms, "
                      f"err {err:.3e}", file=sys.stderr, flush=True)
            tree.free()
    print(json.dumps({"ablation": rows, "samples_per_subdomain": 1, "group": 64, "steps": args.steps,
                      "git_sha": git_sha(), "csrc_sha256_16": csrc_hash()}))


def main():
    args = parse()
    if args.ablation:
        if args.gpus != 1:
            sys.exit(2)
        ablation(args)
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "queries are independent, so several GPUs would each evaluate a share of them", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    import paper_2506_02219_amd as P
    if not os.path.exists(P.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    cfg = CONFIGS[args.config]
    kernel = cfg["kernel"]
    S = args.samples or cfg["samples"]
    do_learned = args.config == "c5" and not args.no_learned and args.branching == 2
    train_clouds, train_gen_s = None, 0.0
    if do_learned:
        t0 = time.time()
        train_clouds = training_surfaces(W.c5_training_seeds()[:args.train_seeds])
        train_gen_s = time.time() - t0
    c4, c4_gen_s = None, 0.0
    if not args.no_batch:
        t0 = time.time()
        c4 = batch_clouds()
        c4_gen_s = time.time() - t0
    t0 = time.time()
    cl = getattr(W, cfg["gen"])()
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    src = torch.from_numpy(cl.sources).to(dev)
    wts = torch.from_numpy(cl.weights).to(dev)
    nrm = None if cl.normals is None else torch.from_numpy(cl.normals).to(dev)
    # the headline sees the queries shuffled (a wavefront's queries share random streams, so
    # neighbouring pixels must not share a wavefront); the comparisons also run on the grid order
    qry_np, perm = W.shuffle_queries(cl.queries, 4242)
    qry = torch.from_numpy(qry_np).to(dev)
    qry_grid = torch.from_numpy(cl.queries).to(dev)
    N = qry.shape[0]
    stream = torch.cuda.current_stream()

    # plain device copy of known size: calibrates the HBM counters of a profiled run
    calib = torch.empty(64 << 20, dtype=torch.float32, device=dev)
    calib2 = torch.empty_like(calib)
    calib2.copy_(calib)

    # --- tree build (timed separately)
    def build(d):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        t = P.sbh_build(src, wts, nrm, branching=d, leaf_size=8)
        torch.cuda.synchronize()
        return t, (time.perf_counter() - tb) * 1e3
    tree, build_ms = build(args.branching)
    tree, build_ms = build(args.branching)  # second build: no first-call overheads

    # --- reference on a fixed query sample
    rng = np.random.Generator(np.random.PCG64(99))
    ns = min(args.err_sample, N)
    sidx = np.sort(rng.choice(N, size=ns, replace=False))
    sidx_t = torch.from_numpy(sidx).to(dev)
    ref = P.sbh_brute(src, wts, nrm, qry[sidx_t].contiguous(), kernel, fp64=True).cpu().numpy()

    out = torch.empty(N, dtype=torch.float32, device=dev)

    def run_sbh(tr, samples, group=args.group):
        P.sbh_eval(tr, qry, kernel, samples=samples, seed=0, group=group, out=out)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(steps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    grid_idx_t = torch.from_numpy(perm[sidx]).to(dev)

    def err_of(fn, idx_t=sidx_t):
        fn()
        torch.cuda.synchronize()
        return float(np.median(rel_errors(out[idx_t].cpu().numpy(), ref, kernel)))

    # --- the timed region: K evaluations of every query
    for _ in range(args.warmup):
        run_sbh(tree, S)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        run_sbh(tree, S)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    qps = N / (ms_per_step * 1e-3)
    err_star = err_of(lambda: run_sbh(tree, S))

    # --- algorithmic work of one launch, from the kernel's own path records
    d = args.branching
    exp = tree.export()

    def work_of(group, rr_mode=0):
        """Algorithmic bytes and flops of one launch, from the kernel's own path records.

        A path's attempted steps are its accepted ones, plus the step its roulette stopped (flag 0).
        Every attempted step costs the roulette of Eq. (5): the selected child's distance and p
        (ROULETTE_FLOPS), reading the child counts (d^3 + 1 words) and the selected child's
        aggregate.  An accepted step at an internal node T adds the swap of Eq. (6): one term per
        non-empty child of T and the weight update (STEP_FLOPS), reading the rest of T's child
        block; an accepted step at a leaf adds one term per point of the leaf.  A roulette stop
        does no swap.  Per query: the subdomain control variates and the final sums."""
        d3 = d ** 3
        paths = torch.empty((N, d3, S, 4), dtype=torch.int32, device=dev)
        P.sbh_eval(tree, qry, kernel, samples=S, seed=0, group=group, out=out, paths=paths, rr_mode=rr_mode)
        torch.cuda.synchronize()
        rec = paths.cpu().numpy().reshape(-1, 4)
        del paths
        rec = rec[rec[:, 0] >= 0]
        steps_acc = rec[:, 2].astype(np.int64)
        flags = rec[:, 3]
        # node lookup by (level, begin)
        key_nodes = exp["level"].astype(np.int64) * (1 << 32) + exp["begin"].astype(np.int64)
        order = np.argsort(key_nodes)
        ks = key_nodes[order]
        parent = exp["parent"].astype(np.int64)
        nch = exp["nchild"].astype(np.int64)
        lev = exp["level"].astype(np.int64)
        cnt = exp["count"].astype(np.int64)
        # cumc[v]: non-empty children summed over v and its ancestors below the root
        cumc = np.zeros(len(nch), np.int64)
        for L in range(1, int(lev.max()) + 1):   # breadth-first: parents come first
            m = lev == L
            cumc[m] = nch[m] + cumc[parent[m]]
        cumc[lev == 0] = 0
        vp = flags == 2
        # the node a path ended at (flags 0 and 1), or the leaf whose point it moved onto (flag 2)
        end_lev = rec[:, 1].astype(np.int64) - vp
        end_key = end_lev * (1 << 32) + rec[:, 0].astype(np.int64)
        pos = np.searchsorted(ks, end_key, side="right") - 1   # flag 2: the leaf holding the point
        end_node = order[np.clip(pos, 0, len(ks) - 1)]
        assert np.all(lev[end_node] == end_lev) and np.all(exp["begin"][end_node] <= rec[:, 0])
        # internal nodes whose swaps were taken: every ancestor of the end node below the root
        # (a leaf's own swap, flag 2, is over its points)
        par = parent[end_node]
        swap_terms = np.where(par > 0, cumc[np.maximum(par, 0)], 0)
        leaf_pts = np.where(vp, cnt[end_node], 0)
        attempted = steps_acc + (flags == 0)
        wind = kernel == 1
        blk_row = 16 * (2 if wind else 1)
        tf = TERM_FLOPS[kernel]
        n_terms = int(swap_terms.sum() + leaf_pts.sum())
        n_att = int(attempted.sum())
        n_acc = int(steps_acc.sum())
        n_int_acc = int((steps_acc - vp).sum())
        alg_flops = float(n_terms * (tf + 1) + n_acc * STEP_FLOPS + n_att * ROULETTE_FLOPS
                          + N * (int(nch[0]) * (tf + 1) + 4))
        alg_bytes = float(n_att * ((d3 + 1) * 4 + blk_row) + (n_terms - n_int_acc - int(vp.sum())) * blk_row
                          + N * (12 + 4 + int(nch[0]) * blk_row + d3 * 4))
        return dict(alg_bytes=alg_bytes, alg_flops=alg_flops, mean_steps=float(steps_acc.mean()),
                    attempted_steps_per_path=float(n_att / len(rec)),
                    children_per_accepted_internal_step=float(swap_terms.sum() / max(n_int_acc, 1)),
                    paths=int(len(rec)), terms=n_terms, accepted=n_acc, attempted=n_att)

    wk = work_of(args.group)
    mean_steps = wk["mean_steps"]
    derivation = {
        "paths_per_launch": wk["paths"], "accepted_steps_per_path": wk["mean_steps"],
        "attempted_steps_per_path": wk["attempted_steps_per_path"],
        "children_per_accepted_internal_step": wk["children_per_accepted_internal_step"],
        "terms_per_launch": wk["terms"], "term_flops": TERM_FLOPS[kernel] + 1, "roulette_flops": ROULETTE_FLOPS,
        "step_flops": STEP_FLOPS,
        "flops": "terms x term_flops + accepted x step_flops + attempted x roulette_flops "
                 "+ queries x (subdomains x term_flops + 4)"}
    if args.group % 64 == 0:
        tflops = wk["alg_flops"] / (ms_per_step * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / FP32_PEAK_TFLOPS, "traffic": None,
                "alg_flops_per_launch": wk["alg_flops"], "kernel": "k_sbh_wave",
                # the build has no packed fp32 instructions: half the peak is what it can issue
                "frac_of_non_packed_fp32": tflops / (FP32_PEAK_TFLOPS / 2), "derivation": derivation}
    else:
        achieved_gbs = wk["alg_bytes"] / (ms_per_step * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None,
                "alg_bytes_per_launch": wk["alg_bytes"], "kernel": "k_sbh_pool", "derivation": derivation}

    # --- the other stream mode (per-query streams vs shared per wavefront), same tree and queries
    other = None
    og = 1 if args.group != 1 else 64
    ms_o = timed(lambda: run_sbh(tree, S, og), args.steps, args.warmup)
    e_o = err_of(lambda: run_sbh(tree, S, og))
    wk_o = work_of(og)
    other = dict(group=og, ms_per_step=ms_o, queries_per_s=N / (ms_o * 1e-3), median_rel_err=e_o,
                 alg_bytes_per_launch=wk_o["alg_bytes"], achieved_alg_GBs=wk_o["alg_bytes"] / (ms_o * 1e-3) / 1e9,
                 alg_flops_per_launch=wk_o["alg_flops"], l2_peak_GBs=L2_PEAK_GBS,
                 frac_of_l2_peak=wk_o["alg_bytes"] / (ms_o * 1e-3) / 1e9 / L2_PEAK_GBS)

    # --- the same estimator on the plane's original pixel order: neighbouring queries share a
    # wavefront (and its random stream); per-query estimates have the same distribution, but
    # neighbours' errors are correlated, which the paper avoids by shuffling
    def run_grid():
        P.sbh_eval(tree, qry_grid, kernel, samples=S, seed=0, group=args.group, out=out)

    grid_order = None
    if not args.no_grid:
        grid_order = dict(group=args.group, ms=timed(run_grid, args.steps, args.warmup),
                          median_rel_err=err_of(run_grid, grid_idx_t))
        grid_order["queries_per_s"] = N / (grid_order["ms"] * 1e-3)

    # --- the tile-shared score proposal on the plane's own order (tiles of 64 neighbouring pixels)
    tile_grid = None
    if not args.no_grid and args.branching == 2:
        def run_tile(samples):
            P.sbh_eval(tree, qry_grid, kernel, samples=samples, seed=0, group=args.group, out=out, proposal=3)

        tile_grid = dict(group=args.group, sweep=[])
        for sv in (1, 2, 4):
            ms_t = timed(lambda: run_tile(sv), args.steps if sv == 1 else 3, args.warmup if sv == 1 else 1)
            tile_grid["sweep"].append(dict(samples=sv, ms=ms_t, median_rel_err=err_of(lambda: run_tile(sv), grid_idx_t)))
        tile_grid["queries_per_s"] = N / (tile_grid["sweep"][0]["ms"] * 1e-3)

    # --- samples-per-subdomain sweep (error / time curve of the stochastic method)
    sweep = None
    if not args.no_sweep:
        sweep = []
        for sv in S_SWEEP:
            ms_s = timed(lambda: run_sbh(tree, sv), 3, 1)
            sweep.append(dict(samples=sv, ms=ms_s, median_rel_err=err_of(lambda: run_sbh(tree, sv))))

    # --- subdomains from the Barnes-Hut cut D(q, beta_low) (Section 3.3.1), on the headline's queries
    cut = None
    if not args.no_cut and args.group % 64 == 0 and args.branching in (2, 4):
        cut = dict(group=args.group, sweep=[])
        for bl in (0.3, 0.5, 0.8):
            def run_cut(bl=bl):
                P.sbh_eval(tree, qry, kernel, beta=bl, samples=S, seed=0, group=args.group, out=out, subdomains=1)
            cut["sweep"].append(dict(beta_low=bl, ms=timed(run_cut, 5, 1), median_rel_err=err_of(run_cut)))

    # --- the walk on compressed interior aggregates (binary16 codes, 8 bytes a child slot in place of
    # the 16 of a float32 centre of mass and mass), same queries and samples as the headline
    compressed = None
    if (not args.no_compressed and args.group % 64 == 0 and args.branching == 2
            and kernel in (P.POTENTIAL, P.SMOOTHDIST)):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ctree = P.sbh_build(src, wts, nrm, branching=2, leaf_size=8, compress=True)
        torch.cuda.synchronize()
        cbuild_ms = (time.perf_counter() - tb) * 1e3

        def run_cmp():
            P.sbh_eval(ctree, qry, kernel, samples=S, seed=0, group=args.group, out=out, compressed=1)

        ms_c = timed(run_cmp, args.steps, args.warmup)
        d3 = 8

        def run_cmp_o():   # the other stream mode, against the uncompressed walk's `other` leg
            P.sbh_eval(ctree, qry, kernel, samples=S, seed=0, group=og, out=out, compressed=1)

        ms_co = timed(run_cmp_o, args.steps, args.warmup)
        compressed = dict(group=args.group, samples=S, ms_per_step=ms_c, queries_per_s=N / (ms_c * 1e-3),
                          median_rel_err=err_of(run_cmp), vs_headline=ms_per_step / ms_c, build_ms=cbuild_ms,
                          other_stream_mode=dict(group=og, ms_per_step=ms_co, median_rel_err=err_of(run_cmp_o),
                                                 vs_uncompressed=ms_o / ms_co),
                          child_block_bytes=d3 * 8, float32_child_block_bytes=d3 * 16,
                          interior_aggregate_bytes=int(ctree.n_blocks) * d3 * 8,
                          float32_interior_aggregate_bytes=int(ctree.n_blocks) * d3 * 16)
        ctree.free()

    # --- second-order node terms (the potential's quadrupole term where a node is far), same queries;
    # an S sweep gives its error / time curve beside the point-mass one
    lod2 = None
    if (not args.no_lod2 and args.group % 64 == 0 and args.branching == 2 and kernel == P.POTENTIAL):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        qtree = P.sbh_build(src, wts, nrm, branching=2, leaf_size=8, quadrupole=True)
        torch.cuda.synchronize()
        qbuild_ms = (time.perf_counter() - tb) * 1e3

        def run_l2(samples=S):
            P.sbh_eval(qtree, qry, kernel, samples=samples, seed=0, group=args.group, out=out, lod=2)

        ms_l = timed(run_l2, args.steps, args.warmup)
        lod2 = dict(group=args.group, samples=S, ms_per_step=ms_l, queries_per_s=N / (ms_l * 1e-3),
                    median_rel_err=err_of(run_l2), vs_headline=ms_per_step / ms_l, build_ms=qbuild_ms,
                    tensor_bytes=int(qtree.n_blocks) * 8 * 32, sweep=[])
        for sv in (2, 4):
            lod2["sweep"].append(dict(samples=sv, ms=timed(lambda: run_l2(sv), 3, 1),
                                      median_rel_err=err_of(lambda: run_l2(sv))))
        qtree.free()

    # --- the roulette voted over each wavefront (rr_mode 3: every query of a tile continues with the
    # largest Eq. (5) p of the tile's queries), same tree and queries, with an S sweep
    voted = None
    if not args.no_vote and args.group % 64 == 0:
        def run_vote(samples=S):
            P.sbh_eval(tree, qry, kernel, samples=samples, seed=0, group=args.group, out=out, rr_mode=3)

        ms_v = timed(run_vote, args.steps, args.warmup)
        wk_v = work_of(args.group, 3)
        tf_v = wk_v["alg_flops"] / (ms_v * 1e-3) / 1e12
        voted = dict(group=args.group, samples=S, ms_per_step=ms_v, queries_per_s=N / (ms_v * 1e-3),
                     median_rel_err=err_of(run_vote), vs_headline=ms_per_step / ms_v,
                     accepted_steps_per_path=wk_v["mean_steps"], alg_flops_per_launch=wk_v["alg_flops"],
                     achieved_TFLOPs=tf_v, frac_of_fp32_peak=tf_v / FP32_PEAK_TFLOPS, sweep=[])
        for sv in (2, 4):
            voted["sweep"].append(dict(samples=sv, ms=timed(lambda: run_vote(sv), 3, 1),
                                       median_rel_err=err_of(lambda: run_vote(sv))))

    # --- float32 brute force over every query (Eq. (1) summed exactly: the paper's third comparator)
    brute = None
    if not args.no_brute:
        bout = torch.empty(N, dtype=torch.float32, device=dev)

        def run_brute():
            P.sbh_brute(src, wts, nrm, qry, kernel, out=bout)

        ms_b = timed(run_brute, 2, 1)
        inter = float(cl.m) * N
        tf_b = BRUTE_FLOPS[kernel] * inter / (ms_b * 1e-3) / 1e12
        brute = dict(kernel="k_brute32" if kernel != P.SMOOTHDIST else "k_brute<2, float>", queries=N,
                     sources=int(cl.m), ms=ms_b, interactions_per_s=inter / (ms_b * 1e-3),
                     flops_per_interaction=BRUTE_FLOPS[kernel], achieved_TFLOPs=tf_b,
                     frac_of_fp32_peak=tf_b / FP32_PEAK_TFLOPS, frac_of_non_packed_fp32=tf_b / (FP32_PEAK_TFLOPS / 2),
                     median_rel_err=float(np.median(rel_errors(bout[sidx_t].cpu().numpy(), ref, kernel))),
                     estimator_speedup=ms_b / ms_per_step)
        del bout

    # --- Barnes-Hut sweeps and equal-error interpolation.  The paper compares the two methods on
    # one query set at a time (a grid, random points), so Barnes-Hut is swept on both orders the
    # estimator is timed on: the shuffled plane (the headline's own queries, in the same order)
    # and the plane's own pixel order (coherent lanes, Barnes-Hut's best case).
    bh = None
    if not args.no_bh:
        bh_tree = tree if args.bh_branching == args.branching else build(args.bh_branching)[0]

        # sweep until Barnes-Hut is well below every error it is compared at
        e_floor = min([err_star] + ([c_["median_rel_err"] for c_ in cut["sweep"]] if cut else [])
                      + ([lod2["median_rel_err"]] if lod2 else []) + ([voted["median_rel_err"]] if voted else []))

        def bh_sweep(qset, idx_t):
            pts = []
            for beta in BETAS:
                def run(beta=beta):
                    P.sbh_eval(bh_tree, qset, kernel, beta=beta, samples=0, out=out)
                ms = timed(run, 3, 1)
                e = err_of(run, idx_t)
                pts.append((beta, ms, e))
                if e < e_floor / 4 and len(pts) > 2:
                    break
            return pts

        def at_error(pts, e_target):
            """Barnes-Hut's time at median error e_target: log-log interpolation between the bracketing betas"""
            t = log_interp([p_[2] for p_ in pts], [p_[1] for p_ in pts], e_target)
            if t is not None:
                return t, "interpolated"
            if pts[0][2] <= e_target:
                return pts[0][1], "upper_bound_at_smallest_beta"
            return None, "not_reached"

        def summary(pts):
            t_eq, kind = at_error(pts, err_star)
            return dict(sweep=[dict(beta=b, ms=round(m, 4), median_rel_err=e) for b, m, e in pts],
                        ms_at_equal_error=None if t_eq is None else round(t_eq, 4),
                        queries_per_s_at_equal_error=None if t_eq is None else N / (t_eq * 1e-3), match=kind), t_eq

        pts_s = bh_sweep(qry, sidx_t)
        pts_g = bh_sweep(qry_grid, grid_idx_t)
        sum_s, t_s = summary(pts_s)
        sum_g, t_g = summary(pts_g)
        if tile_grid is not None:
            # Barnes-Hut (same pixel order) at the tile-proposal estimator's (lower) error
            e1 = tile_grid["sweep"][0]["median_rel_err"]
            tb = at_error(pts_g, e1)[0]
            tile_grid["bh_ms_at_this_error"] = tb
            tile_grid["speedup_vs_bh_at_this_error"] = None if tb is None else tb / tile_grid["sweep"][0]["ms"]
        if cut is not None:
            for c_ in cut["sweep"]:
                tb = at_error(pts_s, c_["median_rel_err"])[0]
                c_["bh_ms_at_this_error"] = tb
                c_["speedup_vs_bh_at_this_error"] = None if tb is None else tb / c_["ms"]
        if voted is not None:
            tb = at_error(pts_s, voted["median_rel_err"])[0]
            voted["bh_ms_at_this_error"] = tb
            voted["speedup_vs_bh_at_this_error"] = None if tb is None else tb / voted["ms_per_step"]
            # the headline estimator (Eq. (5)) at the voted roulette's error, from its S sweep
            if sweep:
                te = log_interp([r["median_rel_err"] for r in sweep], [r["ms"] for r in sweep], voted["median_rel_err"])
                voted["eq5_ms_at_this_error"] = te
                voted["speedup_vs_eq5_at_this_error"] = None if te is None else te / voted["ms_per_step"]
        if lod2 is not None:
            tb = at_error(pts_s, lod2["median_rel_err"])[0]
            lod2["bh_ms_at_this_error"] = tb
            lod2["speedup_vs_bh_at_this_error"] = None if tb is None else tb / lod2["ms_per_step"]
        if grid_order is not None:
            tb = at_error(pts_g, grid_order["median_rel_err"])[0]
            grid_order["bh_ms_at_this_error"] = tb
            grid_order["speedup_vs_bh_at_this_error"] = None if tb is None else tb / grid_order["ms"]
        bh = dict(branching=args.bh_branching, shuffled=sum_s, grid_order=sum_g,
                  # the headline's queries, order and error for both methods
                  speedup_stochastic_vs_bh=None if t_s is None else t_s / ms_per_step,
                  # Barnes-Hut on the coherent pixel order against the headline (shuffled) estimator
                  speedup_stochastic_vs_bh_on_grid_order=None if t_g is None else t_g / ms_per_step)

    # --- learned proposal: trained on the held-out surfaces, evaluated on this one
    learned = None
    if do_learned:
        from paper_2506_02219_amd import learned as L
        torch.cuda.synchronize()
        tl = time.perf_counter()
        Xs, Ts, Cs = [], [], []
        # the last training surface is held out for validation (model selection); the others train
        val_pts, val_w = train_clouds[-1]
        train_clouds = train_clouds[:-1]
        for i, (tp, tw) in enumerate(train_clouds):
            tt = P.sbh_build(torch.from_numpy(tp).to(dev), torch.from_numpy(tw).to(dev), None, branching=2,
                             leaf_size=8)
            r = np.random.Generator(np.random.PCG64(7000 + i))
            tq = np.zeros((args.train_queries, 3), np.float32)
            tq[:, :2] = r.uniform(-1.5, 1.5, (args.train_queries, 2))
            X, Tg, Cn = L.training_rows(tt, torch.from_numpy(tq).to(dev), kernel, seed=8000 + i)
            Xs.append(X); Ts.append(Tg); Cs.append(Cn)
            tt.free()
        X, Tg, Cn = torch.cat(Xs), torch.cat(Ts), torch.cat(Cs)
        del Xs, Ts, Cs, train_clouds
        torch.cuda.synchronize()
        rows_ms = (time.perf_counter() - tl) * 1e3
        # validation: median relative error of the learned estimator (S = 1) on 8192 pixels of the
        # plane over the held-out surface, against float64 brute force
        vt = P.sbh_build(torch.from_numpy(val_pts).to(dev), torch.from_numpy(val_w).to(dev), None, branching=2,
                         leaf_size=8)
        vr = np.random.Generator(np.random.PCG64(7100))
        vq = torch.from_numpy(cl.queries[np.sort(vr.choice(N, size=8192, replace=False))]).to(dev)
        vref = P.sbh_brute(torch.from_numpy(val_pts).to(dev), torch.from_numpy(val_w).to(dev), None, vq, kernel,
                           fp64=True).cpu().numpy()
        vout = torch.empty(vq.shape[0], dtype=torch.float32, device=dev)

        def validate(params):
            errs = []
            for b_ in range(4):
                P.sbh_eval(vt, vq, kernel, samples=1, seed=77, batch=b_, group=1, out=vout, mlp=params)
                errs.append(rel_errors(vout.cpu().numpy(), vref, kernel))
            return float(np.median(np.concatenate(errs)))

        prm = L.init_params(1)
        loss0 = L.mean_loss(prm, X, Tg, Cn)
        torch.cuda.synchronize()
        tt0 = time.perf_counter()
        prm, val_hist = L.train_selected(prm, X, Tg, Cn, args.train_steps, validate, chunks=8,
                                         batch_rows=args.train_batch, lr=args.train_lr, seed=2)
        torch.cuda.synchronize()
        train_ms = (time.perf_counter() - tt0) * 1e3
        loss1 = L.mean_loss(prm, X, Tg, Cn)
        vt.free()

        def proposal_curve(prop, params):
            """(samples, ms, median error) of proposal 1 or 2, and its speed at equal error to the plain method"""
            def run(samples):
                P.sbh_eval(tree, qry, kernel, samples=samples, seed=0, group=1, out=out, mlp=params, proposal=prop)
            cur = []
            for sv in (1, 2, 4):
                ms_l = timed(lambda: run(sv), args.steps if sv == 1 else 3, args.warmup if sv == 1 else 1)
                cur.append(dict(samples=sv, ms=ms_l, median_rel_err=err_of(lambda: run(sv))))
            c1 = cur[0]
            # the plain method's time at this method's error, interpolated over its samples sweep
            t_plain = None
            if sweep:
                t_plain = log_interp([p["median_rel_err"] for p in sweep], [p["ms"] for p in sweep],
                                     c1["median_rel_err"])
            # this method's time at the plain method's error: interpolated over its own sweep, or (when one
            # sample already beats it) scaled down by the 1/S law of the variance
            t_eq = log_interp([p["median_rel_err"] for p in cur], [p["ms"] for p in cur], err_star)
            how = "interpolated"
            if t_eq is None and c1["median_rel_err"] <= err_star:
                t_eq, how = c1["ms"] * (c1["median_rel_err"] / err_star) ** 2, "extrapolated_1_over_S"
            return dict(group=1, sweep=cur, plain_ms_at_this_error=t_plain,
                        speedup_vs_plain_at_this_error=None if t_plain is None else t_plain / c1["ms"],
                        ms_at_plain_error=t_eq, match=how if t_eq is not None else "not_reached",
                        queries_per_s_at_plain_error=None if t_eq is None else N / (t_eq * 1e-3))

        learned = dict(
            train_surfaces=args.train_seeds - 1, train_queries_per_surface=args.train_queries, train_rows=int(X.shape[0]),
            train_steps=args.train_steps, train_batch=args.train_batch, lr=args.train_lr,
            surface_generation_s=train_gen_s, rows_ms=rows_ms, train_ms=train_ms,
            loss_untrained=loss0, loss_selected=loss1, validation=[dict(steps=k, median_rel_err=v) for k, v in val_hist],
            validation_surface_seed=W.c5_training_seeds()[args.train_seeds - 1],
            network=proposal_curve(1, prm), score_only=proposal_curve(2, None))
        del X, Tg, Cn

    # --- batched evaluation of 64 clouds of uneven size (one launch per kernel group, graph replay)
    batched = None
    if c4 is not None:
        trees_b, qs_b, ks_b = [], [], []
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        for srcs, ws, ns, qq, kk in c4:
            trees_b.append(P.sbh_build(torch.from_numpy(srcs).to(dev), torch.from_numpy(ws).to(dev),
                                       None if ns is None else torch.from_numpy(ns).to(dev), branching=2,
                                       leaf_size=8))
            qs_b.append(torch.from_numpy(qq).to(dev))
            ks_b.append(kk)
        torch.cuda.synchronize()
        build_all_ms = (time.perf_counter() - tb0) * 1e3
        NB = sum(q.shape[0] for q in qs_b)
        outs_seq = [torch.empty(q.shape[0], dtype=torch.float32, device=dev) for q in qs_b]

        def run_seq():
            for t_, q_, k_, o_ in zip(trees_b, qs_b, ks_b, outs_seq):
                P.sbh_eval(t_, q_, k_, samples=S, seed=0, group=64, out=o_)

        ms_seq = timed(run_seq, 5, 1)
        tp0 = time.perf_counter()
        plan = P.Batch(trees_b, qs_b, ks_b, samples=S, group=64)
        plan_ms = (time.perf_counter() - tp0) * 1e3
        ms_batch = timed(lambda: plan.launch(0, 0), args.steps, args.warmup)
        plan.launch(0, 0)
        run_seq()
        torch.cuda.synchronize()
        identical = all(bool(torch.equal(torch.nan_to_num(a, nan=1e30), torch.nan_to_num(b, nan=1e30)))
                        for a, b in zip(plan.outs, outs_seq))
        batched = dict(workload="64 clouds of log-uniform sizes (sources 2^12..2^20, queries 2^14..2^18), "
                                "kernels cycling potential / winding / smooth distance",
                       clouds=len(qs_b), queries=int(NB), sources=int(sum(t_.n_points for t_ in trees_b)),
                       samples_per_subdomain=S, group=64, generate_s=c4_gen_s, build_all_ms=build_all_ms,
                       sequential_ms=ms_seq, sequential_queries_per_s=NB / (ms_seq * 1e-3),
                       batched_ms=ms_batch, batched_queries_per_s=NB / (ms_batch * 1e-3),
                       speedup_batched_vs_sequential=ms_seq / ms_batch, plan_create_ms=plan_ms,
                       autotuned=plan.config, identical_to_sequential=identical)
        plan.free()
        for t_ in trees_b:
            t_.free()
        del trees_b, qs_b, outs_seq, c4

    # --- CPU baseline: the FP64 oracle on the host cores, on a bounded sample
    cpu = None
    if not args.no_cpu:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        ot = oracle.Tree(cl.sources, cl.weights, cl.normals, d=args.branching, leaf_size=8)
        nsamp = min(N, 20000)
        tc = time.perf_counter()
        ot.sbh(qry_np[:nsamp], kernel, samples=S, seed=0, group=args.group, index=np.arange(nsamp), threads=threads)
        per_q = (time.perf_counter() - tc) / nsamp
        # the whole query set (or a prefix of it), repeated until about cpu_seconds of work
        nsamp = int(min(N, max(nsamp, args.cpu_seconds / max(per_q, 1e-9))))
        reps = max(1, int(args.cpu_seconds / max(per_q * nsamp, 1e-9)))
        tc = time.perf_counter()
        for _ in range(reps):
            ot.sbh(qry_np[:nsamp], kernel, samples=S, seed=0, group=args.group, index=np.arange(nsamp),
                   threads=threads)
        cpu_s = time.perf_counter() - tc
        nsamp_total = nsamp * reps
        # the same oracle on one thread, on a prefix of the same queries (about a quarter of the time)
        n1 = int(min(N, max(256, args.cpu_seconds / 4 / max(per_q * threads, 1e-9))))
        tc = time.perf_counter()
        ot.sbh(qry_np[:n1], kernel, samples=S, seed=0, group=args.group, index=np.arange(n1), threads=1)
        one_s = time.perf_counter() - tc
        cpu = dict(value=nsamp_total / cpu_s, unit="queries/s", cores=threads, kind="oracle",
                   sample=f"first {nsamp} of {N} queries x {reps} repetitions, same tree, seed and streams, "
                          f"{cpu_s:.1f} s",
                   single_thread=dict(value=n1 / one_s, unit="queries/s", cores=1,
                                      sample=f"first {n1} of {N} queries, {one_s:.1f} s"))

    prof = os.path.join(ROOT, "profiles", f"pmc_sbh_eval_{args.config}_d{args.branching}_g{args.group}.json")
    if os.path.exists(prof):
        with open(prof) as f:
            pm = json.load(f)
        if pm.get("csrc_hash") == csrc_hash() and pm.get("samples") == S:
            # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters, scaled by what the same
            # counters read for a plain copy of known size
            roof["traffic"] = (pm["fetch_kib"] * pm["fetch_factor"] + pm["write_kib"] * pm["write_factor"]) * 1024.0

    line = {
        "metric": "queries/s at fixed median rel. error vs brute force (plain vs learned, vs det. BH)",
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cl.name, "sources": int(cl.m), "queries": int(N), "kernel": ["potential", "winding", "smoothdist"][kernel],
                   "samples_per_subdomain": S, "branching": args.branching, "leaf_size": 8, "group": args.group,
                   "seed": 0},
        "median_rel_err": err_star,
        "err_sample": ns,
        "interactions_per_s": qps * cl.m,
        "build_ms": build_ms,
        "wall_ms_timed_region": wall_ms,
        "mean_accepted_steps_per_path": mean_steps,
        "attempted_steps_per_path": wk["attempted_steps_per_path"],
        "other_stream_mode": other,
        "grid_order": grid_order,
        "tile_score_grid_order": tile_grid,
        "cut_subdomains": cut,
        "compressed_aggregates": compressed,
        "second_order_lod": lod2,
        "voted_roulette": voted,
        "brute_force": brute,
        "sbh_sweep": sweep,
        "bh": bh,
        "learned": learned,
        "batched": batched,
        "roofline": roof,
        "cpu_baseline": cpu,
        "generate_s": gen_s,
        "git_sha": git_sha(),
        "csrc_sha256_16": csrc_hash(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
