"""Stochastic Barnes-Hut on MI355X: Python binding of libsbh.

Argument marshalling only.  Every step of the method runs in the HIP
kernels of libsbh.so (built from csrc/ by build_lib.py); PyTorch supplies
device memory and the current stream.  The names follow the C ABI in
include/sbh.h.  If the library is missing this module raises; there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbh.so")

POTENTIAL, WINDING, SMOOTHDIST = 0, 1, 2
MLP_NPARAM, MLP_GRAD_SIZE = 1608, 1610
KERNELS = {"potential": POTENTIAL, "winding": WINDING, "smoothdist": SMOOTHDIST}


class BuildOpts(C.Structure):
    _fields_ = [("branching", C.c_int32), ("leaf_size", C.c_int32), ("max_level", C.c_int32), ("compress", C.c_int32),
                ("quadrupole", C.c_int32)]


class EvalOpts(C.Structure):
    _fields_ = [("eps", C.c_float), ("alpha", C.c_float), ("group", C.c_int32), ("rr_mode", C.c_int32),
                ("proposal", C.c_int32), ("batch", C.c_uint32), ("paths", C.c_void_p), ("mlp", C.c_void_p),
                ("subdomains", C.c_int32), ("compressed", C.c_int32), ("lod", C.c_int32)]


class BatchItem(C.Structure):
    _fields_ = [("tree", C.c_void_p), ("queries", C.c_void_p), ("out", C.c_void_p), ("nq", C.c_int64),
                ("kernel", C.c_int32), ("reserved", C.c_int32)]


class BatchConfig(C.Structure):
    _fields_ = [("tile_waves", C.c_int32), ("waves_per_simd", C.c_int32), ("heavy_first", C.c_int32),
                ("ms", C.c_float)]


class TreeDesc(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("n_nodes", C.c_int64), ("n_blocks", C.c_int64),
                ("depth", C.c_int32), ("branching", C.c_int32), ("leaf_size", C.c_int32),
                ("max_level", C.c_int32), ("has_normals", C.c_int32), ("lo", C.c_float * 3),
                ("side", C.c_float), ("inv_side", C.c_float)]


class SbhError(RuntimeError):
    def __init__(self, call, status, message):
        super().__init__(f"{call} failed: {status}: {message}")
        self.status = status


_lib = None


def lib():
    """Load libsbh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with paper_2506_02219_amd/build_lib.py")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, u32, u64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float
        L.sbh_build_opts_default.argtypes = [P]
        L.sbh_build_opts_default.restype = None
        L.sbh_eval_opts_default.argtypes = [P]
        L.sbh_eval_opts_default.restype = None
        L.sbh_build.argtypes = [P, P, P, i64, P, P, P]
        L.sbh_build.restype = i32
        L.sbh_eval.argtypes = [P, P, i64, i32, f32, i32, u64, P, P, P]
        L.sbh_eval.restype = i32
        L.sbh_brute.argtypes = [P, P, P, i64, P, i64, i32, P, i32, P, P]
        L.sbh_brute.restype = i32
        L.sbh_tree_info.argtypes = [P, P]
        L.sbh_tree_info.restype = i32
        L.sbh_tree_export.argtypes = [P] + [P] * 12
        L.sbh_tree_export.restype = i32
        L.sbh_tree_export_compressed.argtypes = [P, P]
        L.sbh_tree_export_compressed.restype = i32
        L.sbh_tree_export_quadrupole.argtypes = [P, P]
        L.sbh_tree_export_quadrupole.restype = i32
        L.sbh_mlp_forward.argtypes = [P, P, i64, P, P]
        L.sbh_mlp_forward.restype = i32
        L.sbh_mlp_pairs.argtypes = [P, P, i64, i32, u64, i32, P, P, P, P, P, P]
        L.sbh_mlp_pairs.restype = i32
        L.sbh_mlp_loss_grad.argtypes = [P, P, P, P, i64, P, P]
        L.sbh_mlp_loss_grad.restype = i32
        L.sbh_mlp_train.argtypes = [P, P, P, P, P, i64, i32, i32, f32, i32, P, P]
        L.sbh_mlp_train.restype = i32
        L.sbh_mlp_train_noalloc.argtypes = [P, P, P, P, P, i64, i32, i32, f32, i32, P, P]
        L.sbh_mlp_train_noalloc.restype = i32
        L.sbh_batch_create.argtypes = [P, i32, i32, P, P, P, P]
        L.sbh_batch_create.restype = i32
        L.sbh_batch_launch.argtypes = [P, u64, u32, P]
        L.sbh_batch_launch.restype = i32
        L.sbh_batch_get_config.argtypes = [P, P]
        L.sbh_batch_get_config.restype = i32
        L.sbh_batch_free.argtypes = [P]
        L.sbh_batch_free.restype = i32
        L.sbh_free.argtypes = [P]
        L.sbh_free.restype = i32
        L.sbh_free_async.argtypes = [P, P]
        L.sbh_free_async.restype = i32
        L.sbh_set_allocator.argtypes = [P, P, P]
        L.sbh_set_allocator.restype = i32
        L.sbh_status_string.argtypes = [i32]
        L.sbh_status_string.restype = C.c_char_p
        L.sbh_last_error.argtypes = []
        L.sbh_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(call, status):
    if status != 0:
        L = lib()
        raise SbhError(call, L.sbh_status_string(status).decode(), L.sbh_last_error().decode())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev(t, name, shape_tail=None, dtype=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != (dtype or torch.float32):
        raise TypeError(f"{name} must be {dtype or torch.float32}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}]")
    return t


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


class Tree:
    """Handle on a device tree (sbh_tree*).  Keeps no reference to its inputs."""

    def __init__(self, handle):
        self._h = handle
        d = TreeDesc()
        _check("sbh_tree_info", lib().sbh_tree_info(self._h, C.byref(d)))
        self.n_points, self.n_nodes, self.n_blocks = d.n_points, d.n_nodes, d.n_blocks
        self.depth, self.branching, self.leaf_size = d.depth, d.branching, d.leaf_size
        self.max_level, self.has_normals = d.max_level, bool(d.has_normals)
        self.lo = np.array(list(d.lo), np.float32)
        self.side, self.inv_side = np.float32(d.side), np.float32(d.inv_side)

    @property
    def handle(self):
        return self._h

    def export(self):
        """Host copy of the node and point arrays (sbh_tree_export)."""
        nn, npt = self.n_nodes, self.n_points
        a = {k: np.zeros(nn, np.int32) for k in ("begin", "count", "level", "digit", "parent", "first_child", "nchild")}
        a["agg"] = np.zeros((nn, 4), np.float32)
        a["dip"] = np.zeros((nn, 4), np.float32)
        a["perm"] = np.zeros(npt, np.uint32)
        a["codes"] = np.zeros(npt, np.uint64)
        a["spread2"] = np.zeros(nn, np.float32)
        p = lambda x: x.ctypes.data_as(C.c_void_p)
        _check("sbh_tree_export", lib().sbh_tree_export(
            self._h, p(a["begin"]), p(a["count"]), p(a["level"]), p(a["digit"]), p(a["parent"]),
            p(a["first_child"]), p(a["nchild"]), p(a["agg"]), p(a["dip"]), p(a["perm"]), p(a["codes"]),
            p(a["spread2"])))
        return a

    def export_compressed(self):
        """The compressed aggregates (sbh_tree_export_compressed) as binary16 values
        [n_blocks, d^3, 4] float32: offsets x, y, z (cell sides) and mass fraction."""
        nb = max(self.n_blocks, 1)
        w = np.zeros((nb, self.branching ** 3, 2), np.uint32)
        _check("sbh_tree_export_compressed", lib().sbh_tree_export_compressed(self._h, w.ctypes.data_as(C.c_void_p)))
        h = np.stack([w[..., 0] & 0xFFFF, w[..., 0] >> 16, w[..., 1] & 0xFFFF, w[..., 1] >> 16], -1).astype(np.uint16)
        return h.view(np.float16).astype(np.float32)

    def export_quadrupole(self):
        """The scaled second-moment tensors (sbh_tree_export_quadrupole) [n_blocks, d^3, 8] float32:
        1.5 Qxx, 1.5 Qyy, 1.5 Qzz, 3 Qxy, 3 Qxz, 3 Qyz, tr(Q) / 2, 0."""
        nb = max(self.n_blocks, 1)
        q = np.zeros((nb, self.branching ** 3, 8), np.float32)
        _check("sbh_tree_export_quadrupole", lib().sbh_tree_export_quadrupole(self._h, q.ctypes.data_as(C.c_void_p)))
        return q

    def free(self):
        if self._h:
            lib().sbh_free(self._h)
            self._h = None

    def free_async(self, stream=None):
        """Stream-ordered release (sbh_free_async) on `stream` (default: the current stream)."""
        if self._h:
            _check("sbh_free_async", lib().sbh_free_async(self._h, _stream(stream)))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# --------------------------------------------------------------------------- allocator
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_alloc_keep = None   # the installed callbacks (kept alive while installed)


def sbh_set_allocator(alloc=None, free=None):
    """Route the library's device allocations through alloc(bytes, stream) -> int pointer (0 on
    failure) and free(ptr, bytes, stream) (sbh_set_allocator); both None restores the default.
    `stream` is the raw hipStream_t handle as an int (0 for the null stream)."""
    global _alloc_keep
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        _check("sbh_set_allocator", lib().sbh_set_allocator(None, None, None))
        _alloc_keep = None
        return

    def _a(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0)) or 0)
        except Exception:
            return 0

    def _f(ptr, nbytes, stream, ctx):
        try:
            free(int(ptr), int(nbytes), int(stream or 0))
        except Exception:
            pass

    keep = (ALLOC_FN(_a), FREE_FN(_f))
    _check("sbh_set_allocator", lib().sbh_set_allocator(C.cast(keep[0], C.c_void_p), C.cast(keep[1], C.c_void_p),
                                                        None))
    _alloc_keep = keep


def use_torch_allocator():
    """Take device memory from PyTorch's caching allocator (on the stream of each call)."""
    import torch

    def _alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream or None)

    def _free(ptr, nbytes, stream):
        torch.cuda.caching_allocator_delete(ptr)

    sbh_set_allocator(_alloc, _free)


def sbh_build(sources, weights, normals=None, branching=2, leaf_size=8, max_level=0, stream=None,
              compress=False, quadrupole=False) -> Tree:
    """Build the tree on the GPU (sbh_build). sources [n,3], weights [n], normals [n,3] or None;
    compress: also store the compressed interior aggregates (branching 2); quadrupole: also store the
    children's second-moment tensors (for lod=2)."""
    _dev(sources, "sources", (3,)); _dev(weights, "weights"); _dev(normals, "normals", (3,))
    n = sources.shape[0]
    if weights.shape != (n,) or (normals is not None and normals.shape[0] != n):
        raise ValueError("sources, weights and normals must have the same length")
    o = BuildOpts(branching, leaf_size, max_level, int(bool(compress)), int(bool(quadrupole)))
    h = C.c_void_p()
    _check("sbh_build", lib().sbh_build(_ptr(sources), _ptr(weights), _ptr(normals), n, C.byref(o),
                                        _stream(stream), C.byref(h)))
    return Tree(h)


def sbh_eval(tree: Tree, queries, kernel, beta=2.0, samples=1, seed=0, eps=1e-3, alpha=100.0, group=1,
             rr_mode=0, batch=0, paths=None, out=None, stream=None, mlp=None, proposal=None, subdomains=0,
             compressed=0, lod=1):
    """Evaluate every query (sbh_eval): samples >= 1 stochastic estimator, samples == 0 Barnes-Hut(beta).
    subdomains: 0 the root's children, 1 the Barnes-Hut cut at beta (group a multiple of 64);
    paths: optional int32 CUDA tensor [nq, d^3, samples, 4] receiving the path records ([nq, 4]
    digests with subdomains = 1);
    mlp: optional float32 CUDA tensor [MLP_NPARAM] selecting the learned proposal (1);
    proposal: 0 uniform path index, 1 learned (needs mlp; parameters that are not all finite fall back
    to the score proposal), 2 score proposal, 3 tile-shared score proposal (group a multiple of 64)
    (default: 1 with mlp, else 0);
    compressed: 1 walks on the compressed aggregates of a tree built with compress=1 (uniform proposal,
    potential or smooth distance; samples <= 32 unless group is a multiple of 64);
    lod: 1 point-mass node terms, 2 adds the potential's quadrupole term where the node is far (a tree
    built with quadrupole=True; d = 2, group a multiple of 64, uniform proposal)."""
    import torch
    _dev(queries, "queries", (3,))
    nq = queries.shape[0]
    if out is None:
        out = torch.empty(nq, dtype=torch.float32, device=queries.device)
    _dev(out, "out")
    if paths is not None:
        _dev(paths, "paths", dtype=torch.int32)
        want = (nq, 4) if subdomains == 1 else (nq, tree.branching ** 3, max(samples, 1), 4)
        if tuple(paths.shape) != want:
            raise ValueError(f"paths must have shape {list(want)}")
    if mlp is not None:
        _dev(mlp, "mlp")
        if tuple(mlp.shape) != (MLP_NPARAM,):
            raise ValueError("mlp must have shape [MLP_NPARAM]")
    if proposal is None:
        proposal = 0 if mlp is None else 1
    o = EvalOpts(eps, alpha, group, rr_mode, int(proposal), batch,
                 None if paths is None else paths.data_ptr(), None if mlp is None else mlp.data_ptr(),
                 int(subdomains), int(compressed), int(lod))
    _check("sbh_eval", lib().sbh_eval(tree.handle, _ptr(queries), nq, int(kernel), float(beta), int(samples),
                                      C.c_uint64(seed), C.byref(o), _stream(stream), _ptr(out)))
    return out


def sbh_brute(sources, weights, normals, queries, kernel, eps=1e-3, alpha=100.0, fp64=False, out=None,
              stream=None):
    """Exact sum Eq. (1) on the GPU (sbh_brute); float64 result when fp64."""
    import torch
    _dev(sources, "sources", (3,)); _dev(weights, "weights"); _dev(normals, "normals", (3,))
    _dev(queries, "queries", (3,))
    nq = queries.shape[0]
    dt = torch.float64 if fp64 else torch.float32
    if out is None:
        out = torch.empty(nq, dtype=dt, device=queries.device)
    _dev(out, "out", dtype=dt)
    o = EvalOpts(eps, alpha, 1, 0, 0, 0, None, None)
    _check("sbh_brute", lib().sbh_brute(_ptr(sources), _ptr(weights), _ptr(normals), sources.shape[0],
                                        _ptr(queries), nq, int(kernel), C.byref(o), int(bool(fp64)),
                                        _stream(stream), _ptr(out)))
    return out


def _params(t, name):
    _dev(t, name)
    if tuple(t.shape) != (MLP_NPARAM,):
        raise ValueError(f"{name} must have shape [MLP_NPARAM]")
    return t


def sbh_mlp_forward(params, features, out=None, stream=None):
    """Logits [n, 8] of the proposal network for feature rows [n, 8] (sbh_mlp_forward)."""
    import torch
    _params(params, "params"); _dev(features, "features", (8,))
    if out is None:
        out = torch.empty_like(features)
    _dev(out, "out", (8,))
    if out.shape[0] != features.shape[0]:
        raise ValueError("out must have as many rows as features")
    _check("sbh_mlp_forward", lib().sbh_mlp_forward(_ptr(params), _ptr(features), features.shape[0],
                                                    _stream(stream), _ptr(out)))
    return out


def sbh_mlp_pairs(tree: Tree, queries, kernel, seed=0, max_depth=None, eps=1e-3, alpha=100.0, stream=None):
    """Training rows along uniform paths (sbh_mlp_pairs): features, targets, counts [rows, 8] and
    where [rows, 4] (int32), rows = nq * 8 * max_depth."""
    import torch
    _dev(queries, "queries", (3,))
    depth = tree.max_level if max_depth is None else int(max_depth)
    rows = queries.shape[0] * 8 * depth
    dev = queries.device
    X = torch.empty(rows, 8, dtype=torch.float32, device=dev)
    Tg = torch.empty_like(X); Cn = torch.empty_like(X)
    where = torch.empty(rows, 4, dtype=torch.int32, device=dev)
    o = EvalOpts(eps, alpha, 1, 0, 0, 0, None, None)
    _check("sbh_mlp_pairs", lib().sbh_mlp_pairs(tree.handle, _ptr(queries), queries.shape[0], int(kernel),
                                                C.c_uint64(seed), depth, C.byref(o), _stream(stream),
                                                _ptr(X), _ptr(Tg), _ptr(Cn), _ptr(where)))
    return X, Tg, Cn, where


def sbh_mlp_loss_grad(params, features, targets, counts, out=None, stream=None):
    """Mean loss and gradient (sbh_mlp_loss_grad): returns [MLP_GRAD_SIZE] (gradient, loss, rows)."""
    import torch
    _params(params, "params")
    for t, nm in ((features, "features"), (targets, "targets"), (counts, "counts")):
        _dev(t, nm, (8,))
    n = features.shape[0]
    if targets.shape[0] != n or counts.shape[0] != n:
        raise ValueError("features, targets and counts must have the same number of rows")
    if out is None:
        out = torch.empty(MLP_GRAD_SIZE, dtype=torch.float32, device=params.device)
    _dev(out, "out")
    _check("sbh_mlp_loss_grad", lib().sbh_mlp_loss_grad(_ptr(params), _ptr(features), _ptr(targets), _ptr(counts),
                                                        n, _stream(stream), _ptr(out)))
    return out


def sbh_mlp_train(params, adam_state, features, targets, counts, steps, batch_rows=4096, lr=1e-3, step0=0,
                  losses=None, stream=None):
    """Adam steps on params in place (sbh_mlp_train); adam_state [2 * MLP_NPARAM]; losses [steps] or None."""
    _params(params, "params"); _dev(adam_state, "adam_state")
    if tuple(adam_state.shape) != (2 * MLP_NPARAM,):
        raise ValueError("adam_state must have shape [2 * MLP_NPARAM]")
    for t, nm in ((features, "features"), (targets, "targets"), (counts, "counts")):
        _dev(t, nm, (8,))
    n = features.shape[0]
    if targets.shape[0] != n or counts.shape[0] != n:
        raise ValueError("features, targets and counts must have the same number of rows")
    if losses is not None:
        _dev(losses, "losses")
        if losses.numel() < steps:
            raise ValueError("losses must hold `steps` values")
    _check("sbh_mlp_train", lib().sbh_mlp_train(_ptr(params), _ptr(adam_state), _ptr(features), _ptr(targets),
                                                _ptr(counts), n, int(steps), int(batch_rows), float(lr), int(step0),
                                                _stream(stream), _ptr(losses)))
    return losses


MLP_NOALLOC_MAX_BATCH_ROWS = 32768


def sbh_mlp_train_noalloc(params, adam_state, features, targets, counts, steps, batch_rows=4096, lr=1e-3,
                          step0=0, losses=None, stream=None):
    """sbh_mlp_train on the library's static device workspace (sbh_mlp_train_noalloc): no allocation;
    batch_rows <= MLP_NOALLOC_MAX_BATCH_ROWS; calls overlapping on one GPU race."""
    _params(params, "params"); _dev(adam_state, "adam_state")
    if tuple(adam_state.shape) != (2 * MLP_NPARAM,):
        raise ValueError("adam_state must have shape [2 * MLP_NPARAM]")
    for t, nm in ((features, "features"), (targets, "targets"), (counts, "counts")):
        _dev(t, nm, (8,))
    n = features.shape[0]
    if targets.shape[0] != n or counts.shape[0] != n:
        raise ValueError("features, targets and counts must have the same number of rows")
    if losses is not None:
        _dev(losses, "losses")
        if losses.numel() < steps:
            raise ValueError("losses must hold `steps` values")
    _check("sbh_mlp_train_noalloc",
           lib().sbh_mlp_train_noalloc(_ptr(params), _ptr(adam_state), _ptr(features), _ptr(targets), _ptr(counts),
                                       n, int(steps), int(batch_rows), float(lr), int(step0), _stream(stream),
                                       _ptr(losses)))
    return losses


class Batch:
    """A batch plan (sbh_batch*): trees, query sets and outputs of many clouds evaluated by one
    launch per group, replayed from a HIP graph.  Keeps references to its trees and tensors."""

    def __init__(self, trees, queries, kernels, samples=1, group=64, eps=1e-3, alpha=100.0, rr_mode=0,
                 config=None, outs=None, stream=None):
        import torch
        if not (len(trees) == len(queries) == len(kernels)):
            raise ValueError("trees, queries and kernels must have the same length")
        self.trees, self.queries = list(trees), list(queries)
        self.outs = list(outs) if outs is not None else [torch.empty(q.shape[0], dtype=torch.float32, device=q.device)
                                                          for q in queries]
        items = (BatchItem * len(trees))()
        for i, (t, q, k, o) in enumerate(zip(self.trees, self.queries, kernels, self.outs)):
            _dev(q, "queries", (3,)); _dev(o, "out")
            if o.shape[0] != q.shape[0]:
                raise ValueError("each output must have one value per query")
            items[i] = BatchItem(t.handle, q.data_ptr(), o.data_ptr(), q.shape[0], int(k), 0)
        o = EvalOpts(eps, alpha, group, rr_mode, 0, 0, None, None)
        cfg = None if config is None else BatchConfig(*config, 0.0)
        h = C.c_void_p()
        _check("sbh_batch_create", lib().sbh_batch_create(items, len(trees), int(samples), C.byref(o),
                                                          None if cfg is None else C.byref(cfg), _stream(stream),
                                                          C.byref(h)))
        self._h = h
        c = BatchConfig()
        _check("sbh_batch_get_config", lib().sbh_batch_get_config(self._h, C.byref(c)))
        self.config = dict(tile_waves=c.tile_waves, waves_per_simd=c.waves_per_simd, heavy_first=c.heavy_first,
                           ms=c.ms)

    def launch(self, seed=0, batch=0, stream=None):
        _check("sbh_batch_launch", lib().sbh_batch_launch(self._h, C.c_uint64(seed), batch, _stream(stream)))
        return self.outs

    def free(self):
        if getattr(self, "_h", None):
            lib().sbh_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sbh_free(tree: Tree):
    tree.free()
