"""FP64 CPU oracle for the stochastic Barnes-Hut estimator.

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
CPU-baseline leg.  The product path (the HIP library and its binding) never
imports this package, and this package imports nothing from the product.

Thin ctypes wrapper over sbh_oracle.c; see that file for the passages of the
paper each function follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

POTENTIAL, WINDING, SMOOTHDIST, LINEAR = 0, 1, 2, 99

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        i64, i32, u32, u64, f64 = C.c_int64, C.c_int, C.c_uint32, C.c_uint64, C.c_double
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_brute.argtypes = [P, P, P, i64, P, i64, i32, f64, f64, P, i32]
        L.orc_tree_build.argtypes = [P, P, P, i64, i32, i32, i32]
        L.orc_tree_build.restype = P
        L.orc_tree_free.argtypes = [P]
        L.orc_sbh_vote.argtypes = [P, P, i64, i32, f64, f64, i32, u64, i32, u32, P, P, P, P, P, P, i32]
        L.orc_sbh_vote_expect.argtypes = [P, P, i64, i32, f64, f64, P, i32]
        L.orc_tree_set_lod.argtypes = [P, i32]
        L.orc_tree_set_lod.restype = i32
        L.orc_tree_quad.argtypes = [P, P]
        L.orc_node_term.argtypes = [P, i32, f64, f64, i64, P]
        L.orc_node_term.restype = f64
        L.orc_tree_set_compressed.argtypes = [P, i32]
        L.orc_tree_set_compressed.restype = i32
        L.orc_tree_compressed.argtypes = [P, P, P]
        L.orc_tree_set_diam_mode.argtypes = [P, i32]
        L.orc_tree_set_diam_mode.restype = i32
        L.orc_tree_num_nodes.argtypes = [P]
        L.orc_tree_num_nodes.restype = i64
        L.orc_tree_meta.argtypes = [P, P]
        L.orc_tree_export.argtypes = [P] + [P] * 11
        L.orc_bh.argtypes = [P, P, i64, i32, f64, f64, f64, i32, P, P, P, i32]
        L.orc_sbh.argtypes = [P, P, i64, i32, f64, f64, i32, u64, i32, u32, i32, P, P, P, i64, P, P, P, P, P, i32]
        L.orc_sbh_expect.argtypes = [P, P, i64, i32, f64, f64, i32, P, i32, P, i32]
        L.orc_sbh_cut.argtypes = [P, P, i64, i32, f64, f64, i32, u64, i32, i32, u32, i32, f64, P, i32, P, P, P, P,
                                  P, i32]
        L.orc_term_sens.argtypes = [i32, f64, f64, P, f64, P, P, P]
        L.orc_refine_all.argtypes = [P, P, i64, i32, f64, f64, P]
        L.orc_mlp_nparam.restype = i32
        L.orc_f16_round.argtypes = [C.c_float]
        L.orc_f16_round.restype = C.c_float
        L.orc_mlp_features.argtypes = [P, P, P, i64, P]
        L.orc_mlp_forward.argtypes = [P, P, i64, i32, P]
        L.orc_mlp_loss_grad.argtypes = [P, P, P, P, i64, i32, P]
        L.orc_mlp_loss_grad.restype = f64
        L.orc_child_targets.argtypes = [P, P, P, i64, i32, f64, f64, P, P]
        L.orc_mlp_pairs.argtypes = [P, i64, u64, i32, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: ctr 4 x uint32, key 2 x uint32 -> 4 x uint32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def brute(sources, weights, normals, queries, kernel, eps=1e-3, alpha=100.0, threads=0):
    """Eq. (1) in FP64 with compensated summation. Returns the raw sum F."""
    s = _f32(sources, (-1, 3)); w = _f32(weights).ravel(); q = _f32(queries, (-1, 3))
    nrm = None if normals is None else _f32(normals, (-1, 3))
    out = np.zeros(q.shape[0], dtype=np.float64)
    lib().orc_brute(_p(s), _p(w), _p(nrm), s.shape[0], _p(q), q.shape[0], kernel, eps, alpha, _p(out), threads)
    return out


def term_sens(kernel, p, m, dip, q, eps=1e-3, alpha=100.0):
    """One term f(p, q) (weight m, dipole dip) and its centre sensitivity |grad_p f| |p|."""
    pp = np.ascontiguousarray(p, np.float64); dd = np.ascontiguousarray(dip, np.float64)
    qq = np.ascontiguousarray(q, np.float64); out = np.zeros(2)
    lib().orc_term_sens(kernel, eps, alpha, _p(pp), float(m), _p(dd), _p(qq), _p(out))
    return float(out[0]), float(out[1])


def smooth_distance(F, alpha=100.0):
    """Smooth-distance post-transform -log(F)/alpha (results section)."""
    F = np.asarray(F, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return -np.log(F) / alpha


class Tree:
    """Oracle tree: d in {2,4,8}, leaf_size, max_level (0 = deepest allowed)."""

    def __init__(self, sources, weights, normals=None, d=2, leaf_size=8, max_level=0):
        self._s = _f32(sources, (-1, 3)); self._w = _f32(weights).ravel()
        self._n = None if normals is None else _f32(normals, (-1, 3))
        h = lib().orc_tree_build(_p(self._s), _p(self._w), _p(self._n), self._s.shape[0], d, leaf_size, max_level)
        if not h:
            raise ValueError("oracle tree build rejected its arguments")
        self._h = C.c_void_p(h)
        meta = np.zeros(10)
        lib().orc_tree_meta(self._h, _p(meta))
        self.lo = meta[0:3].astype(np.float32)
        self.side = np.float32(meta[3]); self.inv_side = np.float32(meta[4])
        self.d = int(meta[5]); self.leaf_size = int(meta[6]); self.max_level = int(meta[7])
        self.depth = int(meta[8]); self.m = int(meta[9])
        self.n_nodes = int(lib().orc_tree_num_nodes(self._h))
        n = self.n_nodes
        self.begin = np.zeros(n, np.int64); self.count = np.zeros(n, np.int64)
        self.level = np.zeros(n, np.int32); self.first_child = np.zeros(n, np.int64)
        self.nchild = np.zeros(n, np.int32); self.digit = np.zeros(n, np.int32)
        self.parent = np.zeros(n, np.int64); self.agg = np.zeros((n, 8)); self.spread2 = np.zeros(n)
        self.perm = np.zeros(self.m, np.int64); self.codes = np.zeros(self.m, np.uint64)
        lib().orc_tree_export(self._h, _p(self.begin), _p(self.count), _p(self.level), _p(self.first_child),
                              _p(self.nchild), _p(self.digit), _p(self.parent), _p(self.agg), _p(self.perm),
                              _p(self.codes), _p(self.spread2))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_tree_free(h)
            self._h = None

    def set_compressed(self, on=True):
        """Use the compressed interior aggregates (binary16 centre-of-mass offsets relative to the
        decoded parent, in units of the node's cell side, and binary16 mass fractions of the decoded
        parent) in every node term and far-field ratio; points stay exact."""
        if lib().orc_tree_set_compressed(self._h, int(bool(on))) != 0:
            raise ValueError("the compressed aggregates exclude lod 2")
        self._cmp = bool(on)

    def compressed(self):
        """(decoded aggregates [n, 4] float64: com xyz, mass; stored codes [n, 4] float32: offsets
        x, y, z and mass fraction, zero for the root)."""
        lib().orc_tree_set_compressed(self._h, 1)
        qa = np.zeros((self.n_nodes, 4)); code = np.zeros((self.n_nodes, 4), np.float32)
        lib().orc_tree_compressed(self._h, _p(qa), _p(code))
        lib().orc_tree_set_compressed(self._h, int(getattr(self, "_cmp", False)))
        return qa, code

    def set_lod(self, lod):
        """Node terms of order 1 (point masses, the default) or 2 (plus the potential's quadrupole
        term wherever the node is far: |q - com| >= |B|)."""
        if lib().orc_tree_set_lod(self._h, int(lod)) != 0:
            raise ValueError("lod must be 1 or 2, and 2 excludes the compressed aggregates")

    def quad(self):
        """Second-moment tensors [n, 6] (xx, yy, zz, xy, xz, yz) about each node's centre of mass."""
        out = np.zeros((self.n_nodes, 6))
        lib().orc_tree_quad(self._h, _p(out))
        return out

    def node_term(self, i, q, kernel=0, eps=1e-3, alpha=100.0):
        """Node i's term at query q under the tree's lod."""
        qq = np.ascontiguousarray(q, dtype=np.float64)
        return lib().orc_node_term(self._h, int(kernel), float(eps), float(alpha), int(i), _p(qq))

    def set_diam_mode(self, mode):
        """The reading of |B| for a study of the paper's wording (0, the default and the one the
        GPU implements: the cell diagonal; 1: the cell side; 2: the diagonal of the axis-aligned
        box of the node's own points, 0 for a single point)."""
        if lib().orc_tree_set_diam_mode(self._h, int(mode)) != 0:
            raise ValueError("diam mode must be 0, 1 or 2")

    @property
    def internal(self):
        return (self.count > self.leaf_size) & (self.level < self.max_level)

    def bh(self, queries, kernel, beta, group=1, eps=1e-3, alpha=100.0, threads=0):
        """Algorithm 1; returns (F, min relative margin |b-beta|/beta, nodes visited per group)."""
        q = _f32(queries, (-1, 3)); n = q.shape[0]
        out = np.zeros(n); mg = np.zeros(n); vis = np.zeros(n, np.int64)
        lib().orc_bh(self._h, _p(q), n, kernel, eps, alpha, float(beta), group, _p(out), _p(mg), _p(vis), threads)
        return out, mg, vis

    def sbh(self, queries, kernel, samples=1, seed=0, group=1, batch=0, rr_mode=0, eps=1e-3, alpha=100.0,
            paths=False, index=None, params=None, tile_queries=None, threads=0):
        """Algorithm 2 driven by Philox; returns dict(F, margin, absum, sens[, paths]).
        index: optional original query indices (random stream ids) of a query subset;
        params: learned proposal; tile_queries: the full query set, selecting the tile-shared
        score proposal (tiles of 64 consecutive indices of it)."""
        q = _f32(queries, (-1, 3)); n = q.shape[0]
        idx = None if index is None else np.ascontiguousarray(index, dtype=np.int64)
        prm = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        out = np.zeros(n); mg = np.zeros(n); ab = np.zeros(n); sn = np.zeros(n)
        d3 = self.d ** 3
        pth = np.zeros((n, d3, samples, 4), np.int32) if paths else None
        tq = None if tile_queries is None else _f32(tile_queries, (-1, 3))
        lib().orc_sbh(self._h, _p(q), n, kernel, eps, alpha, samples, seed, group, batch, rr_mode, _p(idx), _p(prm),
                      _p(tq), 0 if tq is None else tq.shape[0], _p(out), _p(mg), _p(ab), _p(sn), _p(pth), threads)
        r = dict(F=out, margin=mg, absum=ab, sens=sn)
        if paths:
            r["paths"] = pth
        return r

    def sbh_vote(self, queries, kernel, samples=1, seed=0, group=64, batch=0, eps=1e-3, alpha=100.0,
                 paths=False, index=None, threads=0):
        """Algorithm 2 with the roulette voted over each tile (rr_mode 3): every query of a tile of 64
        consecutive indices (sharing one stream: group a multiple of 64) continues with the largest
        Eq. (5) probability among the tile's queries.  index: original indices of the queries (whole
        tiles, in order); returns dict(F, margin, absum, sens[, paths])."""
        q = _f32(queries, (-1, 3)); n = q.shape[0]
        idx = None if index is None else np.ascontiguousarray(index, dtype=np.int64)
        out = np.zeros(n); mg = np.zeros(n); ab = np.zeros(n); sn = np.zeros(n)
        d3 = self.d ** 3
        pth = np.zeros((n, d3, samples, 4), np.int32) if paths else None
        lib().orc_sbh_vote(self._h, _p(q), n, kernel, eps, alpha, samples, seed, group, batch, _p(idx), _p(out),
                           _p(mg), _p(ab), _p(sn), _p(pth), threads)
        r = dict(F=out, margin=mg, absum=ab, sens=sn)
        if paths:
            r["paths"] = pth
        return r

    def vote_expect(self, queries, kernel, eps=1e-3, alpha=100.0, threads=0):
        """Exact expectation (Theorem 1) of the one-sample estimator with the roulette voted over tiles
        of 64 consecutive queries."""
        q = _f32(queries, (-1, 3)); out = np.zeros(q.shape[0])
        lib().orc_sbh_vote_expect(self._h, _p(q), q.shape[0], kernel, eps, alpha, _p(out), threads)
        return out

    def sbh_cut(self, queries, kernel, beta_low, samples=1, seed=0, group=64, vote=64, batch=0, rr_mode=0,
                eps=1e-3, alpha=100.0, index=None, expect=False, threads=0):
        """The estimator stratified by the Barnes-Hut cut D(q, beta_low), voted over groups of `vote`
        consecutive queries (Section 3.3.1); returns dict(F, margin, absum, sens, digest [n, 4]:
        subdomains, leaves summed exactly, accepted steps, sum of end levels).  expect: the exact
        expectation (Theorem 1) instead of a sample."""
        q = _f32(queries, (-1, 3)); n = q.shape[0]
        idx = None if index is None else np.ascontiguousarray(index, dtype=np.int64)
        out = np.zeros(n); mg = np.zeros(n); ab = np.zeros(n); sn = np.zeros(n)
        dg = np.zeros((n, 4), np.int32)
        lib().orc_sbh_cut(self._h, _p(q), n, kernel, eps, alpha, samples, seed, group, vote, batch, rr_mode,
                          float(beta_low), _p(idx), int(bool(expect)), _p(out), _p(mg), _p(ab), _p(sn), _p(dg),
                          threads)
        return dict(F=out, margin=mg, absum=ab, sens=sn, digest=dg)

    def expect(self, queries, kernel, rr_mode=0, eps=1e-3, alpha=100.0, params=None, tiles=False, threads=0):
        """Exact expectation of the one-sample estimator (Theorem 1), optionally with the learned
        proposal or the tile-shared score proposal (tiles of 64 consecutive queries)."""
        q = _f32(queries, (-1, 3)); out = np.zeros(q.shape[0])
        prm = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        lib().orc_sbh_expect(self._h, _p(q), q.shape[0], kernel, eps, alpha, rr_mode, _p(prm), int(bool(tiles)),
                             _p(out), threads)
        return out

    def mlp_features(self, nodes, queries):
        """Proposal features (float64 [n, 8]) of (internal node, query) pairs."""
        nd = np.ascontiguousarray(nodes, np.int64)
        q = _f32(queries, (-1, 3)); out = np.zeros((len(nd), 8))
        lib().orc_mlp_features(self._h, _p(nd), _p(q), len(nd), _p(out))
        return out

    def mlp_pairs(self, nq, seed=0, lmax=None):
        """Training (query, node) pairs along uniform paths: node [nq, d^3, lmax] (-1 = none)."""
        lmax = self.max_level if lmax is None else lmax
        d3 = self.d ** 3
        nd = np.zeros((nq, d3, lmax), np.int64)
        lib().orc_mlp_pairs(self._h, nq, seed, lmax, _p(nd))
        return nd

    def training_set(self, queries, kernel, seed=0, lmax=None, eps=1e-3, alpha=100.0):
        """Features (float32), targets and child counts of every training pair
        (rows [nq*d^3*lmax], valid mask)."""
        q = _f32(queries, (-1, 3))
        nd = self.mlp_pairs(q.shape[0], seed, lmax)
        rows = nd.reshape(-1)
        valid = rows >= 0
        qi = np.repeat(np.arange(q.shape[0]), nd.shape[1] * nd.shape[2])
        X = np.zeros((rows.size, 8), np.float32); Tg = np.zeros_like(X); Cn = np.zeros_like(X)
        if valid.any():
            X[valid] = self.mlp_features(rows[valid], q[qi[valid]]).astype(np.float32)
            Tg[valid], Cn[valid] = self.child_targets(rows[valid], q[qi[valid]], kernel, eps, alpha)
        return X, Tg, Cn, valid

    def child_targets(self, nodes, queries, kernel, eps=1e-3, alpha=100.0):
        """Normalised per-slot residual targets and child counts for internal nodes."""
        nd = np.ascontiguousarray(nodes, np.int64); q = _f32(queries, (-1, 3))
        tg = np.zeros((len(nd), 8), np.float32); cn = np.zeros((len(nd), 8), np.float32)
        lib().orc_child_targets(self._h, _p(nd), _p(q), len(nd), kernel, eps, alpha, _p(tg), _p(cn))
        return tg, cn

    def refine_all(self, queries, kernel, eps=1e-3, alpha=100.0):
        """Telescoping sum with every node refined (Eqs. (3)-(4))."""
        q = _f32(queries, (-1, 3)); out = np.zeros(q.shape[0])
        lib().orc_refine_all(self._h, _p(q), q.shape[0], kernel, eps, alpha, _p(out))
        return out


MLP_NPARAM = 1608
MLP_LAMBDA = 0.125


def f16_round(x):
    return float(lib().orc_f16_round(float(x)))


def mlp_forward(params, x, mode=1):
    """Logits of the proposal network for feature rows x [n, 8] (mode 1: binary16 emulation)."""
    prm = np.ascontiguousarray(params, np.float32); xx = _f32(x, (-1, 8))
    z = np.zeros((xx.shape[0], 8))
    lib().orc_mlp_forward(_p(prm), _p(xx), xx.shape[0], mode, _p(z))
    return z


def mlp_loss_grad(params, x, targets, counts, mode=0):
    """Mean soft cross-entropy and its float64 gradient."""
    prm = np.ascontiguousarray(params, np.float32); xx = _f32(x, (-1, 8))
    tg = _f32(targets, (-1, 8)); cn = _f32(counts, (-1, 8))
    g = np.zeros(MLP_NPARAM)
    loss = lib().orc_mlp_loss_grad(_p(prm), _p(xx), _p(tg), _p(cn), xx.shape[0], mode, _p(g))
    return loss, g
