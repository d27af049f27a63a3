"""Seeded synthetic inputs for the stochastic Barnes-Hut workloads.

This module only draws inputs (sources, weights, normals, queries).  It holds
none of the estimator's arithmetic and is the one module that both the FP64
oracle tests and the HIP path use.  Every generator is a pure function of its
seed (NumPy PCG64), so a test on the CPU and a run on the GPU see the same
bytes.

The paper's own datasets (the scanned and modelled meshes of its results
section) are not available; the shapes below stand in for them with the same
sizes: 2^20..2^22 oriented surface samples carrying area weights, queries on a
1000 x 1000 slice plane or uniform in a box (results section, "Applications"
and Table 1).

Workloads
---------
c1  4096 sources uniform in [0,1]^3, weights U[0.5,1.5]; 4096 queries uniform
    in [-0.5,1.5]^3; softened potential.
c2  2^20 area-uniform samples of a closed star-shaped surface (radius
    1 + 0.15 g, g a random real spherical-harmonic field of degrees 1..6
    scaled to unit RMS over the sphere) with outward normals and area
    weights; queries: the 1000 x 1000 pixel centres of z=0 over [-1.5,1.5]^2.
c3  2^22 area-uniform samples of the surface of a union of 32 random
    ellipsoids in [0,1]^3 (semi-axes U[0.05,0.3], random rotations), area
    weights; 2^20 queries uniform in [-0.2,1.2]^3.
c4  64 clouds with log-uniform sizes (sources 2^12..2^20, queries
    2^14..2^18); kernel and geometry cycle potential / winding / smooth.
c5  2^22 samples of a c2-style surface (seed 5000; seeds 5001..5016 for
    training clouds); potential kernel on the z=0 plane.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

POTENTIAL, WINDING, SMOOTHDIST = 0, 1, 2


@dataclasses.dataclass
class Cloud:
    """One source set with its queries. All arrays are float32, C-contiguous."""
    sources: np.ndarray            # [M,3]
    weights: np.ndarray            # [M]
    normals: np.ndarray | None     # [M,3] unit outward normals, or None
    queries: np.ndarray            # [N,3]
    kernel: int                    # POTENTIAL / WINDING / SMOOTHDIST
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.sources.shape[0])

    @property
    def n(self) -> int:
        return int(self.queries.shape[0])


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ----------------------------------------------------------------------------
# Basic shapes
# ----------------------------------------------------------------------------

def uniform_cube(m: int, n: int, seed: int, src_box=(0.0, 1.0), qry_box=(-0.5, 1.5),
                 wlo=0.5, whi=1.5) -> Cloud:
    rng = np.random.Generator(np.random.PCG64(seed))
    src = rng.uniform(src_box[0], src_box[1], size=(m, 3))
    w = rng.uniform(wlo, whi, size=m)
    q = rng.uniform(qry_box[0], qry_box[1], size=(n, 3))
    return Cloud(_f32(src), _f32(w), None, _f32(q), POTENTIAL, name=f"uniform{m}x{n}")


def plane_queries(res: int = 1000, half: float = 1.5, z: float = 0.0) -> np.ndarray:
    """Pixel centres of a res x res grid on the plane z=const over [-half,half]^2,
    row-major (y outer, x inner)."""
    t = (np.arange(res, dtype=np.float64) + 0.5) * (2.0 * half / res) - half
    yy, xx = np.meshgrid(t, t, indexing="ij")
    q = np.stack([xx.ravel(), yy.ravel(), np.full(res * res, z)], axis=1)
    return _f32(q)


def shuffle_queries(q: np.ndarray, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Seeded permutation of a query set. Returns (shuffled, perm) with
    shuffled[i] = q[perm[i]]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(q.shape[0])
    return _f32(q[perm]), perm


# ----------------------------------------------------------------------------
# Icosphere + real spherical harmonics (star-shaped surfaces)
# ----------------------------------------------------------------------------

def icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere by `level` 1:4 subdivisions; faces are counter-clockwise
    seen from outside (outward orientation). 20*4^level faces."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for _ in range(level):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
        e.sort(axis=1)
        key = e[:, 0] * (1 << 32) + e[:, 1]
        uk, inv = np.unique(key, return_inverse=True)
        a = uk >> 32
        b = uk & ((1 << 32) - 1)
        mid = v[a] + v[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = v.shape[0]
        v = np.concatenate([v, mid], axis=0)
        nf = f.shape[0]
        m01 = base + inv[:nf]
        m12 = base + inv[nf:2 * nf]
        m20 = base + inv[2 * nf:]
        f = np.concatenate([
            np.stack([f[:, 0], m01, m20], 1),
            np.stack([f[:, 1], m12, m01], 1),
            np.stack([f[:, 2], m20, m12], 1),
            np.stack([m01, m12, m20], 1)], axis=0)
    return v, f


def _real_sph_harm_basis(lmax: int, dirs: np.ndarray, lmin: int = 1) -> np.ndarray:
    """Orthonormal real spherical harmonics Y_lm(dir) for lmin<=l<=lmax, as
    columns. dirs: [K,3] unit vectors."""
    from scipy.special import sph_harm_y
    polar = np.arccos(np.clip(dirs[:, 2], -1.0, 1.0))
    azim = np.arctan2(dirs[:, 1], dirs[:, 0])
    cols = []
    for l in range(lmin, lmax + 1):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), polar, azim)
            if m > 0:
                cols.append(math.sqrt(2.0) * (-1) ** m * y.real)
            elif m < 0:
                cols.append(math.sqrt(2.0) * (-1) ** m * y.imag)
            else:
                cols.append(y.real)
    return np.stack(cols, axis=1)


def star_radius_fn(seed: int, lmax: int = 6, amp: float = 0.15):
    """r(dir) = 1 + amp * g(dir), g = sum_{l=1..lmax} c_lm Y_lm with
    c ~ N(0,1), rescaled so that g has unit RMS over the sphere (for an
    orthonormal basis, mean(g^2) = sum c^2 / (4 pi))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ncoef = (lmax + 1) ** 2 - 1
    c = rng.standard_normal(ncoef)
    c *= math.sqrt(4.0 * math.pi / float(np.sum(c * c)))

    def radius(dirs):
        return 1.0 + amp * (_real_sph_harm_basis(lmax, dirs) @ c)
    return radius


def sample_triangles(v: np.ndarray, f: np.ndarray, m: int, rng) -> tuple:
    """m area-uniform samples on a triangle mesh: triangle chosen with
    probability proportional to area, uniform barycentric point. Returns
    (points, unit face normals, total area). Normals follow face winding."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    cr = np.cross(b - a, c - a)
    dbl = np.linalg.norm(cr, axis=1)
    area = 0.5 * dbl
    total = float(area.sum())
    cdf = np.cumsum(area)
    cdf /= cdf[-1]
    tri = np.searchsorted(cdf, rng.random(m), side="right")
    tri = np.minimum(tri, f.shape[0] - 1)
    r1 = np.sqrt(rng.random(m))
    r2 = rng.random(m)
    pts = (1 - r1)[:, None] * a[tri] + (r1 * (1 - r2))[:, None] * b[tri] + (r1 * r2)[:, None] * c[tri]
    nrm = cr[tri] / dbl[tri][:, None]
    return pts, nrm, total


def star_surface(m: int, seed: int, level: int = 7, amp: float = 0.15):
    """Area-uniform oriented samples of a random star-shaped closed surface
    (icosphere of `level`, radially displaced). Returns points, outward
    normals, area weights (total area / m), and the radius function."""
    radius = star_radius_fn(seed, amp=amp)
    v, f = icosphere(level)
    r = radius(v)
    if np.min(r) <= 0.05:
        raise ValueError("star surface radius not positive; choose another seed")
    vd = v * r[:, None]
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    pts, nrm, total = sample_triangles(vd, f, m, rng)
    w = np.full(m, total / m)
    return pts, nrm, w, radius


# ----------------------------------------------------------------------------
# Union of ellipsoids
# ----------------------------------------------------------------------------

def _random_rotations(k: int, rng) -> np.ndarray:
    """Uniform random rotations from unit quaternions (normalised Gaussians)."""
    qv = rng.standard_normal((k, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], 1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], 1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], 1)], 1)


def _ellipsoid_area(a, b, c):
    # Thomsen's approximation (relative error below about 1.1%); it only sets
    # the per-ellipsoid sampling proportions and the weight scale.
    p = 1.6075
    return 4 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3) ** (1 / p)


def ellipsoid_union(m: int, seed: int, k: int = 32, amin=0.05, amax=0.3):
    """Area-uniform samples of the boundary of a union of k random ellipsoids.

    Each sample: choose an ellipsoid with probability proportional to its
    (approximate) area, draw an area-uniform point on it by rejection on the
    area element of the sphere-to-ellipsoid map, and drop it when it lies
    strictly inside another ellipsoid. Weight = estimated union area / m.
    Returns (points, outward normals, weights, description dict)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.random((k, 3))
    axes = rng.uniform(amin, amax, size=(k, 3))
    rots = _random_rotations(k, rng)
    areas = np.array([_ellipsoid_area(*ax) for ax in axes])
    cdf = np.cumsum(areas) / areas.sum()
    out_p, out_n = [], []
    got = 0
    drawn = 0
    kept = 0
    while got < m:
        batch = max(1 << 16, int((m - got) * 1.6))
        e = np.minimum(np.searchsorted(cdf, rng.random(batch), side="right"), k - 1)
        u = rng.standard_normal((batch, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        ax = axes[e]
        # area element of x = A u on the unit sphere is prod(a) * |A^{-1} u|
        g = np.prod(ax, axis=1) * np.linalg.norm(u / ax, axis=1)
        gmax = np.prod(ax, axis=1) / np.min(ax, axis=1)
        acc = rng.random(batch) * gmax < g
        e, u, ax = e[acc], u[acc], ax[acc]
        local = u * ax
        nloc = u / ax
        nloc /= np.linalg.norm(nloc, axis=1, keepdims=True)
        R = rots[e]
        pts = np.einsum("kij,kj->ki", R, local) + centres[e]
        nrm = np.einsum("kij,kj->ki", R, nloc)
        inside_other = np.zeros(pts.shape[0], dtype=bool)
        for i in range(k):
            d = (pts - centres[i]) @ rots[i]          # into ellipsoid i's frame
            s = np.sum((d / axes[i]) ** 2, axis=1)
            inside_other |= (s < 1.0 - 1e-9) & (e != i)
        drawn += pts.shape[0]
        kept_mask = ~inside_other
        kept += int(kept_mask.sum())
        pts, nrm = pts[kept_mask], nrm[kept_mask]
        take = min(m - got, pts.shape[0])
        out_p.append(pts[:take])
        out_n.append(nrm[:take])
        got += take
    pts = np.concatenate(out_p)
    nrm = np.concatenate(out_n)
    union_area = float(areas.sum()) * kept / max(drawn, 1)
    w = np.full(m, union_area / m)
    return pts, nrm, w, dict(centres=centres, axes=axes, rots=rots, union_area=union_area)


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

def c1(seed: int = 1001) -> Cloud:
    cl = uniform_cube(4096, 4096, seed)
    cl.name = "c1_uniform4096_potential"
    cl.meta = dict(eps=1e-3, beta=2.0, samples=1, leaf_size=8)
    return cl


def c2(seed: int = 1002, m: int = 1 << 20, res: int = 1000) -> Cloud:
    pts, nrm, w, radius = star_surface(m, seed)
    q = plane_queries(res, 1.5, 0.0)
    cl = Cloud(_f32(pts), _f32(w), _f32(nrm), q, WINDING, name="c2_star2^20_winding_plane1000")
    cl.meta = dict(beta=2.0, samples=1, leaf_size=8, radius=radius)
    return cl


def c3(seed: int = 1003, m: int = 1 << 22, n: int = 1 << 20) -> Cloud:
    pts, nrm, w, info = ellipsoid_union(m, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    q = rng.uniform(-0.2, 1.2, size=(n, 3))
    cl = Cloud(_f32(pts), _f32(w), _f32(nrm), _f32(q), SMOOTHDIST, name="c3_ellipsoids2^22_smooth")
    cl.meta = dict(alpha=100.0, samples=(1, 4), leaf_size=8, **info)
    return cl


def c5(seed: int = 5000, m: int = 1 << 22, res: int = 1000) -> Cloud:
    pts, nrm, w, radius = star_surface(m, seed)
    q = plane_queries(res, 1.5, 0.0)
    cl = Cloud(_f32(pts), _f32(w), _f32(nrm), q, POTENTIAL, name="c5_star2^22_potential_plane1000")
    cl.meta = dict(eps=1e-3, beta=2.0, samples=1, leaf_size=8, radius=radius)
    return cl


def c5_training_seeds():
    return list(range(5001, 5017))


def c4_specs(seed: int = 2000, count: int = 64):
    """Sizes and kernels of the batched workload (cheap: no geometry)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ms = np.rint(2.0 ** rng.uniform(12, 20, size=count)).astype(np.int64)
    ns = np.rint(2.0 ** rng.uniform(14, 18, size=count)).astype(np.int64)
    return [dict(index=b, m=int(ms[b]), n=int(ns[b]), kernel=b % 3, seed=seed + b) for b in range(count)]


def c4_cloud(spec: dict) -> Cloud:
    m, n, kern, s = spec["m"], spec["n"], spec["kernel"], spec["seed"]
    rng = np.random.Generator(np.random.PCG64(s))
    if kern == POTENTIAL:
        cl = uniform_cube(m, n, s)
    elif kern == WINDING:
        pts, nrm, w, _ = star_surface(m, s, level=5)
        q = rng.uniform(-1.5, 1.5, size=(n, 3))
        cl = Cloud(_f32(pts), _f32(w), _f32(nrm), _f32(q), WINDING)
    else:
        pts, nrm, w, _ = ellipsoid_union(m, s, k=8)
        q = rng.uniform(-0.2, 1.2, size=(n, 3))
        cl = Cloud(_f32(pts), _f32(w), _f32(nrm), _f32(q), SMOOTHDIST)
    cl.name = f"c4_cloud{spec['index']}"
    return cl


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c5": c5}
