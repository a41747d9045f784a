"""Boundary meshes of the kind the paper's 3D Laplace BEM problems live on.

The paper's experiments discretise integral equations on surfaces with the
d=3 Laplace kernel (Sec. 6.1, "Mathematical problems") but do not publish the
geometries.  The stand-in used here is the unit sphere triangulated by
repeated midpoint subdivision of an icosahedron, one degree of freedom per
flat triangle (its centroid, with the flat triangle's area as quadrature
weight).  Ellipsoids are the same triangulation with the vertices scaled per
axis.

Everything in this file is input generation only.
"""
from __future__ import annotations

import itertools

import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _icosahedron():
    """Vertices (0,+-1,+-phi) in the three cyclic orders and the 20 faces.

    Faces are the vertex triples that are mutually at edge length 2 (before
    normalisation), enumerated in lexicographic index order so the mesh is
    deterministic without relying on a convex-hull library.
    """
    v = []
    for a, b in itertools.product((-1.0, 1.0), (-_PHI, _PHI)):
        v.append((0.0, a, b))
        v.append((a, b, 0.0))
        v.append((b, 0.0, a))
    v = np.array(v, dtype=np.float64)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    adj = np.abs(d - 2.0) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    assert len(faces) == 20
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, np.array(faces, dtype=np.int64)


def _subdivide(verts, faces):
    """Split every triangle into four at its edge midpoints (projected to the
    unit sphere)."""
    verts = [tuple(p) for p in verts]
    cache = {}

    def mid(a, b):
        key = (a, b) if a < b else (b, a)
        idx = cache.get(key)
        if idx is None:
            p = (np.array(verts[a]) + np.array(verts[b])) * 0.5
            p /= np.linalg.norm(p)
            verts.append(tuple(p))
            idx = len(verts) - 1
            cache[key] = idx
        return idx

    out = []
    for a, b, c in faces:
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        out.extend([(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)])
    return np.array(verts, dtype=np.float64), np.array(out, dtype=np.int64)


def _mesh(level):
    v, f = _icosahedron()
    for _ in range(level):
        v, f = _subdivide(v, f)
    return v, f


def _centroids_areas(v, f):
    p0, p1, p2 = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    cen = (p0 + p1 + p2) / 3.0
    area = 0.5 * np.linalg.norm(np.cross(p1 - p0, p2 - p0), axis=1)
    return np.ascontiguousarray(cen), np.ascontiguousarray(area)


def icosphere(level: int):
    """Flat-triangle centroids (n x 3) and areas (n) of the level-`level`
    icosphere; n = 20 * 4**level."""
    v, f = _mesh(level)
    return _centroids_areas(v, f)


def ellipsoid_surface(level: int, semi_axes):
    """Same triangulation with vertices scaled by the semi-axes (a, b, c)."""
    v, f = _mesh(level)
    v = v * np.asarray(semi_axes, dtype=np.float64)[None, :]
    return _centroids_areas(v, f)


def segment(n: int, a: float = 0.0, b: float = 1.0):
    """Midpoints (n x 3, second and third coordinates zero) and lengths of the
    uniform partition of [a, b] into n panels: the d = 1 domain."""
    h = (b - a) / n
    xyz = np.zeros((n, 3))
    xyz[:, 0] = a + (np.arange(n) + 0.5) * h
    return xyz, np.full(n, h)


def circle(n: int, radius: float = 0.5):
    """Chord midpoints (n x 3, third coordinate zero) and chord lengths of the
    regular n-gon inscribed in the circle of the given radius (vertex k at
    angle 2 pi k / n): the d = 2 boundary.  With radius <= 0.5 every pair
    of points is within unit distance."""
    th = 2.0 * np.pi * np.arange(n + 1) / n
    v = radius * np.stack([np.cos(th), np.sin(th)], axis=1)
    mid = 0.5 * (v[:-1] + v[1:])
    xyz = np.zeros((n, 3))
    xyz[:, :2] = mid
    return xyz, np.linalg.norm(v[1:] - v[:-1], axis=1)


def rhs_uniform(seed: int, n: int):
    """x ~ U(-1, 1), drawn from numpy's PCG64 generator."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def rhs_normal(seed: int, n: int, nrhs: int):
    """n x nrhs standard normal right-hand sides, column-major (Fortran)."""
    b = np.random.default_rng(seed).standard_normal((n, nrhs))
    return np.asfortranarray(b)


# Workload descriptions: geometry level, leaf size, eta, truncation and RHS.
CONFIGS = {
    # n=1280, leaf 32, eta 2, fixed rank 8, FP64; RHS = A x_true.
    "c1": dict(level=3, leaf=32, eta=2.0, fixed_rank=8, eps=0.0, cap=32,
               precision="fp64", rhs="axtrue", seed=0, nrhs=1),
    # n=20480, leaf 64, eta 2, eps 1e-6 (cap 32), FP64, 8 normal RHS.
    "c2": dict(level=5, leaf=64, eta=2.0, fixed_rank=0, eps=1e-6, cap=32,
               precision="fp64", rhs="normal", seed=1, nrhs=8),
    # n=81920, leaf 64, eta 2, eps 1e-5 (cap 32), mixed precision, 32 RHS.
    "c3": dict(level=6, leaf=64, eta=2.0, fixed_rank=0, eps=1e-5, cap=32,
               precision="mixed", rhs="normal", seed=2, nrhs=32),
    # small companions used by the parity tests (same rules, smaller n)
    "s1": dict(level=3, leaf=32, eta=2.0, fixed_rank=0, eps=1e-6, cap=32,
               precision="fp64", rhs="normal", seed=11, nrhs=4),
    "s2": dict(level=4, leaf=32, eta=2.0, fixed_rank=0, eps=1e-6, cap=32,
               precision="fp64", rhs="normal", seed=12, nrhs=4),
}


def config_inputs(name: str):
    """Return (xyz, area, cfg) for a named workload."""
    cfg = dict(CONFIGS[name])
    xyz, area = icosphere(cfg["level"])
    return xyz, area, cfg


def ellipsoid_batch_spec(count=256, seed=3):
    """Levels in {3,4,5} and semi-axes ~ U(0.5, 2) for a batch of matrices."""
    rng = np.random.default_rng(seed)
    levels = rng.integers(3, 6, size=count)
    axes = rng.uniform(0.5, 2.0, size=(count, 3))
    return levels, axes


def serving_trace(seed=5, rate=50.0, duration=60.0,
                  sizes=(1280, 5120, 20480, 81920),
                  probs=(0.4, 0.3, 0.2, 0.1), repeat_frac=0.3, max_rhs=64):
    """Poisson arrivals with sizes, RHS counts and repeat flags."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        n = int(rng.choice(sizes, p=probs))
        nrhs = int(rng.integers(1, max_rhs + 1))
        rep = bool(rng.uniform() < repeat_frac)
        jobs.append(dict(t=t, n=n, nrhs=nrhs, repeat=rep,
                         rhs_seed=int(rng.integers(0, 2**31 - 1))))
    return jobs
