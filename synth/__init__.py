"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds inputs: closed triangulated surfaces, incident-wave
parameters, random density histories.  It holds none of the time-domain BEM
arithmetic (no element integrals, B-splines, FMM or marching), so that the CPU
oracle and the GPU path can both consume it without sharing method code.

Surfaces are returned as (xyz, tri): float64 vertex coordinates (nv, 3) and
int32 vertex indices (nt, 3), each triangle counter-clockwise when seen from
outside the scatterer (outward normal by the right-hand rule).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "icosahedron", "icosphere", "geodesic_sphere", "ellipsoid", "rounded_cube",
    "octahedron", "mean_edge_length", "incident_params", "random_history",
    "workload",
]


def icosahedron():
    """Regular icosahedron with vertices on the unit sphere (20 faces)."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int32)
    return _orient_outward(v, f)


def octahedron():
    """Regular octahedron with vertices on the unit sphere (8 faces)."""
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64)
    f = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                  [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int32)
    return _orient_outward(v, f)


def _orient_outward(v, f):
    """Flip any face whose right-hand normal points towards the centroid of the body."""
    f = f.copy()
    c0 = v.mean(axis=0)
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    nrm = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0
    flip = np.einsum("ij,ij->i", nrm, cen - c0) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def icosphere(level: int):
    """Icosahedron refined `level` times by 4-way midpoint subdivision, projected to r=1.

    level 2 -> 320 faces, level 4 -> 5120, level 5 -> 20480, level 6 -> 81920.
    """
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            k = cache.get(key)
            if k is None:
                m = (np.asarray(verts[i]) + np.asarray(verts[j])) * 0.5
                m /= np.linalg.norm(m)
                verts.append(tuple(m))
                k = len(verts) - 1
                cache[key] = k
            return k

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int32)
    return np.array(verts, dtype=np.float64), f


def geodesic_sphere(freq: int):
    """Frequency-`freq` geodesic sphere: each icosahedron face split into freq^2 triangles.

    Ns = 20 * freq^2; vertices projected to the unit sphere.
    """
    v0, f0 = icosahedron()
    verts: list[np.ndarray] = []
    index: dict[tuple, int] = {}

    def vid(p):
        q = p / np.linalg.norm(p)
        key = tuple(np.round(q, 12))
        k = index.get(key)
        if k is None:
            verts.append(q)
            k = len(verts) - 1
            index[key] = k
        return k

    faces = []
    n = freq
    for a, b, c in f0:
        A, B, C = v0[a], v0[b], v0[c]
        grid = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                p = A + (B - A) * (i / n) + (C - A) * (j / n)
                grid[(i, j)] = vid(p)
        for i in range(n):
            for j in range(n - i):
                faces.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j + 1 < n:
                    faces.append((grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]))
    return _orient_outward(np.array(verts), np.array(faces, dtype=np.int32))


def ellipsoid(freq: int, axes=(1.0, 1.0, 1.0)):
    """Geodesic sphere of frequency `freq` scaled to semi-axes `axes`."""
    v, f = geodesic_sphere(freq)
    return v * np.asarray(axes, dtype=np.float64)[None, :], f


def rounded_cube(freq: int, half=1.0, exponent=8.0):
    """Superellipsoid |x|^e+|y|^e+|z|^e = half^e, by radial projection of a geodesic sphere."""
    v, f = geodesic_sphere(freq)
    s = (np.abs(v) ** exponent).sum(axis=1) ** (1.0 / exponent)
    return v / s[:, None] * half, f


def mean_edge_length(xyz, tri) -> float:
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    return float(np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1).mean())


def incident_params(xyz, seed: int = 0, f0: float = 1.0, sigma: float = 0.5, t0: float | None = None,
                    kind: str = "gauss_mod"):
    """Parameters of a plane incident pulse.

    kind "gauss_mod": u(x,t) = exp(-(p-t0)^2/(2 sigma^2)) cos(2 pi f0 (p-t0)),
    p = t - (k.x + rb)/c, with k a unit vector drawn from a seeded normal
    distribution and rb the largest vertex radius, so the pulse is ~0 on the
    surface at t=0 when t0 = 8 sigma.
    kind "raised_cos": u(x,t) = 0.5 (1 - Cos(2 pi (c t - k.x - rb)/lam)), with
    Cos equal to cos on [0, 2 pi] and 1 elsewhere, lam = sigma.
    """
    rng = np.random.default_rng(seed)
    k = rng.normal(size=3)
    k /= np.linalg.norm(k)
    rb = float(np.linalg.norm(xyz, axis=1).max())
    return {"kind": kind, "dir": k, "f0": float(f0), "sigma": float(sigma),
            "t0": float(8.0 * sigma if t0 is None else t0), "rb": rb}


def random_history(ns: int, nsteps: int, seed: int = 0, smooth: bool = True):
    """Seeded random density coefficients of shape (nsteps, ns)."""
    rng = np.random.default_rng(seed)
    if not smooth:
        return rng.standard_normal((nsteps, ns))
    t = np.arange(nsteps)[:, None]
    ph = rng.uniform(0, 2 * np.pi, size=(1, ns))
    fr = rng.uniform(0.02, 0.1, size=(1, ns))
    amp = rng.standard_normal((1, ns))
    return amp * np.sin(2 * np.pi * fr * t + ph) + 0.1 * rng.standard_normal((nsteps, ns))


def batch_workload(n: int = 64, seed0: int = 0):
    """Independent scatterers: per seed, a coin picks an ellipsoid (semi-axes
    uniform in [0.5, 2]) or a rounded cube (half side uniform in [0.5, 2]); the
    face count Ns = 20 f^2 with f = round(sqrt(Ns'/20)) for Ns' log-uniform in
    [500, 8000]; Nt uniform in [128, 512]; B-spline order d in {1, 2};
    Burton-Miller, Neumann; c = 1, dt = mean edge; plane Gaussian pulse with a
    seeded direction."""
    out = []
    for k in range(n):
        rng = np.random.default_rng(seed0 + k)
        ns_target = float(np.exp(rng.uniform(np.log(500.0), np.log(8000.0))))
        freq = int(np.clip(round(np.sqrt(ns_target / 20.0)), 5, 20))
        if rng.uniform() < 0.5:
            shape = "ellipsoid"
            xyz, tri = ellipsoid(freq, rng.uniform(0.5, 2.0, size=3))
        else:
            shape = "rounded_cube"
            xyz, tri = rounded_cube(freq, half=float(rng.uniform(0.5, 2.0)))
        nt = int(rng.integers(128, 513))
        d = int(rng.integers(1, 3))
        dt = mean_edge_length(xyz, tri)
        out.append(dict(xyz=xyz, tri=tri, shape=shape, freq=freq, ns=tri.shape[0], nt=nt, d=d, bie=1, bc=1, c=1.0,
                        dt=dt, inc=incident_params(xyz, seed=seed0 + k)))
    return out


def workload(name: str):
    """Named workloads: surface, wave speed, step, order and problem type.

    small  : icosphere level 2 (320 faces), d=1, Nt=64, Burton-Miller, Dirichlet, direct
    sphere5k: icosphere level 4 (5120 faces), d=2, Nt=256, Burton-Miller, Neumann, FMM
              depth 4, 4 Chebyshev nodes per axis in space and in time
    """
    if name == "small":
        xyz, tri = icosphere(2)
        cfg = dict(d=1, nt=64, bie=1, bc=0, use_fmm=0, depth=0, p_s=0, p_t=0)
    elif name == "sphere5k":
        xyz, tri = icosphere(4)
        cfg = dict(d=2, nt=256, bie=1, bc=1, use_fmm=1, depth=4, p_s=4, p_t=4)
    elif name == "sphere20k":
        xyz, tri = icosphere(5)
        cfg = dict(d=2, nt=1024, bie=1, bc=1, use_fmm=1, depth=5, p_s=4, p_t=4)
    elif name == "sphere82k":
        xyz, tri = icosphere(6)
        cfg = dict(d=2, nt=2048, bie=1, bc=1, use_fmm=1, depth=6, p_s=5, p_t=5)
    else:
        raise KeyError(name)
    c = 1.0
    dt = mean_edge_length(xyz, tri) / c
    cfg.update(xyz=xyz, tri=tri, c=c, dt=dt, inc=incident_params(xyz, seed=0))
    return cfg
