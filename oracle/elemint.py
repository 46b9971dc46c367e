"""ORACLE (test infrastructure): ctypes front end of the closed-form element integrals in elemint.c.

Geometry convention: the mesh stores triangles counter-clockwise seen from
outside the scatterer (outward normal nhat).  The paper's normal n points the
other way (into the scatterer), collocation points are face centroids, and
the self pair is the one-sided limit on the side n points to.
"""
import ctypes
import os

import numpy as np
import scipy.sparse as sp

from . import build as _build

_lib = None


def configure(L):
    """Declare the argument types of the oracle's C entry points on a loaded library."""
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(ctypes.c_long)
    L.oracle_face_terms.argtypes = [dp, dp, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp]
    L.oracle_elem.argtypes = [dp, dp, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, dp]
    L.oracle_dist_range.argtypes = [dp, dp, dp, dp]
    L.oracle_windows.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, ip, ip]
    L.oracle_fill.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_double, ip, ip, lp, dp]
    L.oracle_windows_rows.argtypes = [ctypes.c_int, ctypes.c_int, ip, dp, dp, ctypes.c_int, ctypes.c_double,
                                      ip, ip]
    L.oracle_fill_rows.argtypes = [ctypes.c_int, ctypes.c_int, ip, dp, dp, dp, ctypes.c_int, ctypes.c_double,
                                   ip, ip, lp, dp]
    L.oracle_windows_points.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, ip, ip]
    L.oracle_fill_points.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_double,
                                     ip, ip, lp, dp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.OUT):
            _build.build()
        _lib = configure(ctypes.CDLL(_build.OUT))
    return _lib


def _p(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


class Geometry:
    """Per-face data the oracle needs: centroids, paper normals, vertex coordinates, areas."""

    def __init__(self, xyz, tri):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int64)
        a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
        cr = np.cross(b - a, c - a)
        self.area = 0.5 * np.linalg.norm(cr, axis=1)
        self.nhat = cr / (2.0 * self.area[:, None])      # outward
        self.n = np.ascontiguousarray(-self.nhat)        # paper normal, into the scatterer
        self.x = np.ascontiguousarray((a + b + c) / 3.0)
        self.tris = np.ascontiguousarray(np.stack([a, b, c], axis=1).reshape(-1, 9))
        self.ns = tri.shape[0]
        self.diam = float(np.max(np.linalg.norm(xyz[:, None, :] - xyz[None, :, :], axis=2))) \
            if xyz.shape[0] <= 4000 else float(2.0 * np.linalg.norm(xyz - xyz.mean(0), axis=1).max())


def face_terms(x, V, n, t, s, d, self_pair=False):
    x, V, n, t = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, V, n, t))
    out = np.zeros(7)
    lib().oracle_face_terms(_p(x), _p(V), _p(n), _p(t), float(s), int(d), int(self_pair), _p(out))
    return out


def elem(x, ni, V, nj, s, d, cdt, self_pair=False):
    """(U, W, Ubar, Wbar) of one (point, element, s = c t_gamma) triple."""
    x, ni, V, nj = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, ni, V, nj))
    out = np.zeros(4)
    lib().oracle_elem(_p(x), _p(ni), _p(V), _p(nj), int(self_pair), float(s), int(d), float(cdt), _p(out))
    return out


def dist_range(x, V):
    x, V = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, V))
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().oracle_dist_range(_p(x), _p(V), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def compact_coefficients(geom: Geometry, d: int, cdt: float):
    """C^{(g)}_ij = sum_kappa w^kappa X^{(g-kappa)}_ij for X in {U, W, Ubar, Wbar}, all pairs.

    Returns (gmax, fams) with fams[f][g] a scipy CSR matrix (ns x ns), f in
    {"U","W","Ubar","Wbar"}, g = 1..gmax.  This is the coefficient of q_j^beta
    (U-families) or u_j^beta (W-families) at time difference g = alpha - beta in
    eq. bie_disc (and its Burton-Miller analogue).
    """
    ns = geom.ns
    glo = np.zeros(ns * ns, dtype=np.int32)
    cnt = np.zeros(ns * ns, dtype=np.int32)
    lib().oracle_windows(ns, _p(geom.x), _p(geom.tris), d, cdt, _p(glo, ctypes.c_int), _p(cnt, ctypes.c_int))
    if cnt.max() + d + 1 > 64:
        raise ValueError("time window too long for the oracle's fixed buffer")
    off = np.zeros(ns * ns, dtype=np.int64)
    off[1:] = np.cumsum(cnt[:-1], dtype=np.int64)
    tot = int(cnt.sum())
    vals = np.zeros((tot, 4))
    lib().oracle_fill(ns, _p(geom.x), _p(geom.n), _p(geom.tris), d, cdt, _p(glo, ctypes.c_int),
                      _p(cnt, ctypes.c_int), _p(off, ctypes.c_long), _p(vals))
    rows = np.repeat(np.repeat(np.arange(ns), ns), cnt)
    cols = np.repeat(np.tile(np.arange(ns), ns), cnt)
    slot = np.arange(tot) - np.repeat(off, cnt)
    g = np.repeat(glo, cnt) + slot
    gmax = int(g.max())
    fams = {}
    for f, name in enumerate(("U", "W", "Ubar", "Wbar")):
        mats = {}
        for gg in range(1, gmax + 1):
            m = g == gg
            mats[gg] = sp.csr_matrix((vals[m, f], (rows[m], cols[m])), shape=(ns, ns))
        fams[name] = mats
    return gmax, fams


def compact_rows(geom: Geometry, d: int, cdt: float, rows):
    """Compact coefficients of the given collocation rows against every element:
    returns (gmax, dense array C[f, r, g, j]) with f in (U, W, Ubar, Wbar), g = 0..gmax (g=0 unused)."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    ns, nr = geom.ns, len(rows)
    glo = np.zeros(nr * ns, dtype=np.int32)
    cnt = np.zeros(nr * ns, dtype=np.int32)
    lib().oracle_windows_rows(ns, nr, _p(rows, ctypes.c_int), _p(geom.x), _p(geom.tris), d, cdt,
                              _p(glo, ctypes.c_int), _p(cnt, ctypes.c_int))
    if cnt.max() + d + 1 > 64:
        raise ValueError("time window too long for the oracle's fixed buffer")
    off = np.zeros(nr * ns, dtype=np.int64)
    off[1:] = np.cumsum(cnt[:-1], dtype=np.int64)
    vals = np.zeros((int(cnt.sum()), 4))
    lib().oracle_fill_rows(ns, nr, _p(rows, ctypes.c_int), _p(geom.x), _p(geom.n), _p(geom.tris), d, cdt,
                           _p(glo, ctypes.c_int), _p(cnt, ctypes.c_int), _p(off, ctypes.c_long), _p(vals))
    g = np.repeat(glo, cnt) + (np.arange(vals.shape[0]) - np.repeat(off, cnt))
    gmax = int(g.max())
    r = np.repeat(np.repeat(np.arange(nr), ns), cnt)
    j = np.repeat(np.tile(np.arange(ns), nr), cnt)
    C = np.zeros((4, nr, gmax + 1, ns))
    for f in range(4):
        C[f, r, g, j] = vals[:, f]
    return gmax, C


def compact_points(geom: Geometry, d: int, cdt: float, pts):
    """Compact coefficients of the single and double layer (U, W families, eq. bie_disc) at
    off-surface points pts (npts x 3) against every element: returns (gmax, C[f, r, g, j]),
    f in (U, W), g = 0..gmax (g = 0 unused)."""
    pts = np.ascontiguousarray(np.atleast_2d(pts), dtype=np.float64)
    ns, npt = geom.ns, pts.shape[0]
    glo = np.zeros(npt * ns, dtype=np.int32)
    cnt = np.zeros(npt * ns, dtype=np.int32)
    lib().oracle_windows_points(ns, npt, _p(pts), _p(geom.tris), d, cdt, _p(glo, ctypes.c_int),
                                _p(cnt, ctypes.c_int))
    if cnt.max() + d + 1 > 64:
        raise ValueError("time window too long for the oracle's fixed buffer")
    off = np.zeros(npt * ns, dtype=np.int64)
    off[1:] = np.cumsum(cnt[:-1], dtype=np.int64)
    vals = np.zeros((int(cnt.sum()), 2))
    lib().oracle_fill_points(ns, npt, _p(pts), _p(geom.n), _p(geom.tris), d, cdt, _p(glo, ctypes.c_int),
                             _p(cnt, ctypes.c_int), _p(off, ctypes.c_long), _p(vals))
    g = np.repeat(glo, cnt) + (np.arange(vals.shape[0]) - np.repeat(off, cnt))
    gmax = int(g.max())
    r = np.repeat(np.repeat(np.arange(npt), ns), cnt)
    j = np.repeat(np.tile(np.arange(ns), npt), cnt)
    C = np.zeros((2, npt, gmax + 1, ns))
    for f in range(2):
        C[f, r, g, j] = vals[:, f]
    return gmax, C
