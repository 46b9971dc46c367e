"""Pins of the oracle's closed-form element integrals (App. B, eq. U_W_BM).

Each check is independent of the closed forms: scipy adaptive quadrature of
the defining integrals, central finite differences of the defining
derivatives, and exact identities of a closed polyhedron (solid angle 4 pi,
divergence theorem).
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import elemint

C4PI = 1.0 / (4.0 * math.pi)


def _tri(seed=0):
    rng = np.random.default_rng(seed)
    V = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.3, 0.9, 0.0]]) + 0.05 * rng.standard_normal((3, 3))
    V[:, 2] = 0.0
    R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    V = V @ R.T + rng.standard_normal(3)
    n = np.cross(V[1] - V[0], V[2] - V[0])
    n /= np.linalg.norm(n)
    return V, n, R


def _brute(x, V, fun, eps=1e-12):
    """int_E fun(r) dS by adaptive quadrature over the triangle's parameter square."""
    e1, e2 = V[1] - V[0], V[2] - V[0]
    jac = np.linalg.norm(np.cross(e1, e2))

    def f(v, u):
        y = V[0] + u * e1 + v * e2
        return fun(np.linalg.norm(x - y)) * jac

    val, _ = integrate.dblquad(f, 0.0, 1.0, 0.0, lambda u: 1.0 - u, epsabs=eps, epsrel=eps)
    return val


def _U(x, V, n, s, d, cdt=1.0, ni=None):
    return elemint.elem(x, n if ni is None else ni, V, n, s, d, cdt)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_U_bruteforce_no_clip(d):
    V, n, _ = _tri(1)
    for k, x in enumerate([V.mean(0) + 0.4 * n + 0.3 * (V[1] - V[0]),
                           V.mean(0) - 0.7 * n, V[2] + 1.5 * (V[2] - V[0]) + 0.02 * n]):
        rmax = max(np.linalg.norm(x - v) for v in V)
        s = rmax * 1.3 + 0.1
        ref = C4PI * _brute(x, V, lambda r: (s - r) ** d / r)
        got = _U(x, V, n, s, d)[0]
        assert abs(got - ref) <= 1e-10 * abs(ref), (k, got, ref)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_U_bruteforce_clipped(d):
    V, n, _ = _tri(2)
    x = V.mean(0) + 0.25 * n + 0.2 * (V[1] - V[2])
    rmin, rmax = elemint.dist_range(x, V)
    for s in np.linspace(rmin, rmax, 6)[1:-1]:
        ref = C4PI * _brute(x, V, lambda r: max(s - r, 0.0) ** d / r, eps=1e-11)
        got = _U(x, V, n, s, d)[0]
        assert abs(got - ref) <= 2e-6 * max(abs(ref), 1e-3 * s ** d), (s, got, ref)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_U_self_polar_bruteforce(d):
    """Singular self integral by nested quadrature in polar coordinates about the centroid."""
    V, n, _ = _tri(3)
    x = V.mean(0)
    for s in (0.2, 0.55, 3.0):
        tot = 0.0
        for a in range(3):
            A, B = V[a], V[(a + 1) % 3]
            e = (B - A) / np.linalg.norm(B - A)
            m = np.cross(n, e)
            p0 = A - x
            h = -np.dot(p0, m)  # distance of the centroid to the edge line (positive)
            th = lambda P: math.atan2(np.dot(P, m), np.dot(P, e))
            ta, tb = th(A - x), th(B - x)
            if tb < ta:
                ta, tb = tb, ta
            nd = -m  # unit in-plane normal pointing from the centroid to the edge line

            def inner(t):
                dirv = math.cos(t) * e + math.sin(t) * m
                rho_e = h / np.dot(dirv, nd)
                top = min(rho_e, s)
                return integrate.quad(lambda r: (s - r) ** d, 0.0, top, epsabs=1e-13, epsrel=1e-13)[0]

            tot += integrate.quad(inner, ta, tb, epsabs=1e-12, epsrel=1e-12, limit=200)[0]
        got = elemint.elem(x, n, V, n, s, d, 1.0, self_pair=True)[0]
        assert abs(got - C4PI * tot) <= 1e-9 * abs(C4PI * tot), (s, got, C4PI * tot)


def _fd_checks(x, V, n, ni, s, d, h=1e-5):
    """Central differences of the closed-form U and W in x and s."""
    def U(xx, ss):
        return elemint.elem(xx, ni, V, n, ss, d, 1.0)[0]

    def W(xx, ss):
        return elemint.elem(xx, ni, V, n, ss, d, 1.0)[1]

    got = elemint.elem(x, ni, V, n, s, d, 1.0)
    W_fd = -(U(x + h * n, s) - U(x - h * n, s)) / (2 * h)
    Ub_fd = (U(x + h * ni, s) - U(x - h * ni, s)) / (2 * h) - (U(x, s + h) - U(x, s - h)) / (2 * h)
    Wb_fd = (W(x + h * ni, s) - W(x - h * ni, s)) / (2 * h) - (W(x, s + h) - W(x, s - h)) / (2 * h)
    return got, np.array([got[0], W_fd, Ub_fd, Wb_fd])


@pytest.mark.parametrize("d", [1, 2])
def test_derivative_families_by_finite_differences(d):
    V, n, _ = _tri(4)
    rng = np.random.default_rng(7)
    pts = [V.mean(0) + 0.3 * n, V.mean(0) - 0.45 * n + 0.2 * (V[0] - V[1]),
           V[1] + 0.4 * (V[1] - V[2]) + 0.05 * n, V.mean(0) + 0.02 * n + 0.1 * (V[2] - V[0])]
    for x in pts:
        ni = rng.standard_normal(3)
        ni /= np.linalg.norm(ni)
        rmin, rmax = elemint.dist_range(x, V)
        for s in (rmin + 0.3 * (rmax - rmin), rmin + 0.8 * (rmax - rmin), 1.2 * rmax + 0.05):
            got, fd = _fd_checks(x, V, n, ni, s, d)
            scale = np.max(np.abs(fd)) + 1e-3
            assert np.all(np.abs(got - fd) <= 2e-6 * scale), (x, s, got, fd)


@pytest.mark.parametrize("d", [1, 2])
def test_self_pair_is_one_sided_limit(d):
    """The self pair equals the limit z -> 0+ along the paper normal; W_ii = (s/c dt)^d / 2."""
    V, n, _ = _tri(5)
    x = V.mean(0)
    for s in (0.15, 0.6, 2.5):
        self_v = elemint.elem(x, n, V, n, s, d, 0.7, self_pair=True)
        near = elemint.elem(x + 1e-7 * n, n, V, n, s, d, 0.7)
        assert np.allclose(self_v, near, rtol=1e-5, atol=1e-6 * np.abs(self_v).max())
        assert abs(self_v[1] - 0.5 * (s / 0.7) ** d) < 1e-13 * (s / 0.7) ** d
        other = elemint.elem(x - 1e-7 * n, n, V, n, s, d, 0.7)
        assert abs(other[1] + 0.5 * (s / 0.7) ** d) < 1e-5 * (s / 0.7) ** d  # jump of the double layer


def _surface(level=1):
    xyz, tri = synth.icosphere(level)
    g = elemint.Geometry(xyz, tri)
    return g


def _one_over_r(x, V, self_pair):
    if not self_pair:
        return _brute(x, V, lambda r: 1.0 / r, eps=1e-11)
    # singular: split into three sub-triangles at x, each integrated in polar form
    tot = 0.0
    for a in range(3):
        A, B = V[a], V[(a + 1) % 3]
        e1, e2 = A - x, B - x
        jac = np.linalg.norm(np.cross(e1, e2))
        # Duffy: y = x + u (e1 + v (e2 - e1)), dS = u jac du dv, r = u |e1 + v (e2-e1)|
        tot += integrate.quad(lambda v: jac / np.linalg.norm(e1 + v * (e2 - e1)), 0.0, 1.0,
                              epsabs=1e-13, epsrel=1e-13)[0]
    return tot


def test_gauss_identities_closed_surface():
    """Closed polyhedron, x_i on the inner side (side of the paper normal), s > diameter:
    d=1: sum_j W_ij = s/(c dt),  sum_j Wbar_ij = -1/(c dt)
    d=2: sum_j W_ij = (s/c dt)^2 - C sum_j h_j int_{E_j} dS/r,
         sum_j Wbar_ij = 2C sum_j (n_i . nhat_j) int_{E_j} dS/r - 8 pi C s
    (solid angle of a closed surface; divergence theorem for the d=2 remainder)."""
    g = _surface(1)
    cdt = 0.37
    s = 2.3  # > diameter 2
    for i in (0, 17, 55):
        tot1 = np.zeros(4)
        tot2 = np.zeros(4)
        vol = 0.0
        grad = 0.0
        for j in range(g.ns):
            V = g.tris[j].reshape(3, 3)
            tot1 += elemint.elem(g.x[i], g.n[i], V, g.n[j], s, 1, cdt, self_pair=(i == j))
            tot2 += elemint.elem(g.x[i], g.n[i], V, g.n[j], s, 2, cdt, self_pair=(i == j))
            ir = _one_over_r(g.x[i], V, i == j)
            h = np.dot(g.nhat[j], V[0] - g.x[i])
            vol += h * ir
            grad += np.dot(g.n[i], g.nhat[j]) * ir
        C2 = 1.0 / (4 * math.pi * cdt ** 2)
        assert abs(tot1[1] - s / cdt) < 1e-11 * s / cdt
        assert abs(tot1[3] + 1.0 / cdt) < 1e-10 / cdt
        assert abs(tot2[1] - ((s / cdt) ** 2 - C2 * vol)) < 1e-9 * (s / cdt) ** 2
        ref = 2 * C2 * grad - 8 * math.pi * C2 * s
        assert abs(tot2[3] - ref) < 1e-9 * abs(8 * math.pi * C2 * s)


# ---------------------------------------------------------------------------
# Planted mistakes: each compiles a copy of the oracle's C source with one
# plausible slip and checks that at least one of the pins above fails on it.

_PLANTS = {
    # App. B's local y taken with the opposite sign (the bracket is odd in y)
    "edge_y_sign": ("double yl = -h;", "double yl = h;"),
    # the foot-point term I_0 of the polar integral dropped
    "no_foot_term": ("out[0] += theta * pospow(s - az, d + 1) / (d + 1);", "out[0] += 0.0;"),
    # edges not clipped to the wavefront r <= s
    "no_clip": ("double lo = x1 > -X ? x1 : -X, hi = x2 < X ? x2 : X;", "double lo = x1, hi = x2;"),
    # double layer with the wrong sign (W = +C dPhi/dz)
    "w_sign": ("out[1] = -C * f[1];", "out[1] = C * f[1];"),
    # Burton-Miller time derivative with the wrong sign (+(1/c) d/dt)
    "bm_time_sign": ("out[2] = C * (nn * f[1] + f[5] - f[3]);", "out[2] = C * (nn * f[1] + f[5] + f[3]);"),
    # in-plane part of the adjoint double layer (tangential divergence theorem) dropped
    "no_tangential_gradient": ("out[3] = -C * (nn * f[2] + f[6] - f[4]);", "out[3] = -C * (nn * f[2] - f[4]);"),
}


def _pins_d2():
    """The fast pins at d = 2 (and d = 1 for the closed-surface identities)."""
    test_U_bruteforce_no_clip(2)
    test_U_bruteforce_clipped(2)
    test_U_self_polar_bruteforce(2)
    test_derivative_families_by_finite_differences(2)
    test_self_pair_is_one_sided_limit(2)
    test_gauss_identities_closed_surface()


def _planted_lib(tmp_path, name):
    import ctypes
    import subprocess
    from oracle import build as obuild
    src = open(os.path.join(os.path.dirname(obuild.OUT), "..", "elemint.c")).read()
    old, new = _PLANTS[name]
    assert src.count(old) == 1, name
    path = tmp_path / f"plant_{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"plant_{name}.so"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", str(path), "-lm", "-o", str(so)], check=True)
    return elemint.configure(ctypes.CDLL(str(so)))


def test_unplanted_pins_pass():
    _pins_d2()


@pytest.mark.parametrize("name", sorted(_PLANTS))
def test_planted_element_integral_mistakes_fail_a_pin(tmp_path, monkeypatch, name):
    monkeypatch.setattr(elemint, "_lib", _planted_lib(tmp_path, name))
    with pytest.raises(AssertionError):
        _pins_d2()
