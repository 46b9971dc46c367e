"""Pins of the oracle's direct marching-on-in-time (eqs. bie_disc, linear, App. A)."""
import math

import numpy as np
import pytest

import synth
from oracle import elemint, mot
from oracle.bspline import weights


def _raw(geom, d, cdt, gstar, fam):
    """Raw X^{(gamma)}_ij, gamma = 1..gstar (not kappa-summed), family index fam."""
    X = np.zeros((gstar + 1, geom.ns, geom.ns))
    for i in range(geom.ns):
        for j in range(geom.ns):
            V = geom.tris[j].reshape(3, 3)
            for gm in range(1, gstar + 1):
                X[gm, i, j] = elemint.elem(geom.x[i], geom.n[i], V, geom.n[j], gm * cdt, d, cdt,
                                           self_pair=(i == j))[fam]
    return X


@pytest.mark.parametrize("d,bie", [(1, 1), (2, 1), (2, 0)])
def test_tau_sigma_form_equals_compact_form(d, bie):
    """App. A: with beta* truncation, sum (U tau~ - W sigma~) == sum_beta (C_U q - C_W u)."""
    xyz, tri = synth.icosphere(1)
    cdt = 0.5
    m = mot.DirectMOT(xyz, tri, 1.0, cdt, d, bie, 0)
    g = m.geom
    gstar = int(math.ceil(2.0 / cdt)) + d + 1          # diameter 2
    XU = _raw(g, d, cdt, gstar, 2 if bie else 0)
    XW = _raw(g, d, cdt, gstar, 3 if bie else 1)
    w = weights(d)
    rng = np.random.default_rng(3)
    nt = 20
    u = rng.standard_normal((nt, g.ns))
    q = rng.standard_normal((nt, g.ns))
    for alpha in (3, 9, 17):
        ref = m.history_rhs(alpha, u, q)
        bstar = max(alpha - gstar, 0)
        b = np.zeros(g.ns)
        for bp in range(bstar, alpha):
            kmax = min(d + 1, bp - bstar)
            ks = range(1, kmax + 1) if bp == alpha - 1 else range(0, kmax + 1)
            tau = sum(w[k] * q[bp - k] for k in ks)
            sig = sum(w[k] * u[bp - k] for k in ks)
            b += XU[alpha - bp] @ tau - XW[alpha - bp] @ sig
        assert np.max(np.abs(b - ref)) <= 1e-12 * np.max(np.abs(ref)), alpha


def _pulsating(level, d, bie, dt_scale=1.0):
    xyz, tri = synth.icosphere(level)
    dt = synth.mean_edge_length(xyz, tri) * dt_scale
    nt = int(math.ceil(10.0 / dt))
    m = mot.DirectMOT(xyz, tri, 1.0, dt, d, bie, mot.DIRICHLET)
    f = lambda t: np.exp(-(t - 4.0) ** 2 / 0.5)
    fp = lambda t: -(t - 4.0) / 0.25 * f(t)
    beta = np.arange(nt - 1)
    ubar = f(dt * (beta + (d + 1) / 2.0))[:, None] * np.ones((1, m.ns))   # Greville quasi-interpolant
    u, q = m.run(nt, None, ubar)
    qrec = mot.reconstruct(q, d)
    ta = dt * np.arange(1, nt)
    qex = (f(ta) + fp(ta))[:, None] * np.ones_like(qrec)   # d/dn u, n into the sphere, u = f(t-(r-1))/r
    return np.linalg.norm(qrec - qex) / np.linalg.norm(qex)


def test_pulsating_sphere_bm_d2_converges_in_h():
    e2 = _pulsating(2, 2, mot.BMBIE)
    e3 = _pulsating(3, 2, mot.BMBIE)
    assert e2 < 0.12 and e3 < 0.06 and e2 / e3 > 1.6, (e2, e3)


def test_pulsating_sphere_bm_d1_converges_in_dt():
    e1 = _pulsating(2, 1, mot.BMBIE, 1.0)
    e2 = _pulsating(2, 1, mot.BMBIE, 0.5)
    assert e1 < 0.3 and e2 < 0.16 and e1 / e2 > 1.6, (e1, e2)


def _late_over_peak(d, bie, bc, nt):
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    inc = synth.incident_params(xyz, seed=0)
    m = mot.DirectMOT(xyz, tri, 1.0, dt, d, bie, bc)
    F = mot.incident(m.geom, inc, 1.0, dt, nt, bie)
    u, q = m.run(nt, F)
    x = np.abs(q if bc == mot.DIRICHLET else u).max(axis=1)
    return x[-10:].max() / max(x[: nt // 3].max(), 1e-300), x.max()


def test_stability_pattern_tables_2_and_3():
    """Qualitative pattern of Tables 2-3 on a small sphere: OBIE with d=2 diverges for
    both conditions; the BMBIE decays for d=1 (Dirichlet) and d=1,2 (Neumann); the
    BMBIE with d=2 does not settle for the Dirichlet problem."""
    late, peak = _late_over_peak(2, mot.OBIE, mot.DIRICHLET, 64)
    assert peak > 1e6
    late, peak = _late_over_peak(2, mot.OBIE, mot.NEUMANN, 100)
    assert peak > 1e6
    assert _late_over_peak(1, mot.BMBIE, mot.DIRICHLET, 128)[0] < 1e-3
    assert _late_over_peak(2, mot.BMBIE, mot.DIRICHLET, 128)[0] > 0.1
    assert _late_over_peak(1, mot.BMBIE, mot.NEUMANN, 128)[0] < 1e-8
    assert _late_over_peak(2, mot.BMBIE, mot.NEUMANN, 128)[0] < 1e-8


def _extinction_residual(level, d, bie):
    xyz, tri = synth.icosphere(level)
    dt = synth.mean_edge_length(xyz, tri)
    nt = int(math.ceil(9.0 / dt))
    m = mot.DirectMOT(xyz, tri, 1.0, dt, d, bie, mot.DIRICHLET)
    inc = synth.incident_params(xyz, seed=1)
    g = m.geom
    k = inc["dir"]
    # incident traces, quasi-interpolated in time at Greville points
    tb = dt * (np.arange(nt - 1) + (d + 1) / 2.0)[:, None]
    p = tb - (g.x @ k + inc["rb"])[None, :] - inc["t0"]
    sg, w = inc["sigma"], 2 * math.pi * inc["f0"]
    env = np.exp(-p * p / (2 * sg * sg))
    uin = env * np.cos(w * p)
    gp = env * (-p / (sg * sg) * np.cos(w * p) - w * np.sin(w * p))
    qin = gp * (-(g.n @ k))[None, :]
    F = mot.incident(g, inc, 1.0, dt, nt, bie)
    res = []
    for alpha in range(1, nt):
        r = F[alpha - 1] + m.history_rhs(alpha, uin, qin) + m.CU[1] @ qin[alpha - 1] - m.CW[1] @ uin[alpha - 1]
        res.append(r)
    return np.linalg.norm(res) / np.linalg.norm(F)


def _extinction_converges(d, bie):
    r1, r2, r3 = (_extinction_residual(level, d, bie) for level in (1, 2, 3))
    return r2 < r1 and r3 < r2 and r3 < 0.5 and r2 / r3 > 1.5, (r1, r2, r3)


@pytest.mark.parametrize("d,bie", [(1, 0), (1, 1), (2, 1)])
def test_extinction_consistency(d, bie):
    """Traces of a field regular inside the scatterer satisfy the discrete equation
    up to a discretisation residual that shrinks under refinement."""
    ok, r = _extinction_converges(d, bie)
    assert ok, r


def _plant_w_sign(m):
    m.CW = {g: -X for g, X in m.CW.items()}


def _plant_gap_shift(m):
    for name in ("CU", "CW"):
        C = getattr(m, name)
        setattr(m, name, {g: C.get(g + 1, 0 * C[g]) for g in C})


def _plant_u_w_swapped(m):
    m.CU, m.CW = m.CW, m.CU


@pytest.mark.parametrize("plant", [_plant_w_sign, _plant_gap_shift, _plant_u_w_swapped])
def test_planted_march_mistakes_fail_the_extinction_pin(monkeypatch, plant):
    """A sign error on the double-layer terms, coefficients taken one time gap late, or
    the two families exchanged each stop the residual from converging."""
    orig = mot.DirectMOT.__init__

    def init(self, *a, **kw):
        orig(self, *a, **kw)
        plant(self)
    monkeypatch.setattr(mot.DirectMOT, "__init__", init)
    ok, r = _extinction_converges(2, mot.BMBIE)
    assert not ok, r


class _Pts:
    """Stand-in for a Geometry: collocation points and paper normals only."""

    def __init__(self, x, n):
        self.x, self.n = np.ascontiguousarray(x), np.ascontiguousarray(n)


def _seeded_points(seed=11, m=40):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(m, 3))
    n = rng.standard_normal((m, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return x, n


@pytest.mark.parametrize("kind", ["raised_cos", "gauss_mod"])
def test_bm_forcing_is_the_bm_operator_of_the_incident_field(kind):
    """(d/dn - (1/c) d/dt) u_in by central differences of the OBIE forcing: in x along the
    paper normal, and in t through the arrival shift rb (u_in depends on c t - k.x - rb)."""
    x, n = _seeded_points()
    c, dt, nt, h = 1.3, 0.05, 120, 1e-6
    inc = {"kind": kind, "dir": np.array([0.6, -0.48, 0.64]), "f0": 1.0, "sigma": 0.5, "t0": 1.5, "rb": 0.2}
    if kind == "raised_cos":
        inc["sigma"] = 0.5       # pulse length Lambda
    bm = mot.incident(_Pts(x, n), inc, c, dt, nt, mot.BMBIE)
    up = mot.incident(_Pts(x + h * n, n), inc, c, dt, nt, mot.OBIE)
    um = mot.incident(_Pts(x - h * n, n), inc, c, dt, nt, mot.OBIE)
    early = dict(inc, rb=inc["rb"] - c * h)      # u_in(x, t + h)
    late = dict(inc, rb=inc["rb"] + c * h)       # u_in(x, t - h)
    ut = (mot.incident(_Pts(x, n), early, c, dt, nt, mot.OBIE)
          - mot.incident(_Pts(x, n), late, c, dt, nt, mot.OBIE)) / (2 * h)
    fd = (up - um) / (2 * h) - ut / c
    scale = np.abs(bm).max()
    assert scale > 1.0
    # the raised cosine is C^1 only: skip samples within 2h of its two kinks
    ok = np.ones_like(bm, dtype=bool)
    if kind == "raised_cos":
        t = dt * np.arange(1, nt)[:, None]
        ph = c * t - (x @ inc["dir"])[None, :] - inc["rb"]
        ok = (np.abs(ph) > 4 * h) & (np.abs(ph - inc["sigma"]) > 4 * h)
    assert np.all(np.abs(bm - fd)[ok] <= 1e-6 * scale)


def test_raised_cosine_pulse_shape():
    """Plane pulse of eq. uin: zero before arrival and after one pulse length, peak 1 at half
    the pulse length, time integral Lambda / (2 c) at every point, and invariant under the
    plane-wave translation (x, t) -> (x + v, t + k.v / c) and under shifts across k."""
    x, n = _seeded_points(5, 25)
    c, lam = 1.7, 0.5
    k = np.array([1.0, 0.0, 0.0])
    inc = {"kind": "raised_cos", "dir": k, "f0": 1.0, "sigma": lam, "t0": 0.0, "rb": 1.5}
    dt, nt = 1e-4, 2 * int(3.0 / 1e-4)
    u = mot.incident(_Pts(x, n), inc, c, dt, nt, mot.OBIE)
    t = dt * np.arange(1, nt)[:, None]
    ph = c * t - (x @ k)[None, :] - inc["rb"]
    assert np.all(u[(ph < 0) | (ph > lam)] == 0.0)
    assert np.all((u >= 0.0) & (u <= 1.0))
    assert np.allclose(u.sum(axis=0) * dt, lam / (2 * c), rtol=1e-6)
    # peak: ph = lam / 2 at t = (x1 + rb + lam / 2) / c
    tp = (x[:, 0] + inc["rb"] + lam / 2) / c
    j = np.rint(tp / dt).astype(int) - 1
    assert np.allclose(u[j, np.arange(len(x))], 1.0, atol=1e-6)
    # plane-wave invariance: a shift v with k.v = 0.3 delays the pulse by 0.3 / c
    rng = np.random.default_rng(2)
    v = rng.standard_normal(3)
    v += (0.3 - v @ k) * k
    shift = int(round(0.3 / c / dt))
    dt2 = 0.3 / c / shift
    u0 = mot.incident(_Pts(x, n), inc, c, dt2, 4000, mot.OBIE)
    u1 = mot.incident(_Pts(x + v, n), inc, c, dt2, 4000 + shift, mot.OBIE)
    assert np.allclose(u1[shift:], u0, atol=1e-12)


_FORCING_PLANTS = [
    # time derivative of the BM operator with the wrong sign
    ("(-kn[None, :] - 1.0)", "(-kn[None, :] + 1.0)"),
    # pulse travelling against its direction
    ("(c * t - kx[None, :] - inc[\"rb\"])", "(c * t + kx[None, :] - inc[\"rb\"])"),
    # pulse length used as a wavenumber
    ("/ lam\n", "* lam\n"),
]


@pytest.mark.parametrize("old,new", _FORCING_PLANTS)
def test_planted_forcing_mistakes_fail_a_pin(monkeypatch, old, new):
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(mot.incident))
    assert src.count(old) == 1, old
    ns = dict(vars(mot))
    exec(compile(src.replace(old, new), "planted_incident", "exec"), ns)
    monkeypatch.setattr(mot, "incident", ns["incident"])
    failed = 0
    for pin in (lambda: test_bm_forcing_is_the_bm_operator_of_the_incident_field("raised_cos"),
                test_raised_cosine_pulse_shape):
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 1
