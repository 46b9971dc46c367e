"""Pins of the oracle's mixed boundary conditions (eq. ibvp with S_u and S_q both non-empty,
phi_j of eq. linear) and of its off-surface field (the Kirchhoff representation with the
operators of eq. bie_disc at a point that is not a collocation point), on the pulsating
sphere: prescribed data u = f(t) on the unit sphere, exact exterior field
u(r, t) = f(t - (r - 1)) / r, q = du/dn = f + f' (n into the sphere)."""
import math

import numpy as np
import pytest

import synth
from oracle import mot


def f(t):
    return np.exp(-(t - 4.0) ** 2 / 0.5)


def fp(t):
    return -(t - 4.0) / 0.25 * f(t)


PTS = np.array([[1.5, 0.0, 0.0], [0.0, 2.5, 0.0], [0.0, 0.0, -1.8], [0.3, 0.2, 0.1]])


def _case(level, d=2):
    xyz, tri = synth.icosphere(level)
    dt = synth.mean_edge_length(xyz, tri)
    nt = int(math.ceil(10.0 / dt))
    tb = dt * (np.arange(nt - 1) + (d + 1) / 2.0)       # Greville quasi-interpolant
    geo_x = mot.DirectMOT.__new__(mot.DirectMOT)
    from oracle.elemint import Geometry
    x = Geometry(xyz, tri).x
    phi = (x[:, 2] > 0).astype(float)                    # q given on the upper half
    pres = np.where(phi[None, :] > 0, (f(tb) + fp(tb))[:, None], f(tb)[:, None])
    m = mot.DirectMOT(xyz, tri, 1.0, dt, d, mot.BMBIE, mot.MIXED, phi=phi)
    u, q = m.run(nt, None, pres)
    ta = dt * np.arange(1, nt)
    urec, qrec = mot.reconstruct(u, d), mot.reconstruct(q, d)
    nm, dm = phi > 0, phi == 0
    eu = np.linalg.norm(urec[:, nm] - f(ta)[:, None]) / np.linalg.norm(np.outer(f(ta), np.ones(nm.sum())))
    eq = np.linalg.norm(qrec[:, dm] - (f(ta) + fp(ta))[:, None]) / \
        np.linalg.norm(np.outer(f(ta) + fp(ta), np.ones(dm.sum())))
    errs = []
    r = np.linalg.norm(PTS, axis=1)
    for tt in (5.0, 6.0):
        a = int(round(tt / dt))
        fld = m.field(PTS, a, u, q)
        ex = np.where(r > 1, f(a * dt - (r - 1)) / np.maximum(r, 1e-300), 0.0)
        errs.append(np.abs(fld - ex))
    return eu, eq, np.max(errs, axis=0)


@pytest.fixture(scope="module")
def levels():
    return _case(2), _case(3)


def test_mixed_problem_converges_to_the_pulsating_sphere(levels):
    (eu2, eq2, _), (eu3, eq3, _) = levels
    assert eu3 < 0.06 and eq3 < 0.09, (eu3, eq3)
    assert eu2 / eu3 > 1.6 and eq2 / eq3 > 1.5, (eu2, eu3, eq2, eq3)


def test_off_surface_field_converges_outside_and_vanishes_inside(levels):
    """Exterior points approach f(t - (r-1))/r; the interior point (extinction: the
    representation gives zero inside the scatterer, the incident field being zero here)
    approaches 0."""
    (_, _, e2), (_, _, e3) = levels
    assert (e3[:3] < 0.04).all() and (e2[:3] / e3[:3] > 1.3).all(), (e2, e3)
    assert e3[3] < 0.05 and e2[3] / e3[3] > 1.5, (e2, e3)


def test_mixed_with_uniform_phi_is_the_pure_problem():
    xyz, tri = synth.icosphere(1)
    dt = synth.mean_edge_length(xyz, tri)
    inc = synth.incident_params(xyz, seed=3)
    nt = 24
    for bc, ph in ((mot.NEUMANN, 1.0), (mot.DIRICHLET, 0.0)):
        a = mot.DirectMOT(xyz, tri, 1.0, dt, 2, mot.BMBIE, bc)
        b = mot.DirectMOT(xyz, tri, 1.0, dt, 2, mot.BMBIE, mot.MIXED, phi=np.full(a.ns, ph))
        F = mot.incident(a.geom, inc, 1.0, dt, nt, mot.BMBIE)
        ua, qa = a.run(nt, F)
        ub, qb = b.run(nt, F)
        assert np.abs(ua - ub).max() <= 1e-13 * max(np.abs(ua).max(), 1.0)
        assert np.abs(qa - qb).max() <= 1e-13 * max(np.abs(qa).max(), 1.0)


def _extinction_errors(level):
    xyz, tri = synth.icosphere(level)
    dt = synth.mean_edge_length(xyz, tri)
    d = 2
    from oracle.elemint import Geometry
    m = mot.DirectMOT.__new__(mot.DirectMOT)
    m.c, m.dt, m.d = 1.0, dt, d
    m.geom = g = Geometry(xyz, tri)
    inc = synth.incident_params(xyz, seed=1)
    k = np.asarray(inc["dir"])
    nt = int(math.ceil(9.0 / dt))
    tb = dt * (np.arange(nt - 1) + (d + 1) / 2.0)[:, None]
    p = tb - (g.x @ k + inc["rb"])[None, :] - inc["t0"]
    sg, w = inc["sigma"], 2 * math.pi * inc["f0"]
    env = np.exp(-p * p / (2 * sg * sg))
    u = env * np.cos(w * p)
    du = env * (-p / (sg * sg) * np.cos(w * p) - w * np.sin(w * p))
    q = du * (-(g.n @ k))[None, :]                      # d/dn with the paper normal n
    pts = np.array([[0.2, -0.1, 0.3], [0.0, 0.0, 0.0], [1.6, 0.3, -0.2], [0.1, -2.0, 0.4]])
    ins, outs = [], []
    for tt in np.arange(4.0, 7.01, 0.25):
        a = int(round(tt / dt))
        fld = m.field(pts, a, u, q)
        pi = a * dt - (pts @ k + inc["rb"]) - inc["t0"]
        uin = np.exp(-pi * pi / (2 * sg * sg)) * np.cos(w * pi)
        ins.append(fld[:2] + uin[:2])
        outs.append(fld[2:])
    return np.abs(ins).max(), np.abs(outs).max()


def test_field_of_the_incident_traces_extinguishes_inside():
    """Extinction consistency of the representation: feeding the incident wave's own traces
    (u = u_in, q = du_in/dn on the surface, quasi-interpolated in time) gives -u_in inside the
    scatterer and 0 outside, up to discretisation error that shrinks under refinement (a sign
    error in either layer, or a wrong time index, leaves an O(1) residual)."""
    i2, o2 = _extinction_errors(2)
    i3, o3 = _extinction_errors(3)
    assert o2 < 0.04 and o3 < 0.01 and o2 / o3 > 3.0, (o2, o3)
    assert i3 < 0.15 and i2 / i3 > 2.0, (i2, i3)
