"""GPU parity of the direct (no-FMM) path through the C ABI against the FP64 oracle.

Tolerances: element-integral tables are compared entry by entry at 1e-12 of the
row's largest magnitude (two independent FP64 routes: closed forms vs
Gauss-Legendre quadrature, agreement measured at ~1e-15); marches at 1e-10
relative L2 over all (step, element) coefficients.
"""
import math

import numpy as np
import pytest

import synth
from oracle import elemint, mot

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _P():
    import paper_2111_05205_amd as P
    return P


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def sphere2():
    xyz, tri = synth.icosphere(2)
    return xyz, tri, synth.mean_edge_length(xyz, tri)


@pytest.mark.parametrize("d,bie", [(1, 1), (2, 1), (1, 0), (2, 0)])
def test_near_table_matches_oracle(sphere2, d, bie):
    P = _P()
    xyz, tri, dt = sphere2
    s = P.TDBEM(xyz, tri, 1.0, dt, d, bie, P.NEUMANN, nt_max=8)
    gmax, fams = elemint.compact_coefficients(elemint.Geometry(xyz, tri), d, dt)
    CU = fams["Ubar" if bie else "U"]
    CW = fams["Wbar" if bie else "W"]
    worst = 0.0
    for i in range(0, s.ns, 3):
        j, g, cu, cw = s.near_row(i)
        ref_u = np.array([CU[gg][i, jj] if gg <= gmax else 0.0 for jj, gg in zip(j, g)])
        ref_w = np.array([CW[gg][i, jj] if gg <= gmax else 0.0 for jj, gg in zip(j, g)])
        scale = max(np.abs(ref_u).max(), np.abs(ref_w).max())
        worst = max(worst, np.abs(cu - ref_u).max() / scale, np.abs(cw - ref_w).max() / scale)
        # every non-zero oracle coefficient of the row is present in the table
        n_ref = sum(CU[gg][i].count_nonzero() for gg in range(1, gmax + 1))
        assert np.count_nonzero(ref_u) == n_ref
    assert worst < 1e-12, worst


@pytest.mark.parametrize("d,bie,bc", [(1, 1, 0), (2, 1, 1), (1, 0, 1)])
def test_history_sum_matches_oracle(sphere2, d, bie, bc):
    P = _P()
    xyz, tri, dt = sphere2
    s = P.TDBEM(xyz, tri, 1.0, dt, d, bie, bc, nt_max=64)
    ref = mot.DirectMOT(xyz, tri, 1.0, dt, d, bie, bc)
    u = synth.random_history(s.ns, 40, seed=1)
    q = synth.random_history(s.ns, 40, seed=2)
    dev = torch.device("cuda")
    for nsteps in (0, 1, 5, 39):
        s.set_history(torch.tensor(u[:nsteps], device=dev) if nsteps else None,
                      torch.tensor(q[:nsteps], device=dev) if nsteps else None)
        got = s.fmm_eval(nsteps + 1).cpu().numpy()
        want = ref.history_rhs(nsteps + 1, u, q)
        if nsteps == 0:
            assert np.all(got == 0.0)
        else:
            assert _rel(got, want) < 1e-12, (nsteps, _rel(got, want))


@pytest.mark.parametrize("kind", ["gauss_mod", "raised_cos"])
@pytest.mark.parametrize("bie", [0, 1])
def test_incident_forcing_matches_oracle(sphere2, kind, bie):
    P = _P()
    xyz, tri, dt = sphere2
    s = P.TDBEM(xyz, tri, 1.0, dt, 1, bie, 0, nt_max=8)
    inc = synth.incident_params(xyz, seed=4, kind=kind)
    got = s.incident_forcing(inc, 1, 63).cpu().numpy()
    want = mot.incident(elemint.Geometry(xyz, tri), inc, 1.0, dt, 64, bie)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("d,bie,bc,nt", [(1, 1, 0, 64), (2, 1, 1, 64), (1, 1, 1, 40), (1, 0, 1, 30)])
def test_march_matches_oracle(sphere2, d, bie, bc, nt):
    """Small sphere (320 faces), incident Gaussian-modulated plane wave; the BM d=1
    Dirichlet case is the small named workload (direct, Nt=64)."""
    P = _P()
    xyz, tri, dt = sphere2
    inc = synth.incident_params(xyz, seed=0)
    s = P.TDBEM(xyz, tri, 1.0, dt, d, bie, bc, nt_max=nt)
    x, info = s.run(nt, inc=inc)
    ref = mot.DirectMOT(xyz, tri, 1.0, dt, d, bie, bc)
    u, q = ref.run(nt, mot.incident(ref.geom, inc, 1.0, dt, nt, bie))
    want = q if bc == 0 else u
    assert info["steps"] == nt - 1 and info["max_resid"] < 1e-11
    assert _rel(x.cpu().numpy(), want) < 1e-10


def test_pulsating_sphere_prescribed_dirichlet(sphere2):
    """Non-homogeneous Dirichlet data through tdbem_step (known current-step part)."""
    P = _P()
    xyz, tri, dt = sphere2
    d, nt = 2, 40
    s = P.TDBEM(xyz, tri, 1.0, dt, d, P.BMBIE, P.DIRICHLET, nt_max=nt)
    ref = mot.DirectMOT(xyz, tri, 1.0, dt, d, mot.BMBIE, mot.DIRICHLET)
    f = lambda t: np.exp(-(t - 4.0) ** 2 / 0.5)
    ubar = f(dt * (np.arange(nt - 1) + 1.5))[:, None] * np.ones((1, s.ns))
    u, q = ref.run(nt, None, ubar)
    dev = torch.device("cuda")
    got = []
    for a in range(1, nt):
        x, inf = s.step(bc_values=torch.tensor(ubar[a - 1], device=dev))
        assert inf["alpha"] == a
        got.append(x.cpu().numpy())
    assert _rel(np.array(got), q) < 1e-10
    hu, hq = s.get_history(nt - 1)
    assert np.array_equal(hu.cpu().numpy(), ubar)


def test_deterministic_and_reset(sphere2):
    P = _P()
    xyz, tri, dt = sphere2
    inc = synth.incident_params(xyz, seed=0)
    s = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=48)
    a, _ = s.run(48, inc=inc)
    s.reset()
    b, _ = s.run(48, inc=inc)
    assert torch.equal(a, b)


def test_error_paths_forced_from_host(sphere2):
    P = _P()
    xyz, tri, dt = sphere2
    inc = synth.incident_params(xyz, seed=0)
    s = P.TDBEM(xyz, tri, 1.0, dt, 1, P.BMBIE, P.DIRICHLET, nt_max=40, gmres_maxiter=1)
    _, info = s.run(40, inc=inc, check=False)
    assert info["rc"] == P._native.E_NOT_CONVERGED
    s2 = P.TDBEM(xyz, tri, 1.0, dt, 1, P.BMBIE, P.DIRICHLET, nt_max=4)
    for _ in range(3):
        s2.step()
    with pytest.raises(P.TDBEMError) as e:
        s2.step()
    assert e.value.code == P._native.E_STATE
    with pytest.raises(P.TDBEMError):
        s2.fmm_eval(7)


def test_march_multi_workgroup_solver_matches_oracle():
    """Ns > 2048 selects the cooperative multi-workgroup GMRES; same parity bar."""
    P = _P()
    xyz, tri = synth.geodesic_sphere(11)             # 2420 faces
    dt = synth.mean_edge_length(xyz, tri)
    nt = 20
    inc = synth.incident_params(xyz, seed=2)
    s = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt)
    x, info = s.run(nt, inc=inc)
    ref = mot.DirectMOT(xyz, tri, 1.0, dt, 2, mot.BMBIE, mot.NEUMANN)
    u, q = ref.run(nt, mot.incident(ref.geom, inc, 1.0, dt, nt, mot.BMBIE))
    assert info["max_resid"] < 1e-11
    assert _rel(x.cpu().numpy(), u) < 1e-10
