"""Mixed boundary conditions (eq. ibvp with S_u and S_q both non-empty, phi_j of eq. linear)
and the off-surface field (Kirchhoff representation with the operators of eq. bie_disc)
through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import mot

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _P():
    import paper_2111_05205_amd as P
    return P


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def mixed_case():
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    from oracle.elemint import Geometry
    x = Geometry(xyz, tri).x
    phi = (x[:, 2] > 0.1).astype(np.int8)               # q given above z = 0.1, u given below
    nt = 40
    inc = synth.incident_params(xyz, seed=6)
    pres = 0.3 * synth.random_history(tri.shape[0], nt - 1, seed=8)
    ref = mot.DirectMOT(xyz, tri, 1.0, dt, 2, mot.BMBIE, mot.MIXED, phi=phi.astype(float))
    F = mot.incident(ref.geom, inc, 1.0, dt, nt, mot.BMBIE)
    u, q = ref.run(nt, F, pres)
    return xyz, tri, dt, phi, nt, F, pres, ref, u, q


def test_mixed_march_matches_oracle(mixed_case):
    P = _P()
    xyz, tri, dt, phi, nt, F, pres, ref, u, q = mixed_case
    s = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, face_bc=phi, nt_max=nt + 1)
    assert s.info()["bc"] == P.MIXED
    dev = torch.device("cuda")
    Fd = torch.tensor(F, device=dev)
    Pd = torch.tensor(pres, device=dev)
    xs = []
    for a in range(1, nt):
        x, info = s.step(forcing=Fd[a - 1].contiguous(), bc_values=Pd[a - 1].contiguous())
        xs.append(x.cpu().numpy())
    gu, gq = (t.cpu().numpy() for t in s.get_history(nt - 1))
    assert _rel(gu, u) < 1e-10 and _rel(gq, q) < 1e-10, (_rel(gu, u), _rel(gq, q))
    # the step output is the unknown: u on phi = 1 faces, q on phi = 0 faces
    unk = np.where(phi[None, :] > 0, u, q)
    assert _rel(np.array(xs), unk) < 1e-10
    s.close()


def test_field_matches_oracle(mixed_case):
    P = _P()
    xyz, tri, dt, phi, nt, F, pres, ref, u, q = mixed_case
    s = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, face_bc=phi, nt_max=nt + 1)
    dev = torch.device("cuda")
    s.set_history(torch.tensor(u, device=dev), torch.tensor(q, device=dev))
    pts = np.array([[1.5, 0.1, -0.2], [0.0, 2.2, 0.3], [-0.1, 0.2, 0.0], [0.4, -0.3, 1.3], [3.0, 0.0, 0.0]])
    for alpha in (10, 25, nt - 1):
        got = s.field(pts, alpha).cpu().numpy()
        want = ref.field(pts, alpha, u, q)
        assert np.abs(got - want).max() <= 1e-10 * max(np.abs(want).max(), 1e-300), (alpha, got, want)
    with pytest.raises(P.TDBEMError):
        s.field(pts, nt)          # rows up to nt-1 are not stored
    s.close()


def test_uniform_mixed_equals_the_pure_condition():
    P = _P()
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    inc = synth.incident_params(xyz, seed=2)
    nt = 30
    for bc, v in ((P.NEUMANN, 1), (P.DIRICHLET, 0)):
        a = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, bc, nt_max=nt)
        b = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, face_bc=np.full(tri.shape[0], v, np.int8), nt_max=nt)
        xa, _ = a.run(nt, inc=inc)
        xb, _ = b.run(nt, inc=inc)
        assert float(torch.linalg.norm(xa - xb) / torch.linalg.norm(xa)) <= 1e-14
        a.close()
        b.close()
    with pytest.raises(P.TDBEMError):
        P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, face_bc=np.full(tri.shape[0], 2, np.int8))
    with pytest.raises(P.TDBEMError):
        P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, face_bc=np.ones(tri.shape[0], np.int8), guess=P.GUESS_MLP)


def test_direct_rows_match_oracle_history_sums():
    """tdbem_direct_rows: the exact history part of b^{alpha-1} at selected rows (every element,
    coefficients on the fly) equals the oracle's direct history sum, for both Burton-Miller
    families; with an FMM context this is the reference its far field is checked against."""
    P = _P()
    xyz, tri = synth.icosphere(3)
    dt = synth.mean_edge_length(xyz, tri)
    ns = tri.shape[0]
    u = synth.random_history(ns, 40, seed=21)
    q = synth.random_history(ns, 40, seed=22)
    ref = mot.DirectMOT(xyz, tri, 1.0, dt, 2, mot.BMBIE, mot.NEUMANN)
    s = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, use_fmm=1, depth=3, p_s=3, p_t=3, nt_max=64)
    dev = torch.device("cuda")
    s.set_history(torch.tensor(u[:35], device=dev), torch.tensor(q[:35], device=dev))
    rows = np.random.default_rng(4).choice(ns, 40, replace=False)
    for alpha in (20, 36):
        got = s.direct_rows(rows, alpha).cpu().numpy()
        want = ref.history_rhs(alpha, u, q)[rows]
        assert _rel(got, want) < 1e-10, (alpha, _rel(got, want))
    s.close()


def test_direct_rows_at_the_benchmarked_size():
    """The same reference at 81 920 faces (the benchmarked instance), 6 sampled rows against the
    oracle's compact coefficients of those rows, computed one row block at a time."""
    P = _P()
    from oracle import elemint
    w = synth.workload("sphere82k")
    ns = w["tri"].shape[0]
    s = P.TDBEM(w["xyz"], w["tri"], w["c"], w["dt"], w["d"], w["bie"], w["bc"], use_fmm=1, depth=6, p_s=3, p_t=3,
                m2l_prec=P.M2L_FP32, nt_max=200)
    u = synth.random_history(ns, 120, seed=23)
    s.set_history(torch.tensor(u, device=torch.device("cuda")), None)
    rows = np.sort(np.random.default_rng(9).choice(ns, 6, replace=False))
    alpha = 121
    got = s.direct_rows(rows, alpha).cpu().numpy()
    g = elemint.Geometry(w["xyz"], w["tri"])
    gmax, C = elemint.compact_rows(g, w["d"], w["c"] * w["dt"], rows)
    want = np.zeros(len(rows))
    for gg in range(2, min(gmax, alpha) + 1):
        want -= C[3, :, gg, :] @ u[alpha - gg]
    assert _rel(got, want) < 1e-10, _rel(got, want)
    s.close()
