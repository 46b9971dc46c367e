"""Stability pattern of the paper's sphere examples (Section 5.1, Tables 2 and 3)
for d = 1, 2 on the smallest of its meshes: sphere of radius 0.5 centred at
(0.5, 0, 0), 2880 faces, dt = 0.04, Nt = 240, raised-cosine plane pulse of
length 0.5 travelling along +x1, direct evaluation.  The paper reports: for the
homogeneous Dirichlet problem the OBIE diverges for every d and the BMBIE runs
for d = 1 only; for the Neumann problem the OBIE runs for d = 1 and diverges for
d = 2, the BMBIE runs for d = 1 and 2.  A march counts as stable when the largest
coefficient over the last fifth of the steps is below that over the first third
(the pulse has long passed), and as unstable when it is more than ten times it
or the solution overflows."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (bie, bc, d) -> stable?   bie 0 = OBIE, 1 = BMBIE; bc 0 = Dirichlet, 1 = Neumann
PATTERN = {(0, 0, 1): False, (0, 0, 2): False, (1, 0, 1): True, (1, 0, 2): False,
           (0, 1, 1): True, (0, 1, 2): False, (1, 1, 1): True, (1, 1, 2): True}


@pytest.fixture(scope="module")
def sphere():
    v, f = synth.geodesic_sphere(12)
    return 0.5 * v + np.array([0.5, 0.0, 0.0]), f


def _growth_ratio(P, s, nt, inc):
    x, ri = s.run(nt, inc=inc, check=False)
    mx = x.abs().max(dim=1).values.cpu().numpy()
    overflow = ri["rc"] == P._native.E_DIVERGED or not np.all(np.isfinite(mx))
    return np.inf if overflow else mx[-nt // 5:].max() / mx[: nt // 3].max()


def _check(key, ratio):
    if PATTERN[key]:
        assert ratio < 1.0, ratio
    else:
        assert ratio > 10.0, ratio


INC = dict(kind="raised_cos", dir=[1.0, 0.0, 0.0], sigma=0.5, t0=0.0, rb=0.0)


@pytest.mark.parametrize("key", sorted(PATTERN))
def test_stability_pattern_of_tables_2_and_3(sphere, key):
    import paper_2111_05205_amd as P
    bie, bc, d = key
    xyz, tri = sphere
    nt = 240
    inc = dict(kind="raised_cos", dir=[1.0, 0.0, 0.0], sigma=0.5, t0=0.0, rb=0.0)
    s = P.TDBEM(xyz, tri, 1.0, 0.04, d, bie, bc, use_fmm=0, nt_max=nt, gmres_tol=1e-10, gmres_maxiter=400)
    x, ri = s.run(nt, inc=inc, check=False)
    mx = x.abs().max(dim=1).values.cpu().numpy()
    overflow = ri["rc"] == P._native.E_DIVERGED or not np.all(np.isfinite(mx))
    ratio = np.inf if overflow else mx[-nt // 5:].max() / mx[: nt // 3].max()
    print(f"bie={bie} bc={bc} d={d}: growth ratio {ratio:.3e}")
    if PATTERN[key]:
        assert not overflow and ratio < 1.0, ratio
    else:
        assert overflow or ratio > 10.0, ratio


def test_growth_check_flags_the_unstable_march(sphere):
    """opts.growth_limit: the d = 2 Burton-Miller Dirichlet march (unstable, Table 2) fails with
    TDBEM_E_DIVERGED once its solution exceeds 10 times the largest value of the rows at least 80
    steps older; the d = 1 march (stable) runs through with the same check; the check changes no
    value of a march it does not stop."""
    import paper_2111_05205_amd as P
    xyz, tri = sphere
    nt = 240
    inc = dict(kind="raised_cos", dir=[1.0, 0.0, 0.0], sigma=0.5, t0=0.0, rb=0.0)
    kw = dict(use_fmm=0, nt_max=nt, gmres_tol=1e-10, gmres_maxiter=400)
    s = P.TDBEM(xyz, tri, 1.0, 0.04, 2, P.BMBIE, P.DIRICHLET, growth_limit=10.0, growth_lag=80, **kw)
    _, ri = s.run(nt, inc=inc, check=False)
    assert ri["rc"] == P._native.E_DIVERGED
    assert "growth_limit" in s.last_error()
    a = P.TDBEM(xyz, tri, 1.0, 0.04, 1, P.BMBIE, P.DIRICHLET, growth_limit=10.0, growth_lag=80, **kw)
    xa, ra = a.run(nt, inc=inc, check=False)
    assert ra["rc"] == 0
    b = P.TDBEM(xyz, tri, 1.0, 0.04, 1, P.BMBIE, P.DIRICHLET, **kw)
    xb, _ = b.run(nt, inc=inc)
    assert torch.equal(xa, xb)
    with pytest.raises(P.TDBEMError):
        P.TDBEM(xyz, tri, 1.0, 0.04, 1, P.BMBIE, P.DIRICHLET, growth_limit=10.0, growth_lag=0, **kw)


@pytest.mark.parametrize("key", sorted(PATTERN))
def test_stability_pattern_with_the_fmm(sphere, key):
    """The FMM rows of Tables 2-3 (p_s = p_t = 4, deepest octree the time step allows)."""
    import paper_2111_05205_amd as P
    bie, bc, d = key
    xyz, tri = sphere
    nt = 240
    s = P.create_fmm(xyz, tri, 1.0, 0.04, d, bie, bc, p_s=4, p_t=4, nt_max=nt, gmres_tol=1e-10, gmres_maxiter=400)
    ratio = _growth_ratio(P, s, nt, INC)
    print(f"FMM bie={bie} bc={bc} d={d}: growth ratio {ratio:.3e}")
    _check(key, ratio)


@pytest.mark.parametrize("level,dt,nt", [(16, 0.03, 320), (24, 0.02, 480)])
def test_stability_pattern_on_the_finer_meshes(level, dt, nt):
    """The 5120- and 11520-face spheres of Section 5.1 (dt = 0.03, 0.02; Nt = 320, 480), direct."""
    import paper_2111_05205_amd as P
    v, f = synth.geodesic_sphere(level)
    xyz = 0.5 * v + np.array([0.5, 0.0, 0.0])
    assert f.shape[0] == 20 * level * level
    for key in sorted(PATTERN):
        bie, bc, d = key
        s = P.TDBEM(xyz, f, 1.0, dt, d, bie, bc, use_fmm=0, nt_max=nt, gmres_tol=1e-10, gmres_maxiter=400)
        ratio = _growth_ratio(P, s, nt, INC)
        print(f"{f.shape[0]} faces bie={bie} bc={bc} d={d}: growth ratio {ratio:.3e}")
        _check(key, ratio)
        s.close()


def test_march_on_the_papers_sphere_matches_the_oracle(sphere):
    """The configuration of the stability study (2880-face sphere, dt = 0.04, raised-cosine
    pulse, Burton-Miller, Dirichlet, d = 2) against the FP64 oracle's direct march, 80 steps."""
    import paper_2111_05205_amd as P
    from oracle import mot
    xyz, tri = sphere
    nt = 80
    ref = mot.DirectMOT(xyz, tri, 1.0, 0.04, 2, mot.BMBIE, mot.DIRICHLET)
    _, q = ref.run(nt, mot.incident(ref.geom, INC, 1.0, 0.04, nt, mot.BMBIE))
    s = P.TDBEM(xyz, tri, 1.0, 0.04, 2, P.BMBIE, P.DIRICHLET, use_fmm=0, nt_max=nt, gmres_tol=1e-13)
    x, info = s.run(nt, inc=INC)
    err = float(np.linalg.norm(x.cpu().numpy() - q) / np.linalg.norm(q))
    print(f"2880 faces, BM Dirichlet d=2, 80 steps: GPU vs oracle {err:.2e}")
    assert err < 1e-10
