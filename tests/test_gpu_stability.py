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
