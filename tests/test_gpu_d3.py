"""Cubic B-splines (d = 3).

The oracle has the closed form of U (App. B, bracket I^3_n) for d = 3 but its
closed-form derivatives stop at d = 2, so the reference for the other families
is built from the oracle's U alone by central differences: W = -dU/dz along the
element normal n_j, Ubar = n_i.grad_x U - dU/ds, Wbar = n_i.grad_x W - dW/ds
(eq. U_W_BM), with steps of 1e-4 of the mean edge and of c dt.  Tolerance, of
the row's largest coefficient: 2e-6 for U and W; 2e-5 for Ubar and Wbar, whose
reference takes nested differences across the wavefront kink (the same
reference at d = 2, against the oracle's closed forms, is off by 4e-6).  Self
pairs (z -> 0+ limit) are compared for U only.  The second test runs the d = 3 rows of
Tables 2-3 on the paper's smallest sphere: every combination is unstable."""
import numpy as np
import pytest

import synth
from oracle import bspline, elemint

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _U(x, ni, V, nj, s, cdt, self_pair=False):
    return elemint.elem(x, ni, V, nj, s, 3, cdt, self_pair)[0] if s > 0.0 else 0.0


def _families(x, ni, V, nj, s, cdt, h, hs):
    def W(xx, ss):
        return -(_U(xx + h * nj, ni, V, nj, ss, cdt) - _U(xx - h * nj, ni, V, nj, ss, cdt)) / (2 * h)
    u = _U(x, ni, V, nj, s, cdt)
    w = W(x, s)
    ub = (_U(x + h * ni, ni, V, nj, s, cdt) - _U(x - h * ni, ni, V, nj, s, cdt)) / (2 * h) \
        - (_U(x, ni, V, nj, s + hs, cdt) - _U(x, ni, V, nj, s - hs, cdt)) / (2 * hs)
    wb = (W(x + h * ni, s) - W(x - h * ni, s)) / (2 * h) - (W(x, s + hs) - W(x, s - hs)) / (2 * hs)
    return np.array([u, w, ub, wb])


@pytest.mark.parametrize("bie", [0, 1])
def test_d3_near_table_against_differenced_oracle(bie):
    import paper_2111_05205_amd as P
    xyz, tri = synth.icosphere(1)
    g = elemint.Geometry(xyz, tri)
    cdt = synth.mean_edge_length(xyz, tri)
    s = P.TDBEM(xyz, tri, 1.0, cdt, 3, bie, P.NEUMANN, use_fmm=0, nt_max=8)
    w = bspline.weights(3)
    h, hs = 1e-4 * cdt, 1e-4 * cdt
    rows = [0, 7, 33, 61, 79]
    worst = 0.0
    for i in rows:
        jj, gg, cu, cw = s.near_row(i)
        scale = max(np.abs(cu).max(), np.abs(cw).max())
        for j, gv, a_u, a_w in zip(jj, gg, cu, cw):
            V = g.tris[j].reshape(3, 3)
            if i == j:
                if bie == 0:
                    ref = sum(w[k] * _U(g.x[i], g.n[i], V, g.n[j], cdt * (gv - k), cdt, True)
                              for k in range(5) if gv - k > 0)
                    worst = max(worst, abs(a_u - ref) / scale)
                continue
            ref = np.zeros(4)
            for k in range(5):
                if gv - k > 0:
                    ref += w[k] * _families(g.x[i], g.n[i], V, g.n[j], cdt * (gv - k), cdt, h, hs)
            ru, rw = (ref[2], ref[3]) if bie else (ref[0], ref[1])
            worst = max(worst, abs(a_u - ru) / scale, abs(a_w - rw) / scale)
    assert worst < (2e-5 if bie else 2e-6), worst


def test_d3_unstable_on_the_papers_sphere():
    import paper_2111_05205_amd as P
    v, f = synth.geodesic_sphere(12)
    xyz = 0.5 * v + np.array([0.5, 0.0, 0.0])
    inc = dict(kind="raised_cos", dir=[1.0, 0.0, 0.0], sigma=0.5, t0=0.0, rb=0.0)
    nt = 240
    for bie in (0, 1):
        for bc in (0, 1):
            sv = P.TDBEM(xyz, f, 1.0, 0.04, 3, bie, bc, use_fmm=0, nt_max=nt, gmres_tol=1e-10, gmres_maxiter=400)
            x, ri = sv.run(nt, inc=inc, check=False)
            mx = x.abs().max(dim=1).values.cpu().numpy()
            overflow = ri["rc"] == P._native.E_DIVERGED or not np.all(np.isfinite(mx))
            ratio = np.inf if overflow else mx[-nt // 5:].max() / mx[: nt // 3].max()
            print(f"d=3 bie={bie} bc={bc}: growth ratio {ratio:.3e}")
            assert overflow or ratio > 10.0
    # the FMM path at d = 3 (p_t must exceed d)
    sv = P.create_fmm(xyz, f, 1.0, 0.04, 3, 1, 1, p_s=4, p_t=4, nt_max=nt, gmres_tol=1e-10, gmres_maxiter=400)
    x, ri = sv.run(nt, inc=inc, check=False)
    mx = x.abs().max(dim=1).values.cpu().numpy()
    overflow = ri["rc"] == P._native.E_DIVERGED or not np.all(np.isfinite(mx))
    assert overflow or mx[-nt // 5:].max() / mx[: nt // 3].max() > 10.0
