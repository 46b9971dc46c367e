"""ORACLE (test infrastructure): direct marching-on-in-time (no FMM), FP64.

Plain definition of the discretised BIEs (eq. bie_disc for the OBIE and its
Burton-Miller analogue with Ubar, Wbar of eq. U_W_BM), collocated at face
centroids and times t_alpha = alpha*dt, alpha = 1..Nt-1, with the incident
field kept as a forcing term (total-field reading of the problem statement):

  0 = f_i^alpha + sum_j sum_{beta=0}^{alpha-1} ( C_U^{(alpha-beta)}_ij q_j^beta
                                              - C_W^{(alpha-beta)}_ij u_j^beta )

C_X^{(g)} = sum_kappa w^kappa X^{(g-kappa)} are the compact (kappa-summed)
coefficients.  The unknown at step alpha is x^{alpha-1} (u on Neumann faces,
q on Dirichlet faces); the per-step matrix A = C_W^{(1)} phi - C_U^{(1)} (1-phi)
= w^{0,d} (W^{(1)} phi - U^{(1)} (1-phi)) is constant (eq. linear), so it is
LU-factorised once.
"""
import numpy as np
import scipy.linalg as sla

from .bspline import weights
from .elemint import Geometry, compact_coefficients, compact_points

OBIE, BMBIE = 0, 1
DIRICHLET, NEUMANN, MIXED = 0, 1, 2


def incident(geom: Geometry, inc: dict, c: float, dt: float, nt: int, bie: int) -> np.ndarray:
    """Forcing f^alpha, alpha = 1..nt-1 (row alpha-1): u_in for the OBIE,
    (d/dn - (1/c) d/dt) u_in with the paper normal for the BMBIE."""
    k = np.asarray(inc["dir"], dtype=np.float64)
    t = dt * np.arange(1, nt)[:, None]
    kx = geom.x @ k
    kn = geom.n @ k
    if inc["kind"] == "gauss_mod":
        p = t - (kx[None, :] + inc["rb"]) / c - inc["t0"]
        sg, w = inc["sigma"], 2.0 * np.pi * inc["f0"]
        env = np.exp(-p * p / (2.0 * sg * sg))
        g = env * np.cos(w * p)
        gp = env * (-p / (sg * sg) * np.cos(w * p) - w * np.sin(w * p))   # d g / d p
        if bie == OBIE:
            return g
        # grad u = g' * (-k/c), du/dt = g'
        return gp * (-kn[None, :] / c) - gp / c
    if inc["kind"] == "raised_cos":
        lam = inc["sigma"]
        a = 2.0 * np.pi * (c * t - kx[None, :] - inc["rb"]) / lam
        inside = (a >= 0.0) & (a <= 2.0 * np.pi)
        u = np.where(inside, 0.5 * (1.0 - np.cos(a)), 0.0)
        du = np.where(inside, 0.5 * np.sin(a), 0.0)          # d u / d a
        if bie == OBIE:
            return u
        return du * (2.0 * np.pi / lam) * (-kn[None, :] - 1.0)
    raise ValueError(inc["kind"])


class DirectMOT:
    """Direct MOT on one closed surface; see module docstring.

    bc = MIXED with phi (ns values, 1 on faces where q is given and u unknown, 0 where u
    is given and q unknown): the boundary S_u / S_q split of eq. ibvp with phi_j as in
    eq. linear, A = C_W^{(1)} diag(phi) - C_U^{(1)} diag(1 - phi)."""

    def __init__(self, xyz, tri, c, dt, d, bie, bc, phi=None):
        self.geom = Geometry(xyz, tri)
        self.c, self.dt, self.d, self.bie, self.bc = float(c), float(dt), int(d), int(bie), int(bc)
        self.gmax, fams = compact_coefficients(self.geom, self.d, self.c * self.dt)
        self.CU = fams["Ubar" if bie == BMBIE else "U"]
        self.CW = fams["Wbar" if bie == BMBIE else "W"]
        if bc == MIXED:
            self.phi = np.asarray(phi, dtype=np.float64)
        else:
            self.phi = np.full(self.geom.ns, 1.0 if bc == NEUMANN else 0.0)
        A = self.CW[1].toarray() * self.phi[None, :] - self.CU[1].toarray() * (1.0 - self.phi)[None, :]
        self.A = A
        self.lu = sla.lu_factor(A)

    @property
    def ns(self):
        return self.geom.ns

    def history_rhs(self, alpha: int, u: np.ndarray, q: np.ndarray) -> np.ndarray:
        """sum_{beta=0}^{alpha-2} (C_U^{(alpha-beta)} q^beta - C_W^{(alpha-beta)} u^beta):
        the part of b^{alpha-1} carried by already-solved steps."""
        b = np.zeros(self.ns)
        for g in range(2, min(self.gmax, alpha) + 1):
            beta = alpha - g
            b += self.CU[g] @ q[beta] - self.CW[g] @ u[beta]
        return b

    def run(self, nt: int, forcing=None, prescribed=None):
        """March alpha = 1..nt-1.  forcing: (nt-1, ns) or None; prescribed: the known
        coefficient per step and face (u on Dirichlet faces, q on Neumann faces), (nt-1, ns)
        or None (= 0).  Returns (u, q), each (nt-1, ns): B-spline coefficients beta = 0..nt-2."""
        ns = self.ns
        ph = self.phi
        u = np.zeros((nt - 1, ns))
        q = np.zeros((nt - 1, ns))
        for alpha in range(1, nt):
            beta = alpha - 1
            b = self.history_rhs(alpha, u, q)
            if forcing is not None:
                b += forcing[beta]
            p = prescribed[beta] if prescribed is not None else np.zeros(ns)
            # the known current-step part: q given on phi = 1 faces, u given on phi = 0 faces
            b += self.CU[1] @ (ph * p) - self.CW[1] @ ((1.0 - ph) * p)
            x = sla.lu_solve(self.lu, b)
            u[beta] = ph * x + (1.0 - ph) * p
            q[beta] = (1.0 - ph) * x + ph * p
        return u, q

    def field(self, pts, alpha: int, u: np.ndarray, q: np.ndarray) -> np.ndarray:
        """Scattered part of the field at off-surface points pts (npts x 3) and time t_alpha from
        the solved coefficients beta = 0..alpha-1 (Kirchhoff representation of the exterior
        field, the operators of eq. bie_disc at a point that is not a collocation point):
        sum_j sum_{g=1}^{alpha} (C_U^{(g)}(x, E_j) q_j^{alpha-g} - C_W^{(g)}(x, E_j) u_j^{alpha-g}).
        Add u_in(x, t_alpha) for the total field; inside the scatterer the sum cancels u_in."""
        gmax, C = compact_points(self.geom, self.d, self.c * self.dt, pts)
        out = np.zeros(C.shape[1])
        for g in range(1, min(gmax, alpha) + 1):
            out += C[0, :, g, :] @ q[alpha - g] - C[1, :, g, :] @ u[alpha - g]
        return out


def reconstruct(coef: np.ndarray, d: int) -> np.ndarray:
    """v(t_alpha) = sum_beta N^{beta,d}(t_alpha) v^beta for alpha = 1..len(coef) (row alpha-1)."""
    w = weights(d)
    nb = coef.shape[0]
    out = np.zeros_like(coef)
    for alpha in range(1, nb + 1):
        for beta in range(max(0, alpha - d - 1), alpha):
            nv = sum(w[k] * max(alpha - k - beta, 0) ** d for k in range(d + 2))
            out[alpha - 1] += nv * coef[beta]
    return out
