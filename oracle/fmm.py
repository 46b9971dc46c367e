"""ORACLE (test infrastructure): plain reference of the interpolation-based
space-time FMM, FP64, numpy.  Written from the paper's Section 3 (eqs.
target, U_intp, Uabmn, target_m2l, m2l, the Burton-Miller evaluation of the
local field) and Section 4 (eqs. m2l_actual, m2l_naive, m2l_near, U_expand,
m2l_expand, Formula 1 with eqs. m2l_rec, L_derivative, m2l_expand_rec1, L_aux,
m2l_expand_rec2, cmp, and Algorithm 1).

Where the paper leaves the construction open, this module takes these readings:
* Interpolation (interp="lagrange", the default): tensor-product Lagrange on
  Chebyshev points of the first kind in each of the eight variables.
  interp="hermite" is the paper's own choice (Section 3, after eq. Uabmn):
  piecewise cubic Hermite interpolation whose nodal slopes are finite
  differences of the nodal values.  Read here as: p >= 3 equispaced nodes
  -1 = w_0 < ... < w_{p-1} = 1, central differences at interior nodes and
  second-order one-sided differences at the two end nodes (so that quadratics
  are reproduced), the end pieces continued outside [-1, 1].
* Octree: root cube centred on the vertex bounding box with half side the
  next power of two of its largest half extent; faces assigned to leaves by
  centroid; near field = the 27 leaves around a face's leaf; interaction
  list (level >= 2) = children of the parent's neighbours that are not
  neighbours.  Offsets of IL cells take 316 values.
* Time hierarchy: M_leaf steps per leaf interval, doubling per level.  A
  source sample tau^{beta} (time t_beta) belongs to level-l interval
  floor((beta+1)/M_l) and a target t_alpha to floor(alpha/M_l) -- the
  classification of the paper's eq. target, where tau^{beta-1} is grouped by
  t_beta.  Source intervals are centred on the sample times they hold, so
  target and source centres differ by ((l-k) M + 1) dt.  M_leaf is the largest
  value for which every same-interval interaction-list pair is exactly zero
  by causality, so intervals only cast to later intervals.
* mu: smallest value for which c (t - s) - r > 0 at every node pair of the
  expansion interval k+mu+1 (all levels, all 316 offsets), so the distant
  future M2L of eq. m2l_expand is exact at the nodes.
* M2M / L2L: re-interpolation between parent and child nodes (not written in
  the paper); M2M at source-interval end, L2L at target-interval start.

Only tests/, the smoke check and the benchmark's CPU-baseline leg use it.
"""
from math import comb

import numpy as np

from .bspline import weights
from .elemint import Geometry, compact_coefficients

OFFSETS = [(a, b, c) for a in range(-3, 4) for b in range(-3, 4) for c in range(-3, 4)
           if max(abs(a), abs(b), abs(c)) >= 2]


def cheb_nodes(p):
    return np.cos((2 * np.arange(p) + 1) * np.pi / (2 * p))


def lagrange(nodes, xi):
    """l_a(xi) for all a: array (len(xi), p)."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    p = len(nodes)
    out = np.ones((xi.size, p))
    for a in range(p):
        for b in range(p):
            if b != a:
                out[:, a] *= (xi - nodes[b]) / (nodes[a] - nodes[b])
    return out


def lagrange_deriv(nodes, xi):
    """d l_a / d xi for all a: array (len(xi), p)."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    p = len(nodes)
    out = np.zeros((xi.size, p))
    for a in range(p):
        for c in range(p):
            if c == a:
                continue
            term = np.full(xi.size, 1.0 / (nodes[a] - nodes[c]))
            for b in range(p):
                if b != a and b != c:
                    term = term * (xi - nodes[b]) / (nodes[a] - nodes[b])
            out[:, a] += term
    return out


def equi_nodes(p):
    if p < 3:
        raise ValueError("the cubic Hermite interpolation needs p >= 3 nodes")
    return np.linspace(-1.0, 1.0, p)


def _fd_slopes(p, h):
    """D (p x p): nodal slopes f'(w_k) ~ sum_a D[k, a] f(w_a) by finite differences."""
    D = np.zeros((p, p))
    for k in range(1, p - 1):
        D[k, k + 1], D[k, k - 1] = 1.0 / (2 * h), -1.0 / (2 * h)
    D[0, :3] = np.array([-3.0, 4.0, -1.0]) / (2 * h)
    D[p - 1, p - 3:] = np.array([1.0, -4.0, 3.0]) / (2 * h)
    return D


def _hermite_parts(nodes, xi):
    """Segment index k, local coordinate t in the segment, node spacing h and slope matrix D."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    p = len(nodes)
    h = nodes[1] - nodes[0]
    k = np.clip(np.floor((xi - nodes[0]) / h).astype(np.int64), 0, p - 2)
    t = (xi - nodes[k]) / h
    return xi, k, t, h, _fd_slopes(p, h)


def hermite_fd(nodes, xi):
    """Cardinal functions of the cubic Hermite interpolation with finite-difference slopes:
    on the segment [w_k, w_k+1] the interpolant is h00 f_k + h01 f_k+1 + h (h10 m_k + h11 m_k+1)
    with the cubic Hermite polynomials h00 .. h11 of t in [0, 1] and slopes m = D f.
    Array (len(xi), p)."""
    xi, k, t, h, D = _hermite_parts(nodes, xi)
    h00, h01 = 2 * t ** 3 - 3 * t ** 2 + 1, -2 * t ** 3 + 3 * t ** 2
    h10, h11 = t ** 3 - 2 * t ** 2 + t, t ** 3 - t ** 2
    rows = np.arange(xi.size)
    out = h * (h10[:, None] * D[k] + h11[:, None] * D[k + 1])
    out[rows, k] += h00
    out[rows, k + 1] += h01
    return out


def hermite_fd_deriv(nodes, xi):
    """d/dxi of hermite_fd: array (len(xi), p)."""
    xi, k, t, h, D = _hermite_parts(nodes, xi)
    d00, d01 = (6 * t ** 2 - 6 * t) / h, (-6 * t ** 2 + 6 * t) / h
    d10, d11 = 3 * t ** 2 - 4 * t + 1, 3 * t ** 2 - 2 * t
    rows = np.arange(xi.size)
    out = d10[:, None] * D[k] + d11[:, None] * D[k + 1]
    out[rows, k] += d00
    out[rows, k + 1] += d01
    return out


def cmp_coef(p, m, k):
    """c_m^p(k) of eq. cmp."""
    return comb(p, m) * ((k - 1) ** (p - m) - 2 * k ** (p - m) + (k + 1) ** (p - m)) * (-1) ** m


def recurrence(k, mu, d, T, ring, R, Lp, aux, Dp):
    """Distant-future part of Algorithm 1 for current interval k, after its near-future
    products: eq. m2l_expand_rec1 (derivatives, with the auxiliaries of k-1), eq. m2l_rec
    (local of interval k+mu+2), eq. m2l_expand_rec2 (auxiliaries).  ring[(l) % R] holds L_l;
    Lp[p] = L^{(p)}, aux[p, m] = L^{(p,m)}, Dp[p] = L^{(p)}_{k+mu+1,k} (p = 1..d)."""
    for p in range(1, d + 1):
        upd = Lp[p] + Dp[p]
        for m in range(0, p - 1):
            upd = upd + cmp_coef(p, m, k) * aux[p, m]
        Lp[p] = upd
    ring[(k + mu + 2) % R] = ring[(k + mu + 1) % R] + sum(Lp[p] * T ** p for p in range(1, d + 1))
    for p in range(2, d + 1):
        for m in range(0, p - 1):
            aux[p, m] = aux[p, m] + Dp[p] * float(k) ** m


def _tensor3(v1, v2, v3):
    """index a1 + p (a2 + p a3) of the product v1[a1] v2[a2] v3[a3] (per row)."""
    n, p = v1.shape
    return (v1[:, None, None, :] * v2[:, None, :, None] * v3[:, :, None, None]).reshape(n, p ** 3)


class ReferenceFMM:
    """History part of the MOT right-hand side with near pairs direct and far pairs by the FMM."""

    def __init__(self, xyz, tri, c, dt, d, bie, depth, p_s, p_t, mu=0, m2l="alg1", bc=None, src_ext=None,
                 near_round=None, interp="lagrange", near_product=None, leaf_ratio=None):
        """near_round: None, or a function applied to both factors (moments and operator) of
        the near-future products (eq. m2l_near) whose operator block is truncated at some node
        pairs and not zero at all of them (where the wavefront crosses the pair's node set),
        e.g. rounding to a lower precision; every other block is a polynomial at the nodes
        or zero, and those products and the derivative products stay exact.
        near_product: None, or a function (X, U) -> X @ U.T as a lower-precision path forms
        the products of those same blocks (e.g. from split factors).
        leaf_ratio: None, or the leaf side in units of c dt: the root cube (centred as usual) gets
        half side leaf_ratio c dt 2^D / 2 with the smallest D >= 2 that holds the mesh, and depth
        is ignored (the sizing under which the operators of a level, in units of c dt and dt,
        depend only on its distance from the leaves)."""
        self.leaf_ratio = leaf_ratio
        self.near_round = near_round
        self.near_product = near_product
        self.geom = g = Geometry(xyz, tri)
        self.bc = bc
        self._src_ext = src_ext
        self.c, self.dt, self.d, self.bie = float(c), float(dt), int(d), int(bie)
        self.D, self.ps, self.pt = int(depth), int(p_s), int(p_t)
        self.m2l = m2l
        self.Cd = 1.0 / (4.0 * np.pi * (self.c * self.dt) ** self.d)
        self.w = weights(self.d)
        if interp == "lagrange":
            self.om_s, self.om_t = cheb_nodes(self.ps), cheb_nodes(self.pt)
            self._l, self._dl = lagrange, lagrange_deriv
        elif interp == "hermite":
            self.om_s, self.om_t = equi_nodes(self.ps), equi_nodes(self.pt)
            self._l, self._dl = hermite_fd, hermite_fd_deriv
        else:
            raise ValueError("interp must be 'lagrange' or 'hermite'")
        self.interp = interp
        self.Ps = self.ps ** 3
        self.P = self.Ps * self.pt
        self._tree(np.asarray(xyz, dtype=np.float64))
        self._hierarchy(mu)
        self._near()
        self._tables()
        self._translations()
        self.reset()

    # ---------------- tree ----------------
    def _tree(self, xyz):
        g, D = self.geom, self.D
        lo, hi = xyz.min(0), xyz.max(0)
        self.center = (lo + hi) / 2.0
        ext = float(((hi - lo) / 2.0).max())
        if self.leaf_ratio:
            hl = 0.5 * self.leaf_ratio * self.c * self.dt
            D = 2
            while D < 12 and hl * 2 ** D < ext:
                D += 1
            self.D = D
            self.H = hl * 2 ** D
        else:
            self.H = 2.0 ** np.ceil(np.log2(ext))
        n = 2 ** D
        idx = np.floor((g.x - (self.center - self.H)) / (2.0 * self.H) * n).astype(np.int64)
        self.leaf_idx = np.clip(idx, 0, n - 1)
        a, b, cc = g.tris[:, 0:3], g.tris[:, 3:6], g.tris[:, 6:9]
        self.e_max = float(max(np.linalg.norm(v - g.x, axis=1).max() for v in (a, b, cc)))
        self.src_ext = 0.0 if self._src_ext is None else float(self._src_ext)
        self.cells, self.cell_of, self.members = [], [], []
        for lev in range(D + 1):
            keys = [tuple(k) for k in (self.leaf_idx >> (D - lev))]
            uniq = sorted(set(keys))
            pos = {k: i for i, k in enumerate(uniq)}
            self.cells.append(uniq)
            self.cell_of.append(np.array([pos[k] for k in keys]))
            mem = [[] for _ in uniq]
            for e, k in enumerate(keys):
                mem[pos[k]].append(e)
            self.members.append(mem)
        # interaction lists, level >= 2
        self.il = {}
        for lev in range(2, D + 1):
            cells = self.cells[lev]
            pos = {k: i for i, k in enumerate(cells)}
            lst = []
            for oi, O in enumerate(cells):
                par = tuple(v >> 1 for v in O)
                for S, si in pos.items():
                    sp = tuple(v >> 1 for v in S)
                    if max(abs(sp[q] - par[q]) for q in range(3)) <= 1 and max(abs(S[q] - O[q]) for q in range(3)) > 1:
                        lst.append((oi, si, tuple(S[q] - O[q] for q in range(3))))
            self.il[lev] = lst
        self.il_by_off = {}
        for lev in range(2, D + 1):
            grp = {}
            for (oi, si, o) in self.il[lev]:
                grp.setdefault(o, ([], []))
                grp[o][0].append(oi)
                grp[o][1].append(si)
            self.il_by_off[lev] = {o: (np.array(a), np.array(b)) for o, (a, b) in grp.items()}
        # parent index and octant (side per axis) of every cell
        self.parent, self.octant = {}, {}
        for lev in range(1, D + 1):
            pos = {k: i for i, k in enumerate(self.cells[lev - 1])}
            self.parent[lev] = np.array([pos[tuple(v >> 1 for v in key)] for key in self.cells[lev]])
            self.octant[lev] = np.array([[1 if (key[q] & 1) else -1 for q in range(3)] for key in self.cells[lev]])

    def cell_center(self, lev, key):
        return self.center - self.H + (np.asarray(key, dtype=np.float64) + 0.5) * (2.0 * self.H / 2 ** lev)

    def hs(self, lev):
        return self.H / 2 ** lev

    def hb(self, lev):
        """Half side of the source interpolation box: the cell, optionally grown by src_ext (e.g.
        the largest distance a face reaches beyond its centroid) so that no source point lies
        outside its box.  Default 0: the box is the cell."""
        return self.hs(lev) + self.src_ext

    # ---------------- time hierarchy ----------------
    def _hierarchy(self, mu):
        cdt = self.c * self.dt
        m_leaf = int(np.floor((2.0 * self.hs(self.D) - self.e_max) / cdt))
        if m_leaf < 1:
            raise ValueError("octree too deep for this time step: leaf interval would be empty")
        self.m_leaf = m_leaf
        self.M = {lev: m_leaf * 2 ** (self.D - lev) for lev in range(self.D + 1)}
        # smallest mu with c (t - s) - r > 0 at every node pair of interval k+mu+1
        need = 1
        for lev in range(2, self.D + 1):
            hs, ht, Ml = self.hs(lev), self.ht(lev), self.M[lev]
            X = hs * np.stack(np.meshgrid(self.om_s, self.om_s, self.om_s, indexing="ij"), -1).reshape(-1, 3)
            Y = X * (self.hb(lev) / hs)
            rmax = 0.0
            for o in OFFSETS:
                y = 2.0 * hs * np.array(o, dtype=float) + Y
                r = np.linalg.norm(X[:, None, :] - y[None, :, :], axis=2)
                rmax = max(rmax, r.max())
            dmin = float((self.om_t[:, None] - self.om_t[None, :]).min())
            m = 1
            while self.c * (((m + 1) * Ml + 1) * self.dt + ht * dmin) - rmax <= 0.0:
                m += 1
            need = max(need, m)
        if mu and mu < need:
            raise ValueError(f"mu={mu} too small, need >= {need}")
        self.mu = int(mu) if mu else need

    def ht(self, lev):
        return self.M[lev] * self.dt / 2.0

    def src_center(self, lev, k):
        Ml = self.M[lev]
        return (k * Ml - 1 + (Ml - 1) / 2.0) * self.dt

    def tgt_center(self, lev, k):
        Ml = self.M[lev]
        return (k * Ml + (Ml - 1) / 2.0) * self.dt

    # ---------------- near field ----------------
    def _near(self):
        g = self.geom
        ns = g.ns
        li = self.leaf_idx
        diff = np.abs(li[:, None, :] - li[None, :, :]).max(axis=2)
        self.near_mask = diff <= 1
        gmax, fams = compact_coefficients(g, self.d, self.c * self.dt)
        self.gmax = gmax
        CU = fams["Ubar" if self.bie else "U"]
        CW = fams["Wbar" if self.bie else "W"]
        mask = self.near_mask
        self.CU = {k: v.multiply(mask).tocsr() for k, v in CU.items()}
        self.CW = {k: v.multiply(mask).tocsr() for k, v in CW.items()}
        self.near_pairs = int(mask.sum())

    # ---------------- element tables ----------------
    def _tables(self):
        g, D = self.geom, self.D
        # P2M: A_jb = int_E l_b, B_jb = int_E n . grad l_b  (degree 3(p_s-1) rule on the triangle)
        nq = max(4, (3 * (self.ps - 1) + 3) // 2)
        xg, wg = np.polynomial.legendre.leggauss(nq)
        u, wu = (xg + 1) / 2, wg / 2
        hs = self.hs(D)
        hb = self.hb(D)
        ns = g.ns
        self.A = np.zeros((ns, self.Ps))
        self.B = np.zeros((ns, self.Ps))
        self.E0 = np.zeros((ns, self.Ps))
        self.E1 = np.zeros((ns, self.Ps))
        for j in range(ns):
            V = g.tris[j].reshape(3, 3)
            area2 = 2.0 * g.area[j]
            cen = self.cell_center(D, self.cells[D][self.cell_of[D][j]])
            pts, wts = [], []
            for a_, wa in zip(u, wu):
                for b_, wb in zip(u, wu):
                    pts.append(V[0] + a_ * (V[1] - V[0]) + a_ * b_ * (V[2] - V[1]))
                    wts.append(wa * wb * a_ * area2)
            pts, wts = np.array(pts), np.array(wts)
            xi = (pts - cen) / hb
            L = [self._l(self.om_s, xi[:, q]) for q in range(3)]
            dL = [self._dl(self.om_s, xi[:, q]) for q in range(3)]
            n = g.n[j]
            val = _tensor3(L[0], L[1], L[2])
            grad = n[0] * _tensor3(dL[0], L[1], L[2]) + n[1] * _tensor3(L[0], dL[1], L[2]) \
                + n[2] * _tensor3(L[0], L[1], dL[2])
            self.A[j] = wts @ val
            self.B[j] = wts @ grad / hb
            xi0 = (g.x[j] - cen) / hs
            L0 = [self._l(self.om_s, [xi0[q]]) for q in range(3)]
            dL0 = [self._dl(self.om_s, [xi0[q]]) for q in range(3)]
            ni = g.n[j]
            self.E0[j] = _tensor3(L0[0], L0[1], L0[2])[0]
            self.E1[j] = (ni[0] * _tensor3(dL0[0], L0[1], L0[2]) + ni[1] * _tensor3(L0[0], dL0[1], L0[2])
                          + ni[2] * _tensor3(L0[0], L0[1], dL0[2]))[0] / hs

    def _translations(self):
        """1-D re-interpolation matrices S[side][a_parent, a_child] = l_{a_parent}(side/2 + om_child/2)."""
        self.Ssp = {sd: self._l(self.om_s, sd / 2.0 + self.om_s / 2.0).T for sd in (-1, 1)}
        # M2M in space: parent source box basis at the child source-box nodes, per level
        self.Msp = {lev: {sd: self._l(self.om_s, (sd * self.hs(lev) + self.hb(lev) * self.om_s)
                                       / self.hb(lev - 1)).T for sd in (-1, 1)}
                    for lev in range(2, self.D + 1)}
        self.Stm = {sd: self._l(self.om_t, sd / 2.0 + self.om_t / 2.0).T for sd in (-1, 1)}
        self._mats = {}

    def m2l_matrix(self, lev, o, gap=None, deriv=0):
        """U_{a,b,m,n}(O,S,I,J) of eq. Uabmn (gap = target minus source interval index), or the
        derivative U^{(p)} of eq. U_expand at the expansion gap mu+1.  Row a + Ps m, column b + Ps n."""
        key = (lev, o, gap, deriv)
        if key in self._mats:
            return self._mats[key]
        hs, ht, Ml = self.hs(lev), self.ht(lev), self.M[lev]
        X = hs * np.stack(np.meshgrid(self.om_s, self.om_s, self.om_s, indexing="ij"), -1).reshape(-1, 3)[:, ::-1]
        Y = 2.0 * hs * np.array(o, dtype=float) + X * (self.hb(lev) / hs)
        r = np.linalg.norm(X[:, None, :] - Y[None, :, :], axis=2)           # (Ps, Ps)
        gp = (self.mu + 1) if deriv else gap
        tdif = (gp * Ml + 1) * self.dt + ht * (self.om_t[:, None] - self.om_t[None, :])   # (pt, pt)
        arg = self.c * tdif[:, None, :, None] - r[None, :, None, :]          # (m, a, n, b)
        if deriv == 0:
            K = np.clip(arg, 0.0, None) ** self.d / r[None, :, None, :]
        else:
            if np.any(arg <= 0.0):
                raise AssertionError("expansion interval not in the distant future")
            K = comb(self.d, deriv) * arg ** (self.d - deriv) / r[None, :, None, :]
        U = K.reshape(self.P, self.P)
        if len(self._mats) * U.nbytes > 1.5e9:
            self._mats.clear()
        self._mats[key] = U
        return U

    # ---------------- march state ----------------
    def reset(self):
        D, P = self.D, self.P
        nc = {lev: len(self.cells[lev]) for lev in range(D + 1)}
        self.mom_cur = {lev: np.zeros((nc[lev], P)) for lev in range(2, D + 1)}
        self.mom_done = {lev: {} for lev in range(2, D + 1)}     # naive variant: all completed moments
        R = self.mu + 3
        self.ring = {lev: np.zeros((R, nc[lev], P)) for lev in range(2, D + 1)}
        self.Lp = {lev: np.zeros((self.d + 1, nc[lev], P)) for lev in range(2, D + 1)}
        self.aux = {lev: np.zeros((self.d + 1, max(self.d - 1, 1), nc[lev], P)) for lev in range(2, D + 1)}
        self.l2l_done = {lev: set() for lev in range(2, D + 1)}
        self.local_cache = {}
        self.n_samples = 0

    def add_sample(self, beta, tau, sigma):
        """P2M of tau^beta, sigma^beta into the leaf interval, then interval-end M2L and M2M."""
        D = self.D
        k = (beta + 1) // self.M[D]
        xi = (beta * self.dt - self.src_center(D, k)) / self.ht(D)
        lt = self._l(self.om_t, [xi])[0]
        per = self.A * tau[:, None] - self.B * sigma[:, None]            # (ns, Ps)
        cellsum = np.zeros((len(self.cells[D]), self.Ps))
        np.add.at(cellsum, self.cell_of[D], per)
        self.mom_cur[D] += self.Cd * (cellsum[:, None, :] * lt[None, :, None]).reshape(-1, self.P)
        self.n_samples = beta + 1
        for lev in range(D, 1, -1):
            Ml = self.M[lev]
            if (beta + 2) % Ml != 0:
                break
            kk = (beta + 2) // Ml - 1                 # completed source interval at this level
            Mk = self.mom_cur[lev]
            if self.m2l == "alg1":
                self._algorithm1(lev, kk, Mk)
            else:
                self.mom_done[lev][kk] = Mk.copy()
                self.local_cache = {}
            if lev > 2:
                self._m2m(lev, Mk, kk)
            self.mom_cur[lev] = np.zeros_like(Mk)

    def _reinterp(self, lev, X, half, transpose):
        """Apply the space-time re-interpolation of every cell of level lev: M2M (child -> parent
        nodes) or, transposed, L2L (parent -> child nodes).  X: (cells, P) in the cell's own layout
        (for L2L: the parent's vector gathered per child)."""
        ps, pt = self.ps, self.pt
        out = np.zeros_like(X)
        oc = self.octant[lev]
        St = self.Stm[half].T if transpose else self.Stm[half]
        for sx in (-1, 1):
            for sy in (-1, 1):
                for sz in (-1, 1):
                    sel = np.where((oc[:, 0] == sx) & (oc[:, 1] == sy) & (oc[:, 2] == sz))[0]
                    if sel.size == 0:
                        continue
                    Sp = self.Ssp if transpose else self.Msp[lev]
                    Sx, Sy, Sz = (Sp[v].T if transpose else Sp[v] for v in (sx, sy, sz))
                    T = X[sel].reshape(-1, pt, ps, ps, ps)          # (cell, n, b3, b2, b1)
                    T = np.einsum("ab,cnzyb->cnzya", Sx, T)
                    T = np.einsum("ab,cnzbx->cnzax", Sy, T)
                    T = np.einsum("ab,cnbyx->cnayx", Sz, T)
                    T = np.einsum("ab,cbzyx->cazyx", St, T)
                    out[sel] = T.reshape(sel.size, -1)
        return out

    def _m2m(self, lev, Mk, k):
        """Moments of source interval k at level lev, re-interpolated into the parents' moments of
        interval k // 2 (k even: the first half of the parent interval)."""
        half = -1 if k % 2 == 0 else 1
        np.add.at(self.mom_cur[lev - 1], self.parent[lev], self._reinterp(lev, Mk, half, False))

    def _algorithm1(self, lev, k, Mk):
        """Algorithm 1 for source interval k at one level (all target cells)."""
        mu, d, R = self.mu, self.d, self.mu + 3
        ring, Lp, aux = self.ring[lev], self.Lp[lev], self.aux[lev]
        nc = len(self.cells[lev])
        Dp = np.zeros((d + 1, nc, self.P))
        for o, (oi, si) in self.il_by_off[lev].items():
            X = Mk[si]
            for l in range(1, mu + 2):
                np.add.at(ring[(k + l) % R], oi, self._near_prod(X, self.m2l_matrix(lev, o, gap=l)))
            for p in range(1, d + 1):
                np.add.at(Dp[p], oi, X @ self.m2l_matrix(lev, o, deriv=p).T)
        T = self.c * self.M[lev] * self.dt
        recurrence(k, mu, d, T, ring, R, Lp, aux, Dp)

    def _near_prod(self, X, U):
        """A near-future product X @ U.T, formed by near_product or from factors rounded by
        near_round where the block is truncated at some node pairs and not zero at all of them."""
        if (U == 0).any() and (U > 0).any():
            if self.near_product is not None:
                return self.near_product(X, U)
            if self.near_round is not None:
                return self.near_round(X) @ self.near_round(U).T
        return X @ U.T

    def _l2l_apply(self, lev_parent, Lpar, k_par):
        """The parent's local of target interval k_par, re-interpolated onto the child level's
        two intervals 2 k_par and 2 k_par + 1: {child interval: (cells, P)}."""
        lev = lev_parent + 1
        G = Lpar[self.parent[lev]]
        return {2 * k_par + (0 if half < 0 else 1): self._reinterp(lev, G, half, True) for half in (-1, 1)}

    def begin_target(self, alpha):
        """Algorithm-1 variant: L2L, top-down, for every level-l target interval that starts at alpha."""
        if self.m2l != "alg1":
            return
        R = self.mu + 3
        for lev in range(2, self.D):
            Ml = self.M[lev]
            if alpha % Ml != 0:
                continue
            kp = alpha // Ml
            for kc, acc in self._l2l_apply(lev, self.ring[lev][kp % R], kp).items():
                self.ring[lev + 1][kc % R] += acc

    def local(self, lev, k):
        """Naive variant: complete local of target interval k (eq. m2l_actual plus L2L from the parent)."""
        key = (lev, k)
        if key in self.local_cache:
            return self.local_cache[key]
        L = np.zeros((len(self.cells[lev]), self.P))
        for kk, Mk in self.mom_done[lev].items():
            if kk >= k:
                continue
            for o, (oi, si) in self.il_by_off[lev].items():
                np.add.at(L, oi, self._near_prod(Mk[si], self.m2l_matrix(lev, o, gap=k - kk)))
        if lev > 2:
            kp = k // 2
            L += self._l2l_apply(lev - 1, self.local(lev - 1, kp), kp)[k]
        self.local_cache[key] = L
        return L

    def far(self, alpha):
        """Far-field part at (x_i, t_alpha): the local field (OBIE) or (d/dn - (1/c) d/dt) of it (BMBIE)."""
        D = self.D
        k = alpha // self.M[D]
        if self.m2l == "alg1":
            L = self.ring[D][k % (self.mu + 3)]
        else:
            L = self.local(D, k)
        tau = (alpha * self.dt - self.tgt_center(D, k)) / self.ht(D)
        lt = self._l(self.om_t, [tau])[0]
        dlt = self._dl(self.om_t, [tau])[0] / self.ht(D)
        Lc = L[self.cell_of[D]].reshape(self.geom.ns, self.pt, self.Ps)   # (i, m, a)
        if self.bie == 0:
            return np.einsum("ima,ia,m->i", Lc, self.E0, lt)
        return np.einsum("ima,ia,m->i", Lc, self.E1, lt) - np.einsum("ima,ia,m->i", Lc, self.E0, dlt) / self.c

    def near(self, alpha, u, q):
        b = np.zeros(self.geom.ns)
        for g in range(2, min(self.gmax, alpha) + 1):
            b += self.CU[g] @ q[alpha - g] - self.CW[g] @ u[alpha - g]
        return b

    def densities(self, beta, u, q):
        """tau^beta, sigma^beta (eqs. tau, sigma without history truncation)."""
        tau = np.zeros(self.geom.ns)
        sig = np.zeros(self.geom.ns)
        for k in range(0, min(self.d + 1, beta) + 1):
            tau += self.w[k] * q[beta - k]
            sig += self.w[k] * u[beta - k]
        return tau, sig

    def history_rhs(self, alpha, u, q):
        """Near + far history part of b^{alpha-1} for a given coefficient history (rows beta)."""
        self.reset()
        for beta in range(0, alpha - 1):
            self.begin_target(beta + 1)
            tau, sig = self.densities(beta, u, q)
            self.add_sample(beta, tau, sig)
        self.begin_target(alpha)
        return self.near(alpha, u, q) + self.far(alpha)

    def run(self, nt, forcing=None):
        """MOT march with near pairs direct and far pairs by this FMM (homogeneous condition
        of the oracle's direct MOT: Neumann -> u unknown, Dirichlet -> q unknown).  The per-step
        matrix only involves pairs closer than c dt, all of which are near pairs."""
        import scipy.linalg as sla
        from .mot import NEUMANN
        if self.bc is None:
            raise ValueError("construct with bc= to march")
        A = (self.CW[1] if self.bc == NEUMANN else -self.CU[1]).toarray()
        lu = sla.lu_factor(A)
        ns = self.geom.ns
        u = np.zeros((nt - 1, ns))
        q = np.zeros((nt - 1, ns))
        self.reset()
        for alpha in range(1, nt):
            beta = alpha - 1
            self.begin_target(alpha)
            b = self.near(alpha, u, q) + self.far(alpha)
            if forcing is not None:
                b = b + forcing[beta]
            x = sla.lu_solve(lu, b)
            if self.bc == NEUMANN:
                u[beta] = x
            else:
                q[beta] = x
            tau, sig = self.densities(beta, u, q)
            self.add_sample(beta, tau, sig)
        return u, q
