/*
 * ORACLE — test infrastructure only.  Nothing in the product library links,
 * loads or calls this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.
 *
 * Closed-form space integrals of the retarded kernels over one flat triangle,
 * in plain FP64 C, written from the paper's Appendix B (evaluation of the
 * spatial integrals in U_ij and W_ij) and from the definitions of the
 * discretised single/double layer (Section 2.4, eqs. discretised_single_layer_
 * potential and discretised_double_layer_potential) and of the Burton-Miller
 * matrices (eq. U_W_BM).
 *
 * Notation.  For a target point x, a triangle E with unit normal n (the paper's
 * normal, used as local z axis), and s = c*t_gamma:
 *   Phi(x,s) = int_E (s-r)_+^d / r dS_y,        r = |x-y|
 * The four coefficient families of a (collocation point i, element j, s) triple:
 *   U    =  C Phi                                (single layer)
 *   W    = -C dPhi/dz                            (double layer, n_y.grad_y)
 *   Ubar =  C ( n_i.grad_x Phi - dPhi/ds )       (BM operator on U)
 *   Wbar = -C ( n_i.grad_x dPhi/dz - d2Phi/dsdz )(BM operator on W)
 * with C = 1/(4 pi (c dt)^d), dz the derivative along n at fixed foot point,
 * and -(1/c) d/dt = -d/ds because s = c (t - t_beta).
 *
 * Phi in polar coordinates about the foot O of x on the plane (App. B):
 *   Phi = Theta (s-|z|)_+^{d+1}/(d+1) + sum_edges I^d_n
 * where Theta is the signed angle the triangle subtends at O (2 pi inside,
 * 0 outside) and I^d_n is the paper's closed-form bracket, evaluated with the
 * local y coordinate of the edge, between the edge end points clipped to the
 * wavefront r <= s.  The in-plane part of grad_x uses the tangential
 * divergence theorem on the flat face:  grad_par Phi = - oint (s-r)_+^d/r nu dl.
 * Derivatives in z and s of the polar and edge parts are differentiated in
 * closed form; endpoint motion of the clip does not contribute because every
 * differentiated integrand vanishes at r = s.
 *
 * Side convention (x_i on the side the paper normal points to, so that the
 * free term is absorbed into the double layer): the self pair is evaluated in
 * the limit z -> 0+.
 */
#include <math.h>
#include <string.h>

#define ORACLE_PI 3.14159265358979323846

static double dot3(const double *a, const double *b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static void sub3(const double *a, const double *b, double *o) { o[0]=a[0]-b[0]; o[1]=a[1]-b[1]; o[2]=a[2]-b[2]; }
static void cross3(const double *a, const double *b, double *o) {
  o[0] = a[1]*b[2] - a[2]*b[1]; o[1] = a[2]*b[0] - a[0]*b[2]; o[2] = a[0]*b[1] - a[1]*b[0];
}
static double pospow(double v, int k) { if (v <= 0.0) return 0.0; double r = 1.0; for (int i = 0; i < k; ++i) r *= v; return r; }

/* Paper's bracket I^d_n at coordinate x of the edge (local y = yl, height z),
 * for d = 1, 2, 3 (App. B), with R := sqrt(y^2+z^2) in log((x+r)/R) so that
 * log((x+r)/R) = asinh(x/R). */
static double paper_bracket(int d, double x, double yl, double z, double s) {
  double r = sqrt(x*x + yl*yl + z*z);
  double rho = sqrt(yl*yl + z*z);
  double at = atan(x / yl);
  double ax = atan(x * z / (yl * r));
  double lg = asinh(x / rho);
  if (d == 1)
    return x*yl/2.0 + (s*s + z*z)/2.0*at - s*z*ax - s*yl*lg;
  if (d == 2)
    return (2.0*(s*s*s + 3.0*s*z*z)*at - 2.0*z*(3.0*s*s + z*z)*ax
            - x*yl*(-6.0*s + r) - yl*(6.0*s*s + yl*yl + 3.0*z*z)*lg) / 6.0;
  /* d == 3 */
  return (x*yl*(18.0*s*s + x*x + 3.0*yl*yl + 6.0*z*z - 6.0*s*r)
          + 3.0*(s*s*s*s + 6.0*s*s*z*z + z*z*z*z)*at
          - 12.0*s*z*(s*s + z*z)*ax
          - 6.0*yl*s*(2.0*s*s + yl*yl + 3.0*z*z)*lg) / 12.0;
}

/* Antiderivatives in x of the derivative integrands (d = 1, 2), with h the
 * signed in-plane distance of O to the edge line (h > 0 when O is on the
 * inner side), rho^2 = h^2 + z^2, R = sqrt(x^2 + rho^2), and the polar weight
 * dtheta = h dx / (x^2 + h^2).  Each was obtained by expanding (s-R)^d in
 * powers of R and integrating term by term:
 *   Pz  = int d/dz[-(s-R)^{d+1}/(d+1)] dtheta
 *   Pzz = int d2/dz2[...] dtheta,  Ps = int d/ds[...] dtheta,  Psz = d/ds Pz
 *   L0  = int (s-R)^d / R dx,      Lz = int d/dz[(s-R)^d/R] dx                */
typedef struct { double Pz, Pzz, Ps, Psz, L0, Lz; } edge_terms;

static void edge_antideriv(int d, double x, double h, double z, double s, edge_terms *o) {
  double rho2 = h*h + z*z;
  double R = sqrt(x*x + rho2);
  double at = atan(x / h);
  double ax = atan(x * z / (h * R));
  double ash = asinh(x / sqrt(rho2));
  double x_r3 = x / (rho2 * R); /* int dx / R^3 */
  if (d == 1) {
    o->Pz  = s*ax - z*at;
    o->Pzz = s*h*x_r3 - at;
    o->Ps  = -s*at + (h*ash + z*ax);
    o->Psz = ax;
    o->L0  = s*ash - x;
    o->Lz  = -z*s*x_r3;
  } else {
    o->Pz  = (s*s + z*z)*ax - 2.0*s*z*at + z*h*ash;
    o->Pzz = s*s*h*x_r3 - 2.0*s*at + h*ash + 2.0*z*ax;
    o->Ps  = -(s*s*at - 2.0*s*(h*ash + z*ax) + (h*x + z*z*at));
    o->Psz = 2.0*s*ax - 2.0*z*at;
    o->L0  = s*s*ash - 2.0*s*x + (x*R + rho2*ash)/2.0;
    o->Lz  = -z*(s*s*x_r3 - ash);
  }
}

/* Raw face quantities:
 *  out[0] Phi, out[1] dPhi/dz, out[2] d2Phi/dz2, out[3] dPhi/ds, out[4] d2Phi/dsdz,
 *  out[5] t.grad_par Phi, out[6] d/dz (t.grad_par Phi)
 * for target x, triangle V (3x3 row-major), unit normal n, in-plane vector t.
 * Derivative outputs (1..6) are only produced for d = 1, 2; Phi for d = 1..3. */
void oracle_face_terms(const double *x, const double *V, const double *n, const double *t,
                       double s, int d, int self, double *out) {
  memset(out, 0, 7 * sizeof(double));
  double e1[3], e2[3], cr[3];
  sub3(V + 3, V, e1); sub3(V + 6, V, e2); cross3(e1, e2, cr);
  int order[3] = {0, 1, 2};
  if (dot3(cr, n) < 0.0) { order[1] = 2; order[2] = 1; } /* counter-clockwise about n */
  double xa[3];
  sub3(x, V, xa);
  double z = self ? 0.0 : dot3(xa, n);
  double O[3] = {x[0] - z*n[0], x[1] - z*n[1], x[2] - z*n[2]};
  double sgnz = (z >= 0.0) ? 1.0 : -1.0;
  double az = fabs(z);
  double theta = 0.0;
  double scale = sqrt(dot3(e1, e1));
  for (int k = 0; k < 3; ++k) {
    const double *A = V + 3 * order[k];
    const double *B = V + 3 * order[(k + 1) % 3];
    double ab[3], e[3], nu[3], ao[3], bo[3];
    sub3(B, A, ab);
    double len = sqrt(dot3(ab, ab));
    e[0] = ab[0]/len; e[1] = ab[1]/len; e[2] = ab[2]/len;
    cross3(e, n, nu);                  /* outward in-plane edge normal */
    sub3(A, O, ao); sub3(B, O, bo);
    double h = dot3(ao, nu);           /* signed distance of O to the edge line */
    double x1 = dot3(ao, e), x2 = dot3(bo, e);
    double yl = -h;                    /* paper's local y = (A-O).(n x e) */
    double rho2 = h*h + z*z;
    int polar = fabs(h) > 1e-12 * scale;
    if (polar) theta += atan(x2 / h) - atan(x1 / h);
    if (s*s <= rho2) continue;         /* wavefront does not reach this edge line */
    double X = sqrt(s*s - rho2);
    double lo = x1 > -X ? x1 : -X, hi = x2 < X ? x2 : X;
    if (lo >= hi) continue;
    if (polar) out[0] += paper_bracket(d, hi, yl, z, s) - paper_bracket(d, lo, yl, z, s);
    if (d <= 2) {
      edge_terms a, b;
      edge_antideriv(d, hi, h, z, s, &b);
      edge_antideriv(d, lo, h, z, s, &a);
      double tn = dot3(t, nu);
      if (polar) {
        out[1] += b.Pz - a.Pz;
        out[2] += b.Pzz - a.Pzz;
        out[3] += b.Ps - a.Ps;
        out[4] += b.Psz - a.Psz;
      }
      out[5] += -tn * (b.L0 - a.L0);
      out[6] += -tn * (b.Lz - a.Lz);
    }
  }
  /* I_0: the part of the polar integral at the foot point */
  out[0] += theta * pospow(s - az, d + 1) / (d + 1);
  if (d <= 2) {
    out[1] += -theta * sgnz * pospow(s - az, d);
    out[2] += theta * d * pospow(s - az, d - 1);
    out[3] += theta * pospow(s - az, d);
    out[4] += -theta * sgnz * d * pospow(s - az, d - 1);
  }
}

/* The four coefficient families {U, W, Ubar, Wbar} at s for collocation point x
 * with paper normal ni, element V with paper normal nj.  cdt = c*dt. */
void oracle_elem(const double *x, const double *ni, const double *V, const double *nj,
                 int self, double s, int d, double cdt, double *out) {
  double nn = dot3(ni, nj);
  double t[3] = {ni[0] - nn*nj[0], ni[1] - nn*nj[1], ni[2] - nn*nj[2]};
  double f[7];
  oracle_face_terms(x, V, nj, t, s, d, self, f);
  double C = 1.0 / (4.0 * ORACLE_PI * pow(cdt, d));
  out[0] = C * f[0];
  out[1] = -C * f[1];
  out[2] = C * (nn * f[1] + f[5] - f[3]);
  out[3] = -C * (nn * f[2] + f[6] - f[4]);
}

/* Distance range [rmin, rmax] from point x to triangle V. */
void oracle_dist_range(const double *x, const double *V, double *rmin, double *rmax) {
  double mx = 0.0;
  for (int k = 0; k < 3; ++k) {
    double d[3]; sub3(x, V + 3*k, d);
    double r = sqrt(dot3(d, d)); if (r > mx) mx = r;
  }
  *rmax = mx;
  /* closest point: inside-projection test, else the nearest point on the edges */
  double e1[3], e2[3], n[3], xa[3];
  sub3(V + 3, V, e1); sub3(V + 6, V, e2); cross3(e1, e2, n);
  double nl = sqrt(dot3(n, n)); n[0] /= nl; n[1] /= nl; n[2] /= nl;
  sub3(x, V, xa);
  double z = dot3(xa, n);
  double p[3] = {x[0] - z*n[0], x[1] - z*n[1], x[2] - z*n[2]};
  int inside = 1;
  for (int k = 0; k < 3; ++k) {
    const double *A = V + 3*k, *B = V + 3*((k+1)%3);
    double ab[3], ap[3], c[3];
    sub3(B, A, ab); sub3(p, A, ap); cross3(ab, ap, c);
    if (dot3(c, n) < 0.0) inside = 0;
  }
  if (inside) { *rmin = fabs(z); return; }
  double best = 1e300;
  for (int k = 0; k < 3; ++k) {
    const double *A = V + 3*k, *B = V + 3*((k+1)%3);
    double ab[3], ax[3];
    sub3(B, A, ab); sub3(x, A, ax);
    double u = dot3(ax, ab) / dot3(ab, ab);
    if (u < 0.0) u = 0.0; if (u > 1.0) u = 1.0;
    double q[3] = {A[0] + u*ab[0] - x[0], A[1] + u*ab[1] - x[1], A[2] + u*ab[2] - x[2]};
    double r = sqrt(dot3(q, q)); if (r < best) best = r;
  }
  *rmin = best;
}

/* B-spline weight w^{kappa,d} = (d+1) / prod_{k != kappa} (k - kappa)  (eq. w). */
static double bspline_w(int kappa, int d) {
  double p = 1.0;
  for (int k = 0; k <= d + 1; ++k) if (k != kappa) p *= (double)(k - kappa);
  return (double)(d + 1) / p;
}

/* Time-difference window of the compact coefficient of pair (i, j):
 * C^{(g)} = sum_kappa w^kappa X^{(g-kappa)} can be non-zero only for
 * rmin/(c dt) < g < rmax/(c dt) + d + 1 (support of the B-spline, Remark
 * support, applied inside the integral as in the derivation of beta*). */
static void window_of(double rmin, double rmax, int d, double cdt, int *glo, int *ghi) {
  int lo = (int)floor(rmin / cdt) + 1;
  int hi = (int)ceil(rmax / cdt + d + 1) - 1;
  if (lo < 1) lo = 1;
  *glo = lo; *ghi = hi;
}

/* Pass 1: window start and length per (row, j), row-major r*ns+j, for the
 * collocation rows rows[0..nrows-1] (rows == NULL: all ns rows).
 * xc: collocation points (ns x 3), tris: vertex coordinates (ns x 9). */
void oracle_windows_rows(int ns, int nrows, const int *rows, const double *xc, const double *tris, int d,
                         double cdt, int *glo, int *cnt) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int r = 0; r < nrows; ++r) {
    int i = rows ? rows[r] : r;
    for (int j = 0; j < ns; ++j) {
      double rmin, rmax;
      if (i == j) { double a; oracle_dist_range(xc + 3*i, tris + 9*j, &a, &rmax); rmin = 0.0; }
      else oracle_dist_range(xc + 3*i, tris + 9*j, &rmin, &rmax);
      int lo, hi; window_of(rmin, rmax, d, cdt, &lo, &hi);
      glo[(long)r*ns + j] = lo; cnt[(long)r*ns + j] = hi - lo + 1;
    }
  }
}

void oracle_windows(int ns, const double *xc, const double *tris, int d, double cdt, int *glo, int *cnt) {
  oracle_windows_rows(ns, ns, 0, xc, tris, d, cdt, glo, cnt);
}

/* Pass 2: compact coefficients for every (row, j) and g in its window.
 * out has 4 families interleaved per slot: out[4*(off[r*ns+j] + k) + f],
 * f = 0 U, 1 W, 2 Ubar, 3 Wbar;  g = glo + k.  nrm: paper normals (ns x 3). */
void oracle_fill_rows(int ns, int nrows, const int *rows, const double *xc, const double *nrm, const double *tris,
                      int d, double cdt, const int *glo, const int *cnt, const long *off, double *out) {
  double w[8];
  for (int k = 0; k <= d + 1; ++k) w[k] = bspline_w(k, d);
#pragma omp parallel for schedule(dynamic, 8)
  for (int r = 0; r < nrows; ++r) {
    int i = rows ? rows[r] : r;
    for (int j = 0; j < ns; ++j) {
      long p = (long)r*ns + j;
      int lo = glo[p], n = cnt[p];
      double X[64][4];
      int gmin = lo - d - 1; if (gmin < 1) gmin = 1;
      int gmax = lo + n - 1;
      if (gmax - gmin + 1 > 64) continue; /* caller rejects such windows */
      for (int g = gmin; g <= gmax; ++g)
        oracle_elem(xc + 3*i, nrm + 3*i, tris + 9*j, nrm + 3*j, i == j, g * cdt, d, cdt, X[g - gmin]);
      for (int k = 0; k < n; ++k) {
        int g = lo + k;
        double acc[4] = {0, 0, 0, 0};
        for (int kap = 0; kap <= d + 1; ++kap) {
          int gg = g - kap;
          if (gg < gmin) continue; /* below the window every term is zero (gg < 1 or no overlap) */
          for (int f = 0; f < 4; ++f) acc[f] += w[kap] * X[gg - gmin][f];
        }
        for (int f = 0; f < 4; ++f) out[4*(off[p] + k) + f] = acc[f];
      }
    }
  }
}

void oracle_fill(int ns, const double *xc, const double *nrm, const double *tris, int d, double cdt,
                 const int *glo, const int *cnt, const long *off, double *out) {
  oracle_fill_rows(ns, ns, 0, xc, nrm, tris, d, cdt, glo, cnt, off, out);
}

/* Off-surface points: windows and compact coefficients of every (point, element)
 * pair, as oracle_windows_rows / oracle_fill_rows with the collocation point
 * replaced by pts[r] (never a self pair).  Only the U and W families are
 * meaningful there (the point has no normal; ni is taken as nj). */
void oracle_windows_points(int ns, int npts, const double *pts, const double *tris, int d, double cdt,
                           int *glo, int *cnt) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int r = 0; r < npts; ++r)
    for (int j = 0; j < ns; ++j) {
      double rmin, rmax;
      oracle_dist_range(pts + 3*r, tris + 9*j, &rmin, &rmax);
      int lo, hi; window_of(rmin, rmax, d, cdt, &lo, &hi);
      glo[(long)r*ns + j] = lo; cnt[(long)r*ns + j] = hi - lo + 1;
    }
}

void oracle_fill_points(int ns, int npts, const double *pts, const double *nrm, const double *tris, int d,
                        double cdt, const int *glo, const int *cnt, const long *off, double *out) {
  double w[8];
  for (int k = 0; k <= d + 1; ++k) w[k] = bspline_w(k, d);
#pragma omp parallel for schedule(dynamic, 8)
  for (int r = 0; r < npts; ++r)
    for (int j = 0; j < ns; ++j) {
      long p = (long)r*ns + j;
      int lo = glo[p], n = cnt[p];
      double X[64][4];
      int gmin = lo - d - 1; if (gmin < 1) gmin = 1;
      int gmax = lo + n - 1;
      if (gmax - gmin + 1 > 64) continue;
      for (int g = gmin; g <= gmax; ++g)
        oracle_elem(pts + 3*r, nrm + 3*j, tris + 9*j, nrm + 3*j, 0, g * cdt, d, cdt, X[g - gmin]);
      for (int k = 0; k < n; ++k) {
        int g = lo + k;
        double acc[2] = {0, 0};
        for (int kap = 0; kap <= d + 1; ++kap) {
          int gg = g - kap;
          if (gg < gmin) continue;
          acc[0] += w[kap] * X[gg - gmin][0];
          acc[1] += w[kap] * X[gg - gmin][1];
        }
        out[2*(off[p] + k)] = acc[0];
        out[2*(off[p] + k) + 1] = acc[1];
      }
    }
}
