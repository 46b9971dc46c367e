// Element integrals of the retarded kernels over one flat triangle, by
// Gauss-Legendre quadrature (FP64), for the near-field coefficient tables.
//
// For a target x, a triangle E with unit normal n (local z axis), and
// s = c t_gamma, let Phi(x,s) = int_E (s-r)_+^d / r dS_y.  The library needs
//   U = C Phi,  W = -C dPhi/dz,  Ubar = C (n_i.grad Phi - dPhi/ds),
//   Wbar = -C (n_i.grad dPhi/dz - d2Phi/dsdz),       C = 1/(4 pi (c dt)^d)
// (single and double layer of the discretised BIE, Section 2.4, and their
// Burton-Miller versions, eq. U_W_BM; -(1/c) d/dt = -d/ds).
//
// Route: polar coordinates about the foot O of x (App. B).  The radial
// integral is done in closed form, int_0^{rho_E} g(r) rho drho = G(R_E) - G(|z|)
// with G' = r g, leaving (i) a foot term proportional to the angle the face
// subtends at O and (ii) one smooth angular integral per edge, which is
// integrated here with composite Gauss-Legendre rules after the substitution
// x = |h| sinh(u) along the edge (h: distance of O to the edge line).  The in-plane gradient uses the tangential
// divergence theorem, grad_par Phi = -oint (s-r)_+^d / r nu dl, integrated
// along each edge in u with x = rho sinh u (so dx / r = du).  Each edge is
// clipped to the wavefront r <= s first, so every integrand is a smooth
// polynomial in r on its interval.  The self pair is the limit z -> 0+ on the
// side n points to.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace tdbem {

// 16-point Gauss-Legendre rule on [-1,1], filled on the host at library load
// (Newton iteration on P_16) and copied to device constant memory.
struct GLRule { double x[16]; double w[16]; };

__host__ __device__ inline double dot3(const double* a, const double* b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
__host__ __device__ inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1]*b[2] - a[2]*b[1]; o[1] = a[2]*b[0] - a[0]*b[2]; o[2] = a[0]*b[1] - a[1]*b[0];
}
__host__ __device__ inline double ipow(double v, int k) { double r = 1.0; for (int i = 0; i < k; ++i) r *= v; return r; }

// Raw quantities: f[0] Phi, f[1] dPhi/dz, f[2] d2Phi/dz2, f[3] dPhi/ds,
// f[4] d2Phi/dsdz, f[5] t.grad_par Phi, f[6] d/dz (t.grad_par Phi).
__host__ __device__ inline void face_terms_gl(const GLRule& gl, const double* x, const double* V,
                                              const double* n, const double* t, double s, int d,
                                              bool self, double* f) {
  for (int k = 0; k < 7; ++k) f[k] = 0.0;
  double e1[3] = {V[3]-V[0], V[4]-V[1], V[5]-V[2]};
  double e2[3] = {V[6]-V[0], V[7]-V[1], V[8]-V[2]};
  double cr[3];
  cross3(e1, e2, cr);
  int ord1 = 1, ord2 = 2;
  if (dot3(cr, n) < 0.0) { ord1 = 2; ord2 = 1; }   // walk the edges counter-clockwise about n
  const double* P[3] = {V, V + 3*ord1, V + 3*ord2};
  double z = self ? 0.0 : ((x[0]-V[0])*n[0] + (x[1]-V[1])*n[1] + (x[2]-V[2])*n[2]);
  double O[3] = {x[0]-z*n[0], x[1]-z*n[1], x[2]-z*n[2]};
  double az = fabs(z), sz = z >= 0.0 ? 1.0 : -1.0;
  double lref = sqrt(dot3(e1, e1));
  double theta = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double* A = P[k];
    const double* B = P[(k + 1) % 3];
    double a[3] = {A[0]-O[0], A[1]-O[1], A[2]-O[2]};
    double b[3] = {B[0]-O[0], B[1]-O[1], B[2]-O[2]};
    double ab[3];
    cross3(a, b, ab);
    theta += atan2(dot3(ab, n), dot3(a, b));              // signed angle subtended at O
    double e[3] = {B[0]-A[0], B[1]-A[1], B[2]-A[2]};
    double len = sqrt(dot3(e, e));
    e[0] /= len; e[1] /= len; e[2] /= len;
    double nu[3];
    cross3(e, n, nu);                                      // outward in-plane normal of the edge
    double h = dot3(a, nu);
    double xa = dot3(a, e), xb = xa + len;
    double rho2 = h*h + z*z;
    if (s*s <= rho2) continue;
    double X = sqrt(s*s - rho2);
    double lo = xa > -X ? xa : -X, hi = xb < X ? xb : X;
    if (lo >= hi) continue;
    // (ii) angular integrals.  dtheta = h dx / (x^2 + h^2); with x = |h| sinh(u)
    // this is sign(h) sech(u) du, analytic in the strip |Im u| < pi/2 whatever
    // the ratio of the edge length to |h|, so composite panels of width <= 0.75
    // converge geometrically.
    if (fabs(h) > 1e-12 * lref) {
      double ah = fabs(h), sh = h > 0.0 ? 1.0 : -1.0;
      double u0 = asinh(lo / ah), u1 = asinh(hi / ah);
      int np = (int)ceil((u1 - u0) / 0.75); if (np < 1) np = 1;
      double hw = (u1 - u0) / (2.0 * np);
      double acc[5] = {0, 0, 0, 0, 0};
      for (int p = 0; p < np; ++p) {
        double mid = u0 + (2*p + 1) * hw;
        for (int q = 0; q < 16; ++q) {
          double u = mid + hw * gl.x[q];
          double ch = cosh(u);
          double R2 = h*h * ch*ch + z*z;
          double R = sqrt(R2);
          double sr = s - R; if (sr < 0.0) sr = 0.0;
          double srd = ipow(sr, d), srd1 = ipow(sr, d - 1);
          double w = sh * gl.w[q] * hw / ch;
          acc[0] += w * (-srd * sr / (d + 1));
          acc[1] += w * (srd * z / R);
          acc[2] += w * (srd / R - d * srd1 * z*z / R2 - srd * z*z / (R2 * R));
          acc[3] += w * (-srd);
          acc[4] += w * (d * srd1 * z / R);
        }
      }
      for (int m = 0; m < 5; ++m) f[m] += acc[m];
    }
    // line integrals along the edge, x = rho sinh(u)
    double tn = dot3(t, nu);
    if (tn != 0.0) {
      double rho = sqrt(rho2);
      double u0 = asinh(lo / rho), u1 = asinh(hi / rho);
      int np = (int)ceil((u1 - u0) / 0.75); if (np < 1) np = 1;
      double hw = (u1 - u0) / (2.0 * np);
      double a0 = 0.0, a1 = 0.0;
      for (int p = 0; p < np; ++p) {
        double mid = u0 + (2*p + 1) * hw;
        for (int q = 0; q < 16; ++q) {
          double u = mid + hw * gl.x[q];
          double R = rho * cosh(u);
          double sr = s - R; if (sr < 0.0) sr = 0.0;
          double srd = ipow(sr, d), srd1 = ipow(sr, d - 1);
          double w = gl.w[q] * hw;
          a0 += w * srd;
          a1 += w * (-z * (d * srd1 / R + srd / (R*R)));
        }
      }
      f[5] += -tn * a0;
      f[6] += -tn * a1;
    }
  }
  // (i) foot terms: G(|z|) part of the radial integral times the subtended angle
  double sa = s - az; if (sa < 0.0) sa = 0.0;
  f[0] += theta * ipow(sa, d + 1) / (d + 1);
  f[1] += -theta * sz * ipow(sa, d);
  f[2] += theta * d * ipow(sa, d - 1) * (s > az ? 1.0 : 0.0);
  f[3] += theta * ipow(sa, d);
  f[4] += -theta * sz * d * ipow(sa, d - 1) * (s > az ? 1.0 : 0.0);
}

// {U, W, Ubar, Wbar} for collocation point x with normal ni, face V with normal nj.
__host__ __device__ inline void elem_families_gl(const GLRule& gl, const double* x, const double* ni,
                                                 const double* V, const double* nj, bool self,
                                                 double s, int d, double Cd, double* out) {
  double nn = dot3(ni, nj);
  double t[3] = {ni[0] - nn*nj[0], ni[1] - nn*nj[1], ni[2] - nn*nj[2]};
  double f[7];
  face_terms_gl(gl, x, V, nj, t, s, d, self, f);
  out[0] = Cd * f[0];
  out[1] = -Cd * f[1];
  out[2] = Cd * (nn * f[1] + f[5] - f[3]);
  out[3] = -Cd * (nn * f[2] + f[6] - f[4]);
}

// Closest and farthest distance from x to triangle V (vertices row-major):
// closest point by barycentric region classification.
__host__ __device__ inline void tri_dist_range(const double* x, const double* V, double* rmin, double* rmax) {
  const double* A = V; const double* B = V + 3; const double* C = V + 6;
  double mx = 0.0;
  for (int k = 0; k < 3; ++k) {
    double dv[3] = {x[0]-V[3*k], x[1]-V[3*k+1], x[2]-V[3*k+2]};
    double r = sqrt(dot3(dv, dv)); if (r > mx) mx = r;
  }
  *rmax = mx;
  double ab[3] = {B[0]-A[0], B[1]-A[1], B[2]-A[2]};
  double ac[3] = {C[0]-A[0], C[1]-A[1], C[2]-A[2]};
  double ap[3] = {x[0]-A[0], x[1]-A[1], x[2]-A[2]};
  double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  double q[3];
  if (d1 <= 0.0 && d2 <= 0.0) { q[0]=A[0]; q[1]=A[1]; q[2]=A[2]; }
  else {
    double bp[3] = {x[0]-B[0], x[1]-B[1], x[2]-B[2]};
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    double cp[3] = {x[0]-C[0], x[1]-C[1], x[2]-C[2]};
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    double vc = d1*d4 - d3*d2, vb = d5*d2 - d1*d6, va = d3*d6 - d5*d4;
    if (d3 >= 0.0 && d4 <= d3) { q[0]=B[0]; q[1]=B[1]; q[2]=B[2]; }
    else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
      double v = d1 / (d1 - d3);
      for (int k = 0; k < 3; ++k) q[k] = A[k] + v*ab[k];
    } else if (d6 >= 0.0 && d5 <= d6) { q[0]=C[0]; q[1]=C[1]; q[2]=C[2]; }
    else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
      double w = d2 / (d2 - d6);
      for (int k = 0; k < 3; ++k) q[k] = A[k] + w*ac[k];
    } else if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
      double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
      for (int k = 0; k < 3; ++k) q[k] = B[k] + w*(C[k]-B[k]);
    } else {
      double den = 1.0 / (va + vb + vc);
      double v = vb * den, w = vc * den;
      for (int k = 0; k < 3; ++k) q[k] = A[k] + ab[k]*v + ac[k]*w;
    }
  }
  double dq[3] = {x[0]-q[0], x[1]-q[1], x[2]-q[2]};
  *rmin = sqrt(dot3(dq, dq));
}

// Window of time differences g with a possibly non-zero compact coefficient:
// rmin/(c dt) < g < rmax/(c dt) + d + 1 (support of N^{beta,d}, Remark support).
__host__ __device__ inline void time_window(double rmin, double rmax, int d, double cdt, int* glo, int* cnt) {
  int lo = (int)floor(rmin / cdt) + 1;
  int hi = (int)ceil(rmax / cdt + d + 1) - 1;
  if (lo < 1) lo = 1;
  *glo = lo;
  *cnt = hi - lo + 1;
}

}  // namespace tdbem
