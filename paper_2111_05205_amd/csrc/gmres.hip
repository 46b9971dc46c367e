// Per-step solve A x = b (eq. linear) by restarted GMRES in FP64.
//
// A is sparse (non-zero only for pairs within c*dt of each other) and
// constant in time; its spectrum is tightly clustered, so GMRES converges in
// about a dozen iterations.  The whole solve runs in ONE workgroup of 1024
// threads (16 wavefronts) per step: the Krylov basis lives in global memory
// (L2-resident for the sizes this kernel serves), the Hessenberg matrix,
// Givens rotations and reduction scratch in LDS, and no host round trip is
// needed.  Orthogonalisation is classical Gram-Schmidt, applied a second time
// only when the first pass removes more than 99% of |W|^2.  The products
// A v read a copy of A padded to the longest row and stored column-major, so
// the loads of a row are independent and consecutive rows are adjacent.
//
// Larger systems use the cooperative variant: NW workgroups of 256 threads,
// guaranteed co-resident by a cooperative launch, each owning a contiguous
// slice of rows.  Every reduction goes through per-workgroup partial sums in
// global memory and a grid barrier (the barrier orders memory at device scope);
// every workgroup then sums the partials in the same order, so the Hessenberg
// matrix, Givens rotations and stopping decision are bitwise identical in all
// workgroups.  Each orthogonalisation pass also carries |W|^2, and a second
// pass runs only when the first removes more than 99% of |W|^2, so an Arnoldi
// step usually takes 2 barriers.
#include "internal.h"

#include <hip/hip_cooperative_groups.h>

#include <algorithm>

namespace tdbem {

constexpr int GM_THREADS = 1024;
constexpr int GM_WAVES = GM_THREADS / 64;
constexpr int GM_MAXM = 32;

struct GmresShared {
  double H[GM_MAXM + 1][GM_MAXM];
  double cs[GM_MAXM], sn[GM_MAXM], g[GM_MAXM + 1], y[GM_MAXM];
  double red[GM_WAVES][GM_MAXM + 1];
  double hv[GM_MAXM + 1];
  double scal[4];
};

__device__ inline double wave_sum(double v) {
  for (int s = 32; s > 0; s >>= 1) v += __shfl_down(v, s, 64);
  return v;
}

// part[k] += V_k[i] w for k <= j, and
// sum_{k <= j} coef[k] V_k[i]: basis rows are read CH at a time with the index
// clamped to j, so every load is issued without a branch (and lands in rows
// already written) and a thread's loads are in flight together.
template <int CH, int NP>
__device__ inline void dot_rows(int ns, int j, const double* __restrict__ V, int i, double w, double (&part)[NP]) {
#pragma unroll
  for (int c = 0; c < GM_MAXM / CH; ++c) {
    if (CH * c <= j) {
      double v[CH];
#pragma unroll
      for (int kk = 0; kk < CH; ++kk) v[kk] = V[(size_t)min(CH * c + kk, j) * ns + i];
#pragma unroll
      for (int kk = 0; kk < CH; ++kk)
        if (CH * c + kk <= j) part[CH * c + kk] += v[kk] * w;
    }
  }
}

template <int CH>
__device__ inline double comb_rows(int ns, int j, const double* __restrict__ V, int i, const double* coef) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < GM_MAXM / CH; ++c) {
    if (CH * c <= j) {
      double v[CH];
#pragma unroll
      for (int kk = 0; kk < CH; ++kk) v[kk] = V[(size_t)min(CH * c + kk, j) * ns + i];
#pragma unroll
      for (int kk = 0; kk < CH; ++kk)
        if (CH * c + kk <= j) s += coef[CH * c + kk] * v[kk];
    }
  }
  return s;
}

// Sum of one value over the block, result broadcast to every thread.
__device__ inline double block_sum(double v, GmresShared& sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh.red[wid][0] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < GM_WAVES; ++w) s += sh.red[w][0];
  return s;
}

// hv[k] = <V_k, w> for k <= j, reduced over the block into sh.hv.
__device__ inline void multi_dot(int ns, int j, const double* __restrict__ V, const double* __restrict__ w,
                                 GmresShared& sh) {
  double part[GM_MAXM];
#pragma unroll
  for (int k = 0; k < GM_MAXM; ++k) part[k] = 0.0;
  for (int i = threadIdx.x; i < ns; i += GM_THREADS) {
    const double wi = w[i];
#pragma unroll
    for (int k = 0; k < GM_MAXM; ++k)
      if (k <= j) part[k] += V[(size_t)k * ns + i] * wi;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < GM_MAXM; ++k) {
    if (k <= j) {
      const double v = wave_sum(part[k]);
      if (lane == 0) sh.red[wid][k] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x <= j) {
    double s = 0.0;
    for (int w2 = 0; w2 < GM_WAVES; ++w2) s += sh.red[w2][threadIdx.x];
    sh.hv[threadIdx.x] = s;
  }
  __syncthreads();
}

// Row i of A v with A padded to W entries per row, column-major ([k][row]):
// consecutive rows are consecutive addresses, and the loads of four entries
// are issued together before their products.
__device__ inline double ell_row(int i, int ns, int W, const int32_t* __restrict__ ec,
                                 const double* __restrict__ ev, const double* __restrict__ v) {
  double s0 = 0.0, s1 = 0.0;
  int k = 0;
  for (; k + 3 < W; k += 4) {
    const int64_t o = (int64_t)k * ns + i;
    const int c0 = ec[o], c1 = ec[o + ns], c2 = ec[o + 2 * ns], c3 = ec[o + 3 * ns];
    const double a0 = ev[o], a1 = ev[o + ns], a2 = ev[o + 2 * ns], a3 = ev[o + 3 * ns];
    const double v0 = v[c0], v1 = v[c1], v2 = v[c2], v3 = v[c3];
    s0 += a0 * v0 + a2 * v2;
    s1 += a1 * v1 + a3 * v3;
  }
  for (; k < W; ++k) {
    const int64_t o = (int64_t)k * ns + i;
    s0 += ev[o] * v[ec[o]];
  }
  return s0 + s1;
}

__device__ inline void spmv(int ns, int W, const int32_t* __restrict__ ec, const double* __restrict__ ev,
                            const double* __restrict__ v, double* __restrict__ y) {
  for (int i = threadIdx.x; i < ns; i += GM_THREADS) y[i] = ell_row(i, ns, W, ec, ev, v);
}

__global__ __launch_bounds__(GM_THREADS) void gmres_kernel(int ns, int W, const int32_t* __restrict__ ec,
                                                            const double* __restrict__ ev,
                                                            const double* __restrict__ b, double* __restrict__ x,
                                                            double* __restrict__ V, int m, int maxit, double tol,
                                                            StepStat* __restrict__ stat,
                                                            const double* __restrict__ xalt) {
  __shared__ GmresShared sh;
  const int tid = threadIdx.x;
  double bn2 = 0.0;
  for (int i = tid; i < ns; i += GM_THREADS) bn2 += b[i] * b[i];
  const double bnorm = sqrt(block_sum(bn2, sh));
  int it = 0;
  double rel = 0.0;
  int flags = 0;
  if (!(bnorm > 0.0)) {
    for (int i = tid; i < ns; i += GM_THREADS) x[i] = 0.0;
    if (!(bnorm == 0.0)) flags |= 2;
  } else {
    const double target = tol * bnorm;
    for (;;) {
      // r = b - A x  -> V_0
      double* V0 = V;
      spmv(ns, W, ec, ev, x, V0);
      double rr = 0.0;
      for (int i = tid; i < ns; i += GM_THREADS) {
        const double r = b[i] - V0[i];
        V0[i] = r;
        rr += r * r;
      }
      double beta = sqrt(block_sum(rr, sh));
      if (it == 0 && xalt) {
        // a second candidate starting point: keep whichever has the smaller residual
        double* V1 = V + ns;
        spmv(ns, W, ec, ev, xalt, V1);
        double ra = 0.0;
        for (int i = tid; i < ns; i += GM_THREADS) {
          const double r = b[i] - V1[i];
          V1[i] = r;
          ra += r * r;
        }
        const double beta_a = sqrt(block_sum(ra, sh));
        if (beta_a < beta || !(beta == beta)) {
          for (int i = tid; i < ns; i += GM_THREADS) {
            x[i] = xalt[i];
            V0[i] = V1[i];
          }
          beta = beta_a;
          flags |= 8;
          __syncthreads();
        }
      }
      if (it == 0 && !(beta <= bnorm)) {
        // the starting point is worse than zero (or not finite): start from x = 0
        for (int i = tid; i < ns; i += GM_THREADS) {
          x[i] = 0.0;
          V0[i] = b[i];
        }
        beta = bnorm;
        flags |= 4;
        __syncthreads();
      }
      rel = beta / bnorm;
      if (!(beta > target) || it >= maxit) {
        if (!(beta == beta)) flags |= 2;
        break;
      }
      for (int i = tid; i < ns; i += GM_THREADS) V0[i] /= beta;
      if (tid == 0) {
        sh.g[0] = beta;
        for (int k = 1; k <= m; ++k) sh.g[k] = 0.0;
      }
      __syncthreads();
      int jlast = -1;
      for (int j = 0; j < m; ++j) {
        double* Vj = V + (size_t)j * ns;
        double* Wv = V + (size_t)(j + 1) * ns;
        spmv(ns, W, ec, ev, Vj, Wv);
        __syncthreads();
        // classical Gram-Schmidt with a second pass only when the first removes
        // more than 99% of |W|^2 (as in the cooperative kernel)
        {
          double w2 = 0.0;
          for (int i = tid; i < ns; i += GM_THREADS) w2 += Wv[i] * Wv[i];
          w2 = block_sum(w2, sh);
          if (tid == 0) sh.scal[3] = w2;  // |W|^2, read by thread 0 below
        }
        for (int pass = 0; pass < 2; ++pass) {
          multi_dot(ns, j, V, Wv, sh);
          if (tid <= j) sh.H[tid][j] = (pass == 0 ? 0.0 : sh.H[tid][j]) + sh.hv[tid];
          if (tid == 0) {
            double hh = 0.0;
            for (int k = 0; k <= j; ++k) hh += sh.hv[k] * sh.hv[k];
            const double ww = sh.scal[3] - hh;
            sh.scal[2] = (pass == 0 && ww >= 0.01 * sh.scal[3]) ? sqrt(ww) : -1.0;
          }
          for (int i = tid; i < ns; i += GM_THREADS) Wv[i] -= comb_rows<4>(ns, j, V, i, sh.hv);
          __syncthreads();
          if (sh.scal[2] >= 0.0) break;
        }
        double hn = sh.scal[2];
        if (!(hn >= 0.0)) {
          double ww = 0.0;
          for (int i = tid; i < ns; i += GM_THREADS) ww += Wv[i] * Wv[i];
          hn = sqrt(block_sum(ww, sh));
        }
        if (hn > 0.0)
          for (int i = tid; i < ns; i += GM_THREADS) Wv[i] /= hn;
        if (tid == 0) {
          sh.H[j + 1][j] = hn;
          for (int k = 0; k < j; ++k) {  // previous rotations
            const double a = sh.H[k][j], c2 = sh.H[k + 1][j];
            sh.H[k][j] = sh.cs[k] * a + sh.sn[k] * c2;
            sh.H[k + 1][j] = -sh.sn[k] * a + sh.cs[k] * c2;
          }
          const double a = sh.H[j][j], c2 = sh.H[j + 1][j];
          const double den = sqrt(a * a + c2 * c2);
          const double cj = den > 0.0 ? a / den : 1.0, sj = den > 0.0 ? c2 / den : 0.0;
          sh.cs[j] = cj;
          sh.sn[j] = sj;
          sh.H[j][j] = cj * a + sj * c2;
          sh.H[j + 1][j] = 0.0;
          sh.g[j + 1] = -sj * sh.g[j];
          sh.g[j] = cj * sh.g[j];
          sh.scal[0] = fabs(sh.g[j + 1]);
          sh.scal[1] = hn;
        }
        __syncthreads();
        ++it;
        jlast = j;
        rel = sh.scal[0] / bnorm;
        if (!(sh.scal[0] > target) || it >= maxit || !(sh.scal[1] > 0.0)) break;
      }
      // x += V y with H y = g (upper triangular, size jlast+1)
      if (tid == 0) {
        for (int k = jlast; k >= 0; --k) {
          double s = sh.g[k];
          for (int l = k + 1; l <= jlast; ++l) s -= sh.H[k][l] * sh.y[l];
          sh.y[k] = s / sh.H[k][k];
        }
      }
      __syncthreads();
      for (int i = tid; i < ns; i += GM_THREADS) x[i] += comb_rows<4>(ns, jlast, V, i, sh.y);
      __syncthreads();
      if (!(rel * bnorm > target) || it >= maxit) {
        if (!(rel == rel)) flags |= 2;
        break;
      }
    }
    if (rel * bnorm > target) flags |= 1;
  }
  if (tid == 0 && stat) {
    stat->iters = it;
    stat->resid = rel;
    stat->flags = flags;
    stat->xmax = 0.0;
  }
}

constexpr int GC_THREADS = 256;

// Two rows per call (i0, i1) so that both rows' loads are in flight together.
__device__ inline void ell_row2(int i0, int i1, int ns, int W, const int32_t* __restrict__ ec,
                                const double* __restrict__ ev, const double* __restrict__ v, double& y0,
                                double& y1) {
  double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
  int k = 0;
  for (; k + 3 < W; k += 4) {
    const int64_t o = (int64_t)k * ns;
    int c0[4], c1[4];
    double e0[4], e1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c0[q] = ec[o + q * ns + i0];
      c1[q] = ec[o + q * ns + i1];
      e0[q] = ev[o + q * ns + i0];
      e1[q] = ev[o + q * ns + i1];
    }
    double x0[4], x1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x0[q] = v[c0[q]];
      x1[q] = v[c1[q]];
    }
    a0 += e0[0] * x0[0] + e0[2] * x0[2];
    b0 += e0[1] * x0[1] + e0[3] * x0[3];
    a1 += e1[0] * x1[0] + e1[2] * x1[2];
    b1 += e1[1] * x1[1] + e1[3] * x1[3];
  }
  for (; k < W; ++k) {
    const int64_t o = (int64_t)k * ns;
    a0 += ev[o + i0] * v[ec[o + i0]];
    a1 += ev[o + i1] * v[ec[o + i1]];
  }
  y0 = a0 + b0;
  y1 = a1 + b1;
}

template <int CH>
__device__ inline void dot_rows2(int ns, int j, const double* __restrict__ V, int i0, int i1, double w0, double w1,
                                 double (&part)[GM_MAXM + 1]) {
#pragma unroll
  for (int c = 0; c < GM_MAXM / CH; ++c) {
    if (CH * c <= j) {
      double v0[CH], v1[CH];
#pragma unroll
      for (int kk = 0; kk < CH; ++kk) {
        const size_t r = (size_t)min(CH * c + kk, j) * ns;
        v0[kk] = V[r + i0];
        v1[kk] = V[r + i1];
      }
#pragma unroll
      for (int kk = 0; kk < CH; ++kk)
        if (CH * c + kk <= j) part[CH * c + kk] += v0[kk] * w0 + v1[kk] * w1;
    }
  }
}

template <int CH>
__device__ inline void comb_rows2(int ns, int j, const double* __restrict__ V, int i0, int i1, const double* coef,
                                  double& s0, double& s1) {
  s0 = 0.0;
  s1 = 0.0;
#pragma unroll
  for (int c = 0; c < GM_MAXM / CH; ++c) {
    if (CH * c <= j) {
      double v0[CH], v1[CH];
#pragma unroll
      for (int kk = 0; kk < CH; ++kk) {
        const size_t r = (size_t)min(CH * c + kk, j) * ns;
        v0[kk] = V[r + i0];
        v1[kk] = V[r + i1];
      }
#pragma unroll
      for (int kk = 0; kk < CH; ++kk)
        if (CH * c + kk <= j) {
          s0 += coef[CH * c + kk] * v0[kk];
          s1 += coef[CH * c + kk] * v1[kk];
        }
    }
  }
}



struct CoopShared {
  double H[GM_MAXM + 1][GM_MAXM];
  double cs[GM_MAXM], sn[GM_MAXM], g[GM_MAXM + 1], y[GM_MAXM];
  double red[GC_THREADS / 64][GM_MAXM + 1];
  double hv[GM_MAXM + 1];
};

// Sum over the grid of per-thread values part[0..n-1] (n <= GM_MAXM+1): wave and
// block reduction, per-workgroup partials to gpart[wg][*], grid barrier, then an
// ordered sum over workgroups into sh.hv (identical in every workgroup).
__device__ inline void grid_multi_sum(int n, const double* part, double* __restrict__ gpart_all, int& flip,
                                      CoopShared& sh, cooperative_groups::grid_group& grid) {
  // two partial buffers used alternately: a buffer is rewritten only two
  // reductions later, after every workgroup has passed the barrier in between
  double* __restrict__ gpart = gpart_all + (size_t)flip * gridDim.x * (GM_MAXM + 1);
  flip ^= 1;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < GM_MAXM + 1; ++k) {
    if (k < n) {
      const double v = wave_sum(part[k]);
      if (lane == 0) sh.red[wid][k] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < n) {
    double s = 0.0;
    for (int w = 0; w < GC_THREADS / 64; ++w) s += sh.red[w][threadIdx.x];
    gpart[blockIdx.x * (GM_MAXM + 1) + threadIdx.x] = s;
  }
  grid.sync();  // orders memory at device scope: the partials are visible after it
  if (threadIdx.x < n) {
    // every workgroup's partial loaded at once, then summed in workgroup order
    const int G = (int)gridDim.x;
    double s = 0.0;
    for (int w0 = 0; w0 < G; w0 += 16) {
      double v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = gpart[min(w0 + q, G - 1) * (GM_MAXM + 1) + threadIdx.x];
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (w0 + q < G) s += v[q];
    }
    sh.hv[threadIdx.x] = s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(GC_THREADS) void gmres_coop_kernel(
    int ns, int W, const int32_t* __restrict__ ec, const double* __restrict__ ev,
    const double* __restrict__ b, double* __restrict__ x, double* __restrict__ V, int m, int maxit, double tol,
    StepStat* __restrict__ stat, double* __restrict__ gpart, const double* __restrict__ xalt) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  __shared__ CoopShared sh;
  const int tid = threadIdx.x;
  const int per = (ns + gridDim.x - 1) / gridDim.x;
  const int r0 = blockIdx.x * per, r1 = min(ns, r0 + per);
  double part[GM_MAXM + 1];
  int flip = 0;
  part[0] = 0.0;
  for (int i = r0 + tid; i < r1; i += GC_THREADS) part[0] += b[i] * b[i];
  grid_multi_sum(1, part, gpart, flip, sh, grid);
  const double bnorm = sqrt(sh.hv[0]);
  int it = 0, flags = 0;
  double rel = 0.0;
  if (!(bnorm > 0.0)) {
    for (int i = r0 + tid; i < r1; i += GC_THREADS) x[i] = 0.0;
    if (!(bnorm == 0.0)) flags |= 2;
  } else {
    const double target = tol * bnorm;
    for (;;) {
      double* V0 = V;
      part[0] = 0.0;
      for (int i = r0 + tid; i < r1; i += GC_THREADS) {
        const double r = b[i] - ell_row(i, ns, W, ec, ev, x);
        V0[i] = r;
        part[0] += r * r;
      }
      grid_multi_sum(1, part, gpart, flip, sh, grid);
      double beta = sqrt(sh.hv[0]);
      if (it == 0 && xalt) {
        // a second candidate starting point: keep whichever has the smaller residual
        // (both norms are grid-wide sums, so every workgroup takes the same branch)
        double* V1 = V + ns;
        part[0] = 0.0;
        for (int i = r0 + tid; i < r1; i += GC_THREADS) {
          const double r = b[i] - ell_row(i, ns, W, ec, ev, xalt);
          V1[i] = r;
          part[0] += r * r;
        }
        grid_multi_sum(1, part, gpart, flip, sh, grid);
        const double beta_a = sqrt(sh.hv[0]);
        if (beta_a < beta || !(beta == beta)) {
          for (int i = r0 + tid; i < r1; i += GC_THREADS) {
            x[i] = xalt[i];
            V0[i] = V1[i];
          }
          beta = beta_a;
          flags |= 8;
        }
      }
      if (it == 0 && !(beta <= bnorm)) {
        // the starting point is worse than zero (or not finite): start from x = 0
        // (beta is the same in every workgroup, so all take this branch together)
        for (int i = r0 + tid; i < r1; i += GC_THREADS) {
          x[i] = 0.0;
          V0[i] = b[i];
        }
        beta = bnorm;
        flags |= 4;
      }
      rel = beta / bnorm;
      if (!(beta > target) || it >= maxit) {
        if (!(beta == beta)) flags |= 2;
        break;
      }
      for (int i = r0 + tid; i < r1; i += GC_THREADS) V0[i] /= beta;
      if (tid == 0) {
        sh.g[0] = beta;
        for (int k = 1; k <= m; ++k) sh.g[k] = 0.0;
      }
      grid.sync();
      int jlast = -1;
      for (int j = 0; j < m; ++j) {
        const double* Vj = V + (size_t)j * ns;
        double* Wv = V + (size_t)(j + 1) * ns;
        // rows two at a time (i1 clamped to i0 past the slice end, its result dropped)
        for (int i0 = r0 + tid; i0 < r1; i0 += 2 * GC_THREADS) {
          const bool has1 = i0 + GC_THREADS < r1;
          const int i1 = has1 ? i0 + GC_THREADS : i0;
          double y0, y1;
          ell_row2(i0, i1, ns, W, ec, ev, Vj, y0, y1);
          Wv[i0] = y0;
          if (has1) Wv[i1] = y1;
        }
        // Classical Gram-Schmidt, repeated only when the first pass cancels
        // badly (the test of Daniel, Gragg, Kaufman and Stewart with eta = 0.1):
        // each pass's reduction also carries |W|^2 (value j+1), and
        // |W - sum h_k V_k|^2 = |W|^2 - sum h_k^2 for orthonormal V_k.  If a pass
        // keeps more than eta^2 of |W|^2, the orthogonality it leaves is within
        // ~eps / eta and the difference is accurate to ~eps / eta^2; otherwise a
        // second pass (whose h_k are at rounding level) follows.  Every workgroup
        // holds the same sums, so all take the same branch.
        double ww = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
          for (int k = 0; k < GM_MAXM + 1; ++k) part[k] = 0.0;
          for (int i0 = r0 + tid; i0 < r1; i0 += 2 * GC_THREADS) {
            const bool has1 = i0 + GC_THREADS < r1;
            const int i1 = has1 ? i0 + GC_THREADS : i0;
            const double w0 = Wv[i0], w1 = has1 ? Wv[i1] : 0.0;
            dot_rows2<8>(ns, j, V, i0, i1, w0, w1, part);
#pragma unroll
            for (int k = 1; k < GM_MAXM + 1; ++k)
              if (k == j + 1) part[k] += w0 * w0 + w1 * w1;
          }
          grid_multi_sum(j + 2, part, gpart, flip, sh, grid);
          if (tid <= j) sh.H[tid][j] = (pass == 0 ? 0.0 : sh.H[tid][j]) + sh.hv[tid];
          double hh = 0.0;
          for (int k = 0; k <= j; ++k) hh += sh.hv[k] * sh.hv[k];
          const double w2 = sh.hv[j + 1];
          ww = w2 - hh;
          for (int i0 = r0 + tid; i0 < r1; i0 += 2 * GC_THREADS) {
            const bool has1 = i0 + GC_THREADS < r1;
            const int i1 = has1 ? i0 + GC_THREADS : i0;
            double c0, c1;
            comb_rows2<8>(ns, j, V, i0, i1, sh.hv, c0, c1);
            Wv[i0] -= c0;
            if (has1) Wv[i1] -= c1;
          }
          if (ww >= 0.01 * w2) break;
        }
        const double hn = ww >= 0.0 ? sqrt(ww) : (ww < 0.0 ? 0.0 : ww);  // NaN stays NaN
        if (hn > 0.0)
          for (int i = r0 + tid; i < r1; i += GC_THREADS) Wv[i] /= hn;
        if (tid == 0) {
          sh.H[j + 1][j] = hn;
          for (int k = 0; k < j; ++k) {
            const double a = sh.H[k][j], c2 = sh.H[k + 1][j];
            sh.H[k][j] = sh.cs[k] * a + sh.sn[k] * c2;
            sh.H[k + 1][j] = -sh.sn[k] * a + sh.cs[k] * c2;
          }
          const double a = sh.H[j][j], c2 = sh.H[j + 1][j];
          const double den = sqrt(a * a + c2 * c2);
          const double cj = den > 0.0 ? a / den : 1.0, sj = den > 0.0 ? c2 / den : 0.0;
          sh.cs[j] = cj;
          sh.sn[j] = sj;
          sh.H[j][j] = cj * a + sj * c2;
          sh.H[j + 1][j] = 0.0;
          sh.g[j + 1] = -sj * sh.g[j];
          sh.g[j] = cj * sh.g[j];
        }
        grid.sync();  // W normalised everywhere; every workgroup's Givens state updated
        ++it;
        jlast = j;
        rel = fabs(sh.g[j + 1]) / bnorm;
        if (!(fabs(sh.g[j + 1]) > target) || it >= maxit || !(hn > 0.0)) break;
      }
      if (tid == 0) {
        for (int k = jlast; k >= 0; --k) {
          double s2 = sh.g[k];
          for (int l = k + 1; l <= jlast; ++l) s2 -= sh.H[k][l] * sh.y[l];
          sh.y[k] = s2 / sh.H[k][k];
        }
      }
      __syncthreads();
      for (int i = r0 + tid; i < r1; i += GC_THREADS) x[i] += comb_rows<8>(ns, jlast, V, i, sh.y);
      grid.sync();
      if (!(rel * bnorm > target) || it >= maxit) {
        if (!(rel == rel)) flags |= 2;
        break;
      }
    }
    if (rel * bnorm > target) flags |= 1;
  }
  if (blockIdx.x == 0 && tid == 0 && stat) {
    stat->iters = it;
    stat->resid = rel;
    stat->flags = flags;
    stat->xmax = 0.0;
  }
}

void launch_gmres(tdbem_ctx* ctx, const double* b, double* x, StepStat* stat, const double* xalt) {
  ProfScope ps(ctx, K_GMRES);
  int m = ctx->opts.gmres_restart;
  if (m > GM_MAXM) m = GM_MAXM;
  if (m < 1) m = 1;
  // a cooperative launch is not captured into a graph: the single-workgroup
  // solver serves captured marches
  const int nwg = ctx->capturing ? 1 : ctx->gmres_wg;
  if (nwg <= 1) {
    gmres_kernel<<<1, GM_THREADS, 0, ctx->stream>>>(ctx->ns, ctx->ell_w, ctx->d_ell_col.p, ctx->d_ell_val.p, b, x,
                                                     ctx->d_V.p, m, ctx->opts.gmres_maxiter, ctx->opts.gmres_tol,
                                                     stat, xalt);
    TDBEM_HIP(hipGetLastError());
    return;
  }
  int ns = ctx->ns, maxit = ctx->opts.gmres_maxiter;
  double tol = ctx->opts.gmres_tol;
  int W = ctx->ell_w;
  const int32_t* ec = ctx->d_ell_col.p;
  const double* ev = ctx->d_ell_val.p;
  double* V = ctx->d_V.p;
  double* gp = ctx->d_gpart.p;
  void* args[] = {&ns, &W, &ec, &ev, &b, &x, &V, &m, &maxit, &tol, &stat, &gp, &xalt};
  TDBEM_HIP(hipLaunchCooperativeKernel((const void*)gmres_coop_kernel, dim3(nwg), dim3(GC_THREADS), args, 0,
                                       ctx->stream));
}

// Largest cooperative grid that is guaranteed co-resident (one workgroup per CU at most).
static int gmres_max_workgroups() {
  int dev = 0, ncu = 0, per = 0;
  TDBEM_HIP(hipGetDevice(&dev));
  TDBEM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  TDBEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)gmres_coop_kernel, GC_THREADS, 0));
  return std::max(1, std::min(ncu * std::max(per, 1), ncu));
}

int gmres_workgroups(int ns) {
  // one workgroup per 512 rows, capped by what is guaranteed co-resident
  if (ns <= 2048) return 1;
  return std::max(1, std::min((ns + 511) / 512, gmres_max_workgroups()));
}

// Time the per-step solve on a fixed right-hand side (all ones, zero start) with
// the single-workgroup kernel and with 128 ... 1024 rows per workgroup of the
// cooperative kernel, and keep the fastest.
void autotune_gmres(tdbem_ctx* ctx) {
  const int ns = ctx->ns;
  if (ns <= 2048) return;
  const int cap = gmres_max_workgroups();
  std::vector<int> cand = {1};  // 1: the single-workgroup kernel (no grid barriers)
  for (int rows : {1024, 512, 256, 128}) {
    const int w = std::max(1, std::min((ns + rows - 1) / rows, cap));
    if (std::find(cand.begin(), cand.end(), w) == cand.end()) cand.push_back(w);
  }
  const int wmax = *std::max_element(cand.begin(), cand.end());
  if (ctx->d_gpart.n < (size_t)2 * wmax * 33) ctx->d_gpart.alloc((size_t)2 * wmax * 33);
  std::vector<double> ones(ns, 1.0);
  TDBEM_HIP(hipMemcpyAsync(ctx->d_b.p, ones.data(), ns * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  hipEvent_t e0, e1;
  TDBEM_HIP(hipEventCreate(&e0));
  TDBEM_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bestw = ctx->gmres_wg;
  const bool prof = ctx->prof;
  ctx->prof = false;
  for (int w : cand) {
    ctx->gmres_wg = w;
    float tot = 0.f;
    for (int r = 0; r < 3; ++r) {
      TDBEM_HIP(hipMemsetAsync(ctx->d_x.p, 0, ns * sizeof(double), ctx->stream));
      TDBEM_HIP(hipEventRecord(e0, ctx->stream));
      launch_gmres(ctx, ctx->d_b.p, ctx->d_x.p, ctx->d_stat.p);
      TDBEM_HIP(hipEventRecord(e1, ctx->stream));
      TDBEM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      TDBEM_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (r > 0) tot += ms;
    }
    if (tot < best) { best = tot; bestw = w; }
  }
  ctx->prof = prof;
  ctx->gmres_wg = bestw;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  TDBEM_HIP(hipMemsetAsync(ctx->d_x.p, 0, ns * sizeof(double), ctx->stream));
  TDBEM_HIP(hipMemsetAsync(ctx->d_stat.p, 0, sizeof(StepStat), ctx->stream));
  TDBEM_HIP(hipStreamSynchronize(ctx->stream));
}

}  // namespace tdbem
