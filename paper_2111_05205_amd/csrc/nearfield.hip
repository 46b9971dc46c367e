// Near-field part of the marching-on-in-time right-hand side.
//
// For each collocation row i and each near element j the library stores the
// compact coefficients C_X^{(g)}_ij = sum_kappa w^{kappa,d} X^{(g-kappa)}_ij
// (X = U, W for the OBIE; Ubar, Wbar for the BMBIE), i.e. the kappa sum of
// eq. bie_disc folded into the matrices instead of the densities (the
// identity of App. A read the other way round).  C^{(g)}_ij can be non-zero
// only for rmin/(c dt) < g < rmax/(c dt) + d + 1 (B-spline support, Remark
// support), so each pair keeps a short window of g values.  The history sum
//   b_i += sum_j sum_{g >= 2} ( C_U^{(g)}_ij q_j^{alpha-g} - C_W^{(g)}_ij u_j^{alpha-g} )
// is HBM-bound: one pass over the coefficient stream per step, history rows
// served from L2.  g = 1 is the unknown step; it forms the constant matrix
// A = w^{0,d} (W^{(1)} phi - U^{(1)} (1 - phi)) of eq. linear.
#include "internal.h"

#include <algorithm>

#include <cmath>

namespace tdbem {

__constant__ GLRule c_gl;

static GLRule make_gl16() {
  GLRule r;
  const int n = 16;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    r.x[i] = x;
    r.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return r;
}

void upload_gl_rule() {
  GLRule r = make_gl16();
  TDBEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gl), &r, sizeof(GLRule)));
}

struct NearParams {
  int d, bie;
  double cdt, Cd;
  BWeights bw;
  int raw;  // store raw X^{(gamma)} (tau form) instead of compact coefficients
};

// One block per row: window (glo, cnt) of every pair of the row.
__global__ void near_window_kernel(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ pj,
                                   const double* __restrict__ xc, const double* __restrict__ tris,
                                   int d, double cdt, int32_t* __restrict__ gw) {
  const int i = blockIdx.x;
  const double x[3] = {xc[3 * i], xc[3 * i + 1], xc[3 * i + 2]};
  for (int64_t p = row_ptr[i] + threadIdx.x; p < row_ptr[i + 1]; p += blockDim.x) {
    const int j = pj[p];
    double rmin, rmax;
    tri_dist_range(x, tris + 9 * (int64_t)j, &rmin, &rmax);
    if (j == i) rmin = 0.0;
    int glo, cnt;
    time_window(rmin, rmax, d, cdt, &glo, &cnt);
    gw[p] = (glo << 16) | cnt;
  }
}

// One block per row: compact coefficients of every pair of the row.
__global__ void near_fill_kernel(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ pj,
                                 const int32_t* __restrict__ gw, const int64_t* __restrict__ off,
                                 const double* __restrict__ xc, const double* __restrict__ nrm,
                                 const double* __restrict__ tris, NearParams P,
                                 double* __restrict__ cu, double* __restrict__ cw) {
  const int i = blockIdx.x;
  const double x[3] = {xc[3 * i], xc[3 * i + 1], xc[3 * i + 2]};
  const double ni[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
  for (int64_t p = row_ptr[i] + threadIdx.x; p < row_ptr[i + 1]; p += blockDim.x) {
    const int j = pj[p];
    const int glo = gw[p] >> 16, cnt = gw[p] & 0xffff;
    const int64_t o = off[p];
    for (int k = 0; k < cnt; ++k) { cu[o + k] = 0.0; cw[o + k] = 0.0; }
    int gmin = glo - P.d - 1;
    if (gmin < 1) gmin = 1;
    const int gmax = glo + cnt - 1;
    for (int gam = gmin; gam <= gmax; ++gam) {
      double X[4];
      elem_families_gl(c_gl, x, ni, tris + 9 * (int64_t)j, nrm + 3 * (int64_t)j, i == j, gam * P.cdt, P.d,
                       P.Cd, X);
      const double xu = P.bie ? X[2] : X[0];
      const double xw = P.bie ? X[3] : X[1];
      if (P.raw) {  // below glo the raw values vanish (the wavefront has not reached E_j)
        if (gam >= glo) { cu[o + gam - glo] = xu; cw[o + gam - glo] = xw; }
        continue;
      }
      for (int kap = 0; kap <= P.d + 1; ++kap) {
        const int g = gam + kap;
        if (g < glo || g > gmax) continue;
        cu[o + g - glo] += P.bw.w[kap] * xu;
        cw[o + g - glo] += P.bw.w[kap] * xw;
      }
    }
  }
}

void build_near_table(tdbem_ctx* ctx, const std::vector<int64_t>& row_ptr, const std::vector<int32_t>& pair_j) {
  const int ns = ctx->ns;
  ctx->npairs = row_ptr[ns];
  ctx->d_row_ptr.alloc(ns + 1);
  ctx->d_pair_j.alloc(ctx->npairs);
  ctx->d_pair_gw.alloc(ctx->npairs);
  ctx->d_pair_off.alloc(ctx->npairs);
  TDBEM_HIP(hipMemcpyAsync(ctx->d_row_ptr.p, row_ptr.data(), (ns + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                           ctx->stream));
  TDBEM_HIP(hipMemcpyAsync(ctx->d_pair_j.p, pair_j.data(), ctx->npairs * sizeof(int32_t), hipMemcpyHostToDevice,
                           ctx->stream));
  near_window_kernel<<<ns, 256, 0, ctx->stream>>>(ctx->d_row_ptr.p, ctx->d_pair_j.p, ctx->d_xc.p, ctx->d_tris.p,
                                                  ctx->d, ctx->cdt, ctx->d_pair_gw.p);
  TDBEM_HIP(hipGetLastError());
  std::vector<int32_t> gw(ctx->npairs);
  TDBEM_HIP(hipMemcpyAsync(gw.data(), ctx->d_pair_gw.p, ctx->npairs * sizeof(int32_t), hipMemcpyDeviceToHost,
                           ctx->stream));
  TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<int64_t> off(ctx->npairs);
  int64_t tot = 0;
  for (int64_t p = 0; p < ctx->npairs; ++p) {
    off[p] = tot;
    int cnt = gw[p] & 0xffff;
    if (cnt <= 0 || cnt > 4096) throw Error(TDBEM_E_INVAL, "time window out of range; is c*dt too small for the mesh?");
    tot += cnt;
  }
  ctx->ncoef = tot;
  TDBEM_HIP(hipMemcpyAsync(ctx->d_pair_off.p, off.data(), ctx->npairs * sizeof(int64_t), hipMemcpyHostToDevice,
                           ctx->stream));
  ctx->d_cu.alloc(tot);
  ctx->d_cw.alloc(tot);
  NearParams P;
  P.d = ctx->d;
  P.bie = ctx->bie;
  P.cdt = ctx->cdt;
  P.Cd = 1.0 / (4.0 * M_PI * std::pow(ctx->cdt, ctx->d));
  P.bw = ctx->bw;
  P.raw = ctx->opts.near_form == 1 ? 1 : 0;
  near_fill_kernel<<<ns, 128, 0, ctx->stream>>>(ctx->d_row_ptr.p, ctx->d_pair_j.p, ctx->d_pair_gw.p,
                                                ctx->d_pair_off.p, ctx->d_xc.p, ctx->d_nrm.p, ctx->d_tris.p, P,
                                                ctx->d_cu.p, ctx->d_cw.p);
  TDBEM_HIP(hipGetLastError());
  TDBEM_HIP(hipStreamSynchronize(ctx->stream));
}

// ---------------------------------------------------------------------------
// Per-step matrix: pairs whose window starts at g = 1.

__global__ void a_count_kernel(int ns, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ gw,
                               int32_t* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  int c = 0;
  for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) c += ((gw[p] >> 16) == 1);
  cnt[i] = c;
}

__global__ void a_fill_kernel(int ns, int bc, double c1, const int8_t* __restrict__ phi,
                              const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ pj,
                              const int32_t* __restrict__ gw, const int64_t* __restrict__ off,
                              const double* __restrict__ cu, const double* __restrict__ cw,
                              const int32_t* __restrict__ a_ptr, int32_t* __restrict__ a_col,
                              double* __restrict__ a_val, double* __restrict__ u1, double* __restrict__ w1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  int k = a_ptr[i];
  for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
    if ((gw[p] >> 16) != 1) continue;
    // C^{(1)} = w^0 X^{(1)} (X^{(0)} = 0): c1 = w^0 when the table holds raw values, else 1
    const double cu1 = c1 * cu[off[p]], cw1 = c1 * cw[off[p]];
    a_col[k] = pj[p];
    // column j: the unknown is u (phi_j = 1: W family) or q (phi_j = 0: -U family)
    const bool ucol = phi ? phi[pj[p]] != 0 : bc == TDBEM_NEUMANN;
    a_val[k] = ucol ? cw1 : -cu1;
    u1[k] = cu1;
    w1[k] = cw1;
    ++k;
  }
}

__global__ void ell_fill_kernel(int ns, int W, const int32_t* __restrict__ ap, const int32_t* __restrict__ ac,
                                const double* __restrict__ av, int32_t* __restrict__ ec, double* __restrict__ ev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int k0 = ap[i], n = ap[i + 1] - k0;
  for (int k = 0; k < W; ++k) {
    ec[(int64_t)k * ns + i] = k < n ? ac[k0 + k] : i;
    ev[(int64_t)k * ns + i] = k < n ? av[k0 + k] : 0.0;
  }
}

void build_step_matrix(tdbem_ctx* ctx) {
  const int ns = ctx->ns;
  DevBuf<int32_t> cnt;
  cnt.alloc(ns);
  a_count_kernel<<<(ns + 255) / 256, 256, 0, ctx->stream>>>(ns, ctx->d_row_ptr.p, ctx->d_pair_gw.p, cnt.p);
  TDBEM_HIP(hipGetLastError());
  std::vector<int32_t> h(ns), ptr(ns + 1);
  TDBEM_HIP(hipMemcpyAsync(h.data(), cnt.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  ptr[0] = 0;
  for (int i = 0; i < ns; ++i) ptr[i + 1] = ptr[i] + h[i];
  ctx->a_nnz = ptr[ns];
  ctx->d_a_ptr.alloc(ns + 1);
  ctx->d_a_col.alloc(ctx->a_nnz);
  ctx->d_a_val.alloc(ctx->a_nnz);
  ctx->d_u1_val.alloc(ctx->a_nnz);
  ctx->d_w1_val.alloc(ctx->a_nnz);
  TDBEM_HIP(hipMemcpyAsync(ctx->d_a_ptr.p, ptr.data(), (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                           ctx->stream));
  a_fill_kernel<<<(ns + 255) / 256, 256, 0, ctx->stream>>>(
      ns, ctx->bc, ctx->opts.near_form == 1 ? ctx->bw.w[0] : 1.0, ctx->bc == TDBEM_MIXED ? ctx->d_phi.p : nullptr,
      ctx->d_row_ptr.p, ctx->d_pair_j.p, ctx->d_pair_gw.p, ctx->d_pair_off.p, ctx->d_cu.p, ctx->d_cw.p,
      ctx->d_a_ptr.p, ctx->d_a_col.p, ctx->d_a_val.p, ctx->d_u1_val.p, ctx->d_w1_val.p);
  TDBEM_HIP(hipGetLastError());
  ctx->ell_w = h.empty() ? 1 : std::max(1, *std::max_element(h.begin(), h.end()));
  ctx->d_ell_col.alloc((size_t)ctx->ell_w * ns);
  ctx->d_ell_val.alloc((size_t)ctx->ell_w * ns);
  ell_fill_kernel<<<(ns + 255) / 256, 256, 0, ctx->stream>>>(ns, ctx->ell_w, ctx->d_a_ptr.p, ctx->d_a_col.p,
                                                             ctx->d_a_val.p, ctx->d_ell_col.p, ctx->d_ell_val.p);
  TDBEM_HIP(hipGetLastError());
  TDBEM_HIP(hipStreamSynchronize(ctx->stream));
}

// ---------------------------------------------------------------------------
// History sum, one 64-wide wavefront per row.

// TAU: the table holds raw X^{(gamma)}, gamma = glo .. ghi, and the kappa sum is
// taken on the densities, tau = sum_kappa w^kappa q^{alpha-gamma-kappa} over the
// kappa with gamma + kappa <= ghi (the pair's last gap: App. A's truncation), as in
// eq. linear; otherwise the table holds the compact coefficients C^{(g)}.
template <class CT, bool TAU>
__global__ __launch_bounds__(256) void near_history_kernel(
    int ns, int alpha, BWeights bw, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ pj,
    const int32_t* __restrict__ gw, const int64_t* __restrict__ off, const CT* __restrict__ cu,
    const CT* __restrict__ cw, const double* __restrict__ hu, const double* __restrict__ hq, int use_u,
    int use_q, const double* __restrict__ base, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= ns) return;
  double acc = 0.0;
  for (int64_t p = row_ptr[i] + lane; p < row_ptr[i + 1]; p += 64) {
    const int j = pj[p];
    const int glo = gw[p] >> 16, cnt = gw[p] & 0xffff;
    const int64_t o = off[p];
    if constexpr (TAU) {
      const int ghi = glo + cnt - 1;
      for (int k = 0; k < cnt; ++k) {
        const int gam = glo + k;
        double tq = 0.0, su = 0.0;
        for (int kap = 0; kap <= bw.d + 1 && gam + kap <= ghi; ++kap) {
          const int beta = alpha - gam - kap;
          if (gam + kap < 2 || beta < 0) continue;  // the unknown step and before the march
          const int64_t h = (int64_t)beta * ns + j;
          if (use_q) tq += bw.w[kap] * hq[h];
          if (use_u) su += bw.w[kap] * hu[h];
        }
        acc += (double)cu[o + k] * tq - (double)cw[o + k] * su;
      }
    } else {
      int k0 = glo >= 2 ? 0 : 2 - glo;  // g = glo + k >= 2
      for (int k = k0; k < cnt; ++k) {
        const int beta = alpha - glo - k;
        if (beta < 0) break;
        const int64_t h = (int64_t)beta * ns + j;
        if (use_q) acc += (double)cu[o + k] * hq[h];
        if (use_u) acc -= (double)cw[o + k] * hu[h];
      }
    }
  }
  for (int s = 32; s > 0; s >>= 1) acc += __shfl_down(acc, s, 64);
  if (lane == 0) out[i] = (base ? base[i] : 0.0) + acc;
}

void launch_near_history(tdbem_ctx* ctx, int alpha, const double* base, double* out) {
  ProfScope ps(ctx, K_NEAR);
  const int rows_per_block = 4;
  const dim3 grid((ctx->ns + rows_per_block - 1) / rows_per_block), block(64 * rows_per_block);
  const bool tau = ctx->opts.near_form == 1, f32 = ctx->opts.near_prec == 1;
  const int uu = ctx->hist_u ? 1 : 0, uq = ctx->hist_q ? 1 : 0;
#define TDBEM_NEAR_ARGS ctx->ns, alpha, ctx->bw, ctx->d_row_ptr.p, ctx->d_pair_j.p, ctx->d_pair_gw.p, ctx->d_pair_off.p
  if (f32 && tau)
    near_history_kernel<float, true><<<grid, block, 0, ctx->stream>>>(TDBEM_NEAR_ARGS, ctx->d_cu32.p, ctx->d_cw32.p,
                                                                      ctx->d_hu.p, ctx->d_hq.p, uu, uq, base, out);
  else if (f32)
    near_history_kernel<float, false><<<grid, block, 0, ctx->stream>>>(TDBEM_NEAR_ARGS, ctx->d_cu32.p, ctx->d_cw32.p,
                                                                       ctx->d_hu.p, ctx->d_hq.p, uu, uq, base, out);
  else if (tau)
    near_history_kernel<double, true><<<grid, block, 0, ctx->stream>>>(TDBEM_NEAR_ARGS, ctx->d_cu.p, ctx->d_cw.p,
                                                                       ctx->d_hu.p, ctx->d_hq.p, uu, uq, base, out);
  else
    near_history_kernel<double, false><<<grid, block, 0, ctx->stream>>>(TDBEM_NEAR_ARGS, ctx->d_cu.p, ctx->d_cw.p,
                                                                        ctx->d_hu.p, ctx->d_hq.p, uu, uq, base, out);
#undef TDBEM_NEAR_ARGS
  TDBEM_HIP(hipGetLastError());
}

__global__ void to_float_kernel(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = (float)a[k];
}

// opts.near_prec = 1: keep only FP32 copies of the near table (after A is built from the FP64 values)
void near_table_to_fp32(tdbem_ctx* ctx) {
  const int64_t n = ctx->ncoef;
  ctx->d_cu32.alloc(std::max<int64_t>(n, 1));
  ctx->d_cw32.alloc(std::max<int64_t>(n, 1));
  if (n > 0) {
    to_float_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(n, ctx->d_cu.p, ctx->d_cu32.p);
    to_float_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(n, ctx->d_cw.p, ctx->d_cw32.p);
    TDBEM_HIP(hipGetLastError());
  }
  TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  ctx->d_cu.release();
  ctx->d_cw.release();
}

// y += scale * M x for M in the sparsity pattern of A.
__global__ void spmv_add_kernel(int ns, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                const double* __restrict__ val, double scale, const double* __restrict__ x,
                                double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  double s = 0.0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * x[col[k]];
  y[i] += scale * s;
}

__global__ void spmv_add_masked_kernel(int ns, const int32_t* __restrict__ ap, const int32_t* __restrict__ ac,
                                       const double* __restrict__ av, double scale, const double* __restrict__ x,
                                       const int8_t* __restrict__ phi, int want, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  double s = 0.0;
  for (int k = ap[i]; k < ap[i + 1]; ++k) {
    const int j = ac[k];
    if ((phi[j] != 0) == (want != 0)) s += av[k] * x[j];
  }
  y[i] += scale * s;
}

void launch_spmv_add_masked(tdbem_ctx* ctx, const double* vals, double scale, const double* xin, int want,
                            double* y) {
  ProfScope ps(ctx, K_OTHER);
  spmv_add_masked_kernel<<<(ctx->ns + 255) / 256, 256, 0, ctx->stream>>>(
      ctx->ns, ctx->d_a_ptr.p, ctx->d_a_col.p, vals, scale, xin, ctx->d_phi.p, want, y);
  TDBEM_HIP(hipGetLastError());
}

// Direct history sums at arbitrary points, one workgroup per point, every
// element summed on the fly (no table): compact coefficients
// C^{(g)}(x, E_j) = sum_kappa w^kappa X^{(g-kappa)}(x, E_j) over each element's window,
// times the stored history,
//   out = sum_j sum_{g=gfirst}^{alpha} (C_U^{(g)} q_j^{alpha-g} - C_W^{(g)} u_j^{alpha-g}).
// Off-surface points (row < 0): the single and double layer (U, W) of eq. bie_disc,
// gfirst = 1.  Collocation rows (row = i): the context's families at x_i with its
// normal (U, W or the Burton-Miller Ubar, Wbar), the self pair as in the near table,
// gfirst = 2 (the history part of b^{alpha-1}, what the FMM approximates).  The raw
// values X^{(gamma)} of the last d+2 gammas sit in a shift register, so each is
// evaluated once.
__global__ __launch_bounds__(256) void direct_points_kernel(int ns, const double* __restrict__ pts,
                                                            const int32_t* __restrict__ rows,
                                                            const double* __restrict__ tris,
                                                            const double* __restrict__ nrm, NearParams P, int alpha,
                                                            const double* __restrict__ hu,
                                                            const double* __restrict__ hq, double* __restrict__ out) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  const int row = rows ? rows[r] : -1;
  const double* xp = row >= 0 ? pts + 3 * (int64_t)row : pts + 3 * (int64_t)r;
  const double x[3] = {xp[0], xp[1], xp[2]};
  const int fu = row >= 0 && P.bie ? 2 : 0, fw = fu + 1, gfirst = row >= 0 ? 2 : 1;
  double acc = 0.0;
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
    double rmin, rmax;
    tri_dist_range(x, tris + 9 * (int64_t)j, &rmin, &rmax);
    if (j == row) rmin = 0.0;
    int glo, cnt;
    time_window(rmin, rmax, P.d, P.cdt, &glo, &cnt);
    const int gmax = min(glo + cnt - 1, alpha);
    if (gmax < max(glo, gfirst)) continue;        // nothing of this element reaches (x, t_alpha) yet
    const double* nj = nrm + 3 * (int64_t)j;
    const double* ni = row >= 0 ? nrm + 3 * (int64_t)row : nj;
    double xu[5] = {0, 0, 0, 0, 0}, xw[5] = {0, 0, 0, 0, 0};  // X^{(gamma - k)}, k = 0..4
    for (int gam = max(glo - P.d - 1, 1); gam <= gmax; ++gam) {
      double X[4];
      elem_families_gl(c_gl, x, ni, tris + 9 * (int64_t)j, nj, j == row, gam * P.cdt, P.d, P.Cd, X);
#pragma unroll
      for (int k = 4; k > 0; --k) { xu[k] = xu[k - 1]; xw[k] = xw[k - 1]; }
      xu[0] = X[fu];
      xw[0] = X[fw];
      if (gam < glo || gam < gfirst) continue;
      double cu = 0.0, cw = 0.0;
#pragma unroll
      for (int kap = 0; kap < 5; ++kap)
        if (kap <= P.d + 1) { cu += P.bw.w[kap] * xu[kap]; cw += P.bw.w[kap] * xw[kap]; }
      const int64_t hrow = (int64_t)(alpha - gam) * ns + j;
      acc += cu * hq[hrow] - cw * hu[hrow];
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[r] = (red[0] + red[1]) + (red[2] + red[3]);
}

static NearParams near_params(const tdbem_ctx* ctx) {
  NearParams P;
  P.d = ctx->d;
  P.bie = ctx->bie;
  P.cdt = ctx->cdt;
  P.Cd = 1.0 / (4.0 * M_PI * std::pow(ctx->cdt, ctx->d));
  P.bw = ctx->bw;
  return P;
}

void launch_field(tdbem_ctx* ctx, int npts, const double* pts, int alpha, double* out) {
  direct_points_kernel<<<npts, 256, 0, ctx->stream>>>(ctx->ns, pts, nullptr, ctx->d_tris.p, ctx->d_nrm.p,
                                                      near_params(ctx), alpha, ctx->d_hu.p, ctx->d_hq.p, out);
  TDBEM_HIP(hipGetLastError());
}

void launch_direct_rows(tdbem_ctx* ctx, int nrows, const int32_t* rows, int alpha, double* out) {
  direct_points_kernel<<<nrows, 256, 0, ctx->stream>>>(ctx->ns, ctx->d_xc.p, rows, ctx->d_tris.p, ctx->d_nrm.p,
                                                       near_params(ctx), alpha, ctx->d_hu.p, ctx->d_hq.p, out);
  TDBEM_HIP(hipGetLastError());
}

void launch_spmv_add(tdbem_ctx* ctx, const double* vals, double scale, const double* xin, double* y) {
  ProfScope ps(ctx, K_OTHER);
  spmv_add_kernel<<<(ctx->ns + 255) / 256, 256, 0, ctx->stream>>>(ctx->ns, ctx->d_a_ptr.p, ctx->d_a_col.p, vals,
                                                                    scale, xin, y);
  TDBEM_HIP(hipGetLastError());
}

}  // namespace tdbem
