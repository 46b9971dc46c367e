// C ABI of the library: context set-up and the marching-on-in-time driver.
//
// Step alpha (collocation time t_alpha, unknown coefficient beta = alpha-1),
// eq. linear with the compact B-spline coefficients:
//   b   = f^alpha + sum_{g>=2} (C_U^{(g)} q^{alpha-g} - C_W^{(g)} u^{alpha-g})   near pairs (direct)
//       + far field at (x_i, t_alpha)                                        far pairs (FMM, L2P)
//       + known current-step part (prescribed boundary coefficients)
//   A x = b                                                                   GMRES, one workgroup
//   store x (u on Neumann faces, q on Dirichlet faces) as row beta
//   P2M of the new sample; interval-end M2M / M2L (Algorithm 1) / L2L           FMM
// Everything runs on the context's stream; tdbem_run issues the whole march
// without host synchronisation and reads the per-step statistics once.
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <utility>

using namespace tdbem;

static thread_local std::string g_create_err;

template <class F>
static int guarded(tdbem_ctx* ctx, F&& f) {
  try {
    f();
    return TDBEM_OK;
  } catch (const Error& e) {
    if (ctx) ctx->err = e.msg; else g_create_err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what(); else g_create_err = e.what();
    return TDBEM_E_INVAL;
  }
}

static void fail(int code, const std::string& m) { throw Error(code, m); }

#define TDBEM_HIP_NOTHROW(call) (void)(call)

namespace tdbem {
void set_global_error(const std::string& msg) { g_create_err = msg; }
}  // namespace tdbem

// ---------------------------------------------------------------------------
// Geometry and mesh validation (host).

static Geometry build_geometry(const tdbem_mesh* mesh) {
  if (!mesh || !mesh->xyz || !mesh->tri) fail(TDBEM_E_INVAL, "mesh arrays are NULL");
  const int nv = mesh->nv, nt = mesh->nt;
  if (nv < 4 || nt < 4) fail(TDBEM_E_INVAL, "mesh needs at least 4 vertices and 4 triangles");
  if (nt > (1 << 27)) fail(TDBEM_E_INVAL, "too many triangles");
  Geometry g;
  g.ns = nt;
  g.xc.resize(3 * (size_t)nt);
  g.nrm.resize(3 * (size_t)nt);
  g.tris.resize(9 * (size_t)nt);
  g.area.resize(nt);
  for (int k = 0; k < 3; ++k) { g.ext_lo[k] = 1e300; g.ext_hi[k] = -1e300; }
  for (int v = 0; v < nv; ++v)
    for (int k = 0; k < 3; ++k) {
      const double c = mesh->xyz[3 * (size_t)v + k];
      if (!std::isfinite(c)) fail(TDBEM_E_INVAL, "non-finite vertex coordinate");
      g.ext_lo[k] = std::min(g.ext_lo[k], c);
      g.ext_hi[k] = std::max(g.ext_hi[k], c);
    }
  std::map<std::pair<int, int>, int> edges;
  double esum = 0.0;
  long ecount = 0;
  for (int t = 0; t < nt; ++t) {
    int id[3];
    for (int k = 0; k < 3; ++k) {
      id[k] = mesh->tri[3 * (size_t)t + k];
      if (id[k] < 0 || id[k] >= nv) fail(TDBEM_E_INVAL, "triangle index out of range");
    }
    if (id[0] == id[1] || id[1] == id[2] || id[0] == id[2]) fail(TDBEM_E_INVAL, "degenerate triangle");
    const double* A = mesh->xyz + 3 * (size_t)id[0];
    const double* B = mesh->xyz + 3 * (size_t)id[1];
    const double* C = mesh->xyz + 3 * (size_t)id[2];
    double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double cr[3];
    cross3(e1, e2, cr);
    const double twoa = std::sqrt(dot3(cr, cr));
    if (!(twoa > 0.0)) fail(TDBEM_E_INVAL, "zero-area triangle");
    g.area[t] = 0.5 * twoa;
    for (int k = 0; k < 3; ++k) {
      g.nrm[3 * (size_t)t + k] = -cr[k] / twoa;  // paper normal: into the scatterer
      g.xc[3 * (size_t)t + k] = (A[k] + B[k] + C[k]) / 3.0;
      g.tris[9 * (size_t)t + k] = A[k];
      g.tris[9 * (size_t)t + 3 + k] = B[k];
      g.tris[9 * (size_t)t + 6 + k] = C[k];
    }
    for (int k = 0; k < 3; ++k) {
      const int a = id[k], b = id[(k + 1) % 3];
      if (++edges[{a, b}] > 1) fail(TDBEM_E_INVAL, "mesh is not consistently oriented (repeated directed edge)");
      const double* P = mesh->xyz + 3 * (size_t)a;
      const double* Q = mesh->xyz + 3 * (size_t)b;
      double dv[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
      const double l = std::sqrt(dot3(dv, dv));
      g.edge_max = std::max(g.edge_max, l);
      if (a < b) { esum += l; ++ecount; }
      double cv[3] = {P[0] - g.xc[3 * (size_t)t], P[1] - g.xc[3 * (size_t)t + 1], P[2] - g.xc[3 * (size_t)t + 2]};
      g.e_max = std::max(g.e_max, std::sqrt(dot3(cv, cv)));
    }
  }
  for (const auto& e : edges)
    if (edges.find({e.first.second, e.first.first}) == edges.end())
      fail(TDBEM_E_INVAL, "mesh is not closed (edge without an opposite edge)");
  g.edge_mean = ecount ? esum / ecount : 0.0;
  return g;
}

static BWeights bspline_weights(int d) {
  BWeights b{};
  b.d = d;
  for (int k = 0; k <= d + 1; ++k) {
    double p = 1.0;
    for (int m = 0; m <= d + 1; ++m)
      if (m != k) p *= (double)(m - k);
    b.w[k] = (double)(d + 1) / p;
  }
  return b;
}

// ---------------------------------------------------------------------------
// Small kernels of the driver.

__global__ void store_step_kernel(int ns, int beta, int bc, const int8_t* __restrict__ phi,
                                  const double* __restrict__ x, const double* __restrict__ bcv,
                                  double* __restrict__ hu, double* __restrict__ hq, StepStat* __restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int64_t r = (int64_t)beta * ns + i;
  const double xv = x[i], pv = bcv ? bcv[i] : 0.0;
  const bool uface = phi ? phi[i] != 0 : bc == TDBEM_NEUMANN;  // u unknown, q given
  if (uface) { hu[r] = xv; hq[r] = pv; }
  else { hq[r] = xv; hu[r] = pv; }
  if (!isfinite(xv) || fabs(xv) > 1e100) atomicOr(&st->flags, 2);
  // max |x| of the step: non-negative doubles order like their bit patterns
  else atomicMax(reinterpret_cast<unsigned long long*>(&st->xmax), (unsigned long long)__double_as_longlong(fabs(xv)));
}

// Growth check of row beta (opts.growth_limit): the reference takes in row beta - lag, then the
// row fails when its largest coefficient exceeds limit times the reference.
__global__ void growth_check_kernel(int beta, int lag, double limit, StepStat* __restrict__ stats,
                                    double* __restrict__ ref) {
  double r = *ref;
  if (beta >= lag) {
    r = fmax(r, stats[beta - lag].xmax);
    *ref = r;
  }
  if (r > 0.0 && stats[beta].xmax > limit * r) atomicOr(&stats[beta].flags, 16);
}

// Rows of the unknown coefficient (u on phi = 1 faces, q on phi = 0 faces) of a
// mixed-condition march.
__global__ void unknown_rows_kernel(int ns, int64_t n, const int8_t* __restrict__ phi, const double* __restrict__ hu,
                                    const double* __restrict__ hq, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  out[k] = phi[k % ns] ? hu[k] : hq[k];
}

// Starting point of the per-step solve: quadratic extrapolation of the last
// three solved coefficient rows (previous row, or zero, early in the march),
// zero, or the previous row.
__global__ void guess_kernel(int ns, int beta, int mode, const double* __restrict__ hu, const double* __restrict__ hq,
                             const int8_t* __restrict__ phi, int bc, double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const double* h = (phi ? phi[i] != 0 : bc == TDBEM_NEUMANN) ? hu : hq;  // history of this face's unknown
  double v = 0.0;
  if (mode == TDBEM_GUESS_ZERO) v = 0.0;
  else if (mode == TDBEM_GUESS_PREV) v = beta >= 1 ? h[(int64_t)(beta - 1) * ns + i] : 0.0;
  else if (beta >= 3)
    v = 3.0 * h[(int64_t)(beta - 1) * ns + i] - 3.0 * h[(int64_t)(beta - 2) * ns + i] + h[(int64_t)(beta - 3) * ns + i];
  else if (beta >= 1)
    v = h[(int64_t)(beta - 1) * ns + i];
  x[i] = v;
}

__global__ void forcing_kernel(int ns, int a0, int n, int bie, double c, double dt, tdbem_incident inc,
                               const double* __restrict__ xc, const double* __restrict__ nrm,
                               double* __restrict__ out) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)n * ns) return;
  const int i = (int)(id % ns);
  const int a = a0 + (int)(id / ns);
  const double t = a * dt;
  const double kx = inc.dir[0] * xc[3 * i] + inc.dir[1] * xc[3 * i + 1] + inc.dir[2] * xc[3 * i + 2];
  const double kn = inc.dir[0] * nrm[3 * i] + inc.dir[1] * nrm[3 * i + 1] + inc.dir[2] * nrm[3 * i + 2];
  double val;
  if (inc.kind == TDBEM_INC_GAUSS_MOD) {
    // u = exp(-p^2 / 2 sigma^2) cos(2 pi f0 p), p = t - (k.x + rb)/c - t0
    const double p = t - (kx + inc.rb) / c - inc.t0;
    const double om = 2.0 * M_PI * inc.f0;
    const double env = exp(-p * p / (2.0 * inc.sigma * inc.sigma));
    const double cs = cos(om * p), sn = sin(om * p);
    if (bie == TDBEM_OBIE) val = env * cs;
    else {
      const double du = env * (-p / (inc.sigma * inc.sigma) * cs - om * sn);  // du/dp
      val = -du * (kn + 1.0) / c;  // grad u = -du k / c, du/dt = du
    }
  } else {
    // u = (1 - cos a)/2 for 0 <= a <= 2 pi, else 0;  a = 2 pi (c t - k.x - rb) / lambda
    const double lam = inc.sigma;
    const double a2 = 2.0 * M_PI * (c * t - kx - inc.rb) / lam;
    const bool in = a2 >= 0.0 && a2 <= 2.0 * M_PI;
    if (bie == TDBEM_OBIE) val = in ? 0.5 * (1.0 - cos(a2)) : 0.0;
    else val = in ? 0.5 * sin(a2) * (2.0 * M_PI / lam) * (-kn - 1.0) : 0.0;
  }
  out[id] = val;
}

namespace tdbem {
void launch_forcing(tdbem_ctx* ctx, const tdbem_incident& inc0, int a0, int n, double* out) {
  tdbem_incident inc = inc0;
  const double nd = std::sqrt(inc.dir[0] * inc.dir[0] + inc.dir[1] * inc.dir[1] + inc.dir[2] * inc.dir[2]);
  if (!(nd > 0.0)) fail(TDBEM_E_INVAL, "incident direction is zero");
  for (int k = 0; k < 3; ++k) inc.dir[k] /= nd;
  if (inc.kind != TDBEM_INC_GAUSS_MOD && inc.kind != TDBEM_INC_RAISED_COS) fail(TDBEM_E_INVAL, "incident kind");
  if (!(inc.sigma > 0.0)) fail(TDBEM_E_INVAL, "incident sigma must be > 0");
  const int64_t tot = (int64_t)n * ctx->ns;
  if (tot == 0) return;
  forcing_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, ctx->stream>>>(ctx->ns, a0, n, ctx->bie, ctx->c, ctx->dt,
                                                                         inc, ctx->d_xc.p, ctx->d_nrm.p, out);
  TDBEM_HIP(hipGetLastError());
}
}  // namespace tdbem

// ---------------------------------------------------------------------------

static tdbem_opts default_opts() {
  tdbem_opts o{};
  o.use_fmm = 0;
  o.depth = 4;
  o.p_s = 4;
  o.p_t = 4;
  o.mu = 0;
  o.m2l_prec = TDBEM_M2L_FP64;
  o.gmres_tol = 1e-12;
  o.gmres_restart = 30;
  o.gmres_maxiter = 300;
  o.nt_max = 4096;
  return o;
}

// One collocation step.  defer: stop the FMM after P2M and M2M and return the number of
// levels whose M2L is still to be launched (fmm_batch_m2l), then fmm_advance_post.
static int do_step(tdbem_ctx* ctx, const double* forcing, const double* bcv, StepStat* stat, bool defer = false) {
  const int alpha = ctx->alpha, beta = alpha - 1;
  if (alpha > ctx->nt_max - 1) fail(TDBEM_E_STATE, "step beyond nt_max");
  launch_near_history(ctx, alpha, forcing, ctx->d_b.p);
  if (ctx->fmm) fmm_far(ctx, alpha, ctx->d_b.p);
  if (bcv) {
    if (ctx->bc == TDBEM_MIXED) {  // q given on phi = 1 faces, u given on phi = 0 faces
      launch_spmv_add_masked(ctx, ctx->d_u1_val.p, 1.0, bcv, 1, ctx->d_b.p);
      launch_spmv_add_masked(ctx, ctx->d_w1_val.p, -1.0, bcv, 0, ctx->d_b.p);
    } else if (ctx->bc == TDBEM_DIRICHLET) {
      launch_spmv_add(ctx, ctx->d_w1_val.p, -1.0, bcv, ctx->d_b.p);
    } else {
      launch_spmv_add(ctx, ctx->d_u1_val.p, 1.0, bcv, ctx->d_b.p);
    }
  }
  const bool use_mlp = (ctx->opts.guess == TDBEM_GUESS_MLP || ctx->opts.guess == TDBEM_GUESS_MLP_ONLY) &&
                       ctx->mlp_loaded && beta >= 4;
  float* feat = nullptr;
  if (beta >= 4 && (use_mlp || ctx->rec_feat)) {
    feat = ctx->rec_feat ? ctx->rec_feat + (size_t)beta * ctx->ns * TDBEM_MLP_IN_PAD : ctx->d_mlp_feat.p;
    launch_mlp_features(ctx, beta, ctx->d_b.p, feat);
  }
  const double* xalt = nullptr;
  if (use_mlp) {
    launch_mlp_guess(ctx, beta, feat, ctx->d_x.p, ctx->d_x_alt.p);
    if (ctx->opts.guess == TDBEM_GUESS_MLP) xalt = ctx->d_x_alt.p;
  } else {
    ProfScope pg(ctx, K_OTHER);
    guess_kernel<<<(ctx->ns + 255) / 256, 256, 0, ctx->stream>>>(
        ctx->ns, beta, ctx->opts.guess, ctx->d_hu.p, ctx->d_hq.p, ctx->bc == TDBEM_MIXED ? ctx->d_phi.p : nullptr,
        ctx->bc, ctx->d_x.p);
    TDBEM_HIP(hipGetLastError());
  }
  launch_gmres(ctx, ctx->d_b.p, ctx->d_x.p, stat, xalt);
  ProfScope* ps = new ProfScope(ctx, K_OTHER);
  store_step_kernel<<<(ctx->ns + 255) / 256, 256, 0, ctx->stream>>>(
      ctx->ns, beta, ctx->bc, ctx->bc == TDBEM_MIXED ? ctx->d_phi.p : nullptr, ctx->d_x.p, bcv, ctx->d_hu.p,
      ctx->d_hq.p, stat);
  if (ctx->opts.growth_limit > 0.0) {
    growth_check_kernel<<<1, 1, 0, ctx->stream>>>(beta, ctx->opts.growth_lag, ctx->opts.growth_limit,
                                                   stat - beta, ctx->d_growth_ref.p);
  }
  delete ps;
  TDBEM_HIP(hipGetLastError());
  if (ctx->bc == TDBEM_MIXED) { ctx->hist_u = true; ctx->hist_q = true; }
  else if (ctx->bc == TDBEM_NEUMANN) { ctx->hist_u = true; if (bcv) ctx->hist_q = true; }
  else { ctx->hist_q = true; if (bcv) ctx->hist_u = true; }
  if (feat && ctx->rec_target) launch_mlp_target(ctx, beta, ctx->rec_target + (size_t)beta * ctx->ns);
  int ndue = 0;
  if (ctx->fmm) {
    if (defer) ndue = fmm_advance_pre(ctx, beta);
    else fmm_advance(ctx, beta);
  }
  ctx->alpha = alpha + 1;
  return ndue;
}

// ---------------------------------------------------------------------------
// March drivers shared by tdbem_run and tdbem_run_batch.

static const double* run_prepare(tdbem_ctx* ctx, int nt, const double* dev_forcing, const tdbem_incident* inc) {
  if (nt < 2 || nt > ctx->nt_max) fail(TDBEM_E_INVAL, "nt out of range [2, nt_max]");
  if (ctx->alpha > nt - 1) fail(TDBEM_E_STATE, "march already past nt-1; call tdbem_reset");
  if (dev_forcing) return dev_forcing;
  if (!inc) return nullptr;
  const size_t need = (size_t)(nt - 1) * ctx->ns;
  if (ctx->d_forc.n < need) ctx->d_forc.alloc(need);
  launch_forcing(ctx, *inc, 1, nt - 1, ctx->d_forc.p);
  return ctx->d_forc.p;
}

static bool use_graph(const tdbem_ctx* ctx) {
  return ctx->opts.graph && ctx->alpha == 1 && !ctx->prof && !ctx->rec_feat;
}

static void march_steps(tdbem_ctx* ctx, int nt, const double* forc) {
  for (int alpha = ctx->alpha; alpha <= nt - 1; ++alpha)
    do_step(ctx, forc ? forc + (size_t)(alpha - 1) * ctx->ns : ctx->d_zero.p, nullptr, ctx->d_stat.p + (alpha - 1));
}

void tdbem::invalidate_graph(tdbem_ctx* ctx) {
  if (ctx->g_exec) (void)hipGraphExecDestroy(ctx->g_exec);
  ctx->g_exec = nullptr;
  ctx->g_nt = 0;
  ctx->g_forc = nullptr;
}

// Capture the march from alpha = 1 to nt-1 into a graph (host work only: the
// launches are recorded, not run) unless one for (nt, forcing) exists.  The
// host-side state a march leaves behind is kept for the replays.
static void ensure_graph(tdbem_ctx* ctx, int nt, const double* forc) {
  if (ctx->g_exec && ctx->g_nt == nt && ctx->g_forc == forc) return;
  invalidate_graph(ctx);
  if (!ctx->cap_stream) TDBEM_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  const hipStream_t user = ctx->stream;
  const int a0 = ctx->alpha;
  const bool hu0 = ctx->hist_u, hq0 = ctx->hist_q;
  ctx->stream = ctx->cap_stream;
  ctx->capturing = true;
  hipGraph_t g = nullptr;
  TDBEM_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  try {
    march_steps(ctx, nt, forc);
  } catch (...) {
    (void)hipStreamEndCapture(ctx->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    ctx->stream = user;
    ctx->capturing = false;
    ctx->alpha = a0;
    ctx->hist_u = hu0;
    ctx->hist_q = hq0;
    throw;
  }
  e = hipStreamEndCapture(ctx->stream, &g);
  ctx->stream = user;
  ctx->capturing = false;
  ctx->g_alpha = ctx->alpha;
  ctx->g_hu = ctx->hist_u;
  ctx->g_hq = ctx->hist_q;
  ctx->alpha = a0;
  ctx->hist_u = hu0;
  ctx->hist_q = hq0;
  if (e != hipSuccess) fail(TDBEM_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&ctx->g_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    ctx->g_exec = nullptr;
    fail(TDBEM_E_DEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(e));
  }
  ctx->g_nt = nt;
  ctx->g_forc = forc;
}

// Issue the march on the context stream: the captured graph, or step by step.
static void run_launch(tdbem_ctx* ctx, int nt, const double* forc) {
  if (use_graph(ctx)) {
    ensure_graph(ctx, nt, forc);
    TDBEM_HIP(hipGraphLaunch(ctx->g_exec, ctx->stream));
    ctx->alpha = ctx->g_alpha;
    ctx->hist_u = ctx->g_hu;
    ctx->hist_q = ctx->g_hq;
  } else {
    march_steps(ctx, nt, forc);
  }
}

// Wait for the march, copy the history out and summarise the per-step records.
static int run_finish(tdbem_ctx* ctx, int nt, int a_first, double* dev_x_hist_out, tdbem_run_info* info,
                      hipEvent_t e0, hipEvent_t e1) {
  const int ns = ctx->ns;
  int rc = TDBEM_OK;
  if (dev_x_hist_out) {
    if (ctx->bc == TDBEM_MIXED) {
      const int64_t n = (int64_t)(nt - 1) * ns;
      unknown_rows_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(ns, n, ctx->d_phi.p, ctx->d_hu.p,
                                                                                ctx->d_hq.p, dev_x_hist_out);
      TDBEM_HIP(hipGetLastError());
    } else {
      const double* src = ctx->bc == TDBEM_NEUMANN ? ctx->d_hu.p : ctx->d_hq.p;
      TDBEM_HIP(hipMemcpyAsync(dev_x_hist_out, src, (size_t)(nt - 1) * ns * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
    }
  }
  std::vector<StepStat> st(nt - 1);
  TDBEM_HIP(hipMemcpyAsync(st.data(), ctx->d_stat.p, (nt - 1) * sizeof(StepStat), hipMemcpyDeviceToHost,
                           ctx->stream));
  TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  float ms = 0.f;
  TDBEM_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tdbem_run_info ri{};
  ri.march_ms = ms;
  for (int a = a_first; a <= nt - 1; ++a) {
    const StepStat& s = st[a - 1];
    ri.steps++;
    ri.total_iters += s.iters;
    ri.max_iters = std::max(ri.max_iters, s.iters);
    ri.max_resid = std::max(ri.max_resid, s.resid);
    if (s.flags & 4) ri.guesses_rejected++;
    if (s.flags & 8) ri.guesses_replaced++;
    if ((s.flags & 2) && rc == TDBEM_OK) {
      rc = TDBEM_E_DIVERGED;
      ctx->err = "non-finite or exploding solution at step " + std::to_string(a);
    } else if ((s.flags & 16) && rc == TDBEM_OK) {
      rc = TDBEM_E_DIVERGED;
      ctx->err = "solution grew beyond growth_limit at step " + std::to_string(a);
    } else if ((s.flags & 1) && rc == TDBEM_OK) {
      rc = TDBEM_E_NOT_CONVERGED;
      ctx->err = "GMRES did not converge at step " + std::to_string(a);
    }
  }
  if (info) *info = ri;
  return rc;
}

extern "C" {

static int create_impl(const tdbem_mesh* mesh, double c, double dt, int d, int bie, int bc, const int8_t* face_bc,
                       const tdbem_opts* opts, void* hip_stream, tdbem_ctx** out) {
  if (!out) { g_create_err = "out is NULL"; return TDBEM_E_INVAL; }
  *out = nullptr;
  tdbem_ctx* ctx = new tdbem_ctx();
  int rc = guarded(nullptr, [&] {
    auto t0 = std::chrono::steady_clock::now();
    if (!(c > 0.0) || !(dt > 0.0)) fail(TDBEM_E_INVAL, "c and dt must be > 0");
    if (d < 1 || d > 3) fail(TDBEM_E_INVAL, "B-spline order d must be 1, 2 or 3");
    if (bie != TDBEM_OBIE && bie != TDBEM_BMBIE) fail(TDBEM_E_INVAL, "bie must be OBIE (0) or BMBIE (1)");
    if (bc != TDBEM_DIRICHLET && bc != TDBEM_NEUMANN && bc != TDBEM_MIXED)
      fail(TDBEM_E_INVAL, "bc must be DIRICHLET (0) or NEUMANN (1)");
    if (bc == TDBEM_MIXED && !face_bc) fail(TDBEM_E_INVAL, "mixed condition without face types");
    ctx->opts = opts ? *opts : default_opts();
    tdbem_opts& o = ctx->opts;
    if (bc == TDBEM_MIXED && (o.guess == TDBEM_GUESS_MLP || o.guess == TDBEM_GUESS_MLP_ONLY))
      fail(TDBEM_E_INVAL, "the learned starting point needs a single boundary condition");
    if (!(o.gmres_tol > 0.0)) o.gmres_tol = 1e-12;
    if (o.gmres_restart <= 0) o.gmres_restart = 30;
    if (o.gmres_maxiter <= 0) o.gmres_maxiter = 300;
    if (o.nt_max <= 1) o.nt_max = 4096;
    if (o.guess < TDBEM_GUESS_EXTRAP || o.guess > TDBEM_GUESS_MLP_ONLY) fail(TDBEM_E_INVAL, "guess must be 0..4");
    if (o.near_form != 0 && o.near_form != 1) fail(TDBEM_E_INVAL, "near_form must be 0 (compact) or 1 (tau form)");
    if (o.near_prec != 0 && o.near_prec != 1) fail(TDBEM_E_INVAL, "near_prec must be 0 (FP64) or 1 (FP32)");
    if (!(o.growth_limit >= 0.0)) fail(TDBEM_E_INVAL, "growth_limit must be >= 0");
    if (o.growth_limit > 0.0 && o.growth_lag < 1) fail(TDBEM_E_INVAL, "growth_lag must be >= 1");
    ctx->stream = (hipStream_t)hip_stream;
    ctx->c = c;
    ctx->dt = dt;
    ctx->cdt = c * dt;
    ctx->d = d;
    ctx->bie = bie;
    ctx->bc = bc;
    ctx->bw = bspline_weights(d);
    ctx->geo = build_geometry(mesh);
    ctx->ns = ctx->geo.ns;
    const int ns = ctx->ns;
    if (bc == TDBEM_MIXED) {
      ctx->phi.assign(face_bc, face_bc + ns);
      for (auto& v : ctx->phi) {
        if (v != 0 && v != 1) fail(TDBEM_E_INVAL, "face types must be 0 (u given) or 1 (q given)");
      }
      ctx->d_phi.alloc(ns);
      TDBEM_HIP(hipMemcpyAsync(ctx->d_phi.p, ctx->phi.data(), ns, hipMemcpyHostToDevice, ctx->stream));
    }
    upload_gl_rule();
    ctx->d_xc.alloc(3 * (size_t)ns);
    ctx->d_nrm.alloc(3 * (size_t)ns);
    ctx->d_tris.alloc(9 * (size_t)ns);
    TDBEM_HIP(hipMemcpyAsync(ctx->d_xc.p, ctx->geo.xc.data(), 3 * ns * sizeof(double), hipMemcpyHostToDevice,
                             ctx->stream));
    TDBEM_HIP(hipMemcpyAsync(ctx->d_nrm.p, ctx->geo.nrm.data(), 3 * ns * sizeof(double), hipMemcpyHostToDevice,
                             ctx->stream));
    TDBEM_HIP(hipMemcpyAsync(ctx->d_tris.p, ctx->geo.tris.data(), 9 * ns * sizeof(double), hipMemcpyHostToDevice,
                             ctx->stream));
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> pair_j;
    if (o.use_fmm) {
      ctx->fmm = fmm_create(ctx);
      fmm_near_pairs(ctx, row_ptr, pair_j);
    } else {
      if ((int64_t)ns * ns > (int64_t)2000000000) fail(TDBEM_E_INVAL, "direct mode limited to ~2e9 pairs");
      row_ptr.resize(ns + 1);
      pair_j.resize((size_t)ns * ns);
      for (int i = 0; i <= ns; ++i) row_ptr[i] = (int64_t)i * ns;
      for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ns; ++j) pair_j[(size_t)i * ns + j] = j;
    }
    build_near_table(ctx, row_ptr, pair_j);
    build_step_matrix(ctx);
    if (o.near_prec == 1) near_table_to_fp32(ctx);
    ctx->nt_max = o.nt_max;
    ctx->d_hu.alloc((size_t)ctx->nt_max * ns);
    ctx->d_hq.alloc((size_t)ctx->nt_max * ns);
    TDBEM_HIP(hipMemsetAsync(ctx->d_hu.p, 0, ctx->d_hu.n * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_hq.p, 0, ctx->d_hq.n * sizeof(double), ctx->stream));
    ctx->d_b.alloc(ns);
    ctx->d_x.alloc(ns);
    ctx->d_zero.alloc(ns);
    ctx->d_V.alloc((size_t)(std::min(ctx->opts.gmres_restart, 32) + 1) * ns);
    ctx->d_stat.alloc(ctx->nt_max);
    ctx->d_growth_ref.alloc(1);
    ctx->gmres_wg = gmres_workgroups(ns);
    ctx->d_gpart.alloc((size_t)2 * std::max(ctx->gmres_wg, 1) * 33);
    TDBEM_HIP(hipMemsetAsync(ctx->d_x.p, 0, ns * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_zero.p, 0, ns * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_stat.p, 0, ctx->nt_max * sizeof(StepStat), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_growth_ref.p, 0, sizeof(double), ctx->stream));
    autotune_gmres(ctx);
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
    ctx->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
  if (rc != TDBEM_OK) {
    tdbem_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return TDBEM_OK;
}

int tdbem_create(const tdbem_mesh* mesh, double c, double dt, int d, int bie, int bc, const tdbem_opts* opts,
                 void* hip_stream, tdbem_ctx** out) {
  if (bc == TDBEM_MIXED) {
    g_create_err = "bc must be DIRICHLET (0) or NEUMANN (1); mixed conditions: tdbem_create_mixed";
    if (out) *out = nullptr;
    return TDBEM_E_INVAL;
  }
  return create_impl(mesh, c, dt, d, bie, bc, nullptr, opts, hip_stream, out);
}

int tdbem_create_mixed(const tdbem_mesh* mesh, double c, double dt, int d, int bie, const int8_t* face_bc,
                       const tdbem_opts* opts, void* hip_stream, tdbem_ctx** out) {
  if (!face_bc) {
    g_create_err = "face_bc is NULL";
    if (out) *out = nullptr;
    return TDBEM_E_INVAL;
  }
  return create_impl(mesh, c, dt, d, bie, TDBEM_MIXED, face_bc, opts, hip_stream, out);
}

int tdbem_field(tdbem_ctx* ctx, int npts, const double* host_pts, int alpha, double* dev_out) {
  if (!ctx) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    if (npts < 0 || (npts > 0 && (!host_pts || !dev_out))) fail(TDBEM_E_INVAL, "field: bad arguments");
    if (alpha < 1 || alpha > ctx->alpha - 1)
      fail(TDBEM_E_INVAL, "field: alpha must be in [1, position - 1] (solved rows 0 .. alpha-1)");
    if (npts == 0) return;
    DevBuf<double> pts;
    pts.alloc(3 * (size_t)npts);
    TDBEM_HIP(hipMemcpyAsync(pts.p, host_pts, 3 * (size_t)npts * sizeof(double), hipMemcpyHostToDevice,
                             ctx->stream));
    launch_field(ctx, npts, pts.p, alpha, dev_out);
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tdbem_direct_rows(tdbem_ctx* ctx, int nrows, const int32_t* host_rows, int alpha, double* dev_out) {
  if (!ctx) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    if (nrows < 0 || (nrows > 0 && (!host_rows || !dev_out))) fail(TDBEM_E_INVAL, "direct_rows: bad arguments");
    if (alpha < 1 || alpha > ctx->alpha) fail(TDBEM_E_INVAL, "direct_rows: alpha must be in [1, position]");
    for (int r = 0; r < nrows; ++r)
      if (host_rows[r] < 0 || host_rows[r] >= ctx->ns) fail(TDBEM_E_INVAL, "direct_rows: row out of range");
    if (nrows == 0) return;
    DevBuf<int32_t> rows;
    rows.alloc(nrows);
    TDBEM_HIP(hipMemcpyAsync(rows.p, host_rows, nrows * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    launch_direct_rows(ctx, nrows, rows.p, alpha, dev_out);
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  });
}

static void prof_collect(tdbem_ctx* ctx) {
  if (!ctx->prof_ev.empty()) TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  for (auto& e : ctx->prof_ev) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.second.first, e.second.second) == hipSuccess) {
      ctx->prof_ms[e.first] += ms;
      ctx->prof_cnt[e.first] += 1;
    }
    ctx->ev_pool.push_back(e.second.first);
    ctx->ev_pool.push_back(e.second.second);
  }
  ctx->prof_ev.clear();
}

int tdbem_profile(tdbem_ctx* ctx, int enable) {
  if (!ctx) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    prof_collect(ctx);
    for (int k = 0; k < 16; ++k) { ctx->prof_ms[k] = 0.0; ctx->prof_cnt[k] = 0; }
    ctx->prof = enable != 0;
    ctx->prof_mask = 0xffffffffu;
  });
}

int tdbem_profile_mask(tdbem_ctx* ctx, unsigned mask) {
  if (!ctx) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    prof_collect(ctx);
    for (int k = 0; k < 16; ++k) { ctx->prof_ms[k] = 0.0; ctx->prof_cnt[k] = 0; }
    ctx->prof = mask != 0;
    ctx->prof_mask = mask;
  });
}

int tdbem_set_m2l_variant(tdbem_ctx* ctx, int n, int choice) {
  if (!ctx || !ctx->fmm) return TDBEM_E_INVAL;
  const int rc = fmm_set_m2l_variant(ctx, n, choice);
  if (rc == TDBEM_OK) invalidate_graph(ctx);
  return rc;
}

int tdbem_profile_read(tdbem_ctx* ctx, double* ms, int64_t* launches, int n) {
  if (!ctx || n < 0 || n > 16) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    prof_collect(ctx);
    for (int k = 0; k < n; ++k) {
      if (ms) ms[k] = ctx->prof_ms[k];
      if (launches) launches[k] = ctx->prof_cnt[k];
    }
  });
}

void tdbem_destroy(tdbem_ctx* ctx) {
  if (!ctx) return;
  for (auto& e : ctx->prof_ev) { (void)hipEventDestroy(e.second.first); (void)hipEventDestroy(e.second.second); }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->fmm) fmm_destroy(ctx->fmm);
  if (ctx->g_exec) (void)hipGraphExecDestroy(ctx->g_exec);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
}

const char* tdbem_last_error(const tdbem_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int tdbem_get_info(const tdbem_ctx* ctx, tdbem_info* info) {
  if (!ctx || !info) return TDBEM_E_INVAL;
  std::memset(info, 0, sizeof(*info));
  info->ns = ctx->ns;
  info->d = ctx->d;
  info->bie = ctx->bie;
  info->bc = ctx->bc;
  info->c = ctx->c;
  info->dt = ctx->dt;
  info->use_fmm = ctx->opts.use_fmm;
  info->near_pairs = ctx->npairs;
  info->near_coefs = ctx->ncoef;
  info->a_nnz = ctx->a_nnz;
  info->setup_ms = ctx->setup_ms;
  info->gmres_workgroups = ctx->gmres_wg;
  if (ctx->fmm) fmm_info(ctx, info);
  return TDBEM_OK;
}

int tdbem_reset(tdbem_ctx* ctx) {
  if (!ctx) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    TDBEM_HIP(hipMemsetAsync(ctx->d_hu.p, 0, ctx->d_hu.n * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_hq.p, 0, ctx->d_hq.n * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_x.p, 0, ctx->ns * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_stat.p, 0, ctx->nt_max * sizeof(StepStat), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_growth_ref.p, 0, sizeof(double), ctx->stream));
    ctx->alpha = 1;
    ctx->hist_u = ctx->hist_q = false;
    if (ctx->fmm) fmm_reset(ctx);
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tdbem_set_history(tdbem_ctx* ctx, int nsteps, const double* dev_u, const double* dev_q) {
  if (!ctx) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    if (nsteps < 0 || nsteps > ctx->nt_max - 1) fail(TDBEM_E_INVAL, "nsteps out of range");
    const size_t bytes = (size_t)nsteps * ctx->ns * sizeof(double);
    TDBEM_HIP(hipMemsetAsync(ctx->d_hu.p, 0, ctx->d_hu.n * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_hq.p, 0, ctx->d_hq.n * sizeof(double), ctx->stream));
    if (dev_u && bytes) TDBEM_HIP(hipMemcpyAsync(ctx->d_hu.p, dev_u, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    if (dev_q && bytes) TDBEM_HIP(hipMemcpyAsync(ctx->d_hq.p, dev_q, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    ctx->hist_u = dev_u != nullptr;
    ctx->hist_q = dev_q != nullptr;
    ctx->alpha = nsteps + 1;
    if (ctx->fmm) {
      fmm_reset(ctx);
      for (int beta = 0; beta < nsteps; ++beta) fmm_advance(ctx, beta);
    }
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tdbem_fmm_eval(tdbem_ctx* ctx, int alpha, double* dev_b_hist) {
  if (!ctx || !dev_b_hist) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    if (alpha < 1 || alpha > ctx->alpha || (ctx->fmm && alpha != ctx->alpha))
      fail(TDBEM_E_STATE, "alpha must be the current march position");
    launch_near_history(ctx, alpha, nullptr, dev_b_hist);
    if (ctx->fmm) fmm_far(ctx, alpha, dev_b_hist);
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tdbem_step(tdbem_ctx* ctx, const double* dev_forcing, const double* dev_bc_values, double* dev_x_out,
               tdbem_step_info* info) {
  if (!ctx) return TDBEM_E_INVAL;
  int rc = TDBEM_OK;
  int r = guarded(ctx, [&] {
    const int alpha = ctx->alpha;
    StepStat* st = ctx->d_stat.p + (alpha - 1);
    do_step(ctx, dev_forcing ? dev_forcing : ctx->d_zero.p, dev_bc_values, st);
    if (dev_x_out)
      TDBEM_HIP(hipMemcpyAsync(dev_x_out, ctx->d_x.p, ctx->ns * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
    StepStat hs;
    TDBEM_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, ctx->stream));
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
    if (info) {
      info->alpha = alpha;
      info->iters = hs.iters;
      info->resid = hs.resid;
    }
    if (hs.flags & 2) { ctx->err = "non-finite or exploding solution at step " + std::to_string(alpha); rc = TDBEM_E_DIVERGED; }
    else if (hs.flags & 16) { ctx->err = "solution grew beyond growth_limit at step " + std::to_string(alpha); rc = TDBEM_E_DIVERGED; }
    else if (hs.flags & 1) { ctx->err = "GMRES did not converge at step " + std::to_string(alpha); rc = TDBEM_E_NOT_CONVERGED; }
  });
  return r != TDBEM_OK ? r : rc;
}

int tdbem_run(tdbem_ctx* ctx, int nt, const double* dev_forcing, const tdbem_incident* inc, double* dev_x_hist_out,
              tdbem_run_info* info) {
  if (!ctx) return TDBEM_E_INVAL;
  int rc = TDBEM_OK;
  int r = guarded(ctx, [&] {
    const int a_first = ctx->alpha;
    const double* forc = run_prepare(ctx, nt, dev_forcing, inc);
    hipEvent_t e0, e1;
    TDBEM_HIP(hipEventCreate(&e0));
    TDBEM_HIP(hipEventCreate(&e1));
    TDBEM_HIP(hipEventRecord(e0, ctx->stream));
    run_launch(ctx, nt, forc);
    TDBEM_HIP(hipEventRecord(e1, ctx->stream));
    rc = run_finish(ctx, nt, a_first, dev_x_hist_out, info, e0, e1);
  });
  return r != TDBEM_OK ? r : rc;
}

int tdbem_run_batch(tdbem_ctx* const* ctxs, int n, const int* nt, const tdbem_incident* inc,
                    double* const* dev_x_hist_out, tdbem_run_info* info, double* wall_ms) {
  if (!ctxs || !nt || n < 0) { g_create_err = "run_batch: ctxs and nt are required"; return TDBEM_E_INVAL; }
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) { g_create_err = "run_batch: NULL context"; return TDBEM_E_INVAL; }
  std::vector<const double*> forc(n);
  std::vector<int> a_first(n);
  std::vector<hipEvent_t> e0(n, nullptr), e1(n, nullptr);
  std::vector<char> graphed(n, 0);
  int first_rc = TDBEM_OK;
  auto note = [&](int rc) { if (rc != TDBEM_OK && first_rc == TDBEM_OK) first_rc = rc; };
  // forcing and (host-side) graph capture before anything is timed
  for (int i = 0; i < n && first_rc == TDBEM_OK; ++i)
    note(guarded(ctxs[i], [&] {
      a_first[i] = ctxs[i]->alpha;
      forc[i] = run_prepare(ctxs[i], nt[i], nullptr, inc ? &inc[i] : nullptr);
      TDBEM_HIP(hipEventCreate(&e0[i]));
      TDBEM_HIP(hipEventCreate(&e1[i]));
      graphed[i] = use_graph(ctxs[i]);
      if (graphed[i]) ensure_graph(ctxs[i], nt[i], forc[i]);
    }));
  if (first_rc == TDBEM_OK) {
    for (int i = 0; i < n; ++i) TDBEM_HIP_NOTHROW(hipStreamSynchronize(ctxs[i]->stream));
    const auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < n; ++i)
      note(guarded(ctxs[i], [&] {
        TDBEM_HIP(hipEventRecord(e0[i], ctxs[i]->stream));
        if (graphed[i]) run_launch(ctxs[i], nt[i], forc[i]);
      }));
    // contexts without a graph: one step of each in turn; FMM contexts that agree on the
    // launch shape share one M2L launch per step (on a stream of the batch, joined to and
    // from the contexts' streams by events)
    int amax = 0;
    for (int i = 0; i < n; ++i) amax = std::max(amax, nt[i] - 1);
    std::vector<tdbem_ctx*> lock;
    std::vector<int> lock_idx;
    for (int i = 0; i < n; ++i)
      if (!graphed[i] && ctxs[i]->fmm) { lock.push_back(ctxs[i]); lock_idx.push_back(i); }
    FmmBatch* fb = nullptr;
    if (lock.size() >= 2) {
      try {
        fb = fmm_batch_create(lock.data(), (int)lock.size());
      } catch (const Error&) {
        fb = nullptr;  // different launch shapes: each context launches its own products
      }
    }
    hipStream_t bst = nullptr;
    std::vector<hipEvent_t> ev_pre;
    hipEvent_t ev_m2l = nullptr;
    if (fb) {
      note(guarded(lock[0], [&] {
        TDBEM_HIP(hipStreamCreateWithFlags(&bst, hipStreamNonBlocking));
        TDBEM_HIP(hipEventCreateWithFlags(&ev_m2l, hipEventDisableTiming));
        ev_pre.assign(lock.size(), nullptr);
        for (auto& e : ev_pre) TDBEM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      }));
    }
    std::vector<int> ndue(lock.size(), 0);
    for (int alpha = 1; alpha <= amax && first_rc == TDBEM_OK; ++alpha) {
      for (int i = 0; i < n; ++i) {
        tdbem_ctx* c = ctxs[i];
        if (graphed[i] || c->alpha != alpha || alpha > nt[i] - 1) continue;
        if (fb && c->fmm) continue;  // stepped below
        note(guarded(c, [&] {
          do_step(c, forc[i] ? forc[i] + (size_t)(alpha - 1) * c->ns : c->d_zero.p, nullptr, c->d_stat.p + (alpha - 1));
        }));
      }
      if (!fb) continue;
      bool any = false;
      for (size_t j = 0; j < lock.size(); ++j) {
        tdbem_ctx* c = lock[j];
        const int i = lock_idx[j];
        ndue[j] = 0;
        if (c->alpha != alpha || alpha > nt[i] - 1) continue;
        note(guarded(c, [&] {
          ndue[j] = do_step(c, forc[i] ? forc[i] + (size_t)(alpha - 1) * c->ns : c->d_zero.p, nullptr,
                            c->d_stat.p + (alpha - 1), true);
          TDBEM_HIP(hipEventRecord(ev_pre[j], c->stream));
          TDBEM_HIP(hipStreamWaitEvent(bst, ev_pre[j], 0));
          // the separable products on the context's stream, beside the batch's dense products
          if (ndue[j] > 0) fmm_advance_sep(c, alpha - 1, ndue[j], c->stream);
        }));
        any = true;
      }
      if (!any || first_rc != TDBEM_OK) continue;
      note(guarded(lock[0], [&] {
        fmm_batch_m2l(fb, ndue.data(), bst);
        TDBEM_HIP(hipEventRecord(ev_m2l, bst));
      }));
      for (size_t j = 0; j < lock.size(); ++j) {
        tdbem_ctx* c = lock[j];
        const int i = lock_idx[j];
        if (c->alpha != alpha + 1 || alpha > nt[i] - 1) continue;  // stepped at this alpha
        note(guarded(c, [&] {
          TDBEM_HIP(hipStreamWaitEvent(c->stream, ev_m2l, 0));
          fmm_advance_post(c, alpha - 1, ndue[j]);
        }));
      }
    }
    if (fb) {
      if (bst) TDBEM_HIP_NOTHROW(hipStreamSynchronize(bst));
      for (auto& e : ev_pre) if (e) (void)hipEventDestroy(e);
      if (ev_m2l) (void)hipEventDestroy(ev_m2l);
      if (bst) (void)hipStreamDestroy(bst);
      fmm_batch_destroy(fb);
    }
    for (int i = 0; i < n; ++i) note(guarded(ctxs[i], [&] { TDBEM_HIP(hipEventRecord(e1[i], ctxs[i]->stream)); }));
    for (int i = 0; i < n; ++i) TDBEM_HIP_NOTHROW(hipStreamSynchronize(ctxs[i]->stream));
    if (wall_ms) *wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < n; ++i) {
      int rc = TDBEM_OK;
      note(guarded(ctxs[i], [&] {
        rc = run_finish(ctxs[i], nt[i], a_first[i], dev_x_hist_out ? dev_x_hist_out[i] : nullptr,
                        info ? &info[i] : nullptr, e0[i], e1[i]);
        e0[i] = e1[i] = nullptr;
      }));
      note(rc);
    }
  }
  for (int i = 0; i < n; ++i) {
    if (e0[i]) (void)hipEventDestroy(e0[i]);
    if (e1[i]) (void)hipEventDestroy(e1[i]);
  }
  return first_rc;
}

// Checkpoint layout: header, then u rows 0..alpha-2, q rows 0..alpha-2, the FMM
// state arrays in fmm_state_buffers order, then the network parameters if loaded.
struct CkptHeader {
  char magic[8];
  int32_t version, ns, d, bie, bc, use_fmm, depth, p_s, p_t, nstate;
  int32_t alpha, hist_u, hist_q, mlp;
  int64_t state_doubles;
  double c, dt;
  int32_t mu, m_leaf, m2l_prec, interp;
  uint64_t mesh_hash;  // FNV-1a over the face vertex coordinates in face order
  double leaf_ratio;   // the tree's sizing (0: bounding box)
};

static uint64_t mesh_hash(const tdbem_ctx* ctx) {
  uint64_t h = 1469598103934665603ull;
  const unsigned char* b = reinterpret_cast<const unsigned char*>(ctx->geo.tris.data());
  const size_t n = ctx->geo.tris.size() * sizeof(double);
  for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
  for (int8_t v : ctx->phi) { h ^= (unsigned char)v; h *= 1099511628211ull; }  // face types (mixed condition)
  return h;
}

static void ckpt_fill_config(const tdbem_ctx* ctx, CkptHeader& h) {
  h.ns = ctx->ns; h.d = ctx->d; h.bie = ctx->bie; h.bc = ctx->bc;
  h.use_fmm = ctx->fmm ? 1 : 0;

  h.p_s = ctx->fmm ? ctx->opts.p_s : 0;
  h.p_t = ctx->fmm ? ctx->opts.p_t : 0;
  h.c = ctx->c; h.dt = ctx->dt;
  tdbem_info info{};
  if (ctx->fmm) fmm_info(ctx, &info);
  h.mu = info.mu; h.m_leaf = info.m_leaf;
  h.depth = ctx->fmm ? info.depth : 0;  // the tree's depth (set by leaf_ratio when that is > 0)
  h.leaf_ratio = ctx->fmm ? ctx->opts.leaf_ratio : 0.0;
  h.m2l_prec = ctx->fmm ? ctx->opts.m2l_prec : 0;
  h.interp = ctx->fmm ? ctx->opts.interp : 0;  // moments and locals are coefficients of this basis
  h.mesh_hash = mesh_hash(ctx);
}

static size_t ckpt_bytes(const tdbem_ctx* ctx, const std::vector<std::pair<double*, size_t>>& st) {
  size_t n = sizeof(CkptHeader) + (size_t)2 * (ctx->alpha - 1) * ctx->ns * sizeof(double);
  for (const auto& b : st) n += b.second * sizeof(double);
  if (ctx->mlp_loaded) n += (size_t)TDBEM_MLP_NPARAM * sizeof(float);
  return n;
}

int tdbem_checkpoint(tdbem_ctx* ctx, void* host_buf, size_t* bytes) {
  if (!ctx || !bytes) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    std::vector<std::pair<double*, size_t>> st;
    if (ctx->fmm) fmm_state_buffers(ctx, st);
    const size_t need = ckpt_bytes(ctx, st);
    if (!host_buf) { *bytes = need; return; }
    if (*bytes < need) {
      *bytes = need;
      fail(TDBEM_E_INVAL, "checkpoint buffer too small (" + std::to_string(need) + " bytes needed)");
    }
    CkptHeader h{};
    std::memcpy(h.magic, "TDBEMCK1", 8);
    h.version = 3;
    ckpt_fill_config(ctx, h);
    h.nstate = (int32_t)st.size();
    h.alpha = ctx->alpha; h.hist_u = ctx->hist_u; h.hist_q = ctx->hist_q; h.mlp = ctx->mlp_loaded;
    for (const auto& b : st) h.state_doubles += (int64_t)b.second;
    char* p = static_cast<char*>(host_buf);
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    const size_t rows = (size_t)(ctx->alpha - 1) * ctx->ns * sizeof(double);
    if (rows) {
      TDBEM_HIP(hipMemcpyAsync(p, ctx->d_hu.p, rows, hipMemcpyDeviceToHost, ctx->stream));
      p += rows;
      TDBEM_HIP(hipMemcpyAsync(p, ctx->d_hq.p, rows, hipMemcpyDeviceToHost, ctx->stream));
      p += rows;
    }
    for (const auto& b : st) {
      TDBEM_HIP(hipMemcpyAsync(p, b.first, b.second * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      p += b.second * sizeof(double);
    }
    if (ctx->mlp_loaded)
      TDBEM_HIP(hipMemcpyAsync(p, ctx->d_mlp_params.p, TDBEM_MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                               ctx->stream));
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
    *bytes = need;
  });
}

int tdbem_restore(tdbem_ctx* ctx, const void* host_buf, size_t bytes) {
  if (!ctx || !host_buf) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    if (bytes < sizeof(CkptHeader)) fail(TDBEM_E_INVAL, "restore: buffer smaller than a checkpoint header");
    CkptHeader h;
    std::memcpy(&h, host_buf, sizeof(h));
    if (std::memcmp(h.magic, "TDBEMCK1", 8) != 0 || h.version != 3) fail(TDBEM_E_INVAL, "restore: not a checkpoint");
    std::vector<std::pair<double*, size_t>> st;
    if (ctx->fmm) fmm_state_buffers(ctx, st);
    int64_t sd = 0;
    for (const auto& b : st) sd += (int64_t)b.second;
    CkptHeader mine{};
    ckpt_fill_config(ctx, mine);
    if (h.ns != mine.ns || h.d != mine.d || h.bie != mine.bie || h.bc != mine.bc || h.use_fmm != mine.use_fmm ||
        h.depth != mine.depth || h.p_s != mine.p_s || h.p_t != mine.p_t || h.mu != mine.mu ||
        h.m_leaf != mine.m_leaf || h.m2l_prec != mine.m2l_prec || h.interp != mine.interp || h.c != mine.c ||
        h.leaf_ratio != mine.leaf_ratio ||
        h.dt != mine.dt || h.nstate != (int32_t)st.size() || h.state_doubles != sd)
      fail(TDBEM_E_INVAL, "restore: checkpoint was taken on a context with a different configuration");
    if (h.mesh_hash != mine.mesh_hash) fail(TDBEM_E_INVAL, "restore: checkpoint was taken on a different mesh");
    if (h.alpha < 1 || h.alpha > ctx->nt_max) fail(TDBEM_E_INVAL, "restore: step beyond this context's nt_max");
    const size_t rows = (size_t)(h.alpha - 1) * ctx->ns * sizeof(double);
    size_t need = sizeof(CkptHeader) + 2 * rows + (size_t)sd * sizeof(double) +
                  (h.mlp ? (size_t)TDBEM_MLP_NPARAM * sizeof(float) : 0);
    if (bytes < need) fail(TDBEM_E_INVAL, "restore: truncated checkpoint");
    const char* p = static_cast<const char*>(host_buf) + sizeof(CkptHeader);
    TDBEM_HIP(hipMemsetAsync(ctx->d_hu.p, 0, ctx->d_hu.n * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_hq.p, 0, ctx->d_hq.n * sizeof(double), ctx->stream));
    if (rows) {
      TDBEM_HIP(hipMemcpyAsync(ctx->d_hu.p, p, rows, hipMemcpyHostToDevice, ctx->stream));
      p += rows;
      TDBEM_HIP(hipMemcpyAsync(ctx->d_hq.p, p, rows, hipMemcpyHostToDevice, ctx->stream));
      p += rows;
    }
    for (const auto& b : st) {
      TDBEM_HIP(hipMemcpyAsync(b.first, p, b.second * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      p += b.second * sizeof(double);
    }
    invalidate_graph(ctx);
    if (h.mlp) {
      mlp_prepare(ctx);
      if (!ctx->d_mlp_params.p) ctx->d_mlp_params.alloc(TDBEM_MLP_NPARAM);
      TDBEM_HIP(hipMemcpyAsync(ctx->d_mlp_params.p, p, TDBEM_MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice,
                               ctx->stream));
      mlp_pack(ctx);
      ctx->mlp_loaded = true;
    }
    TDBEM_HIP(hipMemsetAsync(ctx->d_stat.p, 0, ctx->nt_max * sizeof(StepStat), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(ctx->d_growth_ref.p, 0, sizeof(double), ctx->stream));
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
    ctx->alpha = h.alpha;
    ctx->hist_u = h.hist_u != 0;
    ctx->hist_q = h.hist_q != 0;
  });
}

int tdbem_get_history(tdbem_ctx* ctx, int nsteps, double* dev_u, double* dev_q) {
  if (!ctx) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    if (nsteps < 0 || nsteps > ctx->nt_max) fail(TDBEM_E_INVAL, "nsteps out of range");
    const size_t bytes = (size_t)nsteps * ctx->ns * sizeof(double);
    if (dev_u && bytes) TDBEM_HIP(hipMemcpyAsync(dev_u, ctx->d_hu.p, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    if (dev_q && bytes) TDBEM_HIP(hipMemcpyAsync(dev_q, ctx->d_hq.p, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tdbem_incident_forcing(tdbem_ctx* ctx, const tdbem_incident* inc, int a0, int n, double* dev_out) {
  if (!ctx || !inc || !dev_out || n < 0) return TDBEM_E_INVAL;
  return guarded(ctx, [&] {
    launch_forcing(ctx, *inc, a0, n, dev_out);
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tdbem_near_row(tdbem_ctx* ctx, int i, int cap, int32_t* j_out, int32_t* g_out, double* cu_out, double* cw_out) {
  if (!ctx) return TDBEM_E_INVAL;
  int count = 0;
  int r = guarded(ctx, [&] {
    if (i < 0 || i >= ctx->ns) fail(TDBEM_E_INVAL, "row out of range");
    int64_t rp[2];
    TDBEM_HIP(hipMemcpy(rp, ctx->d_row_ptr.p + i, 2 * sizeof(int64_t), hipMemcpyDeviceToHost));
    const int64_t np = rp[1] - rp[0];
    std::vector<int32_t> pj(np), gw(np);
    std::vector<int64_t> off(np);
    TDBEM_HIP(hipMemcpy(pj.data(), ctx->d_pair_j.p + rp[0], np * sizeof(int32_t), hipMemcpyDeviceToHost));
    TDBEM_HIP(hipMemcpy(gw.data(), ctx->d_pair_gw.p + rp[0], np * sizeof(int32_t), hipMemcpyDeviceToHost));
    TDBEM_HIP(hipMemcpy(off.data(), ctx->d_pair_off.p + rp[0], np * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < np; ++p) {
      const int glo = gw[p] >> 16, cnt = gw[p] & 0xffff;
      std::vector<double> cu(cnt), cw(cnt);
      if (ctx->opts.near_prec == 1) {
        std::vector<float> fu(cnt), fw(cnt);
        TDBEM_HIP(hipMemcpy(fu.data(), ctx->d_cu32.p + off[p], cnt * sizeof(float), hipMemcpyDeviceToHost));
        TDBEM_HIP(hipMemcpy(fw.data(), ctx->d_cw32.p + off[p], cnt * sizeof(float), hipMemcpyDeviceToHost));
        for (int k = 0; k < cnt; ++k) { cu[k] = fu[k]; cw[k] = fw[k]; }
      } else {
        TDBEM_HIP(hipMemcpy(cu.data(), ctx->d_cu.p + off[p], cnt * sizeof(double), hipMemcpyDeviceToHost));
        TDBEM_HIP(hipMemcpy(cw.data(), ctx->d_cw.p + off[p], cnt * sizeof(double), hipMemcpyDeviceToHost));
      }
      for (int k = 0; k < cnt; ++k) {
        if (count < cap) {
          if (j_out) j_out[count] = pj[p];
          if (g_out) g_out[count] = glo + k;
          if (cu_out) cu_out[count] = cu[k];
          if (cw_out) cw_out[count] = cw[k];
        }
        ++count;
      }
    }
  });
  return r != TDBEM_OK ? r : count;
}

}  // extern "C"
