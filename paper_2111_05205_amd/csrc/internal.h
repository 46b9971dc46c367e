// Internal declarations of the MI355X time-domain BEM library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tdbem.h"
#include "elemint_gl.h"

#define TDBEM_HIP(call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      throw tdbem::Error(TDBEM_E_DEVICE, std::string(#call) + ": " +           \
                                             hipGetErrorString(e_));           \
    }                                                                          \
  } while (0)

namespace tdbem {

struct Error {
  int code;
  std::string msg;
  Error(int c, std::string m) : code(c), msg(std::move(m)) {}
};

// Device buffer owned by a context.
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    release();
    n = count;
    if (count == 0) return;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
      p = nullptr;
      n = 0;
      throw Error(TDBEM_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  ~DevBuf() { release(); }
};

// Per-step record kept on the device during a march.
struct StepStat {
  int iters;
  int flags;    // bit0: not converged, bit1: non-finite, bit2/3: starting point rejected/replaced, bit4: growth
  double resid;
  double xmax;  // max_i |x_i| of the step (reset by the solve, raised by the store)
};

struct Fmm;  // space-time FMM state (fmm.hip)

// B-spline weights w^{kappa,d} (eq. w), d <= 4.
struct BWeights { double w[6]; int d; };

struct Geometry {
  int ns = 0;
  std::vector<double> xc;    // ns x 3 collocation points (centroids)
  std::vector<double> nrm;   // ns x 3 paper normals (into the scatterer)
  std::vector<double> tris;  // ns x 9 vertex coordinates
  std::vector<double> area;
  double edge_max = 0.0, edge_mean = 0.0;
  double ext_lo[3], ext_hi[3];  // vertex bounding box
  double e_max = 0.0;           // largest centroid-to-vertex distance
};

}  // namespace tdbem

struct tdbem_ctx {
  std::string err;
  hipStream_t stream = nullptr;
  int ns = 0, d = 1, bie = 1, bc = 0;
  double c = 1.0, dt = 1.0, cdt = 1.0;
  tdbem_opts opts{};
  tdbem::BWeights bw{};
  tdbem::Geometry geo;
  double setup_ms = 0.0;

  // device geometry
  tdbem::DevBuf<double> d_xc, d_nrm, d_tris;

  // near-field table, CSR by collocation row i
  int64_t npairs = 0, ncoef = 0;
  tdbem::DevBuf<int64_t> d_row_ptr;    // ns+1
  tdbem::DevBuf<int32_t> d_pair_j;     // npairs
  tdbem::DevBuf<int32_t> d_pair_gw;    // npairs: (glo << 16) | cnt
  tdbem::DevBuf<int64_t> d_pair_off;   // npairs: first coefficient
  tdbem::DevBuf<double> d_cu, d_cw;    // ncoef each: compact C_U^{(g)}, C_W^{(g)} (raw X^{(gamma)} for the tau form)
  tdbem::DevBuf<float> d_cu32, d_cw32; // the same rounded to FP32 (opts.near_prec = 1; the FP64 arrays are released)

  // per-step matrix A and the g=1 blocks, CSR
  int64_t a_nnz = 0;
  tdbem::DevBuf<int32_t> d_a_ptr, d_a_col;
  tdbem::DevBuf<double> d_a_val, d_u1_val, d_w1_val;
  // the per-step matrix again for the solver, padded to ell_w entries per row and
  // stored column-major ([k][row]; padding: column = row, value = 0)
  int ell_w = 0;
  tdbem::DevBuf<int32_t> d_ell_col;
  tdbem::DevBuf<double> d_ell_val;

  // mixed boundary condition (bc == TDBEM_MIXED): phi_j = 1 where q is given and u unknown, 0 where u is given
  tdbem::DevBuf<int8_t> d_phi;
  std::vector<int8_t> phi;

  // history [beta][element], beta = 0..nt_max-2
  int nt_max = 0;
  tdbem::DevBuf<double> d_hu, d_hq;
  int alpha = 1;        // next collocation step
  bool hist_u = false;  // any non-zero u stored
  bool hist_q = false;  // any non-zero q stored

  // work
  tdbem::DevBuf<double> d_b, d_x, d_V, d_forc, d_zero, d_gpart;
  int gmres_wg = 1;  // workgroups of the per-step solve (1: single-workgroup kernel)
  tdbem::DevBuf<tdbem::StepStat> d_stat;
  tdbem::DevBuf<double> d_growth_ref;  // largest max|x| of the rows up to beta - growth_lag (growth check)

  tdbem::Fmm* fmm = nullptr;

  // learned initial guess
  bool mlp_loaded = false;
  tdbem::DevBuf<float> d_mlp_params;   // packed FP32 parameters
  tdbem::DevBuf<uint16_t> d_mlp_wpk;   // hidden-layer weights as bf16 matrix-core fragments (march forward)
  tdbem::DevBuf<float> d_mlp_feat, d_mlp_y;
  tdbem::DevBuf<double> d_x_alt;       // extrapolated starting point offered beside the network's
  tdbem::DevBuf<double> d_mlp_diag, d_mlp_s, d_area;
  double mlp_geo[5] = {0, 0, 0, 0, 0};  // 1/h^2, bounding-box centre (3), 1/R
  float* rec_feat = nullptr;           // caller-owned training records (tdbem_mlp_record)
  float* rec_target = nullptr;

  // captured march (opts.graph): replayed by later runs with the same nt and forcing
  hipStream_t cap_stream = nullptr;  // non-blocking stream used only while capturing
  bool capturing = false;
  hipGraphExec_t g_exec = nullptr;
  int g_nt = 0;
  const double* g_forc = nullptr;
  int g_alpha = 1;
  bool g_hu = false, g_hq = false;

  // kernel timing (tdbem_profile)
  bool prof = false;
  uint32_t prof_mask = 0xffffffffu;  // categories bracketed while profiling
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_ev;
  std::vector<hipEvent_t> ev_pool;  // events of collected brackets, reused (created once, destroyed with the context)
  double prof_ms[16] = {0};
  int64_t prof_cnt[16] = {0};
};

namespace tdbem {

enum ProfKind { K_NEAR = 0, K_GMRES = 1, K_L2P = 2, K_P2M = 3, K_M2L_GEMM = 4, K_M2L_RED = 5, K_M2M = 6, K_L2L = 7,
                K_OTHER = 8, K_MLP = 9, K_M2L_DERIV = 10 };

// Brackets the launches in its scope with events when profiling is enabled.
struct ProfScope {
  tdbem_ctx* c;
  int kind;
  hipStream_t s;  // the stream the bracketed launches go to (default: the context's)
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(tdbem_ctx* ctx, int k, hipStream_t stream = nullptr) : c(ctx), kind(k), s(stream ? stream : ctx->stream) {
    if (c->prof && ((c->prof_mask >> k) & 1u) && take(e0) && take(e1)) (void)hipEventRecord(e0, s);
  }
  bool take(hipEvent_t& e) {
    if (!c->ev_pool.empty()) {
      e = c->ev_pool.back();
      c->ev_pool.pop_back();
      return true;
    }
    return hipEventCreate(&e) == hipSuccess;
  }
  ~ProfScope() {
    if (c->prof && e0 && e1) {
      (void)hipEventRecord(e1, s);
      c->prof_ev.push_back({kind, {e0, e1}});
    }
  }
};

// nearfield.hip
void build_near_table(tdbem_ctx* ctx, const std::vector<int64_t>& row_ptr, const std::vector<int32_t>& pair_j);
void build_step_matrix(tdbem_ctx* ctx);
void launch_near_history(tdbem_ctx* ctx, int alpha, const double* base, double* out);
void near_table_to_fp32(tdbem_ctx* ctx);
void launch_spmv_add(tdbem_ctx* ctx, const double* vals, double scale, const double* xin, double* y);
// y += scale * vals x restricted to the columns j with phi_j == want
void launch_spmv_add_masked(tdbem_ctx* ctx, const double* vals, double scale, const double* xin, int want, double* y);
// scattered field at npts device points (3 each) at t_alpha from the stored history
void launch_field(tdbem_ctx* ctx, int npts, const double* pts, int alpha, double* out);
// exact (direct, every element) history part of b^{alpha-1} at nrows device row indices
void launch_direct_rows(tdbem_ctx* ctx, int nrows, const int32_t* rows, int alpha, double* out);
void upload_gl_rule();

// gmres.hip
// xalt: NULL or a second starting point; the solve starts from whichever of x,
// xalt has the smaller residual (from zero when both are worse than zero)
void launch_gmres(tdbem_ctx* ctx, const double* b, double* x, StepStat* stat, const double* xalt = nullptr);
int gmres_workgroups(int ns);
void autotune_gmres(tdbem_ctx* ctx);  // pick the solver's workgroup count by timing (Ns > 2048)

// api.hip
void set_global_error(const std::string& msg);  // message for tdbem_last_error(NULL)
void launch_forcing(tdbem_ctx* ctx, const tdbem_incident& inc, int a0, int n, double* out);

// the captured march (if any) refers to buffers and choices that are about to
// change: drop it so the next graph run records the march again
void invalidate_graph(tdbem_ctx* ctx);

// mlp.hip
void mlp_prepare(tdbem_ctx* ctx);  // per-context buffers of the guess (diagonal of A, areas)
void mlp_pack(tdbem_ctx* ctx);     // refresh d_mlp_wpk from d_mlp_params (stream-ordered)
// features of unknown row beta (>= 4) from the stored history and b into feat (Ns x 16); scale into d_mlp_s
void launch_mlp_features(tdbem_ctx* ctx, int beta, const double* b, float* feat);
// x = quadratic extrapolation of the last three rows + s * network(feat); xe = the extrapolation
void launch_mlp_guess(tdbem_ctx* ctx, int beta, const float* feat, double* x, double* xe);
// training target of row beta (after it has been stored)
void launch_mlp_target(tdbem_ctx* ctx, int beta, float* target);

// fmm.hip
Fmm* fmm_create(tdbem_ctx* ctx);
void fmm_destroy(Fmm* f);
void fmm_reset(tdbem_ctx* ctx);
// add the far field at target step alpha to out (Ns)
void fmm_far(tdbem_ctx* ctx, int alpha, double* out);
// the coefficient row beta has been stored: update moments and run interval-end translations
void fmm_advance(tdbem_ctx* ctx, int beta);
// the same in three parts: P2M and M2M (returns the number of levels whose interval ends),
// their M2L launch (fmm_advance or fmm_batch_m2l), then everything after the products
int fmm_advance_pre(tdbem_ctx* ctx, int beta);
void fmm_advance_sep(tdbem_ctx* ctx, int beta, int ndue, hipStream_t st);  // separable products, beside the M2L
void fmm_advance_post(tdbem_ctx* ctx, int beta, int ndue);
// contexts marching in lock step with one M2L launch per step for all of them (equal P,
// mu, precision and M_leaf; fmm_batch_create throws otherwise)
struct FmmBatch;
FmmBatch* fmm_batch_create(tdbem_ctx* const* ctxs, int n);
void fmm_batch_destroy(FmmBatch* b);
// the products of ndue[i] levels of context i (0: none) in one launch on st
void fmm_batch_m2l(FmmBatch* b, const int* ndue, hipStream_t st);
void fmm_info(const tdbem_ctx* ctx, tdbem_info* info);
int fmm_set_m2l_variant(tdbem_ctx* ctx, int n, int choice);
void fmm_near_pairs(const tdbem_ctx* ctx, std::vector<int64_t>& row_ptr, std::vector<int32_t>& pair_j);
// device arrays that carry FMM state from one step to the next (moments, locals, recurrence terms)
void fmm_state_buffers(const tdbem_ctx* ctx, std::vector<std::pair<double*, size_t>>& out);

}  // namespace tdbem
