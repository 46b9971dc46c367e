/*
 * tdbem.h — C ABI of the MI355X time-domain boundary element library.
 *
 * The library solves the exterior initial-boundary value problem of the 3-D
 * wave equation (paper: Section 2.1, eq. ibvp) on a closed surface of flat
 * triangles with piecewise-constant densities in space and a uniform B-spline
 * basis of order d in time (Section 2.3, eqs. u_bspline, decompose, w), by
 * collocation at face centroids and times t_alpha = alpha*dt, alpha = 1..Nt-1.
 * Either the ordinary BIE (eq. bie) or the Burton-Miller BIE (eq. bmbie, with
 * the matrices of eq. U_W_BM) is marched in time (eq. linear).  The history
 * part of the right-hand side is evaluated directly for near pairs (eq.
 * linear, compact B-spline form) and, when enabled, by the interpolation-based
 * space-time FMM for far pairs (Section 3, eqs. target, U_intp, m2l; Section 4,
 * Formula 1 and Algorithm 1).
 *
 * Conventions
 *  - Status: every int-returning call returns TDBEM_OK (0) or a negative
 *    TDBEM_E_* code; tdbem_last_error() then holds a message for that context.
 *  - Pointers named dev_* are HIP device pointers (e.g. torch.Tensor.data_ptr())
 *    that must stay valid until the call returns; the library works on the
 *    HIP stream given at creation and synchronises that stream before
 *    returning from every call, so results are ready on return.
 *  - Host pointers (mesh arrays, info structs) are read or written only during
 *    the call.  The caller owns every buffer passed in; the library copies the
 *    mesh at creation and owns all device tables and the density history
 *    until tdbem_destroy().
 *  - Mesh orientation: triangles counter-clockwise seen from OUTSIDE the
 *    scatterer.  Internally the paper's normal n points into the scatterer
 *    (this makes the free term part of the double layer, Section 2.4), so
 *    q = du/dn is reported with that inward n.
 *  - Array layouts are row-major; time-by-element arrays are [step][element].
 *  - One context per host thread; distinct contexts are independent.
 */
#ifndef TDBEM_H
#define TDBEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque handle of one solver instance (created by tdbem_create, freed by tdbem_destroy). */
struct tdbem_ctx;

enum {
  TDBEM_OK = 0,
  TDBEM_E_INVAL = -1,         /* bad argument or mesh */
  TDBEM_E_NOMEM = -2,         /* device allocation failed */
  TDBEM_E_DEVICE = -3,        /* HIP runtime error */
  TDBEM_E_NOT_CONVERGED = -4, /* per-step GMRES did not reach its tolerance */
  TDBEM_E_DIVERGED = -5,      /* non-finite or exploding solution, or growth beyond opts.growth_limit */
  TDBEM_E_STATE = -6          /* call out of order (e.g. step beyond nt_max) */
};

typedef enum { TDBEM_OBIE = 0, TDBEM_BMBIE = 1 } tdbem_bie;          /* eq. bie / eq. bmbie */
/* u given (q unknown) / q given (u unknown) on every face; MIXED: per face, see tdbem_create_mixed */
typedef enum { TDBEM_DIRICHLET = 0, TDBEM_NEUMANN = 1, TDBEM_MIXED = 2 } tdbem_bc;
/* Precision of the near-future M2L products (Section 4, eq. m2l_near, blocks
 * l = 1..mu+1): FP64, FP32, or BF16 operators and moments (rounded to nearest)
 * on the BF16 matrix cores, or BF16X3: each factor split as x = hi + lo with hi,
 * lo in bf16 (lo the rounded remainder), products hi*hi + hi*lo + lo*hi on the
 * BF16 matrix cores (the lo*lo term, ~2^-16 of the product, is dropped; the same
 * bytes as FP32).  All but FP64 accumulate in FP32.  The derivative products
 * U^{(p)} M (eq. L_l,k), which feed the recurrence of Formula 1 over every later
 * interval, are FP64 in every case (evaluated exactly through the separable form of
 * U^{(p)}); moments, locals, recurrence, near field and solve are FP64. */
typedef enum { TDBEM_M2L_FP64 = 0, TDBEM_M2L_FP32 = 1, TDBEM_M2L_BF16 = 2, TDBEM_M2L_BF16X3 = 3 } tdbem_m2l_prec;
typedef enum { TDBEM_INC_GAUSS_MOD = 0, TDBEM_INC_RAISED_COS = 1 } tdbem_inc_kind;
/* Starting point of the per-step GMRES solve (the paper names no solver):
 * EXTRAP quadratic extrapolation of the last three solved rows (default),
 * ZERO, PREV the previous row, MLP the learned guess (tdbem_mlp_load; falls
 * back to EXTRAP for the first four rows or when no network is loaded).  With
 * MLP the solve computes the residuals of the network's proposal and of the
 * extrapolation and starts from the smaller; any starting point whose residual
 * exceeds |b| is replaced by zero. */
/* MLP_ONLY starts from the network's proposal alone (no comparison with the
 * extrapolation; still zero when the proposal's residual exceeds |b|): the
 * mode that measures what the network itself predicts. */
typedef enum { TDBEM_GUESS_EXTRAP = 0, TDBEM_GUESS_ZERO = 1, TDBEM_GUESS_PREV = 2, TDBEM_GUESS_MLP = 3,
               TDBEM_GUESS_MLP_ONLY = 4 } tdbem_guess;

typedef struct {
  int32_t nv, nt;        /* vertices, triangles */
  const double *xyz;     /* host, nv x 3 */
  const int32_t *tri;    /* host, nt x 3, CCW seen from outside */
} tdbem_mesh;

typedef struct {
  int use_fmm;       /* 0: every pair evaluated directly (near-field kernel); 1: FMM for far pairs */
  int depth;         /* octree depth: root level 0, leaves at level `depth` (FMM only, >= 2) */
  int p_s, p_t;      /* Chebyshev nodes per axis in space and in time (FMM only) */
  int mu;            /* near-future intervals (Section 4.2); 0 = smallest valid value */
  int m2l_prec;      /* tdbem_m2l_prec */
  double gmres_tol;  /* relative residual of the per-step solve (default 1e-12) */
  int gmres_restart; /* default 30 */
  int gmres_maxiter; /* default 300 */
  int nt_max;        /* largest Nt the context will march (sizes the history), default 4096 */
  int guess;         /* tdbem_guess */
  int graph;         /* 1: tdbem_run from a reset context captures the whole march into a HIP graph once and
                        replays it on later runs with the same nt and forcing (per-step solves then use the
                        single-workgroup GMRES kernel; profiling and training records run without the graph) */
  int near_form;     /* near-field history sum: 0 compact coefficients C^{(g)} = sum_kappa w^kappa X^{(g-kappa)}
                        (default); 1 the tau/sigma form of eq. linear: raw X^{(gamma)} times
                        tau = sum_kappa w^kappa q (sigma likewise), truncated at each pair's last gap (App. A).
                        Equal in exact arithmetic; the kappa sum is taken in the coefficients (once, FP64) or in
                        the densities at every step (Section 5.1.3, cancellation of significant digits) */
  int near_prec;     /* 0: near-field coefficients stored in FP64 (default); 1: rounded to FP32 (study of that
                        cancellation; the sums stay FP64) */
  int interp;        /* FMM interpolation in each of the eight variables (eq. U_intp), tdbem_interp */
  double growth_limit; /* > 0: growth check of the march (the instability of Section 5.1 shows as a solution
                          that keeps growing after the incident pulse has passed): step beta fails with
                          TDBEM_E_DIVERGED when max_i |x_i^beta| exceeds growth_limit times the largest
                          max_i |x_i^gamma| over gamma <= beta - growth_lag; 0: off (only non-finite or
                          |x| > 1e100 fail) */
  int growth_lag;    /* steps between the checked row and the newest reference row (>= 1 when growth_limit > 0) */
  double leaf_ratio; /* > 0 (FMM): normalised operators.  The octree's leaf side is leaf_ratio * c * dt (the
                        depth follows from the mesh extent and opts.depth is ignored) and the dense near-future
                        M2L operators are formed in units of c*dt and dt.  U of eq. Uabmn is homogeneous of
                        degree d-1 in (x, c t), so in these units a level's operators depend only on its
                        distance from the leaves: contexts on one device with equal leaf_ratio, M_leaf, mu, d,
                        p_s, p_t, interp and m2l_prec share them (process-wide, held while any such context
                        lives), and each context scales its products by (c dt)^(d-1).  0: per-context
                        operators in physical units (default) */
} tdbem_opts;

/* Interpolation functions l_a of eq. U_intp.  LAGRANGE: polynomials on the p Chebyshev
 * points of the first kind.  HERMITE: the paper's choice (Section 3, after eq. Uabmn):
 * piecewise cubic Hermite interpolation on p >= 3 equispaced nodes (both ends
 * included) whose nodal slopes are finite differences of the nodal values (central
 * inside, second-order one-sided at the ends; quadratics are reproduced), the end
 * pieces continued outside the node range. */
enum tdbem_interp { TDBEM_INTERP_LAGRANGE = 0, TDBEM_INTERP_HERMITE = 1 };

typedef struct {
  int kind;          /* tdbem_inc_kind */
  double dir[3];     /* propagation direction (normalised by the library) */
  double f0, sigma;  /* GAUSS_MOD: centre frequency and envelope width; RAISED_COS: sigma = pulse length */
  double t0, rb;     /* GAUSS_MOD: delay; both: phase offset rb (arrival shift along dir) */
} tdbem_incident;

typedef struct {
  int alpha;         /* collocation step just solved */
  int iters;         /* GMRES iterations */
  double resid;      /* final relative residual estimate */
} tdbem_step_info;

typedef struct {
  int steps;            /* solves performed (nt-1) */
  int total_iters;      /* GMRES iterations over the march */
  int max_iters;        /* largest per-step iteration count */
  double max_resid;     /* largest final relative residual */
  double march_ms;      /* wall time of the march on the context stream (HIP events) */
  int guesses_rejected; /* steps whose starting point had a larger residual than zero (solve started from 0) */
  int guesses_replaced; /* GUESS_MLP: steps where the extrapolation had the smaller residual and was used instead */
} tdbem_run_info;

typedef struct {
  int ns;               /* elements */
  int d, bie, bc;
  double c, dt;
  int use_fmm, depth, p_s, p_t, mu, m_leaf;
  int64_t near_pairs;   /* (i,j) pairs evaluated directly */
  int64_t near_coefs;   /* compact coefficients per family in the near table */
  int64_t a_nnz;        /* non-zeros of the per-step matrix */
  int64_t il_pairs[16]; /* interaction-list pairs per level (FMM) */
  int64_t m2l_matrix_bytes;
  double setup_ms;
  int m2l_variant[16];  /* [n], n = 1..depth-1: autotuned M2L launch for the n finest levels ending an interval
                           together, 2 * tile + persistent; tile (columns x K step x operator rows per
                           workgroup) 0 128x16x128, 1 64x16x128, 2 64x32x128, 3 32x16x128, 4 32x32x128,
                           5 32x16x256, 6 64x16x256, 7 32x32x256 (moment tile shared through LDS);
                           8 32x16x128, 9 32x16x256, 10 64x16x128, 11 64x16x256 (each lane reads its
                           moments directly, no LDS or barrier in the K loop); BF16 contexts use these
                           four shapes with K steps of 32, and 12 .. 15, the same four with the moment
                           fragments staged through LDS once per workgroup, 16 128x32x128 and
                           17 128x32x256 likewise */
  int gmres_workgroups; /* workgroups of the per-step solve (1: single-workgroup kernel; autotuned above 2048 faces) */
  int64_t m2l_dense_blocks[16]; /* per level: sum over interaction pairs of the near-future gaps evaluated as dense
                                   P x P products (the wavefront crosses the pair's node set there; the other gaps
                                   are zero at every node pair, or wavefront-free and evaluated in separable form) */
  int m2l_ops_users[16];        /* per level: live contexts that use this level's dense operator set (1: its own;
                                   more: shared normalised operators, opts.leaf_ratio) */
} tdbem_info;

/* Build a context: copies and validates the mesh (closed, consistently
 * oriented, non-degenerate), precomputes the near-field compact coefficients
 * C^{(g)}_ij = sum_kappa w^kappa X^{(g-kappa)}_ij (App. A, App. B) in FP64 on the
 * device, the constant per-step matrix A (eq. linear), and with use_fmm the
 * octree, space-time hierarchy and M2L operators (Section 3, Remark precomp).
 * d in {1, 2, 3} (the paper finds d = 3 unstable).  c > 0, dt > 0.  hip_stream: hipStream_t or NULL (null stream).
 * opts NULL = defaults.  On success *out owns all device memory.
 * Errors: TDBEM_E_INVAL (bad argument or mesh), TDBEM_E_NOMEM, TDBEM_E_DEVICE. */
int tdbem_create(const tdbem_mesh *mesh, double c, double dt, int d, int bie, int bc,
                 const tdbem_opts *opts, void *hip_stream, struct tdbem_ctx **out);

/* tdbem_create for a mixed boundary condition (Section 2.1, eq. ibvp with both S_u and
 * S_q non-empty): face_bc (host, mesh->nt values) is phi_j of eq. linear, 1 where q is
 * given and u unknown, 0 where u is given and q unknown.  The per-step matrix takes
 * column j from the W family where phi_j = 1 and from -U where phi_j = 0; the
 * prescribed coefficients passed to tdbem_step (dev_bc_values) are q on phi = 1 faces
 * and u on phi = 0 faces; the solution rows (tdbem_step's dev_x_out, tdbem_run's
 * history) hold u on phi = 1 faces and q on phi = 0 faces.  The learned starting point
 * is not available (TDBEM_E_INVAL for guess MLP / MLP_ONLY).  tdbem_info.bc reports
 * TDBEM_MIXED.  Errors as tdbem_create, and TDBEM_E_INVAL for a NULL face_bc or values
 * other than 0 and 1. */
int tdbem_create_mixed(const tdbem_mesh *mesh, double c, double dt, int d, int bie, const int8_t *face_bc,
                       const tdbem_opts *opts, void *hip_stream, struct tdbem_ctx **out);

/* Field at points off the surface from the solved history (the Kirchhoff representation:
 * the single and double layer of eq. bie_disc, not their Burton-Miller combination,
 * evaluated at a point that is not a collocation point):
 *   dev_out[r] = sum_j sum_{g=1}^{alpha} (C_U^{(g)}(x_r, E_j) q_j^{alpha-g} - C_W^{(g)}(x_r, E_j) u_j^{alpha-g}),
 * compact coefficients C^{(g)} = sum_kappa w^kappa X^{(g-kappa)} at x_r.  Outside the
 * scatterer this is the scattered field at (x_r, t_alpha) (add u_in for the total field);
 * inside it equals -u_in (extinction).  Every element is summed directly (the FMM is not
 * used): O(npts Ns window) element integrals.  host_pts: npts x 3 host doubles, not on the
 * surface; 1 <= alpha <= (current position) - 1; dev_out: npts doubles. */
int tdbem_field(struct tdbem_ctx *ctx, int npts, const double *host_pts, int alpha, double *dev_out);

/* Exact history part of b^{alpha-1} (the quantity tdbem_fmm_eval returns) at selected
 * collocation rows, every element summed directly with compact coefficients computed on
 * the fly (no table, no FMM): for checking the FMM's far field at sampled rows where a
 * direct context would not fit.  host_rows: nrows row indices (host); 1 <= alpha <=
 * current position; dev_out: nrows doubles.  O(nrows Ns window) element integrals. */
int tdbem_direct_rows(struct tdbem_ctx *ctx, int nrows, const int32_t *host_rows, int alpha, double *dev_out);

/* Free every device buffer of the context.  NULL is ignored. */
void tdbem_destroy(struct tdbem_ctx *ctx);

/* Message of the last failing call on ctx (or of the last failed create when ctx is NULL). */
const char *tdbem_last_error(const struct tdbem_ctx *ctx);

/* Fill *info with sizes and derived parameters of the context. */
int tdbem_get_info(const struct tdbem_ctx *ctx, tdbem_info *info);

/* Return to the initial state (alpha = 1, zero history, zero FMM moments/locals). */
int tdbem_reset(struct tdbem_ctx *ctx);

/* Replace the stored history by nsteps coefficient rows beta = 0..nsteps-1
 * (dev_u, dev_q: nsteps x Ns each; NULL = zeros) and position the march at
 * alpha = nsteps + 1.  Moments and locals are rebuilt from the new history. */
int tdbem_set_history(struct tdbem_ctx *ctx, int nsteps, const double *dev_u, const double *dev_q);

/* History part of b^{alpha-1} (eq. linear) from the stored coefficients
 * beta <= alpha-2:  sum_j sum_beta (C_U^{(alpha-beta)} q_j^beta - C_W^{(alpha-beta)} u_j^beta)
 * (Burton-Miller matrices for the BMBIE), near pairs directly and far pairs by
 * the FMM when enabled.  alpha must equal the current march position
 * (1 <= alpha <= nsteps stored + 1).  dev_b_hist: Ns doubles, written. */
int tdbem_fmm_eval(struct tdbem_ctx *ctx, int alpha, double *dev_b_hist);

/* One step alpha -> alpha+1: b = forcing + history (near + far) + known
 * current-step part, solve A x = b by GMRES (FP64), store x^{alpha-1} (u on
 * Neumann faces, q on Dirichlet faces) and the prescribed coefficient, and
 * advance the FMM (P2M, M2M, M2L by Algorithm 1, L2L).
 * dev_forcing: Ns doubles f^alpha (u_in, or (d/dn - (1/c) d/dt) u_in for the
 * BMBIE, with the inward normal), or NULL for zero.  dev_bc_values: Ns
 * prescribed coefficients at beta = alpha-1 (u for Dirichlet, q for
 * Neumann), NULL = homogeneous.  dev_x_out: Ns doubles or NULL.
 * Errors: TDBEM_E_STATE past nt_max, TDBEM_E_NOT_CONVERGED, TDBEM_E_DIVERGED. */
int tdbem_step(struct tdbem_ctx *ctx, const double *dev_forcing, const double *dev_bc_values,
               double *dev_x_out, tdbem_step_info *info);

/* March from the current position to alpha = nt-1 (normally from a fresh or
 * reset context: nt-1 solves).  Forcing: dev_forcing ((nt-1) x Ns, row alpha-1)
 * if not NULL, else the incident wave *inc evaluated on the device, else zero.
 * dev_x_hist_out: (nt-1) x Ns solution coefficients, or NULL.  Homogeneous
 * boundary condition.  info may be NULL. */
int tdbem_run(struct tdbem_ctx *ctx, int nt, const double *dev_forcing, const tdbem_incident *inc,
              double *dev_x_hist_out, tdbem_run_info *info);

/* March n independent contexts together (many scatterers on one GPU).
 * Context i marches from its current position to alpha = nt[i]-1 under the
 * incident wave inc[i] (inc NULL: zero forcing), homogeneous boundary
 * condition, like tdbem_run.  Contexts created with opts.graph = 1 launch
 * their captured march graphs; the others are stepped in lock-step, one step
 * of every context in turn.  Contexts on distinct HIP streams run
 * concurrently.  dev_x_hist_out: NULL or n pointers ((nt[i]-1) x Ns each, or
 * NULL); info: NULL or n records.  *wall_ms (may be NULL): host wall time from
 * the first launch to the end of the last context.  Returns the first error;
 * each context's message is in its tdbem_last_error. */
int tdbem_run_batch(struct tdbem_ctx *const *ctxs, int n, const int *nt, const tdbem_incident *inc,
                    double *const *dev_x_hist_out, tdbem_run_info *info, double *wall_ms);

/* Checkpoint of the march state into caller-owned host memory: the position
 * alpha, the solved coefficient rows beta = 0..alpha-2 (u and q), the FMM state
 * carried between steps (partial moments, locals ring, recurrence terms of every
 * level) and the learned-guess parameters if loaded.  host_buf NULL: *bytes
 * receives the size needed.  Otherwise *bytes is the buffer size on entry and
 * the size written on return; too small: TDBEM_E_INVAL with the size needed
 * in *bytes. */
int tdbem_checkpoint(struct tdbem_ctx *ctx, void *host_buf, size_t *bytes);

/* Continue from a checkpoint: the context must have been created with the same
 * mesh size, d, BIE, boundary condition and FMM parameters (else TDBEM_E_INVAL);
 * the next tdbem_step / tdbem_run continues at the checkpoint's alpha and gives
 * the same results as the uninterrupted march. */
int tdbem_restore(struct tdbem_ctx *ctx, const void *host_buf, size_t bytes);

/* Copy the stored coefficients beta = 0..nsteps-1 to dev_u, dev_q (nsteps x Ns each; either may be NULL). */
int tdbem_get_history(struct tdbem_ctx *ctx, int nsteps, double *dev_u, double *dev_q);

/* Device evaluation of the incident forcing f^alpha for alpha = a0..a0+n-1 into
 * dev_out (n x Ns): u_in (OBIE) or (d/dn - (1/c) d/dt) u_in (BMBIE) at the
 * collocation points, inward normal. */
int tdbem_incident_forcing(struct tdbem_ctx *ctx, const tdbem_incident *inc, int a0, int n, double *dev_out);

/* Diagnostic access to the near-field compact coefficients of row i:
 * writes up to cap entries (j, g, C_U^{(g)}_ij, C_W^{(g)}_ij) to host arrays;
 * returns the number of entries of the row (>= 0) or an error code. With
 * opts.near_form = 1 the entries are the raw X_U^{(g)}, X_W^{(g)} instead, and
 * with opts.near_prec = 1 they are the stored FP32 values widened to FP64. */
int tdbem_near_row(struct tdbem_ctx *ctx, int i, int cap, int32_t *j_out, int32_t *g_out,
                   double *cu_out, double *cw_out);

/* Kernel timing.  While enabled, every kernel launch of the context is
 * bracketed by HIP events on the context stream and attributed to a category:
 * 0 near-field history sum, 1 GMRES solve, 2 L2P, 3 P2M (with densities),
 * 4 M2L products, 5 M2L reduction + recurrence, 6 M2M, 7 L2L, 8 other,
 * 9 learned guess (scale, features, network, proposal), 10 M2L derivative
 * products (time moments and the separable U^{(p)} products; 4 holds the
 * near-future products).
 * tdbem_profile(ctx, 1) clears the accumulators; tdbem_profile_read() waits
 * for the stream and writes per-category total milliseconds and launch counts
 * (arrays of n <= 16 entries). */
#define TDBEM_PROF_KINDS 11
int tdbem_profile(struct tdbem_ctx *ctx, int enable);
int tdbem_profile_read(struct tdbem_ctx *ctx, double *ms, int64_t *launches, int n);
/* Like tdbem_profile(ctx, 1) but only the categories whose bit is set in mask
 * are bracketed (fewer events in the stream); mask 0 disables profiling. */
int tdbem_profile_mask(struct tdbem_ctx *ctx, unsigned mask);

/* Override the autotuned M2L launch for the n finest levels ending an interval
 * together (n = 1 .. depth-1; tdbem_info.m2l_variant reports the current one):
 * choice = 2 * tile + persistent, tile 0 .. 11 as listed at m2l_variant.  For
 * tests and tuning studies; the results are the same for every choice up to
 * summation order.  TDBEM_E_INVAL without an FMM, for n or choice out of range,
 * or for tiles 8 .. 11 when p_s^3 p_t is not a multiple of 4. */
int tdbem_set_m2l_variant(struct tdbem_ctx *ctx, int n, int choice);

/* ------------------------------------------------------------------------
 * Learned initial guess (not part of the paper: the per-step system of eq.
 * linear is solved by GMRES here, and a small network proposes where each
 * solve starts; GMRES still runs to its tolerance, so the solution does not
 * depend on the guess).
 *
 * Network: per element, 12 inputs -> three ReLU layers of width 256 -> one
 * output.  Weights and every layer input are rounded to bfloat16 (nearest,
 * ties to even) before entering a product; products are accumulated in FP32
 * on the matrix cores; biases are FP32.
 *
 * Parameters: one packed FP32 vector of TDBEM_MLP_NPARAM floats, blocks in
 * this order, W[o][i] mapping input i to output o (row-major):
 *   W1 [256][16] (input columns 12..15 are padding and should stay 0), b1 [256],
 *   W2 [256][256], b2 [256], W3 [256][256], b3 [256], W4 [256], b4 [1].
 * Features (dev_feat): n x 16 FP32 per element, columns 12..15 ignored:
 *   0..3  backward differences of the last four solved rows x1..x4 of the
 *         unknown: x1, x1 - x2, x1 - 2 x2 + x3, x1 - 3 x2 + 3 x3 - x4, over s
 *   4     (b_i / A_ii - e_i) / s  (Jacobi-scaled right-hand side of the step
 *         relative to the extrapolation e defined below)
 *   5..7  outward unit normal
 *   8     area / h^2              (h = mean edge length)
 *   9..11 (centroid - bounding-box centre) / R   (R = largest vertex distance from it)
 * with s the root mean square of x1..x4 and b_i / A_ii together.  The output
 * y corrects the quadratic extrapolation e = 3 x^{beta-1} - 3 x^{beta-2} + x^{beta-3}:
 * the proposal is x^beta = e + s y (e where y is not finite), and the training
 * target is (x^beta - e) / s.
 * All calls below enqueue on hip_stream (NULL = null stream) and return
 * after that stream has finished them; every pointer is caller-owned. */
#define TDBEM_MLP_IN 12
#define TDBEM_MLP_IN_PAD 16
#define TDBEM_MLP_WIDTH 256
#define TDBEM_MLP_NPARAM 136193

/* Forward pass over n rows: dev_y (n) = network(dev_feat (n x 16)).
 * dev_act: NULL, or 3 x n x 256 bf16 (uint16) that receives the rounded
 * hidden activations h1, h2, h3 for tdbem_mlp_backward. */
int tdbem_mlp_forward(const float *dev_params, int n, const float *dev_feat, float *dev_y,
                      uint16_t *dev_act, void *hip_stream);

/* The same forward pass with the network installed in ctx by tdbem_mlp_load
 * (or tdbem_restore), through the march's kernel, which reads the hidden
 * layers' weights pre-rounded to bf16 in matrix-core fragment order: dev_y (n)
 * equals tdbem_mlp_forward of the installed parameters bit for bit.  Runs on
 * the context's stream.  TDBEM_E_INVAL if no network is installed. */
int tdbem_mlp_forward_loaded(struct tdbem_ctx *ctx, int n, const float *dev_feat, float *dev_y);

/* FP32 floats of workspace tdbem_mlp_backward needs for n rows. */
size_t tdbem_mlp_workspace_floats(int n);

/* Gradient of sum_r dy_r y_r with respect to the parameters (rounding taken
 * as the identity), written to dev_grad (TDBEM_MLP_NPARAM floats, overwritten).
 * dev_act from the forward pass of the same parameters and features.
 * dev_work: tdbem_mlp_workspace_floats(n) floats.  Deterministic. */
int tdbem_mlp_backward(const float *dev_params, int n, const float *dev_feat, const uint16_t *dev_act,
                       const float *dev_dy, float *dev_grad, float *dev_work, size_t work_floats,
                       void *hip_stream);

/* Largest n accepted by tdbem_mlp_backward_noalloc. */
#define TDBEM_MLP_NOALLOC_MAX_ROWS 8192

/* tdbem_mlp_backward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid hipMalloc): no workspace argument, and no allocation of any kind in
 * the call.  The intermediate results (activation gradients, per-split weight
 * gradient partials) live in one library-owned device array of fixed size
 * (29.6 MB per GPU, held from the first call on that GPU until the process
 * ends), shared by every call on that GPU: calls that overlap on one GPU race
 * and must be serialised by the caller.  Arguments and results as for
 * tdbem_mlp_backward (bit for bit the same gradient).
 * Errors: TDBEM_E_INVAL for n > TDBEM_MLP_NOALLOC_MAX_ROWS or bad pointers. */
int tdbem_mlp_backward_noalloc(const float *dev_params, int n, const float *dev_feat, const uint16_t *dev_act,
                               const float *dev_dy, float *dev_grad, void *hip_stream);

/* Mean squared error over n rows: dev_loss[0] = mean (y - t)^2 and
 * dev_dy = 2 (y - t) / n.  Deterministic. */
int tdbem_mlp_mse(int n, const float *dev_y, const float *dev_t, float *dev_dy, float *dev_loss,
                  void *hip_stream);

/* One Adam step (number t >= 1, bias-corrected) on TDBEM_MLP_NPARAM
 * parameters with first/second moment buffers dev_m, dev_v (zero before t = 1). */
int tdbem_mlp_adam_step(float *dev_params, const float *dev_grad, float *dev_m, float *dev_v, int t, float lr,
                        float beta1, float beta2, float eps, void *hip_stream);

/* Copy a parameter vector into the context; with opts.guess = TDBEM_GUESS_MLP
 * the march starts each solve from the network's proposal (rows beta >= 4). */
int tdbem_mlp_load(struct tdbem_ctx *ctx, const float *dev_params);

/* Record training pairs during later steps: for every solved row beta >= 4,
 * dev_feat + beta*Ns*16 receives the features and dev_target + beta*Ns the
 * target (caller-owned, nt_max x Ns x 16 and nt_max x Ns FP32; other rows are
 * not written).  NULL, NULL stops recording. */
int tdbem_mlp_record(struct tdbem_ctx *ctx, float *dev_feat, float *dev_target);

#ifdef __cplusplus
}
#endif
#endif /* TDBEM_H */
