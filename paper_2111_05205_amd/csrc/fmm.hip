// Interpolation-based space-time FMM for the far part of the history sum
// (paper Section 3: eqs. target, U_intp, Uabmn, target_m2l, m2l and the
// Burton-Miller evaluation of the local field; Section 4: near-future M2L,
// eq. m2l_near, derivative products, eq. L_l,k, and the O(Nt) recurrence of
// Formula 1 / Algorithm 1).
//
// Space: octree over the vertex bounding box (root half side rounded up to a
// power of two), faces assigned to leaves by centroid, near field = the 27
// leaves around a face's leaf, interaction lists on levels 2..depth with 316
// possible relative offsets.  Time: M_leaf steps per leaf interval (the
// largest value for which same-interval interaction-list pairs vanish by
// causality), doubling per level; a source sample tau^{beta} belongs to
// interval floor((beta+1)/M) (grouped by t_{beta+1} as in eq. target), a
// target t_alpha to floor(alpha/M); intervals are centred on the times they
// hold.  Interpolation in each of the eight variables: tensor Lagrange on
// Chebyshev points (first kind), or the cubic Hermite interpolation with
// finite-difference slopes on equispaced nodes that the paper used (Section 3,
// after eq. Uabmn); P = p_s^3 p_t coefficients per cell.
//
// Per sample beta (after the solve of step beta+1):
//   P2M        leaf moments of the current source interval       (HBM-bound, small)
//   at the end of a level's source interval k (every level ending then together):
//     M2M      child -> parent re-interpolation (parent-centric, no atomics), first:
//              it only reads the children's moments
//     M2L      offset-batched dense products: for every interaction pair,
//              [U_{k+1,k}; ...; U_{k+mu+1,k}; U^{(1)}; ...; U^{(d)}] M_k(S)
//              written to a per-pair staging buffer, one launch for all those
//              levels (FP32 contexts: P2M and M2M also keep an FP32 copy of the moments)
//     reduce   per target cell: near-future locals L_{k+l} += ..., and the
//              derivative products                                      (HBM-bound)
//     recurrence of Algorithm 1 (eqs. m2l_expand_rec1, m2l_rec, m2l_expand_rec2)
//              per (cell, coefficient)
//   L2L        at the start of a parent's target interval, parent -> child
//   L2P        at each target step: field or Burton-Miller operator of it
#include "internal.h"

#include <algorithm>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

namespace tdbem {

constexpr int MAXP = 8;  // nodes per axis

struct NodeSet { double s[MAXP], t[MAXP]; int interp; };  // nodes in space and time, TDBEM_INTERP_*

// Slope coefficient D[row][a] of the finite-difference nodal slopes on equispaced
// nodes of spacing h: central differences inside, second-order one-sided at the ends.
__host__ __device__ inline double fd_slope(int p, double h, int row, int a) {
  const double s = 0.5 / h;
  if (row == 0) return a == 0 ? -3.0 * s : a == 1 ? 4.0 * s : a == 2 ? -s : 0.0;
  if (row == p - 1) return a == p - 1 ? 3.0 * s : a == p - 2 ? -4.0 * s : a == p - 3 ? s : 0.0;
  return a == row + 1 ? s : a == row - 1 ? -s : 0.0;
}

// Cardinal function l_a(x) of the cubic Hermite interpolation with those slopes and
// its derivative: on the segment [om_k, om_k+1], with t = (x - om_k)/h, the
// interpolant is h00 f_k + h01 f_k+1 + h (h10 m_k + h11 m_k+1), m = D f; the end
// pieces are continued outside [om_0, om_{p-1}].
__host__ __device__ inline void hermite_fd(const double* om, int p, int a, double x, double* val, double* der) {
  const double h = om[1] - om[0];
  int k = (int)floor((x - om[0]) / h);
  k = k < 0 ? 0 : k > p - 2 ? p - 2 : k;
  const double t = (x - om[k]) / h, t2 = t * t, t3 = t2 * t;
  const double dk = fd_slope(p, h, k, a), dk1 = fd_slope(p, h, k + 1, a);
  double v = h * ((t3 - 2.0 * t2 + t) * dk + (t3 - t2) * dk1);
  double g = (3.0 * t2 - 4.0 * t + 1.0) * dk + (3.0 * t2 - 2.0 * t) * dk1;
  if (a == k) { v += 2.0 * t3 - 3.0 * t2 + 1.0; g += (6.0 * t2 - 6.0 * t) / h; }
  if (a == k + 1) { v += -2.0 * t3 + 3.0 * t2; g += (6.0 * t - 6.0 * t2) / h; }
  *val = v;
  *der = g;
}

// bfloat16 bits of x: rounded to float, then to nearest bf16, ties to even (NaN stays NaN).
__device__ inline uint16_t bf16_rne(double x) {
  const float f = (float)x;
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// The second bf16 term of x = hi + lo: the rounded remainder x - hi (split products).
__device__ inline uint16_t bf16_lo(double x, uint16_t hi) {
  return bf16_rne(x - (double)__uint_as_float((uint32_t)hi << 16));
}

// The dense near-future operators of one level (eq. m2l_near, the gaps gf .. g0-1 of
// each offset) with their gap ranges and storage offsets.  In normalised units
// (lengths / (c dt), times / dt) they depend only on the level's distance from the
// leaves, and contexts that agree on it share one set.
struct LevelOps {
  std::vector<std::array<int, 3>> slots;  // offsets the operators are formed for
  std::vector<int> gf, g0;                // gap range of each slot's dense blocks
  std::vector<int64_t> uoff;              // first operator element of each slot (nslot + 1 entries)
  int64_t tot = 0;                        // elements of one operator copy
  DevBuf<double> Uf;                      // FP64 operators in MFMA fragment order
  DevBuf<float> U32;                      // FP32 (mixed precision)
  DevBuf<uint16_t> U16;                   // BF16 fragments (split products: the second terms after tot)
};

struct FmmLevel {
  int ncell = 0;
  std::vector<std::array<int, 3>> key;      // integer cell coordinates
  std::vector<int> parent;                  // index in level-1
  std::vector<int> octant;                  // bit q set: upper half along axis q
  // interaction pairs sorted by target cell
  int64_t npair = 0;
  std::vector<int> il_ptr;                  // ncell+1
  std::vector<int> il_src, il_slot;         // npair
  std::vector<std::array<int, 3>> slot_off; // offset vector of each matrix slot present at this level
  // device
  DevBuf<int32_t> d_il_ptr, d_parent, d_octant, d_child_ptr, d_child;
  DevBuf<int32_t> d_il_src;                 // source cell of each interaction pair (sorted by target cell)
  DevBuf<int32_t> d_tiles128, d_tiles64, d_tiles32;  // GEMM column tiles (slot, first, count) by width
  DevBuf<int32_t> d_pairs_by_slot;          // pair indices grouped by slot
  DevBuf<int32_t> d_src_by_slot;            // their source cells (so the two loads are independent)
  int ntiles128 = 0, ntiles64 = 0, ntiles32 = 0;
  std::shared_ptr<LevelOps> ops;            // dense near-future operators (own, or shared)
  std::vector<int> canon;                   // slot of this level -> slot of ops
  DevBuf<double> d_stage;                   // FP64 per-pair products
  DevBuf<float> d_stage32;                  // FP32 / BF16 per-pair products
  DevBuf<double> d_Ktf;                     // derivative products' spatial kernels r^{-1} (and r, d = 3), fragment order
  DevBuf<double> d_tm, d_tsum;              // time moments [j][cell][b] and their node sums [j][cell]
  DevBuf<double> d_V;                       // separable pair products [product][pair][Psr]
  // Per slot (offset): the near-future gaps gf .. g0-1 have node pairs on both sides of the
  // wavefront and are dense operator blocks; gaps before gf are zero at every node pair,
  // gaps from g0 on are wavefront-free (separable).
  std::vector<int> gf, g0;
  DevBuf<int64_t> d_uoff;                   // first operator element of each slot's dense blocks
  DevBuf<int32_t> d_srows, d_soff;          // dense rows of each slot; their first row in a pair's products
  DevBuf<int32_t> d_items[3][2];            // (tile, row block) work items by tile width (128/64/32) and rows (128/256)
  int nitems[3][2] = {};
  DevBuf<int32_t> d_items_sep;              // (tile, 0) for every 32-column tile (separable products)
  DevBuf<int32_t> d_pair_gr;                // per interaction pair (target order): gf | g0 << 16
  DevBuf<int32_t> d_sep_order;              // each target cell's pairs in order of g0 (stable)
  // (cell, gap) entries with dense blocks and their pairs (the reduction of the dense products)
  DevBuf<int32_t> d_red_cg, d_red_ptr, d_red_pairs;
  int nred = 0;
  int64_t dense_blocks = 0;                 // sum over interaction pairs of their dense blocks
  DevBuf<double> d_mom, d_ring, d_lp, d_aux, d_dp;
  DevBuf<float> d_mom32;                    // FP32 copy of the moments, written by P2M / M2M (FP32 M2L)
  DevBuf<uint16_t> d_mom16;                 // BF16 M2L: moments [cell][Pp] (zero padded; split products: two copies)
};

struct Fmm {
  int D = 0, ps = 0, pt = 0, Ps = 0, P = 0, G = 0, mu = 0, R = 0, m_leaf = 1;
  // precision of the near-future products: 0 FP64, 1 FP32, 2 BF16 (both with FP32
  // accumulation); the derivative products are FP64 in every case
  int prec = 0;
  int interp = TDBEM_INTERP_LAGRANGE;
  double leaf_ratio = 0.0;                 // > 0: leaf side / (c dt), normalised (shareable) operators
  double oscale = 1.0;                     // factor of the dense products: (c dt)^(d-1) with normalised operators
  int Gn = 0;                              // near-future operator blocks, mu + 1
  int Pp = 0;                              // row stride of the BF16 moment copy: P rounded up to 32
  int Pr = 0;                              // row pitch of a gap's P rows in the operator stacks and staged products
  int Psr = 0;                             // row pitch of a pair's Ps separable products
  double H = 0, center[3] = {0, 0, 0}, e_max = 0;
  double om_s[MAXP], om_t[MAXP];
  NodeSet nodes{};                         // the same, as a kernel argument
  std::vector<FmmLevel> lev;               // 0..D
  std::vector<int> leaf_of;                // element -> leaf cell
  std::vector<int> leaf_ptr, leaf_elems;   // leaf -> elements (CSR)
  DevBuf<int32_t> d_leaf_of, d_leaf_ptr, d_leaf_elems;
  DevBuf<double> d_A, d_B, d_E0, d_E1;     // P2M / L2P tables, ns x Ps
  DevBuf<double> d_tau, d_sig;
  DevBuf<double> d_S, d_T;                 // 1-D re-interpolation matrices [side][parent][child]
  double Cd = 0;
  int m2l_choice[16] = {0};                // per number of levels in a launch: 2 * tile variant + persistent
  int persistent_grid = 0;                 // workgroups of a persistent M2L launch
};

// ---------------------------------------------------------------------------
// Host helpers

static void cheb(int p, double* om) {
  for (int a = 0; a < p; ++a) om[a] = std::cos((2.0 * a + 1.0) * M_PI / (2.0 * p));
}

static void equispaced(int p, double* om) {
  for (int a = 0; a < p; ++a) om[a] = -1.0 + 2.0 * a / (p - 1);
}

static double lag(const double* om, int p, int a, double x) {
  double v = 1.0;
  for (int b = 0; b < p; ++b)
    if (b != a) v *= (x - om[b]) / (om[a] - om[b]);
  return v;
}

static double dlag(const double* om, int p, int a, double x) {
  double s = 0.0;
  for (int c = 0; c < p; ++c) {
    if (c == a) continue;
    double t = 1.0 / (om[a] - om[c]);
    for (int b = 0; b < p; ++b)
      if (b != a && b != c) t *= (x - om[b]) / (om[a] - om[b]);
    s += t;
  }
  return s;
}

// l_a(x) and l_a'(x) of the context's interpolation
static double basis(const Fmm* f, const double* om, int p, int a, double x, double* der = nullptr) {
  if (f->interp == TDBEM_INTERP_HERMITE) {
    double v, g;
    hermite_fd(om, p, a, x, &v, &g);
    if (der) *der = g;
    return v;
  }
  if (der) *der = dlag(om, p, a, x);
  return lag(om, p, a, x);
}

static uint64_t morton(int x, int y, int z) {
  uint64_t m = 0;
  for (int b = 0; b < 21; ++b) {
    m |= (uint64_t)((x >> b) & 1) << (3 * b);
    m |= (uint64_t)((y >> b) & 1) << (3 * b + 1);
    m |= (uint64_t)((z >> b) & 1) << (3 * b + 2);
  }
  return m;
}

static int64_t key64(int x, int y, int z) { return ((int64_t)x << 42) | ((int64_t)y << 21) | (int64_t)z; }

static double hs_of(const Fmm* f, int l) { return f->H / (double)(1 << l); }

// ---------------------------------------------------------------------------
// Device kernels


// U[slot][g*P + row][col] for one level.  row = a1 + ps(a2 + ps(a3 + ps m)), col likewise (b, n).
__global__ void m2l_matrix_kernel(int ps, int pt, int P, int G, int mu, int d, double c, double hs, double ht,
                                  double dt, int Ml, NodeSet nodes, const int32_t* __restrict__ slot_off,
                                  double* __restrict__ U) {
  const int slot = blockIdx.z;
  const int g = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)P * P) return;
  const int row = (int)(idx / P), col = (int)(idx % P);
  const int Ps = ps * ps * ps;
  const int a = row % Ps, m = row / Ps, b = col % Ps, n = col / Ps;
  const int a1 = a % ps, a2 = (a / ps) % ps, a3 = a / (ps * ps);
  const int b1 = b % ps, b2 = (b / ps) % ps, b3 = b / (ps * ps);
  const int ox = slot_off[3 * slot], oy = slot_off[3 * slot + 1], oz = slot_off[3 * slot + 2];
  // y - x between source node b of cell O+o and target node a of cell O
  const double dx = 2.0 * hs * ox + hs * (nodes.s[b1] - nodes.s[a1]);
  const double dy = 2.0 * hs * oy + hs * (nodes.s[b2] - nodes.s[a2]);
  const double dz = 2.0 * hs * oz + hs * (nodes.s[b3] - nodes.s[a3]);
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  // near future, target interval k + (g+1) (eq. Uabmn)
  const double tds = ((g + 1) * (double)Ml + 1.0) * dt + ht * (nodes.t[m] - nodes.t[n]);
  double arg = c * tds - r;
  if (arg < 0.0) arg = 0.0;
  U[((int64_t)slot * G + g) * P * P + idx] = ipow(arg, d) / r;
}

// Spatial kernels of the separable products between target node a and source
// node b of a cell pair at offset `slot` (cell half side hs): K[0] = 1/r, K[1] = r
// (d >= 2), K[2] = r^2 (d = 3); row-major [kernel][slot][a][b] (converted to MFMA
// fragment order afterwards).
__global__ void m2l_spatial_kernel(int ps, int nk, double hs, NodeSet nodes, const int32_t* __restrict__ slot_off,
                                   int nslot, double* __restrict__ Kt) {
  const int Ps = ps * ps * ps;
  const int slot = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Ps * Ps) return;
  const int a = idx / Ps, b = idx % Ps;
  const int a1 = a % ps, a2 = (a / ps) % ps, a3 = a / (ps * ps);
  const int b1 = b % ps, b2 = (b / ps) % ps, b3 = b / (ps * ps);
  const int ox = slot_off[3 * slot], oy = slot_off[3 * slot + 1], oz = slot_off[3 * slot + 2];
  const double dx = 2.0 * hs * ox + hs * (nodes.s[b1] - nodes.s[a1]);
  const double dy = 2.0 * hs * oy + hs * (nodes.s[b2] - nodes.s[a2]);
  const double dz = 2.0 * hs * oz + hs * (nodes.s[b3] - nodes.s[a3]);
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  Kt[(int64_t)slot * Ps * Ps + idx] = 1.0 / r;
  if (nk > 1) Kt[((int64_t)nslot + slot) * Ps * Ps + idx] = r;
  if (nk > 2) Kt[((int64_t)2 * nslot + slot) * Ps * Ps + idx] = r * r;
}

// P2M / L2P element tables on the device.  Triangle quadrature: collapsed
// (Duffy) tensor Gauss-Legendre with nq points per direction, exact for the
// polynomial degree 3(p_s-1) of the tensor basis.
struct QuadRule { double x[16]; double w[16]; int n; };

__global__ void elem_tables_kernel(int ns, int ps, double hs, NodeSet nodes, QuadRule q,
                                   const double* __restrict__ tris, const double* __restrict__ nrm,
                                   const double* __restrict__ xc, const double* __restrict__ cell_center,
                                   const int32_t* __restrict__ leaf_of, double* __restrict__ A,
                                   double* __restrict__ B, double* __restrict__ E0, double* __restrict__ E1) {
  const int e = blockIdx.x;
  const int Ps = ps * ps * ps;
  const int b = threadIdx.x;
  if (b >= Ps) return;
  const int b1 = b % ps, b2 = (b / ps) % ps, b3 = b / (ps * ps);
  const double* V = tris + 9 * (int64_t)e;
  const double* cc = cell_center + 3 * (int64_t)leaf_of[e];
  const double* n = nrm + 3 * (int64_t)e;
  double e1[3] = {V[3] - V[0], V[4] - V[1], V[5] - V[2]};
  double e2[3] = {V[6] - V[3], V[7] - V[4], V[8] - V[5]};
  double cr[3];
  cross3(e1, e2, cr);
  const double area2 = sqrt(dot3(cr, cr));
  double sa = 0.0, sb = 0.0;
  for (int i = 0; i < q.n; ++i) {
    const double u = q.x[i];
    for (int j = 0; j < q.n; ++j) {
      const double v = q.x[j];
      const double w = q.w[i] * q.w[j] * u * area2;
      double xi[3];
      for (int k = 0; k < 3; ++k) xi[k] = (V[k] + u * e1[k] + u * v * e2[k] - cc[k]) / hs;
      double l[3], dl[3];
      const int bb[3] = {b1, b2, b3};
      for (int k = 0; k < 3; ++k) {
        double val = 1.0, der = 0.0;
        if (nodes.interp == TDBEM_INTERP_HERMITE) {
          hermite_fd(nodes.s, ps, bb[k], xi[k], &val, &der);
        } else {
          for (int o = 0; o < ps; ++o) {
            if (o == bb[k]) continue;
            const double f = 1.0 / (nodes.s[bb[k]] - nodes.s[o]);
            der = der * (xi[k] - nodes.s[o]) * f + val * f;
            val *= (xi[k] - nodes.s[o]) * f;
          }
        }
        l[k] = val;
        dl[k] = der;
      }
      sa += w * l[0] * l[1] * l[2];
      sb += w * (n[0] * dl[0] * l[1] * l[2] + n[1] * l[0] * dl[1] * l[2] + n[2] * l[0] * l[1] * dl[2]);
    }
  }
  A[(int64_t)e * Ps + b] = sa;
  B[(int64_t)e * Ps + b] = sb / hs;
  // L2P: basis and its normal derivative at the collocation point
  double xi[3], l[3], dl[3];
  const int bb[3] = {b1, b2, b3};
  for (int k = 0; k < 3; ++k) {
    xi[k] = (xc[3 * (int64_t)e + k] - cc[k]) / hs;
    double val = 1.0, der = 0.0;
    if (nodes.interp == TDBEM_INTERP_HERMITE) {
      hermite_fd(nodes.s, ps, bb[k], xi[k], &val, &der);
    } else {
      for (int o = 0; o < ps; ++o) {
        if (o == bb[k]) continue;
        const double f = 1.0 / (nodes.s[bb[k]] - nodes.s[o]);
        der = der * (xi[k] - nodes.s[o]) * f + val * f;
        val *= (xi[k] - nodes.s[o]) * f;
      }
    }
    l[k] = val;
    dl[k] = der;
  }
  E0[(int64_t)e * Ps + b] = l[0] * l[1] * l[2];
  E1[(int64_t)e * Ps + b] = (n[0] * dl[0] * l[1] * l[2] + n[1] * l[0] * dl[1] * l[2] + n[2] * l[0] * l[1] * dl[2]) / hs;
}

// tau^beta and sigma^beta (eqs. tau, sigma, full kappa sum).
__global__ void densities_kernel(int ns, int beta, int d, BWeights bw, const double* __restrict__ hu,
                                 const double* __restrict__ hq, int use_u, int use_q, double* __restrict__ tau,
                                 double* __restrict__ sig) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  double t = 0.0, s = 0.0;
  const int kmax = min(d + 1, beta);
  for (int k = 0; k <= kmax; ++k) {
    const int64_t r = (int64_t)(beta - k) * ns + i;
    if (use_q) t += bw.w[k] * hq[r];
    if (use_u) s += bw.w[k] * hu[r];
  }
  tau[i] = t;
  sig[i] = s;
}

struct TimeWeights { double w[MAXP]; double dw[MAXP]; };

// P2M of one sample into the leaf moments: one block per leaf, thread per spatial node.
// first: this sample opens the leaf's source interval, so the moments are
// assigned rather than accumulated (no clearing pass between intervals).
__global__ void p2m_kernel(int Ps, int pt, int first, double Cd, TimeWeights tw, const int32_t* __restrict__ leaf_ptr,
                           const int32_t* __restrict__ leaf_elems, const double* __restrict__ A,
                           const double* __restrict__ B, const double* __restrict__ tau,
                           const double* __restrict__ sig, double* __restrict__ mom,
                           float* __restrict__ mom32, uint16_t* __restrict__ mom16, int Pp, int64_t lo16) {
  const int S = blockIdx.x;
  const int P = Ps * pt;
  for (int b = threadIdx.x; b < Ps; b += blockDim.x) {
    double acc = 0.0;
    for (int k = leaf_ptr[S]; k < leaf_ptr[S + 1]; ++k) {
      const int e = leaf_elems[k];
      acc += A[(int64_t)e * Ps + b] * tau[e] - B[(int64_t)e * Ps + b] * sig[e];
    }
    acc *= Cd;
    for (int n = 0; n < pt; ++n) {
      const int64_t ix = (int64_t)S * P + b + Ps * n;
      const double v = (first ? 0.0 : mom[ix]) + acc * tw.w[n];
      mom[ix] = v;
      if (mom32) mom32[ix] = (float)v;  // FP32 products read this copy; the last write of an interval is final
      if (mom16) {  // likewise the BF16 products (and, lo16 > 0, the second term of the split products)
        const int64_t j = (int64_t)S * Pp + b + Ps * n;
        const uint16_t h = bf16_rne(v);
        mom16[j] = h;
        if (lo16) mom16[lo16 + j] = bf16_lo(v, h);
      }
    }
  }
}

// Apply the separable re-interpolation to one P-vector held in LDS:
// along axis 0 (x), 1 (y), 2 (z) with ps x ps matrices and along time with pt x pt.
// Mx[q][i][j]: output index i, input index j.  Works in place between buf0/buf1; returns the buffer holding the result.
__device__ double* apply_sep(double* buf0, double* buf1, int ps, int pt, const double* Mx, const double* My,
                             const double* Mz, const double* Mt) {
  const int Ps = ps * ps * ps, P = Ps * pt;
  double* in = buf0;
  double* out = buf1;
  for (int ax = 0; ax < 4; ++ax) {
    const double* Mm = ax == 0 ? Mx : ax == 1 ? My : ax == 2 ? Mz : Mt;
    const int len = ax < 3 ? ps : pt;
    const int stride = ax == 0 ? 1 : ax == 1 ? ps : ax == 2 ? ps * ps : Ps;
    for (int idx = threadIdx.x; idx < P; idx += blockDim.x) {
      const int i = (idx / stride) % len;
      const int base = idx - i * stride;
      double s = 0.0;
      for (int j = 0; j < len; ++j) s += Mm[i * len + j] * in[base + j * stride];
      out[idx] = s;
    }
    __syncthreads();
    double* t = in; in = out; out = t;
  }
  return in;
}

// M2M: one block per parent cell; sums its children's re-interpolated moments.
// S[side][parent a][child b] (side 0: lower half, 1: upper), T likewise for time.
// half 0 (the first child interval of the parent's) assigns, half 1 accumulates.
__global__ void m2m_kernel(int ps, int pt, int half, const int32_t* __restrict__ child_ptr,
                           const int32_t* __restrict__ child, const int32_t* __restrict__ octant,
                           const double* __restrict__ S, const double* __restrict__ T,
                           const double* __restrict__ mom_c, double* __restrict__ mom_p,
                           float* __restrict__ mom32_p, uint16_t* __restrict__ mom16_p, int Pp, int64_t lo16) {
  extern __shared__ double sm[];
  const int Ps = ps * ps * ps, P = Ps * pt;
  double* b0 = sm;
  double* b1 = sm + P;
  const int p = blockIdx.x;
  double acc[4] = {0, 0, 0, 0};
  const int per = (P + blockDim.x - 1) / blockDim.x;
  for (int k = child_ptr[p]; k < child_ptr[p + 1]; ++k) {
    const int cidx = child[k];
    const int oc = octant[cidx];
    for (int idx = threadIdx.x; idx < P; idx += blockDim.x) b0[idx] = mom_c[(int64_t)cidx * P + idx];
    __syncthreads();
    const double* Mx = S + (oc & 1) * ps * ps;
    const double* My = S + ((oc >> 1) & 1) * ps * ps;
    const double* Mz = S + ((oc >> 2) & 1) * ps * ps;
    const double* Mt = T + half * pt * pt;
    double* res = apply_sep(b0, b1, ps, pt, Mx, My, Mz, Mt);
    for (int q = 0; q < per; ++q) {
      const int idx = threadIdx.x + q * blockDim.x;
      if (idx < P) acc[q] += res[idx];
    }
    __syncthreads();
  }
  for (int q = 0; q < per; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < P) {
      const double v = (half == 0 ? 0.0 : mom_p[(int64_t)p * P + idx]) + acc[q];
      mom_p[(int64_t)p * P + idx] = v;
      if (mom32_p) mom32_p[(int64_t)p * P + idx] = (float)v;
      if (mom16_p) {
        const int64_t j = (int64_t)p * Pp + idx;
        const uint16_t h = bf16_rne(v);
        mom16_p[j] = h;
        if (lo16) mom16_p[lo16 + j] = bf16_lo(v, h);
      }
    }
  }
}

// L2L: one block per child cell; adds the parent's local of interval kp into the
// child's intervals 2kp and 2kp+1.  St/Tt: transposed matrices [side][child a][parent a'].
__global__ void l2l_kernel(int ps, int pt, int R, int kp, const int32_t* __restrict__ parent,
                           const int32_t* __restrict__ octant, const double* __restrict__ St,
                           const double* __restrict__ Tt, const double* __restrict__ ring_p, int ncell_p,
                           double* __restrict__ ring_c, int ncell_c) {
  extern __shared__ double sm[];
  const int Ps = ps * ps * ps, P = Ps * pt;
  double* b0 = sm;
  double* b1 = sm + P;
  const int c = blockIdx.x;
  const int oc = octant[c];
  const double* src = ring_p + ((int64_t)(kp % R) * ncell_p + parent[c]) * P;
  for (int half = 0; half < 2; ++half) {
    for (int idx = threadIdx.x; idx < P; idx += blockDim.x) b0[idx] = src[idx];
    __syncthreads();
    const double* Mx = St + (oc & 1) * ps * ps;
    const double* My = St + ((oc >> 1) & 1) * ps * ps;
    const double* Mz = St + ((oc >> 2) & 1) * ps * ps;
    const double* Mt = Tt + half * pt * pt;
    double* res = apply_sep(b0, b1, ps, pt, Mx, My, Mz, Mt);
    const int kc = 2 * kp + half;
    double* dst = ring_c + ((int64_t)(kc % R) * ncell_c + c) * P;
    for (int idx = threadIdx.x; idx < P; idx += blockDim.x) dst[idx] += res[idx];
    __syncthreads();
  }
}

// M2L products on the matrix cores.  For each column tile (offset slot, first
// pair, count <= 128) and each block of 128 operator rows:
//   stage[pair][row] = sum_col U[slot][row][col] * mom[src(pair)][col],   rows = G*P.
// The moments of the tile's source cells are gathered into LDS, so each block
// of U is read once per column tile.  Four waves each own 32 rows x (16 NCB)
// columns as 2 x NCB blocks of 16 x 16 MFMA accumulators; K advances in steps
// of KS.  FP64 uses v_mfma_f64_16x16x4 (D row = 4 r + lane/16), FP32
// v_mfma_f32_16x16x4 (D row = 4 (lane/16) + r); in both, A[i][k] sits in lane
// i + 16 k and B[k][j] in lane j + 16 k.  The operators are stored in that
// fragment order with consecutive k blocks interleaved per lane, so each wave
// streams its A fragments straight into registers with 16-byte loads, one
// (FP64) or two (FP32) K steps ahead; the gathered moments go through LDS.
// A workgroup covers 64 RPW operator rows (4 waves x RPW row blocks of 16).
constexpr int MB_NMAX = 128;     // widest column tile

typedef double dbl4_t __attribute__((ext_vector_type(4)));
typedef float flt4_t __attribute__((ext_vector_type(4)));
typedef double dbl2_t __attribute__((ext_vector_type(2)));

// k blocks of 4 operator columns, padded to a multiple of 4 so that a lane's
// consecutive k blocks form one 16-byte load (4 FP32 or 2 FP64 values).
static inline int m2l_kblocks(int P) { return ((P + 3) / 4 + 3) / 4 * 4; }
template <class T> struct Vec16;
template <> struct Vec16<float> { typedef flt4_t type; static constexpr int n = 4; };
template <> struct Vec16<double> { typedef dbl2_t type; static constexpr int n = 2; };

template <class T> struct Mfma;
// kTransposed: the product is formed as (moments^T U^T) so that the output tile's
// lanes hold consecutive operator rows of one pair (coalesced staging stores).
template <> struct Mfma<double> {
  typedef dbl4_t acc_t;
  static constexpr bool kTransposed = true;
  static __device__ inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct Mfma<float> {
  typedef flt4_t acc_t;
  static constexpr bool kTransposed = false;
  static __device__ inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Operators in MFMA fragment order, V = 16 / sizeof(T) k blocks interleaved per lane:
// Uf[slot][rb][kb / V][lane][kb % V] = U[16 rb + lane%16][16 (kb/4) + 4 (lane/16) + kb%4]: the
// fragment of MFMA k-substep q of a 16-column block gives lane group kk = lane/16 column
// 4 kk + q, so a lane's four substeps are four consecutive columns.  Rows padded to
// RB = ceil(GP/16) blocks and columns to KB = m2l_kblocks(P) blocks (zeros).  A lane's A
// fragments of V consecutive k blocks are then one 16-byte load, and a wave's load is
// 1 KB of contiguous memory.
// row0, GP: GP rows of each slot's G P x P operator stack (GPsrc rows) from source row
// row0, each gap's P rows at a pitch of Pr rows (rows P .. Pr-1 of a gap are zeros).
template <class T>
__global__ void to_fragments_kernel(int P, int Pr, int GPsrc, int row0, int GP, int RB, int KB,
                                    const double* __restrict__ U, T* __restrict__ Uf) {
  constexpr int V = Vec16<T>::n;
  const int slot = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)RB * KB * 64;
  if (idx >= per) return;
  const int e = (int)(idx % V), lane = (int)((idx / V) & 63);
  const int64_t blk = idx / (64 * V);
  const int kb = (int)(blk % (KB / V)) * V + e, rb = (int)(blk / (KB / V));
  const int row = rb * 16 + (lane & 15), col = 16 * (kb >> 2) + 4 * (lane >> 4) + (kb & 3);
  const int gi = row / Pr, a = row - gi * Pr;
  const double v = (row < GP && a < P && col < P) ? U[((int64_t)slot * GPsrc + row0 + gi * P + a) * P + col] : 0.0;
  Uf[(int64_t)slot * per + idx] = (T)v;
}

// One M2L launch covers every level whose source interval ends at this step:
// per level, its column tiles (at the launch's tile width), operators, moments
// and staging; work items are (level, row block, tile), numbered level by level.
constexpr int M2L_MAXLEV = 12;
struct M2LLevelWork {
  const int32_t* tiles;          // (slot, first pair, count) per tile
  const int32_t* pairs_by_slot;
  const int32_t* src_by_slot;
  const void* Uf;                // T operators in fragment order
  const double* mom;
  const float* mom32;            // FP32 copy of mom (FP32 products only)
  const uint16_t* mom16;         // BF16 copy of mom, row stride Pp (BF16 products only)
  const void* Uf_lo;             // split BF16 products: second bf16 term of the operators (layout of Uf)
  const uint16_t* mom16_lo;      // and of the moments (layout of mom16)
  void* stage;                   // T per-pair products
  int ntiles;
  int item0;                     // first work item of this level
  // Per-slot operator stacks (NULL: every slot has GP rows at slot * per, staged from row 0,
  // and item i is (tile i % ntiles, row block i / ntiles)):
  const int32_t* items;          // (tile, row block) per work item
  const int64_t* uoff;           // first operator element of each slot
  const int32_t* srows;          // operator rows of each slot
  const int32_t* soff;           // row of a pair's staged products where the slot's rows start
};

// A work item's column tile and row block, and the operator stack of its slot.
struct ItemGeom { int tile, rowblk, rows, soff; int64_t uoff; };
__device__ inline ItemGeom item_geom(const M2LLevelWork& Lw, int local, int GP, int64_t per) {
  ItemGeom g;
  if (Lw.items) {
    g.tile = Lw.items[2 * local];
    g.rowblk = Lw.items[2 * local + 1];
  } else {
    g.tile = local % Lw.ntiles;
    g.rowblk = local / Lw.ntiles;
  }
  const int slot = Lw.tiles[3 * g.tile];
  if (Lw.uoff) {
    g.uoff = Lw.uoff[slot];
    g.rows = Lw.srows[slot];
    g.soff = Lw.soff[slot];
  } else {
    g.uoff = (int64_t)slot * per;
    g.rows = GP;
    g.soff = 0;
  }
  return g;
}
struct M2LWork {
  M2LLevelWork lev[M2L_MAXLEV];
  int nlev;
  int total;                     // work items over all levels
  // several contexts in one launch: nlev descriptors in device memory, entry e's items
  // numbered from gitem0[e] (NULL: the nlev descriptors above)
  const M2LLevelWork* glev;
  const int32_t* gitem0;
};

// The level descriptor of work item `item` (GLEV: from the device table; a separate
// instantiation, so that the usual launch reads its descriptors from the kernel arguments).
template <bool GLEV>
__device__ inline const M2LLevelWork& item_level(const M2LWork& W, int item) {
  if constexpr (GLEV) {
    int lo = 0, hi = W.nlev - 1;  // the last entry whose first item is <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (W.gitem0[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    return W.glev[lo];
  } else {
    int lv = 0;
    while (lv + 1 < W.nlev && item >= W.lev[lv + 1].item0) ++lv;
    return W.lev[lv];
  }
}

// Waves per SIMD that the register allocation aims at for FP32 (without a
// target the compiler parks values in the accumulation registers and lands a
// wave short; FP64 and the widest tiles would spill, so they keep 1).
template <class T, int NCB, int KS, int RPW, bool PERS>
constexpr int m2l_waves() {
  return sizeof(T) == 8 || NCB == 8 ? 1 : PERS ? (NCB == 2 ? 2 : 1) : (NCB == 2 && KS == 16) ? 3 : 2;
}

template <class T, int NCB, int KS, int RPW, bool PERS, bool GLEV = false>
__global__ __launch_bounds__(256, (m2l_waves<T, NCB, KS, RPW, PERS>())) void m2l_mfma_kernel(int P, int GP, int RB, int KB, M2LWork W) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int BN = NCB * 16;              // columns (interaction pairs) per tile
  constexpr int LD = BN + 4;                // LDS row stride of the moment tile
  constexpr int BPT = KS * BN / 256;        // moment values loaded per thread per K step
  constexpr int TPC = 256 / BN;             // threads per column
  constexpr int QS = KS / 4;                // MFMA k-substeps per K step
  __shared__ T Bs[2][KS][LD];
  __shared__ int src[BN], pid[BN];
  const int total = W.total;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // PERS: a grid smaller than the work, workgroup b takes items b, b + grid, ...
  // (a grid that is a multiple of 8 keeps each workgroup on one XCD for all its
  // items); otherwise one item per workgroup and no loop (fewer live registers).
  int w = blockIdx.x;
  do {
  // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs, so
  // give each XCD a contiguous range of (row block, column tile) items with the
  // tiles of one offset adjacent; the second tile of an offset then finds that
  // row block of U in the XCD's L2.
  const int q8 = total / 8, r8 = total % 8, x8 = w % 8;
  const int item = x8 * q8 + min(x8, r8) + w / 8;
  const M2LLevelWork& Lw = item_level<GLEV>(W, item);
  const int local = item - Lw.item0;
  const int64_t per = (int64_t)RB * KB * 64;
  const ItemGeom ig = item_geom(Lw, local, GP, per);
  const int tile = ig.tile, rowblk = ig.rowblk, rows = ig.rows, RBs = (rows + 15) >> 4;
  const int32_t* __restrict__ tiles = Lw.tiles;
  const int32_t* __restrict__ pairs_by_slot = Lw.pairs_by_slot;
  const int32_t* __restrict__ src_by_slot = Lw.src_by_slot;
  const T* __restrict__ Uf = static_cast<const T*>(Lw.Uf);
  const double* __restrict__ mom = Lw.mom;
  T* __restrict__ stage = static_cast<T*>(Lw.stage) + ig.soff;
  const int first = tiles[3 * tile + 1], cnt = tiles[3 * tile + 2];
  if constexpr (PERS) __syncthreads();  // the previous item's readers of src / pid / Bs are done
  const int rb0 = (rowblk * 4 + wave) * RPW;             // this wave: row blocks rb0 .. rb0+RPW-1
  if (tid < BN) {
    const int p = tid < cnt ? pairs_by_slot[first + tid] : -1;
    pid[tid] = p;
    src[tid] = tid < cnt ? src_by_slot[first + tid] : -1;
  }
  __syncthreads();
  // Row blocks past the operator's end (rb >= RBs) read the last block again:
  // their products are never stored.  k blocks past KB likewise read the last
  // block and meet zero moments, so every load below is unconditional.
  typedef typename Vec16<T>::type vec_t;
  constexpr int V = Vec16<T>::n;
  static_assert(QS % V == 0, "a K step spans whole 16-byte groups");
  const vec_t* Ar[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
    Ar[r] = reinterpret_cast<const vec_t*>(Uf + ig.uoff + ((int64_t)min(rb0 + r, RBs - 1) * KB) * 64) + lane;
  const int ncb = (cnt + 15) >> 4;                                             // live column blocks
  acc_t acc[RPW][NCB];
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  const int bc = tid / TPC, bk = (tid % TPC) * BPT;
  const int bsrc = src[bc];
  // B values come from the moments in the products' own precision (FP32 contexts keep
  // an FP32 copy: half the bytes of the FP64 moments, the same values once rounded)
  typedef std::conditional_t<sizeof(T) == 4, float, double> MT;
  const MT* mrow = (sizeof(T) == 4 ? reinterpret_cast<const MT*>(Lw.mom32) : reinterpret_cast<const MT*>(mom)) +
                   (int64_t)(bsrc >= 0 ? bsrc : 0) * P;
  // DEPTH K steps ahead in registers (DEPTH sets, used in turn): A fragments
  // (QS k-blocks x 2 row blocks) and this thread's BPT raw moment values of the
  // B tile.  The moments are masked and converted only when they are written
  // to LDS one step before their use, so with DEPTH = 2 the loads of the two
  // following steps stay in flight across each step's products.  (FP64 keeps
  // DEPTH = 1: the second set costs it occupancy.)
  // DEPTH + 1 register sets rotate so that no set is copied: step s reads set
  // s % NSET while the loads of step s + DEPTH fill set (s + DEPTH) % NSET.
  constexpr int DEPTH = (sizeof(T) == 4 && RPW == 2) ? 2 : 1;
  constexpr int NSET = DEPTH + 1;
  T fa[NSET][RPW][QS];
  MT fb[NSET][BPT];
  auto load = [&](int set, int k0) {
    const int g0 = (k0 >> 2) / V;
#pragma unroll
    for (int g = 0; g < QS / V; ++g) {
      const int kg = min(g0 + g, KB / V - 1);
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const vec_t a = Ar[r][(int64_t)kg * 64];
#pragma unroll
        for (int e = 0; e < V; ++e) fa[set][r][g * V + e] = a[e];
      }
    }
#pragma unroll
    for (int i = 0; i < BPT; ++i) fb[set][i] = mrow[min(k0 + bk + i, P - 1)];
  };
  auto stage_b = [&](int set, int k0, int b) {
#pragma unroll
    for (int i = 0; i < BPT; ++i)
      Bs[b][bk + i][bc] = (bsrc >= 0 && k0 + bk + i < P) ? (T)fb[set][i] : T(0);
  };
  // the products of one K step; full: every column block of the tile is live
  auto products = [&](auto full, const T (&ca)[RPW][QS], int b) {
    T bf[QS][NCB];
#pragma unroll
    for (int q = 0; q < QS; ++q)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        bf[q][cb] = Bs[b][16 * (q >> 2) + 4 * (lane >> 4) + (q & 3)][cb * 16 + (lane & 15)];
#pragma unroll
    for (int q = 0; q < QS; ++q) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        if (decltype(full)::value || cb < ncb) {
#pragma unroll
          for (int r = 0; r < RPW; ++r) {
            if constexpr (Mfma<T>::kTransposed)  // A = moment tile (pair cb*16 + lane%16)
              acc[r][cb] = Mfma<T>::op(bf[q][cb], ca[r][q], acc[r][cb]);
            else
              acc[r][cb] = Mfma<T>::op(ca[r][q], bf[q][cb], acc[r][cb]);
          }
        }
      }
    }
  };
#pragma unroll
  for (int h = 0; h < DEPTH; ++h) load(h, h * KS);  // in bounds past P too (clamped)
  stage_b(0, 0, 0);
  __syncthreads();
  int buf = 0;
  const int nsteps = (P + KS - 1) / KS;
  // K step s, whose fragments are in set h = s % NSET.  steady: the loads
  // DEPTH steps ahead and the LDS tile of the next step both exist, so neither
  // is behind a branch and the memory counters wait only for what the step needs.
  auto step = [&](auto hc, int s, auto steady) {
    constexpr int h = decltype(hc)::value;
    constexpr bool st = decltype(steady)::value;
    if (st || s + DEPTH < nsteps) load((h + DEPTH) % NSET, (s + DEPTH) * KS);
    if (sizeof(T) == 4 && ncb == NCB) products(std::true_type{}, fa[h], buf);
    else products(std::false_type{}, fa[h], buf);
    // the other LDS buffer was last read in the previous step, before its barrier
    if (st || s + 1 < nsteps) stage_b((h + 1) % NSET, (s + 1) * KS, buf ^ 1);
    __syncthreads();
    buf ^= 1;
  };
  typedef std::integral_constant<int, 0> set0;
  typedef std::integral_constant<int, 1> set1;
  typedef std::integral_constant<int, 2 % NSET> set2;
  int s = 0;
  for (; s + NSET - 1 + DEPTH < nsteps; s += NSET) {
    step(set0{}, s, std::true_type{});
    step(set1{}, s + 1, std::true_type{});
    if constexpr (NSET == 3) step(set2{}, s + 2, std::true_type{});
  }
  for (; s < nsteps; ++s) {
    const int j = s % NSET;
    if (j == 0) step(set0{}, s, std::false_type{});
    else if (j == 1) step(set1{}, s, std::false_type{});
    else step(set2{}, s, std::false_type{});
  }
#pragma unroll
  for (int h = 0; h < RPW; ++h)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      if (cb >= ncb) continue;
      if constexpr (Mfma<T>::kTransposed) {
        // lane holds operator row lane%16 of pairs 4 r + lane/16 (r = 0..3)
        const int row = (rb0 + h) * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int pr = pid[cb * 16 + 4 * r + (lane >> 4)];
          if (pr >= 0 && row < rows) stage[(int64_t)pr * GP + row] = acc[h][cb][r];
        }
        continue;
      }
      const int p = pid[cb * 16 + (lane & 15)];
      if constexpr (sizeof(T) == 4) {
        // FP32 output: the lane holds rows 4 (lane/16) .. +3 of its pair, so write
        // them as one 16-byte vector (the four lanes of a pair: 64 contiguous bytes)
        const int row0 = (rb0 + h) * 16 + 4 * (lane >> 4);
        if (p >= 0 && ((GP | ig.soff) & 3) == 0 && row0 + 3 < rows) {
          *reinterpret_cast<flt4_t*>(stage + (int64_t)p * GP + row0) = acc[h][cb];
          continue;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (rb0 + h) * 16 + Mfma<T>::row(lane, r);
        if (p >= 0 && row < rows) stage[(int64_t)p * GP + row] = acc[h][cb][r];
      }
    }
    if constexpr (!PERS) break;
    w += gridDim.x;
  } while (w < total);
}

// The same products without LDS or barriers in the K loop: every lane loads
// its B fragments straight from the moments.  With the operator layout above,
// lane (n = lane%16, kk = lane/16) needs moments 4 kk .. 4 kk + 3 of the 16-column
// block for its four k-substeps, one contiguous read per column block (16 bytes
// from the FP32 copy of the moments, 32 bytes in FP64),
// so each wave runs its K loop on its own (the four waves of a workgroup only
// share the tile's pair list, read once into LDS for the epilogue).  K steps of
// 16; P a multiple of 4.  The moment loads are clamped into the row and masked
// (column live, k < P) when they are used.
template <class T, int NCB, int RPW, bool PERS>
constexpr int m2l_direct_waves() {
  return sizeof(T) == 8 || PERS || NCB != 2 ? 1 : RPW == 2 ? 3 : 2;
}

template <class T, int NCB, int RPW, bool PERS, bool GLEV = false>
__global__ __launch_bounds__(256, (m2l_direct_waves<T, NCB, RPW, PERS>())) void m2l_direct_kernel(
    int P, int GP, int RB, int KB, M2LWork W) {
  typedef typename Mfma<T>::acc_t acc_t;
  typedef typename Vec16<T>::type vec_t;
  constexpr int V = Vec16<T>::n;
  constexpr int QS = 4;                     // k-substeps per K step of 16
  constexpr int BN = NCB * 16;
  __shared__ int pid[BN];
  const int total = W.total;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kk4 = 4 * (lane >> 4);
  int w = blockIdx.x;
  do {
  const int q8 = total / 8, r8 = total % 8, x8 = w % 8;
  const int item = x8 * q8 + min(x8, r8) + w / 8;
  const M2LLevelWork& Lw = item_level<GLEV>(W, item);
  const int local = item - Lw.item0;
  const int64_t per = (int64_t)RB * KB * 64;
  const ItemGeom ig = item_geom(Lw, local, GP, per);
  const int tile = ig.tile, rowblk = ig.rowblk, rows = ig.rows, RBs = (rows + 15) >> 4;
  const int32_t* __restrict__ tiles = Lw.tiles;
  const int32_t* __restrict__ pairs_by_slot = Lw.pairs_by_slot;
  const int32_t* __restrict__ src_by_slot = Lw.src_by_slot;
  const T* __restrict__ Uf = static_cast<const T*>(Lw.Uf);
  const double* __restrict__ mom = Lw.mom;
  T* __restrict__ stage = static_cast<T*>(Lw.stage) + ig.soff;
  const int first = tiles[3 * tile + 1], cnt = tiles[3 * tile + 2];
  if constexpr (PERS) __syncthreads();  // the previous item's readers of pid are done
  const int rb0 = (rowblk * 4 + wave) * RPW;
  if (tid < BN) pid[tid] = tid < cnt ? pairs_by_slot[first + tid] : -1;
  // this lane's moment rows (column cb*16 + lane%16 of each column block), in
  // the product's precision: FP32 tiles read the FP32 copy of the moments
  const T* mbase;
  if constexpr (sizeof(T) == 4) mbase = Lw.mom32;
  else mbase = mom;
  const T* brow[NCB];
  bool blive[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int col = cb * 16 + (lane & 15);
    blive[cb] = col < cnt;
    brow[cb] = mbase + (int64_t)src_by_slot[first + min(col, cnt - 1)] * P;
  }
  const vec_t* Ar[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
    Ar[r] = reinterpret_cast<const vec_t*>(Uf + ig.uoff + ((int64_t)min(rb0 + r, RBs - 1) * KB) * 64) + lane;
  const int ncb = (cnt + 15) >> 4;
  acc_t acc[RPW][NCB];
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  constexpr int DEPTH = (sizeof(T) == 4 && RPW == 2) ? 2 : 1;
  constexpr int NSET = DEPTH + 1;
  typedef T mvec_t __attribute__((ext_vector_type(4)));
  T fa[NSET][RPW][QS];
  mvec_t fb[NSET][NCB];
  auto load = [&](int set, int k0) {
    const int g0 = (k0 >> 2) / V;
#pragma unroll
    for (int g = 0; g < QS / V; ++g) {
      const int kg = min(g0 + g, KB / V - 1);
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const vec_t a = Ar[r][(int64_t)kg * 64];
#pragma unroll
        for (int e = 0; e < V; ++e) fa[set][r][g * V + e] = a[e];
      }
    }
    const int off = min(k0 + kk4, P - 4);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) fb[set][cb] = *reinterpret_cast<const mvec_t*>(brow[cb] + off);
  };
  auto products = [&](auto full, int set, int k0) {
    const bool kin = k0 + kk4 < P;
#pragma unroll
    for (int q = 0; q < QS; ++q) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        if (decltype(full)::value || cb < ncb) {
          const T bv = (blive[cb] && kin) ? fb[set][cb][q] : T(0);
#pragma unroll
          for (int r = 0; r < RPW; ++r) {
            if constexpr (Mfma<T>::kTransposed)
              acc[r][cb] = Mfma<T>::op(bv, fa[set][r][q], acc[r][cb]);
            else
              acc[r][cb] = Mfma<T>::op(fa[set][r][q], bv, acc[r][cb]);
          }
        }
      }
    }
  };
#pragma unroll
  for (int h = 0; h < DEPTH; ++h) load(h, h * 16);  // in bounds past P too (clamped)
  const int nsteps = (P + 15) / 16;
  auto step = [&](auto hc, int s, auto steady) {
    constexpr int h = decltype(hc)::value;
    constexpr bool st = decltype(steady)::value;
    if (st || s + DEPTH < nsteps) load((h + DEPTH) % NSET, (s + DEPTH) * 16);
    if (sizeof(T) == 4 && ncb == NCB) products(std::true_type{}, h, s * 16);
    else products(std::false_type{}, h, s * 16);
  };
  typedef std::integral_constant<int, 0> set0;
  typedef std::integral_constant<int, 1> set1;
  typedef std::integral_constant<int, 2 % NSET> set2;
  int s = 0;
  for (; s + NSET - 1 + DEPTH < nsteps; s += NSET) {
    step(set0{}, s, std::true_type{});
    step(set1{}, s + 1, std::true_type{});
    if constexpr (NSET == 3) step(set2{}, s + 2, std::true_type{});
  }
  for (; s < nsteps; ++s) {
    const int j = s % NSET;
    if (j == 0) step(set0{}, s, std::false_type{});
    else if (j == 1) step(set1{}, s, std::false_type{});
    else step(set2{}, s, std::false_type{});
  }
  __syncthreads();  // pid written by the first BN threads
#pragma unroll
  for (int h = 0; h < RPW; ++h)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      if (cb >= ncb) continue;
      if constexpr (Mfma<T>::kTransposed) {
        const int row = (rb0 + h) * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int pr = pid[cb * 16 + 4 * r + (lane >> 4)];
          if (pr >= 0 && row < rows) stage[(int64_t)pr * GP + row] = acc[h][cb][r];
        }
        continue;
      }
      const int p = pid[cb * 16 + (lane & 15)];
      if constexpr (sizeof(T) == 4) {
        const int row0 = (rb0 + h) * 16 + 4 * (lane >> 4);
        if (p >= 0 && ((GP | ig.soff) & 3) == 0 && row0 + 3 < rows) {
          *reinterpret_cast<flt4_t*>(stage + (int64_t)p * GP + row0) = acc[h][cb];
          continue;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (rb0 + h) * 16 + Mfma<T>::row(lane, r);
        if (p >= 0 && row < rows) stage[(int64_t)p * GP + row] = acc[h][cb][r];
      }
    }
    if constexpr (!PERS) break;
    w += gridDim.x;
  } while (w < total);
}

// BF16 near-future products (v_mfma_f32_16x16x32_bf16, FP32 accumulation):
// A[i][k] sits in lane i + 16 (k / 8), element k % 8, B[k][j] in lane j + 16 (k / 8),
// element k % 8, D[4 (lane / 16) + r][lane % 16] in accumulator element r.
// Operators in that fragment order, K steps of 32 columns:
//   U16[slot][rb][kb][lane][e] = U[16 rb + lane % 16][32 kb + 8 (lane / 16) + e]
// (rows padded to RB blocks, columns to KB32 steps, zeros), so a lane's A fragment
// of a K step is one 16-byte load and a wave's is 1 KB of contiguous memory; each
// lane reads its B fragment (8 consecutive moments of its column's source cell)
// as one 16-byte load from the zero-padded BF16 moment copy.  No LDS in the K
// loop; fragments of the next K step are loaded while the current one multiplies.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

template <int NCB, int RPW, bool PERS, bool X3, bool GLEV = false>
__global__ __launch_bounds__(256, 2) void m2l_bf16_kernel(int Pp, int GP, int RB, int KB32, M2LWork W) {
  typedef float f4_t __attribute__((ext_vector_type(4)));
  constexpr int BN = NCB * 16;
  __shared__ int pid[BN];
  const int total = W.total;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, k8 = 8 * (lane >> 4);
  int w = blockIdx.x;
  do {
  const int q8 = total / 8, r8 = total % 8, x8 = w % 8;
  const int item = x8 * q8 + min(x8, r8) + w / 8;
  const M2LLevelWork& Lw = item_level<GLEV>(W, item);
  const int local = item - Lw.item0;
  const ItemGeom ig = item_geom(Lw, local, GP, (int64_t)RB * KB32 * 512);
  const int tile = ig.tile, rowblk = ig.rowblk, rows = ig.rows, RBs = (rows + 15) >> 4;
  const int32_t* __restrict__ tiles = Lw.tiles;
  const int32_t* __restrict__ pairs_by_slot = Lw.pairs_by_slot;
  const int32_t* __restrict__ src_by_slot = Lw.src_by_slot;
  float* __restrict__ stage = static_cast<float*>(Lw.stage) + ig.soff;
  const int first = tiles[3 * tile + 1], cnt = tiles[3 * tile + 2];
  if constexpr (PERS) __syncthreads();  // the previous item's readers of pid are done
  const int rb0 = (rowblk * 4 + wave) * RPW;
  if (tid < BN) pid[tid] = tid < cnt ? pairs_by_slot[first + tid] : -1;
  const uint4* brow[NCB];
  bool blive[NCB];
  int64_t boff[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int col = cb * 16 + (lane & 15);
    blive[cb] = col < cnt;
    boff[cb] = (int64_t)src_by_slot[first + min(col, cnt - 1)] * Pp + k8;
    brow[cb] = reinterpret_cast<const uint4*>(Lw.mom16 + boff[cb]);
  }
  const uint4* Ar[RPW];
  int64_t aoff[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    aoff[r] = (int64_t)min(rb0 + r, RBs - 1) * KB32 * 64 + lane;
    Ar[r] = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(Lw.Uf) + ig.uoff) + aoff[r];
  }
  // X3: x = hi + lo in bf16 for both factors, products hi*hi + hi*lo + lo*hi (lo*lo dropped)
  const uint4* Arl[X3 ? RPW : 1];
  const uint4* browl[X3 ? NCB : 1];
  if constexpr (X3) {
#pragma unroll
    for (int r = 0; r < RPW; ++r)
      Arl[r] = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(Lw.Uf_lo) + ig.uoff) + aoff[r];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) browl[cb] = reinterpret_cast<const uint4*>(Lw.mom16_lo + boff[cb]);
  }
  f4_t acc[RPW][NCB];
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  uint4 fa[2][RPW], fb[2][NCB];
  uint4 fal[2][X3 ? RPW : 1], fbl[2][X3 ? NCB : 1];
  auto load = [&](int set, int s) {
#pragma unroll
    for (int r = 0; r < RPW; ++r) fa[set][r] = Ar[r][(int64_t)s * 64];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) fb[set][cb] = brow[cb][4 * s];
    if constexpr (X3) {
#pragma unroll
      for (int r = 0; r < RPW; ++r) fal[set][r] = Arl[r][(int64_t)s * 64];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) fbl[set][cb] = browl[cb][4 * s];
    }
  };
  auto products = [&](int set) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const uint4 bz = blive[cb] ? fb[set][cb] : uint4{0u, 0u, 0u, 0u};
      const bf16x8_t bv = __builtin_bit_cast(bf16x8_t, bz);
      if constexpr (X3) {
        const uint4 bzl = blive[cb] ? fbl[set][cb] : uint4{0u, 0u, 0u, 0u};
        const bf16x8_t bvl = __builtin_bit_cast(bf16x8_t, bzl);
#pragma unroll
        for (int r = 0; r < RPW; ++r) {  // the two small terms first
          acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, fal[set][r]), bv,
                                                               acc[r][cb], 0, 0, 0);
          acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, fa[set][r]), bvl,
                                                               acc[r][cb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r)
        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, fa[set][r]), bv,
                                                             acc[r][cb], 0, 0, 0);
    }
  };
  load(0, 0);
  int s = 0;
  for (; s + 2 <= KB32; s += 2) {
    load(1, s + 1 < KB32 ? s + 1 : s);
    products(0);
    if (s + 2 < KB32) load(0, s + 2);
    if (s + 1 < KB32) products(1);
  }
  if (s < KB32) products(0);
  __syncthreads();  // pid written by the first BN threads
#pragma unroll
  for (int h = 0; h < RPW; ++h)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int p = pid[cb * 16 + (lane & 15)];
      const int row0 = (rb0 + h) * 16 + 4 * (lane >> 4);
      if (p < 0) continue;
      if (((GP | ig.soff) & 3) == 0 && row0 + 3 < rows) {
        *reinterpret_cast<f4_t*>(stage + (int64_t)p * GP + row0) = acc[h][cb];
        continue;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (row0 + r < rows) stage[(int64_t)p * GP + row0 + r] = acc[h][cb][r];
    }
    if constexpr (!PERS) break;
    w += gridDim.x;
  } while (w < total);
}

// One 1 KB fragment chunk from global memory straight into LDS: lane l copies the
// 16 bytes at g (its own address) to lds + 16 l (lds the same for the whole wave).
__device__ __forceinline__ void copy_to_lds16(const uint4* g, uint4* lds) {
  __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 0);
}

// The same products with the moment fragments staged through LDS: per K step the
// workgroup copies each of its NCB column blocks' fragments (hi, and lo for X3) once,
// instead of once per wave, from global memory straight into one of two LDS buffers
// (global_load_lds_dwordx4: no registers in between; one barrier per step, which also
// waits for the copies; the buffer written at step s was last read at step s - 1).
// Columns past the tile's pairs repeat its last pair (finite values, never stored).
template <int NCB, int RPW, bool PERS, bool X3, bool GLEV = false>
__global__ __launch_bounds__(256, 2) void m2l_bf16_lds_kernel(int Pp, int GP, int RB, int KB32, M2LWork W) {
  typedef float f4_t __attribute__((ext_vector_type(4)));
  constexpr int BN = NCB * 16;
  constexpr int NH = X3 ? 2 : 1;           // hi (and lo) copies of the moments
  constexpr int NF = NH * NCB * 64;        // B fragments (16 bytes each) per K step
  constexpr int FPT = (NF + 255) / 256;    // of them per thread
  __shared__ int pid[BN];
  // one LDS object per buffer, so that reads of one need not wait for copies into the other
  __shared__ uint4 Bs0[NF], Bs1[NF];
  const int total = W.total;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int w = blockIdx.x;
  do {
  const int q8 = total / 8, r8 = total % 8, x8 = w % 8;
  const int item = x8 * q8 + min(x8, r8) + w / 8;
  const M2LLevelWork& Lw = item_level<GLEV>(W, item);
  const int local = item - Lw.item0;
  const ItemGeom ig = item_geom(Lw, local, GP, (int64_t)RB * KB32 * 512);
  const int tile = ig.tile, rowblk = ig.rowblk, rows = ig.rows, RBs = (rows + 15) >> 4;
  const int32_t* __restrict__ tiles = Lw.tiles;
  const int32_t* __restrict__ pairs_by_slot = Lw.pairs_by_slot;
  const int32_t* __restrict__ src_by_slot = Lw.src_by_slot;
  float* __restrict__ stage = static_cast<float*>(Lw.stage) + ig.soff;
  const int first = tiles[3 * tile + 1], cnt = tiles[3 * tile + 2];
  if constexpr (PERS) __syncthreads();  // the previous item's readers of pid and the buffers are done
  const int rb0 = (rowblk * 4 + wave) * RPW;
  if (tid < BN) pid[tid] = tid < cnt ? pairs_by_slot[first + tid] : -1;
  // this wave's B chunks: c = wave + 4 i -> copy h = c / NCB, column block cb = c % NCB (lane l: 16 bytes)
  const uint4* bsrc[FPT];
#pragma unroll
  for (int i = 0; i < FPT; ++i) {
    const int c = min(wave + 4 * i, NH * NCB - 1);  // chunks past NH NCB are not copied
    const int h = c / NCB, cb = c % NCB, l = lane;
    const int col = cb * 16 + (l & 15);
    const uint16_t* base = h ? Lw.mom16_lo : Lw.mom16;
    bsrc[i] = reinterpret_cast<const uint4*>(base + (int64_t)src_by_slot[first + min(col, cnt - 1)] * Pp +
                                             8 * (l >> 4));
  }
  const uint4* Ar[RPW];
  const uint4* Arl[X3 ? RPW : 1];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int64_t aoff = (int64_t)min(rb0 + r, RBs - 1) * KB32 * 64 + lane;
    Ar[r] = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(Lw.Uf) + ig.uoff) + aoff;
    if constexpr (X3) Arl[r] = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(Lw.Uf_lo) + ig.uoff) + aoff;
  }
  f4_t acc[RPW][NCB];
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  uint4 fa[2][RPW], fal[2][X3 ? RPW : 1];
  auto load_a = [&](int set, int s) {
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      fa[set][r] = Ar[r][(int64_t)s * 64];
      if constexpr (X3) fal[set][r] = Arl[r][(int64_t)s * 64];
    }
  };
  auto copy_b = [&](auto bufc, int s) {
    uint4* Bd = decltype(bufc)::value ? Bs1 : Bs0;
#pragma unroll
    for (int i = 0; i < FPT; ++i)
      if (wave + 4 * i < NH * NCB) copy_to_lds16(bsrc[i] + 4 * s, Bd + (wave + 4 * i) * 64);
  };
  auto products = [&](auto setc) {
    constexpr int set = decltype(setc)::value;
    const uint4* Bb = set ? Bs1 : Bs0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const bf16x8_t bv = __builtin_bit_cast(bf16x8_t, Bb[cb * 64 + lane]);
      if constexpr (X3) {
        const bf16x8_t bvl = __builtin_bit_cast(bf16x8_t, Bb[(NCB + cb) * 64 + lane]);
#pragma unroll
        for (int r = 0; r < RPW; ++r) {  // the two small terms first
          acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, fal[set][r]), bv,
                                                               acc[r][cb], 0, 0, 0);
          acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, fa[set][r]), bvl,
                                                               acc[r][cb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r)
        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, fa[set][r]), bv,
                                                             acc[r][cb], 0, 0, 0);
    }
  };
  // K step s uses register set s % 2 and LDS buffer s % 2
  auto step = [&](auto setc, int s) {
    constexpr int set = decltype(setc)::value;
    if (s + 1 < KB32) {
      load_a(set ^ 1, s + 1);
      copy_b(std::integral_constant<int, set ^ 1>{}, s + 1);
    }
    products(setc);
    __syncthreads();
  };
  load_a(0, 0);
  copy_b(std::integral_constant<int, 0>{}, 0);
  __syncthreads();
  for (int s = 0; s < KB32; s += 2) {
    step(std::integral_constant<int, 0>{}, s);
    if (s + 1 < KB32) step(std::integral_constant<int, 1>{}, s + 1);
  }
#pragma unroll
  for (int h = 0; h < RPW; ++h)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int p = pid[cb * 16 + (lane & 15)];
      const int row0 = (rb0 + h) * 16 + 4 * (lane >> 4);
      if (p < 0) continue;
      if (((GP | ig.soff) & 3) == 0 && row0 + 3 < rows) {
        *reinterpret_cast<f4_t*>(stage + (int64_t)p * GP + row0) = acc[h][cb];
        continue;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (row0 + r < rows) stage[(int64_t)p * GP + row0 + r] = acc[h][cb][r];
    }
    if constexpr (!PERS) break;
    w += gridDim.x;
  } while (w < total);
}

// Operators in the BF16 fragment order above (rows as in to_fragments_kernel).
// Uf_lo: NULL, or where the second bf16 term of each value goes (split products).
__global__ void to_fragments_bf16_kernel(int P, int Pr, int GPsrc, int row0, int GP, int RB, int KB32,
                                         const double* __restrict__ U, uint16_t* __restrict__ Uf,
                                         uint16_t* __restrict__ Uf_lo) {
  const int slot = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)RB * KB32 * 512;
  if (idx >= per) return;
  const int e = (int)(idx & 7), lane = (int)((idx >> 3) & 63);
  const int64_t blk = idx >> 9;
  const int kb = (int)(blk % KB32), rb = (int)(blk / KB32);
  const int row = rb * 16 + (lane & 15), col = 32 * kb + 8 * (lane >> 4) + e;
  const int gi = row / Pr, a = row - gi * Pr;
  const double v = (row < GP && a < P && col < P) ? U[((int64_t)slot * GPsrc + row0 + gi * P + a) * P + col] : 0.0;
  const uint16_t h = bf16_rne(v);
  Uf[(int64_t)slot * per + idx] = h;
  if (Uf_lo) Uf_lo[(int64_t)slot * per + idx] = bf16_lo(v, h);
}

// Row pitch of a gap's P rows in the operator stacks and the staged products: a
// multiple of 16 (each 16-row MFMA output piece of a pair is an aligned 64-byte
// FP32 segment) where that adds at most 1/32, else of 4 (aligned 16-byte stores).
static int row_pitch(int P) {
  const int r16 = (P + 15) / 16 * 16;
  return (r16 - P) * 32 <= P ? r16 : (P + 3) / 4 * 4;
}

// Tile variants of the M2L products: (columns per tile, K step, row blocks per
// wave).  The variant and whether the launch is persistent are chosen by
// timing (autotuning).
constexpr int M2L_VARIANTS = 18;
constexpr int M2L_FIRST_DIRECT = 8;  // variants from here on use m2l_direct_kernel (P % 4 == 0)
constexpr int M2L_FIRST_BF16_LDS = 12;  // BF16 only: moments staged in LDS (8 .. 11's shapes, and 128 columns)
static const int kVariantCols[M2L_VARIANTS] = {128, 64, 64, 32, 32, 32, 64, 32, 32, 32, 64, 64, 32, 32, 64, 64,
                                               128, 128};
static const int kVariantRpw[M2L_VARIANTS] = {2, 2, 2, 2, 2, 4, 4, 4, 2, 4, 2, 4, 2, 4, 2, 4, 2, 4};

template <class T, bool PERS, bool GLEV = false>
static void launch_m2l_tile(int v, int grid, hipStream_t st, int P, int GP, int RB, int KB, const M2LWork& W) {
  switch (v) {
    case 0: m2l_mfma_kernel<T, 8, 16, 2, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 1: m2l_mfma_kernel<T, 4, 16, 2, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 2: m2l_mfma_kernel<T, 4, 32, 2, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 3: m2l_mfma_kernel<T, 2, 16, 2, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 4: m2l_mfma_kernel<T, 2, 32, 2, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 5: m2l_mfma_kernel<T, 2, 16, 4, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 6: m2l_mfma_kernel<T, 4, 16, 4, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 7: m2l_mfma_kernel<T, 2, 32, 4, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 8: m2l_direct_kernel<T, 2, 2, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 9: m2l_direct_kernel<T, 2, 4, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    case 10: m2l_direct_kernel<T, 4, 2, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
    default: m2l_direct_kernel<T, 4, 4, PERS, GLEV><<<grid, 256, 0, st>>>(P, GP, RB, KB, W); break;
  }
}

// BF16 contexts use the tile shapes of variants 8 .. 11 (columns x rows per workgroup), and
// 12 .. 17, those shapes and 128 x 128, 128 x 256 with the moment fragments staged in LDS.
template <bool PERS, bool X3, bool GLEV = false>
static void launch_m2l_bf16_tile(int v, int grid, hipStream_t st, int Pp, int GP, int RB, int KB32, const M2LWork& W) {
  switch (v) {
    case 8: m2l_bf16_kernel<2, 2, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
    case 9: m2l_bf16_kernel<2, 4, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
    case 10: m2l_bf16_kernel<4, 2, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
    case 11: m2l_bf16_kernel<4, 4, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
    case 12: m2l_bf16_lds_kernel<2, 2, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
    case 13: m2l_bf16_lds_kernel<2, 4, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
    case 14: m2l_bf16_lds_kernel<4, 2, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
    case 15: m2l_bf16_lds_kernel<4, 4, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
    case 16: m2l_bf16_lds_kernel<8, 2, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
    default: m2l_bf16_lds_kernel<8, 4, PERS, X3, GLEV><<<grid, 256, 0, st>>>(Pp, GP, RB, KB32, W); break;
  }
}

template <class T>
static void launch_m2l_variant(int v, bool persistent, int grid, hipStream_t st, int P, int GP, int RB, int KB,
                               const M2LWork& W) {
  if (persistent) launch_m2l_tile<T, true>(v, grid, st, P, GP, RB, KB, W);
  else launch_m2l_tile<T, false>(v, grid, st, P, GP, RB, KB, W);
}

// Reduce the staged near-future products per target cell and gap.  Block e takes
// the e-th (cell, gap index g) that has dense blocks (red_cg = cell, g per entry) and
// sums over its pairs red_pairs[red_ptr[e] .. red_ptr[e+1]) (target order), four
// coefficients per thread (Pr is a multiple of 4, rows P .. Pr-1 are zeros), in FP64
// with four partial sums; the sum goes into the local L_{k+g+1}.
template <class ST>
__global__ __launch_bounds__(256) void m2l_reduce_kernel(int P, int Pr, int Gn, int R, int k, int ncell,
                                                         const int32_t* __restrict__ red_cg,
                                                         const int32_t* __restrict__ red_ptr,
                                                         const int32_t* __restrict__ red_pairs,
                                                         const ST* __restrict__ stage, double scale,
                                                         double* __restrict__ ring) {
  typedef ST v4_t __attribute__((ext_vector_type(4)));
  const int e = blockIdx.x;
  const int a0 = 4 * (blockIdx.y * blockDim.x + threadIdx.x);
  if (a0 >= P) return;
  const int O = red_cg[2 * e], g = red_cg[2 * e + 1];
  const int q0 = red_ptr[e], q1 = red_ptr[e + 1];
  const int64_t ld = (int64_t)Gn * Pr;
  const ST* sp = stage + (int64_t)g * Pr + a0;
  double s0[4] = {0, 0, 0, 0}, s1[4] = {0, 0, 0, 0}, s2[4] = {0, 0, 0, 0}, s3[4] = {0, 0, 0, 0};
  int q = q0;
  // FP32 rows: eight in flight (pair q + j goes to partial sum j mod 4); FP64 rows are twice
  // the registers, and four in flight keep the occupancy up
  if constexpr (sizeof(ST) == 4) {
    for (; q + 7 < q1; q += 8) {
      v4_t v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = *reinterpret_cast<const v4_t*>(sp + red_pairs[q + j] * ld);
#pragma unroll
      for (int j = 0; j < 8; j += 4)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          s0[c] += (double)v[j][c];
          s1[c] += (double)v[j + 1][c];
          s2[c] += (double)v[j + 2][c];
          s3[c] += (double)v[j + 3][c];
        }
    }
  }
  for (; q + 3 < q1; q += 4) {
    const v4_t v0 = *reinterpret_cast<const v4_t*>(sp + red_pairs[q] * ld);
    const v4_t v1 = *reinterpret_cast<const v4_t*>(sp + red_pairs[q + 1] * ld);
    const v4_t v2 = *reinterpret_cast<const v4_t*>(sp + red_pairs[q + 2] * ld);
    const v4_t v3 = *reinterpret_cast<const v4_t*>(sp + red_pairs[q + 3] * ld);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      s0[c] += (double)v0[c];
      s1[c] += (double)v1[c];
      s2[c] += (double)v2[c];
      s3[c] += (double)v3[c];
    }
  }
  for (; q < q1; ++q) {
    const v4_t v0 = *reinterpret_cast<const v4_t*>(sp + red_pairs[q] * ld);
#pragma unroll
    for (int c = 0; c < 4; ++c) s0[c] += (double)v0[c];
  }
  double* L = ring + ((int64_t)((k + g + 1) % R) * ncell + O) * P + a0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (a0 + c < P) L[c] += scale * ((s0[c] + s1[c]) + (s2[c] + s3[c]));
}

// Time moments of the completed source interval's moments, per cell:
// S[j][cell][b] = sum_n (ht w_n)^j M[cell][b + Ps n], j = 0..d (ht w_n: the
// source node's time from the interval centre), and their node sums
// Ssum[j][cell] = sum_b S[j][cell][b].  One 64-lane wave per cell.
__global__ __launch_bounds__(64) void m2l_time_moments_kernel(int Ps, int pt, int d, double ht, NodeSet nodes,
                                                              int ncell, const double* __restrict__ mom,
                                                              double* __restrict__ S, double* __restrict__ Ssum) {
  const int cell = blockIdx.x, lane = threadIdx.x;
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = lane; b < Ps; b += 64) {
    const double* M = mom + (int64_t)cell * Ps * pt + b;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int n = 0; n < pt; ++n) {
      const double v = M[(int64_t)Ps * n], tn = ht * nodes.t[n];
      double tp = 1.0;
      for (int j = 0; j <= d; ++j) { acc[j] += tp * v; tp *= tn; }
    }
    for (int j = 0; j <= d; ++j) {
      S[((int64_t)j * ncell + cell) * Ps + b] = acc[j];
      part[j] += acc[j];
    }
  }
  for (int j = 0; j <= d; ++j) {
    double v = part[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) Ssum[(int64_t)j * ncell + cell] = v;
  }
}

// Separable part of M2L.  Wherever c (t - s) - r > 0 at every node pair of an
// offset's cell pair and time gap, the operator entry there is the polynomial
// (c (A_m - B_n) - r_ab)^d / r_ab (no truncation at any node): A_m the target
// node time, B_n = ht w_n the source node time, both from the source interval's
// centre.  The trinomial expansion then gives
//   (U M)[a, m] = sum_{i+j+k=q} q!/(i! j! k!) (c A_m)^i (-c)^j (-1)^k V_{k,j}[a],   q = d,
//   V_{k,j}[a] = sum_b r_ab^{k-1} S_j[b],   S_j[b] = sum_n B_n^j M[b, n],
// with the same V for every such gap, and the derivative products of Algorithm 1,
// L^{(p)}_{k+mu+1,k} = U^{(p)} M (eq. L_l,k; entries C(d,p) (c (A_m - B_n) - r_ab)^{d-p} / r_ab
// at the expansion gap mu+1), follow from the same V with q = d - p.  This is the
// interpolated operator itself, factored: no approximation beyond the paper's.
// The pair products V_{0,j} = K_{1/r} S_j, V_{2,j} = K_r S_j, V_{3,j} = K_{r^2} S_j
// run on the FP64 matrix cores (launch_sep_products); V_{1,j} (kernel r^0) is the
// node sum of S_j.  This kernel, one workgroup per target cell and a thread per
// target node a, walks the near-future gaps g = 1 .. mu+1 in order, adds the V of
// the pairs whose first wavefront-free gap g0 is g, and adds the expansion of the
// running sum into L_{k+g}; after gap mu+1 every pair is in, and the sum gives the
// derivative products.  FP64 throughout.
// V: [product][pair][Psr] (row pitch Psr >= Ps) in the order (0, 0..d), (2, 0..d-2), (3, 0..d-3).
__device__ inline int sep_vidx(int k, int j, int d) {
  return k == 0 ? j : k == 2 ? d + 1 + j : d + 1 + (d - 1) + j;
}

// Wc is indexed with constants only (loops of fixed trip count, q folds in the
// unrolled callers), so it stays in registers.
__device__ __forceinline__ double sep_expand(int q, double cA, double c, const double (&Wc)[4][4]) {
  double val = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j + k > q) continue;
      const int i = q - j - k;
      double coef = 1.0;  // q! / (i! j! k!)
      for (int t = 2; t <= q; ++t) coef *= t;
      for (int t = 2; t <= i; ++t) coef /= t;
      for (int t = 2; t <= j; ++t) coef /= t;
      for (int t = 2; t <= k; ++t) coef /= t;
      double term = coef * ((j + k) & 1 ? -1.0 : 1.0);
      for (int t = 0; t < i; ++t) term *= cA;
      for (int t = 0; t < j; ++t) term *= c;
      val += term * Wc[k][j];
    }
  return val;
}

template <int D>
__global__ void m2l_sep_expand_kernel(int Ps, int Psr, int pt, int mu, int R, int ks, double c, double dt, int Ml,
                                      double ht, NodeSet nodes, int ncell, int64_t npair,
                                      const int32_t* __restrict__ il_ptr, const int32_t* __restrict__ il_src,
                                      const int32_t* __restrict__ pair_gr, const int32_t* __restrict__ sep_order,
                                      const double* __restrict__ V, const double* __restrict__ Ssum,
                                      double* __restrict__ ring, double* __restrict__ dp) {
  const int O = blockIdx.x;
  const int p0 = il_ptr[O], p1 = il_ptr[O + 1];
  const int P = Ps * pt;
  // one pair's terms, loaded before any of them is added (so that several pairs' loads overlap)
  struct Terms { double v[4][4]; };
  auto fetch = [&](int p, int a, Terms& t) {
#pragma unroll
    for (int j = 0; j <= D; ++j) t.v[0][j] = V[((int64_t)sep_vidx(0, j, D) * npair + p) * Psr + a];
#pragma unroll
    for (int j = 0; j + 1 <= D; ++j) t.v[1][j] = Ssum[(int64_t)j * ncell + il_src[p]];
#pragma unroll
    for (int j = 0; j + 2 <= D; ++j) t.v[2][j] = V[((int64_t)sep_vidx(2, j, D) * npair + p) * Psr + a];
#pragma unroll
    for (int j = 0; j + 3 <= D; ++j) t.v[3][j] = V[((int64_t)sep_vidx(3, j, D) * npair + p) * Psr + a];
  };
  for (int a = threadIdx.x; a < Ps; a += blockDim.x) {
    double Wc[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    auto add = [&](const Terms& t) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if ((k == 0 && j <= D) || (k == 1 && j + 1 <= D) || (k >= 2 && j + k <= D)) Wc[k][j] += t.v[k][j];
    };
    // the cell's pairs in order of their first wavefront-free gap g0 (target order within a g0)
    int q = p0;
    for (int g = 1; g <= mu + 1; ++g) {
      int qe = q;
      while (qe < p1 && (pair_gr[sep_order[qe]] >> 16) == g) ++qe;
      for (; q + 1 < qe; q += 2) {
        Terms t0, t1;
        fetch(sep_order[q], a, t0);
        fetch(sep_order[q + 1], a, t1);
        add(t0);
        add(t1);
      }
      if (q < qe) {
        Terms t0;
        fetch(sep_order[q], a, t0);
        add(t0);
        ++q;
      }
      if (q == p0) continue;  // no pair added yet (the same for every thread)
      double* L = ring + ((int64_t)((ks + g) % R) * ncell + O) * P + a;
      for (int m = 0; m < pt; ++m) {
        const double cA = c * ((g * (double)Ml + 1.0) * dt + ht * nodes.t[m]);
        L[(int64_t)Ps * m] += sep_expand(D, cA, c, Wc);
      }
    }
    // derivative products at the expansion gap mu+1: every pair is in Wc
#pragma unroll
    for (int pp = 1; pp <= D; ++pp) {
      double binom = 1.0;
      for (int t = 0; t < pp; ++t) binom = binom * (D - t) / (t + 1);
      for (int m = 0; m < pt; ++m) {
        const double cA = c * (((mu + 1) * (double)Ml + 1.0) * dt + ht * nodes.t[m]);
        dp[((int64_t)(pp - 1) * ncell + O) * P + a + (int64_t)Ps * m] = binom * sep_expand(D - pp, cA, c, Wc);
      }
    }
  }
}

// Recurrence of Algorithm 1 for source interval k, per (cell, coefficient):
// eq. m2l_expand_rec1 (derivatives L^{(p)}, using the auxiliaries L^{(p,m)} of
// k-1 with the coefficients c_m^p(k) of eq. cmp), eq. m2l_rec (local of interval
// k+mu+2), eq. m2l_expand_rec2 (auxiliaries += L^{(p)}_{k+mu+1,k} k^m).
// d <= 3: auxiliaries (p, m) = (2, 0), (3, 0), (3, 1) stored at (p-1)(p-2)/2 + m.
__device__ inline double cmp_coef(int p, int m, double k) {
  double bin = 1.0;
  for (int q = 0; q < m; ++q) bin = bin * (p - q) / (q + 1);
  const int e = p - m;
  double km1 = 1.0, k0 = 1.0, kp1 = 1.0;
  for (int q = 0; q < e; ++q) { km1 *= k - 1.0; k0 *= k; kp1 *= k + 1.0; }
  return bin * (km1 - 2.0 * k0 + kp1) * ((m & 1) ? -1.0 : 1.0);
}

__global__ void m2l_recurrence_kernel(int P, int mu, int d, int R, int k, double T, int ncell,
                                      const double* __restrict__ dp, double* __restrict__ ring,
                                      double* __restrict__ lp, double* __restrict__ aux) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)ncell * P;
  if (idx >= n) return;
  const double kd = (double)k;
  double Lnew[4] = {0, 0, 0, 0};
  for (int q = 1; q <= d; ++q) {
    double v = lp[(q - 1) * n + idx] + dp[(q - 1) * n + idx];
    for (int m = 0; m <= q - 2; ++m) v += cmp_coef(q, m, kd) * aux[((q - 1) * (q - 2) / 2 + m) * n + idx];
    Lnew[q] = v;
    lp[(q - 1) * n + idx] = v;
  }
  double next = ring[(int64_t)((k + mu + 1) % R) * n + idx];
  double Tp = 1.0;
  for (int q = 1; q <= d; ++q) { Tp *= T; next += Lnew[q] * Tp; }
  ring[(int64_t)((k + mu + 2) % R) * n + idx] = next;
  for (int q = 2; q <= d; ++q) {
    double km = 1.0;
    for (int m = 0; m <= q - 2; ++m) {
      aux[((q - 1) * (q - 2) / 2 + m) * n + idx] += dp[(q - 1) * n + idx] * km;
      km *= kd;
    }
  }
}

// L2P: far field at (x_i, t_alpha) from the leaf local of the current interval.
// One 64-lane wave per leaf cell: lane a takes basis functions a, a + 64, ...;
// the local is combined in time once per leaf (value and time derivative), then
// every element of the leaf takes a coalesced dot product with its table row.
constexpr int L2P_MAXA = (MAXP * MAXP * MAXP + 63) / 64;
__global__ __launch_bounds__(64) void l2p_kernel(int Ps, int pt, int bie, double inv_c, TimeWeights tw,
                                                 const int32_t* __restrict__ leaf_ptr,
                                                 const int32_t* __restrict__ leaf_elems, const double* __restrict__ E0,
                                                 const double* __restrict__ E1, const double* __restrict__ L,
                                                 double* __restrict__ out) {
  const int leaf = blockIdx.x, lane = threadIdx.x;
  const int e_begin = leaf_ptr[leaf], e_end = leaf_ptr[leaf + 1];
  if (e_begin == e_end) return;
  const double* Lc = L + (int64_t)leaf * Ps * pt;
  double lw[L2P_MAXA], ldw[L2P_MAXA];
#pragma unroll
  for (int t = 0; t < L2P_MAXA; ++t) {
    const int a = lane + 64 * t;
    double v0 = 0.0, v1 = 0.0;
    if (a < Ps)
      for (int m = 0; m < pt; ++m) {
        const double v = Lc[a + Ps * m];
        v0 += v * tw.w[m];
        v1 += v * tw.dw[m];
      }
    lw[t] = v0;
    ldw[t] = v1;
  }
  for (int e = e_begin; e < e_end; ++e) {
    const int el = leaf_elems[e];
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < L2P_MAXA; ++t) {
      const int a = lane + 64 * t;
      if (a < Ps) {
        if (bie) s += E1[(int64_t)el * Ps + a] * lw[t] - inv_c * E0[(int64_t)el * Ps + a] * ldw[t];
        else s += E0[(int64_t)el * Ps + a] * lw[t];
      }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) out[el] += s;
  }
}

// ---------------------------------------------------------------------------
// Set-up

static void build_tree(tdbem_ctx* ctx, Fmm* f) {
  const Geometry& g = ctx->geo;
  double ext = 0.0;
  for (int k = 0; k < 3; ++k) {
    f->center[k] = 0.5 * (g.ext_lo[k] + g.ext_hi[k]);
    ext = std::max(ext, 0.5 * (g.ext_hi[k] - g.ext_lo[k]));
  }
  if (!(ext > 0.0)) throw Error(TDBEM_E_INVAL, "degenerate mesh extent");
  if (f->leaf_ratio > 0.0) {
    // leaf half side leaf_ratio * c dt / 2; the fewest levels whose root holds the mesh
    const double hl = 0.5 * f->leaf_ratio * ctx->cdt;
    int D = 2;
    while (D < 12 && hl * (double)(1 << D) < ext) ++D;
    if (hl * (double)(1 << D) < ext) throw Error(TDBEM_E_INVAL, "leaf_ratio too small for this mesh (depth > 12)");
    f->D = D;
    f->H = hl * (double)(1 << D);
  } else {
    f->H = std::pow(2.0, std::ceil(std::log2(ext)));
  }
  const int ns = g.ns, D = f->D;
  f->e_max = g.e_max;
  const int n = 1 << D;
  std::vector<std::array<int, 3>> li(ns);
  for (int e = 0; e < ns; ++e)
    for (int k = 0; k < 3; ++k) {
      int v = (int)std::floor((g.xc[3 * e + k] - (f->center[k] - f->H)) / (2.0 * f->H) * n);
      li[e][k] = std::min(std::max(v, 0), n - 1);
    }
  f->lev.assign(D + 1, FmmLevel());
  std::vector<std::vector<int>> cell_of(D + 1, std::vector<int>(ns));
  for (int l = 0; l <= D; ++l) {
    FmmLevel& L = f->lev[l];
    std::vector<std::pair<uint64_t, std::array<int, 3>>> ks;
    ks.reserve(ns);
    for (int e = 0; e < ns; ++e) {
      std::array<int, 3> k3 = {li[e][0] >> (D - l), li[e][1] >> (D - l), li[e][2] >> (D - l)};
      ks.push_back({morton(k3[0], k3[1], k3[2]), k3});
    }
    std::sort(ks.begin(), ks.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    ks.erase(std::unique(ks.begin(), ks.end(), [](const auto& a, const auto& b) { return a.first == b.first; }),
             ks.end());
    L.ncell = (int)ks.size();
    std::unordered_map<int64_t, int> pos;
    for (int i = 0; i < L.ncell; ++i) {
      L.key.push_back(ks[i].second);
      pos[key64(ks[i].second[0], ks[i].second[1], ks[i].second[2])] = i;
    }
    for (int e = 0; e < ns; ++e)
      cell_of[l][e] = pos[key64(li[e][0] >> (D - l), li[e][1] >> (D - l), li[e][2] >> (D - l))];
    if (l >= 1) {
      std::unordered_map<int64_t, int> ppos;
      const FmmLevel& Pl = f->lev[l - 1];
      for (int i = 0; i < Pl.ncell; ++i) ppos[key64(Pl.key[i][0], Pl.key[i][1], Pl.key[i][2])] = i;
      L.parent.resize(L.ncell);
      L.octant.resize(L.ncell);
      for (int i = 0; i < L.ncell; ++i) {
        const auto& k = L.key[i];
        L.parent[i] = ppos[key64(k[0] >> 1, k[1] >> 1, k[2] >> 1)];
        L.octant[i] = (k[0] & 1) | ((k[1] & 1) << 1) | ((k[2] & 1) << 2);
      }
    }
    // interaction lists
    if (l >= 2) {
      std::unordered_map<int64_t, int> slot_of;
      L.il_ptr.assign(L.ncell + 1, 0);
      for (int O = 0; O < L.ncell; ++O) {
        const auto& k = L.key[O];
        const int px = k[0] >> 1, py = k[1] >> 1, pz = k[2] >> 1;
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz)
              for (int cx = 0; cx < 2; ++cx)
                for (int cy = 0; cy < 2; ++cy)
                  for (int cz = 0; cz < 2; ++cz) {
                    const int sx = 2 * (px + dx) + cx, sy = 2 * (py + dy) + cy, sz = 2 * (pz + dz) + cz;
                    const int ox = sx - k[0], oy = sy - k[1], oz = sz - k[2];
                    if (std::max({std::abs(ox), std::abs(oy), std::abs(oz)}) <= 1) continue;
                    auto it = pos.find(key64(sx, sy, sz));
                    if (sx < 0 || sy < 0 || sz < 0 || it == pos.end()) continue;
                    const int64_t ok = key64(ox + 8, oy + 8, oz + 8);
                    auto st = slot_of.find(ok);
                    int slot;
                    if (st == slot_of.end()) {
                      slot = (int)L.slot_off.size();
                      slot_of[ok] = slot;
                      L.slot_off.push_back({ox, oy, oz});
                    } else {
                      slot = st->second;
                    }
                    L.il_src.push_back(it->second);
                    L.il_slot.push_back(slot);
                  }
        L.il_ptr[O + 1] = (int)L.il_src.size();
      }
      L.npair = (int64_t)L.il_src.size();
    }
  }
  // leaf membership
  f->leaf_of = cell_of[D];
  const int nl = f->lev[D].ncell;
  f->leaf_ptr.assign(nl + 1, 0);
  for (int e = 0; e < ns; ++e) f->leaf_ptr[f->leaf_of[e] + 1]++;
  for (int i = 0; i < nl; ++i) f->leaf_ptr[i + 1] += f->leaf_ptr[i];
  f->leaf_elems.resize(ns);
  std::vector<int> fill(f->leaf_ptr.begin(), f->leaf_ptr.end() - 1);
  for (int e = 0; e < ns; ++e) f->leaf_elems[fill[f->leaf_of[e]]++] = e;
}

static void build_hierarchy(tdbem_ctx* ctx, Fmm* f) {
  const double cdt = ctx->cdt;
  const int m_leaf = (int)std::floor((2.0 * hs_of(f, f->D) - f->e_max) / cdt);
  if (m_leaf < 1)
    throw Error(TDBEM_E_INVAL, "octree too deep for this time step: leaves must be wider than c*dt plus the "
                               "largest centroid-to-vertex distance");
  f->m_leaf = m_leaf;
  // smallest mu with c (t - s) - r > 0 for every node pair of interval k+mu+1, every level and offset
  // (normalised operators: lengths in units of c dt and times in units of dt, so that
  // every context with the same normalised hierarchy finds the same mu)
  const bool nrm = f->leaf_ratio > 0.0;
  const double cc = nrm ? 1.0 : ctx->c, dtt = nrm ? 1.0 : ctx->dt;
  int need = 1;
  for (int l = 2; l <= f->D; ++l) {
    const double Ml = (double)m_leaf * (1 << (f->D - l)), ht = Ml * dtt / 2.0;
    const double hs = nrm ? 0.5 * f->leaf_ratio * (double)(1 << (f->D - l)) : hs_of(f, l);
    double smin = 1e300, smax = -1e300, tmin = 1e300;
    for (int a = 0; a < f->ps; ++a) { smin = std::min(smin, f->om_s[a]); smax = std::max(smax, f->om_s[a]); }
    for (int m = 0; m < f->pt; ++m)
      for (int n = 0; n < f->pt; ++n) tmin = std::min(tmin, f->om_t[m] - f->om_t[n]);
    // largest node distance over all 316 offsets: offset 3 per axis, node spread (smax - smin)
    const double ax = 6.0 * hs + hs * (smax - smin);
    const double rmax = std::sqrt(3.0) * ax;
    int m = 1;
    while (cc * (((m + 1) * Ml + 1.0) * dtt + ht * tmin) - rmax <= 0.0) ++m;
    need = std::max(need, m);
  }
  if (ctx->opts.mu > 0 && ctx->opts.mu < need)
    throw Error(TDBEM_E_INVAL, "mu too small for this hierarchy (need " + std::to_string(need) + ")");
  f->mu = ctx->opts.mu > 0 ? ctx->opts.mu : need;
  f->G = f->mu + 1 + ctx->d;
  f->Gn = f->mu + 1;
  f->R = f->mu + 3;
}

static QuadRule gauss_legendre01(int n) {
  QuadRule q;
  q.n = n;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
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
    q.x[i] = 0.5 * (x + 1.0);
    q.w[i] = 0.5 * 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return q;
}

template <class T>
static void upload(DevBuf<T>& buf, const std::vector<T>& v, hipStream_t s) {
  buf.alloc(v.size());
  if (!v.empty()) TDBEM_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Levels D, D-1, ..., D-n+1 end a source interval together (n = 1..D-1): one
// launch does their near-future products.  choice = 2 * variant + persistent.
static int cols_index(int cols) { return cols == 128 ? 0 : cols == 64 ? 1 : 2; }

// The work descriptor of level l for tile variant v; false if the level has no items.
static bool level_work(const Fmm* f, int l, int v, int item0, M2LLevelWork& Lw, int& nitems) {
  const bool lo = f->prec == 1, b16 = f->prec >= 2, x3 = f->prec == 3;
  const int rows = 64 * kVariantRpw[v];
  const int cols = kVariantCols[v], ci = cols_index(cols), ri = rows == 128 ? 0 : 1;
  const FmmLevel& L = f->lev[l];
  if (L.npair == 0 || L.nitems[ci][ri] == 0) return false;
  Lw = M2LLevelWork{};
  {
    Lw.ntiles = cols == 128 ? L.ntiles128 : cols == 64 ? L.ntiles64 : L.ntiles32;
    Lw.tiles = cols == 128 ? L.d_tiles128.p : cols == 64 ? L.d_tiles64.p : L.d_tiles32.p;
    Lw.pairs_by_slot = L.d_pairs_by_slot.p;
    Lw.src_by_slot = L.d_src_by_slot.p;
    Lw.mom = L.d_mom.p;
    Lw.mom32 = L.d_mom32.p;
    Lw.mom16 = L.d_mom16.p;
    const LevelOps& ops = *L.ops;
    if (x3) {  // second terms after the first (same layouts)
      Lw.Uf_lo = ops.U16.p + ops.tot;
      Lw.mom16_lo = L.d_mom16.p + L.d_mom16.n / 2;
    }
    if (lo) { Lw.Uf = ops.U32.p; Lw.stage = L.d_stage32.p; }
    else if (b16) { Lw.Uf = ops.U16.p; Lw.stage = L.d_stage32.p; }
    else { Lw.Uf = ops.Uf.p; Lw.stage = L.d_stage.p; }
    Lw.items = L.d_items[ci][ri].p;
    Lw.uoff = L.d_uoff.p;
    Lw.srows = L.d_srows.p;
    Lw.soff = L.d_soff.p;
    Lw.item0 = item0;
    nitems = L.nitems[ci][ri];
  }
  return true;
}

// Launch of a filled work descriptor (tile variant and persistence from choice).
static void launch_m2l_work(const Fmm* f, int choice, const M2LWork& W, hipStream_t st) {
  const int P = f->P, G = f->Gn, GP = G * f->Pr;
  const bool lo = f->prec == 1, b16 = f->prec >= 2, x3 = f->prec == 3;
  const int v = choice >> 1, persistent = choice & 1;
  const int RB = (GP + 15) / 16, KB = m2l_kblocks(P);
  const int total = W.total;
  if (total == 0) return;
  if (W.glev) {  // several contexts: one item per workgroup, descriptors from the device table
    if (b16) {
      const int KB32 = (P + 31) / 32;
      if (x3) launch_m2l_bf16_tile<false, true, true>(v, total, st, f->Pp, GP, RB, KB32, W);
      else launch_m2l_bf16_tile<false, false, true>(v, total, st, f->Pp, GP, RB, KB32, W);
    } else if (lo) launch_m2l_tile<float, false, true>(v, total, st, P, GP, RB, KB, W);
    else launch_m2l_tile<double, false, true>(v, total, st, P, GP, RB, KB, W);
    TDBEM_HIP(hipGetLastError());
    return;
  }
  const bool pers = persistent && total > f->persistent_grid;
  const int grid = pers ? f->persistent_grid : total;
  if (b16) {
    const int KB32 = (P + 31) / 32;
    if (x3) {
      if (pers) launch_m2l_bf16_tile<true, true>(v, grid, st, f->Pp, GP, RB, KB32, W);
      else launch_m2l_bf16_tile<false, true>(v, grid, st, f->Pp, GP, RB, KB32, W);
    } else {
      if (pers) launch_m2l_bf16_tile<true, false>(v, grid, st, f->Pp, GP, RB, KB32, W);
      else launch_m2l_bf16_tile<false, false>(v, grid, st, f->Pp, GP, RB, KB32, W);
    }
  } else if (lo) launch_m2l_variant<float>(v, pers, grid, st, P, GP, RB, KB, W);
  else launch_m2l_variant<double>(v, pers, grid, st, P, GP, RB, KB, W);
  TDBEM_HIP(hipGetLastError());
}

static void launch_m2l_levels(const Fmm* f, int n, int choice, hipStream_t st) {
  M2LWork W{};
  int total = 0;
  for (int l = f->D; l > f->D - n && l >= 2; --l) {
    int ni = 0;
    if (level_work(f, l, choice >> 1, total, W.lev[W.nlev], ni)) {
      ++W.nlev;
      total += ni;
    }
  }
  W.total = total;
  launch_m2l_work(f, choice, W, st);
}

// Separable pair products of one level (see m2l_sep_expand_kernel):
// V_{0,j} = K_{1/r} S_j, V_{2,j} = K_r S_j, V_{3,j} = K_{r^2} S_j, FP64 on the
// matrix cores with the near-future products' tiles (32 pairs of one offset,
// LDS-staged time moments), each product a "level" of one launch.
static void launch_sep_products(const Fmm* f, const FmmLevel& L, int d, hipStream_t st) {
  const int Ps = f->Ps, nslot = (int)L.slot_off.size();
  const int RBk = (Ps + 15) / 16, KBk = m2l_kblocks(Ps);
  const int64_t perk = (int64_t)RBk * KBk * 64;
  const int nrb = (Ps + 127) / 128;  // 128 operator rows per workgroup (tile 32 x 16 x 128)
  M2LWork W{};
  int total = 0;
  // products in the order of sep_vidx: (K_{1/r}, S_0..S_d), (K_r, S_0..S_{d-2}), (K_{r^2}, S_0..S_{d-3})
  int vk[8], vj[8], nv = 0;
  for (int j = 0; j <= d; ++j) { vk[nv] = 0; vj[nv++] = j; }
  for (int j = 0; j + 2 <= d; ++j) { vk[nv] = 1; vj[nv++] = j; }
  for (int j = 0; j + 3 <= d; ++j) { vk[nv] = 2; vj[nv++] = j; }
  for (int v = 0; v < nv; ++v) {
    M2LLevelWork& Lw = W.lev[W.nlev++];
    const int j = vj[v], kern = vk[v];
    Lw.ntiles = L.ntiles32;
    Lw.tiles = L.d_tiles32.p;
    Lw.pairs_by_slot = L.d_pairs_by_slot.p;
    Lw.src_by_slot = L.d_src_by_slot.p;
    Lw.mom = L.d_tm.p + (int64_t)j * L.ncell * Ps;
    Lw.mom32 = nullptr;
    Lw.mom16 = nullptr;
    Lw.Uf = L.d_Ktf.p + (int64_t)kern * nslot * perk;
    Lw.stage = L.d_V.p + (int64_t)v * L.npair * f->Psr;
    Lw.item0 = total;
    total += Lw.ntiles * nrb;
  }
  W.total = total;
  if (total == 0) return;
  // rows Ps .. Psr-1 of a pair (zero operator rows) are written too
  m2l_mfma_kernel<double, 2, 16, 2, false><<<total, 256, 0, st>>>(Ps, f->Psr, RBk, KBk, W);
  TDBEM_HIP(hipGetLastError());
}

// Autotuner table shared by all contexts of the process: the fastest
// (tile variant, persistent) for a launch, keyed by operator size P, blocks G,
// precision, levels in the launch and the work size in powers of two.
struct M2LKey {
  int P, G, f32, nlev, bucket;
  bool operator<(const M2LKey& o) const {
    return std::tie(P, G, f32, nlev, bucket) < std::tie(o.P, o.G, o.f32, o.nlev, o.bucket);
  }
};
static std::mutex g_tune_mu;
static std::map<M2LKey, int> g_tune_table;

static int m2l_work_items(const Fmm* f, int n, int v) {
  const int ci = cols_index(kVariantCols[v]), ri = kVariantRpw[v] == 2 ? 0 : 1;
  int total = 0;
  for (int l = f->D; l > f->D - n && l >= 2; --l) total += f->lev[l].nitems[ci][ri];
  return total;
}

static void autotune_m2l(Fmm* f, hipStream_t st) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  for (int n = 1; n <= f->D - 1; ++n) {
    const int items = m2l_work_items(f, n, 1);
    int bucket = 0;
    while ((1 << bucket) < items) ++bucket;
    const M2LKey key{f->P, f->Gn, f->prec, n, bucket};
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_table.find(key);
      if (it != g_tune_table.end()) { f->m2l_choice[n] = it->second; continue; }
    }
    if (!e0) {
      TDBEM_HIP(hipEventCreate(&e0));
      TDBEM_HIP(hipEventCreate(&e1));
    }
    float best = 1e30f;
    int bestc = f->prec >= 2 ? 2 * M2L_FIRST_DIRECT : 2;  // 64 x 16 x 128 (BF16: 32 x 128), one item per workgroup
    for (int c = 0; c < 2 * M2L_VARIANTS; ++c) {
      if ((c & 1) && m2l_work_items(f, n, c >> 1) <= f->persistent_grid) continue;
      if ((c >> 1) >= M2L_FIRST_DIRECT && f->P % 4 != 0 && f->prec < 2) continue;
      if ((c >> 1) >= M2L_FIRST_BF16_LDS && f->prec < 2) continue;
      if ((c >> 1) < M2L_FIRST_DIRECT && f->prec >= 2) continue;  // BF16: the four LDS-free shapes
      launch_m2l_levels(f, n, c, st);  // warm-up
      TDBEM_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < 2; ++r) launch_m2l_levels(f, n, c, st);
      TDBEM_HIP(hipEventRecord(e1, st));
      TDBEM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      TDBEM_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) { best = ms; bestc = c; }
    }
    f->m2l_choice[n] = bestc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_table[key] = bestc;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
}

// Gap range of each slot's dense blocks: gap g (1..mu+1) of an offset is zero at
// every node pair while c (t - s) <= r there (g < gf), a polynomial at every node
// pair once c (t - s) > r everywhere (g >= g0), and a dense block in between, with
// the node coordinates of m2l_matrix_kernel (lengths and times in the units of c, dt, hs).
static void gap_ranges(const Fmm* f, const std::vector<std::array<int, 3>>& slots, double c, double dt, double hs,
                       double Ml, std::vector<int>& gfv, std::vector<int>& g0v) {
  const int nslot = (int)slots.size(), ps = f->ps, Ps = f->Ps;
  const double ht = Ml * dt / 2.0;
  double dmin = 1e300, dmax = -1e300;
  for (int m = 0; m < f->pt; ++m)
    for (int n = 0; n < f->pt; ++n) {
      dmin = std::min(dmin, f->om_t[m] - f->om_t[n]);
      dmax = std::max(dmax, f->om_t[m] - f->om_t[n]);
    }
  gfv.assign(nslot, 1);
  g0v.assign(nslot, 1);
  for (int sl = 0; sl < nslot; ++sl) {
    double rmin = 1e300, rmax = 0.0;
    const auto& o = slots[sl];
    for (int a = 0; a < Ps; ++a)
      for (int b = 0; b < Ps; ++b) {
        const int aa[3] = {a % ps, (a / ps) % ps, a / (ps * ps)}, bb[3] = {b % ps, (b / ps) % ps, b / (ps * ps)};
        double r2 = 0.0;
        for (int q = 0; q < 3; ++q) {
          const double dq = 2.0 * hs * o[q] + hs * (f->om_s[bb[q]] - f->om_s[aa[q]]);
          r2 += dq * dq;
        }
        const double r = std::sqrt(r2);
        rmin = std::min(rmin, r);
        rmax = std::max(rmax, r);
      }
    int gf = f->mu + 2, g0 = f->mu + 2;
    for (int g = f->mu + 1; g >= 1; --g) {
      const double t0 = (g * Ml + 1.0) * dt;
      if (c * (t0 + ht * dmax) - rmin > 0.0) gf = g;
      if (c * (t0 + ht * dmin) - rmax > 0.0) g0 = g;
    }
    if (g0 > f->mu + 1) throw Error(TDBEM_E_INVAL, "expansion gap not past the wavefront for some offset");
    gfv[sl] = std::min(gf, g0);
    g0v[sl] = g0;
  }
}

// The dense operators of ops.slots at one level: gap ranges, then each slot's FP64
// (mu+1)-block stack built in a one-slot buffer and its dense rows converted to the
// products' precision and fragment order (no copy of the whole level in FP64).
static void build_level_ops(const tdbem_ctx* ctx, const Fmm* f, LevelOps& ops, double c, double dt, double hs,
                            double Ml, hipStream_t st) {
  const int P = f->P, Pr = f->Pr, G = f->Gn, nslot = (int)ops.slots.size();
  gap_ranges(f, ops.slots, c, dt, hs, Ml, ops.gf, ops.g0);
  const int KB = m2l_kblocks(P), KB32 = (P + 31) / 32;
  ops.uoff.assign(nslot + 1, 0);
  for (int sl = 0; sl < nslot; ++sl) {
    const int rows = (ops.g0[sl] - ops.gf[sl]) * Pr, RBs = (rows + 15) / 16;
    ops.uoff[sl + 1] = ops.uoff[sl] + (f->prec >= 2 ? (int64_t)RBs * KB32 * 512 : (int64_t)RBs * KB * 64);
  }
  ops.tot = std::max<int64_t>(ops.uoff[nslot], 1);
  const size_t tot = (size_t)ops.tot;
  if (f->prec >= 2) ops.U16.alloc((f->prec == 3 ? 2 : 1) * tot);  // split products: second terms after tot
  else if (f->prec == 1) ops.U32.alloc(tot);
  else ops.Uf.alloc(tot);
  std::vector<int32_t> so;
  for (auto& v : ops.slots) { so.push_back(v[0]); so.push_back(v[1]); so.push_back(v[2]); }
  DevBuf<int32_t> d_so;
  upload(d_so, so, st);
  DevBuf<double> d_U;  // one slot's (mu+1) P x P near-future operators
  d_U.alloc((size_t)G * P * P);
  for (int sl = 0; sl < nslot; ++sl) {
    const int rows = (ops.g0[sl] - ops.gf[sl]) * Pr, RBs = (rows + 15) / 16, row0 = (ops.gf[sl] - 1) * P;
    if (rows == 0) continue;
    dim3 grid((unsigned)(((int64_t)P * P + 255) / 256), G, 1);
    m2l_matrix_kernel<<<grid, 256, 0, st>>>(f->ps, f->pt, P, G, f->mu, ctx->d, c, hs, Ml * dt / 2.0, dt, (int)Ml,
                                            f->nodes, d_so.p + 3 * sl, d_U.p);
    TDBEM_HIP(hipGetLastError());
    const int64_t n = ops.uoff[sl + 1] - ops.uoff[sl];
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (f->prec >= 2)
      to_fragments_bf16_kernel<<<nb, 256, 0, st>>>(P, Pr, G * P, row0, rows, RBs, KB32, d_U.p, ops.U16.p + ops.uoff[sl],
                                                   f->prec == 3 ? ops.U16.p + tot + ops.uoff[sl] : nullptr);
    else if (f->prec == 1)
      to_fragments_kernel<float><<<nb, 256, 0, st>>>(P, Pr, G * P, row0, rows, RBs, KB, d_U.p,
                                                     ops.U32.p + ops.uoff[sl]);
    else
      to_fragments_kernel<double><<<nb, 256, 0, st>>>(P, Pr, G * P, row0, rows, RBs, KB, d_U.p,
                                                      ops.Uf.p + ops.uoff[sl]);
    TDBEM_HIP(hipGetLastError());
  }
  TDBEM_HIP(hipStreamSynchronize(st));  // the one-slot buffer and d_so are released at return
}

// The 316 interaction-list offsets (cells one box apart excluded), in a fixed order.
static const std::vector<std::array<int, 3>>& all_offsets() {
  static const std::vector<std::array<int, 3>> v = [] {
    std::vector<std::array<int, 3>> o;
    for (int x = -3; x <= 3; ++x)
      for (int y = -3; y <= 3; ++y)
        for (int z = -3; z <= 3; ++z)
          if (std::max({std::abs(x), std::abs(y), std::abs(z)}) >= 2) o.push_back({x, y, z});
    return o;
  }();
  return v;
}

// Normalised operator sets shared between contexts: (device, p_s, p_t, interp, d, mu,
// precision, M_l, h_s / (c dt)).  The map holds no reference: a set lives while a context uses it.
typedef std::tuple<int, int, int, int, int, int, int, int, double> OpsKey;
static std::mutex g_ops_mu;
static std::map<OpsKey, std::weak_ptr<LevelOps>> g_ops_cache;

// The level's operators: its own set in physical units, or (opts.leaf_ratio > 0) the
// normalised set of the 316 offsets shared with every context that agrees on the key.
static void level_ops(const tdbem_ctx* ctx, Fmm* f, int l, hipStream_t st) {
  FmmLevel& L = f->lev[l];
  const double Ml = (double)f->m_leaf * (1 << (f->D - l));
  const int nslot = (int)L.slot_off.size();
  L.canon.assign(nslot, 0);
  if (f->leaf_ratio > 0.0) {
    const double hsn = 0.5 * f->leaf_ratio * (double)(1 << (f->D - l));  // h_s / (c dt), exact
    int dev = 0;
    TDBEM_HIP(hipGetDevice(&dev));
    const OpsKey key{dev, f->ps, f->pt, f->interp, ctx->d, f->mu, f->prec, (int)Ml, hsn};
    std::lock_guard<std::mutex> lk(g_ops_mu);
    L.ops = g_ops_cache[key].lock();
    if (!L.ops) {
      L.ops = std::make_shared<LevelOps>();
      L.ops->slots = all_offsets();
      build_level_ops(ctx, f, *L.ops, 1.0, 1.0, hsn, Ml, st);
      g_ops_cache[key] = L.ops;
    }
    const auto& all = all_offsets();
    for (int sl = 0; sl < nslot; ++sl)
      L.canon[sl] = (int)(std::find(all.begin(), all.end(), L.slot_off[sl]) - all.begin());
  } else {
    L.ops = std::make_shared<LevelOps>();
    L.ops->slots = L.slot_off;
    build_level_ops(ctx, f, *L.ops, ctx->c, ctx->dt, hs_of(f, l), Ml, st);
    for (int sl = 0; sl < nslot; ++sl) L.canon[sl] = sl;
  }
}

// Per context, from the level's operator set: each slot's gap range, dense rows and
// operator offset, the per-pair gap ranges in target order, and the work items of the
// dense products (each slot's gaps gf .. g0-1).
static void classify_gaps(const tdbem_ctx* ctx, Fmm* f, int l, const std::vector<int32_t>& tiles128,
                          const std::vector<int32_t>& tiles64, const std::vector<int32_t>& tiles32, hipStream_t st) {
  (void)ctx;
  FmmLevel& L = f->lev[l];
  const int nslot = (int)L.slot_off.size(), Pr = f->Pr;
  const LevelOps& ops = *L.ops;
  L.gf.assign(nslot, 1);
  L.g0.assign(nslot, 1);
  std::vector<int32_t> srows(std::max(nslot, 1), 0), soff(std::max(nslot, 1), 0);
  std::vector<int64_t> uoff(std::max(nslot, 1), 0);
  for (int sl = 0; sl < nslot; ++sl) {
    const int c = L.canon[sl];
    L.gf[sl] = ops.gf[c];
    L.g0[sl] = ops.g0[c];
    srows[sl] = (L.g0[sl] - L.gf[sl]) * Pr;
    soff[sl] = (L.gf[sl] - 1) * Pr;
    uoff[sl] = ops.uoff[c];
  }
  upload(L.d_srows, srows, st);
  upload(L.d_soff, soff, st);
  upload(L.d_uoff, uoff, st);
  std::vector<int32_t> gr(std::max<int64_t>(L.npair, 1), 0);
  L.dense_blocks = 0;
  for (int64_t p = 0; p < L.npair; ++p) {
    const int sl = L.il_slot[p];
    gr[p] = L.gf[sl] | (L.g0[sl] << 16);
    L.dense_blocks += L.g0[sl] - L.gf[sl];
  }
  upload(L.d_pair_gr, gr, st);
  {  // each target cell's pairs in order of g0, target order within one g0
    std::vector<int32_t> order(std::max<int64_t>(L.npair, 1), 0);
    for (int O = 0; O < L.ncell; ++O) {
      const int b = L.il_ptr[O], e = L.il_ptr[O + 1];
      for (int p = b; p < e; ++p) order[p] = p;
      std::stable_sort(order.begin() + b, order.begin() + e,
                       [&](int x, int y) { return L.g0[L.il_slot[x]] < L.g0[L.il_slot[y]]; });
    }
    upload(L.d_sep_order, order, st);
  }
  {
    std::vector<int32_t> cg, rptr(1, 0), rp;
    rp.reserve((size_t)L.dense_blocks);
    for (int O = 0; O < L.ncell; ++O)
      for (int g = 0; g < f->Gn; ++g) {
        const size_t before = rp.size();
        for (int p = L.il_ptr[O]; p < L.il_ptr[O + 1]; ++p) {
          const int sl = L.il_slot[p];
          if (g + 1 >= L.gf[sl] && g + 1 < L.g0[sl]) rp.push_back(p);
        }
        if (rp.size() == before) continue;
        cg.push_back(O);
        cg.push_back(g);
        rptr.push_back((int32_t)rp.size());
      }
    L.nred = (int)rptr.size() - 1;
    if (rp.empty()) rp.push_back(0);
    if (cg.empty()) cg.assign(2, 0);
    upload(L.d_red_cg, cg, st);
    upload(L.d_red_ptr, rptr, st);
    upload(L.d_red_pairs, rp, st);
  }
  const std::vector<int32_t>* tl[3] = {&tiles128, &tiles64, &tiles32};
  for (int ci = 0; ci < 3; ++ci)
    for (int ri = 0; ri < 2; ++ri) {
      const int rows = ri == 0 ? 128 : 256;
      const std::vector<int32_t>& t = *tl[ci];
      const int nt = (int)t.size() / 3;
      int maxrb = 0;
      for (int sl = 0; sl < nslot; ++sl) maxrb = std::max(maxrb, (srows[sl] + rows - 1) / rows);
      std::vector<int32_t> items;
      for (int rb = 0; rb < maxrb; ++rb)
        for (int ti = 0; ti < nt; ++ti)
          if (rb < (srows[t[3 * ti]] + rows - 1) / rows) {
            items.push_back(ti);
            items.push_back(rb);
          }
      L.nitems[ci][ri] = (int)items.size() / 2;
      if (items.empty()) items.assign(2, 0);
      upload(L.d_items[ci][ri], items, st);
    }
}

Fmm* fmm_create(tdbem_ctx* ctx) {
  const tdbem_opts& o = ctx->opts;
  if (!(o.leaf_ratio >= 0.0)) throw Error(TDBEM_E_INVAL, "leaf_ratio must be >= 0");
  if (o.leaf_ratio == 0.0 && (o.depth < 2 || o.depth > 12)) throw Error(TDBEM_E_INVAL, "depth must be in [2, 12]");
  if (o.p_s < 2 || o.p_s > MAXP || o.p_t < 2 || o.p_t > MAXP)
    throw Error(TDBEM_E_INVAL, "p_s and p_t must be in [2, 8]");
  if (o.p_t <= ctx->d) throw Error(TDBEM_E_INVAL, "p_t must exceed the B-spline order d");
  if (o.interp != TDBEM_INTERP_LAGRANGE && o.interp != TDBEM_INTERP_HERMITE)
    throw Error(TDBEM_E_INVAL, "interp must be LAGRANGE (0) or HERMITE (1)");
  if (o.interp == TDBEM_INTERP_HERMITE && (o.p_s < 3 || o.p_t < 3))
    throw Error(TDBEM_E_INVAL, "the cubic Hermite interpolation needs p_s, p_t >= 3");
  if (o.m2l_prec != TDBEM_M2L_FP64 && o.m2l_prec != TDBEM_M2L_FP32 && o.m2l_prec != TDBEM_M2L_BF16 &&
      o.m2l_prec != TDBEM_M2L_BF16X3)
    throw Error(TDBEM_E_INVAL, "m2l_prec must be FP64 (0), FP32 (1) or BF16 (2)");
  Fmm* f = new Fmm();
  try {
    f->D = o.depth;  // with leaf_ratio > 0 the tree sets it
    f->leaf_ratio = o.leaf_ratio;
    f->oscale = o.leaf_ratio > 0.0 ? std::pow(ctx->cdt, ctx->d - 1) : 1.0;
    f->prec = o.m2l_prec;
    f->ps = o.p_s;
    f->pt = o.p_t;
    f->Ps = f->ps * f->ps * f->ps;
    f->P = f->Ps * f->pt;
    f->Pp = (f->P + 31) / 32 * 32;
    f->Pr = row_pitch(f->P);
    f->Psr = (f->Ps + 15) / 16 * 16;
    f->interp = o.interp;
    if (f->interp == TDBEM_INTERP_HERMITE) {
      equispaced(f->ps, f->om_s);
      equispaced(f->pt, f->om_t);
    } else {
      cheb(f->ps, f->om_s);
      cheb(f->pt, f->om_t);
    }
    f->Cd = 1.0 / (4.0 * M_PI * std::pow(ctx->cdt, ctx->d));
    build_tree(ctx, f);
    build_hierarchy(ctx, f);
    hipStream_t st = ctx->stream;
    const int ns = ctx->ns, P = f->P, G = f->Gn;
    NodeSet& nodes = f->nodes;
    for (int a = 0; a < f->ps; ++a) nodes.s[a] = f->om_s[a];
    for (int a = 0; a < f->pt; ++a) nodes.t[a] = f->om_t[a];
    nodes.interp = f->interp;
    // element tables
    const FmmLevel& LL = f->lev[f->D];
    std::vector<double> cc(3 * (size_t)LL.ncell);
    const double hsl = hs_of(f, f->D);
    for (int i = 0; i < LL.ncell; ++i)
      for (int k = 0; k < 3; ++k) cc[3 * i + k] = f->center[k] - f->H + (LL.key[i][k] + 0.5) * 2.0 * hsl;
    DevBuf<double> d_cc;
    upload(d_cc, cc, st);
    std::vector<int32_t> leaf_of(f->leaf_of.begin(), f->leaf_of.end());
    std::vector<int32_t> leaf_ptr(f->leaf_ptr.begin(), f->leaf_ptr.end());
    std::vector<int32_t> leaf_elems(f->leaf_elems.begin(), f->leaf_elems.end());
    upload(f->d_leaf_of, leaf_of, st);
    upload(f->d_leaf_ptr, leaf_ptr, st);
    upload(f->d_leaf_elems, leaf_elems, st);
    f->d_A.alloc((size_t)ns * f->Ps);
    f->d_B.alloc((size_t)ns * f->Ps);
    f->d_E0.alloc((size_t)ns * f->Ps);
    f->d_E1.alloc((size_t)ns * f->Ps);
    const int nq = std::max(4, (3 * (f->ps - 1) + 3) / 2);
    QuadRule q = gauss_legendre01(nq);
    elem_tables_kernel<<<ns, ((f->Ps + 63) / 64) * 64, 0, st>>>(ns, f->ps, hsl, nodes, q, ctx->d_tris.p,
                                                                  ctx->d_nrm.p, ctx->d_xc.p, d_cc.p, f->d_leaf_of.p,
                                                                  f->d_A.p, f->d_B.p, f->d_E0.p, f->d_E1.p);
    TDBEM_HIP(hipGetLastError());
    f->d_tau.alloc(ns);
    f->d_sig.alloc(ns);
    // re-interpolation matrices: S[side][parent a][child b] = l_a(side/2 + om_b/2), side 0 -> -1
    std::vector<double> S(2 * f->ps * f->ps), T(2 * f->pt * f->pt), St(S.size()), Tt(T.size());
    for (int sd = 0; sd < 2; ++sd) {
      const double sgn = sd ? 1.0 : -1.0;
      for (int a = 0; a < f->ps; ++a)
        for (int b = 0; b < f->ps; ++b) {
          const double v = basis(f, f->om_s, f->ps, a, 0.5 * sgn + 0.5 * f->om_s[b]);
          S[sd * f->ps * f->ps + a * f->ps + b] = v;
          St[sd * f->ps * f->ps + b * f->ps + a] = v;
        }
      for (int a = 0; a < f->pt; ++a)
        for (int b = 0; b < f->pt; ++b) {
          const double v = basis(f, f->om_t, f->pt, a, 0.5 * sgn + 0.5 * f->om_t[b]);
          T[sd * f->pt * f->pt + a * f->pt + b] = v;
          Tt[sd * f->pt * f->pt + b * f->pt + a] = v;
        }
    }
    std::vector<double> ST(S);
    ST.insert(ST.end(), T.begin(), T.end());
    ST.insert(ST.end(), St.begin(), St.end());
    ST.insert(ST.end(), Tt.begin(), Tt.end());
    upload(f->d_S, ST, st);
    // per-level device data
    for (int l = 1; l <= f->D; ++l) {
      FmmLevel& L = f->lev[l];
      std::vector<int32_t> par(L.parent.begin(), L.parent.end()), oc(L.octant.begin(), L.octant.end());
      upload(L.d_parent, par, st);
      upload(L.d_octant, oc, st);
    }
    for (int l = 1; l < f->D; ++l) {  // children CSR of level l cells (from level l+1)
      FmmLevel& L = f->lev[l];
      const FmmLevel& C = f->lev[l + 1];
      std::vector<int32_t> ptr(L.ncell + 1, 0), ch(C.ncell);
      for (int c = 0; c < C.ncell; ++c) ptr[C.parent[c] + 1]++;
      for (int i = 0; i < L.ncell; ++i) ptr[i + 1] += ptr[i];
      std::vector<int32_t> fl(ptr.begin(), ptr.end() - 1);
      for (int c = 0; c < C.ncell; ++c) ch[fl[C.parent[c]]++] = c;
      upload(L.d_child_ptr, ptr, st);
      upload(L.d_child, ch, st);
    }
    for (int l = 2; l <= f->D; ++l) {
      FmmLevel& L = f->lev[l];
      std::vector<int32_t> ilp(L.il_ptr.begin(), L.il_ptr.end());
      upload(L.d_il_ptr, ilp, st);
      std::vector<int32_t> ils(L.il_src.begin(), L.il_src.end());
      upload(L.d_il_src, ils, st);
      const int nslot = (int)L.slot_off.size();
      std::vector<std::vector<int32_t>> by(nslot);
      for (int64_t p = 0; p < L.npair; ++p) by[L.il_slot[p]].push_back((int32_t)p);
      std::vector<int32_t> flat, tiles128, tiles64, tiles32;
      for (int sl = 0; sl < nslot; ++sl) {
        const int first = (int)flat.size();
        flat.insert(flat.end(), by[sl].begin(), by[sl].end());
        for (int width : {128, 64, 32}) {
          std::vector<int32_t>& tl = width == 128 ? tiles128 : width == 64 ? tiles64 : tiles32;
          for (int s0 = 0; s0 < (int)by[sl].size(); s0 += width) {
            tl.push_back(sl);
            tl.push_back(first + s0);
            tl.push_back(std::min(width, (int)by[sl].size() - s0));
          }
        }
      }
      L.ntiles128 = (int)tiles128.size() / 3;
      L.ntiles64 = (int)tiles64.size() / 3;
      L.ntiles32 = (int)tiles32.size() / 3;
      upload(L.d_tiles128, tiles128, st);
      upload(L.d_tiles64, tiles64, st);
      upload(L.d_tiles32, tiles32, st);
      upload(L.d_pairs_by_slot, flat, st);
      std::vector<int32_t> flat_src(flat.size());
      for (size_t i = 0; i < flat.size(); ++i) flat_src[i] = L.il_src[flat[i]];
      upload(L.d_src_by_slot, flat_src, st);
      std::vector<int32_t> so;
      for (auto& v : L.slot_off) { so.push_back(v[0]); so.push_back(v[1]); so.push_back(v[2]); }
      DevBuf<int32_t> d_so;
      upload(d_so, so, st);
      const int nk = 1 + (ctx->d >= 2 ? 1 : 0) + (ctx->d >= 3 ? 1 : 0);
      DevBuf<double> d_K;  // row-major spatial kernels (set-up only)
      d_K.alloc((size_t)std::max(nslot, 1) * nk * f->Ps * f->Ps);
      if (nslot > 0) {
        dim3 gk((unsigned)((f->Ps * f->Ps + 255) / 256), nslot);
        m2l_spatial_kernel<<<gk, 256, 0, st>>>(f->ps, nk, hs_of(f, l), nodes, d_so.p, nslot, d_K.p);
        TDBEM_HIP(hipGetLastError());
        const int RBk = (f->Ps + 15) / 16, KBk = m2l_kblocks(f->Ps);
        const int64_t perk = (int64_t)RBk * KBk * 64;
        L.d_Ktf.alloc((size_t)nk * nslot * perk);
        dim3 gfk((unsigned)((perk + 255) / 256), nk * nslot);
        to_fragments_kernel<double><<<gfk, 256, 0, st>>>(f->Ps, f->Ps, f->Ps, 0, f->Ps, RBk, KBk, d_K.p, L.d_Ktf.p);
        TDBEM_HIP(hipGetLastError());
        TDBEM_HIP(hipStreamSynchronize(st));
      }
      L.d_tm.alloc((size_t)L.ncell * (ctx->d + 1) * f->Ps);
      L.d_tsum.alloc((size_t)L.ncell * (ctx->d + 1));
      const int nv = (ctx->d + 1) + std::max(0, ctx->d - 1) + std::max(0, ctx->d - 2);
      L.d_V.alloc((size_t)std::max<int64_t>(L.npair, 1) * nv * f->Psr);
      level_ops(ctx, f, l, st);
      classify_gaps(ctx, f, l, tiles128, tiles64, tiles32, st);
      L.d_mom.alloc((size_t)L.ncell * P);
      if (f->prec == 1) {
        L.d_mom32.alloc((size_t)L.ncell * P);
        TDBEM_HIP(hipMemsetAsync(L.d_mom32.p, 0, L.d_mom32.n * sizeof(float), st));
      }
      if (f->prec >= 2) {  // the padding columns P .. Pp-1 stay zero; split products: two terms
        L.d_mom16.alloc((size_t)(f->prec == 3 ? 2 : 1) * L.ncell * f->Pp);
        TDBEM_HIP(hipMemsetAsync(L.d_mom16.p, 0, L.d_mom16.n * sizeof(uint16_t), st));
      }
      L.d_ring.alloc((size_t)f->R * L.ncell * P);
      L.d_lp.alloc((size_t)ctx->d * L.ncell * P);
      L.d_aux.alloc((size_t)std::max(1, ctx->d * (ctx->d - 1) / 2) * L.ncell * P);  // L^{(p,m)}, m <= p-2
      L.d_dp.alloc((size_t)ctx->d * L.ncell * P);
      if (f->prec != 0) L.d_stage32.alloc((size_t)std::max<int64_t>(L.npair, 1) * G * f->Pr);
      else L.d_stage.alloc((size_t)std::max<int64_t>(L.npair, 1) * G * f->Pr);
      for (DevBuf<double>* b : {&L.d_mom, &L.d_ring, &L.d_lp, &L.d_aux})
        TDBEM_HIP(hipMemsetAsync(b->p, 0, b->n * sizeof(double), st));
      TDBEM_HIP(hipStreamSynchronize(st));  // temporaries (d_so) are released at scope end
    }
    TDBEM_HIP(hipStreamSynchronize(st));
    {
      int dev = 0, ncu = 0;
      TDBEM_HIP(hipGetDevice(&dev));
      TDBEM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      f->persistent_grid = std::max(8, (ncu * 2 / 8) * 8);  // two workgroups per CU, a multiple of 8
    }
    autotune_m2l(f, st);
    return f;
  } catch (...) {
    delete f;
    throw;
  }
}

void fmm_destroy(Fmm* f) { delete f; }

void fmm_reset(tdbem_ctx* ctx) {
  Fmm* f = ctx->fmm;
  for (int l = 2; l <= f->D; ++l) {
    FmmLevel& L = f->lev[l];
    TDBEM_HIP(hipMemsetAsync(L.d_mom.p, 0, L.d_mom.n * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(L.d_ring.p, 0, L.d_ring.n * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(L.d_lp.p, 0, L.d_lp.n * sizeof(double), ctx->stream));
    TDBEM_HIP(hipMemsetAsync(L.d_aux.p, 0, L.d_aux.n * sizeof(double), ctx->stream));
  }
}

void fmm_state_buffers(const tdbem_ctx* ctx, std::vector<std::pair<double*, size_t>>& out) {
  const Fmm* f = ctx->fmm;
  for (int l = 2; l <= f->D; ++l) {
    const FmmLevel& L = f->lev[l];
    out.push_back({L.d_mom.p, L.d_mom.n});
    out.push_back({L.d_ring.p, L.d_ring.n});
    out.push_back({L.d_lp.p, L.d_lp.n});
    out.push_back({L.d_aux.p, L.d_aux.n});
  }
}

static TimeWeights time_weights(const Fmm* f, double xi, double ht) {
  TimeWeights tw{};
  for (int m = 0; m < f->pt; ++m) {
    double der = 0.0;
    tw.w[m] = basis(f, f->om_t, f->pt, m, xi, &der);
    tw.dw[m] = der / ht;
  }
  return tw;
}

void fmm_far(tdbem_ctx* ctx, int alpha, double* out) {
  Fmm* f = ctx->fmm;
  const int D = f->D;
  const FmmLevel& L = f->lev[D];
  const int Ml = f->m_leaf;
  const int k = alpha / Ml;
  const double ht = Ml * ctx->dt / 2.0;
  const double center = (k * (double)Ml + (Ml - 1) / 2.0) * ctx->dt;
  TimeWeights tw = time_weights(f, (alpha * ctx->dt - center) / ht, ht);
  const double* Lk = L.d_ring.p + (int64_t)(k % f->R) * L.ncell * f->P;
  ProfScope ps(ctx, K_L2P);
  l2p_kernel<<<L.ncell, 64, 0, ctx->stream>>>(f->Ps, f->pt, ctx->bie, 1.0 / ctx->c, tw, f->d_leaf_ptr.p,
                                               f->d_leaf_elems.p, f->d_E0.p, f->d_E1.p, Lk, out);
  TDBEM_HIP(hipGetLastError());
}



static int sep_threads(int P) { return std::min(1024, ((P + 63) / 64) * 64); }

// Levels whose source interval ends after sample beta: D, D-1, ..., D-n+1.
static int due_levels(const Fmm* f, int beta) {
  int ndue = 0;
  for (int l = f->D; l >= 2; --l) {
    const int Ml = f->m_leaf * (1 << (f->D - l));
    if ((beta + 2) % Ml != 0) break;
    ++ndue;
  }
  return ndue;
}

void fmm_advance(tdbem_ctx* ctx, int beta) {
  // all on the context's stream: running the separable products on a second stream beside
  // the dense ones gained 1% on one large context and serialised the captured marches of a
  // many-context batch
  Fmm* f = ctx->fmm;
  const int ndue = fmm_advance_pre(ctx, beta);
  if (ndue > 0) {
    fmm_advance_sep(ctx, beta, ndue, ctx->stream);
    ProfScope ps(ctx, K_M2L_GEMM);
    launch_m2l_levels(f, ndue, f->m2l_choice[ndue], ctx->stream);
  }
  fmm_advance_post(ctx, beta, ndue);
}

int fmm_advance_pre(tdbem_ctx* ctx, int beta) {
  Fmm* f = ctx->fmm;
  hipStream_t st = ctx->stream;
  const int D = f->D, P = f->P;
  // densities of the new sample and P2M into the leaf source interval
  ProfScope* p2m_scope = new ProfScope(ctx, K_P2M);
  densities_kernel<<<(ctx->ns + 255) / 256, 256, 0, st>>>(ctx->ns, beta, ctx->d, ctx->bw, ctx->d_hu.p, ctx->d_hq.p,
                                                           ctx->hist_u ? 1 : 0, ctx->hist_q ? 1 : 0, f->d_tau.p,
                                                           f->d_sig.p);
  TDBEM_HIP(hipGetLastError());
  {
    const int Ml = f->m_leaf;
    const int k = (beta + 1) / Ml;
    const double ht = Ml * ctx->dt / 2.0;
    const double center = (k * (double)Ml - 1.0 + (Ml - 1) / 2.0) * ctx->dt;
    TimeWeights tw = time_weights(f, (beta * ctx->dt - center) / ht, ht);
    FmmLevel& L = f->lev[D];
    const int first = (beta + 1) % Ml == 0;
    p2m_kernel<<<L.ncell, ((f->Ps + 63) / 64) * 64, 0, st>>>(f->Ps, f->pt, first, f->Cd, tw, f->d_leaf_ptr.p,
                                                              f->d_leaf_elems.p, f->d_A.p, f->d_B.p, f->d_tau.p,
                                                              f->d_sig.p, L.d_mom.p, L.d_mom32.p, L.d_mom16.p, f->Pp,
                                                              f->prec == 3 ? (int64_t)L.ncell * f->Pp : 0);
    TDBEM_HIP(hipGetLastError());
  }
  delete p2m_scope;
  const double* S = f->d_S.p;
  const double* T = S + 2 * f->ps * f->ps;
  const size_t shm = 2 * (size_t)P * sizeof(double);
  const int ndue = due_levels(f, beta);
  if (ndue > 0) {
    // M2M first (bottom-up: a parent's moments are complete before its own
    // products); it only reads each level's moments, so one M2L launch can then
    // take every due level
    for (int l = D; l > D - ndue && l > 2; --l) {
      const int Ml = f->m_leaf * (1 << (D - l));
      const int k = (beta + 2) / Ml - 1;
      FmmLevel& L = f->lev[l];
      FmmLevel& Pl = f->lev[l - 1];
      ProfScope ps(ctx, K_M2M);
      m2m_kernel<<<Pl.ncell, sep_threads(P), shm, st>>>(f->ps, f->pt, k & 1, Pl.d_child_ptr.p, Pl.d_child.p,
                                                         L.d_octant.p, S, T, L.d_mom.p, Pl.d_mom.p, Pl.d_mom32.p,
                                                         Pl.d_mom16.p, f->Pp, f->prec == 3 ? (int64_t)Pl.ncell * f->Pp : 0);
      TDBEM_HIP(hipGetLastError());
    }
  }
  return ndue;
}

// Separable products of the due levels (the wavefront-free near-future gaps and the
// derivative products L^{(p)}_{k+mu+1,k}, FP64) on stream st.  They read the moments and
// write the locals and derivative terms, which the dense products do not touch, so in a
// lock-step batch they run on each context's stream beside the batch's dense products;
// the reduction of the dense products comes after them.
void fmm_advance_sep(tdbem_ctx* ctx, int beta, int ndue, hipStream_t st) {
  Fmm* f = ctx->fmm;
  const int D = f->D;
  for (int l = D; l > D - ndue; --l) {
    const int Ml = f->m_leaf * (1 << (D - l));
    const int k = (beta + 2) / Ml - 1;  // completed source interval at level l
    FmmLevel& L = f->lev[l];
    if (L.npair == 0) continue;
    ProfScope ps(ctx, K_M2L_DERIV, st);
    const double ht = Ml * ctx->dt / 2.0;
    m2l_time_moments_kernel<<<L.ncell, 64, 0, st>>>(f->Ps, f->pt, ctx->d, ht, f->nodes, L.ncell, L.d_mom.p,
                                                    L.d_tm.p, L.d_tsum.p);
    TDBEM_HIP(hipGetLastError());
    launch_sep_products(f, L, ctx->d, st);
    auto expand = ctx->d == 1 ? m2l_sep_expand_kernel<1> : ctx->d == 2 ? m2l_sep_expand_kernel<2>
                                                                       : m2l_sep_expand_kernel<3>;
    expand<<<L.ncell, std::min(256, ((f->Ps + 63) / 64) * 64), 0, st>>>(
        f->Ps, f->Psr, f->pt, f->mu, f->R, k, ctx->c, ctx->dt, Ml, ht, f->nodes, L.ncell, L.npair, L.d_il_ptr.p,
        L.d_il_src.p, L.d_pair_gr.p, L.d_sep_order.p, L.d_V.p, L.d_tsum.p, L.d_ring.p, L.d_dp.p);
    TDBEM_HIP(hipGetLastError());
  }
}

void fmm_advance_post(tdbem_ctx* ctx, int beta, int ndue) {
  Fmm* f = ctx->fmm;
  hipStream_t st = ctx->stream;
  const int D = f->D, P = f->P;
  const double* S = f->d_S.p;
  const double* T = S + 2 * f->ps * f->ps;
  const double* St = T + 2 * f->pt * f->pt;
  const double* Tt = St + 2 * f->ps * f->ps;
  (void)T;
  const size_t shm = 2 * (size_t)P * sizeof(double);
  if (ndue > 0) {
    for (int l = D; l > D - ndue; --l) {
      const int Ml = f->m_leaf * (1 << (D - l));
      const int k = (beta + 2) / Ml - 1;  // completed source interval at level l
      FmmLevel& L = f->lev[l];
      if (L.npair > 0) {
        ProfScope ps(ctx, K_M2L_RED);
        if (L.nred > 0) {
          const int nthr = (P + 3) / 4, bs = std::min(256, (nthr + 63) / 64 * 64);
          dim3 g2((unsigned)L.nred, (unsigned)((nthr + bs - 1) / bs));
          if (f->prec != 0)
            m2l_reduce_kernel<float><<<g2, bs, 0, st>>>(P, f->Pr, f->Gn, f->R, k, L.ncell, L.d_red_cg.p,
                                                         L.d_red_ptr.p, L.d_red_pairs.p, L.d_stage32.p, f->oscale,
                                                         L.d_ring.p);
          else
            m2l_reduce_kernel<double><<<g2, bs, 0, st>>>(P, f->Pr, f->Gn, f->R, k, L.ncell, L.d_red_cg.p,
                                                          L.d_red_ptr.p, L.d_red_pairs.p, L.d_stage.p, f->oscale,
                                                          L.d_ring.p);
          TDBEM_HIP(hipGetLastError());
        }
        const int64_t nrec = (int64_t)L.ncell * P;
        m2l_recurrence_kernel<<<(unsigned)((nrec + 255) / 256), 256, 0, st>>>(P, f->mu, ctx->d, f->R, k,
                                                                               ctx->c * Ml * ctx->dt, L.ncell,
                                                                               L.d_dp.p, L.d_ring.p, L.d_lp.p,
                                                                               L.d_aux.p);
        TDBEM_HIP(hipGetLastError());
      }
    }
  }
  // L2L for the target intervals that start at the next step, top-down
  const int anext = beta + 2;
  for (int l = 2; l < D; ++l) {
    const int Ml = f->m_leaf * (1 << (D - l));
    if (anext % Ml != 0) continue;
    FmmLevel& Pl = f->lev[l];
    FmmLevel& C = f->lev[l + 1];
    ProfScope ps(ctx, K_L2L);
    l2l_kernel<<<C.ncell, sep_threads(P), shm, st>>>(f->ps, f->pt, f->R, anext / Ml, C.d_parent.p, C.d_octant.p, St,
                                                      Tt, Pl.d_ring.p, Pl.ncell, C.d_ring.p, C.ncell);
    TDBEM_HIP(hipGetLastError());
  }
}

// Several contexts in lock step: the due levels of all of them in one M2L launch.
// The launch shape (P, mu + 1 blocks, precision, tile variant) is common, so the
// contexts must agree on P, mu and precision; equal M_leaf makes their interval ends
// coincide.  Descriptor tables are built once per distinct pattern of due levels
// and kept on the device.
struct FmmBatch {
  std::vector<tdbem_ctx*> ctxs;
  int choice = 0;                          // tile variant (2 * variant + persistent)
  struct Table { DevBuf<M2LLevelWork> lev; DevBuf<int32_t> item0; int nlev = 0, total = 0; };
  std::map<std::vector<int>, std::unique_ptr<Table>> tables;
};

FmmBatch* fmm_batch_create(tdbem_ctx* const* ctxs, int n) {
  if (n < 1) throw Error(TDBEM_E_INVAL, "empty batch");
  const Fmm* f0 = ctxs[0]->fmm;
  for (int i = 0; i < n; ++i) {
    const Fmm* f = ctxs[i]->fmm;
    if (!f || f->P != f0->P || f->Gn != f0->Gn || f->prec != f0->prec || f->m_leaf != f0->m_leaf ||
        f->Pp != f0->Pp)
      throw Error(TDBEM_E_INVAL, "batch M2L: contexts differ in P, mu, precision or M_leaf");
  }
  auto* b = new FmmBatch();
  b->ctxs.assign(ctxs, ctxs + n);
  // the tile of the context with the most interaction pairs, for its leaf-level launch
  int best = 0;
  int64_t most = -1;
  for (int i = 0; i < n; ++i) {
    const Fmm* f = ctxs[i]->fmm;
    if (f->lev[f->D].npair > most) { most = f->lev[f->D].npair; best = i; }
  }
  b->choice = ctxs[best]->fmm->m2l_choice[1] & ~1;  // one item per workgroup (the grid covers all items)
  return b;
}

void fmm_batch_destroy(FmmBatch* b) { delete b; }

void fmm_batch_m2l(FmmBatch* b, const int* ndue, hipStream_t st) {
  const int n = (int)b->ctxs.size();
  std::vector<int> key(ndue, ndue + n);
  auto it = b->tables.find(key);
  if (it == b->tables.end()) {
    std::vector<M2LLevelWork> lev;
    std::vector<int32_t> first;
    int total = 0;
    for (int i = 0; i < n; ++i) {
      const Fmm* f = b->ctxs[i]->fmm;
      for (int l = f->D; l > f->D - ndue[i] && l >= 2; --l) {
        M2LLevelWork Lw{};
        int ni = 0;
        if (!level_work(f, l, b->choice >> 1, total, Lw, ni)) continue;
        lev.push_back(Lw);
        first.push_back(total);
        total += ni;
      }
    }
    auto t = std::make_unique<FmmBatch::Table>();
    t->nlev = (int)lev.size();
    t->total = total;
    if (!lev.empty()) {
      t->lev.alloc(lev.size());
      t->item0.alloc(first.size());
      TDBEM_HIP(hipMemcpy(t->lev.p, lev.data(), lev.size() * sizeof(M2LLevelWork), hipMemcpyHostToDevice));
      TDBEM_HIP(hipMemcpy(t->item0.p, first.data(), first.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    it = b->tables.emplace(key, std::move(t)).first;
  }
  const FmmBatch::Table& t = *it->second;
  if (t.total == 0) return;
  M2LWork W{};
  W.nlev = t.nlev;
  W.total = t.total;
  W.glev = t.lev.p;
  W.gitem0 = t.item0.p;
  launch_m2l_work(b->ctxs[0]->fmm, b->choice, W, st);
}

void fmm_info(const tdbem_ctx* ctx, tdbem_info* info) {
  const Fmm* f = ctx->fmm;
  info->depth = f->D;
  info->p_s = f->ps;
  info->p_t = f->pt;
  info->mu = f->mu;
  info->m_leaf = f->m_leaf;
  int64_t bytes = 0;
  for (int n = 1; n < f->D && n < 16; ++n) info->m2l_variant[n] = f->m2l_choice[n];
  for (int l = 2; l <= f->D && l < 16; ++l) {
    info->il_pairs[l] = f->lev[l].npair;
    info->m2l_dense_blocks[l] = f->lev[l].dense_blocks;
    const LevelOps* ops = f->lev[l].ops.get();
    info->m2l_ops_users[l] = (int)f->lev[l].ops.use_count();
    if (ops) bytes += (int64_t)ops->Uf.n * sizeof(double) + (int64_t)ops->U32.n * sizeof(float) +
                      (int64_t)ops->U16.n * sizeof(uint16_t);
  }
  info->m2l_matrix_bytes = bytes;
}

int fmm_set_m2l_variant(tdbem_ctx* ctx, int n, int choice) {
  Fmm* f = ctx->fmm;
  if (!f || n < 1 || n > f->D - 1 || n >= 16 || choice < 0 || choice >= 2 * M2L_VARIANTS) return TDBEM_E_INVAL;
  if ((choice >> 1) >= M2L_FIRST_DIRECT && f->P % 4 != 0 && f->prec < 2) return TDBEM_E_INVAL;
  if ((choice >> 1) >= M2L_FIRST_BF16_LDS && f->prec < 2) return TDBEM_E_INVAL;
  if ((choice >> 1) < M2L_FIRST_DIRECT && f->prec >= 2) return TDBEM_E_INVAL;
  f->m2l_choice[n] = choice;
  return TDBEM_OK;
}

void fmm_near_pairs(const tdbem_ctx* ctx, std::vector<int64_t>& row_ptr, std::vector<int32_t>& pair_j) {
  const Fmm* f = ctx->fmm;
  const FmmLevel& L = f->lev[f->D];
  std::unordered_map<int64_t, int> pos;
  for (int i = 0; i < L.ncell; ++i) pos[key64(L.key[i][0], L.key[i][1], L.key[i][2])] = i;
  const int ns = ctx->ns;
  row_ptr.assign(ns + 1, 0);
  pair_j.clear();
  for (int i = 0; i < ns; ++i) {
    const auto& k = L.key[f->leaf_of[i]];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          auto it = pos.find(key64(k[0] + dx, k[1] + dy, k[2] + dz));
          if (k[0] + dx < 0 || k[1] + dy < 0 || k[2] + dz < 0 || it == pos.end()) continue;
          const int c = it->second;
          for (int q = f->leaf_ptr[c]; q < f->leaf_ptr[c + 1]; ++q) pair_j.push_back(f->leaf_elems[q]);
        }
    row_ptr[i + 1] = (int64_t)pair_j.size();
  }
}

}  // namespace tdbem
