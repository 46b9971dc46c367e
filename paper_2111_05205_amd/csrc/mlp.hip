// Learned initial guess of the per-step solve.
//
// A per-element network (12 inputs, three ReLU layers of width 256, one
// output) proposes where GMRES starts at each step; GMRES still runs to its
// tolerance.  Weights and layer inputs are rounded to bfloat16 and multiplied
// on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation).  Training
// kernels: backward (FP32 matrix cores on the bf16-rounded operands, rounding
// taken as the identity), mean squared error and Adam.  March-side kernels:
// features, proposal and training-record targets.
//
// Matrix-core lane layouts used below (16x16 output tiles, 64 lanes, lane l):
//   bf16 16x16x16: A[i][k] at lane i + 16 (k / 4), element k % 4;
//                  B[k][j] at lane j + 16 (k / 4), element k % 4
//   bf16 16x16x32: the same with 8 elements per lane (k / 8, k % 8)
//   f32  16x16x4:  A[i][k] at lane i + 16 k;  B[k][j] at lane j + 16 k
//   output (both): D[4 (l / 16) + r][l % 16] in accumulator element r
#include "internal.h"

#include <cmath>
#include <mutex>
#include <string>

namespace tdbem {
namespace {

constexpr int NIN = TDBEM_MLP_IN;
constexpr int NINP = TDBEM_MLP_IN_PAD;
constexpr int WID = TDBEM_MLP_WIDTH;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + WID * NINP;
constexpr int OFF_W2 = OFF_B1 + WID;
constexpr int OFF_B2 = OFF_W2 + WID * WID;
constexpr int OFF_W3 = OFF_B2 + WID;
constexpr int OFF_B3 = OFF_W3 + WID * WID;
constexpr int OFF_W4 = OFF_B3 + WID;
constexpr int OFF_B4 = OFF_W4 + WID;
constexpr int NPARAM = OFF_B4 + 1;
static_assert(NPARAM == TDBEM_MLP_NPARAM, "packed parameter layout");
static_assert(OFF_W2 % 4 == 0 && OFF_W3 % 4 == 0, "16-byte aligned weight rows");

constexpr int FR = 64;          // rows per workgroup (backward)
constexpr int FFR = 32;         // rows per workgroup (forward)
constexpr int HS = WID + 8;     // LDS row stride of bf16 activations (elements)
constexpr int DS = WID + 4;     // LDS row stride of FP32 gradients
constexpr int WG_SPLIT = 8;     // row splits of the weight-gradient products

typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline float round_bf16(float f) { return from_bf16(to_bf16(f)); }

// ---------------------------------------------------------------------------
// Forward: one workgroup (4 waves) per FR rows; activations stay in LDS as
// bf16; wave w computes output neurons [64 w, 64 w + 64) for all FR rows.  The
// weight fragments of the next K step are loaded while the current one is
// multiplied.

// PK: the hidden layers' weights come pre-rounded in matrix-core fragment
// order (wpk, see mlp_pack_kernel): a wave fetches all of a layer's fragments
// for its 64 neurons at once (32 x 16 bytes per lane), the next layer's while
// the current one is multiplied, so the weight stream costs one memory
// latency per layer instead of one per K step.
template <int FR, bool PK>
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float* __restrict__ P, int n,
                                                      const float* __restrict__ feat, float* __restrict__ y,
                                                      uint16_t* __restrict__ act, const uint4* __restrict__ wpk) {
  constexpr int RT = FR / 16;     // row tiles per wave
  constexpr int TPR = 256 / FR;   // threads per row in the output layer
  __shared__ __align__(16) uint16_t H[2][FR * HS];
  __shared__ float w4s[WID];  // output-layer weights, bf16-rounded
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = blockIdx.x * FR;
  for (int e = tid; e < FR * NINP; e += 256) {
    const int r = e / NINP, k = e % NINP;
    float v = 0.f;
    if (row0 + r < n && k < NIN) v = feat[(int64_t)(row0 + r) * NINP + k];
    H[0][r * HS + k] = to_bf16(v);
  }
  for (int k = tid; k < WID; k += 256) w4s[k] = round_bf16(P[OFF_W4 + k]);
  const float b4 = P[OFF_B4];
  // packed fragments of hidden layer 1 or 2: [layer][tile 16][kstep 8][lane 64]
  uint4 wq[8][4];
  auto fetch = [&](int hl) {
    if constexpr (PK) {
      const uint4* base = wpk + (size_t)hl * 16 * 8 * 64;
#pragma unroll
      for (int st = 0; st < 8; ++st)
#pragma unroll
        for (int t = 0; t < 4; ++t) wq[st][t] = base[((w * 4 + t) * 8 + st) * 64 + lane];
    }
  };
  fetch(0);
  __syncthreads();
  for (int layer = 0; layer < 3; ++layer) {
    const int K = layer == 0 ? NINP : WID;
    const float* W = P + (layer == 0 ? OFF_W1 : layer == 1 ? OFF_W2 : OFF_W3);
    const float* B = P + (layer == 0 ? OFF_B1 : layer == 1 ? OFF_B2 : OFF_B3);
    const uint16_t* Hin = H[layer & 1];
    uint16_t* Hout = H[(layer + 1) & 1];
    f4 acc[4][RT];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < RT; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    float4 bias[4];  // loaded ahead of the products
    for (int a = 0; a < 4; ++a) bias[a] = *reinterpret_cast<const float4*>(B + w * 64 + a * 16 + 4 * lk);
    if (layer == 0) {
      // K = 16 (12 inputs and padding): one v_mfma_f32_16x16x16_bf16 step
      s4 av[4], bv[RT];
      for (int t = 0; t < 4; ++t) {
        const float4 wv = *reinterpret_cast<const float4*>(W + (int64_t)(w * 64 + t * 16 + li) * K + 4 * lk);
        av[t] = s4{(short)to_bf16(wv.x), (short)to_bf16(wv.y), (short)to_bf16(wv.z), (short)to_bf16(wv.w)};
      }
      for (int b = 0; b < RT; ++b)
        bv[b] = __builtin_bit_cast(s4, *reinterpret_cast<const uint2*>(Hin + (b * 16 + li) * HS + 4 * lk));
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < RT; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
    } else if (PK) {
      // K = 256 in 8 steps of v_mfma_f32_16x16x32_bf16 on the fetched fragments
#pragma unroll
      for (int st = 0; st < 8; ++st) {
        b8 av[4], bv[RT];
#pragma unroll
        for (int t = 0; t < 4; ++t) av[t] = __builtin_bit_cast(b8, wq[st][t]);
#pragma unroll
        for (int b = 0; b < RT; ++b)
          bv[b] = __builtin_bit_cast(b8, *reinterpret_cast<const uint4*>(Hin + (b * 16 + li) * HS + 32 * st + 8 * lk));
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < RT; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
      if (layer == 1) fetch(1);  // the last hidden layer's fragments, while this layer finishes
    } else {
      // K = 256 in 8 steps of v_mfma_f32_16x16x32_bf16: A[i][k] at lane i + 16 (k / 8), element k % 8
      float4 wn[4][2];
      for (int t = 0; t < 4; ++t)
        for (int h = 0; h < 2; ++h)
          wn[t][h] = *reinterpret_cast<const float4*>(W + (int64_t)(w * 64 + t * 16 + li) * K + 8 * lk + 4 * h);
      for (int k0 = 0; k0 < K; k0 += 32) {
        b8 av[4], bv[RT];
        for (int t = 0; t < 4; ++t) {
          const uint4 pk = uint4{(uint32_t)to_bf16(wn[t][0].x) | ((uint32_t)to_bf16(wn[t][0].y) << 16),
                                 (uint32_t)to_bf16(wn[t][0].z) | ((uint32_t)to_bf16(wn[t][0].w) << 16),
                                 (uint32_t)to_bf16(wn[t][1].x) | ((uint32_t)to_bf16(wn[t][1].y) << 16),
                                 (uint32_t)to_bf16(wn[t][1].z) | ((uint32_t)to_bf16(wn[t][1].w) << 16)};
          av[t] = __builtin_bit_cast(b8, pk);
        }
        if (k0 + 32 < K)
          for (int t = 0; t < 4; ++t)
            for (int h = 0; h < 2; ++h)
              wn[t][h] = *reinterpret_cast<const float4*>(W + (int64_t)(w * 64 + t * 16 + li) * K + k0 + 32 + 8 * lk +
                                                          4 * h);
        for (int b = 0; b < RT; ++b)
          bv[b] = __builtin_bit_cast(b8, *reinterpret_cast<const uint4*>(Hin + (b * 16 + li) * HS + k0 + 8 * lk));
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < RT; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    for (int a = 0; a < 4; ++a) {
      const int o0 = w * 64 + a * 16 + 4 * lk;
      for (int b = 0; b < RT; ++b) {
        const int r = b * 16 + li;
        const uint16_t h0 = to_bf16(fmaxf(acc[a][b][0] + bias[a].x, 0.f));
        const uint16_t h1 = to_bf16(fmaxf(acc[a][b][1] + bias[a].y, 0.f));
        const uint16_t h2 = to_bf16(fmaxf(acc[a][b][2] + bias[a].z, 0.f));
        const uint16_t h3 = to_bf16(fmaxf(acc[a][b][3] + bias[a].w, 0.f));
        const uint2 pk = uint2{(uint32_t)h0 | ((uint32_t)h1 << 16), (uint32_t)h2 | ((uint32_t)h3 << 16)};
        *reinterpret_cast<uint2*>(Hout + r * HS + o0) = pk;
        if (act && row0 + r < n) *reinterpret_cast<uint2*>(act + ((int64_t)layer * n + row0 + r) * WID + o0) = pk;
      }
    }
    __syncthreads();
  }
  // output layer (h3 is in H[1]): TPR lanes per row, WID / TPR inputs each
  const int r = tid / TPR, q = tid % TPR;
  float s = 0.f;
  for (int k = q * (WID / TPR); k < (q + 1) * (WID / TPR); ++k) s += w4s[k] * from_bf16(H[1][r * HS + k]);
  for (int m = 1; m < TPR; m <<= 1) s += __shfl_xor(s, m);
  if (q == 0 && row0 + r < n) y[row0 + r] = s + b4;
}

// ---------------------------------------------------------------------------
// Backward through the activations: dz3 = dy (x) W4 masked by h3 > 0, then
// dz2 = (dz3 W3) masked by h2 > 0, dz1 = (dz2 W2) masked by h1 > 0.
// dz: [3][n][256] (index 0 = dz1).  One workgroup per 64 rows.

__global__ __launch_bounds__(256) void mlp_bwd_data_kernel(const float* __restrict__ P, int n,
                                                           const uint16_t* __restrict__ act,
                                                           const float* __restrict__ dy, float* __restrict__ dz) {
  __shared__ __align__(16) float D[FR * DS];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = blockIdx.x * FR;
  for (int e = tid; e < FR * WID; e += 256) {
    const int r = e / WID, k = e % WID;
    float v = 0.f;
    if (row0 + r < n) {
      const int64_t idx = ((int64_t)2 * n + row0 + r) * WID + k;
      if (from_bf16(act[idx]) > 0.f) v = dy[row0 + r] * round_bf16(P[OFF_W4 + k]);
      dz[idx] = v;
    }
    D[r * DS + k] = v;
  }
  __syncthreads();
  for (int L = 0; L < 2; ++L) {
    const float* W = P + (L == 0 ? OFF_W3 : OFF_W2);
    const int li_out = L == 0 ? 1 : 0;  // dz index written; its mask is activation index li_out
    f4 acc[4][4];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    for (int o0 = 0; o0 < WID; o0 += 4) {
      float av[4], bv[4];
      for (int t = 0; t < 4; ++t) {
        av[t] = round_bf16(W[(int64_t)(o0 + lk) * WID + w * 64 + t * 16 + li]);  // A[kin][o] = W[o][kin]
        bv[t] = D[(t * 16 + li) * DS + o0 + lk];                                // B[o][row] = dz[row][o]
      }
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
    for (int a = 0; a < 4; ++a) {
      const int k0 = w * 64 + a * 16 + 4 * lk;
      for (int b = 0; b < 4; ++b) {
        const int r = b * 16 + li;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (row0 + r < n) {
          const int64_t idx = ((int64_t)li_out * n + row0 + r) * WID + k0;
          const uint2 hm = *reinterpret_cast<const uint2*>(act + idx);
          const uint16_t hh[4] = {(uint16_t)(hm.x & 0xffff), (uint16_t)(hm.x >> 16), (uint16_t)(hm.y & 0xffff),
                                  (uint16_t)(hm.y >> 16)};
          for (int e = 0; e < 4; ++e) v[e] = from_bf16(hh[e]) > 0.f ? acc[a][b][e] : 0.f;
          *reinterpret_cast<float4*>(dz + idx) = float4{v[0], v[1], v[2], v[3]};
        }
        for (int e = 0; e < 4; ++e) D[r * DS + k0 + e] = v[e];
      }
    }
    __syncthreads();
  }
}

// Weight gradients, split over rows: part[s][p] for split s.
// Tasks 0..3: W1 tiles (64 outputs x 16 inputs), 4..19: W2 tiles (64 x 64),
// 20..35: W3 tiles, 36: biases and W4.  Wave w of a tile task owns outputs
// [o0 + 16 w, o0 + 16 w + 16).
constexpr int WG_TASKS = 37;

__global__ __launch_bounds__(256) void mlp_wgrad_kernel(int n, const float* __restrict__ feat,
                                                        const uint16_t* __restrict__ act,
                                                        const float* __restrict__ dz, const float* __restrict__ dy,
                                                        float* __restrict__ part) {
  const int task = blockIdx.x, split = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int chunk = (n + WG_SPLIT - 1) / WG_SPLIT;
  const int rb = split * chunk, re = min(n, rb + chunk);
  float* out = part + (int64_t)split * NPARAM;
  if (task == WG_TASKS - 1) {
    // column sums: b1, b2, b3 (dz), W4 (dy h3), b4 (dy)
    const int k = tid;
    float s1 = 0.f, s2 = 0.f, s3 = 0.f, s4v = 0.f, s5 = 0.f;
    for (int r = rb; r < re; ++r) {
      s1 += dz[((int64_t)0 * n + r) * WID + k];
      s2 += dz[((int64_t)1 * n + r) * WID + k];
      s3 += dz[((int64_t)2 * n + r) * WID + k];
      const float g = dy[r];
      s4v += g * from_bf16(act[((int64_t)2 * n + r) * WID + k]);
      if (k == 0) s5 += g;
    }
    out[OFF_B1 + k] = s1;
    out[OFF_B2 + k] = s2;
    out[OFF_B3 + k] = s3;
    out[OFF_W4 + k] = s4v;
    if (k == 0) out[OFF_B4] = s5;
    return;
  }
  int layer, o0, kt0, ktiles;
  if (task < 4) { layer = 0; o0 = task * 64; kt0 = 0; ktiles = 1; }
  else if (task < 20) { layer = 1; o0 = ((task - 4) / 4) * 64; kt0 = ((task - 4) % 4) * 64; ktiles = 4; }
  else { layer = 2; o0 = ((task - 20) / 4) * 64; kt0 = ((task - 20) % 4) * 64; ktiles = 4; }
  const int K = layer == 0 ? NINP : WID;
  const int woff = layer == 0 ? OFF_W1 : layer == 1 ? OFF_W2 : OFF_W3;
  const float* dzl = dz + (int64_t)layer * n * WID;
  const uint16_t* hin = layer == 0 ? nullptr : act + (int64_t)(layer - 1) * n * WID;
  f4 acc[4];
  for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
  const int orow = o0 + 16 * w + li;
  for (int r0 = rb; r0 < re; r0 += 4) {
    const int r = r0 + lk;
    const bool ok = r < re;
    const float av = ok ? dzl[(int64_t)r * WID + orow] : 0.f;  // A[o][r] = dz[r][o]
    for (int t = 0; t < ktiles; ++t) {
      const int k = kt0 + 16 * t + li;
      float bv = 0.f;                                         // B[r][k] = h_in[r][k]
      if (ok) {
        if (layer == 0) bv = k < NIN ? round_bf16(feat[(int64_t)r * NINP + k]) : 0.f;
        else bv = from_bf16(hin[(int64_t)r * WID + k]);
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
    }
  }
  for (int t = 0; t < ktiles; ++t)
    for (int e = 0; e < 4; ++e) {
      const int o = o0 + 16 * w + 4 * lk + e;
      const int k = kt0 + 16 * t + li;
      out[woff + o * K + k] = acc[t][e];
    }
}

__global__ void mlp_reduce_kernel(const float* __restrict__ part, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float s = 0.f;
  for (int k = 0; k < WG_SPLIT; ++k) s += part[(int64_t)k * NPARAM + p];
  grad[p] = s;
}

__global__ __launch_bounds__(1024) void mlp_mse_kernel(int n, const float* __restrict__ y,
                                                       const float* __restrict__ t, float* __restrict__ dy,
                                                       float* __restrict__ loss) {
  __shared__ double sh[1024];
  const int tid = threadIdx.x;
  double acc = 0.0;
  const float sc = 2.f / (float)(n > 0 ? n : 1);
  for (int i = tid; i < n; i += 1024) {
    const float e = y[i] - t[i];
    dy[i] = sc * e;
    acc += (double)e * e;
  }
  sh[tid] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  if (tid == 0) loss[0] = (float)(sh[0] / (n > 0 ? n : 1));
}

__global__ void mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1,
                                float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---------------------------------------------------------------------------
// March side.

__global__ void diag_kernel(int ns, const int32_t* __restrict__ ap, const int32_t* __restrict__ ac,
                            const double* __restrict__ av, double* __restrict__ diag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  double d = 0.0;
  for (int k = ap[i]; k < ap[i + 1]; ++k)
    if (ac[k] == i) d = av[k];
  diag[i] = d;
}

// s = sqrt((sum_{k=1..4} |x^{beta-k}|^2 + |b / diag|^2) / (5 ns)), one workgroup.
__global__ __launch_bounds__(1024) void mlp_scale_kernel(int ns, int beta, const double* __restrict__ h,
                                                         const double* __restrict__ b,
                                                         const double* __restrict__ diag, double* __restrict__ s) {
  __shared__ double sh[16];
  const int tid = threadIdx.x;
  double acc = 0.0;
#pragma unroll 4
  for (int i = tid; i < ns; i += 1024) {  // unrolled: several rows' loads in flight
    for (int k = 1; k <= 4; ++k) {
      const double x = h[(int64_t)(beta - k) * ns + i];
      acc += x * x;
    }
    const double bj = b[i] / diag[i];
    acc += bj * bj;
  }
  for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if ((tid & 63) == 0) sh[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sh[w];
    s[0] = sqrt(t / (5.0 * ns));
  }
}

struct FeatGeo { double inv_h2, cen[3], inv_r; };

__global__ void mlp_features_kernel(int ns, int beta, const double* __restrict__ h, const double* __restrict__ b,
                                    const double* __restrict__ diag, const double* __restrict__ xc,
                                    const double* __restrict__ nrm, const double* __restrict__ area, FeatGeo g,
                                    const double* __restrict__ s, float* __restrict__ feat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const double sv = s[0];
  const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
  float f[NINP];
  const double x1 = h[(int64_t)(beta - 1) * ns + i], x2 = h[(int64_t)(beta - 2) * ns + i];
  const double x3 = h[(int64_t)(beta - 3) * ns + i], x4 = h[(int64_t)(beta - 4) * ns + i];
  // backward differences of the history and the Jacobi-scaled rhs relative to the extrapolation
  f[0] = (float)(x1 * inv);
  f[1] = (float)((x1 - x2) * inv);
  f[2] = (float)((x1 - 2.0 * x2 + x3) * inv);
  f[3] = (float)((x1 - 3.0 * x2 + 3.0 * x3 - x4) * inv);
  f[4] = (float)((b[i] / diag[i] - (3.0 * x1 - 3.0 * x2 + x3)) * inv);
  for (int k = 0; k < 3; ++k) f[5 + k] = (float)(-nrm[3 * i + k]);  // outward = -(paper normal)
  f[8] = (float)(area[i] * g.inv_h2);
  for (int k = 0; k < 3; ++k) f[9 + k] = (float)((xc[3 * i + k] - g.cen[k]) * g.inv_r);
  for (int k = NIN; k < NINP; ++k) f[k] = 0.f;
  float4* o = reinterpret_cast<float4*>(feat + (int64_t)i * NINP);
  for (int q = 0; q < 4; ++q) o[q] = float4{f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]};
}

// Value at beta of the parabola through rows beta-1, beta-2, beta-3.
__device__ inline double extrapolated(const double* __restrict__ h, int beta, int ns, int i) {
  return 3.0 * h[(int64_t)(beta - 1) * ns + i] - 3.0 * h[(int64_t)(beta - 2) * ns + i] + h[(int64_t)(beta - 3) * ns + i];
}

// The network corrects the extrapolation: x = extrapolation + s y.
__global__ void mlp_guess_kernel(int ns, int beta, const double* __restrict__ h, const double* __restrict__ s,
                                 const float* __restrict__ y, double* __restrict__ x, double* __restrict__ xe) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const double base = extrapolated(h, beta, ns, i);
  const float yi = y[i];
  x[i] = isfinite(yi) ? base + s[0] * (double)yi : base;
  if (xe) xe[i] = base;
}

__global__ void mlp_target_kernel(int ns, int beta, const double* __restrict__ h, const double* __restrict__ s,
                                  float* __restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const double sv = s[0];
  const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
  t[i] = (float)((h[(int64_t)beta * ns + i] - extrapolated(h, beta, ns, i)) * inv);
}

void launch_fwd(const float* P, int n, const float* feat, float* y, uint16_t* act, hipStream_t st,
                const uint4* wpk = nullptr) {
  if (n <= 0) return;
  if (wpk)
    mlp_fwd_kernel<FFR, true><<<(n + FFR - 1) / FFR, 256, 0, st>>>(P, n, feat, y, act, wpk);
  else
    mlp_fwd_kernel<FFR, false><<<(n + FFR - 1) / FFR, 256, 0, st>>>(P, n, feat, y, act, nullptr);
  TDBEM_HIP(hipGetLastError());
}

// Hidden-layer weights W2, W3 rounded to bf16 in the fragment order of
// v_mfma_f32_16x16x32_bf16 (A[i][k] at lane i + 16 (k / 8), element k % 8):
// wpk[layer][tile t][kstep s][lane] holds W[16 t + lane%16][32 s + 8 (lane/16) + e], e = 0..7.
__global__ void mlp_pack_kernel(const float* __restrict__ P, uint4* __restrict__ wpk) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // (layer, t, s, lane)
  if (idx >= 2 * 16 * 8 * 64) return;
  const int lane = idx & 63, s = (idx >> 6) & 7, t = (idx >> 9) & 15, layer = idx >> 13;
  const float* W = P + (layer == 0 ? OFF_W2 : OFF_W3) + (int64_t)(16 * t + (lane & 15)) * WID + 32 * s + 8 * (lane >> 4);
  uint32_t h[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) h[e] = to_bf16(W[e]);
  wpk[idx] = uint4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
}

}  // namespace

static FeatGeo feat_geo(const tdbem_ctx* ctx) {
  const Geometry& G = ctx->geo;
  FeatGeo g{};
  for (int k = 0; k < 3; ++k) g.cen[k] = 0.5 * (G.ext_lo[k] + G.ext_hi[k]);
  double r2 = 0.0;
  for (size_t v = 0; v < G.tris.size() / 3; ++v) {
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double dd = G.tris[3 * v + k] - g.cen[k];
      d2 += dd * dd;
    }
    r2 = std::max(r2, d2);
  }
  g.inv_r = 1.0 / std::sqrt(r2);
  g.inv_h2 = 1.0 / (G.edge_mean * G.edge_mean);
  return g;
}

void mlp_prepare(tdbem_ctx* ctx) {
  const int ns = ctx->ns;
  if (ctx->d_mlp_diag.n == (size_t)ns) return;
  const FeatGeo g = feat_geo(ctx);
  ctx->mlp_geo[0] = g.inv_h2;
  for (int k = 0; k < 3; ++k) ctx->mlp_geo[1 + k] = g.cen[k];
  ctx->mlp_geo[4] = g.inv_r;
  ctx->d_mlp_diag.alloc(ns);
  ctx->d_mlp_s.alloc(1);
  ctx->d_area.alloc(ns);
  ctx->d_mlp_feat.alloc((size_t)ns * NINP);
  ctx->d_mlp_y.alloc(ns);
  ctx->d_x_alt.alloc(ns);
  TDBEM_HIP(hipMemcpyAsync(ctx->d_area.p, ctx->geo.area.data(), ns * sizeof(double), hipMemcpyHostToDevice,
                           ctx->stream));
  diag_kernel<<<(ns + 255) / 256, 256, 0, ctx->stream>>>(ns, ctx->d_a_ptr.p, ctx->d_a_col.p, ctx->d_a_val.p,
                                                         ctx->d_mlp_diag.p);
  TDBEM_HIP(hipGetLastError());
  TDBEM_HIP(hipStreamSynchronize(ctx->stream));
}

void launch_mlp_features(tdbem_ctx* ctx, int beta, const double* b, float* feat) {
  ProfScope ps(ctx, K_MLP);
  const int ns = ctx->ns;
  const double* h = ctx->bc == TDBEM_NEUMANN ? ctx->d_hu.p : ctx->d_hq.p;
  mlp_scale_kernel<<<1, 1024, 0, ctx->stream>>>(ns, beta, h, b, ctx->d_mlp_diag.p, ctx->d_mlp_s.p);
  TDBEM_HIP(hipGetLastError());
  FeatGeo geo{};
  geo.inv_h2 = ctx->mlp_geo[0];
  for (int k = 0; k < 3; ++k) geo.cen[k] = ctx->mlp_geo[1 + k];
  geo.inv_r = ctx->mlp_geo[4];
  mlp_features_kernel<<<(ns + 255) / 256, 256, 0, ctx->stream>>>(ns, beta, h, b, ctx->d_mlp_diag.p, ctx->d_xc.p,
                                                                  ctx->d_nrm.p, ctx->d_area.p, geo, ctx->d_mlp_s.p,
                                                                  feat);
  TDBEM_HIP(hipGetLastError());
}

void launch_mlp_guess(tdbem_ctx* ctx, int beta, const float* feat, double* x, double* xe) {
  ProfScope ps(ctx, K_MLP);
  const int ns = ctx->ns;
  const double* h = ctx->bc == TDBEM_NEUMANN ? ctx->d_hu.p : ctx->d_hq.p;
  launch_fwd(ctx->d_mlp_params.p, ns, feat, ctx->d_mlp_y.p, nullptr, ctx->stream,
             reinterpret_cast<const uint4*>(ctx->d_mlp_wpk.p));
  mlp_guess_kernel<<<(ns + 255) / 256, 256, 0, ctx->stream>>>(ns, beta, h, ctx->d_mlp_s.p, ctx->d_mlp_y.p, x,
                                                               xe);
  TDBEM_HIP(hipGetLastError());
}

void launch_mlp_target(tdbem_ctx* ctx, int beta, float* target) {
  ProfScope ps(ctx, K_MLP);
  const int ns = ctx->ns;
  const double* h = ctx->bc == TDBEM_NEUMANN ? ctx->d_hu.p : ctx->d_hq.p;
  mlp_target_kernel<<<(ns + 255) / 256, 256, 0, ctx->stream>>>(ns, beta, h, ctx->d_mlp_s.p, target);
  TDBEM_HIP(hipGetLastError());
}

void mlp_pack(tdbem_ctx* ctx) {
  if (!ctx->d_mlp_wpk.p) ctx->d_mlp_wpk.alloc((size_t)2 * WID * WID);
  mlp_pack_kernel<<<(2 * 16 * 8 * 64 + 255) / 256, 256, 0, ctx->stream>>>(
      ctx->d_mlp_params.p, reinterpret_cast<uint4*>(ctx->d_mlp_wpk.p));
  TDBEM_HIP(hipGetLastError());
}

// Scratch of tdbem_mlp_backward_noalloc: dz (3 x n x 256) followed by the
// WG_SPLIT x NPARAM weight-gradient partials, sized for the row maximum
// (29.6 MB).  Each GPU the library runs on holds its own copy until the
// process ends.  In host code the name is not a device address: kernels get the
// per-device address from hipGetSymbolAddress.
constexpr size_t NOALLOC_FLOATS = (size_t)3 * TDBEM_MLP_NOALLOC_MAX_ROWS * WID + (size_t)WG_SPLIT * NPARAM;
__device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of this GPU's scratch, looked up once per device with that device current.
float* noalloc_scratch() {
  int dev = 0;
  TDBEM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) throw Error(TDBEM_E_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(TDBEM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace tdbem

using namespace tdbem;

template <class F>
static int mlp_guarded(F&& f) {
  try {
    f();
    return TDBEM_OK;
  } catch (const Error& e) {
    set_global_error(e.msg);
    return e.code;
  }
}

extern "C" {

int tdbem_mlp_forward(const float* dev_params, int n, const float* dev_feat, float* dev_y, uint16_t* dev_act,
                      void* hip_stream) {
  return mlp_guarded([&] {
    if (!dev_params || n < 0 || (n > 0 && (!dev_feat || !dev_y))) throw Error(TDBEM_E_INVAL, "mlp_forward: bad arguments");
    if ((reinterpret_cast<uintptr_t>(dev_params) | reinterpret_cast<uintptr_t>(dev_feat)) & 15)
      throw Error(TDBEM_E_INVAL, "mlp_forward: parameters and features must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(dev_act) & 7) throw Error(TDBEM_E_INVAL, "mlp_forward: act must be 8-byte aligned");
    hipStream_t st = (hipStream_t)hip_stream;
    launch_fwd(dev_params, n, dev_feat, dev_y, dev_act, st);
    TDBEM_HIP(hipStreamSynchronize(st));
  });
}

int tdbem_mlp_forward_loaded(tdbem_ctx* ctx, int n, const float* dev_feat, float* dev_y) {
  if (!ctx) return TDBEM_E_INVAL;
  try {
    if (!ctx->mlp_loaded) throw Error(TDBEM_E_INVAL, "mlp_forward_loaded: no network installed");
    if (n < 0 || (n > 0 && (!dev_feat || !dev_y))) throw Error(TDBEM_E_INVAL, "mlp_forward_loaded: bad arguments");
    if (reinterpret_cast<uintptr_t>(dev_feat) & 15)
      throw Error(TDBEM_E_INVAL, "mlp_forward_loaded: features must be 16-byte aligned");
    launch_fwd(ctx->d_mlp_params.p, n, dev_feat, dev_y, nullptr, ctx->stream,
               reinterpret_cast<const uint4*>(ctx->d_mlp_wpk.p));
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
    return TDBEM_OK;
  } catch (const Error& e) {
    ctx->err = e.msg;
    return e.code;
  }
}

size_t tdbem_mlp_workspace_floats(int n) {
  return (size_t)3 * (size_t)(n > 0 ? n : 0) * WID + (size_t)WG_SPLIT * NPARAM;
}

int tdbem_mlp_backward(const float* dev_params, int n, const float* dev_feat, const uint16_t* dev_act,
                       const float* dev_dy, float* dev_grad, float* dev_work, size_t work_floats, void* hip_stream) {
  return mlp_guarded([&] {
    if (!dev_params || !dev_grad || !dev_work || n < 0 || (n > 0 && (!dev_feat || !dev_act || !dev_dy)))
      throw Error(TDBEM_E_INVAL, "mlp_backward: bad arguments");
    if (work_floats < tdbem_mlp_workspace_floats(n)) throw Error(TDBEM_E_INVAL, "mlp_backward: workspace too small");
    if ((reinterpret_cast<uintptr_t>(dev_work) | reinterpret_cast<uintptr_t>(dev_act)) & 15)
      throw Error(TDBEM_E_INVAL, "mlp_backward: workspace and act must be 16-byte aligned");
    hipStream_t st = (hipStream_t)hip_stream;
    float* dz = dev_work;
    float* part = dev_work + (size_t)3 * n * WID;
    if (n > 0) {
      mlp_bwd_data_kernel<<<(n + FR - 1) / FR, 256, 0, st>>>(dev_params, n, dev_act, dev_dy, dz);
      TDBEM_HIP(hipGetLastError());
    }
    mlp_wgrad_kernel<<<dim3(WG_TASKS, WG_SPLIT), 256, 0, st>>>(n, dev_feat, dev_act, dz, dev_dy, part);
    TDBEM_HIP(hipGetLastError());
    mlp_reduce_kernel<<<(NPARAM + 255) / 256, 256, 0, st>>>(part, dev_grad);
    TDBEM_HIP(hipGetLastError());
    TDBEM_HIP(hipStreamSynchronize(st));
  });
}

// Backward pass without allocation: the activation gradients and the per-split
// weight-gradient partials live in one file-scope device array (the same kernels
// as tdbem_mlp_backward, which takes them in a caller workspace).  Every launch
// writes every element it later reads, so nothing needs clearing between calls.
int tdbem_mlp_backward_noalloc(const float* dev_params, int n, const float* dev_feat, const uint16_t* dev_act,
                               const float* dev_dy, float* dev_grad, void* hip_stream) {
  return mlp_guarded([&] {
    if (!dev_params || !dev_grad || n < 0 || (n > 0 && (!dev_feat || !dev_act || !dev_dy)))
      throw Error(TDBEM_E_INVAL, "mlp_backward_noalloc: bad arguments");
    if (n > TDBEM_MLP_NOALLOC_MAX_ROWS)
      throw Error(TDBEM_E_INVAL, "mlp_backward_noalloc: n = " + std::to_string(n) + " exceeds the maximum of " +
                                     std::to_string(TDBEM_MLP_NOALLOC_MAX_ROWS) + " rows");
    if (reinterpret_cast<uintptr_t>(dev_act) & 15)
      throw Error(TDBEM_E_INVAL, "mlp_backward_noalloc: act must be 16-byte aligned");
    float* work = noalloc_scratch();
    hipStream_t st = (hipStream_t)hip_stream;
    float* dz = work;
    float* part = work + (size_t)3 * n * WID;
    if (n > 0) {
      mlp_bwd_data_kernel<<<(n + FR - 1) / FR, 256, 0, st>>>(dev_params, n, dev_act, dev_dy, dz);
      TDBEM_HIP(hipGetLastError());
    }
    mlp_wgrad_kernel<<<dim3(WG_TASKS, WG_SPLIT), 256, 0, st>>>(n, dev_feat, dev_act, dz, dev_dy, part);
    TDBEM_HIP(hipGetLastError());
    mlp_reduce_kernel<<<(NPARAM + 255) / 256, 256, 0, st>>>(part, dev_grad);
    TDBEM_HIP(hipGetLastError());
    TDBEM_HIP(hipStreamSynchronize(st));
  });
}

int tdbem_mlp_mse(int n, const float* dev_y, const float* dev_t, float* dev_dy, float* dev_loss, void* hip_stream) {
  return mlp_guarded([&] {
    if (n < 0 || !dev_loss || (n > 0 && (!dev_y || !dev_t || !dev_dy))) throw Error(TDBEM_E_INVAL, "mlp_mse: bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    mlp_mse_kernel<<<1, 1024, 0, st>>>(n, dev_y, dev_t, dev_dy, dev_loss);
    TDBEM_HIP(hipGetLastError());
    TDBEM_HIP(hipStreamSynchronize(st));
  });
}

int tdbem_mlp_adam_step(float* dev_params, const float* dev_grad, float* dev_m, float* dev_v, int t, float lr,
                        float beta1, float beta2, float eps, void* hip_stream) {
  return mlp_guarded([&] {
    if (!dev_params || !dev_grad || !dev_m || !dev_v || t < 1) throw Error(TDBEM_E_INVAL, "mlp_adam_step: bad arguments");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
      throw Error(TDBEM_E_INVAL, "mlp_adam_step: need 0 <= beta < 1 and eps > 0");
    const float bc1 = (float)(1.0 - std::pow((double)beta1, t));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, t));
    hipStream_t st = (hipStream_t)hip_stream;
    mlp_adam_kernel<<<(NPARAM + 255) / 256, 256, 0, st>>>(dev_params, dev_grad, dev_m, dev_v, lr, beta1, beta2, eps,
                                                          bc1, bc2);
    TDBEM_HIP(hipGetLastError());
    TDBEM_HIP(hipStreamSynchronize(st));
  });
}

int tdbem_mlp_load(tdbem_ctx* ctx, const float* dev_params) {
  if (!ctx) return TDBEM_E_INVAL;
  try {
    if (!dev_params) throw Error(TDBEM_E_INVAL, "mlp_load: parameters are NULL");
    mlp_prepare(ctx);
    invalidate_graph(ctx);  // a captured march may predate the network
    if (!ctx->d_mlp_params.p) ctx->d_mlp_params.alloc(NPARAM);  // reloads copy in place
    TDBEM_HIP(hipMemcpyAsync(ctx->d_mlp_params.p, dev_params, NPARAM * sizeof(float), hipMemcpyDeviceToDevice,
                             ctx->stream));
    mlp_pack(ctx);
    TDBEM_HIP(hipStreamSynchronize(ctx->stream));
    ctx->mlp_loaded = true;
    return TDBEM_OK;
  } catch (const Error& e) {
    ctx->err = e.msg;
    return e.code;
  }
}

int tdbem_mlp_record(tdbem_ctx* ctx, float* dev_feat, float* dev_target) {
  if (!ctx) return TDBEM_E_INVAL;
  try {
    if ((dev_feat == nullptr) != (dev_target == nullptr))
      throw Error(TDBEM_E_INVAL, "mlp_record: give both buffers or neither");
    if (reinterpret_cast<uintptr_t>(dev_feat) & 15) throw Error(TDBEM_E_INVAL, "mlp_record: features must be 16-byte aligned");
    if (dev_feat) mlp_prepare(ctx);
    ctx->rec_feat = dev_feat;
    ctx->rec_target = dev_target;
    return TDBEM_OK;
  } catch (const Error& e) {
    ctx->err = e.msg;
    return e.code;
  }
}

}  // extern "C"
