// Surrogate network for ln k_s: an ensemble of MLPs 6 -> 128 -> 128 -> 128 -> 1
// (SiLU), trained and queried with the kernels below.
//
// Numerics, two precisions chosen per model: FP32 master weights always.
//  - BF16: BF16 copies of the weights (round to nearest even) feed the
//    forward pass; the two 128x128 layers run on v_mfma_f32_16x16x16_bf16
//    (BF16 inputs, FP32 accumulation); hidden activations are rounded to
//    BF16 before entering the next layer.
//  - FP32: the master weights and FP32 activations throughout; the 128x128
//    layers run on v_mfma_f32_16x16x4_f32.
// In both the 6-wide input layer and the 128-wide output dot run in FP32.  Inputs are the six
// physical quantities (LET, b, V, gap, dose per pulse, pulse rate),
// standardised as (log x - mu) / sigma.  Optionally the network learns the
// residual of ln k_s over an analytic baseline, -ln f_Jaffe - ln f_Boag:
// Jaffe's collection efficiency of a track parallel to the field (eq.
// Jaffe_noangle, with the averaged D and mu) times Boag's ln(1+u)/u for the
// uniform dose; the baseline is evaluated here in FP64.  The output is the
// standardised residual.  Training: mean squared error over each minibatch,
// backward in FP32 (with BF16 the casts pass gradients straight through),
// Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"
#include "reduce.h"

namespace it {
namespace {

constexpr int kH = 128, kIn = 6;
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH * kH, ow4 = ob3 + kH, ob4 = ow4 + kH, kP = ob4 + 1;  // 34049
constexpr int kPpad = (kP + 63) / 64 * 64;
constexpr int kTileS = 64;       // samples per forward block (4 waves x 16)
constexpr int kActStride = kH + 4;  // padded BF16 row (avoids LDS bank conflicts)

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kGL = 32;  // Gauss-Legendre nodes of the Jaffe integral

struct Header {
  int32_t members, step;
  float mu[kIn], sigma[kIn], lo[kIn], hi[kIn];
  float t_mu, t_sigma;
  int32_t use_baseline;
  int32_t precision;  // IT_MLP_BF16 or IT_MLP_FP32
  // averaged diffusion and mobility, alpha, W [eV], mu+ + mu-, ion pairs
  // per cm^3 and mGy
  double D, mu_avg, alpha, W, mu_sum, pairs_per_mGy;
  double gl_x[kGL], gl_w[kGL];  // nodes and weights on [-1, 1]
};

struct Model {  // device pointers carved from the model buffer
  Header* hdr;
  float* master;      // [M][kP]
  float* m;           // [M][kP]
  float* v;           // [M][kP]
  unsigned short* w;  // [M][kPpad] BF16
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t model_bytes(int M) {
  return align256(sizeof(Header)) + 3 * align256((size_t)M * kP * sizeof(float)) +
         align256((size_t)M * kPpad * sizeof(unsigned short));
}

Model carve_model(void* base, int M) {
  char* p = (char*)base;
  Model md;
  md.hdr = (Header*)p;
  p += align256(sizeof(Header));
  md.master = (float*)p;
  p += align256((size_t)M * kP * sizeof(float));
  md.m = (float*)p;
  p += align256((size_t)M * kP * sizeof(float));
  md.v = (float*)p;
  p += align256((size_t)M * kP * sizeof(float));
  md.w = (unsigned short*)p;
  return md;
}

struct TrainWs {  // per member: [M][n][...]
  float *z, *a1, *a2, *a3, *h1, *h2, *h3, *y, *dy, *d1, *d2, *d3, *grad, *loss, *base;
};

size_t train_ws_bytes(int M, int64_t n) {
  const size_t nh = (size_t)M * n * kH * sizeof(float);
  return 9 * align256(nh) + align256((size_t)M * n * kIn * 4) + 2 * align256((size_t)M * n * 4) +
         align256((size_t)M * kP * 4) + align256((size_t)M * 4) + align256((size_t)n * 4);
}

TrainWs carve_train(void* base, int M, int64_t n) {
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    float* r = (float*)p;
    p += align256(bytes);
    return r;
  };
  const size_t nh = (size_t)M * n * kH * sizeof(float);
  TrainWs w;
  w.a1 = take(nh);
  w.a2 = take(nh);
  w.a3 = take(nh);
  w.h1 = take(nh);
  w.h2 = take(nh);
  w.h3 = take(nh);
  w.d1 = take(nh);
  w.d2 = take(nh);
  w.d3 = take(nh);
  w.z = take((size_t)M * n * kIn * 4);
  w.y = take((size_t)M * n * 4);
  w.dy = take((size_t)M * n * 4);
  w.grad = take((size_t)M * kP * 4);
  w.loss = take((size_t)M * 4);
  w.base = take((size_t)n * 4);
  return w;
}

// Analytic baseline of ln k_s for one query (FP64): -ln f_J - ln f_B with
// f_J = (y1/y2) e^{-y1} [Ei(y1 + ln(1+y2)) - Ei(y1)], written as
// (y1/y2) int_0^{ln(1 + ln(1+y2)/y1)} exp(y1 (e^w - 1)) dw (no overflow for
// large y1), y1 = 8 pi D/(alpha N0), y2 = 2 d D/(mu b^2 E), N0 = LET/W, and
// f_B = ln(1+u)/u with u = alpha/(mu+ + mu-) n0 d^2/V.  The quadrature is
// summed in four parts of kGL/4 nodes (added in order), so that four
// threads can share a query.
struct BaseArgs {
  double y1, y2, upper;
};

__device__ inline BaseArgs base_args(const Header& H, const float* x) {
  const double let = x[0], b = x[1], V = x[2], d = x[3];
  const double E = V / d;
  const double N0 = let * 1.0e7 / H.W;
  BaseArgs a;
  a.y1 = 8.0 * M_PI * H.D / (H.alpha * N0);
  a.y2 = 2.0 * d * H.D / (H.mu_avg * b * b * E);
  a.upper = log1p(log1p(a.y2) / a.y1);
  return a;
}

__device__ inline double base_part(const Header& H, const BaseArgs& a, int part) {
  double s = 0.0;
  for (int q = part * (kGL / 4); q < (part + 1) * (kGL / 4); ++q) {
    const double w = 0.5 * a.upper * (H.gl_x[q] + 1.0);
    s += H.gl_w[q] * exp(a.y1 * expm1(w));
  }
  return s;
}

__device__ inline double base_finish(const Header& H, const float* x, const BaseArgs& a, double sum) {
  const double V = x[2], d = x[3], dose = x[4];
  const double fJ = a.y1 / a.y2 * (sum * 0.5 * a.upper);
  const double u = H.alpha / H.mu_sum * dose * H.pairs_per_mGy * d * d / V;
  const double fB = u > 0.0 ? log1p(u) / u : 1.0;
  return -log(fJ) - log(fB);
}

__device__ double baseline(const Header& H, const float* x) {
  const BaseArgs a = base_args(H, x);
  const double p0 = base_part(H, a, 0), p1 = base_part(H, a, 1), p2 = base_part(H, a, 2), p3 = base_part(H, a, 3);
  return base_finish(H, x, a, ((p0 + p1) + p2) + p3);
}

// Baseline of the 64 samples of a tile with all 256 threads: wave p sums
// quadrature part p of sample s0 + lane into part[p][lane]; after a barrier
// thread s < 64 calls base_of.
__device__ inline void base_parts(const Header& H, const float* __restrict__ X, int64_t n, int64_t s0,
                                  double (*part)[kTileS]) {
  const int p = threadIdx.x / 64, s = threadIdx.x % 64;
  const int64_t gs = s0 + s;
  part[p][s] = H.use_baseline && gs < n ? base_part(H, base_args(H, X + gs * kIn), p) : 0.0;
}

__device__ inline double base_of(const Header& H, const float* __restrict__ X, int64_t gs,
                                 const double (*part)[kTileS], int s) {
  if (!H.use_baseline) return 0.0;
  const float* x = X + gs * kIn;
  return base_finish(H, x, base_args(H, x), ((part[0][s] + part[1][s]) + part[2][s]) + part[3][s]);
}

__device__ inline unsigned short to_bf16(float f) {  // round to nearest even
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
// The logistic function 1/(1 + e^-a) from the hardware base-2 exponential
// (e^-a = 2^(-a log2 e)) and reciprocal: a few instructions instead of a
// full-precision exponential and division, about 1e-6 relative for the
// pre-activations the network sees (the rounding of -a log2 e dominates).
// Large |a| saturate correctly: 2^(+big) = inf gives 0, 2^(-big) = 0 gives 1.
__device__ inline float logistic(float a) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-a * 1.44269504088896341f));
}
__device__ inline float silu(float a) { return a * logistic(a); }
__device__ inline float dsilu(float a) {
  const float s = logistic(a);
  return s * (1.0f + a * (1.0f - s));
}

struct ForwardOut {  // optional stores of the training forward (member slices)
  float *z, *a1, *a2, *a3, *h1, *h2, *h3, *y;
};

// ---------------------------------------------------------------------------
// FP32 models.  Every kernel runs 256 threads on a tile of 64 samples of one
// member; wave w owns samples 16w..16w+15 of the tile.  The training kernel
// stages the 128 x 128 weights of a layer in LDS (wl[o][i], rows padded to
// kWS), read from global memory into registers one layer ahead (64 values
// per thread, element tid + 256 u of the matrix), so that their latency
// hides behind the previous layer; the query kernel stages them in halves
// (forward_query_f32).  Products run on v_mfma_f32_16x16x4f32 (A[i][k]: lane
// i + 16 k, B[k][j]: lane j + 16 k, D[i][j]: lane j + 16 (i/4), item i % 4),
// four 16-wide output tiles per pass sharing the A operand, k taken 4 at a
// time in increasing order.  Every per-element value a thread computes sits
// at (sample 16w + 4 (lane/16) + v, unit 16 t + lane % 16), v = 0..3, t =
// 0..7, the D layout, in every layer: so the pre-activations a thread
// stores in the forward pass are read back, in the backward pass, by that
// same thread.
constexpr int kWS = kH + 4;

// The small parameters of a member (W1 and b1, b2, b3, w4, b4), staged in
// LDS once per tile: three contiguous runs of the parameter vector.
struct SmallP {
  float w1b1[kH * kIn + kH];  // W1 [128][6], then b1
  float b2[kH];
  float b3w4b4[2 * kH + 1];   // b3, w4, b4
};

__device__ inline void sload(const float* __restrict__ master, SmallP& sp) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = tid + 256 * u;
    if (q < kH * kIn + kH) sp.w1b1[q] = master[oW1 + q];
  }
  if (tid < kH) sp.b2[tid] = master[ob2 + tid];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = tid + 256 * u;
    if (q < 2 * kH + 1) sp.b3w4b4[q] = master[ob3 + q];
  }
}

struct WRegs {
  float v[64];
};

__device__ inline void wload(WRegs& r, const float* __restrict__ W) {
#pragma unroll
  for (int u = 0; u < 64; ++u) r.v[u] = W[threadIdx.x + 256 * u];
}

__device__ inline void wstore(const WRegs& r, float (*wl)[kWS]) {
#pragma unroll
  for (int u = 0; u < 64; ++u) {
    const int q = threadIdx.x + 256 * u;
    wl[q / kH][q % kH] = r.v[u];
  }
}

// acc[u] += in[16w + i][k] * B[k][16 (t0 + u) + j] over k = 0..127, with
// B[k][j] = wl[j][k] (forward: out = in W^T) or wl[k][j] (backward:
// out = in W).
template <bool BWD>
__device__ inline void mfma_pass(const float (*in)[kActStride], const float (*wl)[kWS], int t0, float4_t* acc) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int arow = wave * 16 + (lane & 15), kq = lane >> 4, j = lane & 15;
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 8
  for (int kk = 0; kk < kH / 4; ++kk) {
    const int k = 4 * kk + kq;
    const float a = in[arow][k];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = (t0 + u) * 16 + j;
      acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, BWD ? wl[k][c] : wl[c][k], acc[u], 0, 0, 0);
    }
  }
}

// Hidden layer 2 or 3 of the training forward pass: out = silu(in W^T + b),
// with stores of the pre-activations and activations.  Ends with a barrier.
__device__ void layer_fwd_f32(const float (*in)[kActStride], float (*out)[kActStride], const float (*wl)[kWS],
                              const float* __restrict__ bias, int64_t n, int64_t s0, float* sa, float* sh) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll 1
  for (int t0 = 0; t0 < kH / 16; t0 += 4) {
    float4_t acc[4];
    mfma_pass<false>(in, wl, t0, acc);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = (t0 + u) * 16 + (lane & 15);
      const float b = bias[o];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int s = wave * 16 + 4 * (lane >> 4) + v;
        const float a = acc[u][v] + b;
        const float h = silu(a);
        out[s][o] = h;
        const int64_t gs = s0 + s;
        if (gs < n) {
          sa[gs * kH + o] = a;
          sh[gs * kH + o] = h;
        }
      }
    }
  }
  __syncthreads();
}

// Backward through a hidden layer: dprev = (d W) * silu'(a_prev), where
// a_prev are the pre-activations this thread stored in the forward pass
// (read before the pass's products, so that the loads overlap them).
// Optional LDS copy (the next layer's input); stores for the weight
// gradients.  Ends with a barrier.
__device__ void layer_bwd_f32(const float (*d)[kActStride], float (*dout)[kActStride], const float (*wl)[kWS],
                              const float* apre, int64_t n, int64_t s0, float* dstore) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll 1
  for (int t0 = 0; t0 < kH / 16; t0 += 4) {
    float ap[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gs = s0 + wave * 16 + 4 * (lane >> 4) + v;
        ap[u][v] = gs < n ? apre[gs * kH + (t0 + u) * 16 + (lane & 15)] : 0.0f;
      }
    float4_t acc[4];
    mfma_pass<true>(d, wl, t0, acc);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = (t0 + u) * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int s = wave * 16 + 4 * (lane >> 4) + v;
        const int64_t gs = s0 + s;
        float dv = 0.0f;
        if (gs < n) {
          dv = acc[u][v] * dsilu(ap[u][v]);
          dstore[gs * kH + o] = dv;
        }
        if (dout) dout[s][o] = dv;
      }
    }
  }
  __syncthreads();
}

// Training forward pass of one FP32 member over samples [s0, s0 + 64),
// storing what the backward pass and the weight gradients read.  On entry
// `pf` holds (or is loading) this member's W2; on return it is loading
// `next` (when not null).  Leaves the standardised outputs in ys[64] and h3
// in act[0].
__device__ void forward_tile_f32(const Header& H, const float* __restrict__ master, const float* __restrict__ X,
                                 int64_t n, int64_t s0, float* zs, float (*act)[kTileS][kActStride],
                                 float (*wl)[kWS], SmallP& sp, float (*yp)[kTileS], float* ys, WRegs& pf,
                                 const float* next, const ForwardOut& st) {
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  sload(master, sp);  // its last readers passed a barrier
  // standardised inputs
  for (int q = tid; q < kTileS * kIn; q += 256) {
    const int s = q / kIn, i = q % kIn;
    const int64_t gs = s0 + s;
    float zv = 0.0f;
    if (gs < n) zv = (logf(X[gs * kIn + i]) - H.mu[i]) / H.sigma[i];
    zs[q] = zv;
    if (gs < n) st.z[gs * kIn + i] = zv;
  }
  __syncthreads();
  // layer 1 (FP32 FMAs, D layout)
#pragma unroll 2
  for (int t = 0; t < kH / 16; ++t) {
    const int o = t * 16 + (lane & 15);
    float w1[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) w1[i] = sp.w1b1[o * kIn + i];
    const float b = sp.w1b1[kH * kIn + o];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = wave * 16 + 4 * (lane >> 4) + v;
      float a = b;
#pragma unroll
      for (int i = 0; i < kIn; ++i) a += w1[i] * zs[s * kIn + i];
      const float h = silu(a);
      act[0][s][o] = h;
      const int64_t gs = s0 + s;
      if (gs < n) {
        st.a1[gs * kH + o] = a;
        st.h1[gs * kH + o] = h;
      }
    }
  }
  wstore(pf, wl);  // W2 (wl's last readers passed a barrier)
  __syncthreads();
  wload(pf, master + oW3);
  layer_fwd_f32(act[0], act[1], wl, sp.b2, n, s0, st.a2, st.h2);
  wstore(pf, wl);  // W3
  __syncthreads();
  if (next) wload(pf, next);
  layer_fwd_f32(act[1], act[0], wl, sp.b3w4b4, n, s0, st.a3, st.h3);
  // output layer: four partial dot products of 32 terms per sample
  {
    const int s = lane, p = wave;
    float y = 0.0f;
#pragma unroll 8
    for (int i = 32 * p; i < 32 * p + 32; ++i) y += sp.b3w4b4[kH + i] * act[0][s][i];
    yp[p][s] = y;
  }
  __syncthreads();
  if (tid < kTileS) {
    const float y = sp.b3w4b4[2 * kH] + (((yp[0][tid] + yp[1][tid]) + yp[2][tid]) + yp[3][tid]);
    ys[tid] = y;
    const int64_t gs = s0 + tid;
    if (gs < n) st.y[gs] = y;
  }
  __syncthreads();
}

// Query form of the FP32 forward pass, sized for two blocks per CU (78 KB of
// LDS): one activation buffer, updated in place (every wave reads and writes
// only its own 16 rows, so a layer's two passes keep their results in
// registers until both have read the input), and each 128 x 128 matrix
// staged in two halves of 64 output rows, one per pass (32 values per
// thread in flight, element tid + 256 u of the half).  Every output is summed
// in the same order as in forward_tile_f32, so both give the same values.
struct WHalf {
  float v[32];
};

__device__ inline void wload_half(WHalf& r, const float* __restrict__ W, int half) {
#pragma unroll
  for (int u = 0; u < 32; ++u) r.v[u] = W[half * 64 * kH + threadIdx.x + 256 * u];
}

__device__ inline void wstore_half(const WHalf& r, float (*wl)[kWS]) {
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    const int q = threadIdx.x + 256 * u;
    wl[q / kH][q % kH] = r.v[u];
  }
}

// One hidden layer of the query form: act = silu(act W^T + b).  On entry pf
// holds half 0 of W and wl is free (its last readers passed a barrier); on
// return pf is loading half 0 of `next` (when not null).  Ends with a
// barrier.
__device__ void layer_query_f32(float (*act)[kActStride], float (*wl)[kWS], const float* bias,
                                const float* __restrict__ W, WHalf& pf, const float* next) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  float4_t acc[2][4];
  wstore_half(pf, wl);
  __syncthreads();
  wload_half(pf, W, 1);
  mfma_pass<false>(act, wl, 0, acc[0]);
  __syncthreads();  // every wave is done with half 0
  wstore_half(pf, wl);
  __syncthreads();
  if (next) wload_half(pf, next, 0);
  mfma_pass<false>(act, wl, 0, acc[1]);
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = h * 64 + u * 16 + (lane & 15);
      const float b = bias[o];
#pragma unroll
      for (int v = 0; v < 4; ++v) act[wave * 16 + 4 * (lane >> 4) + v][o] = silu(acc[h][u][v] + b);
    }
  __syncthreads();
}

// Query forward pass of one FP32 member over samples [s0, s0 + 64): pf holds
// (or is loading) half 0 of this member's W2 on entry and is loading `next`
// on return.  Leaves the standardised outputs in ys[64].
__device__ void forward_query_f32(const Header& H, const float* __restrict__ master, const float* __restrict__ X,
                                  int64_t n, int64_t s0, float* zs, float (*act)[kActStride], float (*wl)[kWS],
                                  SmallP& sp, float (*yp)[kTileS], float* ys, WHalf& pf, const float* next) {
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  sload(master, sp);  // its last readers passed a barrier
  for (int q = tid; q < kTileS * kIn; q += 256) {
    const int s = q / kIn, i = q % kIn;
    const int64_t gs = s0 + s;
    zs[q] = gs < n ? (logf(X[gs * kIn + i]) - H.mu[i]) / H.sigma[i] : 0.0f;
  }
  __syncthreads();
#pragma unroll 2
  for (int t = 0; t < kH / 16; ++t) {
    const int o = t * 16 + (lane & 15);
    float w1[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) w1[i] = sp.w1b1[o * kIn + i];
    const float b = sp.w1b1[kH * kIn + o];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = wave * 16 + 4 * (lane >> 4) + v;
      float a = b;
#pragma unroll
      for (int i = 0; i < kIn; ++i) a += w1[i] * zs[s * kIn + i];
      act[s][o] = silu(a);
    }
  }
  layer_query_f32(act, wl, sp.b2, master + oW2, pf, master + oW3);
  layer_query_f32(act, wl, sp.b3w4b4, master + oW3, pf, next);
  {
    const int s = lane, p = wave;
    float y = 0.0f;
#pragma unroll 8
    for (int i = 32 * p; i < 32 * p + 32; ++i) y += sp.b3w4b4[kH + i] * act[s][i];
    yp[p][s] = y;
  }
  __syncthreads();
  if (tid < kTileS) ys[tid] = sp.b3w4b4[2 * kH] + (((yp[0][tid] + yp[1][tid]) + yp[2][tid]) + yp[3][tid]);
  __syncthreads();
}

// One FP32 training step's per-sample work for a tile of 64 samples of one
// member: the forward pass (storing what the weight gradients need), the
// loss gradient dy = 2 (y - t_std) / n, and the pre-activation gradients of
// the three hidden layers.  The baseline of each sample is written by the
// member-0 blocks (the loss kernel reads it).
__global__ __launch_bounds__(256) void train_tile_f32_kernel(Model md, const float* __restrict__ X,
                                                             const float* __restrict__ t, int64_t n, TrainWs ws) {
  __shared__ float zs[kTileS * kIn];
  __shared__ float act[2][kTileS][kActStride];
  __shared__ float wl[kH][kWS];
  __shared__ SmallP sp;
  __shared__ float yp[4][kTileS];
  __shared__ float ys[kTileS], dys[kTileS];
  __shared__ double bp[4][kTileS];
  const Header& H = *md.hdr;
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int m = blockIdx.y;
  const int64_t s0 = (int64_t)blockIdx.x * kTileS;
  const float* master = md.master + (size_t)m * kP;
  const size_t nh = (size_t)n * kH;
  const ForwardOut st{ws.z + (size_t)m * n * kIn, ws.a1 + m * nh, ws.a2 + m * nh, ws.a3 + m * nh,
                      ws.h1 + m * nh, ws.h2 + m * nh, ws.h3 + m * nh, ws.y + (size_t)m * n};
  WRegs pf;
  wload(pf, master + oW2);
  // the baseline and target of each sample, while W2 is on its way
  base_parts(H, X, n, s0, bp);
  __syncthreads();
  const int64_t gt = s0 + tid;
  float ty = 0.0f;
  if (tid < kTileS && gt < n) {
    const float base = (float)base_of(H, X, gt, bp, tid);
    if (m == 0) ws.base[gt] = base;
    ty = (t[gt] - base - H.t_mu) / H.t_sigma;
  }
  forward_tile_f32(H, master, X, n, s0, zs, act, wl, sp, yp, ys, pf, master + oW2, st);
  if (tid < kTileS) {
    float dy = 0.0f;
    if (gt < n) {
      dy = 2.0f * (ys[tid] - ty) / (float)n;
      ws.dy[(size_t)m * n + gt] = dy;
    }
    dys[tid] = dy;
  }
  __syncthreads();
  // d3 = dy w4 silu'(a3) -> act[1]; the pre-activations are read first
  float* d3 = ws.d3 + m * nh;
  float a3[kH / 16][4];
#pragma unroll
  for (int tt = 0; tt < kH / 16; ++tt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gs = s0 + wave * 16 + 4 * (lane >> 4) + v;
      a3[tt][v] = gs < n ? st.a3[gs * kH + tt * 16 + (lane & 15)] : 0.0f;
    }
#pragma unroll
  for (int tt = 0; tt < kH / 16; ++tt) {
    const int o = tt * 16 + (lane & 15);
    const float w4 = sp.b3w4b4[kH + o];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = wave * 16 + 4 * (lane >> 4) + v;
      const int64_t gs = s0 + s;
      float dv = 0.0f;
      if (gs < n) {
        dv = dys[s] * w4 * dsilu(a3[tt][v]);
        d3[gs * kH + o] = dv;
      }
      act[1][s][o] = dv;
    }
  }
  __syncthreads();
  layer_bwd_f32(act[1], act[0], wl, st.a2, n, s0, ws.d2 + m * nh);  // wl holds W3
  wstore(pf, wl);                                                   // W2
  __syncthreads();
  layer_bwd_f32(act[0], nullptr, wl, st.a1, n, s0, ws.d1 + m * nh);
}

// ---------------------------------------------------------------------------
// BF16 models: hidden activations rounded to BF16 before the next layer,
// the 128 x 128 layers on v_mfma_f32_16x16x16_bf16.
//
// Forward pass of one member over samples [s0, s0 + 64) (256 threads).
// Leaves the standardised outputs in ys[64] (LDS).
template <bool STORE>
__device__ void forward_tile_bf16(const Header& H, const float* __restrict__ master,
                                  const unsigned short* __restrict__ w, const float* __restrict__ X, int64_t n,
                                  int64_t s0, float* zs /*[64][6]*/, unsigned short (*act)[kTileS][kActStride],
                                  float* ys, const ForwardOut& st) {
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  // standardised inputs
  for (int q = tid; q < kTileS * kIn; q += 256) {
    const int s = q / kIn, i = q % kIn;
    const int64_t gs = s0 + s;
    float zv = 0.0f;
    if (gs < n) zv = (logf(X[gs * kIn + i]) - H.mu[i]) / H.sigma[i];
    zs[q] = zv;
    if (STORE && gs < n) st.z[gs * kIn + i] = zv;
  }
  __syncthreads();
  // layer 1 (FP32 arithmetic on the BF16 weights)
  for (int q = tid; q < kTileS * kH; q += 256) {
    const int s = q / kH, o = q % kH;
    float a = master[ob1 + o];
#pragma unroll
    for (int i = 0; i < kIn; ++i) a += from_bf16(w[oW1 + o * kIn + i]) * zs[s * kIn + i];
    const unsigned short h = to_bf16(silu(a));
    act[0][s][o] = h;
    const int64_t gs = s0 + s;
    if (STORE && gs < n) {
      st.a1[gs * kH + o] = a;
      st.h1[gs * kH + o] = from_bf16(h);
    }
  }
  __syncthreads();
  // layers 2 and 3: wave w owns samples 16w..16w+15
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const int oW = layer == 0 ? oW2 : oW3, ob = layer == 0 ? ob2 : ob3;
    const unsigned short (*in)[kActStride] = act[layer];
    unsigned short (*out)[kActStride] = act[1 - layer];
    float* sa = layer == 0 ? st.a2 : st.a3;
    float* sh = layer == 0 ? st.h2 : st.h3;
    const int arow = wave * 16 + (lane & 15);  // A: sample row of this lane
    const int kq = 4 * (lane >> 4);            // A/B: k offset within the 16-wide step
#pragma unroll 1
    for (int nt = 0; nt < kH / 16; ++nt) {
      float4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
      const int bo = nt * 16 + (lane & 15);  // B: output column of this lane
#pragma unroll
      for (int kk = 0; kk < kH / 16; ++kk) {
        const int k = kk * 16 + kq;
        short4_t a, b;
        a[0] = (short)in[arow][k];
        a[1] = (short)in[arow][k + 1];
        a[2] = (short)in[arow][k + 2];
        a[3] = (short)in[arow][k + 3];
        const unsigned short* wr = w + oW + bo * kH + k;
        b[0] = (short)wr[0];
        b[1] = (short)wr[1];
        b[2] = (short)wr[2];
        b[3] = (short)wr[3];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
      }
      // D[i][j]: sample i = 4 (lane/16) + v, output j = lane % 16
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int s = wave * 16 + 4 * (lane >> 4) + v;
        const float a = acc[v] + master[ob + bo];
        const unsigned short h = to_bf16(silu(a));
        out[s][bo] = h;
        const int64_t gs = s0 + s;
        if (STORE && gs < n) {
          sa[gs * kH + bo] = a;
          sh[gs * kH + bo] = from_bf16(h);
        }
      }
    }
    __syncthreads();
  }
  // output layer (FP32 dot); act[0] holds h3
  if (tid < kTileS) {
    float y = master[ob4];
    for (int i = 0; i < kH; ++i) y += from_bf16(w[ow4 + i]) * from_bf16(act[0][tid][i]);
    ys[tid] = y;
    const int64_t gs = s0 + tid;
    if (STORE && gs < n) st.y[gs] = y;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void forward_train_bf16_kernel(Model md, const float* X, int64_t n, TrainWs ws) {
  if (blockIdx.y == 0 && threadIdx.x < kTileS) {  // baseline of each sample (member independent)
    const int64_t gs = (int64_t)blockIdx.x * kTileS + threadIdx.x;
    if (gs < n) ws.base[gs] = md.hdr->use_baseline ? (float)baseline(*md.hdr, X + gs * kIn) : 0.0f;
  }
  __shared__ float zs[kTileS * kIn];
  __shared__ unsigned short act[2][kTileS][kActStride];
  __shared__ float ys[kTileS];
  const int m = blockIdx.y;
  const size_t nh = (size_t)n * kH;
  ForwardOut st{ws.z + (size_t)m * n * kIn, ws.a1 + m * nh, ws.a2 + m * nh, ws.a3 + m * nh,
                ws.h1 + m * nh, ws.h2 + m * nh, ws.h3 + m * nh, ws.y + (size_t)m * n};
  forward_tile_bf16<true>(*md.hdr, md.master + (size_t)m * kP, md.w + (size_t)m * kPpad, X, n,
                          (int64_t)blockIdx.x * kTileS, zs, act, ys, st);
}

// Per-sample deltas of a BF16 model: dy = 2 (y - t)/n, then the
// pre-activation gradients of the three hidden layers (block of 128
// threads = hidden units; the casts pass gradients straight through).
__global__ __launch_bounds__(128) void delta_bf16_kernel(Model md, const float* t, int64_t n, TrainWs ws) {
  __shared__ float d[kH];
  const int m = blockIdx.y, o = threadIdx.x;
  const int64_t s = blockIdx.x;
  const size_t nh = (size_t)n * kH, row = m * nh + (size_t)s * kH;
  const unsigned short* w = md.w + (size_t)m * kPpad;
  const float ty = (t[s] - ws.base[s] - md.hdr->t_mu) / md.hdr->t_sigma;
  const float dy = 2.0f * (ws.y[(size_t)m * n + s] - ty) / (float)n;
  if (o == 0) ws.dy[(size_t)m * n + s] = dy;
  float da = dy * from_bf16(w[ow4 + o]) * dsilu(ws.a3[row + o]);
  ws.d3[row + o] = da;
  d[o] = da;
  __syncthreads();
  float g = 0.0f;
  for (int j = 0; j < kH; ++j) g += from_bf16(w[oW3 + j * kH + o]) * d[j];
  da = g * dsilu(ws.a2[row + o]);
  ws.d2[row + o] = da;
  __syncthreads();
  d[o] = da;
  __syncthreads();
  g = 0.0f;
  for (int j = 0; j < kH; ++j) g += from_bf16(w[oW2 + j * kH + o]) * d[j];
  ws.d1[row + o] = g * dsilu(ws.a1[row + o]);
}

// ---------------------------------------------------------------------------
// Weight gradients G[o][i] = sum_s delta[s][o] * in[s][i] (in[s][K] = 1
// gives the bias) of the four layers, in one launch: block x of the grid
// walks the jobs' 16 x 16 tiles of (o, i) in turn, block y is the member.
struct GradJob {
  const float* delta;  // [n][rows_d]
  int rows_d;          // width of delta rows (128 or 1)
  const float* in;     // [n][K]
  int K;
  int nO;              // outputs (128 or 1)
  int w_off, b_off;    // parameter offsets of weights [nO][K] and bias [nO]
  size_t delta_stride, in_stride;  // member strides
  int tiles_x, first;  // tiles along i; first block of the job
};

struct GradJobs {
  GradJob job[4];
};

// One 16 x 16 tile of G per block on FP32 MFMA (v_mfma_f32_16x16x4f32,
// A[i][k]: lane i + 16 k, B[k][j]: lane j + 16 k, D[i][j]: lane j + 16 (i/4),
// item i % 4): A = delta (outputs x samples), B = inputs (samples x inputs,
// the column after the last input is 1 for the bias).  The block's 4 waves
// take interleaved groups of 4 samples, sum them in fixed order through LDS:
// deterministic.
__global__ __launch_bounds__(256) void wgrad_kernel(GradJobs jobs, int64_t n, float* grad) {
  __shared__ float part[4][16][16];
  int jn = 0;
#pragma unroll
  for (int q = 1; q < 4; ++q)
    if ((int)blockIdx.x >= jobs.job[q].first) jn = q;
  const GradJob& job = jobs.job[jn];
  const int m = blockIdx.y;
  const float* __restrict__ delta = job.delta + m * job.delta_stride;
  const float* __restrict__ in = job.in + m * job.in_stride;
  const int tile = blockIdx.x - job.first;
  const int o0 = (tile / job.tiles_x) * 16, i0 = (tile % job.tiles_x) * 16;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = lane & 15, k = lane >> 4;
  const int o = o0 + r, i = i0 + r;  // A row (output) and B column (input) of this lane
  const bool o_ok = o < job.nO;
  const float bias_one = i == job.K ? 1.0f : 0.0f;
  float4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
  // samples sb + k with the wave-uniform base sb = 16 g + 4 wave, g = 0, 1,
  // ...: each MFMA takes 4 samples; loop bounds are uniform over the wave
  constexpr int kU = 32;  // MFMAs per unrolled group (loads issued ahead)
  int64_t sb = 4 * wave;
  for (; sb + 16 * (kU - 1) + 3 < n; sb += 16 * kU) {
    float a[kU], b[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t su = sb + 16 * u + k;
      a[u] = o_ok ? delta[su * job.rows_d + o] : 0.0f;
      b[u] = i < job.K ? in[su * job.K + i] : bias_one;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
  }
  for (; sb < n; sb += 16) {  // the tail: one group of 4 samples per MFMA, missing samples as zeros
    const int64_t su = sb + k;
    const bool in_range = su < n;
    const float a = in_range && o_ok ? delta[su * job.rows_d + o] : 0.0f;
    const float b = in_range ? (i < job.K ? in[su * job.K + i] : bias_one) : 0.0f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) part[wave][4 * k + v][r] = acc[v];  // D[4k + v][r]
  __syncthreads();
  {
    const int oo = threadIdx.x / 16, ii = threadIdx.x % 16;
    const float g = ((part[0][oo][ii] + part[1][oo][ii]) + part[2][oo][ii]) + part[3][oo][ii];
    const int og = o0 + oo, ig = i0 + ii;
    if (og < job.nO && ig <= job.K) {
      float* gm = grad + (size_t)m * kP;
      if (ig < job.K) gm[job.w_off + og * job.K + ig] = g;
      else gm[job.b_off + og] = g;
    }
  }
}
__global__ void adam_kernel(Model md, const float* grad, int M, float lr, int step) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)M * kP) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = grad[q];
  const float m = b1 * md.m[q] + (1.0f - b1) * g;
  const float v = b2 * md.v[q] + (1.0f - b2) * g * g;
  md.m[q] = m;
  md.v[q] = v;
  const float mh = m / (1.0f - powf(b1, (float)step));
  const float vh = v / (1.0f - powf(b2, (float)step));
  const float p = md.master[q] - lr * mh / (sqrtf(vh) + eps);
  md.master[q] = p;
  const int64_t mem = q / kP, k = q % kP;
  md.w[mem * kPpad + k] = to_bf16(p);
}

__global__ void to_bf16_kernel(Model md, int M) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)M * kP) return;
  md.w[(q / kP) * kPpad + q % kP] = to_bf16(md.master[q]);
}

__global__ __launch_bounds__(1024) void loss_kernel(Model md, const float* t, int64_t n, TrainWs ws) {
  const int m = blockIdx.x;
  __shared__ float part[16];
  float s = 0.0f;
  for (int64_t q = threadIdx.x; q < n; q += 1024) {
    const float r = ws.y[(size_t)m * n + q] - (t[q] - ws.base[q] - md.hdr->t_mu) / md.hdr->t_sigma;
    s += r * r;
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float tot = 0.0f;
    for (int w = 0; w < 16; ++w) tot += part[w];
    ws.loss[m] = tot / (float)n;
  }
}

// Ensemble query: mean and spread (max - min) of ln k_s over the members,
// out-of-box test of the standardised inputs, fallback flag and the number
// of flagged queries per block.  Per tile of 64 queries, after the members'
// forward passes (LDS ys, summed into ysum/ymin/ymax).
__device__ inline void query_finish(const Header& H, const float* __restrict__ X, int64_t n, int64_t s0,
                                    float spread_tol, const float* zs, float* ysum, float* ymin, float* ymax,
                                    double (*bp)[kTileS], float* mean, float* spread, unsigned char* fallback,
                                    int* cnt, int* block_count) {
  const int tid = threadIdx.x;
  base_parts(H, X, n, s0, bp);
  __syncthreads();
  if (tid < kTileS && s0 + tid < n) {
    const int64_t gs = s0 + tid;
    const float base = (float)base_of(H, X, gs, bp, tid);
    ysum[tid] += (float)H.members * base;
    ymin[tid] += base;
    ymax[tid] += base;
    bool out = false;
    for (int i = 0; i < kIn; ++i) {
      const float z = zs[tid * kIn + i];
      out = out || !(z >= H.lo[i] && z <= H.hi[i]);
    }
    const float sp = ymax[tid] - ymin[tid];
    mean[gs] = ysum[tid] / (float)H.members;
    spread[gs] = sp;
    const bool fb = out || !(sp <= spread_tol);
    fallback[gs] = fb ? 1 : 0;
    if (fb) atomicAdd(cnt, 1);
  }
  __syncthreads();
  if (tid == 0) block_count[blockIdx.x] = *cnt;
}

__device__ inline void query_accumulate(const Header& H, int m, const float* ys, float* ysum, float* ymin,
                                        float* ymax) {
  const int tid = threadIdx.x;
  if (tid < kTileS) {
    const float v = ys[tid] * H.t_sigma + H.t_mu;
    ysum[tid] = m == 0 ? v : ysum[tid] + v;
    ymin[tid] = m == 0 ? v : fminf(ymin[tid], v);
    ymax[tid] = m == 0 ? v : fmaxf(ymax[tid], v);
  }
  __syncthreads();
}

// Two blocks per CU (78 KB of LDS each, at most 256 registers per lane).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void query_f32_kernel(
    Model md, const float* __restrict__ X, int64_t n, float spread_tol, float* mean, float* spread,
    unsigned char* fallback, int* block_count) {
  __shared__ float zs[kTileS * kIn];
  __shared__ float act[kTileS][kActStride];
  __shared__ float wl[kH / 2][kWS];
  __shared__ SmallP sp;
  __shared__ float yp[4][kTileS];
  __shared__ float ys[kTileS], ymin[kTileS], ymax[kTileS], ysum[kTileS];
  __shared__ double bp[4][kTileS];
  __shared__ int cnt;
  const Header& H = *md.hdr;
  const int64_t s0 = (int64_t)blockIdx.x * kTileS;
  if (threadIdx.x == 0) cnt = 0;
  WHalf pf;
  wload_half(pf, md.master + oW2, 0);
  for (int m = 0; m < H.members; ++m) {
    const float* master = md.master + (size_t)m * kP;
    const float* next = m + 1 < H.members ? master + kP + oW2 : nullptr;
    forward_query_f32(H, master, X, n, s0, zs, act, wl, sp, yp, ys, pf, next);
    query_accumulate(H, m, ys, ysum, ymin, ymax);
  }
  query_finish(H, X, n, s0, spread_tol, zs, ysum, ymin, ymax, bp, mean, spread, fallback, &cnt, block_count);
}

__global__ __launch_bounds__(256) void query_bf16_kernel(Model md, const float* __restrict__ X, int64_t n,
                                                         float spread_tol, float* mean, float* spread,
                                                         unsigned char* fallback, int* block_count) {
  __shared__ float zs[kTileS * kIn];
  __shared__ unsigned short act[2][kTileS][kActStride];
  __shared__ float ys[kTileS], ymin[kTileS], ymax[kTileS], ysum[kTileS];
  __shared__ double bp[4][kTileS];
  __shared__ int cnt;
  const Header& H = *md.hdr;
  const int64_t s0 = (int64_t)blockIdx.x * kTileS;
  if (threadIdx.x == 0) cnt = 0;
  const ForwardOut none{};
  for (int m = 0; m < H.members; ++m) {
    forward_tile_bf16<false>(H, md.master + (size_t)m * kP, md.w + (size_t)m * kPpad, X, n, s0, zs, act, ys,
                             none);
    query_accumulate(H, m, ys, ysum, ymin, ymax);
  }
  query_finish(H, X, n, s0, spread_tol, zs, ysum, ymin, ymax, bp, mean, spread, fallback, &cnt, block_count);
}
// Ordered compaction of the flagged query indices: an exclusive scan of the
// per-block counts (one block), then each block writes its flagged indices
// in order.
__global__ __launch_bounds__(1024) void scan_kernel(const int* block_count, int nblocks, int* block_off,
                                                    int64_t* total) {
  __shared__ int buf[1024];
  int carry = 0;
  for (int b0 = 0; b0 < nblocks; b0 += 1024) {
    const int b = b0 + threadIdx.x;
    const int v = b < nblocks ? block_count[b] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
      const int u = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += u;
      __syncthreads();
    }
    if (b < nblocks) block_off[b] = carry + buf[threadIdx.x] - v;
    const int last = buf[1023];
    __syncthreads();
    carry += last;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kTileS) void scatter_kernel(const unsigned char* fallback, int64_t n,
                                                         const int* block_off, int64_t* idx) {
  const int64_t s0 = (int64_t)blockIdx.x * kTileS;
  const int64_t gs = s0 + threadIdx.x;
  const bool f = gs < n && fallback[gs];
  const unsigned long long mask = __ballot(f);
  if (f) {
    const unsigned long long below = mask & ((1ull << threadIdx.x) - 1ull);
    idx[block_off[blockIdx.x] + __popcll(below)] = gs;
  }
}

__global__ void baseline_kernel(Model md, const float* X, int64_t n, double* out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = baseline(*md.hdr, X + q * kIn);
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on the
// Legendre polynomial (three-term recursion).
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace
}  // namespace it

using namespace it;

extern "C" {

int it_mlp_model_bytes(int32_t members, size_t* bytes) {
  if (!bytes || members < 1 || members > 64) return IT_EINVAL;
  *bytes = model_bytes(members);
  return IT_OK;
}

int it_mlp_init(void* d_model, int32_t members, const float* h_params, const float* h_norm, const double* h_phys,
                int32_t precision, void* stream_) {
  clear_stale_error();
  if (!d_model || !h_params || !h_norm || members < 1 || members > 64) return IT_EINVAL;
  if (precision != IT_MLP_BF16 && precision != IT_MLP_FP32) return IT_EINVAL;
  hipStream_t s = (hipStream_t)stream_;
  Model md = carve_model(d_model, members);
  Header h;
  std::memset(&h, 0, sizeof(h));
  h.members = members;
  h.precision = precision;
  for (int i = 0; i < kIn; ++i) {
    h.mu[i] = h_norm[i];
    h.sigma[i] = h_norm[kIn + i];
    h.lo[i] = h_norm[2 * kIn + i];
    h.hi[i] = h_norm[3 * kIn + i];
    if (!(h.sigma[i] > 0.0f) || !(h.lo[i] <= h.hi[i])) return IT_EINVAL;
  }
  h.t_mu = h_norm[4 * kIn];
  h.t_sigma = h_norm[4 * kIn + 1];
  if (!(h.t_sigma > 0.0f)) return IT_EINVAL;
  if (h_phys) {
    h.use_baseline = 1;
    h.D = h_phys[0];
    h.mu_avg = h_phys[1];
    h.alpha = h_phys[2];
    h.W = h_phys[3];
    h.mu_sum = h_phys[4];
    h.pairs_per_mGy = h_phys[5];
    for (int q = 0; q < 6; ++q)
      if (!(std::isfinite(h_phys[q]) && h_phys[q] > 0.0)) return IT_EINVAL;
    gauss_legendre(kGL, h.gl_x, h.gl_w);
  }
  if (hipMemcpyAsync(md.hdr, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(md.master, h_params, (size_t)members * kP * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(md.m, 0, (size_t)members * kP * 4, s) != hipSuccess ||
      hipMemsetAsync(md.v, 0, (size_t)members * kP * 4, s) != hipSuccess)
    return IT_EHIP;
  hipLaunchKernelGGL(to_bf16_kernel, dim3((members * kP + 255) / 256), dim3(256), 0, s, md, members);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return IT_EHIP;
  return IT_OK;
}

int it_mlp_train_ws_bytes(int32_t members, int64_t n, size_t* bytes) {
  if (!bytes || members < 1 || members > 64 || n < 1) return IT_EINVAL;
  *bytes = train_ws_bytes(members, n);
  return IT_OK;
}

static int launch_grad(const Model& md, int M, bool f32, const float* X, const float* t, int64_t n,
                       const TrainWs& w, hipStream_t s) {
  const int nb = (int)((n + kTileS - 1) / kTileS);
  if (f32) {
    hipLaunchKernelGGL(train_tile_f32_kernel, dim3(nb, M), dim3(256), 0, s, md, X, t, n, w);
  } else {
    hipLaunchKernelGGL(forward_train_bf16_kernel, dim3(nb, M), dim3(256), 0, s, md, X, n, w);
    hipLaunchKernelGGL(delta_bf16_kernel, dim3((unsigned)n, M), dim3(kH), 0, s, md, t, n, w);
  }
  const size_t nh = (size_t)n * kH;
  GradJobs jobs = {{
      {w.d3, kH, w.h2, kH, kH, oW3, ob3, nh, nh, 0, 0},
      {w.d2, kH, w.h1, kH, kH, oW2, ob2, nh, nh, 0, 0},
      {w.d1, kH, w.z, kIn, kH, oW1, ob1, nh, (size_t)n * kIn, 0, 0},
      {w.dy, 1, w.h3, kH, 1, ow4, ob4, (size_t)n, nh, 0, 0},
  }};
  int blocks = 0;
  for (GradJob& g : jobs.job) {
    g.tiles_x = (g.K + 1 + 15) / 16;
    g.first = blocks;
    blocks += g.tiles_x * ((g.nO + 15) / 16);
  }
  hipLaunchKernelGGL(wgrad_kernel, dim3(blocks, M), dim3(256), 0, s, jobs, n, w.grad);
  return hipGetLastError() == hipSuccess ? IT_OK : IT_EHIP;
}

int it_mlp_grad(const void* d_model, int32_t members, const float* d_X, const float* d_t, int64_t n,
                float* d_grad, float* h_loss, void* d_ws, size_t ws_bytes, void* stream_) {
  clear_stale_error();
  if (!d_model || !d_X || !d_t || !d_grad || n < 1 || members < 1 || members > 64) return IT_EINVAL;
  if (!d_ws || ws_bytes < train_ws_bytes(members, n)) return IT_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream_;
  Model md = carve_model((void*)d_model, members);
  TrainWs w = carve_train(d_ws, members, n);
  Header h;
  if (hipMemcpyAsync(&h, md.hdr, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return IT_EHIP;
  int rc = launch_grad(md, members, h.precision == IT_MLP_FP32, d_X, d_t, n, w, s);
  if (rc) return rc;
  if (hipMemcpyAsync(d_grad, w.grad, (size_t)members * kP * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return IT_EHIP;
  if (h_loss) {
    hipLaunchKernelGGL(loss_kernel, dim3(members), dim3(1024), 0, s, md, d_t, n, w);
    if (hipMemcpyAsync(h_loss, w.loss, members * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return IT_EHIP;
  }
  return hipStreamSynchronize(s) == hipSuccess ? IT_OK : IT_EHIP;
}

int it_mlp_train(void* d_model, int32_t members, const float* d_X, const float* d_t, int64_t n, int64_t batch,
                 int32_t steps, float lr, float lr_final, int32_t log_every, float* h_loss, void* d_ws,
                 size_t ws_bytes, void* stream_) {
  clear_stale_error();
  if (!d_model || !d_X || !d_t || n < 1 || steps < 0 || members < 1 || members > 64 || !(lr > 0.0f) ||
      !(lr_final > 0.0f) || batch < 0 || batch > n)
    return IT_EINVAL;
  const int64_t rows = batch ? batch : n;
  if (n % rows) return IT_EINVAL;  // the minibatches tile the data
  if (!d_ws || ws_bytes < train_ws_bytes(members, rows)) return IT_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream_;
  Model md = carve_model(d_model, members);
  TrainWs w = carve_train(d_ws, members, rows);
  Header h;
  if (hipMemcpyAsync(&h, md.hdr, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return IT_EHIP;
  const int64_t nbatch = n / rows;
  int nlog = 0;
  for (int k = 0; k < steps; ++k) {
    // minibatch: the next contiguous window of the data, continuing across calls
    const int64_t b0 = ((h.step + k) % nbatch) * rows;
    const float* X = d_X + b0 * kIn;
    const float* t = d_t + b0;
    int rc = launch_grad(md, members, h.precision == IT_MLP_FP32, X, t, rows, w, s);
    if (rc) return rc;
    if (h_loss && log_every > 0 && k % log_every == 0) {
      hipLaunchKernelGGL(loss_kernel, dim3(members), dim3(1024), 0, s, md, t, rows, w);
      if (hipMemcpyAsync(h_loss + (size_t)nlog * members, w.loss, members * 4, hipMemcpyDeviceToHost, s) !=
          hipSuccess)
        return IT_EHIP;
      ++nlog;
    }
    // cosine decay from lr to lr_final over the steps of this call
    const double frac = steps > 1 ? (double)k / (double)(steps - 1) : 0.0;
    const double lr0 = lr, lr1 = lr_final;  // in FP64: the end points are exact
    const float lr_k = (float)(lr1 + 0.5 * (lr0 - lr1) * (1.0 + std::cos(M_PI * frac)));
    hipLaunchKernelGGL(adam_kernel, dim3((members * kP + 255) / 256), dim3(256), 0, s, md, w.grad, members, lr_k,
                       h.step + k + 1);
    if (hipGetLastError() != hipSuccess) return IT_EHIP;
  }
  h.step += steps;
  if (hipMemcpyAsync(md.hdr, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess) return IT_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? IT_OK : IT_EHIP;
}

int it_mlp_baseline(const void* d_model, const float* d_X, int64_t n, double* d_out, void* stream_) {
  clear_stale_error();
  if (!d_model || n < 0 || (n > 0 && (!d_X || !d_out))) return IT_EINVAL;
  if (n == 0) return IT_OK;
  hipStream_t s = (hipStream_t)stream_;
  Model md = carve_model((void*)d_model, 1);  // only the header is read
  hipLaunchKernelGGL(baseline_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, md, d_X, n, d_out);
  return hipGetLastError() == hipSuccess ? IT_OK : IT_EHIP;
}

int it_mlp_query_ws_bytes(int64_t nq, size_t* bytes) {
  if (!bytes || nq < 0) return IT_EINVAL;
  const int64_t nb = (nq + kTileS - 1) / kTileS;
  *bytes = align256((size_t)nb * 4) * 2 + 256;
  return IT_OK;
}

}  // extern "C"

namespace it {
namespace {

// The query with its scratch (per-tile fallback counts and offsets, the
// total) at d_ws, it_mlp_query_ws_bytes(nq) bytes.
int query(const void* d_model, const float* d_X, int64_t nq, float spread_tol, float* d_mean, float* d_spread,
          unsigned char* d_fallback, int64_t* d_fallback_idx, int64_t* h_nfallback, void* d_ws, hipStream_t s) {
  if (nq == 0) {
    if (h_nfallback) *h_nfallback = 0;
    return IT_OK;
  }
  Model md = carve_model((void*)d_model, 1);  // header and first arrays; members read from the header
  Header h;
  if (hipMemcpyAsync(&h, md.hdr, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return IT_EHIP;
  md = carve_model((void*)d_model, h.members);
  const int nb = (int)((nq + kTileS - 1) / kTileS);
  char* p = (char*)d_ws;
  int* counts = (int*)p;
  int* offs = (int*)(p + align256((size_t)nb * 4));
  int64_t* total = (int64_t*)(p + 2 * align256((size_t)nb * 4));
  if (h.precision == IT_MLP_FP32)
    hipLaunchKernelGGL(query_f32_kernel, dim3(nb), dim3(256), 0, s, md, d_X, nq, spread_tol, d_mean, d_spread,
                       d_fallback, counts);
  else
    hipLaunchKernelGGL(query_bf16_kernel, dim3(nb), dim3(256), 0, s, md, d_X, nq, spread_tol, d_mean, d_spread,
                       d_fallback, counts);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, counts, nb, offs, total);
  if (d_fallback_idx)
    hipLaunchKernelGGL(scatter_kernel, dim3(nb), dim3(kTileS), 0, s, d_fallback, nq, offs, d_fallback_idx);
  if (hipGetLastError() != hipSuccess) return IT_EHIP;
  if (h_nfallback) {
    if (hipMemcpyAsync(h_nfallback, total, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return IT_EHIP;
  }
  return IT_OK;
}

// Scratch of the allocation-free query: a file-scope device array, one copy
// per GPU, held until the process ends.  Its device address is taken once
// per device (with that device current) and kept: in host code the array's
// name is only a stand-in for it.  Nothing in it needs to start at zero
// (every query tile writes its own count, the scan writes the offsets and
// the total).
constexpr int64_t kStaticQueries = IT_MLP_QUERY_STATIC_MAX;
constexpr size_t kStaticScratchBytes = 2 * (((size_t)kStaticQueries / kTileS * 4 + 255) / 256 * 256) + 256;
__device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

void* static_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    scratch_ptr[dev] = ptr;
  }
  return scratch_ptr[dev];
}

}  // namespace
}  // namespace it

extern "C" {

int it_mlp_query(const void* d_model, const float* d_X, int64_t nq, float spread_tol, float* d_mean,
                 float* d_spread, unsigned char* d_fallback, int64_t* d_fallback_idx, int64_t* h_nfallback,
                 void* d_ws, size_t ws_bytes, void* stream_) {
  clear_stale_error();
  if (!d_model || nq < 0 || (nq > 0 && (!d_X || !d_mean || !d_spread || !d_fallback))) return IT_EINVAL;
  size_t need;
  it_mlp_query_ws_bytes(nq, &need);
  if (!d_ws || ws_bytes < need) return IT_EWORKSPACE;
  return query(d_model, d_X, nq, spread_tol, d_mean, d_spread, d_fallback, d_fallback_idx, h_nfallback, d_ws,
               (hipStream_t)stream_);
}

int it_mlp_query_static(const void* d_model, const float* d_X, int64_t nq, float spread_tol, float* d_mean,
                        float* d_spread, unsigned char* d_fallback, int64_t* d_fallback_idx, int64_t* h_nfallback,
                        void* stream_) {
  clear_stale_error();
  if (!d_model || nq < 0 || nq > kStaticQueries || (nq > 0 && (!d_X || !d_mean || !d_spread || !d_fallback)))
    return IT_EINVAL;
  size_t need;
  it_mlp_query_ws_bytes(nq, &need);
  if (need > kStaticScratchBytes) return IT_EINVAL;
  void* ws = static_scratch();
  if (!ws) return IT_EHIP;
  return query(d_model, d_X, nq, spread_tol, d_mean, d_spread, d_fallback, d_fallback_idx, h_nfallback, ws,
               (hipStream_t)stream_);
}

}  // extern "C"
