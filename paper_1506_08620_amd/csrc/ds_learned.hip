// Learned replacement of the Direct table (not from the paper): a monotone CDF
// model routes a query to one of S segments, a per-segment linear fit
// predicts its index, recorded error bounds give a window, and a branch-free
// binary search inside the window finds the index exactly.
//
// Exactness does not depend on the quality of the model:
//   * the feature u(z) and the router y(u) are non-decreasing functions of z,
//     evaluated by the same device code for the keys at build time and for
//     the queries, so routing is monotone: if the keys X_a .. X_{b-1} route to
//     segment s, every query routed to s has its index in [a-1, b-1];
//   * the fit's prediction is non-decreasing in z too, so the key errors over
//     [a-1, b] bound the query's index relative to the prediction;
//   * every result is verified against X_i <= z < X_{i+1}; a failure (never
//     expected) falls back to a full binary search and is counted.
//
// Network: u -> 32 -> 32 -> 1, hidden units clamp(x, 0, 1), weights kept
// >= 0 (projected after every Adam step), so y(u) is monotone.  Training
// minimises the mean squared error of y(u(X_i)) against i / N with
// hand-written forward/backward kernels (one thread per sample, deterministic
// per-workgroup partial gradients) and an Adam kernel.  At search time the
// 32x32 layer runs on the matrix cores (v_mfma_f32_32x32x2f32), 32 queries
// per wave and pass.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <type_traits>
#include <vector>

#include "ds_batched_internal.h"
#include "ds_ops.h"

namespace ds {

constexpr int kHid = 32;
constexpr int kParams = 2 * kHid + kHid * kHid + kHid + kHid + 1;  // 1153
static_assert(kParams == kRouterParams, "router parameter count");
constexpr int oW1 = 0, oB1 = 32, oW2 = 64, oB2 = 64 + 1024, oW3 = 64 + 1024 + 32, oB3 = 64 + 1024 + 64;
constexpr int kTrainBlock = 256;

// per-segment fit: prediction p = a (z - zc) + b (relative to lo), window
// [lo + floor(p) + dmin - 1, lo + floor(p) + dmax] clipped to [lo, hi]
struct alignas(16) SegFit {
  double zc;
  float a, b;
  int32_t dmin, dmax, lo, hi;
};
static_assert(sizeof(SegFit) == kSegFitBytes, "segment record size");

struct LearnedModel {
  float* params = nullptr;      // kParams
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* partial = nullptr;     // per-workgroup gradients
  float* loss_partial = nullptr;
  float* feat = nullptr;        // u of every key
  int32_t* route = nullptr;     // segment of every key
  int32_t* first = nullptr;     // nseg + 1: first key of each segment
  SegFit* segs = nullptr;
  float* steps = nullptr;       // compiled router: nseg step positions (see router_steps_kernel)
  uint32_t* grid = nullptr;     // compiled router: 2^log2g grid cells over u (grid_segment)
  int32_t log2g = 0;
  void* samples = nullptr;      // S[j] = X_{E j} (single-array search)
  int64_t nsamples = 0;
  unsigned long long* fallbacks = nullptr;
  int32_t nseg = 0;
  int32_t identity = 0;         // ablation: y = u
  int32_t router = 0;           // kRouteTable, kRouteF16 or kRouteF32
  double delta = 0, flo = 0, fscale = 0;
  int64_t max_err = 0;
  double mean_log2_window = 0;
  double final_loss = 0;
};

namespace {

using floatx16 = float __attribute__((ext_vector_type(16)));

// Monotone feature of a query: the bit pattern of d = max(z - X_0, 0) + delta
// read as an integer is a non-decreasing, roughly logarithmic function of d;
// it is scaled to [0, 1] and rounded to f32.  Every step is non-decreasing.
__host__ __device__ __forceinline__ float feature(double z, double X0, double delta, double flo, double fscale) {
  double d = z - X0;
  d = std::fmax(d, 0.0) + delta;
  int64_t bits;
  __builtin_memcpy(&bits, &d, 8);
  const double f = (static_cast<double>(bits) - flo) * fscale;
  return static_cast<float>(std::fmin(std::fmax(f, 0.0), 1.0));
}

__device__ __forceinline__ float clamp01(float x) { return std::fmin(std::fmax(x, 0.0f), 1.0f); }

// Router weights held in registers by one lane.  Lane l works on query
// q = l % 32 and on the hidden units k = 2 kk + l / 32 of layer 1; for the
// 32x32 layer it supplies row j = l % 32 of W2 (A operand) and its own h1
// values (B operand); the output tile D[j][q] lands in lane q + 32 ((j / 4) % 2),
// register (j % 4) + 4 (j / 8).
struct RouterRegs {
  float w1[16], b1[16], w2[16], w3[16];
  floatx16 b2;
  float b3;
};

__device__ __forceinline__ int out_row(int r, int half) { return (r & 3) + 4 * half + 8 * (r >> 2); }

__device__ void load_router(const float* __restrict__ p, RouterRegs& R) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int m = lane & 31;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 2 * kk + half;
    R.w1[kk] = p[oW1 + k];
    R.b1[kk] = p[oB1 + k];
    R.w2[kk] = p[oW2 + m * kHid + k];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int j = out_row(r, half);
    R.b2[r] = p[oB2 + j];
    R.w3[r] = p[oW3 + j];
  }
  R.b3 = p[oB3];
}

// y(u) for the query of lane l % 32; all 64 lanes must call it, and lanes l
// and l ^ 32 must pass the same u.  Both lanes return the same y.
__device__ __forceinline__ float router_tail(const floatx16& acc, const RouterRegs& R) {
  float part = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) part = std::fma(R.w3[r], clamp01(acc[r]), part);
  const float other = __shfl_xor(part, 32, 64);
  return (part + other) + R.b3;  // a + b == b + a exactly, so both lanes agree
}

__device__ __forceinline__ float router_y(float u, const RouterRegs& R) {
  floatx16 acc = R.b2;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const float h1 = clamp01(std::fma(R.w1[kk], u, R.b1[kk]));
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(R.w2[kk], h1, acc, 0, 0, 0);
  }
  return router_tail(acc, R);
}

// Two independent 32-query passes interleaved, so each matrix instruction has
// the other chain's instruction to overlap with.  Each result is computed by
// exactly the same operations as router_y.
__device__ __forceinline__ void router_y2(float ua, float ub, const RouterRegs& R, float* ya, float* yb) {
  floatx16 acc_a = R.b2, acc_b = R.b2;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const float ha = clamp01(std::fma(R.w1[kk], ua, R.b1[kk]));
    const float hb = clamp01(std::fma(R.w1[kk], ub, R.b1[kk]));
    acc_a = __builtin_amdgcn_mfma_f32_32x32x2f32(R.w2[kk], ha, acc_a, 0, 0, 0);
    acc_b = __builtin_amdgcn_mfma_f32_32x32x2f32(R.w2[kk], hb, acc_b, 0, 0, 0);
  }
  *ya = router_tail(acc_a, R);
  *yb = router_tail(acc_b, R);
}

// The same network with the 32x32 layer's inputs (h1 and W2) rounded to
// FP16 and FP32 accumulation (v_mfma_f32_32x32x8f16, 4 instructions per pass
// instead of 16).  Rounding is monotone and W2 stays >= 0, so this router is
// monotone as well; it is a different (slightly coarser) function of u, and a
// model built with it is searched with it.  Lane l supplies, for block kb,
// the units k = 8 kb + 4 (l / 32) + c, c = 0..3.
using half4 = _Float16 __attribute__((ext_vector_type(4)));

struct RouterRegs16 {
  float w1[16], b1[16], w3[16];
  half4 w2[4];
  floatx16 b2;
  float b3;
};

__device__ void load_router16(const float* __restrict__ p, RouterRegs16& R) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int m = lane & 31;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = 8 * kb + 4 * half + c;
      R.w1[4 * kb + c] = p[oW1 + k];
      R.b1[4 * kb + c] = p[oB1 + k];
      R.w2[kb][c] = static_cast<_Float16>(p[oW2 + m * kHid + k]);
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int j = out_row(r, half);
    R.b2[r] = p[oB2 + j];
    R.w3[r] = p[oW3 + j];
  }
  R.b3 = p[oB3];
}

__device__ __forceinline__ float router_tail16(const floatx16& acc, const RouterRegs16& R) {
  float part = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) part = std::fma(R.w3[r], clamp01(acc[r]), part);
  const float other = __shfl_xor(part, 32, 64);
  return (part + other) + R.b3;
}

__device__ __forceinline__ void router16_y2(float ua, float ub, const RouterRegs16& R, float* ya, float* yb) {
  floatx16 acc_a = R.b2, acc_b = R.b2;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    half4 ha, hb;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      ha[c] = static_cast<_Float16>(clamp01(std::fma(R.w1[4 * kb + c], ua, R.b1[4 * kb + c])));
      hb[c] = static_cast<_Float16>(clamp01(std::fma(R.w1[4 * kb + c], ub, R.b1[4 * kb + c])));
    }
    acc_a = __builtin_amdgcn_mfma_f32_32x32x8f16(R.w2[kb], ha, acc_a, 0, 0, 0);
    acc_b = __builtin_amdgcn_mfma_f32_32x32x8f16(R.w2[kb], hb, acc_b, 0, 0, 0);
  }
  *ya = router_tail16(acc_a, R);
  *yb = router_tail16(acc_b, R);
}

// The FP16 router with its half-wave-uniform values (layer 1, b2, layer 3:
// lanes of one half of a wave use the same 16 of each) read from LDS, and only
// the lane's own row of W2 in registers.  The operations and their order are
// those of router16_y2, so y is bit-identical; what changes is the register
// footprint (about 30 fewer), which leaves the scheduler room to overlap the
// window search's loads.
struct RouterShared16 {
  float w1[2][16], b1[2][16], w3[2][16], b2[2][16];
  float b3;
};

// called by every thread of the workgroup (blockDim.x >= 64); a barrier must
// follow before use
__device__ void fill_router_shared16(const float* __restrict__ p, RouterShared16* S, half4* w2) {
  const int t = threadIdx.x;
  if (t < 64) {
    const int half = t >> 5, i = t & 31;
    if (i < 16) {
      const int k = 8 * (i >> 2) + 4 * half + (i & 3);
      S->w1[half][i] = p[oW1 + k];
      S->b1[half][i] = p[oB1 + k];
    } else {
      const int r = i - 16;
      const int j = out_row(r, half);
      S->b2[half][r] = p[oB2 + j];
      S->w3[half][r] = p[oW3 + j];
    }
    if (t == 0) S->b3 = p[oB3];
  }
  const int lane = t & 63, half = lane >> 5, m = lane & 31;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int c = 0; c < 4; ++c) w2[kb][c] = static_cast<_Float16>(p[oW2 + m * kHid + 8 * kb + 4 * half + c]);
}

__device__ __forceinline__ float router_tail16_shared(const floatx16& acc, const RouterShared16* S, int half) {
  float part = 0.0f;
  const float4* w3 = reinterpret_cast<const float4*>(S->w3[half]);
#pragma unroll
  for (int r4 = 0; r4 < 4; ++r4) {
    const float4 w = w3[r4];
    part = std::fma(w.x, clamp01(acc[4 * r4 + 0]), part);
    part = std::fma(w.y, clamp01(acc[4 * r4 + 1]), part);
    part = std::fma(w.z, clamp01(acc[4 * r4 + 2]), part);
    part = std::fma(w.w, clamp01(acc[4 * r4 + 3]), part);
  }
  const float other = __shfl_xor(part, 32, 64);
  return (part + other) + S->b3;
}

__device__ __forceinline__ float route_pair_shared16(float u_mine, const half4* w2, const RouterShared16* S) {
  const int half = (threadIdx.x & 63) >> 5;
  const float u_other = __shfl_xor(u_mine, 32, 64);
  const float ua = half ? u_other : u_mine, ub = half ? u_mine : u_other;
  floatx16 acc_a;
  const float4* b2 = reinterpret_cast<const float4*>(S->b2[half]);
#pragma unroll
  for (int r4 = 0; r4 < 4; ++r4) {
    const float4 v = b2[r4];
    acc_a[4 * r4 + 0] = v.x;
    acc_a[4 * r4 + 1] = v.y;
    acc_a[4 * r4 + 2] = v.z;
    acc_a[4 * r4 + 3] = v.w;
  }
  floatx16 acc_b = acc_a;
  const float4* w1 = reinterpret_cast<const float4*>(S->w1[half]);
  const float4* b1 = reinterpret_cast<const float4*>(S->b1[half]);
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const float4 w = w1[kb], b = b1[kb];
    const float wv[4] = {w.x, w.y, w.z, w.w}, bv[4] = {b.x, b.y, b.z, b.w};
    half4 ha, hb;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      ha[c] = static_cast<_Float16>(clamp01(std::fma(wv[c], ua, bv[c])));
      hb[c] = static_cast<_Float16>(clamp01(std::fma(wv[c], ub, bv[c])));
    }
    acc_a = __builtin_amdgcn_mfma_f32_32x32x8f16(w2[kb], ha, acc_a, 0, 0, 0);
    acc_b = __builtin_amdgcn_mfma_f32_32x32x8f16(w2[kb], hb, acc_b, 0, 0, 0);
  }
  const float ya = router_tail16_shared(acc_a, S, half);
  const float yb = router_tail16_shared(acc_b, S, half);
  return half ? yb : ya;
}

// y for the query of this lane (lane l: query l of the 64-query group), with
// the two 32-query passes of either router precision
template <bool F16>
__device__ __forceinline__ float route_pair(float u_mine, const void* regs) {
  const int half = (threadIdx.x & 63) >> 5;
  const float u_other = __shfl_xor(u_mine, 32, 64);
  float ya, yb;
  if constexpr (F16) {
    router16_y2(half ? u_other : u_mine, half ? u_mine : u_other, *static_cast<const RouterRegs16*>(regs), &ya, &yb);
  } else {
    router_y2(half ? u_other : u_mine, half ? u_mine : u_other, *static_cast<const RouterRegs*>(regs), &ya, &yb);
  }
  return half ? yb : ya;
}

// Segment coordinate of a key or query: three quarters of the network's output
// plus a quarter of the feature itself.  The network places segments by key
// count, which squeezes a sparse region of the key domain (a long tail) into a
// few segments, although queries spread uniformly in z land mostly there; the
// feature term keeps a share of the segments spread by the feature, which is
// roughly logarithmic in z.  Both terms are non-decreasing in z and each
// rounding is monotone, so the coordinate is non-decreasing in z.  Keys (build)
// and queries (search) go through this same function.
__device__ __forceinline__ float route_coord(float y_net, float u) { return 0.75f * y_net + 0.25f * u; }

__device__ __forceinline__ int32_t segment_of(float y, int32_t nseg) {
  const float s = std::floor(std::fmin(std::fmax(y * static_cast<float>(nseg), 0.0f), static_cast<float>(nseg - 1)));
  return static_cast<int32_t>(s);
}

// Prediction of a segment's fit, as an index offset relative to seg.lo; the
// same code serves the bound computation (keys) and the search (queries).
template <typename T>
__device__ __forceinline__ int32_t seg_predict(const SegFit& sg, T z) {
  const float d = static_cast<float>(static_cast<double>(z) - sg.zc);
  float p = std::fma(sg.a, d, sg.b);
  p = std::fmin(std::fmax(p, -2.0f), static_cast<float>(sg.hi - sg.lo + 2));
  return static_cast<int32_t>(std::floor(p));
}

// How keys and queries are routed to segments.  The network's segment is a
// non-decreasing step function of the scalar f32 feature u with at most nseg
// steps, so it is fully described by where each step lies:
//   kRouteTable  (default) the FP32 network's steps, found once at build time
//                by bisection over the f32 values of u with the network itself
//                (router_steps_kernel); a key or query is then routed by a
//                search of that table (table_segment) -- the same function as
//                evaluating the FP32 network, at a fraction of the cost
//   kRouteF16    the network evaluated per query on the matrix cores, 32x32
//                layer with FP16 inputs and FP32 accumulation
//   kRouteF32    the same with FP32 inputs
// The identity router of the ablation (y = u) needs no table.
constexpr int kRouteTable = 0, kRouteF16 = 1, kRouteF32 = 2;

// The compiled router's segment of u: the largest t with steps[t] <= u, where
// steps[0] = -inf and steps is non-decreasing (a branch-free bisection; the
// probe index stays below nseg).
__device__ __forceinline__ int32_t table_segment(float u, const float* steps, int32_t nseg) {
  int32_t lo = 0, n = nseg;
  while (n > 1) {
    const int32_t half = n >> 1;
    lo = (steps[lo + half] <= u) ? lo + half : lo;
    n -= half;
  }
  return lo;
}

// A uniform grid over u speeds the table up: cell c of G = 2^k cells holds
// u in [c 2^-k, (c + 1) 2^-k) (u = 1 falls in the last cell), and
// grid[c] = s_lo | (s_hi - s_lo) << 16 with s_lo and s_hi the table segments of
// the cell's lowest and highest u.  The segment of u is then found by the same
// bisection restricted to [s_lo, s_hi] (steps[s_lo] <= u < steps[s_hi + 1]),
// usually 0 to 3 probes instead of log2(nseg): the same result as
// table_segment.  u * 2^k is exact, so the cell is exact.
__device__ __forceinline__ int32_t grid_segment(float u, const float* steps, const uint32_t* grid, int32_t log2g) {
  const int32_t g = 1 << log2g;
  const int32_t c = std::min(static_cast<int32_t>(u * static_cast<float>(g)), g - 1);
  const uint32_t e = grid[c];
  int32_t lo = static_cast<int32_t>(e & 0xffffu), n = static_cast<int32_t>(e >> 16) + 1;
  while (n > 1) {
    const int32_t half = n >> 1;
    lo = (steps[lo + half] <= u) ? lo + half : lo;
    n -= half;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// build kernels

// Kernels below serve one array, or, when given the batch's totals (and its
// LearnMeta), every learned array of a batch at once: blockIdx.y (blockIdx.x
// for the one-workgroup kernels) selects the model slot, and lm[slot] gives the
// array's keys and feature constants.
template <typename T>
__global__ void feature_kernel(const T* __restrict__ X, int64_t n, double X0, double delta, double flo, double fscale,
                               float* __restrict__ u) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    u[i] = feature(static_cast<double>(X[i]), X0, delta, flo, fscale);
}

__device__ __forceinline__ uint32_t mix32(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return static_cast<uint32_t>(x);
}

constexpr int kLd = kHid + 1;  // padded row of the per-wave LDS tiles

// Gradient sums of one wave (lane layout of the 32x32 MFMA tiles).
struct GradAcc {
  floatx16 g2;                         // dL/dW2, D[j][k] in the output layout
  float gw1, gb1, gb2, gw3, gb3, ls;  // per lane: unit n = lane % 32, samples of half lane / 32
};

// Forward and backward pass of one wave over its 64 training samples, added
// into acc.  sample(q, &u, &t) gives sample q's feature and target and whether
// it exists.  The parameters are in LDS (sp); w2f / w2b hold the lane's row of
// W2 and of its transpose; TA, TB, sv are the wave's own tiles.  Every wave of
// the workgroup must call it together (it holds workgroup barriers).
//   forward   h1 = clamp(W1 u + b1), a2 = W2 h1 + b2 (MFMA), y = W3 clamp(a2) + b3
//   backward  dy = 2 (y - t) / batch, da2 = dy W3 [0 < h2 < 1], dW2 += da2 h1^T (MFMA
//             over the 64 samples), da1 = W2^T da2 [0 < h1 < 1] (MFMA), dW1, db1, dW3,
//             db3 as sums over the samples
template <class Sample>
__device__ __forceinline__ void wave_grad(const float* sp, const float (&w2f)[16], const float (&w2b)[16],
                                          float (*TA)[kLd], float (*TB)[kLd], float (*sv)[3], float inv_b,
                                          Sample sample, GradAcc& acc) {
  const int lane = threadIdx.x & 63, n = lane & 31, h = lane >> 5;
  float st_h2[2][16], st_da1[2][16];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int q = p * 32 + n;
    float u = 0.0f, t = 0.0f;
    const bool valid = sample(q, &u, &t);
    float h1[16];
    floatx16 acc2;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int un = out_row(r, h);
      h1[r] = clamp01(std::fma(sp[oW1 + un], u, sp[oB1 + un]));
      acc2[r] = sp[oB2 + un];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(w2f[r], h1[r], acc2, 0, 0, 0);
    float part = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) part = std::fma(sp[oW3 + out_row(r, h)], clamp01(acc2[r]), part);
    const float y = (part + __shfl_xor(part, 32, 64)) + sp[oB3];  // the same sum in both lanes
    const float dy = valid ? 2.0f * (y - t) * inv_b : 0.0f;
    const float l = valid ? (y - t) * (y - t) * inv_b : 0.0f;
    float da2[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int un = out_row(r, h);
      const float h2 = clamp01(acc2[r]);
      st_h2[p][r] = h2;
      // clamp(a) lies strictly inside (0, 1) exactly when a does, so the unit outputs give the masks
      da2[r] = (h2 > 0.0f && h2 < 1.0f) ? dy * sp[oW3 + un] : 0.0f;
      TA[q][un] = da2[r];
      TB[q][un] = h1[r];
    }
    floatx16 d1;
#pragma unroll
    for (int r = 0; r < 16; ++r) d1[r] = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) d1 = __builtin_amdgcn_mfma_f32_32x32x2f32(w2b[r], da2[r], d1, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) st_da1[p][r] = (h1[r] > 0.0f && h1[r] < 1.0f) ? d1[r] : 0.0f;
    if (h == 0) {
      sv[q][0] = dy;
      sv[q][1] = u;
      sv[q][2] = l;
    }
  }
  __syncthreads();
  // dW2[j][k] += sum_s da2[s][j] h1[s][k]: K = the wave's 64 samples, two per instruction
  // (lane half h supplies sample 2i + h); db2 from the same reads
#pragma unroll 8
  for (int i = 0; i < 32; ++i) {
    const float a = TA[2 * i + h][n];
    acc.gb2 += a;
    acc.g2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, TB[2 * i + h][n], acc.g2, 0, 0, 0);
  }
  __syncthreads();
  // phase 2: the tiles now hold h2 and da1
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      TA[p * 32 + n][out_row(r, h)] = st_h2[p][r];
      TB[p * 32 + n][out_row(r, h)] = st_da1[p][r];
    }
  }
  __syncthreads();
  // lane (n, h): unit n over the samples s = 2i + h
  for (int i = 0; i < 32; ++i) {
    const int s2 = 2 * i + h;
    const float da1 = TB[s2][n], dy = sv[s2][0];
    acc.gw1 = std::fma(da1, sv[s2][1], acc.gw1);
    acc.gb1 += da1;
    acc.gw3 = std::fma(dy, TA[s2][n], acc.gw3);
    acc.gb3 += dy;
    acc.ls += sv[s2][2];
  }
  __syncthreads();
}

// The waves' gradients added in wave order into red[0 .. kParams] (kParams = the
// loss); red is the workgroup's tile A, free once wave_grad returned.  The two
// lane halves of each wave are combined first.  Ends with a barrier.
template <int kWaves>
__device__ __forceinline__ void reduce_waves(GradAcc& acc, float* red) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, n = lane & 31, h = lane >> 5;
  acc.gw1 += __shfl_xor(acc.gw1, 32, 64);
  acc.gb1 += __shfl_xor(acc.gb1, 32, 64);
  acc.gw3 += __shfl_xor(acc.gw3, 32, 64);
  acc.gb2 += __shfl_xor(acc.gb2, 32, 64);
  acc.gb3 += __shfl_xor(acc.gb3, 32, 64);
  acc.ls += __shfl_xor(acc.ls, 32, 64);
  float* mine = red + w * (kParams + 1);
#pragma unroll
  for (int r = 0; r < 16; ++r) mine[oW2 + out_row(r, h) * kHid + n] = acc.g2[r];
  if (h == 0) {
    mine[oW1 + n] = acc.gw1;
    mine[oB1 + n] = acc.gb1;
    mine[oB2 + n] = acc.gb2;
    mine[oW3 + n] = acc.gw3;
    if (n == 0) {
      mine[oB3] = acc.gb3;
      mine[kParams] = acc.ls;
    }
  }
  __syncthreads();
  for (int k = tid; k <= kParams; k += kWaves * 64) {
    float v = red[k];
#pragma unroll
    for (int ww = 1; ww < kWaves; ++ww) v += red[ww * (kParams + 1) + k];
    red[k] = v;  // only thread k reads and writes column k
  }
  __syncthreads();
}

// the lane's rows of W2 (forward) and of its transpose (backward) from LDS
__device__ __forceinline__ void load_w2_rows(const float* sp, float (&w2f)[16], float (&w2b)[16]) {
  const int lane = threadIdx.x & 63, n = lane & 31, h = lane >> 5;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int u = out_row(r, h);
    w2f[r] = sp[oW2 + n * kHid + u];  // A of the forward: W2[n][u]
    w2b[r] = sp[oW2 + u * kHid + n];  // A of the backward: W2[u][n]
  }
}

// the training sample j of a step: a key drawn by a counter-based hash of
// (seed, step, j), its feature and its target i / (n - 1)
__device__ __forceinline__ int64_t draw_index(int64_t n_keys, uint64_t seed, int64_t step, int64_t j) {
  const uint64_t key = seed * 0x9E3779B97F4A7C15ull + static_cast<uint64_t>(step) * 0x100000001B3ull +
                       static_cast<uint64_t>(j);
  return static_cast<int64_t>(mix32(key) % static_cast<uint32_t>(n_keys));
}

__device__ __forceinline__ float key_target(int64_t idx, int64_t n_keys) {
  return static_cast<float>(static_cast<double>(idx) / static_cast<double>(n_keys - 1));
}

__device__ __forceinline__ void draw_sample(const float* feat, int64_t n_keys, uint64_t seed, int64_t step, int64_t j,
                                            float* u, float* t) {
  const int64_t idx = draw_index(n_keys, seed, step, j);
  *u = feat[idx];
  *t = key_target(idx, n_keys);
}

// One training step's gradient over a batch, split over workgroups of
// kTrainBlock samples: each writes its sum (and its loss) to partial[part];
// adam_kernel adds the parts in order.  Samples are given (u_in, t_in) or drawn
// (draw_sample).
__global__ void __launch_bounds__(kTrainBlock) train_step_kernel(
    const float* __restrict__ params, const float* __restrict__ feat, int64_t n_keys, uint64_t seed, int64_t step,
    int32_t batch, const float* __restrict__ u_in, const float* __restrict__ t_in, float* __restrict__ partial,
    float* __restrict__ loss_partial) {
  constexpr int kWaves = kTrainBlock / 64;
  __shared__ float sp[kParams];
  __shared__ float tileA[kWaves][64][kLd];  // da2, then h2
  __shared__ float tileB[kWaves][64][kLd];  // h1, then da1
  __shared__ float svec[kWaves][64][3];     // dy, u, loss per sample
  const int tid = threadIdx.x, w = tid >> 6;
  for (int k = tid; k < kParams; k += kTrainBlock) sp[k] = params[k];
  __syncthreads();
  float w2f[16], w2b[16];
  load_w2_rows(sp, w2f, w2b);
  GradAcc acc{};
  auto sample = [&](int q, float* u, float* t) {
    const int64_t j = (int64_t)blockIdx.x * kTrainBlock + w * 64 + q;
    if (j >= batch) return false;
    if (u_in) {
      *u = u_in[j];
      *t = t_in[j];
    } else {
      draw_sample(feat, n_keys, seed, step, j, u, t);
    }
    return true;
  };
  wave_grad(sp, w2f, w2b, tileA[w], tileB[w], svec[w], 1.0f / static_cast<float>(batch), sample, acc);
  float* red = &tileA[0][0][0];  // kWaves x (kParams + 1) floats
  static_assert(kWaves * (kParams + 1) <= kWaves * 64 * kLd, "reduction fits the tile");
  reduce_waves<kWaves>(acc, red);
  float* out = partial + (int64_t)blockIdx.x * kParams;
  for (int k = tid; k <= kParams; k += kTrainBlock) {
    if (k < kParams)
      out[k] = red[k];
    else
      loss_partial[blockIdx.x] = red[k];
  }
}

// Adam step of one parameter with its gradient g (step t >= 1), then the
// projection of the weights onto w >= 0 that keeps the router monotone
__device__ __forceinline__ float adam_update(int k, float p, float g, float* m, float* v, float lr, int64_t t) {
  constexpr float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  const float mk = beta1 * m[k] + (1.0f - beta1) * g;
  const float vk = beta2 * v[k] + (1.0f - beta2) * g * g;
  m[k] = mk;
  v[k] = vk;
  const float bc1 = 1.0f - std::pow(beta1, static_cast<float>(t));
  const float bc2 = 1.0f - std::pow(beta2, static_cast<float>(t));
  p = p - lr * (mk / bc1) / (std::sqrt(vk / bc2) + eps);
  const bool is_weight = (k < oB1) || (k >= oW2 && k < oB2) || (k >= oW3 && k < oB3);
  return is_weight ? std::fmax(p, 0.0f) : p;
}

// step size of step st of steps: 2e-3 cosine-decayed to 5 % of it
__host__ __device__ __forceinline__ float train_rate(float lr, int64_t st, int64_t steps) {
  const float frac = static_cast<float>(st) / static_cast<float>(steps);
  return lr * (0.05f + 0.95f * 0.5f * (1.0f + std::cos(3.14159265f * frac)));
}

// The whole training of the batched form in one launch: workgroup k trains the
// model of learned slot k for every step (kBatchLearnSamples samples a step, in
// kBatchTrainPasses passes of its kBatchTrainBlock lanes), sums the gradient of
// its waves and passes in a fixed order, and applies the Adam step itself; the
// parameters stay in LDS between steps.  No workgroup waits for another.  The
// feature of each drawn key is computed from the key (the same function as
// feature_kernel's).
constexpr int kBatchTrainBlock = 512;
constexpr int kBatchTrainPasses = kBatchLearnSamples / kBatchTrainBlock;

template <typename T>
__global__ void __launch_bounds__(kBatchTrainBlock) batched_train_kernel(float* __restrict__ params,
                                                                         float* __restrict__ adam_m,
                                                                         float* __restrict__ adam_v,
                                                                         const T* __restrict__ X,
                                                                         const LearnMeta* __restrict__ lm,
                                                                         const PlanTotals* __restrict__ tot,
                                                                         uint64_t seed0, int32_t steps, float lr) {
  const int slot = blockIdx.x;
  if (slot >= tot->n_learned) return;
  constexpr int kWaves = kBatchTrainBlock / 64;
  __shared__ float sp[kParams];
  __shared__ float tileA[kWaves][64][kLd];
  __shared__ float tileB[kWaves][64][kLd];
  __shared__ float svec[kWaves][64][3];
  static_assert(kWaves * (kParams + 1) <= kWaves * 64 * kLd, "reduction fits the tile");
  const LearnMeta L = lm[slot];
  const T* Xa = X + L.x_off;
  const int64_t n_keys = int64_t(L.N) + 1;
  const uint64_t seed = seed0 + 0x632BE59BD9B4E019ull * static_cast<uint64_t>(slot + 1);
  float* p = params + (int64_t)slot * kParams;
  float* m = adam_m + (int64_t)slot * kParams;
  float* v = adam_v + (int64_t)slot * kParams;
  const int tid = threadIdx.x, w = tid >> 6;
  for (int k = tid; k < kParams; k += kBatchTrainBlock) sp[k] = p[k];
  __syncthreads();
  const float inv_b = 1.0f / static_cast<float>(kBatchLearnSamples);
  // The draws do not depend on the parameters: the keys of the next pass
  // (lane sample q = 32 p + lane % 32, p = 0, 1) are loaded while this one is
  // worked on, so the key reads do not wait between the passes' barriers.
  const int n32 = tid & 31;
  int64_t idx_next[2];
  T key_next[2];
  auto fetch = [&](int32_t st, int pass) {
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
      idx_next[pp] = draw_index(n_keys, seed, st, int64_t(pass) * kBatchTrainBlock + w * 64 + 32 * pp + n32);
      key_next[pp] = Xa[idx_next[pp]];
    }
  };
  if (steps > 0) fetch(0, 0);
  for (int32_t st = 0; st < steps; ++st) {
    float w2f[16], w2b[16];
    load_w2_rows(sp, w2f, w2b);
    GradAcc acc{};
    for (int pass = 0; pass < kBatchTrainPasses; ++pass) {
      const int64_t idx[2] = {idx_next[0], idx_next[1]};
      const T key[2] = {key_next[0], key_next[1]};
      if (pass + 1 < kBatchTrainPasses) fetch(st, pass + 1);
      else if (st + 1 < steps) fetch(st + 1, 0);
      auto sample = [&](int q, float* u, float* t) {
        const int pp = q >= 32 ? 1 : 0;
        *u = feature(static_cast<double>(key[pp]), L.X0, L.delta, L.flo, L.fscale);
        *t = key_target(idx[pp], n_keys);
        return true;
      };
      wave_grad(sp, w2f, w2b, tileA[w], tileB[w], svec[w], inv_b, sample, acc);
    }
    float* red = &tileA[0][0][0];
    reduce_waves<kWaves>(acc, red);
    const float lr_t = train_rate(lr, st, steps);
    for (int k = tid; k < kParams; k += kBatchTrainBlock) sp[k] = adam_update(k, sp[k], red[k], m, v, lr_t, st + 1);
    __syncthreads();
  }
  for (int k = tid; k < kParams; k += kBatchTrainBlock) p[k] = sp[k];
}

// Sums the per-workgroup gradients in a fixed order (deterministic), then,
// unless grad_out is given, applies one Adam step and projects the weights
// onto w >= 0.
__global__ void __launch_bounds__(1024) adam_kernel(float* __restrict__ params, float* __restrict__ m,
                                                    float* __restrict__ v, const float* __restrict__ partial,
                                                    int32_t n_parts, float lr, int64_t t, float* __restrict__ grad_out) {
  for (int k = threadIdx.x; k < kParams; k += blockDim.x) {
    // the parts in order, eight loads in flight at a time
    float g = 0.0f;
    int b = 0;
    for (; b + 8 <= n_parts; b += 8) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = partial[(int64_t)(b + u) * kParams + k];
#pragma unroll
      for (int u = 0; u < 8; ++u) g += x[u];
    }
    for (; b < n_parts; ++b) g += partial[(int64_t)b * kParams + k];
    if (grad_out) {
      grad_out[k] = g;
      continue;
    }
    params[k] = adam_update(k, params[k], g, m, v, lr, t);
  }
}

__global__ void sum_kernel(const float* __restrict__ parts, int32_t n, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s += parts[i];
    *out = s;
  }
}

// segment of every key through the search-time router (MFMA), 64 keys per wave
template <bool F16>
__global__ void __launch_bounds__(256) route_keys_kernel(const float* __restrict__ params,
                                                         const float* __restrict__ feat, int64_t n,
                                                         int32_t nseg, int32_t identity, int32_t* __restrict__ route,
                                                         float* __restrict__ y_out) {
  typename std::conditional<F16, RouterRegs16, RouterRegs>::type R;
  if constexpr (F16)
    load_router16(params, R);
  else
    load_router(params, R);
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; wave * 64 < n; wave += waves) {
    const int64_t i = wave * 64 + lane;
    const float u_mine = i < n ? feat[i] : 1.0f;
    const float y = identity ? u_mine : route_pair<F16>(u_mine, &R);
    if (i < n) {
      route[i] = segment_of(identity ? y : route_coord(y, u_mine), nseg);
      if (y_out) y_out[i] = y;
    }
  }
}

// The FP32 network's segment of u, segment_of(route_coord(y(u), u)); every
// lane of the wave must call it (the router works on 64 inputs at once).
__device__ __forceinline__ int32_t net_segment(float u, const RouterRegs& R, int32_t nseg) {
  return segment_of(route_coord(route_pair<false>(u, &R), u), nseg);
}

// Compiling the router, step 1: the network's segment at the 2^kp + 1 points
// u_c = c 2^-kp, c = 0 .. 2^kp (exact floats), into probe[c].  With tot,
// blockIdx.y is the model slot of the batched form.
__global__ void __launch_bounds__(256) router_probe_kernel(const float* __restrict__ params, int32_t nseg,
                                                           int32_t kp, int32_t* __restrict__ probe,
                                                           const PlanTotals* __restrict__ tot) {
  if (tot) {
    if (int(blockIdx.y) >= tot->n_learned) return;
    params += (int64_t)blockIdx.y * kParams;
    probe += (int64_t)blockIdx.y * (nseg + 1);
  }
  RouterRegs R;
  load_router(params, R);
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t np = (1 << kp) + 1;
  const float u = std::ldexp(static_cast<float>(std::min(c, np - 1)), -kp);
  const int32_t sg = net_segment(u, R, nseg);
  if (c < np) probe[c] = sg;
}

// Step 2: lane t (1 <= t < nseg) finds the smallest f32 u in [0, 1] whose
// segment is at least t (2.0f when no u reaches t; steps[0] = -inf).  The
// probes bracket it: with c the first probe point whose segment is >= t, the
// network is non-decreasing, so the answer lies in (u_(c-1), u_c], and a
// bisection over the bit patterns of that interval (ordered like the values)
// finds it -- the same value as a bisection over all of [0, 1], in 12 to 23
// rounds instead of 31.  The wave evaluates the network while any of its lanes
// is still bisecting.  The steps are then made non-decreasing
// (router_table_kernel), so the table is a non-decreasing step function even
// if some rounding were not monotone.
__global__ void __launch_bounds__(256) router_steps_kernel(const float* __restrict__ params, int32_t nseg,
                                                           int32_t kp, const int32_t* __restrict__ probe,
                                                           float* __restrict__ steps,
                                                           const PlanTotals* __restrict__ tot) {
  if (tot) {
    if (int(blockIdx.y) >= tot->n_learned) return;
    params += (int64_t)blockIdx.y * kParams;
    probe += (int64_t)blockIdx.y * (nseg + 1);
    steps += (int64_t)blockIdx.y * nseg;
  }
  RouterRegs R;
  load_router(params, R);
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t np = (1 << kp) + 1;
  // c = #{probes < t}: the probe points are in order of u
  int32_t c = 0, n = np;
  while (n > 0) {
    const int32_t half = n >> 1;
    const bool below = probe[c + half] < t;
    c = below ? c + half + 1 : c;
    n = below ? n - half - 1 : half;
  }
  uint32_t lo = 1, hi = 0;  // an empty interval: nothing to bisect
  float found = 2.0f;       // no u reaches t
  if (c == 0) {
    found = 0.0f;
  } else if (c < np) {
    lo = __float_as_uint(std::ldexp(static_cast<float>(c - 1), -kp)) + 1;
    hi = __float_as_uint(std::ldexp(static_cast<float>(c), -kp));  // its segment is >= t
  }
  while (__ballot(lo < hi)) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    const int32_t sg = net_segment(__uint_as_float(mid), R, nseg);
    if (lo < hi) {
      if (sg >= t) hi = mid;
      else lo = mid + 1;
    }
  }
  if (c > 0 && c < np) found = __uint_as_float(lo);
  if (t == 0) steps[0] = -std::numeric_limits<float>::infinity();
  else if (t < nseg) steps[t] = found;
}

// Step 3, one workgroup per model: the steps made non-decreasing (a prefix
// maximum: each thread's run of steps, then a scan of the run maxima across the
// workgroup), then the grid cells of grid_segment from them.
constexpr int kTableBlock = 1024;

__global__ void __launch_bounds__(kTableBlock) router_table_kernel(float* __restrict__ steps, int32_t nseg,
                                                                   int32_t log2g, uint32_t* __restrict__ grid,
                                                                   const PlanTotals* __restrict__ tot) {
  if (tot) {
    if (int(blockIdx.x) >= tot->n_learned) return;
    steps += (int64_t)blockIdx.x * nseg;
    grid += (int64_t)blockIdx.x << log2g;
  }
  __shared__ float st[kBatchMaxSegments];
  __shared__ float wave_max[kTableBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int per = (nseg + kTableBlock - 1) / kTableBlock;
  const int a = std::min(nseg, tid * per), b = std::min(nseg, a + per);
  float run = -std::numeric_limits<float>::infinity();
  for (int k = a; k < b; ++k) {
    run = std::fmax(run, steps[k]);
    st[k] = run;
  }
  // inclusive scan (max) of the run maxima over the wave, then over the waves
  float x = run;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float y = __shfl_up(x, o, 64);
    if (lane >= o) x = std::fmax(x, y);
  }
  if (lane == 63) wave_max[w] = x;
  __syncthreads();
  float before = -std::numeric_limits<float>::infinity();  // max of every earlier thread's run
  for (int ww = 0; ww < w; ++ww) before = std::fmax(before, wave_max[ww]);
  const float up = __shfl_up(x, 1, 64);
  if (lane > 0) before = std::fmax(before, up);
  for (int k = a; k < b; ++k) {
    st[k] = std::fmax(st[k], before);
    steps[k] = st[k];
  }
  __syncthreads();
  const int32_t g = 1 << log2g;
  const float scale = std::ldexp(1.0f, -log2g);
  for (int32_t cc = tid; cc < g; cc += kTableBlock) {
    const float u0 = static_cast<float>(cc) * scale;
    const float u1 = (cc == g - 1) ? 1.0f : std::nextafter(static_cast<float>(cc + 1) * scale, 0.0f);
    const int32_t s0 = table_segment(u0, st, nseg), s1 = table_segment(u1, st, nseg);
    grid[cc] = static_cast<uint32_t>(s0) | (static_cast<uint32_t>(s1 - s0) << 16);
  }
}

// segment of every key through the compiled router
__global__ void route_keys_table_kernel(const float* __restrict__ steps, const float* __restrict__ feat, int64_t n,
                                        int32_t nseg, int32_t* __restrict__ route) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    route[i] = table_segment(feat[i], steps, nseg);
}

// the queries' routing of the compiled router (grid_segment), for checking
__global__ void route_query_table_kernel(const float* __restrict__ steps, const uint32_t* __restrict__ grid,
                                         int32_t log2g, const float* __restrict__ feat, int64_t n,
                                         int32_t* __restrict__ route) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    route[i] = grid_segment(feat[i], steps, grid, log2g);
}

// first[s] = #{i : route_i < s} for s in [0, nseg]
__global__ void seg_first_kernel(const int32_t* __restrict__ route, int64_t n, int32_t nseg,
                                 int32_t* __restrict__ first) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t prev = (i == 0) ? -1 : route[i - 1];
    const int32_t cur = (i == n) ? nseg : route[i];
    for (int32_t s = prev + 1; s <= cur; ++s) first[s] = static_cast<int32_t>(i);
  }
}

// Copy n 32-bit words from global memory to LDS with 4-byte moves, four
// loads in flight per lane.  The router's step table and grid sit after nseg
// entries, so their addresses are 4-byte but, for nseg not a multiple of 4,
// not 16-byte aligned (stage_bytes needs 16).
__device__ __forceinline__ void stage_words(void* dst, const void* src, int64_t n) {
  const uint32_t* s = static_cast<const uint32_t*>(src);
  uint32_t* d = static_cast<uint32_t*>(dst);
  const int64_t B = blockDim.x;
  int64_t k = threadIdx.x;
  for (; k + 3 * B < n; k += 4 * B) {
    const uint32_t w0 = s[k], w1 = s[k + B], w2 = s[k + 2 * B], w3 = s[k + 3 * B];
    d[k] = w0;
    d[k + B] = w1;
    d[k + 2 * B] = w2;
    d[k + 3 * B] = w3;
  }
  for (; k < n; k += B) d[k] = s[k];
}

// The batched form of feature_kernel + route_keys_kernel + seg_first_kernel in
// one pass, with no per-key feature or route array: each wave takes a contiguous range of at least 8
// of the array's 64-key groups, and each key i routed to segment r with its
// predecessor in segment p writes first[s] = i for s in (p, r]; the last key
// also writes first[s] = n for s above its segment.  A lane's predecessor is
// the lane before it or, for lane 0, the last key of the previous group (the
// wave routes the key before its range first).  The keys of the next
// kRouteGroups groups are loaded before the current ones are routed, so each
// lane keeps up to 2 kRouteGroups loads in flight; each key's feature is
// computed as feature_kernel computes it.  With the compiled router the keys'
// order is used: a key's table segment (the last step <= its feature) is
// non-decreasing along the sorted keys, so a group's keys lie between the
// segment carried from the key before it and that of its last key, found by
// galloping up the steps from the carried one (one LDS read when the group
// crosses no step); only a group that crosses steps searches them per lane.  The compiled router's step
// table and grid are staged in LDS first (a few dozen KiB at most), and each
// model's keys are shared by kRouteBlocks workgroups of 1024 lanes.  Routing
// is the same function as route_keys_table_kernel's.
constexpr int kRouteBlock = 1024;
constexpr int kRouteBlocks = 8;
constexpr int kRouteGroups = 4;

// dynamic LDS of route_first_kernel<false>: the step table, then the grid
int64_t route_first_lds(int32_t nseg, int32_t log2g) { return int64_t(nseg) * 4 + (int64_t(4) << log2g); }

template <bool IDENT, typename T>
__global__ void __launch_bounds__(kRouteBlock) route_first_kernel(const float* __restrict__ steps_all,
                                                                  const uint32_t* __restrict__ grid_all, int32_t log2g,
                                                                  const T* __restrict__ X, int32_t nseg,
                                                                  int32_t* __restrict__ first,
                                                                  const LearnMeta* __restrict__ lm,
                                                                  const PlanTotals* __restrict__ tot) {
  extern __shared__ __attribute__((aligned(16))) unsigned char rlds[];
  const int slot = blockIdx.y;
  if (slot >= tot->n_learned) return;  // uniform across the workgroup
  const float* steps = reinterpret_cast<const float*>(rlds);
  const uint32_t* grid = reinterpret_cast<const uint32_t*>(rlds + int64_t(nseg) * 4);
  if (!IDENT) {
    stage_words(rlds, steps_all + (int64_t)slot * nseg, nseg);
    stage_words(rlds + int64_t(nseg) * 4, grid_all + ((int64_t)slot << log2g), int64_t(1) << log2g);
    __syncthreads();
  }
  const LearnMeta L = lm[slot];
  X += L.x_off;
  first += (int64_t)slot * (nseg + 1);
  const int64_t n = int64_t(L.N) + 1;  // keys
  const int64_t ngroups = (n + 63) / 64;
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x / 64);
  const int64_t per = std::max<int64_t>((ngroups + waves - 1) / waves, 8);
  const int64_t g0 = (int64_t(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x / 64)) * per;
  const int64_t g1 = std::min(ngroups, g0 + per);
  if (g0 >= g1) return;  // uniform across the wave; no barrier below
  const int lane = threadIdx.x & 63;
  auto segment = [&](float u) { return IDENT ? segment_of(u, nseg) : grid_segment(u, steps, grid, log2g); };
  auto feat = [&](T x) { return feature(static_cast<double>(x), L.X0, L.delta, L.flo, L.fscale); };
  // the last step <= u among steps [lo, hi] (steps[lo] <= u)
  auto last_step_le = [&](float u, int32_t lo, int32_t hi) {
    int32_t cnt = hi - lo + 1;
    while (cnt > 1) {
      const int32_t half = cnt >> 1;
      lo = (steps[lo + half] <= u) ? lo + half : lo;
      cnt -= half;
    }
    return lo;
  };
  auto key_at = [&](int64_t i) { return X[std::min(i, n - 1)]; };  // lanes past the last key read it again
  // the key before the range
  int32_t carry = (g0 > 0) ? segment(feat(X[g0 * 64 - 1])) : -1;
  T xn[kRouteGroups];
#pragma unroll
  for (int k = 0; k < kRouteGroups; ++k) xn[k] = key_at((g0 + k) * 64 + lane);
  for (int64_t grp = g0; grp < g1; grp += kRouteGroups) {
    T x[kRouteGroups];
#pragma unroll
    for (int k = 0; k < kRouteGroups; ++k) x[k] = xn[k];
    if (grp + kRouteGroups < g1) {
#pragma unroll
      for (int k = 0; k < kRouteGroups; ++k) xn[k] = key_at((grp + kRouteGroups + k) * 64 + lane);
    }
#pragma unroll
    for (int k = 0; k < kRouteGroups; ++k) {
      if (grp + k >= g1) break;  // uniform across the wave
      const int64_t i = (grp + k) * 64 + lane;
      const float u = feat(x[k]);
      int32_t r;
      if (IDENT) {
        r = segment_of(u, nseg);
      } else {
        // lanes past the array's last key hold that key, so lane 63 holds the group's largest
        const float u_last = __shfl(u, 63, 64);
        const int32_t r_lo = std::max(carry, 0);  // steps[0] = -inf
        int32_t hi = r_lo, step = 1;
        while (hi + 1 < nseg && steps[hi + 1] <= u_last) {  // gallop: the same steps in every lane
          const int32_t probe = std::min(hi + step, nseg - 1);
          if (steps[probe] <= u_last) {
            hi = probe;
            step *= 2;
          } else {
            hi = last_step_le(u_last, hi, probe - 1);
            break;
          }
        }
        r = (hi == r_lo) ? r_lo : last_step_le(u, r_lo, hi);
      }
      int32_t p = __shfl_up(r, 1, 64);
      if (lane == 0) p = carry;
      if (i < n) {
        for (int32_t sg = p + 1; sg <= r; ++sg) first[sg] = static_cast<int32_t>(i);
        if (i == n - 1)
          for (int32_t sg = r + 1; sg <= nseg; ++sg) first[sg] = static_cast<int32_t>(n);
      }
      carry = __shfl(r, 63, 64);  // used only when the group is whole
    }
  }
}

// least-squares line of index against z for the keys of one segment (f64
// sums over centred z), then the key errors over [lo, hi + 1].
//
// seg_fit_kernel: one wave per kFitSegs consecutive segments and one wave per
// workgroup, so that a wave retires as soon as its segments are done.  The
// wave reads the kFitSegs + 1 boundaries in one load; a short segment's keys
// (fit range up to 128) are loaded once for both passes, longer ones loop with
// 8 loads per lane in flight.  The kernel is bound by instruction issue (half
// the segments are empty or hold one key), so a segment's butterflies span
// only the lanes that hold its keys, and one key needs no sums.  (Four
// segments per wave, their loads issued together, took 1.06x as long.)  In the
// batched form, a segment whose fit range exceeds kFitLongKeys keys is queued for
// seg_fit_long_kernel instead, which gives it a workgroup of kLongBlock lanes:
// segment sizes are very uneven (clusters route tens of thousands of keys to
// one segment), and a single wave walking such a segment set the whole
// launch's time (for 2048 segments of each of the 256 mixture arrays: 374 us
// with no queue, 249 + 70 us for the two kernels at 8192 keys, 221 + 165 at
// 2048, 277 + 52 at 16384).  Reductions run in a fixed
// order (with L lanes, lane t holds a + t, a + t + L, ...; a butterfly over
// the wave, then the waves in order), so the fits do not depend on timing.
constexpr int kFitLanes = 64;
constexpr int kFitRounds = 2;
constexpr int kFitUnroll = 8;
constexpr int kFitSegs = 4;                                     // segments per wave
constexpr int kFitGroupLanes = kFitLanes / kFitSegs;           // lanes per short segment
constexpr int kFitGroupRounds = 4;                             // keys per lane of a short segment
constexpr int kFitGroupKeys = kFitGroupLanes * kFitGroupRounds;  // a short segment's fit range, at most
constexpr int kLongBlock = 1024;

// the keys [a, b) of a segment and the range [lo, last] of its error pass
struct FitSpan {
  int64_t a, b, lo, hi, last;
  bool fast;  // last - lo < kFitLanes * kFitRounds: values loaded once
};

__device__ __forceinline__ FitSpan fit_span(int64_t a, int64_t b, int64_t N) {
  FitSpan sp;
  sp.a = a;
  sp.b = b;
  sp.lo = std::max<int64_t>(0, std::min<int64_t>(a - 1, N - 1));
  sp.hi = std::max<int64_t>(sp.lo, std::min<int64_t>(b - 1, N - 1));
  sp.last = std::min(sp.hi + 1, N);
  sp.fast = sp.last - sp.lo < kFitLanes * kFitRounds;
  return sp;
}

struct FitSums {
  double sz, szz, siz;
};

template <typename T>
__device__ __forceinline__ void add_key(FitSums& s, int64_t i, T x, int64_t lo, double zc) {
  const double dz = static_cast<double>(x) - zc;
  s.sz += dz;
  s.szz += dz * dz;
  s.siz += static_cast<double>(i - lo) * dz;
}

// the sums over keys [from, to) taken by lane t of L lanes, in rounds of
// kFitUnroll loads issued together (the last round's loads predicated, so a
// remainder costs one round trip, not one per key)
template <typename T, int L>
__device__ __forceinline__ void add_keys(const T* __restrict__ X, int64_t from, int64_t to, int64_t lo, double zc,
                                         int t, FitSums& s) {
  for (int64_t i = from + t; i < to; i += kFitUnroll * L) {
    T x[kFitUnroll];
#pragma unroll
    for (int u = 0; u < kFitUnroll; ++u) x[u] = (i + u * L < to) ? X[i + u * L] : T(0);
#pragma unroll
    for (int u = 0; u < kFitUnroll; ++u)
      if (i + u * L < to) add_key(s, i + u * L, x[u], lo, zc);
  }
}

// The butterfly width for values held by lanes [0, cnt) (lanes above hold the
// reduction's identity): the levels o = top, top / 2, ..., 1 cover lanes
// [0, 2 top), and the levels above would only combine identities (adding an
// exact zero, or taking the min / max with the empty bound).
__device__ __forceinline__ int butterfly_top(int64_t cnt) {
  int top = 0;  // covers one lane
  while (top < kFitLanes / 2 && (top ? 2 * int64_t(top) : 1) < cnt) top = top ? 2 * top : 1;
  return top;
}

__device__ __forceinline__ double lane0(double x) {
  uint64_t b;
  __builtin_memcpy(&b, &x, 8);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b >> 32));
  b = (uint64_t(hi) << 32) | lo;
  __builtin_memcpy(&x, &b, 8);
  return x;
}

// the sums over lanes [0, 2 top), then lane 0's in every lane (the whole wave
// must be active)
__device__ __forceinline__ void wave_sum(FitSums& s, int top = kFitLanes / 2) {
  for (int o = top; o > 0; o >>= 1) {
    s.sz += __shfl_xor(s.sz, o, kFitLanes);
    s.szz += __shfl_xor(s.szz, o, kFitLanes);
    s.siz += __shfl_xor(s.siz, o, kFitLanes);
  }
  s.sz = lane0(s.sz);
  s.szz = lane0(s.szz);
  s.siz = lane0(s.siz);
}

// the line of the sums (every lane holds the same sums and computes the same
// fit); n and the sum of (i - lo) over the keys [a, b) have closed forms
__device__ __forceinline__ SegFit line_fit(const FitSpan& sp, double zc, const FitSums& s) {
  const double n = static_cast<double>(sp.b - sp.a);
  const double si_ = n * (static_cast<double>(sp.a + sp.b - 1) * 0.5 - static_cast<double>(sp.lo));
  double slope = 0, icpt = 0;
  if (n >= 2) {
    const double var = s.szz - s.sz * s.sz / n;
    const double cov = s.siz - si_ * s.sz / n;
    slope = (var > 0) ? cov / var : 0.0;
    if (!(slope > 0)) slope = 0;  // monotone prediction
    icpt = (si_ - slope * s.sz) / n;
  } else if (n == 1) {
    icpt = si_;
  }
  SegFit f{};
  f.zc = zc;
  f.a = static_cast<float>(slope);
  f.b = static_cast<float>(icpt);
  f.lo = static_cast<int32_t>(sp.lo);
  f.hi = static_cast<int32_t>(sp.hi);
  return f;
}

template <typename T>
__device__ __forceinline__ void err_key(const SegFit& f, int64_t i, T x, int64_t lo, int32_t& dmin, int32_t& dmax) {
  const int32_t d = static_cast<int32_t>(i - lo) - seg_predict<T>(f, x);
  dmin = std::min(dmin, d);
  dmax = std::max(dmax, d);
}

// the error bounds over keys [lo, last] taken by lane t of L lanes, in rounds
// as add_keys
template <typename T, int L>
__device__ __forceinline__ void err_keys(const T* __restrict__ X, int64_t lo, int64_t last, const SegFit& f, int t,
                                         int32_t& dmin, int32_t& dmax) {
  for (int64_t i = lo + t; i <= last; i += kFitUnroll * L) {
    T x[kFitUnroll];
#pragma unroll
    for (int u = 0; u < kFitUnroll; ++u) x[u] = (i + u * L <= last) ? X[i + u * L] : T(0);
#pragma unroll
    for (int u = 0; u < kFitUnroll; ++u)
      if (i + u * L <= last) err_key(f, i + u * L, x[u], lo, dmin, dmax);
  }
}

__device__ __forceinline__ void wave_minmax(int32_t& dmin, int32_t& dmax, int top = kFitLanes / 2) {
  for (int o = top; o > 0; o >>= 1) {
    dmin = std::min(dmin, __shfl_xor(dmin, o, kFitLanes));
    dmax = std::max(dmax, __shfl_xor(dmax, o, kFitLanes));
  }
  dmin = __builtin_amdgcn_readfirstlane(dmin);
  dmax = __builtin_amdgcn_readfirstlane(dmax);
}

// the fit and error bounds of one segment by one wave, from its span, its
// values v[r] = X[lo + lane + 64 r] when sp.fast, and its centre zc = X[a]
// (X[lo] when empty)
template <typename T>
__device__ __forceinline__ SegFit fit_one(const T* __restrict__ X, const FitSpan& sp, const T (&v)[kFitRounds],
                                          double zc, int lane) {
  // a segment's keys sit in lanes [0, cnt) when sp.fast and cnt <= 64
  const int top = sp.fast ? butterfly_top(sp.last - sp.lo + 1) : kFitLanes / 2;
  FitSums s{0, 0, 0};
  if (sp.b - sp.a >= 2) {  // one key gives zero sums (its centre is itself)
    if (sp.fast) {
#pragma unroll
      for (int r = 0; r < kFitRounds; ++r) {
        const int64_t i = sp.lo + lane + kFitLanes * r;
        if (i >= sp.a && i < sp.b) add_key(s, i, v[r], sp.lo, zc);
      }
    } else {
      add_keys<T, kFitLanes>(X, sp.a, sp.b, sp.lo, zc, lane, s);
    }
    wave_sum(s, top);
  }
  SegFit f = line_fit(sp, zc, s);
  int32_t dmin = 1 << 30, dmax = -(1 << 30);
  if (sp.fast) {
#pragma unroll
    for (int r = 0; r < kFitRounds; ++r) {
      const int64_t i = sp.lo + lane + kFitLanes * r;
      if (i <= sp.last) err_key(f, i, v[r], sp.lo, dmin, dmax);
    }
  } else {
    err_keys<T, kFitLanes>(X, sp.lo, sp.last, f, lane, dmin, dmax);
  }
  wave_minmax(dmin, dmax, top);
  f.dmin = dmin;
  f.dmax = dmax;
  return f;
}

// The fit and error bounds of a short segment (fit range of at most
// kFitGroupKeys keys) by the kFitGroupLanes lanes of one group of a wave: the
// same sums, line and bounds as fit_one, with the butterflies inside the group,
// so the groups of a wave fit their segments with the same instructions.
// Every lane of the group holds the result; live = false gives an unused one.
template <typename T>
__device__ __forceinline__ SegFit fit_grouped(const T* __restrict__ X, const FitSpan& sp, bool live, int gl) {
  T v[kFitGroupRounds];
#pragma unroll
  for (int r = 0; r < kFitGroupRounds; ++r) {
    const int64_t i = sp.lo + gl + kFitGroupLanes * r;
    v[r] = (live && i <= sp.last) ? X[i] : T(0);
  }
  const double zc = live ? static_cast<double>(X[(sp.a < sp.b) ? sp.a : sp.lo]) : 0.0;
  FitSums s{0, 0, 0};
#pragma unroll
  for (int r = 0; r < kFitGroupRounds; ++r) {
    const int64_t i = sp.lo + gl + kFitGroupLanes * r;
    if (live && i >= sp.a && i < sp.b) add_key(s, i, v[r], sp.lo, zc);
  }
#pragma unroll
  for (int o = kFitGroupLanes / 2; o > 0; o >>= 1) {
    s.sz += __shfl_xor(s.sz, o, kFitGroupLanes);
    s.szz += __shfl_xor(s.szz, o, kFitGroupLanes);
    s.siz += __shfl_xor(s.siz, o, kFitGroupLanes);
  }
  SegFit f = line_fit(sp, zc, s);
  int32_t dmin = 1 << 30, dmax = -(1 << 30);
#pragma unroll
  for (int r = 0; r < kFitGroupRounds; ++r) {
    const int64_t i = sp.lo + gl + kFitGroupLanes * r;
    if (live && i <= sp.last) err_key(f, i, v[r], sp.lo, dmin, dmax);
  }
#pragma unroll
  for (int o = kFitGroupLanes / 2; o > 0; o >>= 1) {
    dmin = std::min(dmin, __shfl_xor(dmin, o, kFitGroupLanes));
    dmax = std::max(dmax, __shfl_xor(dmax, o, kFitGroupLanes));
  }
  f.dmin = dmin;
  f.dmax = dmax;
  return f;
}

// segments [kFitSegs x, kFitSegs (x + 1)) of the model, x = blockIdx.x: the
// short ones by lane groups, kFitSegs at once (group q takes segment
// kFitSegs x + q), then each longer one by the whole wave; with long_list
// (batched form), the long ones are queued there (count in tot->long_segs)
// for seg_fit_long_kernel
template <typename T>
__global__ void __launch_bounds__(kFitLanes, 7) seg_fit_kernel(const T* __restrict__ X, int64_t N,
                                                               const int32_t* __restrict__ first,
                                                               SegFit* __restrict__ segs, int32_t nseg,
                                                               const LearnMeta* __restrict__ lm,
                                                               PlanTotals* __restrict__ tot,
                                                               LongSeg* __restrict__ long_list) {
  static_assert(kFitSegs * kFitGroupLanes == kFitLanes, "one lane group per segment of the wave");
  const int slot = blockIdx.y;
  if (lm) {
    if (slot >= tot->n_learned) return;
    const LearnMeta L = lm[slot];
    X += L.x_off;
    N = L.N;
    first += (int64_t)slot * (nseg + 1);
    segs += (int64_t)slot * nseg;
  }
  const int32_t s0 = static_cast<int32_t>(blockIdx.x) * kFitSegs;
  const int lane = threadIdx.x;
  // first[s0 .. s0 + kFitSegs] (clamped to first[nseg]) in one load
  const int32_t fl = first[std::min(s0 + std::min(lane, kFitSegs), nseg)];
  {
    const int q = lane / kFitGroupLanes, gl = lane % kFitGroupLanes;
    const FitSpan sp = fit_span(__shfl(fl, q, kFitLanes), __shfl(fl, q + 1, kFitLanes), N);
    const bool mine = s0 + q < nseg && sp.last - sp.lo < kFitGroupKeys;
    if (__ballot(mine)) {  // the whole wave takes part in the groups' butterflies
      const SegFit f = fit_grouped<T>(X, sp, mine, gl);
      if (mine && gl == 0) segs[s0 + q] = f;
    }
  }
#pragma unroll 1
  for (int k = 0; k < kFitSegs; ++k) {
    if (s0 + k >= nseg) break;  // uniform across the wave
    const int64_t a = __builtin_amdgcn_readfirstlane(__shfl(fl, k, kFitLanes));
    const int64_t b = __builtin_amdgcn_readfirstlane(__shfl(fl, k + 1, kFitLanes));
    const FitSpan sp = fit_span(a, b, N);
    if (sp.last - sp.lo < kFitGroupKeys) continue;  // fitted by its group
    if (long_list && sp.last - sp.lo + 1 > kFitLongKeys) {
      if (lane == 0) long_list[atomicAdd(&tot->long_segs, 1u)] = LongSeg{slot, s0 + k};
      continue;
    }
    T v[kFitRounds];
#pragma unroll
    for (int r = 0; r < kFitRounds; ++r) {
      const int64_t i = sp.lo + lane + kFitLanes * r;
      v[r] = (sp.fast && i <= sp.last) ? X[i] : T(0);
    }
    const double zc = static_cast<double>(X[(a < b) ? a : sp.lo]);
    const SegFit f = fit_one<T>(X, sp, v, zc, lane);
    if (lane == 0) segs[s0 + k] = f;
  }
}

int32_t fit_blocks(int32_t nseg) { return (nseg + kFitSegs - 1) / kFitSegs; }

// The queued long segments, one workgroup of kLongBlock lanes at a time each
// (workgroup x takes entries x, x + gridDim.x, ...).
template <typename T>
__global__ void __launch_bounds__(kLongBlock) seg_fit_long_kernel(const T* __restrict__ X,
                                                                  const int32_t* __restrict__ first_all,
                                                                  SegFit* __restrict__ segs_all, int32_t nseg,
                                                                  const LearnMeta* __restrict__ lm,
                                                                  const PlanTotals* __restrict__ tot,
                                                                  const LongSeg* __restrict__ list) {
  constexpr int kW = kLongBlock / 64;
  __shared__ double red[3][kW];
  __shared__ int32_t redi[2][kW];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t count = tot->long_segs;
  for (uint32_t e = blockIdx.x; e < count; e += gridDim.x) {  // uniform across the workgroup
    const LongSeg ls = list[e];
    const LearnMeta L = lm[ls.slot];
    const T* Xa = X + L.x_off;
    const int32_t* first = first_all + (int64_t)ls.slot * (nseg + 1);
    const FitSpan sp = fit_span(first[ls.s], first[ls.s + 1], L.N);
    const double zc = static_cast<double>(Xa[(sp.a < sp.b) ? sp.a : sp.lo]);
    FitSums s{0, 0, 0};
    add_keys<T, kLongBlock>(Xa, sp.a, sp.b, sp.lo, zc, tid, s);
    wave_sum(s);
    if (lane == 0) {
      red[0][w] = s.sz;
      red[1][w] = s.szz;
      red[2][w] = s.siz;
    }
    __syncthreads();
    FitSums t{0, 0, 0};
    for (int ww = 0; ww < kW; ++ww) {
      t.sz += red[0][ww];
      t.szz += red[1][ww];
      t.siz += red[2][ww];
    }
    SegFit f = line_fit(sp, zc, t);
    int32_t dmin = 1 << 30, dmax = -(1 << 30);
    err_keys<T, kLongBlock>(Xa, sp.lo, sp.last, f, tid, dmin, dmax);
    wave_minmax(dmin, dmax);
    if (lane == 0) {
      redi[0][w] = dmin;
      redi[1][w] = dmax;
    }
    __syncthreads();
    if (tid == 0) {
      for (int ww = 0; ww < kW; ++ww) {
        dmin = std::min(dmin, redi[0][ww]);
        dmax = std::max(dmax, redi[1][ww]);
      }
      f.dmin = dmin;
      f.dmax = dmax;
      segs_all[(int64_t)ls.slot * nseg + ls.s] = f;
    }
    __syncthreads();  // red and redi are reused by the next entry
  }
}


// ---------------------------------------------------------------------------
// search

template <typename T>
struct LearnedArgs {
  const T* X;
  const T* S;  // samples X_{E j} (single-array search)
  const float* params;
  const SegFit* segs;
  const float* steps;  // compiled router (kRouteTable)
  const uint32_t* grid;
  int32_t log2g;
  unsigned long long* fallbacks;
  const T* z;
  int32_t* out;
  int64_t M;
  double X0d, delta, flo, fscale;
  T X0, XN;
  int32_t N, nseg, identity, pad;
};

// Window of candidate indices for z from its segment: [q + dmin - 1, q + dmax]
// relative to lo, kept inside [lo, hi].
template <typename T>
__device__ __forceinline__ void query_window(T z, int32_t seg, const SegFit* segs, int32_t* L, int32_t* U) {
  const SegFit sg = segs[seg];
  const int32_t q = seg_predict<T>(sg, z);
  *L = std::min(std::max(sg.lo, sg.lo + q + sg.dmin - 1), sg.hi);
  *U = std::min(std::max(*L, sg.lo + q + sg.dmax), sg.hi);
}


// Values of X after X_N that the search may read (+inf): the block read by
// the sample search can start at the block after the last one of X_N's.
constexpr int64_t kLearnScanPad = 32;

template <typename T>
using vec16b = T __attribute__((ext_vector_type(16 / sizeof(T))));

// The end of the search of a window [L, U] of a single array, through its
// sample array S (S[j] = X_{E j}, E = 64 / sizeof(T) keys per 64-byte block of
// X, +inf past the end): the samples jL + 1 .. jU + 1 of the window's blocks
// (64 bytes of S, which stays in L2: N bytes in f64) give the block js of the
// answer, whose E values are then read as one 64-byte block and counted.
// Instead of the dependent probes of a bisection into X and one or two lines
// of X, a query reads 64 bytes of S and one block of X, and a window inside
// one block reads that block alone (plus the next value when all of the
// block's values are <= z).
//
// sample_block returns js and the window's blocks [jL, jU] after narrowing.
// The samples read are 64 bytes of S: the aligned line that holds sample
// jL + 1 when it holds sample jU + 1 too, else the 64 bytes from the 16-byte
// word of sample jL + 1 (a window of up to SE - V + 1 blocks, 7 in f64 and 13
// in f32; longer windows are first narrowed by bisection on S), all issued
// before any is used.  S is non-decreasing, so the samples <= z among them form a
// prefix: with A of them, the samples jL + 1 .. jU + 1 that are <= z are
// those before s0 + A, and no per-sample test of the window's ends is needed.
template <typename T>
__device__ __forceinline__ int32_t sample_block(T z, int32_t L, int32_t U, const T* __restrict__ S, int32_t* jL_out,
                                                int32_t* jU_out) {
  constexpr int E = 64 / int(sizeof(T));   // keys per 64-byte block of X
  constexpr int SE = 64 / int(sizeof(T));  // samples per 64 bytes of S
  constexpr int V = 16 / int(sizeof(T));   // samples per 16-byte word
  int32_t jL = L / E, jU = U / E;
  while (jU + 1 > ((jL + 1) & ~(V - 1)) + SE - 1) {  // windows of more than SE - V + 1 blocks only
    const int32_t m = jL + ((jU - jL + 1) >> 1);
    const bool c = S[m] <= z;
    jL = c ? m : jL;
    jU = c ? jU : m - 1;
  }
  // a window inside one block reads no samples: the block decides unless all
  // of its values are <= z (then the next value, the first of the next block)
  int32_t c1 = 0;
  if (jU > jL) {
    // the 64-byte-aligned line of sample jL + 1 when it holds jU + 1 too (one
    // request to L2), else the 64 bytes from jL + 1's 16-byte word (two)
    const int32_t s64 = (jL + 1) & ~(SE - 1);
    const int32_t s0 = (jU + 1 <= s64 + SE - 1) ? s64 : ((jL + 1) & ~(V - 1));
    const vec16b<T>* p = reinterpret_cast<const vec16b<T>*>(S + s0);
    vec16b<T> x[SE / V];
#pragma unroll
    for (int v = 0; v < SE / V; ++v) x[v] = p[v];
    int32_t A = 0;
#pragma unroll
    for (int v = 0; v < SE / V; ++v)
#pragma unroll
      for (int e = 0; e < V; ++e) A += (x[v][e] <= z) ? 1 : 0;
    c1 = std::max(0, std::min(jU + 1, s0 + A - 1) - jL);
  }
  *jL_out = jL;
  *jU_out = jU;
  return jL + c1;
}

// The result from the count c2 of values <= z in block js: with c2 values
// <= z, X_{E js + c2 - 1} <= z < X_{E js + c2} has been read when
// 1 <= c2 <= E - 1, or when c2 = E and the sample js + 1 was read (else it is
// read here); *certified tells whether that holds, whatever the model
// predicted.
template <typename T>
__device__ __forceinline__ int32_t block_result(T z, int32_t jL, int32_t jU, int32_t js, int32_t c2,
                                                const T* __restrict__ X, bool* certified) {
  constexpr int E = 64 / int(sizeof(T));
  bool upper = c2 <= E - 1 || (jU > jL && js <= jU);  // the value after the answer was read
  if (c2 == E && jU == jL) upper = z < X[int64_t(js + 1) * E];
  *certified = c2 >= 1 && upper;
  return js * E + c2 - 1;
}

// sample_block, then each lane reads its own block (four 16-byte loads).
template <typename T>
__device__ __forceinline__ int32_t sample_search(T z, int32_t L, int32_t U, const T* __restrict__ X,
                                                 const T* __restrict__ S, bool* certified) {
  constexpr int E = 64 / int(sizeof(T));
  constexpr int V = 16 / int(sizeof(T));
  int32_t jL, jU;
  const int32_t js = sample_block<T>(z, L, U, S, &jL, &jU);
  const vec16b<T>* q = reinterpret_cast<const vec16b<T>*>(X + int64_t(js) * E);
  int32_t c2 = 0;
#pragma unroll
  for (int v = 0; v < E / V; ++v) {
    const vec16b<T> x = q[v];
#pragma unroll
    for (int e = 0; e < V; ++e) c2 += (x[e] <= z) ? 1 : 0;
  }
  return block_result<T>(z, jL, jU, js, c2, X, certified);
}

// Sum of v over the four lanes of each quad (lanes 4k .. 4k + 3), in every
// lane of the quad: two DPP quad permutations, [1,0,3,2] then [2,3,0,1].
__device__ __forceinline__ int32_t quad_sum(int32_t v) {
  v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  v += __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  return v;
}

// Value of lane r of each quad (lanes 4k .. 4k + 3), in every lane of the
// quad: a DPP quad permutation [r, r, r, r] per 32-bit word.  r must be a
// constant after unrolling.
__device__ __forceinline__ int32_t quad_bcast32(int32_t v, int r) {
  switch (r) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0x00, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x55, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_mov_dpp(v, 0xAA, 0xF, 0xF, false);
    default: return __builtin_amdgcn_mov_dpp(v, 0xFF, 0xF, 0xF, false);
  }
}

template <typename U>
__device__ __forceinline__ U quad_bcast(U v, int r) {
  static_assert(sizeof(U) % 4 == 0, "32-bit words");
  int32_t w[sizeof(U) / 4];
  __builtin_memcpy(w, &v, sizeof(U));
#pragma unroll
  for (int i = 0; i < int(sizeof(U) / 4); ++i) w[i] = quad_bcast32(w[i], r);
  __builtin_memcpy(&v, w, sizeof(U));
  return v;
}

// How many of the E values of block blk of X (values blk E .. blk E + E - 1)
// are <= z, for the query of every lane.  All 64 lanes must take part with a
// valid block.  The blocks are read cooperatively, inside each quad: in round
// r the four lanes of a quad read 16 bytes each of the block of the quad's
// lane r (its block and z broadcast by DPP), so each load instruction touches
// 16 blocks (a lane reading its own block makes four loads that each touch
// 64).  The quad's counts are summed by DPP and lane r keeps round r's sum.
// coop_issue issues the four loads; coop_count counts once they are needed,
// so the caller can issue other loads in between.
// MASK: only the positions e_lo .. e_hi of the query's block count (the
// block of a packed buffer holds values of neighbouring arrays).
template <typename T, bool MASK>
struct CoopBlock {
  vec16b<T> x[4];
  int32_t bounds;  // MASK: e_lo | e_hi << 8 of this lane's query
};

template <typename T, bool MASK, typename I>
__device__ __forceinline__ void coop_issue(const T* __restrict__ X, I blk, int32_t e_lo, int32_t e_hi,
                                           CoopBlock<T, MASK>& c) {
  constexpr int E = 64 / int(sizeof(T));
  constexpr int V = 16 / int(sizeof(T));
  const int sub = threadIdx.x & 3;
  if constexpr (MASK) c.bounds = e_lo | (e_hi << 8);
#pragma unroll
  for (int r = 0; r < 4; ++r) {  // every load is issued before any value is used
    const I b = quad_bcast(blk, r);
    c.x[r] = *reinterpret_cast<const vec16b<T>*>(X + int64_t(b) * E + sub * V);
  }
}

// z (and the bounds) of round r's query are broadcast again here rather than
// held from coop_issue, which keeps fewer registers live while the loads are
// in flight.
template <typename T, bool MASK>
__device__ __forceinline__ int32_t coop_count(const CoopBlock<T, MASK>& c, T z) {
  constexpr int V = 16 / int(sizeof(T));
  const int sub = threadIdx.x & 3;
  int32_t mine = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const T zr = quad_bcast(z, r);
    const int32_t bd = MASK ? quad_bcast32(c.bounds, r) : 0;
    int32_t n = 0;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int pos = sub * V + e;
      const bool in = MASK ? (pos >= (bd & 0xff) && pos <= (bd >> 8)) : true;
      n += (in && c.x[r][e] <= zr) ? 1 : 0;
    }
    n = quad_sum(n);
    mine = (sub == r) ? n : mine;
  }
  return mine;
}

template <typename T, bool MASK = false, typename I>
__device__ __forceinline__ int32_t coop_block_count(const T* __restrict__ X, I blk, T z, int32_t e_lo = 0,
                                                    int32_t e_hi = 0) {
  CoopBlock<T, MASK> c;
  coop_issue<T, MASK>(X, blk, e_lo, e_hi, c);
  return coop_count<T, MASK>(c, z);
}

// Samples of the single-array search: S[j] = X_{E j} for E j < nX (X padded
// with +inf), +inf beyond.
template <typename T>
__global__ void samples_kernel(const T* __restrict__ X, int64_t nX, T* __restrict__ S, int64_t nS) {
  constexpr int E = 64 / int(sizeof(T));
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nS) S[j] = (j * E < nX) ? X[j * E] : std::numeric_limits<T>::infinity();
}

// The sample search for an array inside a packed buffer Xp of total_x values
// (array values at x_off .. x_off + N, no padding between arrays): blocks and
// samples are those of the whole buffer, S[J] = Xp[E J], and only samples
// whose value belongs to the array are counted (blocks after the first one of
// the array, up to the block holding X_N); the samples read are the 64 bytes
// from the 16-byte word of sample jL + 1, as in sample_block.  The answer's
// block is scanned with the values outside the array masked, read value by
// value where the buffer is not 16-byte aligned or the block passes its end
// (COOP: when no lane's block passes the end of an aligned buffer, the wave
// reads the blocks cooperatively, coop_issue / coop_count; every lane of the
// wave must then take part).  between() is called once, by the whole wave
// together, after the block's loads are issued where they are cooperative
// (before them otherwise): the caller's next loads then do not hold up this
// count.
// Certification as in sample_search, over the array's own values.
// The array's place in the packed buffer, the same for every lane of a tile:
// its values start at Xb[xr] (Xb = Xp + E xb, the start of the block that
// holds its first value, xr < E), its samples are Sb[j] = S[xb + j], and
// blocks j with E j + E <= lim lie inside the buffer.  Block indices below
// are relative to xb, so they fit 32 bits.
template <typename T>
struct PackedArray {
  const T* Xb;
  const T* Sb;
  int32_t xr, N;
  int32_t lim;  // total_x - E xb, capped at INT32_MAX
};

template <typename T>
__device__ __forceinline__ PackedArray<T> packed_array(const T* Xp, const T* S, int64_t x_off, int32_t N,
                                                       int64_t total_x) {
  constexpr int64_t E = 64 / int64_t(sizeof(T));
  const int64_t xb = x_off / E;
  PackedArray<T> pa;
  pa.Xb = Xp + xb * E;
  pa.Sb = S + xb;
  pa.xr = static_cast<int32_t>(x_off - xb * E);
  pa.N = N;
  pa.lim = static_cast<int32_t>(std::min<int64_t>(total_x - xb * E, INT32_MAX));
  return pa;
}

template <typename T, bool COOP, typename F>
__device__ __forceinline__ int32_t sample_search_packed(T z, int32_t L, int32_t U, const PackedArray<T>& pa,
                                                        bool* certified, F&& between) {
  constexpr int E = 64 / int(sizeof(T));
  constexpr int SE = 64 / int(sizeof(T));
  constexpr int V = 16 / int(sizeof(T));
  const T* __restrict__ S = pa.Sb;
  const int32_t jlast = (pa.xr + pa.N) / E;  // block holding X_N
  // 0 <= L <= U: the divisions are shifts
  int32_t jL = static_cast<int32_t>(static_cast<uint32_t>(pa.xr + L) / E);
  int32_t jU = static_cast<int32_t>(static_cast<uint32_t>(pa.xr + U) / E);
  while (jU + 1 > ((jL + 1) & ~(V - 1)) + SE - 1) {
    const int32_t m = jL + ((jU - jL + 1) >> 1);  // jL < m <= jU: S[m] is a value of the array
    const bool c = S[m] <= z;
    jL = c ? m : jL;
    jU = c ? jU : m - 1;
  }
  const int32_t jt = std::min(jU + 1, jlast);  // samples jL + 1 .. jt are counted
  // the 64-byte-aligned line of sample jL + 1 when it holds jt too, else the
  // 64 bytes from jL + 1's 16-byte word
  const int32_t s64 = (jL + 1) & ~(SE - 1);
  const int32_t s0 = (jt <= s64 + SE - 1) ? s64 : ((jL + 1) & ~(V - 1));
  const vec16b<T>* p = reinterpret_cast<const vec16b<T>*>(S + s0);
  vec16b<T> xs[SE / V];
#pragma unroll
  for (int v = 0; v < SE / V; ++v) xs[v] = p[v];
  // sample s0 + i counts when jL < s0 + i <= jt, i.e. (s0 - jL - 1) + i in [0, jt - jL)
  const int32_t d = s0 - jL - 1;
  const uint32_t span = static_cast<uint32_t>(jt - jL);
  int32_t c1 = 0;
#pragma unroll
  for (int v = 0; v < SE / V; ++v)
#pragma unroll
    for (int e = 0; e < V; ++e) c1 += (static_cast<uint32_t>(d + v * V + e) < span && xs[v][e] <= z) ? 1 : 0;
  const int32_t js = jL + c1;
  const int32_t k0 = js * E;  // the block's first value, relative to Xb
  const int32_t e_lo = std::max(0, pa.xr - k0);
  const int32_t e_hi = std::min(E - 1, pa.xr + pa.N - k0);
  const bool aligned = (reinterpret_cast<uintptr_t>(pa.Xb) & 15) == 0;
  int32_t c2 = 0;
  if (COOP && aligned && !__ballot(k0 + E > pa.lim)) {
    // every lane's block lies inside the buffer: the wave reads them cooperatively
    CoopBlock<T, true> cb;
    coop_issue<T, true>(pa.Xb, js, e_lo, e_hi, cb);
    between();
    c2 = coop_count<T, true>(cb, z);
  } else {
    between();  // by the whole wave, before the lanes part
    if (aligned && k0 + E <= pa.lim) {
      const vec16b<T>* q = reinterpret_cast<const vec16b<T>*>(pa.Xb + k0);
#pragma unroll
      for (int v = 0; v < E / V; ++v) {
        const vec16b<T> x = q[v];
#pragma unroll
        for (int e = 0; e < V; ++e) c2 += (v * V + e >= e_lo && v * V + e <= e_hi && x[e] <= z) ? 1 : 0;
      }
    } else {
      for (int32_t e = e_lo; e <= e_hi; ++e) c2 += (pa.Xb[k0 + e] <= z) ? 1 : 0;
    }
  }
  *certified = c2 >= 1 && (c2 <= e_hi - e_lo || js + 1 <= jt);
  return k0 + e_lo + c2 - 1 - pa.xr;
}

// Index of z by the classic binary search over the whole array, for a query
// whose window search could not certify its result (counted).
template <typename T>
__device__ int32_t full_search_counted(T z, const T* __restrict__ X, int32_t N, unsigned long long* fallbacks) {
  atomicAdd(fallbacks, 1ull);
  int32_t lo = 0, nn = N;
  while (nn > 1) {
    const int32_t h = nn >> 1;
    const bool c = z >= X[lo + h];
    lo = c ? lo + h : lo;
    nn = c ? nn - h : h;
  }
  return lo;
}

// One 64-query group per wave and iteration; the next group's queries are
// loaded before this group is worked on.  A query is routed to its segment
// (the compiled router's grid and steps in LDS, or the network evaluated on
// the matrix cores), takes its window from the segment's fit, finds the
// 64-byte block of X that holds its answer from the samples of the window's
// blocks, and counts that block's values <= z (COOP: four lanes read each
// block together); a result that could not be certified (never expected)
// takes a full binary search and is counted.
template <typename T, int ROUTE, bool COOP>
__global__ void __launch_bounds__(1024) learned_search_kernel(LearnedArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  RouterShared16* Sp = nullptr;  // FP16 router's shared values (no static LDS in the other modes)
  const int64_t seg_bytes = int64_t(a.nseg) * sizeof(SegFit);
  stage_bytes(smem, reinterpret_cast<const unsigned char*>(a.segs), seg_bytes);
  const SegFit* segs = reinterpret_cast<const SegFit*>(smem);
  const float* steps = reinterpret_cast<const float*>(smem + seg_bytes);
  const uint32_t* grid = reinterpret_cast<const uint32_t*>(smem + seg_bytes + int64_t(a.nseg) * 4);
  // FP16 router: half-wave-uniform values in LDS, W2 rows in registers
  half4 w2[4];
  RouterRegs R;
  if constexpr (ROUTE == kRouteTable) {
    if (!a.identity) {
      stage_words(smem + seg_bytes, a.steps, a.nseg);
      stage_words(smem + seg_bytes + int64_t(a.nseg) * 4, a.grid, int64_t(1) << a.log2g);
    }
  } else if constexpr (ROUTE == kRouteF16) {
    __shared__ RouterShared16 S;
    Sp = &S;
    fill_router_shared16(a.params, Sp, w2);
  } else {
    load_router(a.params, R);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t stride = waves * 64;
  int64_t base = wave * 64;
  // the load is unconditional (the index clamped to the last query; the lanes
  // past M discard their result), so the compiler can leave the next group's
  // load in flight: under a branch it could not count it and would wait for it
  auto load_z = [&](int64_t q) { return __builtin_nontemporal_load(a.z + std::min(q, a.M - 1)); };
  T z = load_z(base + lane);
  for (; base < a.M; base += stride) {
    // the per-lane read loads the next group at once; the cooperative one
    // after its block loads, so that waiting for the samples does not
    // wait for the next group (loads complete in order)
    T z_next;
    if constexpr (!COOP) z_next = load_z(base + stride + lane);
    const float u = feature(static_cast<double>(z), a.X0d, a.delta, a.flo, a.fscale);
    int32_t seg;
    if constexpr (ROUTE == kRouteTable) {
      seg = a.identity ? segment_of(u, a.nseg) : grid_segment(u, steps, grid, a.log2g);
    } else {
      float y_net;
      if constexpr (ROUTE == kRouteF16) {
        asm volatile("" ::: "memory");  // keeps the LDS reads of the router inside the loop
        y_net = route_pair_shared16(u, w2, Sp);
      } else {
        y_net = route_pair<false>(u, &R);
      }
      seg = segment_of(a.identity ? u : route_coord(y_net, u), a.nseg);
    }
    int32_t L, U;
    query_window<T>(z, seg, segs, &L, &U);
    bool certified;
    int32_t i;
    if constexpr (COOP) {
      int32_t jL, jU;
      const int32_t js = sample_block<T>(z, L, U, a.S, &jL, &jU);
      CoopBlock<T, false> cb;
      coop_issue<T, false>(a.X, js, 0, 0, cb);
      z_next = load_z(base + stride + lane);
      i = block_result<T>(z, jL, jU, js, coop_count<T, false>(cb, z), a.X, &certified);
    } else {
      i = sample_search<T>(z, L, U, a.X, a.S, &certified);
    }
    if ((z >= a.X0) && (z < a.XN) && !certified) i = full_search_counted<T>(z, a.X, a.N, a.fallbacks);
    i = (z >= a.XN) ? a.N : i;
    i = (z >= a.X0) ? i : -1;
    if (base + lane < a.M) __builtin_nontemporal_store(i, a.out + base + lane);
    z = z_next;
  }
}

// Xp[from .. to - 1] = +inf
template <typename T>
__global__ void fill_inf_kernel(T* __restrict__ Xp, int64_t from, int64_t to) {
  const int64_t k = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < to) Xp[k] = std::numeric_limits<T>::infinity();
}

// Largest grid of the compiled router (cells) and the most segments of a
// single-array model: its search stages the fits (32 bytes each), the steps
// (4 bytes each) and the grid (4 bytes per cell) in one workgroup's LDS.
constexpr int32_t kMaxLog2Grid = 12;
constexpr int32_t kMaxLearnSegments = 4096;
// 2048 segments (64 KiB of fits, 8 KiB of steps, 8 KiB of grid) leave room
// for two 1024-thread workgroups per CU
constexpr int32_t kDefaultLearnSegments = 2048;
constexpr int64_t kLearnLdsBudget = 160 * 1024;

// probe points of the router compilation: 2^kp + 1 <= nseg + 1
int32_t probe_log2(int32_t nseg) {
  int32_t k = 0;
  while ((2 << k) <= nseg) ++k;
  return k;
}

// grid cells for nseg segments: as many cells as segments (rounded up to a
// power of two), at most 4096, and fewer where the LDS budget requires
int32_t grid_log2(int32_t nseg, int64_t budget) {
  int32_t k = 0;
  while (k < kMaxLog2Grid && (1 << k) < nseg) ++k;
  while (k > 0 && int64_t(nseg) * (int64_t(sizeof(SegFit)) + 4) + (int64_t(4) << k) > budget) --k;
  return k;
}

// the network's parameters, the segment fits and, for the compiled router, its step table and grid
int64_t learned_model_bytes(const LearnedModel* L) {
  const bool table = L->router == kRouteTable && !L->identity;
  return int64_t(kParams) * 4 + int64_t(L->nseg) * (int64_t(sizeof(SegFit)) + (table ? 4 : 0)) +
         (table ? (int64_t(4) << L->log2g) : 0);
}

// The starting point of a model: the network is set to a piecewise-linear CDF
// of the array's keys.  With u_q the feature of the key at position q N / 64
// (q = 0 .. 64), layer-1 unit k rises from 0 to 1 over [u_2k, u_2k+2], the
// k-th 32-quantile interval.  Layer 2 then spends its units where that is
// least linear: the kInitSplit intervals whose median feature u_2k+1 lies
// farthest from the middle of the interval are split there (two units, one
// rising over each half, each weighted 1/64 in the output), and one more unit
// sums the ramps of all the other intervals (weighted by their share).  So
// y(u_2k) = k / 32 and, in a split interval, y(u_2k+1) = (2k + 1) / 64: a tight
// cluster of keys gets ramps (and so segments) of its own from the start,
// which training from a generic starting point (ramps spread evenly over u)
// does not achieve in the steps the build can afford.  Every weight is >= 0:
// the network is monotone.  Adam's moments start at zero.  One workgroup of 64
// lanes per model: the single array's (lm null), or learned slot blockIdx.x of
// a batch.
constexpr int kInitSplit = 15;  // (kHid - 1) / 2: two layer-2 units per split, one for the rest

template <typename T>
__global__ void __launch_bounds__(64) init_params_kernel(float* __restrict__ params, float* __restrict__ m,
                                                         float* __restrict__ v, const T* __restrict__ X, int64_t N,
                                                         double X0, double delta, double flo, double fscale,
                                                         const LearnMeta* __restrict__ lm,
                                                         const PlanTotals* __restrict__ tot) {
  static_assert(2 * kInitSplit + 1 <= kHid, "layer-2 units");
  if (lm) {
    const int slot = blockIdx.x;
    if (slot >= tot->n_learned) return;
    const LearnMeta L = lm[slot];
    X += L.x_off;
    N = L.N;
    X0 = L.X0;
    delta = L.delta;
    flo = L.flo;
    fscale = L.fscale;
    params += (int64_t)slot * kParams;
    m += (int64_t)slot * kParams;
    v += (int64_t)slot * kParams;
  }
  const int t = threadIdx.x;
  auto feat = [&](int64_t pos) { return feature(static_cast<double>(X[pos]), X0, delta, flo, fscale); };
  // u_q for lane q < 64, and u_64 (the last key) in every lane
  const float uq = feat((int64_t(t) * N + 32) / 64);
  const float u_end = feat(N);
  // interval k = lane t < kHid: its ends and median
  const int k = t & (kHid - 1);
  const float lo = __shfl(uq, 2 * k, 64), mid = __shfl(uq, 2 * k + 1, 64);
  const float hi = (k + 1 < kHid) ? __shfl(uq, 2 * k + 2, 64) : u_end;
  const float w1 = 1.0f / std::fmax(hi - lo, 0x1p-24f);
  const float b1 = -lo * w1;
  // where the median sits in the ramp, as layer 1 computes it
  const float tm = clamp01(std::fma(w1, mid, b1));
  const bool can_split = tm > 0x1p-20f && tm < 1.0f - 0x1p-20f;
  const float score = can_split ? std::fabs(tm - 0.5f) : -1.0f;
  // rank of the score among the intervals (ties by interval index)
  int rank = 0;
  for (int j2 = 0; j2 < kHid; ++j2) {
    const float sj = __shfl(score, j2, 64);
    rank += (sj > score || (sj == score && j2 < k)) ? 1 : 0;
  }
  const bool split = t < kHid && can_split && rank < kInitSplit;
  const uint64_t split_mask = __ballot(split);
  const int n_split = __popcll(split_mask);
  const int n_rest = kHid - n_split;
  if (t < kHid) {
    params[oW1 + t] = w1;
    params[oB1 + t] = b1;
    for (int j2 = 0; j2 < kHid; ++j2) params[oW2 + j2 * kHid + t] = 0.0f;
    params[oB2 + t] = 0.0f;
    params[oW3 + t] = 0.0f;
  }
  __syncthreads();
  if (t < kHid) {
    if (split) {
      // the r-th split interval drives units 1 + 2r (its first half) and 2 + 2r (its second)
      const int r = __popcll(split_mask & ((uint64_t(1) << t) - 1));
      const int j1 = 1 + 2 * r, j2 = 2 + 2 * r;
      params[oW2 + j1 * kHid + t] = 1.0f / tm;
      params[oW2 + j2 * kHid + t] = 1.0f / (1.0f - tm);
      params[oB2 + j2] = -tm / (1.0f - tm);
      params[oW3 + j1] = 1.0f / (2 * kHid);
      params[oW3 + j2] = 1.0f / (2 * kHid);
    } else {
      params[oW2 + 0 * kHid + t] = 1.0f / static_cast<float>(n_rest);  // unit 0 sums the rest
    }
    if (t == 0) params[oW3 + 0] = static_cast<float>(n_rest) / kHid;
  }
  if (t == 0) params[oB3] = 0.0f;
  for (int q = t; q < kParams; q += blockDim.x) {
    m[q] = 0.0f;
    v[q] = 0.0f;
  }
}

template <typename T>
ds_status learned_build_typed(ds_index* h, const ds_build_opts* o, hipStream_t s) {
  LearnedModel* L = new (std::nothrow) LearnedModel();
  if (!L) return DS_ERR_OOM;
  h->learned = L;
  const int64_t N = h->N;
  const int64_t n = N + 1;
  {
    // the handle's copy of X gets kLearnScanPad values of +inf after X_N for the search's block scan
    T* Xp = nullptr;
    if (hipMalloc(&Xp, size_t(n + kLearnScanPad) * sizeof(T)) != hipSuccess) return DS_ERR_OOM;
    if (hipMemcpyAsync(Xp, h->X, size_t(n) * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess) {
      (void)hipFree(Xp);
      return DS_ERR_HIP;
    }
    fill_inf_kernel<T><<<dim3(1), dim3(64), 0, s>>>(Xp, n, n + kLearnScanPad);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      (void)hipFree(Xp);
      return DS_ERR_HIP;
    }
    (void)hipFree(h->X);
    h->X = Xp;
    h->nX = n + kLearnScanPad;
  }
  {
    // samples of every 64-byte block of X, plus two 64-byte lines of +inf
    constexpr int64_t E = 64 / int64_t(sizeof(T));
    L->nsamples = ((h->nX + E - 1) / E + 2 * E + E - 1) / E * E;
    if (hipMalloc(&L->samples, size_t(L->nsamples) * sizeof(T)) != hipSuccess) return DS_ERR_OOM;
    samples_kernel<T><<<dim3((unsigned)((L->nsamples + 255) / 256)), dim3(256), 0, s>>>(
        static_cast<const T*>(h->X), h->nX, static_cast<T*>(L->samples), L->nsamples);
    DS_HIP_CHECK(hipGetLastError());
  }
  const T* X = static_cast<const T*>(h->X);
  T ends[2];
  DS_HIP_CHECK(hipMemcpyAsync(&ends[0], X, sizeof(T), hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipMemcpyAsync(&ends[1], X + N, sizeof(T), hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipStreamSynchronize(s));
  h->X0 = ends[0];
  h->XN = ends[1];
  const double range = static_cast<double>(ends[1]) - static_cast<double>(ends[0]);
  L->delta = std::max(range * 0x1p-40, 1e-300);
  {
    double d0 = L->delta, d1 = range + L->delta;
    int64_t b0, b1;
    std::memcpy(&b0, &d0, 8);
    std::memcpy(&b1, &d1, 8);
    L->flo = static_cast<double>(b0);
    L->fscale = 1.0 / (static_cast<double>(b1) - L->flo);
  }
  const int32_t nseg = o->learn_segments > 0 ? o->learn_segments : kDefaultLearnSegments;
  if (nseg < 1 || nseg > kMaxLearnSegments) return DS_ERR_ARG;
  L->nseg = nseg;
  L->identity = (o->learn_epochs < 0) ? 1 : 0;
  L->router = (o->learn_flags & DS_LEARN_FP32_ROUTER) ? kRouteF32
             : (o->learn_flags & DS_LEARN_EVAL_ROUTER) ? kRouteF16
                                                       : kRouteTable;
  const int32_t batch = o->learn_batch > 0 ? o->learn_batch : 8192;
  const int32_t epochs = o->learn_epochs > 0 ? o->learn_epochs : (o->learn_epochs == 0 ? 60 : 0);
  const float lr = o->learn_rate > 0 ? o->learn_rate : 2e-3f;
  const int32_t n_parts = (batch + kTrainBlock - 1) / kTrainBlock;
  if (hipMalloc(&L->params, kParams * 4) != hipSuccess || hipMalloc(&L->adam_m, kParams * 4) != hipSuccess ||
      hipMalloc(&L->adam_v, kParams * 4) != hipSuccess ||
      hipMalloc(&L->partial, size_t(n_parts) * kParams * 4) != hipSuccess ||
      hipMalloc(&L->loss_partial, size_t(n_parts) * 4 + 4) != hipSuccess ||
      hipMalloc(&L->feat, size_t(n) * 4) != hipSuccess || hipMalloc(&L->route, size_t(n) * 4) != hipSuccess ||
      hipMalloc(&L->first, size_t(nseg + 1) * 4) != hipSuccess ||
      hipMalloc(&L->segs, size_t(nseg) * sizeof(SegFit)) != hipSuccess ||
      hipMalloc(&L->steps, size_t(nseg) * 4) != hipSuccess ||
      hipMalloc(&L->grid, size_t(4) << kMaxLog2Grid) != hipSuccess ||
      hipMalloc(&L->fallbacks, 8) != hipSuccess)
    return DS_ERR_OOM;
  // the starting point: the keys' piecewise-linear CDF at their 32-quantiles
  init_params_kernel<T><<<dim3(1), dim3(64), 0, s>>>(L->params, L->adam_m, L->adam_v, X, n - 1,
                                                     static_cast<double>(ends[0]), L->delta, L->flo, L->fscale,
                                                     nullptr, nullptr);
  DS_HIP_CHECK(hipGetLastError());
  const unsigned long long zero = 0;
  DS_HIP_CHECK(hipMemcpyAsync(L->fallbacks, &zero, 8, hipMemcpyHostToDevice, s));
  feature_kernel<T><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(X, n, static_cast<double>(ends[0]),
                                                                             L->delta, L->flo, L->fscale, L->feat);
  DS_HIP_CHECK(hipGetLastError());
  // training: epochs passes of n / batch steps, cosine-decayed step size
  const int64_t steps = L->identity ? 0 : std::max<int64_t>(1, int64_t(epochs) * ((n + batch - 1) / batch));
  for (int64_t st = 0; st < steps; ++st) {
    train_step_kernel<<<dim3(n_parts), dim3(kTrainBlock), 0, s>>>(L->params, L->feat, n, o->seed, st, batch, nullptr,
                                                                  nullptr, L->partial, L->loss_partial);
    adam_kernel<<<dim3(1), dim3(1024), 0, s>>>(L->params, L->adam_m, L->adam_v, L->partial, n_parts,
                                               train_rate(lr, st, steps), st + 1, nullptr);
  }
  DS_HIP_CHECK(hipGetLastError());
  if (steps > 0) {
    float* dloss = L->loss_partial + n_parts;
    sum_kernel<<<1, 64, 0, s>>>(L->loss_partial, n_parts, dloss);
    float fl = 0;
    DS_HIP_CHECK(hipMemcpyAsync(&fl, dloss, 4, hipMemcpyDeviceToHost, s));
    DS_HIP_CHECK(hipStreamSynchronize(s));
    L->final_loss = fl;
  }
  // route the keys with the search-time router, then segments, fits and bounds
  if (L->router == kRouteTable && !L->identity) {
    const int32_t kp = probe_log2(nseg);  // L->first (nseg + 1 entries) holds the probes until the fits
    router_probe_kernel<<<dim3((unsigned)(((1 << kp) + 1 + 255) / 256)), dim3(256), 0, s>>>(L->params, nseg, kp,
                                                                                         L->first, nullptr);
    router_steps_kernel<<<dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, s>>>(L->params, nseg, kp, L->first,
                                                                                 L->steps, nullptr);
    L->log2g = grid_log2(nseg, kLearnLdsBudget);
    router_table_kernel<<<dim3(1), dim3(kTableBlock), 0, s>>>(L->steps, nseg, L->log2g, L->grid, nullptr);
    route_keys_table_kernel<<<dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s>>>(
        L->steps, L->feat, n, nseg, L->route);
  } else if (L->router == kRouteF16) {
    route_keys_kernel<true><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(L->params, L->feat, n, nseg,
                                                                                  L->identity, L->route, nullptr);
  } else {
    // the FP32 network, or the identity router (routed by the same kernel)
    route_keys_kernel<false><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(L->params, L->feat, n, nseg,
                                                                                   L->identity, L->route, nullptr);
  }
  seg_first_kernel<<<dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s>>>(L->route, n, nseg, L->first);
  seg_fit_kernel<T><<<dim3(fit_blocks(nseg)), dim3(kFitLanes), 0, s>>>(X, N, L->first, L->segs, nseg, nullptr,
                                                                         nullptr, nullptr);
  DS_HIP_CHECK(hipGetLastError());
  std::vector<SegFit> host(nseg);
  DS_HIP_CHECK(hipMemcpyAsync(host.data(), L->segs, size_t(nseg) * sizeof(SegFit), hipMemcpyDeviceToHost, s));
  std::vector<int32_t> firsts(nseg + 1);
  DS_HIP_CHECK(hipMemcpyAsync(firsts.data(), L->first, size_t(nseg + 1) * 4, hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipStreamSynchronize(s));
  int64_t max_err = 0;
  double wsum = 0, wcnt = 0;
  for (int32_t k = 0; k < nseg; ++k) {
    const SegFit& f = host[k];
    max_err = std::max<int64_t>(max_err, std::max(std::abs(int64_t(f.dmin)), std::abs(int64_t(f.dmax))));
    const int64_t width = std::min<int64_t>(int64_t(f.dmax) - f.dmin + 2, int64_t(f.hi) - f.lo + 1);
    const double keys = std::max(1, firsts[k + 1] - firsts[k]);
    wsum += keys * std::log2(static_cast<double>(std::max<int64_t>(1, width)));
    wcnt += keys;
  }
  L->max_err = max_err;
  L->mean_log2_window = wcnt > 0 ? wsum / wcnt : 0;
  // training scratch is no longer needed
  (void)hipFree(L->partial);
  (void)hipFree(L->route);
  (void)hipFree(L->first);
  L->partial = nullptr;
  L->route = nullptr;
  L->first = nullptr;
  h->info.model_bytes = learned_model_bytes(L);
  return DS_OK;
}

template <typename T>
ds_status learned_search_typed(ds_index* h, const void* z, int64_t M, int32_t* out, hipStream_t s) {
  LearnedModel* L = h->learned;
  LearnedArgs<T> a{};
  a.X = static_cast<const T*>(h->X);
  a.S = static_cast<const T*>(L->samples);
  a.params = L->params;
  a.segs = L->segs;
  a.steps = L->steps;
  a.grid = L->grid;
  a.log2g = L->log2g;
  a.fallbacks = L->fallbacks;
  a.z = static_cast<const T*>(z);
  a.out = out;
  a.M = M;
  a.X0d = h->X0;
  a.delta = L->delta;
  a.flo = L->flo;
  a.fscale = L->fscale;
  a.X0 = T(h->X0);
  a.XN = T(h->XN);
  a.N = static_cast<int32_t>(h->N);
  a.nseg = L->nseg;
  a.identity = L->identity;
  const bool table = L->router == kRouteTable && !L->identity;
  const int lds = static_cast<int>(int64_t(L->nseg) * (sizeof(SegFit) + (table ? 4 : 0)) +
                                   (table ? (int64_t(4) << L->log2g) : 0));
  // ds_tune.stage 1: each lane reads its own samples and block of X; else (0,
  // 2) the same samples, and the blocks of X read cooperatively by the quads
  const bool coop = !(h->tune_set && h->tune.stage == 1);
  auto kern = L->router == kRouteTable ? (coop ? learned_search_kernel<T, kRouteTable, true>
                                               : learned_search_kernel<T, kRouteTable, false>)
              : L->router == kRouteF16 ? (coop ? learned_search_kernel<T, kRouteF16, true>
                                               : learned_search_kernel<T, kRouteF16, false>)
                                      : (coop ? learned_search_kernel<T, kRouteF32, true>
                                              : learned_search_kernel<T, kRouteF32, false>);
  if (lds > 64 * 1024)
    DS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     lds));
  const int block = (h->tune_set && h->tune.block) ? h->tune.block : 1024;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  // six workgroups per resident slot, each restaging the tables: measured
  // 5-10 % faster than one persistent workgroup per slot on the clustered f64
  // array (the waves of a CU then start their groups at different times
  // rather than all routing, then all waiting on memory, together)
  const int64_t need = (M + block - 1) / block;
  int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(need, int64_t(6) * per_cu * num_cus())));
  if (h->tune_set && h->tune.grid) grid = h->tune.grid;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, a);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

}  // namespace

ds_status learned_build(ds_index* h, const ds_build_opts* o, hipStream_t s) {
  return h->dt == DS_F32 ? learned_build_typed<float>(h, o, s) : learned_build_typed<double>(h, o, s);
}

ds_status learned_search(ds_index* h, const void* z, int64_t M, int32_t* out, hipStream_t s) {
  if (!h->learned) return DS_ERR_ARG;
  return h->dt == DS_F32 ? learned_search_typed<float>(h, z, M, out, s)
                         : learned_search_typed<double>(h, z, M, out, s);
}

void learned_free(ds_index* h) {
  LearnedModel* L = h->learned;
  if (!L) return;
  for (void* p : {static_cast<void*>(L->params), static_cast<void*>(L->adam_m), static_cast<void*>(L->adam_v),
                  static_cast<void*>(L->partial), static_cast<void*>(L->loss_partial), static_cast<void*>(L->feat),
                  static_cast<void*>(L->route), static_cast<void*>(L->first), static_cast<void*>(L->segs),
                  static_cast<void*>(L->steps), static_cast<void*>(L->grid),
                  static_cast<void*>(L->samples), static_cast<void*>(L->fallbacks)})
    if (p) (void)hipFree(p);
  delete L;
  h->learned = nullptr;
}

// ---------------------------------------------------------------------------
// batched learned method: every learned array of a batch has its own model
// slot; all slots are initialised, trained (one launch per step for all of
// them), routed and fitted together, then searched by a persistent kernel
// that pulls the learned arrays' query tiles.

namespace {

constexpr int kBatchLearnBlock = 1024;

// LDS of the batched learned search: the current model's fits, router steps
// and router grid
int64_t batch_learned_lds(int32_t nseg, int32_t log2g) {
  return int64_t(nseg) * (kSegFitBytes + 4) + (int64_t(4) << log2g);
}

// A value equal in every lane of the wave, as a scalar (both 32-bit halves
// through readfirstlane).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint64_t u = static_cast<uint64_t>(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
  return static_cast<int64_t>((uint64_t(hi) << 32) | lo);
}

template <typename T, bool IDENT>
__global__ void __launch_bounds__(kBatchLearnBlock, 8) batch_learned_search_kernel(BatchLearned b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  // the current and the next tile (claimed by wave 0 while the others work),
  // with their 64-query group counters
  __shared__ int64_t s_tile[2];
  __shared__ int32_t s_k[2];
  __shared__ int32_t s_grp[2];
  const ArrMeta<T>* meta = static_cast<const ArrMeta<T>*>(b.meta);
  const int queue = blockIdx.x % kNumQueues;
  const int64_t total = b.tot->total_tiles;
  if (b.tot->learned_tiles == 0) return;  // no learned array
  const int lane = threadIdx.x & 63;
  const SegFit* segs = reinterpret_cast<const SegFit*>(smem);
  const float* steps = reinterpret_cast<const float*>(smem + int64_t(b.nseg) * kSegFitBytes);
  const uint32_t* grid = reinterpret_cast<const uint32_t*>(smem + int64_t(b.nseg) * (kSegFitBytes + 4));
  auto claim_tile = [&](int slot) {  // by wave 0
    // Each queue (one per XCD) owns a contiguous eighth of the tile order,
    // so the workgroups of one XCD share the few arrays of their range in
    // that XCD's L2; a queue whose range is done takes from the next ones.
    long long gl = total;
    if (threadIdx.x == 0) {
      for (int t = 0; t < kNumQueues; ++t) {
        const int qq = (queue + t) % kNumQueues;
        const int64_t lo = total * qq / kNumQueues, hi = total * (qq + 1) / kNumQueues;
        const int64_t li = atomicAdd(&b.tot->lqueue[qq], 1u);
        if (lo + li < hi) {
          gl = lo + li;
          break;
        }
      }
    }
    const int64_t g = __shfl(gl, 0, 64);
    // the last array whose first tile is <= g
    const int32_t k = (g < total) ? wave_last_le(b.tile_off, b.K, g) : -1;
    if (threadIdx.x == 0) {
      s_tile[slot] = g;
      s_k[slot] = k;
    }
  };
  if (threadIdx.x < 64) claim_tile(0);
  if (threadIdx.x == 0) s_grp[0] = 0;
  __syncthreads();
  int32_t cur = -1;
  for (int bf = 0;; bf ^= 1) {
    // the tile and its array are the same for the whole workgroup: read from
    // LDS into scalar registers, so the array's metadata is loaded once into
    // scalar registers too instead of into every lane's vector registers
    const int64_t g = uniform64(s_tile[bf]);
    const int32_t k = __builtin_amdgcn_readfirstlane(s_k[bf]);
    if (g >= total) break;
    const ArrMeta<T>& m = meta[k];
    const bool learned = m.method == DS_METHOD_LEARNED;
    const int32_t slot = m.slot;
    if (learned && slot != cur) {
      // every wave is past the previous tile's end barrier
      stage_bytes(smem, static_cast<const unsigned char*>(b.segs) + (int64_t)slot * b.nseg * kSegFitBytes,
                  int64_t(b.nseg) * kSegFitBytes);
      if (!IDENT) {
        stage_words(smem + int64_t(b.nseg) * kSegFitBytes, b.steps_tab + (int64_t)slot * b.nseg, b.nseg);
        stage_words(smem + int64_t(b.nseg) * (kSegFitBytes + 4), b.grid + ((int64_t)slot << b.log2g),
                    int64_t(1) << b.log2g);
      }
      __syncthreads();
      cur = slot;
    }
    if (threadIdx.x == 0) s_grp[bf ^ 1] = 0;
    if (threadIdx.x < 64) claim_tile(bf ^ 1);
    if (!learned) {
      __syncthreads();  // the next tile is claimed
      continue;
    }
    const LearnMeta lm = b.lmeta[slot];
    LearnedArgs<T> a{};
    a.X = static_cast<const T*>(b.X) + m.x_off;
    a.fallbacks = &b.tot->fallbacks;
    a.X0 = m.X0;
    a.XN = m.XN;
    a.N = m.N;
    a.nseg = b.nseg;
    const PackedArray<T> pa = packed_array<T>(static_cast<const T*>(b.X), static_cast<const T*>(b.samples), m.x_off,
                                              m.N, b.total_x);
    const int64_t q0 = m.q_off + (g - m.t_off) * b.tile;
    const int64_t q1 = std::min(m.q_end, q0 + b.tile);
    const int32_t ngrp = static_cast<int32_t>((q1 - q0 + 63) >> 6);
    const T* z = static_cast<const T*>(b.z);
    // waves claim the tile's 64-query groups one at a time, so they finish the
    // tile within one group of each other; the next group is claimed and its
    // queries loaded before the current one is worked on
    auto claim = [&]() {
      int32_t c = 0;
      if (lane == 0) c = atomicAdd(&s_grp[bf], 1);
      return __shfl(c, 0, 64);
    };
    // the query loads are unconditional (index clamped to the tile's last query,
    // q1 > q0), so the next group's load stays in flight while this one is worked on
    auto load_q = [&](int32_t grp) {
      return __builtin_nontemporal_load(z + std::min(q0 + int64_t(grp) * 64 + lane, q1 - 1));
    };
    int32_t gi = claim();
    T zq = load_q(gi);
    while (gi < ngrp) {
      const int64_t q = q0 + int64_t(gi) * 64 + lane;
      // the next group is claimed and its queries loaded once this group's
      // block loads are in flight (loads complete in order: issued earlier,
      // they would hold up the wait for the samples)
      int32_t gn;
      T z_next;
      auto next = [&]() {
        gn = claim();
        z_next = load_q(gn);
      };
      const float u = feature(static_cast<double>(zq), lm.X0, lm.delta, lm.flo, lm.fscale);
      const int32_t seg = IDENT ? segment_of(u, b.nseg) : grid_segment(u, steps, grid, b.log2g);
      int32_t L, U;
      query_window<T>(zq, seg, segs, &L, &U);
      bool certified;
      int32_t i = sample_search_packed<T, true>(zq, L, U, pa, &certified, next);
      if ((zq >= a.X0) && (zq < a.XN) && !certified) i = full_search_counted<T>(zq, a.X, a.N, a.fallbacks);
      i = (zq >= a.XN) ? a.N : i;
      i = (zq >= a.X0) ? i : -1;
      if (q < q1) __builtin_nontemporal_store(i, b.out + q);
      zq = z_next;
      gi = gn;
    }
    __syncthreads();  // every wave is done with this array's tables before they may change, and the next tile
                      // is claimed
  }
}

template <typename T>
ds_status batched_learned_build_typed(const BatchLearned& b, hipStream_t s) {
  const int K = b.K;
  // the samples were written by the build's pass over the keys (gaps_kernel)
  const T* X = static_cast<const T*>(b.X);
  if (!b.identity)
    init_params_kernel<T><<<dim3(K), dim3(64), 0, s>>>(b.params, b.adam_m, b.adam_v, X, 0, 0, 0, 0, 0, b.lmeta,
                                                       b.tot);
  // every step of every model's training in one launch (one workgroup per model)
  if (b.steps > 0)
    batched_train_kernel<T><<<dim3(K), dim3(kBatchTrainBlock), 0, s>>>(b.params, b.adam_m, b.adam_v, X, b.lmeta,
                                                                       b.tot, b.seed, b.steps, 2e-3f);
  DS_HIP_CHECK(hipGetLastError());
  if (b.identity) {
    route_first_kernel<true, T><<<dim3(kRouteBlocks, K), dim3(kRouteBlock), 0, s>>>(b.steps_tab, b.grid, b.log2g, X,
                                                                                   b.nseg, b.first, b.lmeta, b.tot);
  } else {
    // each trained network compiled to its step table and grid, then the keys routed through them
    // (each model's entries of `first` hold its probes until the keys are routed)
    const int32_t kp = probe_log2(b.nseg);
    router_probe_kernel<<<dim3((unsigned)(((1 << kp) + 1 + 255) / 256), K), dim3(256), 0, s>>>(b.params, b.nseg, kp,
                                                                                            b.first, b.tot);
    router_steps_kernel<<<dim3((unsigned)((b.nseg + 255) / 256), K), dim3(256), 0, s>>>(b.params, b.nseg, kp, b.first,
                                                                                      b.steps_tab, b.tot);
    router_table_kernel<<<dim3(K), dim3(kTableBlock), 0, s>>>(b.steps_tab, b.nseg, b.log2g, b.grid, b.tot);
    route_first_kernel<false, T><<<dim3(kRouteBlocks, K), dim3(kRouteBlock), route_first_lds(b.nseg, b.log2g), s>>>(
        b.steps_tab, b.grid, b.log2g, X, b.nseg, b.first, b.lmeta, b.tot);
  }
  seg_fit_kernel<T><<<dim3(fit_blocks(b.nseg), K), dim3(kFitLanes), 0, s>>>(
      X, 0, b.first, static_cast<SegFit*>(b.segs), b.nseg, b.lmeta, b.tot, b.longs);
  seg_fit_long_kernel<T><<<dim3(static_cast<unsigned>(2 * num_cus())), dim3(kLongBlock), 0, s>>>(
      X, b.first, static_cast<SegFit*>(b.segs), b.nseg, b.lmeta, b.tot, b.longs);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

template <typename T>
ds_status batched_learned_search_typed(const BatchLearned& b, hipStream_t s) {
  auto kern = b.identity ? batch_learned_search_kernel<T, true> : batch_learned_search_kernel<T, false>;
  const int lds = static_cast<int>(batch_learned_lds(b.nseg, b.log2g));
  if (lds > 64 * 1024)
    DS_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     lds));
  int per_cu = 0;
  const int block = kBatchLearnBlock;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int grid = per_cu * num_cus();
  grid = std::max(kNumQueues, grid / kNumQueues * kNumQueues);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, b);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

}  // namespace

// the batched search kernel's own LDS (tile claims) is kept out of the budget
// The batched search's grid: small enough that two workgroups fit one CU's LDS
// (fits, steps, grid and about 1 KiB of static LDS each) when the fits and
// steps leave room for a grid of at least 64 cells, else as large as one
// workgroup allows.
int32_t batch_grid_log2(int32_t nseg) {
  const int64_t half = kLearnLdsBudget / 2 - 1024;
  if (int64_t(nseg) * (int64_t(sizeof(SegFit)) + 4) + (int64_t(4) << 6) <= half) return grid_log2(nseg, half);
  return grid_log2(nseg, kLearnLdsBudget - 1024);
}

ds_status batched_learned_build(const BatchLearned& b, int dtype, hipStream_t s) {
  if (b.nseg < 1 || b.nseg > kBatchMaxSegments || batch_learned_lds(b.nseg, b.log2g) > kLearnLdsBudget - 1024)
    return DS_ERR_ARG;
  return dtype == DS_F32 ? batched_learned_build_typed<float>(b, s) : batched_learned_build_typed<double>(b, s);
}

ds_status batched_learned_search(const BatchLearned& b, int dtype, hipStream_t s) {
  return dtype == DS_F32 ? batched_learned_search_typed<float>(b, s) : batched_learned_search_typed<double>(b, s);
}


void learned_fill_info(const ds_index* h, ds_info_t* in) {
  const LearnedModel* L = h->learned;
  if (!L) return;
  in->model_bytes = learned_model_bytes(L);
  in->x_bytes += L->nsamples * int64_t(h->dt == DS_F32 ? 4 : 8);  // the search's sample array
  in->max_err = L->max_err;
  in->mean_log2_window = L->mean_log2_window;
}

ds_status learned_fallbacks(const ds_index* h, uint64_t* count) {
  const LearnedModel* L = h->learned;
  unsigned long long f = 0;
  if (L && L->fallbacks) DS_HIP_CHECK(hipMemcpy(&f, L->fallbacks, 8, hipMemcpyDeviceToHost));
  *count = f;
  return DS_OK;
}

}  // namespace ds

extern "C" {

ds_status ds_learned_grad(const float* params_dev, const float* u_dev, const float* t_dev, int32_t batch,
                          float* grad_dev, float* loss_dev, hipStream_t s) {
  if (!params_dev || !u_dev || !t_dev || !grad_dev || batch < 1) return DS_ERR_ARG;
  const int32_t n_parts = (batch + ds::kTrainBlock - 1) / ds::kTrainBlock;
  float* partial = nullptr;
  float* lp = nullptr;
  if (hipMalloc(&partial, size_t(n_parts) * ds::kParams * 4) != hipSuccess) return DS_ERR_OOM;
  if (hipMalloc(&lp, size_t(n_parts) * 4) != hipSuccess) {
    (void)hipFree(partial);
    return DS_ERR_OOM;
  }
  ds::train_step_kernel<<<dim3(n_parts), dim3(ds::kTrainBlock), 0, s>>>(params_dev, nullptr, 1, 0, 0, batch, u_dev,
                                                                        t_dev, partial, lp);
  ds::adam_kernel<<<dim3(1), dim3(1024), 0, s>>>(nullptr, nullptr, nullptr, partial, n_parts, 0, 1, grad_dev);
  if (loss_dev) ds::sum_kernel<<<1, 64, 0, s>>>(lp, n_parts, loss_dev);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(partial);
  (void)hipFree(lp);
  return e == hipSuccess ? DS_OK : DS_ERR_HIP;
}

ds_status ds_learned_forward(const float* params_dev, const float* u_dev, int64_t n, int32_t fp16_router, float* y_dev,
                             hipStream_t s) {
  if (!params_dev || !u_dev || !y_dev || n < 0) return DS_ERR_ARG;
  if (n == 0) return DS_OK;
  int32_t* route = nullptr;
  if (hipMalloc(&route, size_t(n) * 4) != hipSuccess) return DS_ERR_OOM;
  if (fp16_router)
    ds::route_keys_kernel<true><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(params_dev, u_dev, n, 4096, 0,
                                                                                      route, y_dev);
  else
    ds::route_keys_kernel<false><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(params_dev, u_dev, n, 4096, 0,
                                                                                       route, y_dev);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(route);
  return e == hipSuccess ? DS_OK : DS_ERR_HIP;
}

ds_status ds_learned_route(ds_handle h, const float* u_dev, int64_t n, int32_t mode, int32_t* seg_dev,
                           hipStream_t s) {
  if (!h || !h->learned || !u_dev || !seg_dev || n < 0 || mode < 0 || mode > 2) return DS_ERR_ARG;
  if (n == 0) return DS_OK;
  const ds::LearnedModel* L = h->learned;
  const bool table = L->router == ds::kRouteTable && !L->identity;
  const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 1 << 16));
  if (mode == 1 || !table) {
    // the network evaluated (FP16 inputs for a handle with the FP16-input router, unless mode 1)
    if (mode != 1 && L->router == ds::kRouteF16)
      ds::route_keys_kernel<true><<<dim3(blocks), dim3(256), 0, s>>>(L->params, u_dev, n, L->nseg, L->identity,
                                                                     seg_dev, nullptr);
    else
      ds::route_keys_kernel<false><<<dim3(blocks), dim3(256), 0, s>>>(L->params, u_dev, n, L->nseg, L->identity,
                                                                      seg_dev, nullptr);
  } else if (mode == 0) {
    ds::route_query_table_kernel<<<dim3(std::min(blocks, 4096u)), dim3(256), 0, s>>>(L->steps, L->grid, L->log2g,
                                                                                     u_dev, n, seg_dev);
  } else {
    ds::route_keys_table_kernel<<<dim3(std::min(blocks, 4096u)), dim3(256), 0, s>>>(L->steps, u_dev, n, L->nseg,
                                                                                     seg_dev);
  }
  DS_HIP_CHECK(hipGetLastError());
  DS_HIP_CHECK(hipStreamSynchronize(s));
  return DS_OK;
}

ds_status ds_learned_model(ds_handle h, float* params_host, int32_t capacity, uint64_t* fallbacks_host,
                           hipStream_t s) {
  if (!h || !h->learned) return DS_ERR_ARG;
  ds::LearnedModel* L = h->learned;
  if (params_host) {
    if (capacity < ds::kParams) return DS_ERR_ARG;
    DS_HIP_CHECK(hipMemcpyAsync(params_host, L->params, ds::kParams * 4, hipMemcpyDeviceToHost, s));
  }
  if (fallbacks_host) {
    unsigned long long f = 0;
    DS_HIP_CHECK(hipMemcpyAsync(&f, L->fallbacks, 8, hipMemcpyDeviceToHost, s));
    DS_HIP_CHECK(hipStreamSynchronize(s));
    *fallbacks_host = f;
  }
  DS_HIP_CHECK(hipStreamSynchronize(s));
  return DS_OK;
}

}  // extern "C"
