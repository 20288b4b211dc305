// Device-side building blocks shared by the single-array and the batched
// search kernels: LDS staging, the query stream loop and the per-query
// operators of every method and layout.
#pragma once

#include "ds_internal.h"

namespace ds {

template <typename T>
using vec4 = T __attribute__((ext_vector_type(4)));
using ivec4 = int __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int64_t round16(int64_t b) { return (b + 15) & ~int64_t(15); }

// Copy n_bytes (multiple of 4) from global to LDS with 16-byte moves, four
// loads in flight per lane before the stores.
__device__ __forceinline__ void stage_bytes(unsigned char* __restrict__ dst, const unsigned char* __restrict__ src,
                                            int64_t n_bytes) {
  const int64_t n16 = n_bytes >> 4;
  const int4* s4 = reinterpret_cast<const int4*>(src);
  int4* d4 = reinterpret_cast<int4*>(dst);
  const int64_t B = blockDim.x;
  int64_t k = threadIdx.x;
  for (; k + 3 * B < n16; k += 4 * B) {
    const int4 a = s4[k], b = s4[k + B], c = s4[k + 2 * B], d = s4[k + 3 * B];
    d4[k] = a;
    d4[k + B] = b;
    d4[k + 2 * B] = c;
    d4[k + 3 * B] = d;
  }
  for (; k < n16; k += B) d4[k] = s4[k];
  const int64_t rem = n_bytes - (n16 << 4);  // 0, 4, 8 or 12
  if ((int64_t)threadIdx.x < (rem >> 2)) {
    reinterpret_cast<int*>(dst + (n16 << 4))[threadIdx.x] = reinterpret_cast<const int*>(src + (n16 << 4))[threadIdx.x];
  }
}

// Streams M queries through op.  VEC: z and out are aligned for 4-element
// vector access; U vectors per lane per iteration keep several independent
// gathers in flight.
template <typename T, int U, bool VEC, class Op>
__device__ __forceinline__ void stream_queries(const T* __restrict__ z, int32_t* __restrict__ out, int64_t M,
                                               const Op& op) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (VEC) {
    const int64_t nvec = M >> 2;
    const vec4<T>* zv = reinterpret_cast<const vec4<T>*>(z);
    ivec4* ov = reinterpret_cast<ivec4*>(out);
    const int64_t step = (int64_t)gridDim.x * blockDim.x * U;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x * U + threadIdx.x; base < nvec; base += step) {
      vec4<T> q[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t v = base + (int64_t)u * blockDim.x;
        if (v < nvec) q[u] = __builtin_nontemporal_load(zv + v);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t v = base + (int64_t)u * blockDim.x;
        if (v < nvec) {
          ivec4 r;
          r.x = op(q[u].x);
          r.y = op(q[u].y);
          r.z = op(q[u].z);
          r.w = op(q[u].w);
          __builtin_nontemporal_store(r, ov + v);
        }
      }
    }
    const int64_t t = (nvec << 2) + gtid;
    if (t < M) out[t] = op(z[t]);
  } else {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = gtid; k < M; k += step) out[k] = op(z[k]);
  }
}

template <typename T, int FORM>
struct DirectOp {
  const T* X;
  const int32_t* Kb;  // points at K_0
  T H, W, X0, vlo, vhi;
  __device__ __forceinline__ int32_t operator()(T z) const { return direct_one<T, FORM>(z, X, Kb, H, W, X0, vlo, vhi); }
};

// RANKCODE layout (see ds.h).  With e = f(z) - jmin, K_j is the running count
// of the 64-cell word plus the popcount of the word's lower bits.  A cell
// without an X_i gives i = K_j - 1 directly (every X_i before it is below z
// and X_{K_j} is above it).  A cell holding X_t (t = K_j) compares the position
// codes of z and X_t: a strict difference decides, equal codes decide when X_t
// is the first float of its code class, and only the remaining case reads X_t.
// The last two lines give -1 below X_0 (and for NaN) and N at or above X_N.
template <typename T, int FORM, bool INTERLEAVED, typename CodeT = uint16_t>
struct RankCodeOp {
  static constexpr int kPosBits = sizeof(CodeT) * 8 - 1;
  const uint64_t* bits;
  const uint32_t* base;
  const RcWord* w16;  // INTERLEAVED: (bits, base) of a word in one 16-byte load
  const CodeT* code;
  const T* Xg;  // X in global memory, for the rare undecided compare
  T H, W, X0, vlo, vhi, XN;
  int32_t jmin, N;
  __device__ __forceinline__ int32_t operator()(T z) const {
    const T v = grid_value<T, FORM>(z, H, W, X0);
    const T jf = std::floor(std::fmin(std::fmax(v, vlo), vhi));
    const int32_t e = static_cast<int32_t>(jf) - jmin;
    const int32_t w = e >> 6;
    const uint32_t b = static_cast<uint32_t>(e) & 63u;
    uint64_t word;
    uint32_t wbase;
    if constexpr (INTERLEAVED) {
      const RcWord rw = w16[w];
      word = rw.bits;
      wbase = rw.base;
    } else {
      word = bits[w];
      wbase = base[w];
    }
    const int32_t t = static_cast<int32_t>(wbase) + __popcll(word & ((uint64_t(1) << b) - 1));
    const bool occupied = (word >> b) & 1u;
    const int32_t c = occupied ? code[t] : 0;  // only occupied cells need the code
    const T cz = cell_code<T, kPosBits>(v, jf);
    const T cx = static_cast<T>(c >> 1);
    const bool first = c & 1;
    int32_t i = t - 1;
    if (occupied) {
      if (cz > cx || (cz == cx && first)) {
        i = t;
      } else if (cz == cx) {
        i = t - 1 + (z >= Xg[t] ? 1 : 0);
      }
    }
    i = (z >= XN) ? N : i;
    return (z >= X0) ? i : -1;
  }
};

// PAIRS layout (Sec. 4.8, algorithm DirectCache): one aligned load gives
// (K_j, X_{K_j}).
template <typename T, int FORM>
struct PairsOp {
  const CachePair<T>* pb;  // points at the pair of cell 0
  T H, W, X0, vlo, vhi;
  __device__ __forceinline__ int32_t operator()(T z) const {
    T v = grid_value<T, FORM>(z, H, W, X0);
    v = std::fmin(std::fmax(v, vlo), vhi);
    const int32_t j = (FORM == DS_FORM_FMA) ? static_cast<int32_t>(std::floor(v)) : static_cast<int32_t>(v);
    const CachePair<T> p = pb[j];
    return p.t - 1 + (z >= p.x ? 1 : 0);
  }
};


// Sec. 3.2.1: i = 0; for k = P, P/2, ..., 1: r = i|k; if z >= Xp_r then i = r.
// Xp is X padded with X_N to 2P entries.  The last two lines extend the
// result to out-of-domain z: min(i, N) gives N at or above X_N, and the
// subtraction gives -1 below X_0 or for NaN.
template <typename T>
struct LeadbitOp {
  const T* Xp;
  int32_t P, N;
  __device__ __forceinline__ int32_t operator()(T z) const {
    int32_t i = 0;
    for (int32_t k = P; k > 0; k >>= 1) {
      const int32_t r = i | k;
      i = (z >= Xp[r]) ? r : i;
    }
    i = i < N ? i : N;
    return i - (z >= Xp[0] ? 0 : 1);
  }
};

// Sec. 3.3 with the size update read as S <- S - H: i = 0; if z >= X_F then
// i = F; J times: H = floor(S/2), F = i + H, if z >= X_F then i = F, S -= H.
// It never reads past X_N and returns N at or above X_N; below X_0 (and NaN)
// the final subtraction gives -1.
template <typename T>
struct OffsetOp {
  const T* X;
  int32_t F0, S0, J;
  __device__ __forceinline__ int32_t operator()(T z) const {
    int32_t i = (z >= X[F0]) ? F0 : 0;
    int32_t S = S0;
    for (int32_t j = 0; j < J; ++j) {
      const int32_t h = S >> 1;
      const int32_t f = i + h;
      i = (z >= X[f]) ? f : i;
      S -= h;
    }
    return i - (z >= X[0] ? 0 : 1);
  }
};

}  // namespace ds
