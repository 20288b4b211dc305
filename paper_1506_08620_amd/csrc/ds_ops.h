// Device-side building blocks shared by the single-array and the batched
// search kernels: LDS staging, the query stream loop and the per-query
// operators of every method and layout.
#pragma once

#include <algorithm>
#include <type_traits>

#include "ds_internal.h"

namespace ds {

template <typename T>
using vec4 = T __attribute__((ext_vector_type(4)));
using ivec4 = int __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int64_t round16(int64_t b) { return (b + 15) & ~int64_t(15); }

// LDS offsets of the RANKCODE layout staged as bits | counts | codes
__host__ __device__ constexpr int64_t rankcode_offsets(int64_t nW, int64_t n_code_bytes, int64_t* base_off,
                                                       int64_t* code_off) {
  *base_off = round16(nW * 8);
  *code_off = *base_off + round16(nW * 4);
  return *code_off + round16(n_code_bytes);
}

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

// An operator with a Gathered type splits a query into three steps that
// stream_queries runs over all of a lane's queries in turn, so that the loads
// of each step are in flight together:
//   g = gather(z)             the table load (plus what the next step needs
//                             from z);
//   i = decide(z, g, &t)      the result, unless t >= 0: then the result is
//                             t - 1 + [z >= X_t] (the rare undecided compare,
//                             always for an in-domain z).
template <class Op, class = void>
struct has_gather : std::false_type {};
template <class Op>
struct has_gather<Op, std::void_t<typename Op::Gathered>> : std::true_type {};

// Vectors of W queries and W results: a lane loads and stores W consecutive
// values with one 16-byte (f32: 4 values) or 16-byte (f64: 2 values) access,
// so one load instruction of a wave covers 1 KiB of contiguous queries and the
// L1 asks the L2 for whole lines (a 32-byte f64 vector per lane would split
// into two 16-byte loads of which each touches every line at half of it,
// doubling the requests of the query stream).
template <typename T, int W>
using vecw = T __attribute__((ext_vector_type(W)));
template <int W>
using ivecw = int __attribute__((ext_vector_type(W)));

// The VEC loop for an operator with a Gathered type: gather, decide and the
// undecided compares each run over all U W queries of a lane in turn, so the
// loads of a step are in flight together.  A vector index past the end is
// clamped to the last vector: every load is in bounds and unconditional
// (which keeps the loop free of branches, so the compiler's waits cover only
// the loads a step needs), and only the stores are guarded.  (Prefetching the
// next iteration's queries measured no faster on MI355X and costs registers.)
template <typename T, int W, int U, class Op>
__device__ __forceinline__ void stream_gathered(const vecw<T, W>* __restrict__ zv, ivecw<W>* __restrict__ ov,
                                                int64_t nvec, const Op& op) {
  const int64_t B = blockDim.x;
  const int64_t step = (int64_t)gridDim.x * B * U;
  const int64_t last = nvec - 1;
  for (int64_t base = (int64_t)blockIdx.x * B * U + threadIdx.x; base < nvec; base += step) {
    vecw<T, W> q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = __builtin_nontemporal_load(zv + std::min<int64_t>(base + u * B, last));
    typename Op::Gathered g[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int l = 0; l < W; ++l) g[u][l] = op.gather(q[u][l]);
    }
    int32_t r[U][W], t[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int l = 0; l < W; ++l) r[u][l] = op.decide(q[u][l], g[u][l], &t[u][l]);
    }
    T x[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int l = 0; l < W; ++l) {
        x[u][l] = T(0);
        if (t[u][l] >= 0) x[u][l] = op.Xg[t[u][l]];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (base + u * B < nvec) {
        ivecw<W> o;
#pragma unroll
        for (int l = 0; l < W; ++l) o[l] = (t[u][l] >= 0) ? t[u][l] - 1 + (q[u][l] >= x[u][l] ? 1 : 0) : r[u][l];
        __builtin_nontemporal_store(o, ov + base + u * B);
      }
    }
  }
}

// Streams M queries through op.  VEC: z is aligned for 4-element vectors and
// out for 16 bytes; a lane handles 4U queries per iteration (f32: U vectors of
// 4, f64: 2U vectors of 2), so several independent gathers are in flight.
template <typename T, int U, bool VEC, class Op>
__device__ __forceinline__ void stream_queries(const T* __restrict__ z, int32_t* __restrict__ out, int64_t M,
                                               const Op& op) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (VEC) {
    constexpr int W = 16 / int(sizeof(T));  // values per 16-byte vector
    constexpr int UV = 4 * U / W;           // vectors per lane and iteration
    const int64_t nvec = M / W;
    const vecw<T, W>* zv = reinterpret_cast<const vecw<T, W>*>(z);
    ivecw<W>* ov = reinterpret_cast<ivecw<W>*>(out);
    if constexpr (has_gather<Op>::value) {
      stream_gathered<T, W, UV>(zv, ov, nvec, op);
    } else {
      const int64_t step = (int64_t)gridDim.x * blockDim.x * UV;
      for (int64_t base = (int64_t)blockIdx.x * blockDim.x * UV + threadIdx.x; base < nvec; base += step) {
        vecw<T, W> q[UV];
#pragma unroll
        for (int u = 0; u < UV; ++u) {
          const int64_t v = base + (int64_t)u * blockDim.x;
          if (v < nvec) q[u] = __builtin_nontemporal_load(zv + v);
        }
#pragma unroll
        for (int u = 0; u < UV; ++u) {
          const int64_t v = base + (int64_t)u * blockDim.x;
          if (v < nvec) {
            ivecw<W> r;
#pragma unroll
            for (int l = 0; l < W; ++l) r[l] = op(q[u][l]);
            __builtin_nontemporal_store(r, ov + v);
          }
        }
      }
    }
    const int64_t t = nvec * W + gtid;
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

// The gap-q search of Sec. 4.7 (eq. (index2); algorithm DirectGap2 for
// q = 2): t = K_j with K_j = max{i : f(X_i) <= j}, i = t - sum_{k<q}
// [z < X_{t-k}].  Xt points at X_0 with at least Q - 1 copies of X_0 before
// it, the left padding the algorithm needs for t < q - 1 (z >= X_0 there, so
// those compares are false).  Q bounds q; the compares are predicated, and
// independent, so their loads are in flight together.  NaN and z < X_0 give
// -1; z >= X_N reaches K_R = N with every compare false.
template <typename T, int FORM, int Q>
struct GapOp {
  const T* Xt;
  const int32_t* Kb;  // points at K_0
  T H, W, X0, vlo, vhi;
  int32_t q;
  __device__ __forceinline__ int32_t operator()(T z) const {
    T v = grid_value<T, FORM>(z, H, W, X0);
    v = std::fmin(std::fmax(v, vlo), vhi);
    const int32_t j = static_cast<int32_t>(std::floor(v));
    const int32_t t = Kb[j];
    int32_t i = t;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (k < q) i -= (z < Xt[t - k]) ? 1 : 0;
    }
    return (z >= X0) ? i : -1;
  }
};

// GAPCODE layout of the gap-q variant (Sec. 4.7) for q <= 15: the grid keeps
// at most q keys per cell, so a cell is described by its key count (CB = 2
// bits for q <= 3, 4 bits for q <= 15; 64 / CB cells per 64-bit word, with
// the count of the keys in earlier cells per word) and each key by the
// RANKCODE position code.  With e = f(z) - jmin and A the first key of cell e
// (the word's count plus its counts below e), keys before A lie in earlier
// cells, so below z, and keys after the cell lie above it: the result is
// A - 1 plus the number of the cell's keys at or below z (at most QMAX), each
// decided from the codes as in RankCodeOp (X read on an undecided tie).
template <int CB>
__device__ __forceinline__ int32_t sum_counts(uint64_t m) {
  if constexpr (CB == 2) {
    return __popcll(m & 0x5555555555555555ull) + 2 * __popcll(m & 0xAAAAAAAAAAAAAAAAull);
  } else {
    return __popcll(m & 0x1111111111111111ull) + 2 * __popcll(m & 0x2222222222222222ull) +
           4 * __popcll(m & 0x4444444444444444ull) + 8 * __popcll(m & 0x8888888888888888ull);
  }
}

template <typename T, int FORM, int CB, int QMAX>
struct GapCodeOp {
  static constexpr int kCells = 64 / CB;            // cells per word
  static constexpr int kLog2Cells = CB == 2 ? 5 : 4;
  static constexpr int kMask = (1 << CB) - 1;
  const uint64_t* counts;
  const uint32_t* base;
  const uint16_t* code;
  const T* Xg;  // X_0 .. X_N in global memory
  T H, W, X0, vlo, vhi, XN;
  int32_t jmin, N;
  __device__ __forceinline__ int32_t operator()(T z) const {
    const T v = grid_value<T, FORM>(z, H, W, X0);
    const T jf = std::floor(std::fmin(std::fmax(v, vlo), vhi));
    const int32_t e = static_cast<int32_t>(jf) - jmin;
    const uint64_t word = counts[e >> kLog2Cells];
    const uint32_t sh = (static_cast<uint32_t>(e) & (kCells - 1)) * CB;
    const uint64_t low = word & ((uint64_t(1) << sh) - 1);
    const int32_t A = static_cast<int32_t>(base[e >> kLog2Cells]) + sum_counts<CB>(low);
    const int32_t c = static_cast<int32_t>((word >> sh) & kMask);  // at most q <= QMAX
    const T cz = cell_code<T>(v, jf);
    int32_t i = A - 1;
#pragma unroll
    for (int k = 0; k < QMAX; ++k) {
      if (k < c) {
        const int32_t cx = code[A + k];
        const T cxp = static_cast<T>(cx >> 1);
        const bool first = cx & 1;
        const bool up = cz > cxp || (cz == cxp && first);
        const bool tie = cz == cxp && !first;
        i += (up || (tie && z >= Xg[A + k])) ? 1 : 0;
      }
    }
    i = (z >= XN) ? N : i;
    return (z >= X0) ? i : -1;
  }
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

// bit 4n + 3 set for each nonzero nibble n: the low three bits of a nibble
// plus 7 carry into its top bit exactly when they are not all zero, and never
// out of the nibble
__device__ __forceinline__ uint32_t nonzero_nibbles32(uint32_t x) {
  return (((x & 0x77777777u) + 0x77777777u) | x) & 0x88888888u;
}

// NIBBLE layout through L1/L2: the chunk of the query's cell is one 16-byte
// gather holding the running count, the occupancy and the bin codes of 24
// cells, so a query touches one cache line of the table (plus X_t when the
// bins tie).  gather() also does all the floating-point work on z and packs
// it into one word (cell in the chunk, bin of z, below X_0), so decide() is
// integer-only.
template <typename T, int FORM>
struct NibbleOp {
  struct Gathered {
    uint4 q;
    uint32_t p;
  };
  static constexpr uint32_t kBelow = 1u << 9;
  const NibChunk* ch;
  const T* Xg;
  T H, W, X0, vlo, vhi, XN;
  int32_t jmin, N;
  const uint4* pre = nullptr;  // the first n_pre chunks again, in LDS
  uint32_t n_pre = 0;
  __device__ __forceinline__ Gathered gather(T z) const {
    const T v = grid_value<T, FORM>(z, H, W, X0);
    const T jf = std::floor(std::fmin(std::fmax(v, vlo), vhi));
    const uint32_t e = static_cast<uint32_t>(static_cast<int32_t>(jf) - jmin);
    const uint32_t k = e / kNibCells;
    Gathered g;
    if (k < n_pre)
      g.q = pre[k];  // an LDS read instead of an L2 access
    else
      g.q = reinterpret_cast<const uint4*>(ch)[k];  // one dwordx4 gather
    // the bin of z (clamped at 0 for z below X_0 and NaN, whose result is -1 anyway)
    const uint32_t bz = static_cast<uint32_t>(std::fmax(cell_bin(v, jf), T(0)));
    g.p = (e - k * kNibCells) | (bz << 5) | (z >= X0 ? 0u : kBelow);
    return g;
  }
  __device__ __forceinline__ int32_t decide(T, const Gathered& g, int32_t* tie) const {
    const uint32_t c = g.p & 31u, cz = (g.p >> 5) & 15u;
    const uint32_t wi = c >> 3, sh = (c & 7u) << 2;
    const uint32_t before = (1u << sh) - 1u;  // nibbles before c in its word
    const uint32_t m0 = wi > 0 ? ~0u : before;
    const uint32_t m1 = wi > 1 ? ~0u : (wi == 1 ? before : 0u);
    const uint32_t m2 = wi == 2 ? before : 0u;
    const uint32_t rank = __popc(nonzero_nibbles32(g.q.x) & m0) + __popc(nonzero_nibbles32(g.q.y) & m1) +
                          __popc(nonzero_nibbles32(g.q.z) & m2);
    const uint32_t w = wi == 0 ? g.q.x : (wi == 1 ? g.q.y : g.q.z);
    const uint32_t nib = (w >> sh) & 15u;
    const int32_t t = static_cast<int32_t>(g.q.w + rank);
    bool up, eq;
    if constexpr (NibCode<T>::kFlag) {
      const uint32_t cx = (nib - 1) >> 1;
      const bool first = (nib - 1) & 1u;
      up = cz > cx || (cz == cx && first);
      eq = cz == cx && !first;
    } else {
      const uint32_t cx = nib - 1;
      up = cz > cx;
      eq = cz == cx;
    }
    // z at or above X_N needs no case of its own: it lies in the last cell (or
    // is clamped to it), which holds X_N = X_t, with a bin >= the bin of X_N,
    // so the codes (or the compare with X_N) give t = N
    const bool occupied = nib != 0;
    const bool below = (g.p & kBelow) != 0;
    *tie = (occupied && eq && !below) ? t : -1;
    const int32_t i = (occupied && up) ? t : t - 1;
    return below ? -1 : i;
  }
  __device__ __forceinline__ int32_t operator()(T z) const {
    int32_t t;
    const int32_t i = decide(z, gather(z), &t);
    return (t >= 0) ? t - 1 + (z >= Xg[t] ? 1 : 0) : i;
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
