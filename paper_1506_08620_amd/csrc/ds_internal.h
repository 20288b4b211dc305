// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "ds.h"

namespace ds {

constexpr int kLdsBytesPerCU = 160 * 1024;     // gfx950 LDS per compute unit (and per workgroup)
constexpr int64_t kL2BytesPerXcd = int64_t(4) << 20;  // MI355X L2 per XCD
constexpr int64_t kDefaultTableCap = int64_t(4) << 30;
constexpr double kTwoPowQ = 2147483648.0;       // Q = 31: grid indices are int32
constexpr int kMaxGapQ = 16;                     // largest q of the gap-q variant
constexpr int kEytLdsBytes = 64 * 1024;          // LDS for the top levels of the Eytzinger tree

// levels of the Eytzinger tree whose nodes (plus the unused slot 0) fit kEytLdsBytes
template <typename T>
__host__ __device__ inline int eyt_lds_levels(int L) {
  int t = 0;
  while (t < L && (int64_t(2) << t) * int64_t(sizeof(T)) <= kEytLdsBytes) ++t;
  return t;
}

#define DS_HIP_CHECK(expr)                                                              \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      std::fprintf(stderr, "ds: %s failed: %s (%s:%d)\n", #expr, hipGetErrorString(e_), \
                   __FILE__, __LINE__);                                                  \
      return DS_ERR_HIP;                                                                 \
    }                                                                                    \
  } while (0)

// ---------------------------------------------------------------------------
// The grid map f of the Direct method, shared by build and search so that
// both evaluate exactly the same floating-point expression.
//   subtraction form (Sec. 4.1, eq. (function)):  v = m(H * m(x - X_0))
//   FMA form (Sec. 4.9, eq. (fma)):               v = fma(H, x, -W), W = m(H X_0)
// f(x) = floor(v).  No contraction is allowed in either form (the library is
// built with -ffp-contract=off); the FMA form uses an explicit fma.
template <typename T, int FORM>
__host__ __device__ __forceinline__ T grid_value(T x, T H, T W, T X0) {
  if constexpr (FORM == DS_FORM_FMA) {
    return std::fma(H, x, -W);
  } else {
    T d = x - X0;
    return H * d;
  }
}

template <typename T, int FORM>
__host__ __device__ __forceinline__ T grid_floor(T x, T H, T W, T X0) {
  return std::floor(grid_value<T, FORM>(x, H, W, X0));
}

// Direct search of one query (Sec. 4.2, algorithm Direct) on tables that may
// live in LDS or in global memory.  Kb points at K_0 (entry jmin is Kb[jmin]).
// The clamp of v to [jmin, R] is done on the float: maxNum(NaN, jmin) = jmin,
// so NaN and z < X_0 land on K_jmin = 0, z >= X_N lands on K_R = N, and the
// float->int conversion is always defined.  The fix step is written
// i = t - 1 + [z >= X_t]: equal to the paper's "t, minus one if z < X_t" for
// every non-NaN z, and -1 for NaN.
template <typename T, int FORM>
__device__ __forceinline__ int32_t direct_one(T z, const T* __restrict__ X, const int32_t* __restrict__ Kb, T H,
                                              T W, T X0, T vlo, T vhi) {
  T v = grid_value<T, FORM>(z, H, W, X0);
  v = std::fmin(std::fmax(v, vlo), vhi);
  int32_t j;
  if constexpr (FORM == DS_FORM_FMA) {
    j = static_cast<int32_t>(std::floor(v));
  } else {
    j = static_cast<int32_t>(v);  // v >= 0 here, truncation is the floor
  }
  const int32_t t = Kb[j];
  const T x = X[t];
  return t - 1 + (z >= x ? 1 : 0);
}

// Position code of a value inside its grid cell: the fraction v - floor(v) in
// units of 2^-B, capped at 2^B - 1 (B = 15 for the 16-bit codes, 7 for the
// 8-bit ones; one more bit of each code is the first-of-class flag).  It is a
// non-decreasing function of v within a cell, computed identically by the
// build and the search, so a strict difference between the codes of z and of
// X_t orders z and X_t.
template <typename T, int B = 15>
__host__ __device__ __forceinline__ T cell_code(T v, T jf) {
  return std::fmin(std::floor((v - jf) * T(1 << B)), T((1 << B) - 1));
}

// the cache-friendly pair of Sec. 4.8: (K_j, X_{K_j}) in one aligned load
template <typename T>
struct alignas(2 * sizeof(T)) CachePair;
template <>
struct alignas(8) CachePair<float> {
  int32_t t;
  float x;
};
template <>
struct alignas(16) CachePair<double> {
  int32_t t;
  int32_t pad;
  double x;
};

// one 64-cell word of the RANKCODE bitmap with its running count, for the
// layout read through L2 (one 16-byte gather per query)
struct alignas(16) RcWord {
  uint64_t bits;
  uint32_t base;
  uint32_t pad;
};

// NIBBLE layout: one 16-byte chunk per 24 grid cells, read with one gather.
// base counts the X_i of earlier cells (it comes last, so that the first two
// code words form an aligned 64-bit register pair); nibble c % 8 of
// nib[c / 8] describes cell 24 k + c: 0 when it holds no X_i, else a code of
// the position of its X_i inside the cell (NibCode).  The rank of a cell is
// base plus the nonzero nibbles before it.
constexpr int kNibCells = 24;
// NIBBLE chunks that a workgroup keeps in LDS when the layout is read through L2
constexpr int64_t kNibPrefixChunks = (156 * 1024) / 16;
// chunks of the NIBBLE layout for nK grid cells
__host__ __device__ constexpr int64_t nibble_chunks(int64_t nK) { return (nK + kNibCells - 1) / kNibCells; }
struct alignas(16) NibChunk {
  uint32_t nib[3];
  uint32_t base;
};

// The 15 nonzero nibble values.  f32 cells hold few floats, so a code keeps
// 7 bins of the position and the first-of-class flag (value 1 + 2 bin +
// first): a query in the bin of X_t that is the first float of its bin is at
// or above X_t.  f64 cells hold very many floats and the flag would almost
// never be set, so all 15 values are bins (value 1 + bin).
template <typename T>
struct NibCode {
  static constexpr bool kFlag = sizeof(T) == 4;
  static constexpr int kBins = kFlag ? 7 : 15;
};

// Bin of a value inside its grid cell: kBins equal bins of the fraction
// v - floor(v), capped at kBins - 1.  Non-decreasing in v within a cell and
// computed identically by the build and the search, like cell_code.
template <typename T>
__host__ __device__ __forceinline__ T cell_bin(T v, T jf) {
  constexpr int B = NibCode<T>::kBins;
  return std::fmin(std::floor((v - jf) * T(B)), T(B - 1));
}

template <typename T>
struct DirectArgs {
  const T* X;         // N+1 values (global)
  const int32_t* K;   // R - jmin + 1 entries (global), K[0] = K_jmin
  T H, W, X0;
  T vlo, vhi;         // jmin and R as T (exact)
  T XN;               // X_N
  int32_t jmin;
  int32_t nK;         // R - jmin + 1
  int32_t nX;         // N + 1
  int32_t N;
  // RANKCODE layout
  const uint64_t* rc_bits;   // nW words, bit b of word w: cell jmin + 64 w + b holds an X_i
  const uint32_t* rc_base;   // nW counts: #{i : f(X_i) < jmin + 64 w}
  const uint16_t* rc_code;   // N+1 codes (allocation padded to a multiple of 8)
  const RcWord* rc_w16;      // nW interleaved words (bits, base)
  const uint8_t* rc_code8;   // N+1 8-bit codes (7-bit position, flag), for the L2 layout
  int32_t nW;
  int32_t gap_q;             // gap-q variant: compares per query
  int64_t x_off;             // index of X_0 in X (gap-q: the left padding)
  // PAIRS layout
  const CachePair<T>* pairs; // nK pairs, pairs[0] for cell jmin
  // NIBBLE layout
  const NibChunk* nib;       // ceil(nK / 24) chunks, chunk 0 starts at cell jmin
  int64_t nib_chunks;
  const T* z;
  int32_t* out;
  int64_t M;
};

template <typename T>
struct BsearchArgs {
  const T* X;         // padded X (leading-bit) or plain X (offset)
  int32_t nX;         // entries of X as stored
  int32_t N;
  int32_t P;          // leading-bit: 2^floor(log2 N)
  int32_t F, S, J;    // offset search constants
  int32_t pad_;
  const T* z;
  int32_t* out;
  int64_t M;
};

struct LearnedModel;  // defined in ds_learned.hip

}  // namespace ds

// The opaque handle behind ds_handle.
struct ds_index {
  int device = 0;
  ds_dtype dt = DS_F32;
  int32_t method = DS_METHOD_DIRECT;
  int32_t form = DS_FORM_SUB;
  int32_t hstart = DS_HSTART_PHI;
  int64_t N = 0;
  // Direct method parameters, exact values of the dtype
  double H = 0, W = 0, X0 = 0, XN = 0;
  int64_t R = 0, jmin = 0;
  int64_t n_updates = 0;
  int32_t refine_h = 0;   // bisect [last infeasible H, grown H] after growth
  int32_t n_refine = 0;   // midpoints the bisection tested
  // device memory
  void* X = nullptr;            // N+1 values (Direct, offset, learned), padded on the right
                                // (leading-bit) or on the left (gap-q: x_off copies of X_0)
  int64_t nX = 0;               // entries in X
  int64_t x_off = 0;            // index of X_0 in X
  int32_t gap_q = 0;            // gap-q variant: number of compares
  int32_t eyt_L = 0;            // Eytzinger layout: levels (X holds 2^L values, X[0] unused)
  int32_t* K = nullptr;         // Direct table
  bool k_in_x = false;          // K lies inside the allocation of X (small builds)
  int64_t nK = 0;
  // RANKCODE layout (see ds.h)
  uint64_t* rc_bits = nullptr;
  uint32_t* rc_base = nullptr;
  uint16_t* rc_code = nullptr;
  ds::RcWord* rc_w16 = nullptr;
  uint8_t* rc_code8 = nullptr;
  int64_t rc_words = 0;
  // PAIRS layout
  void* pairs = nullptr;
  // NIBBLE layout
  ds::NibChunk* nib = nullptr;
  int64_t nib_chunks = 0;
  // GAPCODE layout of the gap-q variant (q <= 15): per 64 / gc_bits cells the
  // key counts (gc_bits = 2 for q <= 3, else 4 bits each) and the count of
  // keys in earlier cells; the codes are rc_code's
  uint64_t* gc_counts = nullptr;
  uint32_t* gc_base = nullptr;
  int64_t gc_words = 0;
  int32_t gc_bits = 0;
  int32_t auto_stage = 2;       // layout the automatic launch uses
  // binary search constants
  int32_t P = 0, F = 0, S = 0, J = 0;
  // learned model (device), owned
  ds::LearnedModel* learned = nullptr;
  // launch shape
  ds_tune tune{};
  bool tune_set = false;
  int32_t staged = 0;           // the PLAIN tables fit in LDS
  ds_info_t info{};
};

namespace ds {
// implemented in ds_search.hip
// cand: a launch shape to use instead of the handle's (nullptr: the handle's)
ds_status launch_search(ds_index* h, const void* z, int64_t M, int32_t* out, hipStream_t s,
                        const ds_tune* cand = nullptr);
bool tables_fit_lds(const ds_index* h);
int64_t rankcode_lds_bytes(const ds_index* h);
int64_t direct_lds_bytes(const ds_index* h, int stage);  // LDS bytes of a Direct layout staged by the search
// implemented in ds_learned.hip
ds_status learned_build(ds_index* h, const ds_build_opts* o, hipStream_t s);
ds_status learned_search(ds_index* h, const void* z, int64_t M, int32_t* out, hipStream_t s);
void learned_free(ds_index* h);
void learned_fill_info(const ds_index* h, ds_info_t* in);
ds_status learned_fallbacks(const ds_index* h, uint64_t* count);  // synchronous device read
int num_cus();
}  // namespace ds
