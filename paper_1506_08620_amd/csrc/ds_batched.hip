// Batched ragged build + search: K independent arrays, each with its own
// queries, handled by a fixed sequence of kernels with no host
// synchronisation and no allocation, so the whole sequence can be captured in
// a HIP graph and replayed.
//
//   1. build       validation, minimum rounded gap and ComputeHR (Sec. 4.4.3)
//                  entirely on the device: two passes over the packed keys in
//                  fixed chunks (the minimum gap; the first pair whose cells
//                  coincide at the starting H) with per-array atomics, then
//                  one workgroup per array that needs growth applies the
//                  growth steps of the sequential algorithm from that pair
//                  and rescans until a pass changes nothing.
//   2. plan        one workgroup: exclusive scans over the arrays of the table
//                  words, codes and query tiles; arrays whose table would not
//                  fit the workspace fall back to the offset binary search
//                  (Sec. 3.3).  It also clears the tile queues.
//   3. rankcode    the RANKCODE layout of every Direct array (bitmap of
//                  occupied cells, running counts, 16-bit position codes):
//                  the occupancy words are cleared, then one pass over the
//                  packed keys in the same chunks sets every key's entries.
//   4. search      persistent workgroups pull query tiles from one queue per
//                  XCD (tiles of an array go to the XCD that took its first
//                  chunk, so that XCD's L2 holds the array's tables); when the
//                  array changes, the workgroup copies the array's tables into
//                  LDS if they fit, else it reads them through L2.
//
// Every array's results are local indices with the same out-of-domain values
// as ds_search; arrays with no value give -1, arrays with one value give -1 or
// 0, and arrays that are not strictly increasing or hold a non-finite value
// give -2 for all their queries.
#include <algorithm>
#include <limits>
#include <mutex>

#include "ds_batched_internal.h"
#include "ds_ops.h"

namespace ds {

namespace {

constexpr int kPlanBlock = 1024;
constexpr int64_t kScanChunk = 4096;  // packed values per workgroup of the build's passes over the keys
constexpr int kMaxGrowthRounds = 4096;

struct WsLayout {
  size_t meta, chunk_first, tile_off, totals, codes, bits, base, end;
  // learned region (present when nseg > 0)
  size_t lmeta, params, adam_m, adam_v, steps, grid, segs, first, longs, samples;
  int64_t words_budget;
  int64_t codes_cap;
  int32_t nseg;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

WsLayout ws_layout(int32_t K, int64_t total_x, int64_t words_budget, int32_t nseg) {
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  L.meta = take(size_t(K) * sizeof(ArrMeta<double>));
  L.chunk_first = take(size_t((total_x + kScanChunk - 1) / kScanChunk + 1) * 4);
  L.tile_off = take(size_t(K + 1) * sizeof(int64_t));
  L.totals = take(sizeof(PlanTotals));
  L.codes_cap = total_x + int64_t(K) * 8 + 8;
  L.codes = take(size_t(L.codes_cap) * 2);
  L.nseg = nseg;
  if (nseg > 0) {
    const size_t P = size_t(kRouterParams) * 4;
    L.lmeta = take(size_t(K) * sizeof(LearnMeta));
    L.params = take(size_t(K) * P);
    L.adam_m = take(size_t(K) * P);
    L.adam_v = take(size_t(K) * P);
    L.steps = take(size_t(K) * size_t(nseg) * 4);
    L.grid = take(size_t(K) * (size_t(4) << batch_grid_log2(nseg)));
    L.segs = take(size_t(K) * size_t(nseg) * kSegFitBytes);
    L.first = take(size_t(K) * size_t(nseg + 1) * 4);
    L.longs = take(size_t(total_x / (kFitLongKeys - 1) + 1) * sizeof(LongSeg));
    // first value of every 64-byte block of the packed X (total_x / 8 values of
    // 8 bytes in f64, total_x / 16 of 4 bytes in f32) and two lines of +inf
    L.samples = take(size_t(total_x) + 512);
  }
  L.words_budget = words_budget;
  L.bits = take(size_t(words_budget) * 8);
  L.base = take(size_t(words_budget) * 4);
  L.end = off;
  return L;
}

// largest words budget whose layout fits in a workspace of the given size
int64_t words_budget_for(int32_t K, int64_t total_x, int32_t nseg, size_t bytes) {
  const WsLayout L0 = ws_layout(K, total_x, 0, nseg);
  if (bytes <= L0.end) return 0;
  int64_t w = int64_t((bytes - L0.end) / 12);
  while (w > 0 && ws_layout(K, total_x, w, nseg).end > bytes) w -= std::max<int64_t>(1, w / 64);
  return std::max<int64_t>(0, w);
}

template <typename T>
__device__ __forceinline__ T next_up_dev(T x) {
  return std::nextafter(x, std::numeric_limits<T>::infinity());
}

// --------------------------------------------------------------------------
// 1. per-array ComputeHR (Sec. 4.4.2 - 4.4.3), in five launches.  The two
//    passes over the keys run over the packed buffer in fixed chunks, so a
//    2^20-key array is read by 256 workgroups at once instead of one:
//   init       one thread per array: X_0, X_N, the accumulators, and the
//              array of each chunk's first value
//   gaps       one workgroup per 4096 packed values: validation flags and
//              the minimum rounded gap of each array met, merged into the
//              array's accumulators with atomics
//   start      one thread per array: H = the float above 1 / min gap, W, and
//              the start's feasibility
//   first_bad  one workgroup per 4096 values: the first pair of each array
//              whose cells coincide at the starting H (atomic minimum);
//              a chunk of an array that is not Direct there is skipped
//   finish     one workgroup per array: ComputeHR's growth from that pair
//              on, for the arrays that have one; R, jmin, the table size
constexpr int kScanBlock = 256;
constexpr int kScanSlots = 1024;      // arrays of a chunk accumulated in LDS before the global atomics
constexpr int kFinishBlock = 256;
constexpr int32_t kNoPair = 0x7fffffff;

// R - jmin + 1 cells at this H exceed cap_cells (0 = no cap)
template <typename T, int FORM>
__device__ __forceinline__ bool over_cap(T H, T W, T X0, T XN, int64_t cap_cells) {
  if (cap_cells <= 0) return false;
  const int64_t cells = static_cast<int64_t>(grid_floor<T, FORM>(XN, H, W, X0)) -
                        static_cast<int64_t>(grid_floor<T, FORM>(X0, H, W, X0)) + 1;
  return cells > cap_cells;
}

// bits of a float >= 0 as an unsigned integer of the same order (for atomicMin)
__device__ __forceinline__ unsigned long long order_bits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ unsigned long long order_bits(double x) {
  return static_cast<unsigned long long>(__double_as_longlong(x));
}
template <typename T>
__device__ __forceinline__ T from_order_bits(unsigned long long b);
template <>
__device__ __forceinline__ float from_order_bits<float>(unsigned long long b) {
  return __uint_as_float(static_cast<uint32_t>(b));
}
template <>
__device__ __forceinline__ double from_order_bits<double>(unsigned long long b) {
  return __longlong_as_double(static_cast<long long>(b));
}

// the array holding packed value g: the largest k in [lo, hi) with
// x_off[k] <= g, given x_off[lo] <= g < x_off[hi] (empty arrays are skipped)
__device__ __forceinline__ int32_t array_of(const int64_t* __restrict__ x_off, int32_t lo, int32_t hi, int64_t g) {
  while (hi - lo > 1) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (x_off[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <typename T>
__global__ void __launch_bounds__(kScanBlock) init_meta_kernel(const int64_t* __restrict__ x_off,
                                                               const int64_t* __restrict__ q_off,
                                                               const T* __restrict__ Xp, int32_t K,
                                                               ArrMeta<T>* __restrict__ meta,
                                                               int32_t* __restrict__ chunk_first) {
  const int32_t k = blockIdx.x * kScanBlock + threadIdx.x;
  if (k >= K) return;
  const int64_t xo = x_off[k];
  const int64_t N = x_off[k + 1] - xo - 1;
  // the chunks whose first value lies in this array (each chunk start lies in exactly one array)
  for (int64_t c = (xo + kScanChunk - 1) / kScanChunk; c * kScanChunk < xo + N + 1; ++c)
    chunk_first[c] = k;
  ArrMeta<T> m{};
  m.x_off = xo;
  m.q_off = q_off[k];
  m.q_end = q_off[k + 1];
  m.N = static_cast<int32_t>(N);
  m.R = -1;
  m.gbits = order_bits(std::numeric_limits<T>::infinity());
  m.flags = 0;
  m.first_bad = kNoPair;
  if (N <= 0) {
    m.method = kBmTrivial;
    m.X0 = (N == 0) ? Xp[xo] : T(0);
  } else {
    m.method = DS_METHOD_DIRECT;  // until the start kernel decides
    m.X0 = Xp[xo];
    m.XN = Xp[xo + N];
  }
  meta[k] = m;
}

template <typename T, bool VECLOAD>
__device__ __forceinline__ void load_group(const T* __restrict__ X, int64_t g0, int64_t total_x,
                                           T (&v)[16 / sizeof(T)]) {
  constexpr int V = 16 / sizeof(T);
  if (VECLOAD && g0 + V <= total_x) {
    const uint4 q = *reinterpret_cast<const uint4*>(X + g0);
    __builtin_memcpy(&v[0], &q, 16);
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) v[e] = (g0 + e < total_x) ? X[g0 + e] : T(0);
  }
}

// The arrays met by this workgroup's chunk: k0 holds its first value, and
// every array of the chunk lies in [k0, hi) with x_off[hi] past the chunk.
struct ChunkArrays {
  int32_t k0, hi;
  bool one;  // the whole chunk lies in array k0
};

__device__ __forceinline__ ChunkArrays chunk_arrays(const int64_t* __restrict__ x_off, int32_t K,
                                                    const int32_t* __restrict__ chunk_first, int64_t total_x) {
  const int64_t c = blockIdx.x;
  const int64_t c1 = std::min((c + 1) * kScanChunk, total_x);
  const int64_t n_chunks = (total_x + kScanChunk - 1) / kScanChunk;
  ChunkArrays a;
  a.k0 = chunk_first[c];
  a.one = x_off[a.k0 + 1] >= c1;
  // the array holding the next chunk's first value ends past this chunk
  a.hi = (c + 1 < n_chunks) ? std::min(chunk_first[c + 1] + 1, K) : K;
  return a;
}

// Visits, in increasing g per lane, every pair (X[g], X[g+1]) of one array
// with g in this workgroup's chunk: vis.begin(k) when a lane enters array k,
// vis.pair(g, a, b) per pair, vis.end() when it leaves.  Lane t holds groups
// of 16 bytes at t, t + 256, ... so each load of a wave is 1 KiB contiguous;
// the loads are issued before the chunk's arrays are looked up.
template <typename T, bool VECLOAD, class Vis>
__device__ __forceinline__ ChunkArrays scan_pairs(const int64_t* __restrict__ x_off, int32_t K,
                                                  const int32_t* __restrict__ chunk_first, const T* __restrict__ X,
                                                  int64_t total_x, Vis& vis, unsigned long long* g_slots = nullptr,
                                                  uint32_t* f_slots = nullptr, T* __restrict__ samples = nullptr) {
  constexpr int V = 16 / sizeof(T);
  constexpr int U = static_cast<int>(kScanChunk / (kScanBlock * V));
  const int64_t c0 = int64_t(blockIdx.x) * kScanChunk;
  const int64_t c1 = std::min(c0 + kScanChunk, total_x);
  ChunkArrays ca;
  if constexpr (Vis::kLookFirst) {
    // a visitor that may skip the whole chunk looks before it loads
    ca = chunk_arrays(x_off, K, chunk_first, total_x);
    if (vis.skip(ca)) return ca;
  }
  T v[U][V], nx[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t g0 = c0 + int64_t(u * kScanBlock + threadIdx.x) * V;
    load_group<T, VECLOAD>(X, g0, total_x, v[u]);
    nx[u] = (g0 + V < total_x) ? X[g0 + V] : T(0);
  }
  if (samples) {
    // the first value of each 64-byte block of the packed buffer (the learned
    // search's samples): the lane whose group starts the block holds it
    constexpr int64_t E = 64 / sizeof(T);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t g0 = c0 + int64_t(u * kScanBlock + threadIdx.x) * V;
      if (g0 % E == 0 && g0 < c1) samples[g0 / E] = v[u][0];
    }
  }
  if constexpr (!Vis::kLookFirst) ca = chunk_arrays(x_off, K, chunk_first, total_x);
  vis.prepare(ca, g_slots, f_slots);
  int32_t k = ca.k0;
  int64_t end = x_off[k + 1];  // one past array k's last value
  vis.begin(k);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t g0 = c0 + int64_t(u * kScanBlock + threadIdx.x) * V;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int64_t g = g0 + e;
      if (g >= c1) continue;
      if (g >= end) {
        vis.end();
        k = array_of(x_off, std::min(k + 1, ca.hi - 1), ca.hi, g);
        end = x_off[k + 1];
        vis.begin(k);
      }
      if (g + 1 < end) vis.pair(g, v[u][e], e + 1 < V ? v[u][e + 1] : nx[u]);
    }
  }
  return ca;
}

template <typename T>
struct GapVis {
  static constexpr bool kLookFirst = false;  // every chunk is scanned
  ArrMeta<T>* meta;
  unsigned long long* s_g;  // per-array slots in LDS for a chunk of many arrays, else null
  uint32_t* s_f;
  int32_t k0;
  int32_t k;
  T x0, gmin;
  uint32_t fl;
  bool any;
  // a chunk of several arrays (few enough for the slots) merges its lanes in LDS first
  __device__ __forceinline__ void prepare(const ChunkArrays& ca, unsigned long long* g_slots, uint32_t* f_slots) {
    s_g = nullptr;
    if (ca.one || ca.hi - ca.k0 > kScanSlots) return;
    s_g = g_slots;
    s_f = f_slots;
    k0 = ca.k0;
    for (int j = threadIdx.x; j < ca.hi - ca.k0; j += kScanBlock) {
      s_g[j] = ~0ull;  // untouched
      s_f[j] = 0;
    }
    __syncthreads();
  }
  __device__ __forceinline__ void begin(int32_t kk) {
    k = kk;
    x0 = meta[kk].X0;
    gmin = std::numeric_limits<T>::infinity();
    fl = 0;
    any = false;
  }
  __device__ __forceinline__ void pair(int64_t, T a, T b) {
    any = true;
    if (!std::isfinite(a) || !std::isfinite(b)) fl |= 1u;
    if (!(a < b)) fl |= 2u;
    const T da = a - x0, db = b - x0;
    if (!(da < db)) fl |= 4u;
    gmin = std::fmin(gmin, db - da);
  }
  __device__ __forceinline__ void flush() const {
    // a gap <= 0 or NaN comes with flag 2 or 4, which decides alone
    const unsigned long long b = order_bits((gmin > T(0)) ? gmin : T(0));
    if (s_g) {
      atomicMin(&s_g[k - k0], b);
      if (fl) atomicOr(&s_f[k - k0], fl);
    } else {
      atomicMin(&meta[k].gbits, b);
      if (fl) atomicOr(&meta[k].flags, fl);
    }
  }
  __device__ __forceinline__ void end() const {
    if (any) flush();
  }
};

// validation flags (1: not finite, 2: not increasing, 4: X_i - X_0 not
// increasing) and the minimum rounded gap min (X_{i+1} - X_0) - (X_i - X_0)
template <typename T, bool VECLOAD>
__global__ void __launch_bounds__(kScanBlock) gaps_kernel(const int64_t* __restrict__ x_off, int32_t K,
                                                          const int32_t* __restrict__ chunk_first,
                                                          const T* __restrict__ Xp, int64_t total_x,
                                                          ArrMeta<T>* __restrict__ meta, T* __restrict__ samples) {
  __shared__ unsigned long long s_g[kScanSlots];
  __shared__ uint32_t s_f[kScanSlots];
  if (samples && blockIdx.x == gridDim.x - 1) {
    // after the last block's sample: two blocks' worth of +inf, which the
    // learned search may read past the buffer's end
    constexpr int64_t E = 64 / sizeof(T);
    const int64_t n_full = (total_x + E - 1) / E;
    if (threadIdx.x < 2 * E) samples[n_full + threadIdx.x] = std::numeric_limits<T>::infinity();
  }
  GapVis<T> vis{meta};
  const ChunkArrays ca = scan_pairs<T, VECLOAD>(x_off, K, chunk_first, Xp, total_x, vis, s_g, s_f, samples);
  if (ca.one) {
    // the whole chunk is one array: one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
      vis.gmin = std::fmin(vis.gmin, __shfl_xor(vis.gmin, off, 64));
      vis.fl |= __shfl_xor(vis.fl, off, 64);
      vis.any = vis.any | (__shfl_xor(static_cast<int>(vis.any), off, 64) != 0);
    }
    if ((threadIdx.x & 63) == 0 && vis.any) vis.flush();
    return;
  }
  vis.end();
  if (!vis.s_g) return;
  __syncthreads();
  for (int j = threadIdx.x; j < ca.hi - ca.k0; j += kScanBlock) {
    if (s_g[j] == ~0ull) continue;
    atomicMin(&meta[ca.k0 + j].gbits, s_g[j]);
    if (s_f[j]) atomicOr(&meta[ca.k0 + j].flags, s_f[j]);
  }
}

// H = the float above 1 / min gap (eq. minhnumeric), W, and whether that start
// is feasible before any growth
template <typename T, int FORM>
__global__ void __launch_bounds__(kScanBlock) start_kernel(int32_t K, int64_t cap_cells,
                                                           ArrMeta<T>* __restrict__ meta) {
  const int32_t k = blockIdx.x * kScanBlock + threadIdx.x;
  if (k >= K) return;
  ArrMeta<T>& m = meta[k];
  if (m.method != DS_METHOD_DIRECT) return;  // no value or one value
  const uint32_t flags = m.flags;
  if (flags & 3u) {
    m.method = kBmInvalid;
    return;
  }
  bool feasible = !(flags & 4u);
  T H = 0, W = 0;
  if (feasible) {
    const T g = from_order_bits<T>(m.gbits);
    const T Hbar = T(1) / g;  // correctly rounded division
    feasible = !std::isinf(Hbar);
    H = next_up_dev(Hbar);
    W = (FORM == DS_FORM_FMA) ? T(H * m.X0) : T(0);
    feasible = feasible && grid_floor<T, FORM>(m.XN, H, W, m.X0) < T(kTwoPowQ);
    // a table already over the Direct cap only grows with H: not Direct
    feasible = feasible && !over_cap<T, FORM>(H, W, m.X0, m.XN, cap_cells);
  }
  if (feasible) {
    m.H = H;
    m.W = W;
  } else {
    m.method = DS_METHOD_BSEARCH_OFFSET;
  }
}

template <typename T, int FORM>
struct FirstBadVis {
  ArrMeta<T>* meta;
  int32_t k;
  T H, W, x0;
  int64_t base;
  bool active;
  // a chunk inside one array that is not Direct at the starting H is skipped
  static constexpr bool kLookFirst = true;
  __device__ __forceinline__ bool skip(const ChunkArrays& ca) const {
    return ca.one && meta[ca.k0].method != DS_METHOD_DIRECT;
  }
  __device__ __forceinline__ void prepare(const ChunkArrays&, unsigned long long*, uint32_t*) {}
  __device__ __forceinline__ void begin(int32_t kk) {
    k = kk;
    const ArrMeta<T>& m = meta[kk];
    active = m.method == DS_METHOD_DIRECT;
    H = m.H;
    W = m.W;
    x0 = m.X0;
    base = m.x_off;
  }
  __device__ __forceinline__ void pair(int64_t g, T a, T b) {
    if (active && grid_floor<T, FORM>(a, H, W, x0) == grid_floor<T, FORM>(b, H, W, x0)) {
      atomicMin(&meta[k].first_bad, static_cast<int32_t>(g + 1 - base));
      active = false;  // later pairs of this lane come after this one
    }
  }
  __device__ __forceinline__ void end() const {}
};

// the first i with floor(m(X_{i-1})) = floor(m(X_i)) at the starting H
template <typename T, int FORM, bool VECLOAD>
__global__ void __launch_bounds__(kScanBlock) first_bad_kernel(const int64_t* __restrict__ x_off, int32_t K,
                                                               const int32_t* __restrict__ chunk_first,
                                                               const T* __restrict__ Xp, int64_t total_x,
                                                               ArrMeta<T>* __restrict__ meta) {
  FirstBadVis<T, FORM> vis{meta};
  (void)scan_pairs<T, VECLOAD>(x_off, K, chunk_first, Xp, total_x, vis);
}

// ComputeHR's growth (Sec. 4.4.3) from the first coinciding pair: one lane
// applies the growth steps of the sequential algorithm to that pair, the
// workgroup finds the next one after it, and a pass over the whole array
// that changes nothing ends the search
template <typename T, int FORM>
__global__ void __launch_bounds__(kFinishBlock) finish_kernel(const T* __restrict__ Xp, int64_t cap_cells,
                                                              ArrMeta<T>* __restrict__ meta) {
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ int64_t s_first[kFinishBlock];
  __shared__ T s_H, s_W;
  __shared__ int s_state;  // 0 continue, 1 infeasible
  ArrMeta<T>& mref = meta[k];
  if (mref.method != DS_METHOD_DIRECT) return;
  const int64_t N = mref.N;
  const T* X = Xp + mref.x_off;
  const T X0 = mref.X0, XN = mref.XN;
  T H = mref.H, W = mref.W;
  T P = next_up_dev(H) - H;
  int32_t n_updates = 0;
  bool feasible = true;
  int64_t bad = mref.first_bad;
  if (bad <= N) {
    if (tid == 0) {
      s_H = H;
      s_W = W;
      s_state = 0;
    }
    __syncthreads();
    int64_t i_start = 1;
    bool changed = false;
    for (int round = 0; round < kMaxGrowthRounds; ++round) {
      H = s_H;
      W = s_W;
      if (round > 0) {
        int64_t first = N + 1;
        for (int64_t i = i_start + tid; i <= N; i += kFinishBlock) {
          if (grid_floor<T, FORM>(X[i - 1], H, W, X0) == grid_floor<T, FORM>(X[i], H, W, X0)) {
            first = i;
            break;
          }
        }
        s_first[tid] = first;
        __syncthreads();
        for (int w = kFinishBlock / 2; w > 0; w >>= 1) {
          if (tid < w) s_first[tid] = std::min(s_first[tid], s_first[tid + w]);
          __syncthreads();
        }
        bad = s_first[0];
        __syncthreads();
      }
      if (bad > N) {
        if (!changed) break;  // a whole pass without change: every pair holds
        changed = false;
        i_start = 1;
        continue;
      }
      if (tid == 0) {
        const T a = X[bad - 1], b = X[bad];
        T h = s_H, ww = s_W;
        int st = 0;
        while (grid_floor<T, FORM>(a, h, ww, X0) == grid_floor<T, FORM>(b, h, ww, X0)) {
          h = h + P;
          if (FORM == DS_FORM_FMA) ww = h * X0;
          if (!(grid_floor<T, FORM>(XN, h, ww, X0) < T(kTwoPowQ)) || over_cap<T, FORM>(h, ww, X0, XN, cap_cells)) {
            st = 1;
            break;
          }
          P = P + P;
          ++n_updates;
        }
        s_H = h;
        s_W = ww;
        s_state = st;
      }
      __syncthreads();
      if (s_state) {
        feasible = false;
        break;
      }
      changed = true;
      i_start = bad + 1;
      if (round == kMaxGrowthRounds - 1) feasible = false;
    }
    H = s_H;
    W = s_W;
  }
  if (tid == 0) {
    if (feasible) {
      mref.H = H;
      mref.W = W;
      mref.R = static_cast<int32_t>(grid_floor<T, FORM>(XN, H, W, X0));
      mref.jmin = static_cast<int32_t>(grid_floor<T, FORM>(X0, H, W, X0));
      const int64_t nK = int64_t(mref.R) - mref.jmin + 1;
      const int64_t nW = (nK + 63) / 64;
      mref.nW = static_cast<int32_t>((nW + 3) / 4 * 4);  // keeps every array's words 16-byte aligned
      mref.n_updates = n_updates;
    } else {
      mref.method = DS_METHOD_BSEARCH_OFFSET;
      mref.H = 0;
      mref.W = 0;
    }
  }
}

// samples: where the learned search's samples go (the first value of each
// 64-byte block of the packed keys, then 2 x 64 / sizeof(T) of +inf), or null
template <typename T, int FORM>
ds_status launch_build(const ds_batch_desc* d, ArrMeta<T>* meta, int32_t* chunk_first, int64_t cap_cells,
                       T* samples, hipStream_t s) {
  const int32_t K = d->num_arrays;
  const T* X = static_cast<const T*>(d->X_dev);
  const dim3 per_array((K + kScanBlock - 1) / kScanBlock);
  init_meta_kernel<T><<<per_array, dim3(kScanBlock), 0, s>>>(d->x_off_dev, d->q_off_dev, X, K, meta, chunk_first);
  DS_HIP_CHECK(hipGetLastError());
  const dim3 chunks(static_cast<uint32_t>((d->total_x + kScanChunk - 1) / kScanChunk));
  const bool vec = (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
  if (chunks.x > 0) {
    if (vec)
      gaps_kernel<T, true><<<chunks, dim3(kScanBlock), 0, s>>>(d->x_off_dev, K, chunk_first, X, d->total_x, meta,
                                                               samples);
    else
      gaps_kernel<T, false><<<chunks, dim3(kScanBlock), 0, s>>>(d->x_off_dev, K, chunk_first, X, d->total_x, meta,
                                                                samples);
    DS_HIP_CHECK(hipGetLastError());
  }
  start_kernel<T, FORM><<<per_array, dim3(kScanBlock), 0, s>>>(K, cap_cells, meta);
  DS_HIP_CHECK(hipGetLastError());
  if (chunks.x > 0) {
    if (vec)
      first_bad_kernel<T, FORM, true><<<chunks, dim3(kScanBlock), 0, s>>>(d->x_off_dev, K, chunk_first, X,
                                                                          d->total_x, meta);
    else
      first_bad_kernel<T, FORM, false><<<chunks, dim3(kScanBlock), 0, s>>>(d->x_off_dev, K, chunk_first, X,
                                                                           d->total_x, meta);
    DS_HIP_CHECK(hipGetLastError());
  }
  finish_kernel<T, FORM><<<dim3(K), dim3(kFinishBlock), 0, s>>>(X, cap_cells, meta);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

// --------------------------------------------------------------------------
// 2. plan: scans over arrays (one workgroup).  Lane t owns the arrays
//    [t C, (t + 1) C), C = ceil(K / 1024): it sums them, one workgroup scan
//    turns the lanes' sums into their first offsets, and the lane walks its
//    arrays again to assign them; a second scan numbers the learned arrays.
//    With tiles_only (a new tile size over arrays already built) only the
//    query tiles are assigned again: methods, tables and slots stay.
__device__ __forceinline__ void plan_scan3(int64_t* s_a, int64_t* s_b, int64_t* s_c, int tid) {
  // inclusive Hillis-Steele scans of three lanes' values at once
  for (int d = 1; d < kPlanBlock; d <<= 1) {
    int64_t a = 0, b = 0, c = 0;
    if (tid >= d) {
      a = s_a[tid - d];
      b = s_b[tid - d];
      c = s_c[tid - d];
    }
    __syncthreads();
    s_a[tid] += a;
    s_b[tid] += b;
    s_c[tid] += c;
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(kPlanBlock) plan_kernel(ArrMeta<T>* __restrict__ meta, int32_t K,
                                                          int64_t* __restrict__ tile_off, PlanTotals* __restrict__ tot,
                                                          int64_t words_budget, int64_t tile, int32_t learn,
                                                          int64_t direct_cap_cells, LearnMeta* __restrict__ lmeta,
                                                          int32_t tiles_only) {
  __shared__ int64_t s_w[kPlanBlock], s_c[kPlanBlock], s_t[kPlanBlock];
  const int tid = threadIdx.x;
  if (tid < kNumQueues) {
    tot->queue[tid] = 0;
    tot->lqueue[tid] = 0;
  }
  if (tid == 0) {
    tot->fallbacks = 0;
    tot->long_segs = 0;
  }
  const int32_t per = (K + kPlanBlock - 1) / kPlanBlock;
  const int32_t kb = static_cast<int32_t>(std::min<int64_t>(K, int64_t(tid) * per));
  const int32_t ke = static_cast<int32_t>(std::min<int64_t>(K, int64_t(kb) + per));
  // pass 1: Direct over the per-array table cap is treated like an infeasible
  // array; the lane's table words, codes and tiles
  // (four arrays at a time, their fields loaded before any is used: the loop is bound by load latency)
  constexpr int kPlanBatch = 4;
  struct Fields {
    int32_t method, R, jmin, nW, N;
    int64_t q_off, q_end;
  };
  auto fields = [&](int32_t k0, Fields (&f)[kPlanBatch]) {
#pragma unroll
    for (int u = 0; u < kPlanBatch; ++u) {
      const ArrMeta<T>& m = meta[std::min(k0 + u, ke - 1)];
      f[u] = Fields{m.method, m.R, m.jmin, m.nW, m.N, m.q_off, m.q_end};
    }
  };
  int64_t sw = 0, sc = 0, st = 0;
  for (int32_t k0 = kb; k0 < ke; k0 += kPlanBatch) {
    Fields f[kPlanBatch];
    fields(k0, f);
#pragma unroll
    for (int u = 0; u < kPlanBatch; ++u) {
      if (k0 + u >= ke) break;
      int32_t method = f[u].method;
      if (!tiles_only) {
        if (method == DS_METHOD_DIRECT && direct_cap_cells > 0 && int64_t(f[u].R) - f[u].jmin + 1 > direct_cap_cells)
          method = DS_METHOD_BSEARCH_OFFSET;
        if (learn && method == DS_METHOD_BSEARCH_OFFSET) method = DS_METHOD_LEARNED;
        if (method != f[u].method) meta[k0 + u].method = method;
      }
      if (method == DS_METHOD_DIRECT) {
        sw += f[u].nW;
        sc += (int64_t(f[u].N) + 1 + 7) / 8 * 8;
      }
      st += (f[u].q_end - f[u].q_off + tile - 1) / tile;
    }
  }
  s_w[tid] = sw;
  s_c[tid] = sc;
  s_t[tid] = st;
  __syncthreads();
  plan_scan3(s_w, s_c, s_t, tid);
  // pass 2: offsets; a table that does not fit the workspace falls back (its
  // words still count in the offsets of the arrays after it)
  int64_t w0 = s_w[tid] - sw, c0 = s_c[tid] - sc, t0 = s_t[tid] - st;
  const int64_t words_total = s_w[kPlanBlock - 1], tiles_total = s_t[kPlanBlock - 1];
  int64_t nl = 0, lt = 0;
  for (int32_t k0 = kb; k0 < ke; k0 += kPlanBatch) {
    Fields f[kPlanBatch];
    fields(k0, f);  // the methods as pass 1 left them
#pragma unroll
    for (int u = 0; u < kPlanBatch; ++u) {
      if (k0 + u >= ke) break;
      ArrMeta<T>& m = meta[k0 + u];
      int32_t method = f[u].method;
      const int64_t nt = (f[u].q_end - f[u].q_off + tile - 1) / tile;
      m.t_off = t0;
      tile_off[k0 + u] = t0;
      t0 += nt;
      if (method == DS_METHOD_DIRECT && !tiles_only) {
        const int64_t nw = f[u].nW, nc = (int64_t(f[u].N) + 1 + 7) / 8 * 8;
        if (w0 + nw > words_budget) {
          method = learn ? DS_METHOD_LEARNED : DS_METHOD_BSEARCH_OFFSET;
          m.method = method;
          m.w_off = 0;
          m.c_off = 0;
        } else {
          m.w_off = w0;
          m.c_off = c0;
        }
        w0 += nw;
        c0 += nc;
      }
      if (method == DS_METHOD_LEARNED) {
        ++nl;
        lt += nt;
      }
    }
  }
  __syncthreads();
  s_w[tid] = nl;
  s_t[tid] = lt;
  s_c[tid] = 0;
  __syncthreads();
  plan_scan3(s_w, s_c, s_t, tid);
  // pass 3: learned arrays take consecutive model slots
  int32_t slot = static_cast<int32_t>(s_w[tid] - nl);
  for (int32_t k = kb; k < ke && nl > 0 && !tiles_only; ++k) {
    ArrMeta<T>& m = meta[k];
    if (m.method != DS_METHOD_LEARNED) continue;
    m.slot = slot;
    LearnMeta lm{};
    lm.X0 = static_cast<double>(m.X0);
    lm.XN = static_cast<double>(m.XN);
    const double range = lm.XN - lm.X0;
    lm.delta = std::fmax(range * 0x1p-40, 1e-300);
    const double d0 = lm.delta, d1 = range + lm.delta;
    int64_t b0, b1;
    __builtin_memcpy(&b0, &d0, 8);
    __builtin_memcpy(&b1, &d1, 8);
    lm.flo = static_cast<double>(b0);
    lm.fscale = 1.0 / (static_cast<double>(b1) - lm.flo);
    lm.x_off = m.x_off;
    lm.N = m.N;
    lm.k = k;
    lmeta[slot] = lm;
    ++slot;
  }
  if (tid == kPlanBlock - 1) {
    tile_off[K] = tiles_total;
    tot->total_tiles = tiles_total;
    tot->learned_tiles = s_t[kPlanBlock - 1];
    if (!tiles_only) {
      tot->words_used = words_total;
      tot->n_learned = static_cast<int32_t>(s_w[kPlanBlock - 1]);
    }
  }
}

// --------------------------------------------------------------------------
// 3. RANKCODE layout of every Direct array (bitmap of occupied cells, running
//    counts, 16-bit position codes), in two launches over the packed values
//    like the build's scans: the pool's occupancy words are cleared, then
//    each value sets its cell's bit, writes its code and the running count of
//    the words whose first cell lies in (cell of X_{i-1}, cell of X_i].
__global__ void __launch_bounds__(kScanBlock) zero_words_kernel(unsigned long long* __restrict__ bits,
                                                                const PlanTotals* __restrict__ tot,
                                                                int64_t words_budget) {
  // the placed arrays' words lie in [0, words_used) (the count also holds
  // arrays that did not fit, hence the budget)
  const int64_t n = std::min(tot->words_used, words_budget);
  const int64_t stride = int64_t(gridDim.x) * kScanBlock * 2;
  for (int64_t w = (int64_t(blockIdx.x) * kScanBlock + threadIdx.x) * 2; w < n; w += stride) {
    if (w + 1 < n)
      *reinterpret_cast<uint4*>(bits + w) = make_uint4(0, 0, 0, 0);  // the pool is 256-byte aligned, w even
    else
      bits[w] = 0ull;
  }
}

template <typename T, int FORM, bool VECLOAD>
__global__ void __launch_bounds__(kScanBlock) rankcode_kernel(const int64_t* __restrict__ x_off, int32_t K,
                                                              const int32_t* __restrict__ chunk_first,
                                                              const T* __restrict__ Xp, int64_t total_x,
                                                              const ArrMeta<T>* __restrict__ meta,
                                                              unsigned long long* __restrict__ bits,
                                                              uint32_t* __restrict__ base,
                                                              uint16_t* __restrict__ codes) {
  constexpr int V = 16 / sizeof(T);
  constexpr int U = static_cast<int>(kScanChunk / (kScanBlock * V));
  const int64_t c0 = int64_t(blockIdx.x) * kScanChunk;
  const int64_t c1 = std::min(c0 + kScanChunk, total_x);
  const int lane = threadIdx.x & 63;
  const ChunkArrays ca = chunk_arrays(x_off, K, chunk_first, total_x);
  int32_t k = ca.k0;
  ArrMeta<T> m = meta[k];
  if (ca.one && m.method != DS_METHOD_DIRECT) return;  // a chunk of a learned or binary-search array
  T v[U][V], pv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t g0 = c0 + int64_t(u * kScanBlock + threadIdx.x) * V;
    load_group<T, VECLOAD>(Xp, g0, total_x, v[u]);
    pv[u] = (g0 > 0 && g0 <= total_x) ? Xp[g0 - 1] : T(0);
  }
  int64_t end = x_off[k + 1];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t g0 = c0 + int64_t(u * kScanBlock + threadIdx.x) * V;
    long long key = -1 - lane;  // global word of acc; distinct negatives never merge
    unsigned long long acc = 0;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int64_t g = g0 + e;
      if (g >= c1) continue;
      if (g >= end) {
        k = array_of(x_off, std::min(k + 1, ca.hi - 1), ca.hi, g);
        end = x_off[k + 1];
        m = meta[k];
      }
      if (m.method != DS_METHOD_DIRECT) continue;
      const int64_t i = g - m.x_off;
      const int64_t nK = int64_t(m.R) - m.jmin + 1;
      const int64_t nWused = (nK + 63) / 64;
      uint32_t* bb = base + m.w_off;
      uint16_t* cb = codes + m.c_off;
      const T x = v[u][e];
      const T gv = grid_value<T, FORM>(x, m.H, m.W, m.X0);
      const T jf = std::floor(gv);
      const int64_t cell = static_cast<int64_t>(jf) - m.jmin;
      const T xp = (e > 0) ? v[u][e > 0 ? e - 1 : 0] : pv[u];
      const int64_t cprev = (i == 0) ? -1 : static_cast<int64_t>(grid_floor<T, FORM>(xp, m.H, m.W, m.X0)) - m.jmin;
      // running counts: words whose first cell lies in (cprev, cell] start at i
      for (int64_t w = (cprev + 1 + 63) / 64; w <= cell / 64 && w < nWused; ++w) bb[w] = static_cast<uint32_t>(i);
      const T c = cell_code<T>(gv, jf);
      const T p = std::nextafter(x, -std::numeric_limits<T>::infinity());
      const T vp = grid_value<T, FORM>(p, m.H, m.W, m.X0);
      const T jp = std::floor(vp);
      const int first = (jp == jf && cell_code<T>(vp, jp) == c) ? 0 : 1;
      cb[i] = static_cast<uint16_t>((static_cast<int>(c) << 1) | first);
      if (i == m.N) {
        for (int64_t w = nWused; w < m.nW; ++w) bb[w] = static_cast<uint32_t>(m.N + 1);  // padding words
        for (int64_t j = m.N + 1; j < (int64_t(m.N) + 1 + 7) / 8 * 8; ++j) cb[j] = 0;
      }
      if (cell >= 0 && cell < nK) {
        const long long word = m.w_off + (cell >> 6);
        const unsigned long long bit = 1ull << (cell & 63);
        if (word == key) {
          acc |= bit;
        } else {
          if (key >= 0) atomicOr(&bits[key], acc);  // an earlier word of this lane's group
          key = word;
          acc = bit;
        }
      }
    }
    // Lanes hold consecutive groups, so their words are non-decreasing across
    // the wave: a segmented OR over lanes that share a word leaves one atomic
    // per word and wave.
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned long long ob = __shfl_down(acc, off, 64);
      const long long ow = __shfl_down(key, off, 64);
      if (lane + off < 64 && ow == key) acc |= ob;
    }
    const long long kprev = __shfl_up(key, 1, 64);
    if (key >= 0 && (lane == 0 || kprev != key)) atomicOr(&bits[key], acc);
  }
}

template <typename T, int FORM>
ds_status launch_rankcode(const ds_batch_desc* d, const WsLayout& L, unsigned char* ws, hipStream_t s) {
  if (L.words_budget > 0) {
    const int64_t blocks = std::min<int64_t>((L.words_budget + 2 * kScanBlock - 1) / (2 * kScanBlock), 4096);
    zero_words_kernel<<<dim3(static_cast<uint32_t>(blocks)), dim3(kScanBlock), 0, s>>>(
        reinterpret_cast<unsigned long long*>(ws + L.bits), reinterpret_cast<const PlanTotals*>(ws + L.totals),
        L.words_budget);
    DS_HIP_CHECK(hipGetLastError());
  }
  const dim3 chunks(static_cast<uint32_t>((d->total_x + kScanChunk - 1) / kScanChunk));
  if (chunks.x == 0) return DS_OK;
  const T* X = static_cast<const T*>(d->X_dev);
  const auto* meta = reinterpret_cast<const ArrMeta<T>*>(ws + L.meta);
  const auto* cf = reinterpret_cast<const int32_t*>(ws + L.chunk_first);
  auto* bits = reinterpret_cast<unsigned long long*>(ws + L.bits);
  auto* base = reinterpret_cast<uint32_t*>(ws + L.base);
  auto* codes = reinterpret_cast<uint16_t*>(ws + L.codes);
  if ((reinterpret_cast<uintptr_t>(X) & 15u) == 0)
    rankcode_kernel<T, FORM, true><<<chunks, dim3(kScanBlock), 0, s>>>(d->x_off_dev, d->num_arrays, cf, X,
                                                                       d->total_x, meta, bits, base, codes);
  else
    rankcode_kernel<T, FORM, false><<<chunks, dim3(kScanBlock), 0, s>>>(d->x_off_dev, d->num_arrays, cf, X,
                                                                        d->total_x, meta, bits, base, codes);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

// --------------------------------------------------------------------------
// 4. persistent search
struct SearchShape {
  int64_t tile;
  int32_t lds_budget;  // bytes of dynamic LDS per workgroup (0: never stage)
  int32_t chunk;       // tiles per queue chunk
};

template <typename T>
__device__ __forceinline__ void stage_values(T* __restrict__ dst, const T* __restrict__ src, int64_t n) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// The queries [q0, q1) of one tile in chunks of 64 QPT, each taken by a wave
// from the LDS counter *next*: a wave that started late (the one that claims
// the next tile) just takes fewer chunks.
template <typename T, int QPT, class Op>
__device__ __forceinline__ void run_tile(const T* __restrict__ z, int32_t* __restrict__ out, int64_t q0, int64_t q1,
                                         const Op& op, int32_t* next) {
  constexpr int64_t kChunkQ = 64 * QPT;
  const int lane = threadIdx.x & 63;
  const int64_t nchunks = (q1 - q0 + kChunkQ - 1) / kChunkQ;
  for (;;) {
    int c = 0;
    if (lane == 0) c = atomicAdd(next, 1);
    c = __shfl(c, 0, 64);
    if (c >= nchunks) break;
    const int64_t q = q0 + int64_t(c) * kChunkQ + lane;
    if (q0 + (int64_t(c) + 1) * kChunkQ <= q1) {
      T v[QPT];
#pragma unroll
      for (int u = 0; u < QPT; ++u) v[u] = __builtin_nontemporal_load(z + q + u * 64);
#pragma unroll
      for (int u = 0; u < QPT; ++u) __builtin_nontemporal_store(op(v[u]), out + q + u * 64);
    } else {
      for (int64_t r = q; r < q1; r += 64) out[r] = op(z[r]);
    }
  }
}

// Persistent workgroups pull tiles from their XCD's queue.  Wave 0 claims the
// next tile (queue atomic, then the tile's array by a 64-way search of the
// tile offsets) while the other waves start on the current one; the claim
// and the tile's chunk counter are double-buffered in LDS, so one barrier per
// tile separates them.
template <typename T, int FORM, int QPT>
__global__ void __launch_bounds__(1024) batch_search_kernel(const ArrMeta<T>* __restrict__ meta, int32_t K,
                                                            const int64_t* __restrict__ tile_off,
                                                            PlanTotals* __restrict__ tot, const T* __restrict__ Xp,
                                                            const unsigned long long* __restrict__ bits,
                                                            const uint32_t* __restrict__ base,
                                                            const uint16_t* __restrict__ codes,
                                                            const T* __restrict__ z, int32_t* __restrict__ out,
                                                            SearchShape sh) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int64_t s_tile[2];
  __shared__ int32_t s_k[2];
  __shared__ int32_t s_next[2];
  const int queue = blockIdx.x % kNumQueues;
  const int64_t total = tot->total_tiles;
  if (tot->learned_tiles == total) return;  // every tile belongs to a learned array
  auto claim = [&](int slot) {  // by wave 0
    unsigned long long li = 0;
    if (threadIdx.x == 0) li = atomicAdd(&tot->queue[queue], 1u);
    li = __shfl(li, 0, 64);
    const int64_t ch = sh.chunk;
    const int64_t g = ((int64_t(li) / ch) * kNumQueues + queue) * ch + (int64_t(li) % ch);
    // the last array whose first tile is <= g
    const int32_t k = (g < total) ? wave_last_le(tile_off, K, g) : -1;
    if (threadIdx.x == 0) {
      s_tile[slot] = g;
      s_k[slot] = k;
    }
  };
  if (threadIdx.x < 64) claim(0);
  if (threadIdx.x == 0) s_next[0] = 0;
  __syncthreads();
  int32_t cur = -1;
  bool staged = false;
  for (int b = 0;; b ^= 1) {
    const int64_t g = s_tile[b];
    const int32_t k = s_k[b];
    if (g >= total) break;
    const ArrMeta<T>& m = meta[k];
    const int64_t q0 = m.q_off + (g - m.t_off) * sh.tile;
    const int64_t q1 = std::min(m.q_end, q0 + sh.tile);
    const int64_t N = m.N;
    // the tables of a new array go to LDS when they fit (every wave is past the
    // previous tile's end barrier)
    const int64_t nW = m.nW;
    const int64_t base_off = round16(nW * 8);
    const int64_t code_off = base_off + round16(nW * 4);
    if (k != cur) {
      if (m.method == DS_METHOD_DIRECT) {
        staged = code_off + round16((N + 1) * 2) <= sh.lds_budget;
        if (staged) {
          stage_bytes(smem, reinterpret_cast<const unsigned char*>(bits + m.w_off), nW * 8);
          stage_bytes(smem + base_off, reinterpret_cast<const unsigned char*>(base + m.w_off), nW * 4);
          stage_bytes(smem + code_off, reinterpret_cast<const unsigned char*>(codes + m.c_off), round16((N + 1) * 2));
        }
      } else if (m.method == DS_METHOD_BSEARCH_OFFSET) {
        staged = (N + 1) * int64_t(sizeof(T)) <= sh.lds_budget;
        if (staged) stage_values(reinterpret_cast<T*>(smem), Xp + m.x_off, N + 1);
      }
      cur = k;
      __syncthreads();
    }
    if (threadIdx.x == 0) s_next[b ^ 1] = 0;
    if (threadIdx.x < 64) claim(b ^ 1);
    if (m.method == DS_METHOD_DIRECT) {
      const T vlo = T(m.jmin), vhi = T(m.R);
      if (staged) {
        RankCodeOp<T, FORM, false> op{reinterpret_cast<const uint64_t*>(smem),
                                      reinterpret_cast<const uint32_t*>(smem + base_off), nullptr,
                                      reinterpret_cast<const uint16_t*>(smem + code_off), Xp + m.x_off, m.H, m.W,
                                      m.X0, vlo, vhi, m.XN, m.jmin, m.N};
        run_tile<T, QPT>(z, out, q0, q1, op, &s_next[b]);
      } else {
        RankCodeOp<T, FORM, false> op{reinterpret_cast<const uint64_t*>(bits + m.w_off), base + m.w_off, nullptr,
                                      codes + m.c_off, Xp + m.x_off, m.H, m.W, m.X0, vlo, vhi, m.XN, m.jmin, m.N};
        run_tile<T, QPT>(z, out, q0, q1, op, &s_next[b]);
      }
    } else if (m.method == DS_METHOD_BSEARCH_OFFSET) {
      const int32_t F = static_cast<int32_t>((N + 1) / 2);
      const int32_t S = static_cast<int32_t>(N + 1 - F);
      int32_t J = 0;
      while ((int64_t(1) << (J + 1)) <= N + 1) ++J;
      OffsetOp<T> op{staged ? reinterpret_cast<const T*>(smem) : Xp + m.x_off, F, S, J};
      run_tile<T, QPT>(z, out, q0, q1, op, &s_next[b]);
    } else if (m.method != DS_METHOD_LEARNED) {  // learned tiles are searched by the learned kernel
      const int32_t fill = (m.method == kBmInvalid) ? -2 : -1;
      const bool one = (m.method == kBmTrivial && N == 0);
      const T x0 = m.X0;
      for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) out[q] = (one && z[q] >= x0) ? 0 : fill;
    }
    __syncthreads();  // the tile is done and the next one claimed
  }
}

template <typename T, int FORM, int QPT>
ds_status launch_search_kernel(const ds_batch_desc* d, const WsLayout& L, unsigned char* ws, const SearchShape& sh,
                               int block, hipStream_t s) {
  auto kern = batch_search_kernel<T, FORM, QPT>;
  const int lds = sh.lds_budget;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  int grid = per_cu * num_cus();
  grid = std::max(kNumQueues, grid / kNumQueues * kNumQueues);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, reinterpret_cast<const ArrMeta<T>*>(ws + L.meta),
                     d->num_arrays, reinterpret_cast<const int64_t*>(ws + L.tile_off),
                     reinterpret_cast<PlanTotals*>(ws + L.totals), static_cast<const T*>(d->X_dev),
                     reinterpret_cast<const unsigned long long*>(ws + L.bits),
                     reinterpret_cast<const uint32_t*>(ws + L.base), reinterpret_cast<const uint16_t*>(ws + L.codes),
                     static_cast<const T*>(d->z_dev), d->out_dev, sh);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

template <typename T, int FORM>
ds_status launch_search_qpt(const ds_batch_desc* d, const WsLayout& L, unsigned char* ws, const SearchShape& sh,
                            int block, int qpt, hipStream_t s) {
  switch (qpt) {
    case 4: return launch_search_kernel<T, FORM, 4>(d, L, ws, sh, block, s);
    case 16: return launch_search_kernel<T, FORM, 16>(d, L, ws, sh, block, s);
    default: return launch_search_kernel<T, FORM, 8>(d, L, ws, sh, block, s);
  }
}

// Queries per work item when none is set: 2^17, or 2^14 when learned models
// are enabled, so that the workgroups of one XCD usually work on the same
// learned array at once and share its keys in that XCD's L2 (each XCD takes a
// contiguous range of the tile order).
int64_t tile_of(const ds_batch_desc* d) {
  if (d->tile > 0) return d->tile;
  return d->learn_segments > 0 ? (int64_t(1) << 14) : (int64_t(1) << 17);
}

SearchShape shape_of(const ds_batch_desc* d) {
  SearchShape sh{};
  sh.tile = tile_of(d);
  sh.lds_budget = d->lds_bytes < 0 ? 0 : (d->lds_bytes > 0 ? std::min(d->lds_bytes, kLdsBytesPerCU - 1024)
                                                            : kLdsBytesPerCU - 1024);
  sh.chunk = 4;
  return sh;
}

WsLayout layout_of(const ds_batch_desc* d) {
  const int32_t nseg = d->learn_segments > 0 ? d->learn_segments : 0;
  return ws_layout(d->num_arrays, d->total_x, words_budget_for(d->num_arrays, d->total_x, nseg, d->workspace_bytes),
                   nseg);
}

template <typename T>
ds_status launch_plan(const ds_batch_desc* d, const WsLayout& L, unsigned char* ws, int64_t tile, hipStream_t s,
                      bool tiles_only = false) {
  const int64_t cap_cells = d->direct_cap_bytes > 0 ? d->direct_cap_bytes / 4 : 0;
  plan_kernel<T><<<dim3(1), dim3(kPlanBlock), 0, s>>>(
      reinterpret_cast<ArrMeta<T>*>(ws + L.meta), d->num_arrays, reinterpret_cast<int64_t*>(ws + L.tile_off),
      reinterpret_cast<PlanTotals*>(ws + L.totals), L.words_budget, tile, L.nseg > 0 ? 1 : 0, cap_cells,
      L.nseg > 0 ? reinterpret_cast<LearnMeta*>(ws + L.lmeta) : nullptr, tiles_only ? 1 : 0);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

BatchLearned learned_of(const ds_batch_desc* d, const WsLayout& L, unsigned char* ws) {
  BatchLearned b{};
  b.meta = ws + L.meta;
  b.tile_off = reinterpret_cast<const int64_t*>(ws + L.tile_off);
  b.tot = reinterpret_cast<PlanTotals*>(ws + L.totals);
  b.K = d->num_arrays;
  b.nseg = L.nseg;
  b.identity = d->learn_steps < 0 ? 1 : 0;
  b.steps = d->learn_steps > 0 ? d->learn_steps : (d->learn_steps == 0 ? kBatchLearnStepsDefault : 0);
  b.log2g = batch_grid_log2(L.nseg);
  b.seed = 0x1506ull;
  b.tile = tile_of(d);
  b.X = d->X_dev;
  b.total_x = d->total_x;
  b.z = d->z_dev;
  b.out = d->out_dev;
  b.lmeta = reinterpret_cast<LearnMeta*>(ws + L.lmeta);
  b.params = reinterpret_cast<float*>(ws + L.params);
  b.adam_m = reinterpret_cast<float*>(ws + L.adam_m);
  b.adam_v = reinterpret_cast<float*>(ws + L.adam_v);
  b.steps_tab = reinterpret_cast<float*>(ws + L.steps);
  b.grid = reinterpret_cast<uint32_t*>(ws + L.grid);
  b.segs = ws + L.segs;
  b.first = reinterpret_cast<int32_t*>(ws + L.first);
  b.longs = reinterpret_cast<LongSeg*>(ws + L.longs);
  b.samples = ws + L.samples;
  return b;
}

// Times the search phase for each launch shape on the arrays already built in
// the workspace; keeps the fastest in *d.
template <typename T, int FORM>
ds_status autotune_batched(ds_batch_desc* d, hipStream_t s) {
  unsigned char* ws = static_cast<unsigned char*>(d->workspace_dev);
  const WsLayout L = layout_of(d);
  hipEvent_t e0, e1;
  DS_HIP_CHECK(hipEventCreate(&e0));
  DS_HIP_CHECK(hipEventCreate(&e1));
  const int tiles[5] = {1 << 16, 1 << 17, 1 << 18, 1 << 19, 1 << 20};
  const int blocks[2] = {512, 1024};
  const int qpts[3] = {4, 8, 16};
  float best = 1e30f;
  ds_batch_desc bd = *d;
  ds_status st = DS_OK;
  for (int ti = 0; ti < 5 && st == DS_OK; ++ti) {
    for (int bi = 0; bi < 2 && st == DS_OK; ++bi) {
      for (int qi = 0; qi < 3 && st == DS_OK; ++qi) {
        ds_batch_desc c = *d;
        c.tile = tiles[ti];
        c.block = blocks[bi];
        c.qpt = qpts[qi];
        const SearchShape sh = shape_of(&c);
        float total = 0;
        for (int r = 0; r < 2 && st == DS_OK; ++r) {
          st = launch_plan<T>(&c, L, ws, sh.tile, s, true);  // re-plans the tiles and clears the queues
          if (st != DS_OK) break;
          if (hipEventRecord(e0, s) != hipSuccess) { st = DS_ERR_HIP; break; }
          st = launch_search_qpt<T, FORM>(&c, L, ws, sh, c.block, c.qpt, s);
          if (st != DS_OK) break;
          if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { st = DS_ERR_HIP; break; }
          float ms = 0;
          if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = DS_ERR_HIP; break; }
          if (r > 0) total += ms;
        }
        if (st == DS_OK && total < best) {
          best = total;
          bd = c;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DS_OK) return st;
  d->tile = bd.tile;
  d->block = bd.block;
  d->qpt = bd.qpt;
  return DS_OK;
}

template <typename T, int FORM>
ds_status run_batched(const ds_batch_desc* d, hipStream_t s) {
  unsigned char* ws = static_cast<unsigned char*>(d->workspace_dev);
  const WsLayout L = layout_of(d);
  const int64_t tile = tile_of(d);
  auto* meta = reinterpret_cast<ArrMeta<T>*>(ws + L.meta);
  const int64_t cap_cells = d->direct_cap_bytes > 0 ? d->direct_cap_bytes / 4 : 0;
  ds_status st = launch_build<T, FORM>(d, meta, reinterpret_cast<int32_t*>(ws + L.chunk_first), cap_cells,
                                       L.nseg > 0 ? reinterpret_cast<T*>(ws + L.samples) : nullptr, s);
  if (st != DS_OK) return st;
  st = launch_plan<T>(d, L, ws, tile, s);
  if (st != DS_OK) return st;
  st = launch_rankcode<T, FORM>(d, L, ws, s);
  if (st != DS_OK) return st;
  if (L.nseg > 0) {
    st = batched_learned_build(learned_of(d, L, ws), d->dtype, s);
    if (st != DS_OK) return st;
  }
  if (d->total_q == 0) return DS_OK;
  const SearchShape sh = shape_of(d);
  const int block = d->block > 0 ? d->block : 1024;
  const int qpt = d->qpt > 0 ? d->qpt : 8;
  st = launch_search_qpt<T, FORM>(d, L, ws, sh, block, qpt, s);
  if (st != DS_OK || L.nseg == 0) return st;
  return batched_learned_search(learned_of(d, L, ws), d->dtype, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// The fixed workspace of ds_search_batched_noalloc.  In host code the name
// `scratch` stands for the symbol, not for device memory: the device address
// of each GPU's copy is looked up once per device and kept in scratch_ptr.
__device__ __align__(256) unsigned char scratch[DS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxScratchDevices] = {};

// the current device's copy of the scratch array
ds_status current_scratch(void** out) {
  int dev = -1;
  DS_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return DS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    DS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return DS_ERR_HIP;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return DS_OK;
}
}  // namespace

}  // namespace ds

extern "C" {

size_t ds_batch_workspace_bytes(int32_t num_arrays, int64_t total_x, int64_t table_budget_entries,
                                int32_t learn_segments) {
  if (num_arrays < 0 || total_x < 0 || table_budget_entries < 0 || learn_segments < 0 ||
      learn_segments > ds::kBatchMaxSegments)
    return 0;
  // each array's words are rounded up to a multiple of 4, plus one partial word
  const int64_t words = table_budget_entries > 0 ? table_budget_entries / 64 + int64_t(num_arrays) * 4 + 16 : 0;
  return ds::ws_layout(num_arrays, total_x, words, learn_segments).end;
}

ds_status ds_search_batched(const ds_batch_desc* d, hipStream_t s) {
  if (!d) return DS_ERR_ARG;
  if (d->dtype != DS_F32 && d->dtype != DS_F64) return DS_ERR_ARG;
  if (d->form != DS_FORM_SUB && d->form != DS_FORM_FMA) return DS_ERR_ARG;
  if (d->num_arrays < 0 || d->total_x < 0 || d->total_q < 0) return DS_ERR_ARG;
  if (d->num_arrays == 0) return DS_OK;
  if (!d->x_off_dev || !d->q_off_dev || !d->workspace_dev) return DS_ERR_ARG;
  if (d->total_x > 0 && !d->X_dev) return DS_ERR_ARG;
  if (d->total_q > 0 && (!d->z_dev || !d->out_dev)) return DS_ERR_ARG;
  if (d->block != 0 && (d->block < 64 || d->block > 1024 || d->block % 64)) return DS_ERR_ARG;
  if (d->qpt != 0 && d->qpt != 4 && d->qpt != 8 && d->qpt != 16) return DS_ERR_ARG;
  if (d->tile < 0) return DS_ERR_ARG;
  if (d->learn_segments < 0 || d->learn_segments > ds::kBatchMaxSegments || d->learn_steps < -1 ||
      d->direct_cap_bytes < 0)
    return DS_ERR_ARG;
  if (d->workspace_bytes < ds_batch_workspace_bytes(d->num_arrays, d->total_x, 0, d->learn_segments))
    return DS_ERR_ARG;
  if (d->dtype == DS_F32)
    return d->form == DS_FORM_FMA ? ds::run_batched<float, DS_FORM_FMA>(d, s) : ds::run_batched<float, DS_FORM_SUB>(d, s);
  return d->form == DS_FORM_FMA ? ds::run_batched<double, DS_FORM_FMA>(d, s) : ds::run_batched<double, DS_FORM_SUB>(d, s);
}

ds_status ds_search_batched_noalloc(const ds_batch_desc* d, hipStream_t s) {
  if (!d) return DS_ERR_ARG;
  if (d->num_arrays < 0 || d->total_x < 0 || d->learn_segments < 0 || d->learn_segments > ds::kBatchMaxSegments)
    return DS_ERR_ARG;
  const size_t need = ds_batch_workspace_bytes(d->num_arrays, d->total_x, 0, d->learn_segments);
  if (need == 0) return DS_ERR_ARG;
  if (need > size_t(DS_NOALLOC_SCRATCH_BYTES)) return DS_ERR_SCRATCH_CAP;
  ds_batch_desc c = *d;
  void* ws = nullptr;
  const ds_status st = ds::current_scratch(&ws);
  if (st != DS_OK) return st;
  c.workspace_dev = ws;
  c.workspace_bytes = DS_NOALLOC_SCRATCH_BYTES;
  return ds_search_batched(&c, s);
}

ds_status ds_batch_autotune(ds_batch_desc* d, hipStream_t s) {
  ds_status st = ds_search_batched(d, s);  // builds every array into the workspace
  if (st != DS_OK) return st;
  if (d->num_arrays == 0 || d->total_q == 0) return DS_OK;
  if (d->dtype == DS_F32)
    return d->form == DS_FORM_FMA ? ds::autotune_batched<float, DS_FORM_FMA>(d, s)
                                  : ds::autotune_batched<float, DS_FORM_SUB>(d, s);
  return d->form == DS_FORM_FMA ? ds::autotune_batched<double, DS_FORM_FMA>(d, s)
                                : ds::autotune_batched<double, DS_FORM_SUB>(d, s);
}

ds_status ds_batch_fallbacks(const ds_batch_desc* d, uint64_t* count_host, hipStream_t s) {
  if (!d || !count_host || !d->workspace_dev || d->num_arrays < 0) return DS_ERR_ARG;
  const ds::WsLayout L = ds::layout_of(d);
  const auto* tot = reinterpret_cast<const ds::PlanTotals*>(static_cast<const unsigned char*>(d->workspace_dev) +
                                                             L.totals);
  unsigned long long v = 0;
  DS_HIP_CHECK(hipMemcpyAsync(&v, &tot->fallbacks, sizeof(v), hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipStreamSynchronize(s));
  *count_host = v;
  return DS_OK;
}

ds_status ds_batch_report(const ds_batch_desc* d, int32_t* method_host, int64_t* R_host, hipStream_t s) {
  if (!d || d->num_arrays < 0) return DS_ERR_ARG;
  if (d->num_arrays == 0) return DS_OK;
  if (!method_host || !R_host || !d->workspace_dev) return DS_ERR_ARG;
  const ds::WsLayout L = ds::layout_of(d);
  const size_t msz = d->dtype == DS_F32 ? sizeof(ds::ArrMeta<float>) : sizeof(ds::ArrMeta<double>);
  unsigned char* host = static_cast<unsigned char*>(std::malloc(msz * size_t(d->num_arrays)));
  if (!host) return DS_ERR_OOM;
  hipError_t e = hipMemcpyAsync(host, static_cast<unsigned char*>(d->workspace_dev) + L.meta,
                                msz * size_t(d->num_arrays), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    std::free(host);
    return DS_ERR_HIP;
  }
  for (int32_t k = 0; k < d->num_arrays; ++k) {
    if (d->dtype == DS_F32) {
      const auto* m = reinterpret_cast<const ds::ArrMeta<float>*>(host) + k;
      method_host[k] = m->method;
      R_host[k] = m->method == DS_METHOD_DIRECT ? m->R : -1;
    } else {
      const auto* m = reinterpret_cast<const ds::ArrMeta<double>*>(host) + k;
      method_host[k] = m->method;
      R_host[k] = m->method == DS_METHOD_DIRECT ? m->R : -1;
    }
  }
  std::free(host);
  return DS_OK;
}

}  // extern "C"
