// Batched ragged build + search: K independent arrays, each with its own
// queries, handled by a fixed sequence of four kernels with no host
// synchronisation and no allocation, so the whole sequence can be captured in
// a HIP graph and replayed.
//
//   1. build_hr    one workgroup per array: validation, minimum rounded gap,
//                  and ComputeHR (Sec. 4.4.3) run entirely on the device: the
//                  workgroup finds the first pair whose cells coincide, one
//                  lane applies the growth steps of the sequential algorithm,
//                  and the scan resumes after that pair; passes repeat until
//                  one changes nothing.
//   2. plan        one workgroup: exclusive scans over the arrays of the table
//                  words, codes and query tiles; arrays whose table would not
//                  fit the workspace fall back to the offset binary search
//                  (Sec. 3.3).  It also clears the tile queues.
//   3. rankcode    one workgroup per Direct array: the RANKCODE layout (bitmap
//                  of occupied cells, running counts, 16-bit position codes).
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

#include "ds_batched_internal.h"
#include "ds_ops.h"

namespace ds {

namespace {

constexpr int kBuildBlock = 1024;
constexpr int kPlanBlock = 1024;
constexpr int kMaxGrowthRounds = 4096;

struct WsLayout {
  size_t meta, tile_off, totals, codes, bits, base, end;
  // learned region (present when nseg > 0)
  size_t lmeta, params, adam_m, adam_v, partial, loss, segs, first, feat, route, samples;
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
    L.partial = take(size_t(K) * kBatchLearnParts * P);
    L.loss = take(size_t(K) * kBatchLearnParts * 4);
    L.segs = take(size_t(K) * size_t(nseg) * kSegFitBytes);
    L.first = take(size_t(K) * size_t(nseg + 1) * 4);
    L.feat = take(size_t(total_x) * 4);
    L.route = take(size_t(total_x) * 4);
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
// 1. per-array ComputeHR
// R - jmin + 1 cells at this H exceed cap_cells (0 = no cap)
template <typename T, int FORM>
__device__ __forceinline__ bool over_cap(T H, T W, T X0, T XN, int64_t cap_cells) {
  if (cap_cells <= 0) return false;
  const int64_t cells = static_cast<int64_t>(grid_floor<T, FORM>(XN, H, W, X0)) -
                        static_cast<int64_t>(grid_floor<T, FORM>(X0, H, W, X0)) + 1;
  return cells > cap_cells;
}

template <typename T, int FORM>
__global__ void __launch_bounds__(kBuildBlock) build_hr_kernel(const int64_t* __restrict__ x_off,
                                                               const int64_t* __restrict__ q_off,
                                                               const T* __restrict__ Xp, int64_t cap_cells,
                                                               ArrMeta<T>* __restrict__ meta) {
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ T s_min[kBuildBlock];
  __shared__ uint32_t s_flags[kBuildBlock];
  __shared__ int64_t s_first[kBuildBlock];
  __shared__ T s_H, s_W;
  __shared__ int s_state;  // 0 continue, 1 infeasible
  const int64_t xo = x_off[k];
  const int64_t n_vals = x_off[k + 1] - xo;
  const int64_t N = n_vals - 1;
  const T* X = Xp + xo;
  ArrMeta<T> m{};
  m.x_off = xo;
  m.q_off = q_off[k];
  m.q_end = q_off[k + 1];
  m.N = static_cast<int32_t>(N);
  if (N <= 0) {
    if (tid == 0) {
      m.method = kBmTrivial;
      m.X0 = (N == 0) ? X[0] : T(0);
      meta[k] = m;
    }
    return;
  }
  const T X0 = X[0];
  const T XN = X[N];
  // validation and minimum rounded gap (Sec. 4.4.2)
  T gmin = std::numeric_limits<T>::infinity();
  uint32_t fl = 0;
  for (int64_t i = tid; i < N; i += kBuildBlock) {
    const T a = X[i], b = X[i + 1];
    if (!std::isfinite(a) || !std::isfinite(b)) fl |= 1u;
    if (!(a < b)) fl |= 2u;
    const T da = a - X0, db = b - X0;
    if (!(da < db)) fl |= 4u;
    gmin = std::fmin(gmin, db - da);
  }
  s_min[tid] = gmin;
  s_flags[tid] = fl;
  __syncthreads();
  for (int w = kBuildBlock / 2; w > 0; w >>= 1) {
    if (tid < w) {
      s_min[tid] = std::fmin(s_min[tid], s_min[tid + w]);
      s_flags[tid] |= s_flags[tid + w];
    }
    __syncthreads();
  }
  const uint32_t flags = s_flags[0];
  const T g = s_min[0];
  m.X0 = X0;
  m.XN = XN;
  if (flags & 3u) {
    if (tid == 0) {
      m.method = kBmInvalid;
      meta[k] = m;
    }
    return;
  }
  bool feasible = !(flags & 4u);
  T H = 0, W = 0, P = 0;
  int32_t n_updates = 0;
  if (feasible) {
    const T Hbar = T(1) / g;  // correctly rounded division
    feasible = !std::isinf(Hbar);
    H = next_up_dev(Hbar);
    W = (FORM == DS_FORM_FMA) ? T(H * X0) : T(0);
    feasible = feasible && grid_floor<T, FORM>(XN, H, W, X0) < T(kTwoPowQ);
    // a table already over the Direct cap only grows with H: not Direct, stop here
    feasible = feasible && !over_cap<T, FORM>(H, W, X0, XN, cap_cells);
    P = next_up_dev(H) - H;
  }
  if (feasible) {
    // growth passes (Sec. 4.4.3); every lane keeps H, W, P in step via LDS
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
      int64_t first = N + 1;
      for (int64_t i = i_start + tid; i <= N; i += kBuildBlock) {
        if (grid_floor<T, FORM>(X[i - 1], H, W, X0) == grid_floor<T, FORM>(X[i], H, W, X0)) {
          first = i;
          break;
        }
      }
      s_first[tid] = first;
      __syncthreads();
      for (int w = kBuildBlock / 2; w > 0; w >>= 1) {
        if (tid < w) s_first[tid] = std::min(s_first[tid], s_first[tid + w]);
        __syncthreads();
      }
      const int64_t bad = s_first[0];
      __syncthreads();
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
      m.H = H;
      m.W = W;
      m.R = static_cast<int32_t>(grid_floor<T, FORM>(XN, H, W, X0));
      m.jmin = static_cast<int32_t>(grid_floor<T, FORM>(X0, H, W, X0));
      const int64_t nK = int64_t(m.R) - m.jmin + 1;
      const int64_t nW = (nK + 63) / 64;
      m.nW = static_cast<int32_t>((nW + 3) / 4 * 4);  // keeps every array's words 16-byte aligned
      m.method = DS_METHOD_DIRECT;
      m.n_updates = n_updates;
    } else {
      m.method = DS_METHOD_BSEARCH_OFFSET;
      m.R = -1;
    }
    meta[k] = m;
  }
}

// --------------------------------------------------------------------------
// 2. plan: scans over arrays (one workgroup)
template <typename T>
__global__ void __launch_bounds__(kPlanBlock) plan_kernel(ArrMeta<T>* __restrict__ meta, int32_t K,
                                                          int64_t* __restrict__ tile_off, PlanTotals* __restrict__ tot,
                                                          int64_t words_budget, int64_t tile, int32_t learn,
                                                          int64_t direct_cap_cells, LearnMeta* __restrict__ lmeta) {
  __shared__ int64_t s_w[kPlanBlock], s_c[kPlanBlock], s_t[kPlanBlock], s_l[kPlanBlock];
  __shared__ int64_t carry_w, carry_c, carry_t, carry_l;
  __shared__ unsigned long long s_ltiles;
  const int tid = threadIdx.x;
  if (tid == 0) {
    carry_w = carry_c = carry_t = carry_l = 0;
    s_ltiles = 0;
  }
  if (tid < kNumQueues) {
    tot->queue[tid] = 0;
    tot->lqueue[tid] = 0;
  }
  if (tid == 0) tot->fallbacks = 0;
  // Direct over the per-array table cap is treated like an infeasible array
  for (int32_t k = tid; k < K; k += kPlanBlock) {
    ArrMeta<T>& m = meta[k];
    if (m.method == DS_METHOD_DIRECT && direct_cap_cells > 0 && int64_t(m.R) - m.jmin + 1 > direct_cap_cells)
      m.method = DS_METHOD_BSEARCH_OFFSET;
    if (learn && m.method == DS_METHOD_BSEARCH_OFFSET) m.method = DS_METHOD_LEARNED;
  }
  __syncthreads();
  for (int32_t base = 0; base < K; base += kPlanBlock) {
    const int32_t k = base + tid;
    int64_t nw = 0, nc = 0, nt = 0;
    if (k < K) {
      const ArrMeta<T>& m = meta[k];
      if (m.method == DS_METHOD_DIRECT) {
        nw = m.nW;
        nc = (int64_t(m.N) + 1 + 7) / 8 * 8;
      }
      nt = (m.q_end - m.q_off + tile - 1) / tile;
    }
    s_w[tid] = nw;
    s_c[tid] = nc;
    s_t[tid] = nt;
    __syncthreads();
    // inclusive Hillis-Steele scans
    for (int d = 1; d < kPlanBlock; d <<= 1) {
      int64_t aw = 0, ac = 0, at = 0;
      if (tid >= d) {
        aw = s_w[tid - d];
        ac = s_c[tid - d];
        at = s_t[tid - d];
      }
      __syncthreads();
      s_w[tid] += aw;
      s_c[tid] += ac;
      s_t[tid] += at;
      __syncthreads();
    }
    if (k < K) {
      ArrMeta<T>& m = meta[k];
      const int64_t w0 = carry_w + s_w[tid] - nw;
      const int64_t c0 = carry_c + s_c[tid] - nc;
      const int64_t t0 = carry_t + s_t[tid] - nt;
      m.t_off = t0;
      tile_off[k] = t0;
      if (m.method == DS_METHOD_DIRECT) {
        if (w0 + nw > words_budget) {
          // the table does not fit the workspace
          m.method = learn ? DS_METHOD_LEARNED : DS_METHOD_BSEARCH_OFFSET;
          m.w_off = 0;
          m.c_off = 0;
        } else {
          m.w_off = w0;
          m.c_off = c0;
        }
      }
    }
    __syncthreads();
    // learned arrays take consecutive model slots
    const int64_t isl = (k < K && meta[k].method == DS_METHOD_LEARNED) ? 1 : 0;
    s_l[tid] = isl;
    __syncthreads();
    for (int d = 1; d < kPlanBlock; d <<= 1) {
      const int64_t a = tid >= d ? s_l[tid - d] : 0;
      __syncthreads();
      s_l[tid] += a;
      __syncthreads();
    }
    if (isl) {
      ArrMeta<T>& m = meta[k];
      atomicAdd(&s_ltiles, static_cast<unsigned long long>(nt));
      const int32_t slot = static_cast<int32_t>(carry_l + s_l[tid] - 1);
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
    }
    __syncthreads();
    if (tid == kPlanBlock - 1) {
      carry_w += s_w[tid];
      carry_c += s_c[tid];
      carry_t += s_t[tid];
      carry_l += s_l[tid];
    }
    __syncthreads();
  }
  if (tid == 0) {
    tile_off[K] = carry_t;
    tot->total_tiles = carry_t;
    tot->learned_tiles = static_cast<int64_t>(s_ltiles);
    tot->words_used = carry_w;
    tot->n_learned = static_cast<int32_t>(carry_l);
  }
}

// --------------------------------------------------------------------------
// 3. per-array RANKCODE layout
template <typename T, int FORM>
__global__ void __launch_bounds__(kBuildBlock) rankcode_kernel(const T* __restrict__ Xp, ArrMeta<T>* __restrict__ meta,
                                                               unsigned long long* __restrict__ bits,
                                                               uint32_t* __restrict__ base,
                                                               uint16_t* __restrict__ codes, int64_t words_budget) {
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  const ArrMeta<T> m = meta[k];
  if (m.method != DS_METHOD_DIRECT) return;
  const T* X = Xp + m.x_off;
  const int64_t N = m.N;
  unsigned long long* wb = bits + m.w_off;
  uint32_t* bb = base + m.w_off;
  uint16_t* cb = codes + m.c_off;
  const int64_t nK = int64_t(m.R) - m.jmin + 1;
  const int64_t nWused = (nK + 63) / 64;
  for (int64_t w = tid; w < m.nW; w += kBuildBlock) {
    wb[w] = 0ull;
    bb[w] = static_cast<uint32_t>(N + 1);  // padding words past the last cell
  }
  const int64_t n_codes = (N + 1 + 7) / 8 * 8;
  for (int64_t i = N + 1 + tid; i < n_codes; i += kBuildBlock) cb[i] = 0;
  __syncthreads();
  // Lanes of a wave hold consecutive i, so their cells (and words) are
  // non-decreasing across the wave: a segmented OR over lanes that share a
  // word leaves one atomic per word and wave instead of one per element.
  const int lane = tid & 63;
  for (int64_t i0 = 0; i0 <= N; i0 += kBuildBlock) {
    const int64_t i = i0 + tid;
    const bool valid = i <= N;
    int64_t word = -1 - lane;  // distinct per invalid lane: never merges
    unsigned long long bitv = 0;
    if (valid) {
      const T x = X[i];
      const T v = grid_value<T, FORM>(x, m.H, m.W, m.X0);
      const T jf = std::floor(v);
      const int64_t e = static_cast<int64_t>(jf) - m.jmin;
      const int64_t eprev =
          (i == 0) ? -1 : static_cast<int64_t>(grid_floor<T, FORM>(X[i - 1], m.H, m.W, m.X0)) - m.jmin;
      if (e >= 0 && e < nK) {
        word = e >> 6;
        bitv = 1ull << (e & 63);
      }
      // running counts: words whose first cell lies in (e_{i-1}, e_i] start at i
      for (int64_t w = (eprev + 1 + 63) / 64; w <= e / 64 && w < nWused; ++w) bb[w] = static_cast<uint32_t>(i);
      const T c = cell_code<T>(v, jf);
      const T p = std::nextafter(x, -std::numeric_limits<T>::infinity());
      const T vp = grid_value<T, FORM>(p, m.H, m.W, m.X0);
      const T jp = std::floor(vp);
      const int first = (jp == jf && cell_code<T>(vp, jp) == c) ? 0 : 1;
      cb[i] = static_cast<uint16_t>((static_cast<int>(c) << 1) | first);
    }
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned long long ob = __shfl_down(bitv, off, 64);
      const long long ow = __shfl_down(static_cast<long long>(word), off, 64);
      if (lane + off < 64 && ow == word) bitv |= ob;
    }
    const long long wprev = __shfl_up(static_cast<long long>(word), 1, 64);
    const bool head = (lane == 0) || (wprev != word);
    if (valid && head && bitv) atomicOr(&wb[word], bitv);
  }
  (void)words_budget;
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

template <typename T, int QPT, class Op>
__device__ __forceinline__ void run_tile(const T* __restrict__ z, int32_t* __restrict__ out, int64_t q0, int64_t q1,
                                         const Op& op) {
  const int64_t B = blockDim.x;
  int64_t q = q0 + threadIdx.x;
  for (; q + (QPT - 1) * B < q1; q += QPT * B) {
    T v[QPT];
#pragma unroll
    for (int u = 0; u < QPT; ++u) v[u] = __builtin_nontemporal_load(z + q + u * B);
#pragma unroll
    for (int u = 0; u < QPT; ++u) __builtin_nontemporal_store(op(v[u]), out + q + u * B);
  }
  for (; q < q1; q += B) out[q] = op(z[q]);
}

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
  __shared__ int64_t s_tile;
  __shared__ int32_t s_k;
  const int queue = blockIdx.x % kNumQueues;
  const int64_t total = tot->total_tiles;
  if (tot->learned_tiles == total) return;  // every tile belongs to a learned array
  int32_t cur = -1;
  bool staged = false;
  for (;;) {
    if (threadIdx.x == 0) {
      const int64_t li = atomicAdd(&tot->queue[queue], 1u);
      const int64_t ch = sh.chunk;
      const int64_t g = ((li / ch) * kNumQueues + queue) * ch + (li % ch);
      int32_t k = -1;
      if (g < total) {
        // last array whose first tile is <= g
        int32_t lo = 0, hi = K - 1;
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if (tile_off[mid] <= g)
            lo = mid;
          else
            hi = mid - 1;
        }
        k = lo;
      }
      s_tile = g;
      s_k = k;
    }
    __syncthreads();
    const int64_t g = s_tile;
    const int32_t k = s_k;
    __syncthreads();  // s_tile is rewritten in the next round
    if (g >= total) break;
    const ArrMeta<T>& m = meta[k];
    const int64_t q0 = m.q_off + (g - m.t_off) * sh.tile;
    const int64_t q1 = std::min(m.q_end, q0 + sh.tile);
    const int64_t N = m.N;
    if (m.method == DS_METHOD_DIRECT) {
      const int64_t nW = m.nW;
      const int64_t code_bytes = round16((N + 1) * 2);
      const int64_t base_off = round16(nW * 8);
      const int64_t code_off = base_off + round16(nW * 4);
      const bool fits = code_off + code_bytes <= sh.lds_budget;
      if (k != cur) {
        if (fits) {
          __syncthreads();
          stage_bytes(smem, reinterpret_cast<const unsigned char*>(bits + m.w_off), nW * 8);
          stage_bytes(smem + base_off, reinterpret_cast<const unsigned char*>(base + m.w_off), nW * 4);
          stage_bytes(smem + code_off, reinterpret_cast<const unsigned char*>(codes + m.c_off), code_bytes);
          __syncthreads();
        }
        cur = k;
        staged = fits;
      }
      const T vlo = T(m.jmin), vhi = T(m.R);
      if (staged) {
        RankCodeOp<T, FORM, false> op{reinterpret_cast<const uint64_t*>(smem),
                                      reinterpret_cast<const uint32_t*>(smem + base_off), nullptr,
                                      reinterpret_cast<const uint16_t*>(smem + code_off), Xp + m.x_off, m.H, m.W,
                                      m.X0, vlo, vhi, m.XN, m.jmin, m.N};
        run_tile<T, QPT>(z, out, q0, q1, op);
      } else {
        RankCodeOp<T, FORM, false> op{reinterpret_cast<const uint64_t*>(bits + m.w_off), base + m.w_off, nullptr,
                                      codes + m.c_off, Xp + m.x_off, m.H, m.W, m.X0, vlo, vhi, m.XN, m.jmin, m.N};
        run_tile<T, QPT>(z, out, q0, q1, op);
      }
    } else if (m.method == DS_METHOD_LEARNED) {
      continue;  // searched by the learned kernel
    } else if (m.method == DS_METHOD_BSEARCH_OFFSET) {
      const bool fits = (N + 1) * int64_t(sizeof(T)) <= sh.lds_budget;
      if (k != cur) {
        if (fits) {
          __syncthreads();
          stage_values(reinterpret_cast<T*>(smem), Xp + m.x_off, N + 1);
          __syncthreads();
        }
        cur = k;
        staged = fits;
      }
      const int32_t F = static_cast<int32_t>((N + 1) / 2);
      const int32_t S = static_cast<int32_t>(N + 1 - F);
      int32_t J = 0;
      while ((int64_t(1) << (J + 1)) <= N + 1) ++J;
      OffsetOp<T> op{staged ? reinterpret_cast<const T*>(smem) : Xp + m.x_off, F, S, J};
      run_tile<T, QPT>(z, out, q0, q1, op);
    } else {
      const int32_t fill = (m.method == kBmInvalid) ? -2 : -1;
      const bool one = (m.method == kBmTrivial && N == 0);
      const T x0 = m.X0;
      for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) out[q] = (one && z[q] >= x0) ? 0 : fill;
    }
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
ds_status launch_plan(const ds_batch_desc* d, const WsLayout& L, unsigned char* ws, int64_t tile, hipStream_t s) {
  const int64_t cap_cells = d->direct_cap_bytes > 0 ? d->direct_cap_bytes / 4 : 0;
  plan_kernel<T><<<dim3(1), dim3(kPlanBlock), 0, s>>>(
      reinterpret_cast<ArrMeta<T>*>(ws + L.meta), d->num_arrays, reinterpret_cast<int64_t*>(ws + L.tile_off),
      reinterpret_cast<PlanTotals*>(ws + L.totals), L.words_budget, tile, L.nseg > 0 ? 1 : 0, cap_cells,
      L.nseg > 0 ? reinterpret_cast<LearnMeta*>(ws + L.lmeta) : nullptr);
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
  b.steps = d->learn_steps > 0 ? d->learn_steps : 10;
  b.fp32_router = 0;
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
  b.partial = reinterpret_cast<float*>(ws + L.partial);
  b.loss = reinterpret_cast<float*>(ws + L.loss);
  b.segs = ws + L.segs;
  b.first = reinterpret_cast<int32_t*>(ws + L.first);
  b.feat = reinterpret_cast<float*>(ws + L.feat);
  b.route = reinterpret_cast<int32_t*>(ws + L.route);
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
          st = launch_plan<T>(&c, L, ws, sh.tile, s);  // re-plans the tiles and clears the queues
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
  const int32_t K = d->num_arrays;
  unsigned char* ws = static_cast<unsigned char*>(d->workspace_dev);
  const WsLayout L = layout_of(d);
  const int64_t wb = L.words_budget;
  const int64_t tile = tile_of(d);
  auto* meta = reinterpret_cast<ArrMeta<T>*>(ws + L.meta);
  const int64_t cap_cells = d->direct_cap_bytes > 0 ? d->direct_cap_bytes / 4 : 0;
  build_hr_kernel<T, FORM><<<dim3(K), dim3(kBuildBlock), 0, s>>>(d->x_off_dev, d->q_off_dev,
                                                                  static_cast<const T*>(d->X_dev), cap_cells, meta);
  DS_HIP_CHECK(hipGetLastError());
  ds_status st = launch_plan<T>(d, L, ws, tile, s);
  if (st != DS_OK) return st;
  rankcode_kernel<T, FORM><<<dim3(K), dim3(kBuildBlock), 0, s>>>(
      static_cast<const T*>(d->X_dev), meta, reinterpret_cast<unsigned long long*>(ws + L.bits),
      reinterpret_cast<uint32_t*>(ws + L.base), reinterpret_cast<uint16_t*>(ws + L.codes), wb);
  DS_HIP_CHECK(hipGetLastError());
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

}  // namespace ds

extern "C" {

size_t ds_batch_workspace_bytes(int32_t num_arrays, int64_t total_x, int64_t table_budget_entries,
                                int32_t learn_segments) {
  if (num_arrays < 0 || total_x < 0 || table_budget_entries < 0 || learn_segments < 0 || learn_segments > 8192)
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
  if (d->learn_segments < 0 || d->learn_segments > 8192 || d->learn_steps < 0 || d->direct_cap_bytes < 0)
    return DS_ERR_ARG;
  if (d->workspace_bytes < ds_batch_workspace_bytes(d->num_arrays, d->total_x, 0, d->learn_segments))
    return DS_ERR_ARG;
  if (d->dtype == DS_F32)
    return d->form == DS_FORM_FMA ? ds::run_batched<float, DS_FORM_FMA>(d, s) : ds::run_batched<float, DS_FORM_SUB>(d, s);
  return d->form == DS_FORM_FMA ? ds::run_batched<double, DS_FORM_FMA>(d, s) : ds::run_batched<double, DS_FORM_SUB>(d, s);
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
