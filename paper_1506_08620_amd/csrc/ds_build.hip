// Build of the Direct-search index on the GPU, and the C entry points that
// create, describe and destroy handles.
//
//   a) validation + minimum rounded gap  (Sec. 4.4.2, eq. (distinguishable-exact)
//      and eq. (minhnumeric)): one pass over X, a block-min reduction and flag OR.
//   b) H growth (Sec. 4.4.3, algorithm ComputeHR): the host owns the scalar
//      recurrence; a parallel kernel finds the first pair i >= i_start whose
//      grid cells coincide under the current H, so the host applies the growth
//      steps in exactly the order of the sequential algorithm.  Passes repeat
//      until one changes nothing, so every pair holds under the final H.
//      On request the interval between the last failing H and the grown one is
//      then bisected (the refinement proposed at the end of Sec. 4.4.3), each
//      midpoint checked by one verify pass over the whole array.
//   c) the table K (Sec. 4, eq. (indexdef)): one workgroup per 256 consecutive
//      X_i computes their cells, then fills the contiguous run of K entries
//      that falls between its first and last cell, each entry found by a
//      binary search over the workgroup's cells in LDS.
#include <algorithm>
#include <chrono>
#include <limits>
#include <new>

#include "ds_internal.h"

namespace ds {

namespace {

constexpr uint32_t kFlagNonFinite = 1u;
constexpr uint32_t kFlagNotSorted = 2u;
constexpr uint32_t kFlagOffsetsNotIncreasing = 4u;

struct BuildScratch {
  unsigned long long min_gap_bits;  // bits of the smallest m(D_{i+1} - D_i) (positive floats order as integers)
  unsigned long long first_bad;     // smallest failing pair index of a verify pass
  uint32_t flags;
  uint32_t pad[3];
};

template <typename T>
struct Bits;
template <>
struct Bits<float> {
  using U = uint32_t;
};
template <>
struct Bits<double> {
  using U = uint64_t;
};

template <typename T>
__device__ __forceinline__ unsigned long long to_bits(T v) {
  typename Bits<T>::U u;
  __builtin_memcpy(&u, &v, sizeof(T));
  return static_cast<unsigned long long>(u);
}

template <typename T>
T from_bits(unsigned long long b) {
  typename Bits<T>::U u = static_cast<typename Bits<T>::U>(b);
  T v;
  std::memcpy(&v, &u, sizeof(T));
  return v;
}

constexpr int kScanBlock = 256;

// One pass over X: finiteness and order of neighbours, and the smallest
// rounded q-gap m(D_{i+q} - D_i) (q = 1 for plain Direct; Sec. 4.7 for q > 1),
// with a flag when some D_{i+q} <= D_i (no grid can then separate X_i and X_{i+q}).
template <typename T>
__global__ void __launch_bounds__(kScanBlock) mingap_kernel(const T* __restrict__ X, int64_t N, int64_t q,
                                                            BuildScratch* __restrict__ scr) {
  const T X0 = X[0];
  T gmin = std::numeric_limits<T>::infinity();
  uint32_t fl = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    const T a = X[i], b = X[i + 1];
    if (!std::isfinite(a) || !std::isfinite(b)) fl |= kFlagNonFinite;
    if (!(a < b)) fl |= kFlagNotSorted;
    if (i + q <= N) {
      const T da = a - X0, dq = X[i + q] - X0;  // D_i = m(X_i - X_0)
      if (!(da < dq)) fl |= kFlagOffsetsNotIncreasing;
      const T g = dq - da;                     // m(D_{i+q} - D_i)
      gmin = std::fmin(gmin, g);
    }
  }
  __shared__ T smin[kScanBlock];
  __shared__ uint32_t sfl[kScanBlock];
  smin[threadIdx.x] = gmin;
  sfl[threadIdx.x] = fl;
  __syncthreads();
  for (int w = kScanBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smin[threadIdx.x] = std::fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      sfl[threadIdx.x] |= sfl[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (sfl[0]) atomicOr(&scr->flags, sfl[0]);
    const T m = smin[0];
    // only positive gaps matter; a non-positive one is reported through the flags
    if (m > T(0)) atomicMin(&scr->min_gap_bits, to_bits<T>(m));
  }
}

// smallest i in [i_start, N] with floor(f(X_{i-q})) == floor(f(X_i)): eq. (cond2)
// for q = 1, eq. (f-monotonic-n) for q > 1 (i_start >= q)
template <typename T, int FORM>
__global__ void __launch_bounds__(kScanBlock) verify_kernel(const T* __restrict__ X, int64_t N, int64_t q,
                                                            int64_t i_start, T H, T W, T X0,
                                                            BuildScratch* __restrict__ scr) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long first = ~0ull;
  for (int64_t i = i_start + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= N; i += stride) {
    const T a = grid_floor<T, FORM>(X[i - q], H, W, X0);
    const T b = grid_floor<T, FORM>(X[i], H, W, X0);
    if (a == b) {
      first = static_cast<unsigned long long>(i);
      break;  // later i of this thread are larger
    }
  }
  if (first != ~0ull) atomicMin(&scr->first_bad, first);
}

constexpr int kFillBlock = 256;

// K_j = min{ i : f(X_i) >= j } for j in [jmin, R]; K[e] holds K_{jmin+e}.
template <typename T, int FORM>
__global__ void __launch_bounds__(kFillBlock) fill_kernel(const T* __restrict__ X, int64_t N, T H, T W, T X0,
                                                          int32_t jmin, int64_t nK, int32_t* __restrict__ K) {
  __shared__ int32_t c[kFillBlock + 1];  // c[0] = f(X_{i0-1}) (jmin-1 for i0 = 0), c[1+t] = f(X_{i0+t})
  const int64_t i0 = (int64_t)blockIdx.x * kFillBlock;
  const int64_t i = i0 + threadIdx.x;
  if (i <= N) c[1 + threadIdx.x] = static_cast<int32_t>(grid_floor<T, FORM>(X[i], H, W, X0));
  if (threadIdx.x == 0)
    c[0] = (i0 == 0) ? jmin - 1 : static_cast<int32_t>(grid_floor<T, FORM>(X[i0 - 1], H, W, X0));
  __syncthreads();
  const int nb = static_cast<int>(std::min<int64_t>(kFillBlock, N + 1 - i0));
  const int64_t jlo = (int64_t)c[0] + 1, jhi = c[nb];
  for (int64_t j = jlo + threadIdx.x; j <= jhi; j += kFillBlock) {
    int lo = 1, hi = nb;  // smallest t in [1, nb] with c[t] >= j
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((int64_t)c[mid] >= j)
        hi = mid;
      else
        lo = mid + 1;
    }
    const int64_t e = j - jmin;
    if (e >= 0 && e < nK) K[e] = static_cast<int32_t>(i0 + lo - 1);  // always true when f is monotone
  }
}

// ---------------------------------------------------------------------------
// The whole Direct build of a small array in one workgroup and one launch, so
// that ds_build makes one allocation and reads one result record: the copy of
// X, validation and the smallest rounded gap (as mingap_kernel), ComputeHR
// (Sec. 4.4.3) as compute_hr does it -- the start value, then passes that
// find the first pair from i on whose cells coincide, grow H at that pair by
// P (doubled after each step, never reset) and go on after it, until a pass
// grows nothing -- then R, jmin and, when it fits kcap cells, the table K
// (eq. (indexdef): i is written into the cells (f(X_{i-1}), f(X_i)]).  The
// same floating-point operations in the same order as the multi-launch build,
// so H, W, R, jmin and K are identical.
constexpr int kSmallBlock = 1024;
constexpr int64_t kSmallBuildMax = 65537;  // values (N + 1) of the one-workgroup build

template <typename T>
struct SmallResult {
  T H, W, X0, XN;
  int64_t R, jmin, n_updates;
  int32_t status;   // ds_status
  int32_t filled;   // K was written (R - jmin + 1 <= kcap)
};

template <typename T, int FORM>
__global__ void __launch_bounds__(kSmallBlock) small_build_kernel(const T* __restrict__ Xin, int64_t N, int32_t hstart,
                                                                  T* __restrict__ X, SmallResult<T>* __restrict__ res,
                                                                  int32_t* __restrict__ K, int64_t kcap) {
  const int tid = threadIdx.x;
  __shared__ T s_min[kSmallBlock / 64];
  __shared__ uint32_t s_fl[kSmallBlock / 64];
  __shared__ unsigned long long s_first;
  __shared__ T s_H, s_W;
  __shared__ int32_t s_status;
  for (int64_t i = tid; i <= N; i += kSmallBlock) X[i] = Xin[i];
  __syncthreads();
  const T X0 = X[0], XN = X[N];
  // validation flags and the smallest rounded gap m(D_{i+1} - D_i)
  T gmin = std::numeric_limits<T>::infinity();
  uint32_t fl = 0;
  for (int64_t i = tid; i < N; i += kSmallBlock) {
    const T a = X[i], b = X[i + 1];
    if (!std::isfinite(a) || !std::isfinite(b)) fl |= kFlagNonFinite;
    if (!(a < b)) fl |= kFlagNotSorted;
    const T da = a - X0, db = b - X0;
    if (!(da < db)) fl |= kFlagOffsetsNotIncreasing;
    gmin = std::fmin(gmin, db - da);
  }
  for (int o = 32; o > 0; o >>= 1) {
    gmin = std::fmin(gmin, __shfl_xor(gmin, o, 64));
    fl |= __shfl_xor(fl, o, 64);
  }
  if ((tid & 63) == 0) {
    s_min[tid >> 6] = gmin;
    s_fl[tid >> 6] = fl;
  }
  __syncthreads();
  if (tid == 0) {
    T g = std::numeric_limits<T>::infinity();
    uint32_t f = 0;
    for (int w = 0; w < kSmallBlock / 64; ++w) {
      g = std::fmin(g, s_min[w]);
      f |= s_fl[w];
    }
    int32_t st = DS_OK;
    if (f & kFlagNonFinite) st = DS_ERR_NONFINITE;
    else if (f & kFlagNotSorted) st = DS_ERR_NOT_SORTED;
    else if (f & kFlagOffsetsNotIncreasing) st = DS_ERR_INFEASIBLE;
    T H = 0, W = 0;
    if (st == DS_OK) {
      const T Hbar = T(1) / g;  // eq. (minhnumeric), correctly rounded
      if (std::isinf(Hbar)) st = DS_ERR_INFEASIBLE;
      H = (hstart == DS_HSTART_HBAR) ? Hbar : std::nextafter(Hbar, std::numeric_limits<T>::infinity());
      W = (FORM == DS_FORM_FMA) ? T(H * X0) : T(0);
      if (st == DS_OK && grid_floor<T, FORM>(XN, H, W, X0) >= T(kTwoPowQ)) st = DS_ERR_INFEASIBLE;
    }
    s_H = H;
    s_W = W;
    s_status = st;
  }
  __syncthreads();
  T P = std::nextafter(s_H, std::numeric_limits<T>::infinity()) - s_H;  // used by thread 0 only
  int64_t n_updates = 0;
  for (;;) {  // passes until none grows H (the same for every thread: shared values)
    if (s_status != DS_OK) break;
    bool changed = false;
    int64_t i_start = 1;
    while (i_start <= N) {
      if (tid == 0) s_first = ~0ull;
      __syncthreads();
      const T H = s_H, W = s_W;
      for (int64_t i = i_start + tid; i <= N; i += kSmallBlock) {
        if (grid_floor<T, FORM>(X[i - 1], H, W, X0) == grid_floor<T, FORM>(X[i], H, W, X0)) {
          atomicMin(&s_first, static_cast<unsigned long long>(i));
          break;  // later i of this thread are larger
        }
      }
      __syncthreads();
      const unsigned long long f = s_first;
      if (f == ~0ull) break;
      const int64_t i = static_cast<int64_t>(f);
      if (tid == 0) {
        T Hc = H, Wc = W;
        const T a = X[i - 1], b = X[i];
        while (grid_floor<T, FORM>(a, Hc, Wc, X0) == grid_floor<T, FORM>(b, Hc, Wc, X0)) {
          Hc = Hc + P;
          if (FORM == DS_FORM_FMA) Wc = Hc * X0;
          if (grid_floor<T, FORM>(XN, Hc, Wc, X0) >= T(kTwoPowQ)) {  // eq. (overflowexact)
            s_status = DS_ERR_INFEASIBLE;
            break;
          }
          P = P + P;
          ++n_updates;
        }
        s_H = Hc;
        s_W = Wc;
      }
      changed = true;
      __syncthreads();
      if (s_status != DS_OK) break;
      i_start = i + 1;
    }
    if (!changed) break;
  }
  __syncthreads();
  const T H = s_H, W = s_W;
  const int32_t st = s_status;
  const int64_t R = st == DS_OK ? static_cast<int64_t>(grid_floor<T, FORM>(XN, H, W, X0)) : 0;
  const int64_t jmin = st == DS_OK ? static_cast<int64_t>(grid_floor<T, FORM>(X0, H, W, X0)) : 0;
  const bool fill = st == DS_OK && R - jmin + 1 <= kcap;
  if (fill) {
    for (int64_t i = tid; i <= N; i += kSmallBlock) {
      const int64_t hi = static_cast<int64_t>(grid_floor<T, FORM>(X[i], H, W, X0));
      const int64_t lo = (i == 0) ? jmin : static_cast<int64_t>(grid_floor<T, FORM>(X[i - 1], H, W, X0)) + 1;
      for (int64_t j = lo; j <= hi; ++j) K[j - jmin] = static_cast<int32_t>(i);
    }
  }
  if (tid == 0) {
    SmallResult<T> r{};
    r.H = H;
    r.W = W;
    r.X0 = X0;
    r.XN = XN;
    r.R = R;
    r.jmin = jmin;
    r.n_updates = n_updates;
    r.status = st;
    r.filled = fill ? 1 : 0;
    *res = r;
  }
}

// K_j = max{ i : f(X_i) <= j } for j in [jmin, R] (eq. (kgeneral), Sec. 4.7);
// K[e] holds K_{jmin+e}.  The workgroup of X_{i0..i0+255} owns the cells from
// f(X_{i0}) up to the one before f(X_{i0+256}) (up to R for the last
// workgroup), and finds each entry by a binary search over its cells in LDS.
template <typename T, int FORM>
__global__ void __launch_bounds__(kFillBlock) fill_max_kernel(const T* __restrict__ X, int64_t N, T H, T W, T X0,
                                                              int32_t jmin, int64_t R, int64_t nK,
                                                              int32_t* __restrict__ K) {
  __shared__ int32_t c[kFillBlock];  // c[t] = f(X_{i0+t})
  __shared__ int64_t jnext;
  const int64_t i0 = (int64_t)blockIdx.x * kFillBlock;
  const int64_t i = i0 + threadIdx.x;
  if (i <= N) c[threadIdx.x] = static_cast<int32_t>(grid_floor<T, FORM>(X[i], H, W, X0));
  if (threadIdx.x == 0)
    jnext = (i0 + kFillBlock <= N) ? static_cast<int64_t>(grid_floor<T, FORM>(X[i0 + kFillBlock], H, W, X0)) : R + 1;
  __syncthreads();
  const int nb = static_cast<int>(std::min<int64_t>(kFillBlock, N + 1 - i0));
  for (int64_t j = (int64_t)c[0] + threadIdx.x; j < jnext; j += kFillBlock) {
    int lo = 0, hi = nb - 1;  // largest t in [0, nb - 1] with c[t] <= j (c[0] <= j)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((int64_t)c[mid] <= j)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t e = j - jmin;
    if (e >= 0 && e < nK) K[e] = static_cast<int32_t>(i0 + lo);  // always true when f is monotone
  }
}

// Xp[0..count-1] = Xp[count]: the left padding of the gap-q search, copies of X_0
template <typename T>
__global__ void pad_left_kernel(T* __restrict__ Xp, int64_t count) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) Xp[k] = Xp[count];
}

// RANKCODE bitmap: one wave per 64 cells.  Cell e holds an X_i exactly when
// K_{e+1} > K_e (K counts the X_i of earlier cells); the last cell holds X_N.
__global__ void __launch_bounds__(256) rank_bits_kernel(const int32_t* __restrict__ K, int64_t nK, int64_t nW,
                                                        uint64_t* __restrict__ bits, uint32_t* __restrict__ base,
                                                        RcWord* __restrict__ w16) {
  const int lane = threadIdx.x & 63;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= nW) return;  // uniform across the wave
  const int64_t e = w * 64 + lane;
  bool occupied = false;
  if (e < nK - 1)
    occupied = K[e + 1] != K[e];
  else if (e == nK - 1)
    occupied = true;
  const uint64_t m = __ballot(occupied);
  if (lane == 0) {
    const uint32_t b0 = static_cast<uint32_t>(K[w * 64]);
    bits[w] = m;
    base[w] = b0;
    RcWord rw;
    rw.bits = m;
    rw.base = b0;
    rw.pad = 0;
    w16[w] = rw;
  }
}

// GAPCODE words (gap-q grid, q <= 15): CB-bit key counts of the L = 64 / CB
// cells jmin + L w .. jmin + L w + L - 1 (the count of cell e is K_e - K_(e-1),
// K_(jmin-1) = -1 with K_j = max{i : f(X_i) <= j}) and the number of keys in
// earlier cells, K_(jmin + L w - 1) + 1.
__global__ void __launch_bounds__(256) gap_words_kernel(const int32_t* __restrict__ K, int64_t nK, int64_t nW,
                                                        int32_t cb, uint64_t* __restrict__ counts,
                                                        uint32_t* __restrict__ base) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nW) return;
  const int L = 64 / cb;
  uint64_t m = 0;
  for (int b = 0; b < L; ++b) {
    const int64_t e = w * L + b;
    if (e >= nK) break;
    const int32_t c = K[e] - (e > 0 ? K[e - 1] : -1);
    m |= static_cast<uint64_t>(c) << (cb * b);
  }
  counts[w] = m;
  base[w] = (w == 0) ? 0u : static_cast<uint32_t>(K[w * L - 1] + 1);
}

// RANKCODE codes: 15-bit position of X_i in its cell, and a flag set when no
// smaller float shares the cell and the position code of X_i.
template <typename T, int FORM>
__global__ void __launch_bounds__(256) rank_code_kernel(const T* __restrict__ X, int64_t N, int64_t n_alloc, T H,
                                                        T W, T X0, uint16_t* __restrict__ code) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_alloc) return;
  if (i > N) {
    code[i] = 0;
    return;
  }
  const T x = X[i];
  const T v = grid_value<T, FORM>(x, H, W, X0);
  const T jf = std::floor(v);
  const T c = cell_code<T>(v, jf);
  const T p = std::nextafter(x, -std::numeric_limits<T>::infinity());
  const T vp = grid_value<T, FORM>(p, H, W, X0);
  const T jp = std::floor(vp);
  const T cp = cell_code<T>(vp, jp);
  const int first = (jp == jf && cp == c) ? 0 : 1;
  code[i] = static_cast<uint16_t>((static_cast<int>(c) << 1) | first);
}

// the same codes with 7 bits of position, for the layout read through L2
template <typename T, int FORM>
__global__ void __launch_bounds__(256) rank_code8_kernel(const T* __restrict__ X, int64_t N, int64_t n_alloc, T H,
                                                         T W, T X0, uint8_t* __restrict__ code) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_alloc) return;
  if (i > N) {
    code[i] = 0;
    return;
  }
  const T x = X[i];
  const T v = grid_value<T, FORM>(x, H, W, X0);
  const T jf = std::floor(v);
  const T c = cell_code<T, 7>(v, jf);
  const T p = std::nextafter(x, -std::numeric_limits<T>::infinity());
  const T vp = grid_value<T, FORM>(p, H, W, X0);
  const T jp = std::floor(vp);
  const int first = (jp == jf && cell_code<T, 7>(vp, jp) == c) ? 0 : 1;
  code[i] = static_cast<uint8_t>((static_cast<int>(c) << 1) | first);
}

// NIBBLE chunks: one thread per 24 cells.  Cell e holds X_{K_e} exactly when
// K_{e+1} > K_e (the last cell holds X_N); its nibble codes the bin of
// X_{K_e} in the cell and, for f32, the first-of-class flag (NibCode).
template <typename T, int FORM>
__global__ void __launch_bounds__(256) nibble_kernel(const T* __restrict__ X, const int32_t* __restrict__ K, int64_t nK,
                                                     int64_t n_chunks, T H, T W, T X0, NibChunk* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_chunks) return;
  const int64_t e0 = k * kNibCells;
  NibChunk ch{};
  ch.base = static_cast<uint32_t>(K[e0]);  // e0 < nK for every chunk
  for (int c = 0; c < kNibCells; ++c) {
    const int64_t e = e0 + c;
    bool occupied = false;
    if (e < nK - 1)
      occupied = K[e + 1] != K[e];
    else if (e == nK - 1)
      occupied = true;
    if (!occupied) continue;
    const T x = X[K[e]];
    const T v = grid_value<T, FORM>(x, H, W, X0);
    const T jf = std::floor(v);
    const uint32_t b = static_cast<uint32_t>(cell_bin(v, jf));
    uint32_t nib = 1u + b;
    if constexpr (NibCode<T>::kFlag) {
      const T p = std::nextafter(x, -std::numeric_limits<T>::infinity());
      const T vp = grid_value<T, FORM>(p, H, W, X0);
      const T jp = std::floor(vp);
      const uint32_t first = (jp == jf && static_cast<uint32_t>(cell_bin(vp, jp)) == b) ? 0u : 1u;
      nib = 1u + 2u * b + first;
    }
    ch.nib[c >> 3] |= nib << (4 * (c & 7));
  }
  out[k] = ch;
}

template <typename T>
__global__ void __launch_bounds__(256) pairs_kernel(const T* __restrict__ X, const int32_t* __restrict__ K, int64_t nK,
                                                    CachePair<T>* __restrict__ pairs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nK) return;
  CachePair<T> p{};
  p.t = K[e];
  p.x = X[p.t];
  pairs[e] = p;
}

// leading-bit padding (Sec. 3.2.1): X_N repeated up to 2^p entries
template <typename T>
__global__ void pad_kernel(T* __restrict__ Xp, int64_t from, int64_t to, T value) {
  const int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < to) Xp[i] = value;
}

int64_t grid_for(int64_t n, int block, int64_t cap) {
  int64_t g = (n + block - 1) / block;
  return std::max<int64_t>(1, std::min(g, cap));
}

template <typename T>
T next_up(T x) {
  return std::nextafter(x, std::numeric_limits<T>::infinity());
}

// The host half of ComputeHR for one form; see the file comment.  q = 1 is
// plain Direct; q > 1 checks the pairs (X_{i-q}, X_i) of Sec. 4.7 instead of
// neighbours, starting from the smallest rounded q-gap g.
template <typename T, int FORM>
ds_status compute_hr(ds_index* h, const T* X, int64_t q, BuildScratch* scr, hipStream_t s, T X0, T XN, T g) {
  const int64_t N = h->N;
  const T one = T(1);
  const T Hbar = one / g;  // eq. (minhnumeric), correctly rounded
  if (std::isinf(Hbar)) return DS_ERR_INFEASIBLE;
  T H = (h->hstart == DS_HSTART_HBAR) ? Hbar : next_up(Hbar);
  T W = (FORM == DS_FORM_FMA) ? T(H * X0) : T(0);
  auto overflow = [&](T Hc, T Wc) { return grid_floor<T, FORM>(XN, Hc, Wc, X0) >= T(kTwoPowQ); };
  if (overflow(H, W)) return DS_ERR_INFEASIBLE;  // eq. (overflowexact)
  T P = next_up(H) - H;
  int64_t n_updates = 0;
  T Hbad = T(0);  // last H seen to fail a pair; 0 = none
  const int64_t vgrid = std::min<int64_t>(grid_for(N, kScanBlock, 1 << 20), int64_t(num_cus()) * 8);
  // smallest failing pair index >= i_start under (Hc, Wc), or -1
  auto first_bad_from = [&](int64_t i_start, T Hc, T Wc, int64_t* first) -> ds_status {
    const unsigned long long none = ~0ull;
    DS_HIP_CHECK(hipMemcpyAsync(&scr->first_bad, &none, sizeof(none), hipMemcpyHostToDevice, s));
    verify_kernel<T, FORM><<<dim3((unsigned)vgrid), dim3(kScanBlock), 0, s>>>(X, N, q, i_start, Hc, Wc, X0, scr);
    DS_HIP_CHECK(hipGetLastError());
    unsigned long long f = 0;
    DS_HIP_CHECK(hipMemcpyAsync(&f, &scr->first_bad, sizeof(f), hipMemcpyDeviceToHost, s));
    DS_HIP_CHECK(hipStreamSynchronize(s));
    *first = (f == none) ? -1 : static_cast<int64_t>(f);
    return DS_OK;
  };
  for (;;) {
    bool changed = false;
    int64_t i_start = q;
    while (i_start <= N) {
      int64_t i = -1;
      ds_status st = first_bad_from(i_start, H, W, &i);
      if (st != DS_OK) return st;
      if (i < 0) break;
      T pair[2];
      DS_HIP_CHECK(hipMemcpyAsync(&pair[0], X + (i - q), sizeof(T), hipMemcpyDeviceToHost, s));
      DS_HIP_CHECK(hipMemcpyAsync(&pair[1], X + i, sizeof(T), hipMemcpyDeviceToHost, s));
      DS_HIP_CHECK(hipStreamSynchronize(s));
      while (grid_floor<T, FORM>(pair[0], H, W, X0) == grid_floor<T, FORM>(pair[1], H, W, X0)) {
        Hbad = H;
        H = H + P;
        if (FORM == DS_FORM_FMA) W = H * X0;
        if (overflow(H, W)) return DS_ERR_INFEASIBLE;
        P = P + P;
        ++n_updates;
        changed = true;
      }
      i_start = i + 1;
    }
    if (!changed) break;
  }
  // The refinement at the end of Sec. 4.4.3: Hbad fails and H holds; keep that
  // invariant while halving [Hbad, H] until the ends are neighbouring floats.
  int32_t n_refine = 0;
  if (h->refine_h && n_updates > 0) {
    T lo = Hbad;
    for (;;) {
      const T mid = lo + (H - lo) / T(2);
      if (!(lo < mid && mid < H)) break;
      ++n_refine;
      const T Wm = (FORM == DS_FORM_FMA) ? T(mid * X0) : T(0);
      bool ok = !overflow(mid, Wm);
      if (ok) {
        int64_t i = -1;
        ds_status st = first_bad_from(q, mid, Wm, &i);
        if (st != DS_OK) return st;
        ok = i < 0;
      }
      if (ok) {
        H = mid;
        W = Wm;
      } else {
        lo = mid;
      }
    }
  }
  h->H = H;
  h->W = W;
  h->X0 = X0;
  h->XN = XN;
  h->R = static_cast<int64_t>(grid_floor<T, FORM>(XN, H, W, X0));
  h->jmin = static_cast<int64_t>(grid_floor<T, FORM>(X0, H, W, X0));
  h->n_updates = n_updates;
  h->n_refine = n_refine;
  return DS_OK;
}

template <typename T, int FORM>
ds_status fill_table(ds_index* h, hipStream_t s) {
  const int64_t blocks = (h->N + 1 + kFillBlock - 1) / kFillBlock;
  fill_kernel<T, FORM><<<dim3((unsigned)blocks), dim3(kFillBlock), 0, s>>>(
      static_cast<const T*>(h->X), h->N, T(h->H), T(h->W), T(h->X0), static_cast<int32_t>(h->jmin), h->nK, h->K);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

template <typename T, int FORM>
ds_status build_rankcode(ds_index* h, hipStream_t s) {
  const int64_t nW = (h->nK + 63) / 64;
  const int64_t n_codes = ((h->N + 1) + 7) / 8 * 8;
  h->rc_words = nW;
  if (hipMalloc(&h->rc_bits, size_t(nW) * 8) != hipSuccess || hipMalloc(&h->rc_base, size_t(nW) * 4) != hipSuccess ||
      hipMalloc(&h->rc_code, size_t(n_codes) * 2) != hipSuccess ||
      hipMalloc(&h->rc_w16, size_t(nW) * sizeof(RcWord)) != hipSuccess ||
      hipMalloc(&h->rc_code8, size_t(n_codes)) != hipSuccess)
    return DS_ERR_OOM;
  rank_bits_kernel<<<dim3((unsigned)((nW * 64 + 255) / 256)), dim3(256), 0, s>>>(h->K, h->nK, nW, h->rc_bits,
                                                                                    h->rc_base, h->rc_w16);
  DS_HIP_CHECK(hipGetLastError());
  rank_code_kernel<T, FORM><<<dim3((unsigned)((n_codes + 255) / 256)), dim3(256), 0, s>>>(
      static_cast<const T*>(h->X), h->N, n_codes, T(h->H), T(h->W), T(h->X0), h->rc_code);
  rank_code8_kernel<T, FORM><<<dim3((unsigned)((n_codes + 255) / 256)), dim3(256), 0, s>>>(
      static_cast<const T*>(h->X), h->N, n_codes, T(h->H), T(h->W), T(h->X0), h->rc_code8);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

template <typename T, int FORM>
ds_status build_nibble(ds_index* h, hipStream_t s) {
  const int64_t n = nibble_chunks(h->nK);
  if (hipMalloc(&h->nib, size_t(n) * sizeof(NibChunk)) != hipSuccess) {
    h->nib = nullptr;
    return DS_ERR_OOM;
  }
  h->nib_chunks = n;
  nibble_kernel<T, FORM><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(
      static_cast<const T*>(h->X), h->K, h->nK, n, T(h->H), T(h->W), T(h->X0), h->nib);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

template <typename T>
ds_status build_pairs(ds_index* h, hipStream_t s) {
  if (hipMalloc(&h->pairs, size_t(h->nK) * sizeof(CachePair<T>)) != hipSuccess) {
    h->pairs = nullptr;
    return DS_ERR_OOM;
  }
  pairs_kernel<T><<<dim3((unsigned)((h->nK + 255) / 256)), dim3(256), 0, s>>>(
      static_cast<const T*>(h->X), h->K, h->nK, static_cast<CachePair<T>*>(h->pairs));
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

// Which layouts to build: the one the automatic launch will use (PLAIN in LDS
// when it fits, else RANKCODE in LDS when it fits, else NIBBLE in LDS when its
// chunks fit, else NIBBLE through L2 with a prefix in LDS: one cache line of
// table per query, against about 1.5 for RANKCODE through L2 and 2 for
// PAIRS), plus whatever the caller asked for.
template <typename T>
ds_status build_layouts(ds_index* h, const ds_build_opts& o, hipStream_t s) {
  h->staged = tables_fit_lds(h) ? 1 : 0;
  const int64_t nW = (h->nK + 63) / 64;
  h->rc_words = nW;
  const bool rc_fits = rankcode_lds_bytes(h) <= kLdsBytesPerCU;
  const bool nib_fits = nibble_chunks(h->nK) * int64_t(sizeof(NibChunk)) <= kLdsBytesPerCU;
  h->auto_stage = h->staged ? 1 : (rc_fits ? 3 : (nib_fits ? 7 : 6));
  const bool want_rc = (o.extra_layouts & DS_LAYOUT_RANKCODE) || h->auto_stage == 3 || h->auto_stage == 5;
  const bool want_pairs = (o.extra_layouts & DS_LAYOUT_PAIRS) || h->auto_stage == 4;
  const bool want_nib = (o.extra_layouts & DS_LAYOUT_NIBBLE) || h->auto_stage == 6 || h->auto_stage == 7;
  if (want_nib) {
    ds_status st = (h->form == DS_FORM_FMA) ? build_nibble<T, DS_FORM_FMA>(h, s) : build_nibble<T, DS_FORM_SUB>(h, s);
    if (st != DS_OK) return st;
  }
  if (want_rc) {
    ds_status st = (h->form == DS_FORM_FMA) ? build_rankcode<T, DS_FORM_FMA>(h, s) : build_rankcode<T, DS_FORM_SUB>(h, s);
    if (st != DS_OK) return st;
  }
  if (want_pairs) {
    ds_status st = build_pairs<T>(h, s);
    if (st != DS_OK) return st;
  }
  return DS_OK;
}

template <typename T>
ds_status build_direct(ds_index* h, const ds_build_opts& o, hipStream_t s) {
  const T* X = static_cast<const T*>(h->X);
  const int64_t N = h->N;
  BuildScratch* scr = nullptr;
  if (hipMalloc(&scr, sizeof(BuildScratch)) != hipSuccess) return DS_ERR_OOM;
  struct Free {
    BuildScratch* p;
    ~Free() { (void)hipFree(p); }
  } guard{scr};
  BuildScratch init{};
  init.min_gap_bits = ~0ull;
  init.first_bad = ~0ull;
  DS_HIP_CHECK(hipMemcpyAsync(scr, &init, sizeof(init), hipMemcpyHostToDevice, s));
  const int64_t grid = std::min<int64_t>(grid_for(N, kScanBlock, 1 << 20), int64_t(num_cus()) * 8);
  mingap_kernel<T><<<dim3((unsigned)grid), dim3(kScanBlock), 0, s>>>(X, N, 1, scr);
  DS_HIP_CHECK(hipGetLastError());
  BuildScratch got{};
  T ends[2];
  DS_HIP_CHECK(hipMemcpyAsync(&got, scr, sizeof(got), hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipMemcpyAsync(&ends[0], X, sizeof(T), hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipMemcpyAsync(&ends[1], X + N, sizeof(T), hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipStreamSynchronize(s));
  if (got.flags & kFlagNonFinite) return DS_ERR_NONFINITE;
  if (got.flags & kFlagNotSorted) return DS_ERR_NOT_SORTED;
  if (got.flags & kFlagOffsetsNotIncreasing) return DS_ERR_INFEASIBLE;
  const T g = from_bits<T>(got.min_gap_bits);
  ds_status st = (h->form == DS_FORM_FMA) ? compute_hr<T, DS_FORM_FMA>(h, X, 1, scr, s, ends[0], ends[1], g)
                                          : compute_hr<T, DS_FORM_SUB>(h, X, 1, scr, s, ends[0], ends[1], g);
  if (st != DS_OK) return st;
  h->nK = h->R - h->jmin + 1;
  const int64_t cap = o.table_cap_bytes > 0 ? o.table_cap_bytes : kDefaultTableCap;
  if (h->nK * int64_t(sizeof(int32_t)) > cap) return DS_ERR_TABLE_CAP;
  if (hipMalloc(&h->K, size_t(h->nK) * sizeof(int32_t)) != hipSuccess) {
    h->K = nullptr;
    return DS_ERR_OOM;
  }
  st = (h->form == DS_FORM_FMA) ? fill_table<T, DS_FORM_FMA>(h, s) : fill_table<T, DS_FORM_SUB>(h, s);
  if (st != DS_OK) return st;
  st = build_layouts<T>(h, o, s);
  if (st != DS_OK) return st;
  DS_HIP_CHECK(hipStreamSynchronize(s));
  return DS_OK;
}

// Direct build of an array of at most kSmallBuildMax values: one allocation
// holds the copy of X, the result record and room for a table of
// max(4 (N + 1), 16384) cells; small_build_kernel does the rest, and the host
// reads the record once.  A table larger than the room gets its own
// allocation and the usual fill.
template <typename T>
ds_status build_direct_small(ds_index* h, const ds_build_opts& o, const void* X_dev, hipStream_t s) {
  const int64_t N = h->N;
  const int64_t cap = o.table_cap_bytes > 0 ? o.table_cap_bytes : kDefaultTableCap;
  const int64_t kcap = std::min<int64_t>(std::max<int64_t>(4 * (N + 1), 16384), cap / int64_t(sizeof(int32_t)));
  const size_t x_bytes = (size_t(N + 1) * sizeof(T) + 255) / 256 * 256;
  const size_t r_bytes = (sizeof(SmallResult<T>) + 255) / 256 * 256;
  unsigned char* arena = nullptr;
  if (hipMalloc(&arena, x_bytes + r_bytes + size_t(kcap) * sizeof(int32_t)) != hipSuccess) return DS_ERR_OOM;
  h->X = arena;
  h->nX = N + 1;
  auto* res = reinterpret_cast<SmallResult<T>*>(arena + x_bytes);
  int32_t* Kin = reinterpret_cast<int32_t*>(arena + x_bytes + r_bytes);
  if (h->form == DS_FORM_FMA)
    small_build_kernel<T, DS_FORM_FMA><<<dim3(1), dim3(kSmallBlock), 0, s>>>(
        static_cast<const T*>(X_dev), N, h->hstart, static_cast<T*>(h->X), res, Kin, kcap);
  else
    small_build_kernel<T, DS_FORM_SUB><<<dim3(1), dim3(kSmallBlock), 0, s>>>(
        static_cast<const T*>(X_dev), N, h->hstart, static_cast<T*>(h->X), res, Kin, kcap);
  DS_HIP_CHECK(hipGetLastError());
  SmallResult<T> r{};
  DS_HIP_CHECK(hipMemcpyAsync(&r, res, sizeof(r), hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipStreamSynchronize(s));
  if (r.status != DS_OK) return static_cast<ds_status>(r.status);
  h->H = r.H;
  h->W = r.W;
  h->X0 = r.X0;
  h->XN = r.XN;
  h->R = r.R;
  h->jmin = r.jmin;
  h->n_updates = r.n_updates;
  h->nK = h->R - h->jmin + 1;
  if (h->nK * int64_t(sizeof(int32_t)) > cap) return DS_ERR_TABLE_CAP;
  ds_status st = DS_OK;
  if (r.filled) {
    h->K = Kin;
    h->k_in_x = true;  // freed with X
  } else {
    if (hipMalloc(&h->K, size_t(h->nK) * sizeof(int32_t)) != hipSuccess) {
      h->K = nullptr;
      return DS_ERR_OOM;
    }
    st = (h->form == DS_FORM_FMA) ? fill_table<T, DS_FORM_FMA>(h, s) : fill_table<T, DS_FORM_SUB>(h, s);
    if (st != DS_OK) return st;
  }
  return build_layouts<T>(h, o, s);
}

// The gap-q variant (Sec. 4.7): the grid only has to satisfy
// f(X_{i+q}) > f(X_i), K_j = max{i : f(X_i) <= j}, and the search makes q
// compares.  X is stored after kMaxGapQ - 1 copies of X_0 (the left padding
// the search reads for K_j < q - 1).  With o.gap_q = 0, q is the smallest
// value in 1..min(16, N) whose grid is feasible and whose table fits the cap
// (the memory-budget choice the section suggests).
template <typename T>
ds_status build_direct_gap(ds_index* h, const ds_build_opts& o, const void* X_dev, hipStream_t s) {
  const int64_t N = h->N;
  const int64_t pad = kMaxGapQ - 1;
  if (hipMalloc(&h->X, size_t(N + 1 + pad) * sizeof(T)) != hipSuccess) {
    h->X = nullptr;
    return DS_ERR_OOM;
  }
  h->nX = N + 1 + pad;
  h->x_off = pad;
  T* Xp = static_cast<T*>(h->X);
  const T* X = Xp + pad;
  DS_HIP_CHECK(hipMemcpyAsync(Xp + pad, X_dev, size_t(N + 1) * sizeof(T), hipMemcpyDeviceToDevice, s));
  pad_left_kernel<T><<<dim3(1), dim3(64), 0, s>>>(Xp, pad);
  DS_HIP_CHECK(hipGetLastError());
  BuildScratch* scr = nullptr;
  if (hipMalloc(&scr, sizeof(BuildScratch)) != hipSuccess) return DS_ERR_OOM;
  struct Free {
    BuildScratch* p;
    ~Free() { (void)hipFree(p); }
  } guard{scr};
  const int64_t cap = o.table_cap_bytes > 0 ? o.table_cap_bytes : kDefaultTableCap;
  const int64_t q_lo = o.gap_q > 0 ? o.gap_q : 1;
  const int64_t q_hi = o.gap_q > 0 ? o.gap_q : std::min<int64_t>(kMaxGapQ, N);
  const int64_t grid = std::min<int64_t>(grid_for(N, kScanBlock, 1 << 20), int64_t(num_cus()) * 8);
  T ends[2];
  DS_HIP_CHECK(hipMemcpyAsync(&ends[0], X, sizeof(T), hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipMemcpyAsync(&ends[1], X + N, sizeof(T), hipMemcpyDeviceToHost, s));
  ds_status st = DS_ERR_INFEASIBLE;
  int64_t q = q_lo;
  for (; q <= q_hi; ++q) {
    BuildScratch init{};
    init.min_gap_bits = ~0ull;
    init.first_bad = ~0ull;
    DS_HIP_CHECK(hipMemcpyAsync(scr, &init, sizeof(init), hipMemcpyHostToDevice, s));
    mingap_kernel<T><<<dim3((unsigned)grid), dim3(kScanBlock), 0, s>>>(X, N, q, scr);
    DS_HIP_CHECK(hipGetLastError());
    BuildScratch got{};
    DS_HIP_CHECK(hipMemcpyAsync(&got, scr, sizeof(got), hipMemcpyDeviceToHost, s));
    DS_HIP_CHECK(hipStreamSynchronize(s));
    if (got.flags & kFlagNonFinite) return DS_ERR_NONFINITE;
    if (got.flags & kFlagNotSorted) return DS_ERR_NOT_SORTED;
    if (got.flags & kFlagOffsetsNotIncreasing) {
      st = DS_ERR_INFEASIBLE;
      continue;
    }
    const T g = from_bits<T>(got.min_gap_bits);
    st = (h->form == DS_FORM_FMA) ? compute_hr<T, DS_FORM_FMA>(h, X, q, scr, s, ends[0], ends[1], g)
                                  : compute_hr<T, DS_FORM_SUB>(h, X, q, scr, s, ends[0], ends[1], g);
    // an infeasible grid (or one past the table cap) tries the next q; any other
    // failure (a HIP call, an allocation) is returned as it is
    if (st == DS_ERR_INFEASIBLE || st == DS_ERR_TABLE_CAP) continue;
    if (st != DS_OK) return st;
    if ((h->R - h->jmin + 1) * int64_t(sizeof(int32_t)) > cap) {
      st = DS_ERR_TABLE_CAP;
      continue;
    }
    break;
  }
  if (st != DS_OK) return st;
  h->gap_q = static_cast<int32_t>(q);
  h->nK = h->R - h->jmin + 1;
  if (hipMalloc(&h->K, size_t(h->nK) * sizeof(int32_t)) != hipSuccess) {
    h->K = nullptr;
    return DS_ERR_OOM;
  }
  const int64_t blocks = (N + 1 + kFillBlock - 1) / kFillBlock;
  if (h->form == DS_FORM_FMA)
    fill_max_kernel<T, DS_FORM_FMA><<<dim3((unsigned)blocks), dim3(kFillBlock), 0, s>>>(
        X, N, T(h->H), T(h->W), T(h->X0), static_cast<int32_t>(h->jmin), h->R, h->nK, h->K);
  else
    fill_max_kernel<T, DS_FORM_SUB><<<dim3((unsigned)blocks), dim3(kFillBlock), 0, s>>>(
        X, N, T(h->H), T(h->W), T(h->X0), static_cast<int32_t>(h->jmin), h->R, h->nK, h->K);
  DS_HIP_CHECK(hipGetLastError());
  if (q <= 15) {
    // GAPCODE: count words and the keys' position codes (codes of the unpadded X)
    h->gc_bits = q <= 3 ? 2 : 4;
    const int64_t cells = 64 / h->gc_bits;
    const int64_t nW = (h->nK + cells - 1) / cells;
    const int64_t n_codes = ((N + 1) + 7) / 8 * 8;
    if (hipMalloc(&h->gc_counts, size_t(nW) * 8) != hipSuccess || hipMalloc(&h->gc_base, size_t(nW) * 4) != hipSuccess ||
        hipMalloc(&h->rc_code, size_t(n_codes) * 2) != hipSuccess)
      return DS_ERR_OOM;
    h->gc_words = nW;
    gap_words_kernel<<<dim3((unsigned)((nW + 255) / 256)), dim3(256), 0, s>>>(h->K, h->nK, nW, h->gc_bits,
                                                                               h->gc_counts, h->gc_base);
    if (h->form == DS_FORM_FMA)
      rank_code_kernel<T, DS_FORM_FMA><<<dim3((unsigned)((n_codes + 255) / 256)), dim3(256), 0, s>>>(
          X, N, n_codes, T(h->H), T(h->W), T(h->X0), h->rc_code);
    else
      rank_code_kernel<T, DS_FORM_SUB><<<dim3((unsigned)((n_codes + 255) / 256)), dim3(256), 0, s>>>(
          X, N, n_codes, T(h->H), T(h->W), T(h->X0), h->rc_code);
    DS_HIP_CHECK(hipGetLastError());
  }
  h->staged = tables_fit_lds(h) ? 1 : 0;
  // PLAIN in LDS when it fits, else GAPCODE in LDS when it fits, else PLAIN through L2
  h->auto_stage = h->staged ? 1 : ((h->gc_counts && direct_lds_bytes(h, 8) <= kLdsBytesPerCU) ? 8 : 2);
  DS_HIP_CHECK(hipStreamSynchronize(s));
  return DS_OK;
}

// Binary-search baselines keep X (offset search) or X padded with X_N up to
// 2^p entries, p = 1 + floor(log2 N) (leading-bit search, Sec. 3.2.1).
template <typename T>
ds_status build_bsearch(ds_index* h, const void* X_dev, hipStream_t s) {
  const int64_t N = h->N;
  int p = 0;
  while ((int64_t(1) << (p + 1)) <= N) ++p;  // p = floor(log2 N)
  h->P = static_cast<int32_t>(int64_t(1) << p);
  // offset search constants (Sec. 3.3): F = floor((N+1)/2), S = N+1-F, J = floor(log2(N+1))
  h->F = static_cast<int32_t>((N + 1) / 2);
  h->S = static_cast<int32_t>(N + 1 - h->F);
  int j = 0;
  while ((int64_t(1) << (j + 1)) <= N + 1) ++j;
  h->J = j;
  const int64_t n_store = (h->method == DS_METHOD_BSEARCH_LEADBIT) ? (int64_t(2) * h->P) : (N + 1);
  if (hipMalloc(&h->X, size_t(n_store) * sizeof(T)) != hipSuccess) {
    h->X = nullptr;
    return DS_ERR_OOM;
  }
  h->nX = n_store;
  DS_HIP_CHECK(hipMemcpyAsync(h->X, X_dev, size_t(N + 1) * sizeof(T), hipMemcpyDeviceToDevice, s));
  if (n_store > N + 1) {
    T xn;
    DS_HIP_CHECK(hipMemcpyAsync(&xn, static_cast<const T*>(X_dev) + N, sizeof(T), hipMemcpyDeviceToHost, s));
    DS_HIP_CHECK(hipStreamSynchronize(s));
    const int64_t cnt = n_store - (N + 1);
    pad_kernel<T><<<dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s>>>(static_cast<T*>(h->X), N + 1, n_store, xn);
    DS_HIP_CHECK(hipGetLastError());
  }
  return DS_OK;
}

// Eytzinger layout (Sec. 3.4): node b of the complete tree of L levels (depth
// d = floor(log2 b), position p = b - 2^d in its level) is the in-order
// element (2p + 1) 2^(L-1-d) - 1 of the padded array X_0..X_N, X_N, ...
template <typename T>
__global__ void eyt_layout_kernel(const T* __restrict__ X, int64_t N, int L, T* __restrict__ Y) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nodes = int64_t(1) << L;
  if (b >= nodes) return;
  if (b == 0) {
    Y[0] = X[0];  // unused slot
    return;
  }
  const int d = 63 - __clzll(static_cast<unsigned long long>(b));
  const int64_t p = b - (int64_t(1) << d);
  const int64_t idx = ((2 * p + 1) << (L - 1 - d)) - 1;
  Y[b] = X[idx <= N ? idx : N];
}

template <typename T>
ds_status build_eytzinger(ds_index* h, const void* X_dev, hipStream_t s) {
  const int64_t N = h->N;
  int L = 1;
  while ((int64_t(1) << L) - 1 < N + 1) ++L;
  const int64_t n = int64_t(1) << L;
  if (hipMalloc(&h->X, size_t(n) * sizeof(T)) != hipSuccess) {
    h->X = nullptr;
    return DS_ERR_OOM;
  }
  h->nX = n;
  h->eyt_L = L;
  eyt_layout_kernel<T><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(static_cast<const T*>(X_dev), N, L,
                                                                                static_cast<T*>(h->X));
  DS_HIP_CHECK(hipGetLastError());
  DS_HIP_CHECK(hipStreamSynchronize(s));
  return DS_OK;
}

// the validation pass alone, for the binary-search methods
template <typename T>
ds_status validate_only(ds_index* h, const void* X_dev, hipStream_t s) {
  BuildScratch* scr = nullptr;
  if (hipMalloc(&scr, sizeof(BuildScratch)) != hipSuccess) return DS_ERR_OOM;
  struct Free {
    BuildScratch* p;
    ~Free() { (void)hipFree(p); }
  } guard{scr};
  BuildScratch init{};
  init.min_gap_bits = ~0ull;
  DS_HIP_CHECK(hipMemcpyAsync(scr, &init, sizeof(init), hipMemcpyHostToDevice, s));
  const int64_t grid = std::min<int64_t>(grid_for(h->N, kScanBlock, 1 << 20), int64_t(num_cus()) * 8);
  mingap_kernel<T><<<dim3((unsigned)grid), dim3(kScanBlock), 0, s>>>(static_cast<const T*>(X_dev), h->N, 1, scr);
  DS_HIP_CHECK(hipGetLastError());
  BuildScratch got{};
  DS_HIP_CHECK(hipMemcpyAsync(&got, scr, sizeof(got), hipMemcpyDeviceToHost, s));
  DS_HIP_CHECK(hipStreamSynchronize(s));
  if (got.flags & kFlagNonFinite) return DS_ERR_NONFINITE;
  if (got.flags & kFlagNotSorted) return DS_ERR_NOT_SORTED;
  T x0;
  DS_HIP_CHECK(hipMemcpy(&x0, X_dev, sizeof(T), hipMemcpyDeviceToHost));
  h->X0 = x0;
  return DS_OK;
}

void free_layouts(ds_index* h) {
  if (h->rc_bits) (void)hipFree(h->rc_bits);
  if (h->rc_base) (void)hipFree(h->rc_base);
  if (h->rc_code) (void)hipFree(h->rc_code);
  if (h->rc_w16) (void)hipFree(h->rc_w16);
  if (h->rc_code8) (void)hipFree(h->rc_code8);
  h->rc_w16 = nullptr;
  h->rc_code8 = nullptr;
  if (h->pairs) (void)hipFree(h->pairs);
  if (h->nib) (void)hipFree(h->nib);
  if (h->gc_counts) (void)hipFree(h->gc_counts);
  if (h->gc_base) (void)hipFree(h->gc_base);
  h->gc_counts = nullptr;
  h->gc_base = nullptr;
  h->gc_words = 0;
  h->gc_bits = 0;
  h->rc_bits = nullptr;
  h->rc_base = nullptr;
  h->rc_code = nullptr;
  h->pairs = nullptr;
  h->nib = nullptr;
  h->nib_chunks = 0;
}

void free_device(ds_index* h) {
  if (h->X) (void)hipFree(h->X);
  if (h->K && !h->k_in_x) (void)hipFree(h->K);
  h->X = nullptr;
  h->K = nullptr;
  h->k_in_x = false;
  free_layouts(h);
  learned_free(h);
}

template <typename T>
ds_status build_typed(ds_index* h, const void* X_dev, const ds_build_opts& o, hipStream_t s) {
  const int64_t N = h->N;
  int method = o.method;
  if (method == DS_METHOD_BSEARCH_LEADBIT || method == DS_METHOD_BSEARCH_OFFSET) {
    ds_status st = validate_only<T>(h, X_dev, s);
    if (st != DS_OK) return st;
    h->method = method;
    return build_bsearch<T>(h, X_dev, s);
  }
  if (method == DS_METHOD_BSEARCH_EYTZINGER) {
    ds_status st = validate_only<T>(h, X_dev, s);
    if (st != DS_OK) return st;
    h->method = method;
    return build_eytzinger<T>(h, X_dev, s);
  }
  if (method == DS_METHOD_LEARNED) {
    h->method = DS_METHOD_LEARNED;
    if (hipMalloc(&h->X, size_t(N + 1) * sizeof(T)) != hipSuccess) return DS_ERR_OOM;
    h->nX = N + 1;
    DS_HIP_CHECK(hipMemcpyAsync(h->X, X_dev, size_t(N + 1) * sizeof(T), hipMemcpyDeviceToDevice, s));
    ds_status st = validate_only<T>(h, h->X, s);
    if (st != DS_OK) return st;
    return learned_build(h, &o, s);
  }
  ds_status st;
  if (method == DS_METHOD_DIRECT_GAP) {
    h->method = DS_METHOD_DIRECT_GAP;
    st = build_direct_gap<T>(h, o, X_dev, s);
  } else {
    // Direct (or AUTO: Direct first)
    h->method = DS_METHOD_DIRECT;
    if (N + 1 <= kSmallBuildMax && !o.refine_h) {
      st = build_direct_small<T>(h, o, X_dev, s);
    } else {
      if (hipMalloc(&h->X, size_t(N + 1) * sizeof(T)) != hipSuccess) return DS_ERR_OOM;
      h->nX = N + 1;
      DS_HIP_CHECK(hipMemcpyAsync(h->X, X_dev, size_t(N + 1) * sizeof(T), hipMemcpyDeviceToDevice, s));
      st = build_direct<T>(h, o, s);
    }
  }
  if (st == DS_OK) return DS_OK;
  const bool can_fall = (st == DS_ERR_INFEASIBLE || st == DS_ERR_TABLE_CAP);
  int fb = o.fallback;
  if (method == DS_METHOD_AUTO && fb == DS_FALLBACK_NONE) fb = DS_FALLBACK_LEARNED;
  if (!can_fall || fb == DS_FALLBACK_NONE) return st;
  // fall back: drop the partial Direct state and build the replacement
  free_layouts(h);
  if (h->K && !h->k_in_x) (void)hipFree(h->K);
  h->K = nullptr;
  h->k_in_x = false;
  h->nK = 0;
  h->H = h->W = 0;
  h->R = h->jmin = 0;
  h->gap_q = 0;
  if (h->x_off != 0) {  // the gap variant's padded copy: replace it by a plain one
    (void)hipFree(h->X);
    h->x_off = 0;
    if (hipMalloc(&h->X, size_t(N + 1) * sizeof(T)) != hipSuccess) {
      h->X = nullptr;
      return DS_ERR_OOM;
    }
    h->nX = N + 1;
    DS_HIP_CHECK(hipMemcpyAsync(h->X, X_dev, size_t(N + 1) * sizeof(T), hipMemcpyDeviceToDevice, s));
  }
  if (fb == DS_FALLBACK_BSEARCH) {
    (void)hipFree(h->X);
    h->X = nullptr;
    h->method = DS_METHOD_BSEARCH_LEADBIT;
    return build_bsearch<T>(h, X_dev, s);
  }
  h->method = DS_METHOD_LEARNED;
  return learned_build(h, &o, s);
}

}  // namespace

int num_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

}  // namespace ds

extern "C" {

ds_status ds_build(const void* X_dev, int64_t N, ds_dtype dt, const ds_build_opts* opts, hipStream_t s,
                   ds_handle* out) {
  if (!X_dev || !out || N < 1 || N > int64_t(2147483646)) return DS_ERR_ARG;
  if (dt != DS_F32 && dt != DS_F64) return DS_ERR_ARG;
  ds_build_opts o{};
  if (opts) o = *opts;
  if (o.method < DS_METHOD_DIRECT || o.method > DS_METHOD_BSEARCH_EYTZINGER) return DS_ERR_ARG;
  if (o.gap_q < 0 || o.gap_q > ds::kMaxGapQ || (o.method == DS_METHOD_DIRECT_GAP && o.gap_q > N)) return DS_ERR_ARG;
  if (o.form != DS_FORM_SUB && o.form != DS_FORM_FMA) return DS_ERR_ARG;
  if (o.hstart != DS_HSTART_PHI && o.hstart != DS_HSTART_HBAR) return DS_ERR_ARG;
  if (o.refine_h != 0 && o.refine_h != 1) return DS_ERR_ARG;
  if (o.fallback < DS_FALLBACK_NONE || o.fallback > DS_FALLBACK_LEARNED) return DS_ERR_ARG;
  if (o.table_cap_bytes < 0) return DS_ERR_ARG;
  if (o.extra_layouts & ~(DS_LAYOUT_RANKCODE | DS_LAYOUT_PAIRS | DS_LAYOUT_NIBBLE)) return DS_ERR_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  ds_index* h = new (std::nothrow) ds_index();
  if (!h) return DS_ERR_OOM;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return DS_ERR_HIP;
  }
  h->dt = dt;
  h->N = N;
  h->form = o.form;
  h->hstart = o.hstart;
  h->refine_h = o.refine_h;
  ds_status st = (dt == DS_F32) ? ds::build_typed<float>(h, X_dev, o, s) : ds::build_typed<double>(h, X_dev, o, s);
  if (st == DS_OK && hipStreamSynchronize(s) != hipSuccess) st = DS_ERR_HIP;
  if (st != DS_OK) {
    (void)hipStreamSynchronize(s);
    ds::free_device(h);
    delete h;
    return st;
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ds_info_t& in = h->info;
  in.method = h->method;
  in.dtype = h->dt;
  in.form = h->form;
  const bool direct_family = h->method == DS_METHOD_DIRECT || h->method == DS_METHOD_DIRECT_GAP;
  in.staged = direct_family ? h->auto_stage : (ds::tables_fit_lds(h) ? 1 : 2);
  if (!direct_family) h->staged = ds::tables_fit_lds(h) ? 1 : 0;
  in.gap_q = h->gap_q;
  in.N = h->N;
  in.H = h->H;
  in.W = h->W;
  in.X0 = h->X0;
  in.R = h->R;
  in.jmin = h->jmin;
  in.n_h_updates = h->n_updates;
  in.n_h_refine = h->n_refine;
  in.table_bytes = h->nK * int64_t(sizeof(int32_t));
  in.x_bytes = h->nX * int64_t(dt == DS_F32 ? 4 : 8);
  in.rankcode_bytes = h->rc_bits ? (h->rc_words * 12 + (h->N + 1) * 2) : 0;
  in.gapcode_bytes = h->gc_counts ? (h->gc_words * 12 + (h->N + 1) * 2) : 0;
  in.pairs_bytes = h->pairs ? h->nK * int64_t(dt == DS_F32 ? 8 : 16) : 0;
  in.nibble_bytes = h->nib ? h->nib_chunks * int64_t(sizeof(ds::NibChunk)) : 0;
  in.build_ms = ms;
  ds::learned_fill_info(h, &in);
  *out = h;
  return DS_OK;
}

ds_status ds_info(ds_handle h, ds_info_t* info) {
  if (!h || !info) return DS_ERR_ARG;
  *info = h->info;
  info->fallback_count = 0;
  if (h->learned) return ds::learned_fallbacks(h, &info->fallback_count);
  return DS_OK;
}

ds_status ds_copy_table(ds_handle h, int32_t* dst_dev, int64_t capacity_entries, hipStream_t s) {
  if (!h || !dst_dev || !h->K || capacity_entries < h->nK) return DS_ERR_ARG;
  DS_HIP_CHECK(hipMemcpyAsync(dst_dev, h->K, size_t(h->nK) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  DS_HIP_CHECK(hipStreamSynchronize(s));
  return DS_OK;
}

ds_status ds_destroy(ds_handle h) {
  if (!h) return DS_ERR_ARG;
  ds::free_device(h);
  delete h;
  return DS_OK;
}

const char* ds_status_str(ds_status st) {
  switch (st) {
    case DS_OK: return "ok";
    case DS_ERR_ARG: return "invalid argument";
    case DS_ERR_NOT_SORTED: return "X is not strictly increasing";
    case DS_ERR_NONFINITE: return "X holds a non-finite value";
    case DS_ERR_INFEASIBLE: return "no feasible grid scale H for this X in this precision";
    case DS_ERR_TABLE_CAP: return "the Direct table would exceed the byte cap";
    case DS_ERR_OOM: return "device allocation failed";
    case DS_ERR_HIP: return "HIP runtime error";
    case DS_ERR_UNSUPPORTED: return "unsupported option";
    case DS_ERR_SCRATCH_CAP: return "the batch needs more workspace than the fixed scratch array holds";
  }
  return "unknown status";
}

}  // extern "C"
