// Search kernels: Direct (Sec. 4.2) and the two branch-free binary-search
// baselines (Sec. 3.2.1 leading-bit with padding, Sec. 3.3 offset-based).
//
// Layout and launch (gfx950):
//   * queries stream through in 4-element vectors per lane (16 B for f32,
//     32 B for f64) with non-temporal loads and stores, so z and out do not
//     evict the tables from L2;
//   * the tables (K and X for Direct, X for binary search) are copied into LDS
//     by every workgroup when they fit in one workgroup's LDS (160 KiB),
//     otherwise they are gathered through L1/L2;
//   * the grid is persistent: as many workgroups as can be resident, each
//     stepping through the query vectors with a grid-sized stride, so the LDS
//     copy is paid once per workgroup.
#include <algorithm>
#include <mutex>

#include "ds_internal.h"

namespace ds {

namespace {

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
template <typename T, int FORM, bool INTERLEAVED>
struct RankCodeOp {
  const uint64_t* bits;
  const uint32_t* base;
  const RcWord* w16;  // INTERLEAVED: (bits, base) of a word in one 16-byte load
  const uint16_t* code;
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
    const T cz = cell_code<T>(v, jf);
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

__host__ __device__ constexpr int64_t rankcode_offsets(int64_t nW, int64_t n_code_bytes, int64_t* base_off,
                                                       int64_t* code_off) {
  *base_off = round16(nW * 8);
  *code_off = *base_off + round16(nW * 4);
  return *code_off + round16(n_code_bytes);
}

// STAGE 1: PLAIN in LDS; 2: PLAIN through L1/L2; 3: RANKCODE in LDS;
// 4: PAIRS through L1/L2; 5: RANKCODE through L1/L2.
template <typename T, int FORM, int STAGE, int U, bool VEC>
__global__ void __launch_bounds__(1024) direct_search_kernel(DirectArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  if constexpr (STAGE == 1 || STAGE == 2) {
    const T* X = a.X;
    const int32_t* K = a.K;
    if constexpr (STAGE == 1) {
      const int64_t xb = round16(int64_t(a.nX) * sizeof(T));
      stage_bytes(smem, reinterpret_cast<const unsigned char*>(a.X), int64_t(a.nX) * sizeof(T));
      stage_bytes(smem + xb, reinterpret_cast<const unsigned char*>(a.K), int64_t(a.nK) * 4);
      __syncthreads();
      X = reinterpret_cast<const T*>(smem);
      K = reinterpret_cast<const int32_t*>(smem + xb);
    }
    DirectOp<T, FORM> op{X, K - a.jmin, a.H, a.W, a.X0, a.vlo, a.vhi};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  } else if constexpr (STAGE == 3) {
    int64_t base_off = 0, code_off = 0;
    const int64_t code_bytes = round16(int64_t(a.N + 1) * 2);
    rankcode_offsets(a.nW, code_bytes, &base_off, &code_off);
    stage_bytes(smem, reinterpret_cast<const unsigned char*>(a.rc_bits), int64_t(a.nW) * 8);
    stage_bytes(smem + base_off, reinterpret_cast<const unsigned char*>(a.rc_base), int64_t(a.nW) * 4);
    stage_bytes(smem + code_off, reinterpret_cast<const unsigned char*>(a.rc_code), code_bytes);
    __syncthreads();
    RankCodeOp<T, FORM, false> op{reinterpret_cast<const uint64_t*>(smem),
                                  reinterpret_cast<const uint32_t*>(smem + base_off),
                                  nullptr,
                                  reinterpret_cast<const uint16_t*>(smem + code_off),
                                  a.X, a.H, a.W, a.X0, a.vlo, a.vhi, a.XN, a.jmin, a.N};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  } else if constexpr (STAGE == 5) {
    RankCodeOp<T, FORM, true> op{nullptr, nullptr, a.rc_w16, a.rc_code, a.X, a.H, a.W, a.X0, a.vlo, a.vhi, a.XN,
                                 a.jmin, a.N};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  } else {
    PairsOp<T, FORM> op{a.pairs - a.jmin, a.H, a.W, a.X0, a.vlo, a.vhi};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  }
}

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

template <typename T, int KIND, int STAGE, int U, bool VEC>
__global__ void __launch_bounds__(1024) bsearch_kernel(BsearchArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const T* X = a.X;
  if constexpr (STAGE == 1) {
    stage_bytes(smem, reinterpret_cast<const unsigned char*>(a.X), int64_t(a.nX) * sizeof(T));
    __syncthreads();
    X = reinterpret_cast<const T*>(smem);
  }
  if constexpr (KIND == DS_METHOD_BSEARCH_LEADBIT) {
    LeadbitOp<T> op{X, a.P, a.N};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  } else {
    OffsetOp<T> op{X, a.F, a.S, a.J};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  }
}

int64_t lds_bytes_needed(const ds_index* h, int stage) {
  const int64_t s = (h->dt == DS_F32) ? 4 : 8;
  if (h->method == DS_METHOD_DIRECT && stage == 3) {
    int64_t b = 0, c = 0;
    return rankcode_offsets(h->rc_words, round16((h->N + 1) * 2), &b, &c);
  }
  if (h->method == DS_METHOD_DIRECT) return round16(h->nX * s) + h->nK * 4;
  if (h->method == DS_METHOD_BSEARCH_LEADBIT || h->method == DS_METHOD_BSEARCH_OFFSET) return round16(h->nX * s);
  return int64_t(1) << 40;
}

struct Shape {
  int block, unroll, stage, grid;
};

// Occupancy-derived persistent grid for one kernel instantiation.
template <class KernelT>
int resident_blocks(KernelT kernel, int block, int lds) {
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (lds > 64 * 1024) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  return per_cu * num_cus();
}

// Default launch shape per layout and precision, from a sweep of block size
// and vectors per lane on MI355X (2^26 queries of the N sweep).
void default_shape(const ds_index* h, int stage, int* block, int* unroll) {
  const bool f32 = h->dt == DS_F32;
  switch (stage) {
    case 1: *block = 256; *unroll = f32 ? 4 : 2; return;
    case 3: {
      const bool one_wg_per_cu = lds_bytes_needed(h, 3) > kLdsBytesPerCU / 2;
      *block = 1024;
      *unroll = (one_wg_per_cu && f32) ? 4 : 1;
      return;
    }
    case 4: *block = f32 ? 256 : 1024; *unroll = f32 ? 4 : 1; return;
    case 5: *block = 512; *unroll = 2; return;
    default: *block = 512; *unroll = 2; return;
  }
}

Shape pick_shape(const ds_index* h, int64_t M) {
  Shape sh{};
  const ds_tune& t = h->tune;
  if (h->tune_set && t.stage) {
    sh.stage = t.stage;
  } else if (h->method == DS_METHOD_DIRECT) {
    sh.stage = h->auto_stage;
  } else {
    sh.stage = h->staged ? 1 : 2;
  }
  int block = 512, unroll = 2;
  if (h->method == DS_METHOD_DIRECT) default_shape(h, sh.stage, &block, &unroll);
  sh.block = (h->tune_set && t.block) ? t.block : block;
  sh.unroll = (h->tune_set && t.unroll) ? t.unroll : unroll;
  sh.grid = (h->tune_set && t.grid) ? t.grid : 0;
  (void)M;
  return sh;
}

template <class KernelT, class ArgsT>
ds_status launch(KernelT kernel, const ArgsT& args, const Shape& sh, int lds, int64_t work_items, hipStream_t s) {
  int grid = sh.grid;
  if (grid <= 0) {
    grid = resident_blocks(kernel, sh.block, lds);
    const int64_t need = (work_items + int64_t(sh.block) - 1) / sh.block;
    grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(grid, need)));
  } else if (lds > 64 * 1024) {
    (void)resident_blocks(kernel, sh.block, lds);  // sets the LDS attribute
  }
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(sh.block), lds, s, args);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

template <typename T, int FORM, int STAGE, bool VEC>
ds_status dispatch_direct_u(const DirectArgs<T>& a, const Shape& sh, int lds, int64_t items, hipStream_t s) {
  switch (sh.unroll) {
    case 1: return launch(direct_search_kernel<T, FORM, STAGE, 1, VEC>, a, sh, lds, items, s);
    case 2: return launch(direct_search_kernel<T, FORM, STAGE, 2, VEC>, a, sh, lds, items, s);
    default: return launch(direct_search_kernel<T, FORM, STAGE, 4, VEC>, a, sh, lds, items, s);
  }
}

template <typename T, int FORM>
ds_status dispatch_direct(const DirectArgs<T>& a, const Shape& sh, bool vec, int lds, hipStream_t s) {
  const int64_t items = vec ? ((a.M >> 2) + sh.unroll - 1) / sh.unroll : a.M;
  switch (sh.stage) {
    case 1:
      return vec ? dispatch_direct_u<T, FORM, 1, true>(a, sh, lds, items, s)
                 : dispatch_direct_u<T, FORM, 1, false>(a, sh, lds, items, s);
    case 3:
      return vec ? dispatch_direct_u<T, FORM, 3, true>(a, sh, lds, items, s)
                 : dispatch_direct_u<T, FORM, 3, false>(a, sh, lds, items, s);
    case 4:
      return vec ? dispatch_direct_u<T, FORM, 4, true>(a, sh, 0, items, s)
                 : dispatch_direct_u<T, FORM, 4, false>(a, sh, 0, items, s);
    case 5:
      return vec ? dispatch_direct_u<T, FORM, 5, true>(a, sh, 0, items, s)
                 : dispatch_direct_u<T, FORM, 5, false>(a, sh, 0, items, s);
    default:
      return vec ? dispatch_direct_u<T, FORM, 2, true>(a, sh, 0, items, s)
                 : dispatch_direct_u<T, FORM, 2, false>(a, sh, 0, items, s);
  }
}

template <typename T, int KIND, int STAGE, bool VEC>
ds_status dispatch_bs_u(const BsearchArgs<T>& a, const Shape& sh, int lds, int64_t items, hipStream_t s) {
  switch (sh.unroll) {
    case 1: return launch(bsearch_kernel<T, KIND, STAGE, 1, VEC>, a, sh, lds, items, s);
    case 2: return launch(bsearch_kernel<T, KIND, STAGE, 2, VEC>, a, sh, lds, items, s);
    default: return launch(bsearch_kernel<T, KIND, STAGE, 4, VEC>, a, sh, lds, items, s);
  }
}

template <typename T, int KIND>
ds_status dispatch_bs(const BsearchArgs<T>& a, const Shape& sh, bool vec, int lds, hipStream_t s) {
  const int64_t items = vec ? ((a.M >> 2) + sh.unroll - 1) / sh.unroll : a.M;
  if (sh.stage == 1) {
    return vec ? dispatch_bs_u<T, KIND, 1, true>(a, sh, lds, items, s)
               : dispatch_bs_u<T, KIND, 1, false>(a, sh, lds, items, s);
  }
  return vec ? dispatch_bs_u<T, KIND, 2, true>(a, sh, 0, items, s)
             : dispatch_bs_u<T, KIND, 2, false>(a, sh, 0, items, s);
}

template <typename T>
T X_N(const ds_index* h) {
  return T(h->XN);
}

template <typename T>
ds_status search_typed(ds_index* h, const void* z, int64_t M, int32_t* out, hipStream_t s) {
  const Shape sh = pick_shape(h, M);
  const bool vec = ((reinterpret_cast<uintptr_t>(z) % (4 * sizeof(T))) == 0) &&
                   ((reinterpret_cast<uintptr_t>(out) % 16) == 0);
  const int lds = (sh.stage == 1 || sh.stage == 3) ? static_cast<int>(lds_bytes_needed(h, sh.stage)) : 0;
  if (h->method == DS_METHOD_DIRECT) {
    DirectArgs<T> a{};
    a.X = static_cast<const T*>(h->X);
    a.K = h->K;
    a.H = T(h->H);
    a.W = T(h->W);
    a.X0 = T(h->X0);
    a.vlo = T(h->jmin);
    a.vhi = T(h->R);
    a.jmin = static_cast<int32_t>(h->jmin);
    a.nK = static_cast<int32_t>(h->nK);
    a.nX = static_cast<int32_t>(h->nX);
    a.N = static_cast<int32_t>(h->N);
    a.XN = X_N<T>(h);
    a.rc_bits = h->rc_bits;
    a.rc_base = h->rc_base;
    a.rc_code = h->rc_code;
    a.rc_w16 = h->rc_w16;
    a.nW = static_cast<int32_t>(h->rc_words);
    a.pairs = static_cast<const CachePair<T>*>(h->pairs);
    a.z = static_cast<const T*>(z);
    a.out = out;
    a.M = M;
    return (h->form == DS_FORM_FMA) ? dispatch_direct<T, DS_FORM_FMA>(a, sh, vec, lds, s)
                                    : dispatch_direct<T, DS_FORM_SUB>(a, sh, vec, lds, s);
  }
  BsearchArgs<T> a{};
  a.X = static_cast<const T*>(h->X);
  a.nX = static_cast<int32_t>(h->nX);
  a.N = static_cast<int32_t>(h->N);
  a.P = h->P;
  a.F = h->F;
  a.S = h->S;
  a.J = h->J;
  a.z = static_cast<const T*>(z);
  a.out = out;
  a.M = M;
  if (h->method == DS_METHOD_BSEARCH_LEADBIT) return dispatch_bs<T, DS_METHOD_BSEARCH_LEADBIT>(a, sh, vec, lds, s);
  return dispatch_bs<T, DS_METHOD_BSEARCH_OFFSET>(a, sh, vec, lds, s);
}

}  // namespace

bool tables_fit_lds(const ds_index* h) { return lds_bytes_needed(h, 1) <= kLdsBytesPerCU; }
int64_t rankcode_lds_bytes(const ds_index* h) { return lds_bytes_needed(h, 3); }

ds_status launch_search(ds_index* h, const void* z, int64_t M, int32_t* out, hipStream_t s) {
  if (h->method == DS_METHOD_LEARNED) return learned_search(h, z, M, out, s);
  return (h->dt == DS_F32) ? search_typed<float>(h, z, M, out, s) : search_typed<double>(h, z, M, out, s);
}

}  // namespace ds

extern "C" {

ds_status ds_search(ds_handle h, const void* z_dev, int64_t M, int32_t* out_dev, hipStream_t s) {
  if (!h || M < 0) return DS_ERR_ARG;
  if (M == 0) return DS_OK;
  if (!z_dev || !out_dev) return DS_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DS_ERR_HIP;
  if (dev != h->device) return DS_ERR_ARG;
  return ds::launch_search(h, z_dev, M, out_dev, s);
}

ds_status ds_autotune(ds_handle h, const void* z_dev, int64_t M, int32_t* out_dev, hipStream_t s, ds_tune* best) {
  if (!h || !z_dev || !out_dev || M <= 0) return DS_ERR_ARG;
  if (h->method == DS_METHOD_LEARNED) return DS_ERR_UNSUPPORTED;
  const int64_t m = std::min<int64_t>(M, int64_t(1) << 24);
  int stages[5];
  int n_stages = 0;
  if (h->method == DS_METHOD_DIRECT) {
    if (h->staged) stages[n_stages++] = 1;
    if (h->rc_code && ds::rankcode_lds_bytes(h) <= ds::kLdsBytesPerCU) stages[n_stages++] = 3;
    if (h->rc_w16) stages[n_stages++] = 5;
    if (h->pairs) stages[n_stages++] = 4;
    stages[n_stages++] = 2;
  } else {
    if (h->staged) stages[n_stages++] = 1;
    stages[n_stages++] = 2;
  }
  const ds_tune saved = h->tune;
  const bool saved_set = h->tune_set;
  hipEvent_t e0, e1;
  DS_HIP_CHECK(hipEventCreate(&e0));
  DS_HIP_CHECK(hipEventCreate(&e1));
  float best_ms = 1e30f;
  ds_tune best_t{};
  ds_status st = DS_OK;
  const int blocks[3] = {256, 512, 1024};
  const int unrolls[3] = {1, 2, 4};
  for (int si = 0; si < n_stages && st == DS_OK; ++si) {
    for (int bi = 0; bi < 3 && st == DS_OK; ++bi) {
      for (int ui = 0; ui < 3 && st == DS_OK; ++ui) {
        ds_tune cand{blocks[bi], unrolls[ui], stages[si], 0};
        h->tune = cand;
        h->tune_set = true;
        st = ds::launch_search(h, z_dev, m, out_dev, s);  // warm-up
        if (st != DS_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) { st = DS_ERR_HIP; break; }
        for (int r = 0; r < 3 && st == DS_OK; ++r) st = ds::launch_search(h, z_dev, m, out_dev, s);
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { st = DS_ERR_HIP; break; }
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = DS_ERR_HIP; break; }
        if (ms < best_ms) {
          best_ms = ms;
          best_t = cand;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DS_OK) {
    h->tune = saved;
    h->tune_set = saved_set;
    return st;
  }
  h->tune = best_t;
  h->tune_set = true;
  if (best) *best = best_t;
  return DS_OK;
}

ds_status ds_set_tune(ds_handle h, const ds_tune* t) {
  if (!h) return DS_ERR_ARG;
  if (!t) {
    h->tune_set = false;
    h->tune = ds_tune{};
    return DS_OK;
  }
  if (t->block != 0 && (t->block < 64 || t->block > 1024 || (t->block % 64) != 0)) return DS_ERR_ARG;
  if (t->unroll != 0 && t->unroll != 1 && t->unroll != 2 && t->unroll != 4) return DS_ERR_ARG;
  if (t->stage < 0 || t->stage > 5) return DS_ERR_ARG;
  if (t->stage == 5 && !h->rc_w16) return DS_ERR_ARG;
  if (t->stage == 1 && !h->staged) return DS_ERR_ARG;
  if (t->stage >= 3 && h->method != DS_METHOD_DIRECT) return DS_ERR_ARG;
  if (t->stage == 3 && (!h->rc_code || ds::rankcode_lds_bytes(h) > ds::kLdsBytesPerCU)) return DS_ERR_ARG;
  if (t->stage == 4 && !h->pairs) return DS_ERR_ARG;
  if (t->grid < 0) return DS_ERR_ARG;
  h->tune = *t;
  h->tune_set = true;
  return DS_OK;
}

}  // extern "C"
