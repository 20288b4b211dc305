// Search kernels: Direct (Sec. 4.2) and the two branch-free binary-search
// baselines (Sec. 3.2.1 leading-bit with padding, Sec. 3.3 offset-based).
//
// Layout and launch (gfx950):
//   * queries stream through in 4-element vectors per lane (16 B for f32,
//     32 B for f64) with non-temporal loads and stores, so z and out do not
//     evict the tables from L2;
//   * the tables (K and X for Direct, X for binary search) are copied into LDS
//     by every workgroup when they fit in one workgroup's LDS (160 KiB),
//     otherwise they are gathered through L1/L2 (the NIBBLE layout keeps its
//     first 156 KiB in LDS even then);
//   * the grid is persistent: as many workgroups as can be resident, each
//     stepping through the query vectors with a grid-sized stride, so the LDS
//     copy is paid once per workgroup.
#include <algorithm>
#include <mutex>

#include "ds_ops.h"

namespace ds {

namespace {


// STAGE 1: PLAIN in LDS; 2: PLAIN through L1/L2; 3: RANKCODE in LDS;
// 4: PAIRS through L1/L2; 5: RANKCODE through L1/L2; 6: NIBBLE through L1/L2
// with its first chunks in LDS; 7: NIBBLE in LDS.
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
    RankCodeOp<T, FORM, true, uint8_t> op{nullptr, nullptr, a.rc_w16, a.rc_code8, a.X, a.H, a.W, a.X0, a.vlo, a.vhi,
                                          a.XN, a.jmin, a.N};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  } else if constexpr (STAGE == 6 || STAGE == 7) {
    // 7: every chunk in LDS; 6: the first kNibPrefixChunks in LDS, the rest
    // through L2 (the L2's line rate bounds this layout, so every chunk served
    // from LDS is an L2 access saved)
    const int64_t n_pre = (STAGE == 7) ? a.nib_chunks : std::min<int64_t>(a.nib_chunks, kNibPrefixChunks);
    stage_bytes(smem, reinterpret_cast<const unsigned char*>(a.nib), n_pre * int64_t(sizeof(NibChunk)));
    __syncthreads();
    NibbleOp<T, FORM> op{a.nib, a.X, a.H, a.W, a.X0, a.vlo, a.vhi, a.XN, a.jmin, a.N};
    op.pre = reinterpret_cast<const uint4*>(smem);
    op.n_pre = static_cast<uint32_t>(n_pre);
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  } else {
    PairsOp<T, FORM> op{a.pairs - a.jmin, a.H, a.W, a.X0, a.vlo, a.vhi};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  }
}

// gap-q (Sec. 4.7) on the PLAIN tables: STAGE 1 = padded X and K in LDS,
// 2 = through L1/L2.  Q = 2 for q <= 2, 4 for q <= 4, 16 for larger q.
template <typename T, int FORM, int STAGE, int U, bool VEC, int Q>
__global__ void __launch_bounds__(1024) gap_search_kernel(DirectArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
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
  if constexpr (STAGE == 8) {
    // GAPCODE in LDS: the count words, their running counts and the key codes
    int64_t base_off = 0, code_off = 0;
    const int64_t code_bytes = round16(int64_t(a.N + 1) * 2);
    rankcode_offsets(a.nW, code_bytes, &base_off, &code_off);
    stage_bytes(smem, reinterpret_cast<const unsigned char*>(a.rc_bits), int64_t(a.nW) * 8);
    stage_bytes(smem + base_off, reinterpret_cast<const unsigned char*>(a.rc_base), int64_t(a.nW) * 4);
    stage_bytes(smem + code_off, reinterpret_cast<const unsigned char*>(a.rc_code), code_bytes);
    __syncthreads();
    GapCodeOp<T, FORM, (Q <= 3 ? 2 : 4), Q> op{reinterpret_cast<const uint64_t*>(smem),
                                           reinterpret_cast<const uint32_t*>(smem + base_off),
                                           reinterpret_cast<const uint16_t*>(smem + code_off), a.X + a.x_off, a.H,
                                           a.W, a.X0, a.vlo, a.vhi, a.XN, a.jmin, a.N};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  } else {
    GapOp<T, FORM, Q> op{X + a.x_off, K - a.jmin, a.H, a.W, a.X0, a.vlo, a.vhi, a.gap_q};
    stream_queries<T, U, VEC>(a.z, a.out, a.M, op);
  }
}

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

template <typename T>
struct EytArgs {
  const T* Y;          // 2^L values, node k at Y[k] (Y[0] unused)
  int32_t L;           // levels
  int32_t lds_levels;  // levels staged in LDS (STAGE 1)
  int32_t N;
  int32_t pad_;
  const T* z;
  int32_t* out;
  int64_t M;
};

// The descent of Sec. 3.4 for one query: k <- 2k + [z >= Y_k] for L levels,
// the first `lt` from Yl (LDS), the rest from Yg.  The leaf k - 2^L counts the
// padded values <= z; the pads equal X_N, so min(count, N + 1) - 1 is the
// result everywhere (-1 below X_0 and for NaN, N at or above X_N).
template <typename T>
__device__ __forceinline__ int32_t eyt_one(T z, const T* Yl, const T* Yg, int lt, int L, int32_t N) {
  uint32_t k = 1;
  for (int d = 0; d < lt; ++d) k = 2 * k + (z >= Yl[k] ? 1u : 0u);
  uint64_t kk = k;
  for (int d = lt; d < L; ++d) kk = 2 * kk + (z >= Yg[kk] ? 1u : 0u);
  const int64_t c = static_cast<int64_t>(kk - (uint64_t(1) << L));
  return static_cast<int32_t>((c < int64_t(N) + 1 ? c : int64_t(N) + 1) - 1);
}

// STAGE 1: the top levels in LDS, the rest through L1/L2; 2: all through
// L1/L2.  A lane descends its 4U queries in lockstep, so the gathers of one
// level are in flight together; vector indices past the end are clamped to
// the last vector and only the stores are guarded.
template <typename T, int STAGE, int U, bool VEC>
__global__ void __launch_bounds__(1024) eytzinger_kernel(EytArgs<T> a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const T* Yl = a.Y;
  int lt = 0;
  if constexpr (STAGE == 1) {
    lt = a.lds_levels;
    stage_bytes(smem, reinterpret_cast<const unsigned char*>(a.Y), (int64_t(1) << lt) * int64_t(sizeof(T)));
    __syncthreads();
    Yl = reinterpret_cast<const T*>(smem);
  }
  const int L = a.L;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (VEC) {
    // 16-byte vectors (4 f32 or 2 f64 queries) so each load of a wave covers
    // 1 KiB of contiguous queries; 4U queries per lane and iteration either way
    constexpr int W = 16 / int(sizeof(T));
    constexpr int UV = 4 * U / W;
    const int64_t nvec = a.M / W;
    const vecw<T, W>* zv = reinterpret_cast<const vecw<T, W>*>(a.z);
    ivecw<W>* ov = reinterpret_cast<ivecw<W>*>(a.out);
    const int64_t B = blockDim.x;
    const int64_t step = (int64_t)gridDim.x * B * UV;
    for (int64_t base = (int64_t)blockIdx.x * B * UV + threadIdx.x; base < nvec; base += step) {
      vecw<T, W> q[UV];
#pragma unroll
      for (int u = 0; u < UV; ++u) q[u] = __builtin_nontemporal_load(zv + std::min<int64_t>(base + u * B, nvec - 1));
      uint32_t k[UV][W];
#pragma unroll
      for (int u = 0; u < UV; ++u)
#pragma unroll
        for (int l = 0; l < W; ++l) k[u][l] = 1;
      for (int d = 0; d < lt; ++d) {
#pragma unroll
        for (int u = 0; u < UV; ++u)
#pragma unroll
          for (int l = 0; l < W; ++l) k[u][l] = 2 * k[u][l] + (q[u][l] >= Yl[k[u][l]] ? 1u : 0u);
      }
      uint64_t kk[UV][W];
#pragma unroll
      for (int u = 0; u < UV; ++u)
#pragma unroll
        for (int l = 0; l < W; ++l) kk[u][l] = k[u][l];
      for (int d = lt; d < L; ++d) {
#pragma unroll
        for (int u = 0; u < UV; ++u)
#pragma unroll
          for (int l = 0; l < W; ++l) kk[u][l] = 2 * kk[u][l] + (q[u][l] >= a.Y[kk[u][l]] ? 1u : 0u);
      }
#pragma unroll
      for (int u = 0; u < UV; ++u) {
        if (base + u * B < nvec) {
          ivecw<W> o;
#pragma unroll
          for (int l = 0; l < W; ++l) {
            const int64_t c = static_cast<int64_t>(kk[u][l] - (uint64_t(1) << L));
            o[l] = static_cast<int32_t>((c < int64_t(a.N) + 1 ? c : int64_t(a.N) + 1) - 1);
          }
          __builtin_nontemporal_store(o, ov + base + u * B);
        }
      }
    }
    const int64_t t = nvec * W + gtid;
    if (t < a.M) a.out[t] = eyt_one(a.z[t], Yl, a.Y, lt, L, a.N);
  } else {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t m = gtid; m < a.M; m += step) a.out[m] = eyt_one(a.z[m], Yl, a.Y, lt, L, a.N);
  }
}

int64_t lds_bytes_needed(const ds_index* h, int stage) {
  const int64_t s = (h->dt == DS_F32) ? 4 : 8;
  if (h->method == DS_METHOD_BSEARCH_EYTZINGER) {
    const int lt = (h->dt == DS_F32) ? eyt_lds_levels<float>(h->eyt_L) : eyt_lds_levels<double>(h->eyt_L);
    return (int64_t(1) << lt) * s;
  }
  if (h->method == DS_METHOD_DIRECT && stage == 3) {
    int64_t b = 0, c = 0;
    return rankcode_offsets(h->rc_words, round16((h->N + 1) * 2), &b, &c);
  }
  if (h->method == DS_METHOD_DIRECT && stage == 7) return nibble_chunks(h->nK) * int64_t(sizeof(NibChunk));
  if (h->method == DS_METHOD_DIRECT_GAP && stage == 8) {
    int64_t b = 0, c = 0;
    return rankcode_offsets(h->gc_words, round16((h->N + 1) * 2), &b, &c);
  }
  if (h->method == DS_METHOD_DIRECT && stage == 6)
    return std::min<int64_t>(nibble_chunks(h->nK), kNibPrefixChunks) * int64_t(sizeof(NibChunk));
  if (h->method == DS_METHOD_DIRECT || h->method == DS_METHOD_DIRECT_GAP) return round16(h->nX * s) + h->nK * 4;
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
    case 8: {  // GAPCODE in LDS, as RANKCODE
      const bool one_wg_per_cu = lds_bytes_needed(h, 8) > kLdsBytesPerCU / 2;
      *block = 1024;
      *unroll = (one_wg_per_cu && f32) ? 4 : 1;
      return;
    }
    case 4: *block = f32 ? 256 : 1024; *unroll = f32 ? 4 : 1; return;
    case 5: *block = 512; *unroll = 2; return;
    case 6: *block = f32 ? 1024 : 512; *unroll = 2; return;  // one workgroup per CU (the LDS prefix)
    case 7:  // two workgroups per CU when the chunks take at most half the LDS
      *block = 1024;
      *unroll = lds_bytes_needed(h, 7) > kLdsBytesPerCU / 2 ? 2 : 1;
      return;
    default: *block = 512; *unroll = 2; return;
  }
}

// The launch shape: the fields of *cand (the autotuner's candidate, which
// never touches the handle) or else of the handle's fixed tune that are set,
// the defaults for the rest.
Shape pick_shape(const ds_index* h, int64_t M, const ds_tune* cand) {
  Shape sh{};
  const bool set = cand != nullptr || h->tune_set;
  const ds_tune& t = cand ? *cand : h->tune;
  if (set && t.stage) {
    sh.stage = t.stage;
  } else if (h->method == DS_METHOD_DIRECT || h->method == DS_METHOD_DIRECT_GAP) {
    sh.stage = h->auto_stage;
  } else {
    sh.stage = h->staged ? 1 : 2;
  }
  int block = 512, unroll = 2;
  if (h->method == DS_METHOD_DIRECT || h->method == DS_METHOD_DIRECT_GAP) default_shape(h, sh.stage, &block, &unroll);
  sh.block = (set && t.block) ? t.block : block;
  sh.unroll = (set && t.unroll) ? t.unroll : unroll;
  sh.grid = (set && t.grid) ? t.grid : 0;
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
    case 6:
      return vec ? dispatch_direct_u<T, FORM, 6, true>(a, sh, lds, items, s)
                 : dispatch_direct_u<T, FORM, 6, false>(a, sh, lds, items, s);
    case 7:
      return vec ? dispatch_direct_u<T, FORM, 7, true>(a, sh, lds, items, s)
                 : dispatch_direct_u<T, FORM, 7, false>(a, sh, lds, items, s);
    default:
      return vec ? dispatch_direct_u<T, FORM, 2, true>(a, sh, 0, items, s)
                 : dispatch_direct_u<T, FORM, 2, false>(a, sh, 0, items, s);
  }
}

template <typename T, int FORM, int STAGE, bool VEC, int Q>
ds_status dispatch_gap_u(const DirectArgs<T>& a, const Shape& sh, int lds, int64_t items, hipStream_t s) {
  switch (sh.unroll) {
    case 1: return launch(gap_search_kernel<T, FORM, STAGE, 1, VEC, Q>, a, sh, lds, items, s);
    case 2: return launch(gap_search_kernel<T, FORM, STAGE, 2, VEC, Q>, a, sh, lds, items, s);
    default: return launch(gap_search_kernel<T, FORM, STAGE, 4, VEC, Q>, a, sh, lds, items, s);
  }
}

template <typename T, int FORM, int Q>
ds_status dispatch_gap_q(const DirectArgs<T>& a, const Shape& sh, bool vec, int lds, hipStream_t s) {
  const int64_t items = vec ? ((a.M >> 2) + sh.unroll - 1) / sh.unroll : a.M;
  if (sh.stage == 8) {  // GAPCODE: 2-bit counts for q <= 3, 4-bit counts for q <= 15
    // the bound on the keys per cell: 3, 4, 8 or 15
    if (a.gap_q <= 3)
      return vec ? dispatch_gap_u<T, FORM, 8, true, 3>(a, sh, lds, items, s)
                 : dispatch_gap_u<T, FORM, 8, false, 3>(a, sh, lds, items, s);
    if (a.gap_q <= 4)
      return vec ? dispatch_gap_u<T, FORM, 8, true, 4>(a, sh, lds, items, s)
                 : dispatch_gap_u<T, FORM, 8, false, 4>(a, sh, lds, items, s);
    if (a.gap_q <= 8)
      return vec ? dispatch_gap_u<T, FORM, 8, true, 8>(a, sh, lds, items, s)
                 : dispatch_gap_u<T, FORM, 8, false, 8>(a, sh, lds, items, s);
    return vec ? dispatch_gap_u<T, FORM, 8, true, 15>(a, sh, lds, items, s)
               : dispatch_gap_u<T, FORM, 8, false, 15>(a, sh, lds, items, s);
  }
  if (sh.stage == 1) {
    return vec ? dispatch_gap_u<T, FORM, 1, true, Q>(a, sh, lds, items, s)
               : dispatch_gap_u<T, FORM, 1, false, Q>(a, sh, lds, items, s);
  }
  return vec ? dispatch_gap_u<T, FORM, 2, true, Q>(a, sh, 0, items, s)
             : dispatch_gap_u<T, FORM, 2, false, Q>(a, sh, 0, items, s);
}

template <typename T, int FORM>
ds_status dispatch_gap(const DirectArgs<T>& a, const Shape& sh, bool vec, int lds, hipStream_t s) {
  if (a.gap_q <= 2) return dispatch_gap_q<T, FORM, 2>(a, sh, vec, lds, s);
  if (a.gap_q <= 4) return dispatch_gap_q<T, FORM, 4>(a, sh, vec, lds, s);
  return dispatch_gap_q<T, FORM, kMaxGapQ>(a, sh, vec, lds, s);
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

template <typename T, int STAGE, bool VEC>
ds_status dispatch_eyt_u(const EytArgs<T>& a, const Shape& sh, int lds, int64_t items, hipStream_t s) {
  switch (sh.unroll) {
    case 1: return launch(eytzinger_kernel<T, STAGE, 1, VEC>, a, sh, lds, items, s);
    case 2: return launch(eytzinger_kernel<T, STAGE, 2, VEC>, a, sh, lds, items, s);
    default: return launch(eytzinger_kernel<T, STAGE, 4, VEC>, a, sh, lds, items, s);
  }
}

template <typename T>
ds_status dispatch_eyt(const EytArgs<T>& a, const Shape& sh, bool vec, int lds, hipStream_t s) {
  const int64_t items = vec ? ((a.M >> 2) + sh.unroll - 1) / sh.unroll : a.M;
  if (sh.stage == 1) {
    return vec ? dispatch_eyt_u<T, 1, true>(a, sh, lds, items, s) : dispatch_eyt_u<T, 1, false>(a, sh, lds, items, s);
  }
  return vec ? dispatch_eyt_u<T, 2, true>(a, sh, 0, items, s) : dispatch_eyt_u<T, 2, false>(a, sh, 0, items, s);
}

template <typename T>
T X_N(const ds_index* h) {
  return T(h->XN);
}

template <typename T>
ds_status search_typed(const ds_index* h, const void* z, int64_t M, int32_t* out, hipStream_t s,
                       const ds_tune* cand) {
  const Shape sh = pick_shape(h, M, cand);
  const bool vec = ((reinterpret_cast<uintptr_t>(z) % (4 * sizeof(T))) == 0) &&
                   ((reinterpret_cast<uintptr_t>(out) % 16) == 0);
  const int lds = (sh.stage == 1 || sh.stage == 3 || sh.stage == 6 || sh.stage == 7 || sh.stage == 8)
                      ? static_cast<int>(lds_bytes_needed(h, sh.stage))
                      : 0;
  if (h->method == DS_METHOD_DIRECT || h->method == DS_METHOD_DIRECT_GAP) {
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
    a.rc_code8 = h->rc_code8;
    a.nW = static_cast<int32_t>(h->rc_words);
    if (h->method == DS_METHOD_DIRECT_GAP) {  // the GAPCODE words take the RANKCODE fields
      a.rc_bits = h->gc_counts;
      a.rc_base = h->gc_base;
      a.nW = static_cast<int32_t>(h->gc_words);
    }
    a.pairs = static_cast<const CachePair<T>*>(h->pairs);
    a.nib = h->nib;
    a.nib_chunks = h->nib_chunks;
    a.gap_q = h->gap_q;
    a.x_off = h->x_off;
    a.z = static_cast<const T*>(z);
    a.out = out;
    a.M = M;
    if (h->method == DS_METHOD_DIRECT_GAP)
      return (h->form == DS_FORM_FMA) ? dispatch_gap<T, DS_FORM_FMA>(a, sh, vec, lds, s)
                                      : dispatch_gap<T, DS_FORM_SUB>(a, sh, vec, lds, s);
    return (h->form == DS_FORM_FMA) ? dispatch_direct<T, DS_FORM_FMA>(a, sh, vec, lds, s)
                                    : dispatch_direct<T, DS_FORM_SUB>(a, sh, vec, lds, s);
  }
  if (h->method == DS_METHOD_BSEARCH_EYTZINGER) {
    EytArgs<T> e{};
    e.Y = static_cast<const T*>(h->X);
    e.L = h->eyt_L;
    e.lds_levels = eyt_lds_levels<T>(h->eyt_L);
    e.N = static_cast<int32_t>(h->N);
    e.z = static_cast<const T*>(z);
    e.out = out;
    e.M = M;
    return dispatch_eyt<T>(e, sh, vec, lds, s);
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
int64_t direct_lds_bytes(const ds_index* h, int stage) { return lds_bytes_needed(h, stage); }
int64_t rankcode_lds_bytes(const ds_index* h) { return lds_bytes_needed(h, 3); }

ds_status launch_search(ds_index* h, const void* z, int64_t M, int32_t* out, hipStream_t s, const ds_tune* cand) {
  if (h->method == DS_METHOD_LEARNED) return learned_search(h, z, M, out, s);
  return (h->dt == DS_F32) ? search_typed<float>(h, z, M, out, s, cand)
                           : search_typed<double>(h, z, M, out, s, cand);
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
  int stages[8];
  int n_stages = 0;
  if (h->method == DS_METHOD_DIRECT) {
    if (h->staged) stages[n_stages++] = 1;
    if (h->rc_code && ds::rankcode_lds_bytes(h) <= ds::kLdsBytesPerCU) stages[n_stages++] = 3;
    if (h->rc_w16) stages[n_stages++] = 5;
    if (h->nib) stages[n_stages++] = 6;
    if (h->nib && ds::direct_lds_bytes(h, 7) <= ds::kLdsBytesPerCU) stages[n_stages++] = 7;
    if (h->pairs) stages[n_stages++] = 4;
    stages[n_stages++] = 2;
  } else {
    if (h->staged) stages[n_stages++] = 1;
    if (h->gc_counts && ds::direct_lds_bytes(h, 8) <= ds::kLdsBytesPerCU) stages[n_stages++] = 8;
    stages[n_stages++] = 2;
  }
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
        const ds_tune cand{blocks[bi], unrolls[ui], stages[si], 0};
        st = ds::launch_search(h, z_dev, m, out_dev, s, &cand);  // warm-up
        if (st != DS_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) { st = DS_ERR_HIP; break; }
        for (int r = 0; r < 3 && st == DS_OK; ++r) st = ds::launch_search(h, z_dev, m, out_dev, s, &cand);
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
  if (st != DS_OK) return st;
  // the handle's tune is written once, with the choice (as ds_set_tune would)
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
  if (t->stage < 0 || t->stage > 8) return DS_ERR_ARG;
  if (h->method == DS_METHOD_LEARNED) {
    // learned: stage 1 = each lane reads its own lines, 2 = the wave reads them cooperatively
    if (t->stage > 2 || t->unroll != 0 || t->grid < 0) return DS_ERR_ARG;
    h->tune = *t;
    h->tune_set = true;
    return DS_OK;
  }
  if ((t->stage == 6 || t->stage == 7) && !h->nib) return DS_ERR_ARG;
  if (t->stage == 7 && ds::direct_lds_bytes(h, 7) > ds::kLdsBytesPerCU) return DS_ERR_ARG;
  if (t->stage == 5 && (!h->rc_w16 || !h->rc_code8)) return DS_ERR_ARG;
  if (t->stage == 1 && !h->staged) return DS_ERR_ARG;
  if (t->stage == 8) {  // GAPCODE: the gap-q variant with q <= 3
    if (h->method != DS_METHOD_DIRECT_GAP || !h->gc_counts || ds::direct_lds_bytes(h, 8) > ds::kLdsBytesPerCU)
      return DS_ERR_ARG;
  } else if (t->stage >= 3 && h->method != DS_METHOD_DIRECT) {
    return DS_ERR_ARG;
  }
  if (t->stage == 3 && (!h->rc_code || ds::rankcode_lds_bytes(h) > ds::kLdsBytesPerCU)) return DS_ERR_ARG;
  if (t->stage == 4 && !h->pairs) return DS_ERR_ARG;
  if (t->grid < 0) return DS_ERR_ARG;
  h->tune = *t;
  h->tune_set = true;
  return DS_OK;
}

}  // extern "C"
