// The two uses of interval search that motivate the problem (Sec. 2), with
// the Direct search fused into the consuming kernel, and the scalar-problem
// device API (ds_device.h):
//   * ds_histogram      samples per interval: the index goes straight into
//                       an LDS-private bin, so queries are read once and no
//                       index is written (bins too many for LDS beside the
//                       tables: up to four passes, each counting a range of
//                       bins in all of LDS with the tables read through L2;
//                       beyond that, one global atomic per sample);
//   * ds_interp_linear  piecewise-linear interpolation: index, then the knots
//                       X_i, X_{i+1}, Y_i, Y_{i+1}, then y, in one pass;
//   * ds_get_view / ds_view_search  the tables as a plain view, searched by a
//                       kernel built on ds_device.h alone.
// The fused kernels use the layout the automatic search uses (PLAIN or
// RANKCODE in LDS, NIBBLE through L2) through the same per-query operators;
// where the search stages NIBBLE in LDS they read it through L2, which leaves
// the LDS to the histogram's bins.
#include <algorithm>
#include <mutex>

#include "ds_ops.h"

namespace ds {

namespace {

// Stages the tables of the layout STAGE (1 = PLAIN in LDS, 3 = RANKCODE in
// LDS, 6 = NIBBLE through L2) and calls body(op, X) with the per-query
// operator and the X the knots are read from (LDS for PLAIN).  Every thread of
// the workgroup must call it (it holds a barrier).
template <typename T, int FORM, int STAGE, class Body>
__device__ __forceinline__ void with_direct_op(const DirectArgs<T>& a, unsigned char* smem, Body body) {
  if constexpr (STAGE == 1) {
    const int64_t xb = round16(int64_t(a.nX) * sizeof(T));
    stage_bytes(smem, reinterpret_cast<const unsigned char*>(a.X), int64_t(a.nX) * sizeof(T));
    stage_bytes(smem + xb, reinterpret_cast<const unsigned char*>(a.K), int64_t(a.nK) * 4);
    __syncthreads();
    const T* X = reinterpret_cast<const T*>(smem);
    const DirectOp<T, FORM> op{X, reinterpret_cast<const int32_t*>(smem + xb) - a.jmin, a.H, a.W, a.X0, a.vlo, a.vhi};
    body(op, X);
  } else if constexpr (STAGE == 3) {
    int64_t base_off = 0, code_off = 0;
    const int64_t code_bytes = round16(int64_t(a.N + 1) * 2);
    rankcode_offsets(a.nW, code_bytes, &base_off, &code_off);
    stage_bytes(smem, reinterpret_cast<const unsigned char*>(a.rc_bits), int64_t(a.nW) * 8);
    stage_bytes(smem + base_off, reinterpret_cast<const unsigned char*>(a.rc_base), int64_t(a.nW) * 4);
    stage_bytes(smem + code_off, reinterpret_cast<const unsigned char*>(a.rc_code), code_bytes);
    __syncthreads();
    const RankCodeOp<T, FORM, false> op{reinterpret_cast<const uint64_t*>(smem),
                                        reinterpret_cast<const uint32_t*>(smem + base_off),
                                        nullptr,
                                        reinterpret_cast<const uint16_t*>(smem + code_off),
                                        a.X, a.H, a.W, a.X0, a.vlo, a.vhi, a.XN, a.jmin, a.N};
    body(op, a.X);
  } else {
    const NibbleOp<T, FORM> op{a.nib, a.X, a.H, a.W, a.X0, a.vlo, a.vhi, a.XN, a.jmin, a.N};
    body(op, a.X);
  }
}

// Calls f(k, z_k) for every query: 16-byte vector loads (4 f32 or 2 f64
// values, so a wave's load covers 1 KiB of contiguous queries) when z is
// aligned (grid-stride over vectors, then the tail), scalar loads otherwise.
template <typename T, class F>
__device__ __forceinline__ void for_each_query(const T* __restrict__ z, int64_t M, bool vec, F f) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  if (vec) {
    constexpr int W = 16 / int(sizeof(T));
    const int64_t nvec = M / W;
    const vecw<T, W>* zv = reinterpret_cast<const vecw<T, W>*>(z);
    for (int64_t v = gtid; v < nvec; v += step) {
      const vecw<T, W> q = __builtin_nontemporal_load(zv + v);
#pragma unroll
      for (int l = 0; l < W; ++l) f(W * v + l, q[l]);
    }
    const int64_t t = nvec * W + gtid;
    if (t < M) f(t, z[t]);
  } else {
    for (int64_t k = gtid; k < M; k += step) f(k, z[k]);
  }
}

// Histogram: LDSBINS keeps N + 2 uint32 bins per workgroup after the staged
// tables (bins_off bytes in) and adds them to the global counters at the end.
template <typename T, int FORM, int STAGE, bool LDSBINS>
__global__ void __launch_bounds__(1024) hist_kernel(DirectArgs<T> a, int64_t bins_off, bool vec,
                                                    unsigned long long* __restrict__ counts) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  uint32_t* bins = reinterpret_cast<uint32_t*>(smem + bins_off);
  const int64_t nb = int64_t(a.N) + 2;
  if constexpr (LDSBINS) {
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) bins[b] = 0;
    __syncthreads();
  }
  with_direct_op<T, FORM, STAGE>(a, smem, [&](const auto& op, const T*) {
    for_each_query<T>(a.z, a.M, vec, [&](int64_t, T z) {
      const int32_t i = op(z);
      if constexpr (LDSBINS)
        atomicAdd(&bins[i + 1], 1u);
      else
        atomicAdd(&counts[i + 1], 1ull);
    });
  });
  if constexpr (LDSBINS) {
    __syncthreads();
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
      const uint32_t c = bins[b];
      if (c) atomicAdd(&counts[b], static_cast<unsigned long long>(c));
    }
  }
}

// Histogram of the bins [b0, b0 + nbl) only, in LDS (all of it), with the
// PLAIN tables read through L2: for arrays whose N + 2 bins fit neither
// beside the staged tables nor in one LDS, a few such passes over the queries
// (one launch each) beat one global atomic per sample.
template <typename T, int FORM>
__global__ void __launch_bounds__(1024) hist_range_kernel(DirectArgs<T> a, int64_t b0, int64_t nbl, bool vec,
                                                          unsigned long long* __restrict__ counts) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  uint32_t* bins = reinterpret_cast<uint32_t*>(smem);
  for (int64_t b = threadIdx.x; b < nbl; b += blockDim.x) bins[b] = 0;
  __syncthreads();
  const DirectOp<T, FORM> op{a.X, a.K - a.jmin, a.H, a.W, a.X0, a.vlo, a.vhi};
  for_each_query<T>(a.z, a.M, vec, [&](int64_t, T z) {
    const int64_t b = int64_t(op(z)) + 1 - b0;
    if (b >= 0 && b < nbl) atomicAdd(&bins[b], 1u);
  });
  __syncthreads();
  for (int64_t b = threadIdx.x; b < nbl; b += blockDim.x) {
    const uint32_t c = bins[b];
    if (c) atomicAdd(&counts[b0 + b], static_cast<unsigned long long>(c));
  }
}

// Piecewise-linear interpolation in T, no contraction (the library is built
// with -ffp-contract=off): the operation order is the one ds.h documents.
template <typename T, int FORM, int STAGE>
__global__ void __launch_bounds__(1024) interp_kernel(DirectArgs<T> a, bool vec, const T* __restrict__ Y,
                                                      T* __restrict__ y) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int32_t N = a.N;
  with_direct_op<T, FORM, STAGE>(a, smem, [&](const auto& op, const T* Xs) {
    for_each_query<T>(a.z, a.M, vec, [&](int64_t k, T z) {
      const int32_t i = op(z);
      T r;
      if (i < 0) {
        r = (z != z) ? z : Y[0];
      } else if (i >= N) {
        r = Y[N];
      } else {
        const T x0 = Xs[i], x1 = Xs[i + 1], y0 = Y[i], y1 = Y[i + 1];
        const T t = (z - x0) / (x1 - x0);
        const T dy = y1 - y0;
        const T p = t * dy;
        r = y0 + p;
      }
      y[k] = r;
    });
  });
}

// The scalar-problem API in use: one thread per query, ds_device.h only.
template <typename T>
__global__ void __launch_bounds__(256) view_search_kernel(const ds_view v, const T* __restrict__ z, int64_t M,
                                                          int32_t* __restrict__ out) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < M; k += step) {
    if constexpr (sizeof(T) == 4)
      out[k] = ds_find_f32(v, z[k]);
    else
      out[k] = ds_find_f64(v, z[k]);
  }
}

template <class KernelT>
int persistent_grid(KernelT kernel, int block, int lds, int64_t work) {
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (lds > 64 * 1024) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize, lds) !=
        hipSuccess)
      return -1;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t need = std::max<int64_t>(1, (work + block - 1) / block);
  return static_cast<int>(std::min<int64_t>(int64_t(per_cu) * num_cus(), need));
}

template <typename T>
DirectArgs<T> direct_args(const ds_index* h, const void* z, int64_t M) {
  DirectArgs<T> a{};
  a.X = static_cast<const T*>(h->X);
  a.K = h->K;
  a.H = T(h->H);
  a.W = T(h->W);
  a.X0 = T(h->X0);
  a.vlo = T(h->jmin);
  a.vhi = T(h->R);
  a.XN = T(h->XN);
  a.jmin = static_cast<int32_t>(h->jmin);
  a.nK = static_cast<int32_t>(h->nK);
  a.nX = static_cast<int32_t>(h->nX);
  a.N = static_cast<int32_t>(h->N);
  a.rc_bits = h->rc_bits;
  a.rc_base = h->rc_base;
  a.rc_code = h->rc_code;
  a.nW = static_cast<int32_t>(h->rc_words);
  a.nib = h->nib;
  a.z = static_cast<const T*>(z);
  a.M = M;
  return a;
}

constexpr int kAppBlock = 1024;

template <typename T, int FORM, int STAGE, bool LDSBINS>
ds_status launch_hist(const DirectArgs<T>& a, int64_t table_lds, int64_t bins_bytes, bool vec, uint64_t* counts,
                      hipStream_t s) {
  auto k = hist_kernel<T, FORM, STAGE, LDSBINS>;
  const int lds = static_cast<int>(LDSBINS ? table_lds + bins_bytes : table_lds);
  const int grid = persistent_grid(k, kAppBlock, lds, vec ? (a.M >> 2) : a.M);
  if (grid < 0) return DS_ERR_HIP;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kAppBlock), lds, s, a, table_lds, vec,
                     reinterpret_cast<unsigned long long*>(counts));
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

constexpr int kHistMaxPasses = 4;

template <typename T, int FORM, int STAGE>
ds_status hist_stage(const ds_index* h, const DirectArgs<T>& a, bool vec, uint64_t* counts, hipStream_t s) {
  const int64_t table_lds = (STAGE == 6) ? 0 : round16(direct_lds_bytes(h, STAGE));
  const int64_t nb = h->N + 2;
  const int64_t bins_bytes = round16(nb * 4);
  if (table_lds + bins_bytes <= kLdsBytesPerCU) return launch_hist<T, FORM, STAGE, true>(a, table_lds, bins_bytes, vec, counts, s);
  const int64_t per_pass = kLdsBytesPerCU / 4;
  const int64_t passes = (nb + per_pass - 1) / per_pass;
  if (passes > kHistMaxPasses) return launch_hist<T, FORM, STAGE, false>(a, table_lds, 0, vec, counts, s);
  auto k = hist_range_kernel<T, FORM>;
  const int lds = static_cast<int>(std::min<int64_t>(nb, per_pass) * 4);
  const int grid = persistent_grid(k, kAppBlock, lds, vec ? (a.M >> 2) : a.M);
  if (grid < 0) return DS_ERR_HIP;
  for (int64_t b0 = 0; b0 < nb; b0 += per_pass) {
    const int64_t nbl = std::min<int64_t>(per_pass, nb - b0);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kAppBlock), lds, s, a, b0, nbl, vec,
                       reinterpret_cast<unsigned long long*>(counts));
    DS_HIP_CHECK(hipGetLastError());
  }
  return DS_OK;
}

template <typename T, int FORM, int STAGE>
ds_status interp_stage(const ds_index* h, const DirectArgs<T>& a, bool vec, const T* Y, T* y, hipStream_t s) {
  auto k = interp_kernel<T, FORM, STAGE>;
  const int lds = static_cast<int>((STAGE == 6) ? 0 : direct_lds_bytes(h, STAGE));
  const int grid = persistent_grid(k, kAppBlock, lds, vec ? (a.M >> 2) : a.M);
  if (grid < 0) return DS_ERR_HIP;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kAppBlock), lds, s, a, vec, Y, y);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

// the automatic layout of a Direct handle: 1 (PLAIN in LDS), 3 (RANKCODE in LDS) or 6 and 7 (NIBBLE,
// read through L2)
template <typename T, int FORM>
ds_status hist_typed(const ds_index* h, const DirectArgs<T>& a, bool vec, uint64_t* counts, hipStream_t s) {
  switch (h->auto_stage) {
    case 1: return hist_stage<T, FORM, 1>(h, a, vec, counts, s);
    case 3: return hist_stage<T, FORM, 3>(h, a, vec, counts, s);
    default: return hist_stage<T, FORM, 6>(h, a, vec, counts, s);
  }
}

template <typename T, int FORM>
ds_status interp_typed(const ds_index* h, const DirectArgs<T>& a, bool vec, const T* Y, T* y, hipStream_t s) {
  switch (h->auto_stage) {
    case 1: return interp_stage<T, FORM, 1>(h, a, vec, Y, y, s);
    case 3: return interp_stage<T, FORM, 3>(h, a, vec, Y, y, s);
    default: return interp_stage<T, FORM, 6>(h, a, vec, Y, y, s);
  }
}

ds_status check_direct(ds_handle h) {
  if (!h) return DS_ERR_ARG;
  if (h->method != DS_METHOD_DIRECT) return DS_ERR_UNSUPPORTED;
  const bool built = (h->auto_stage == 1) || (h->auto_stage == 3 && h->rc_code) ||
                     ((h->auto_stage == 6 || h->auto_stage == 7) && h->nib);
  if (!built) return DS_ERR_UNSUPPORTED;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DS_ERR_HIP;
  return dev == h->device ? DS_OK : DS_ERR_ARG;
}

}  // namespace

}  // namespace ds

extern "C" {

ds_status ds_get_view(ds_handle h, ds_view* v) {
  if (!h || !v) return DS_ERR_ARG;
  if (h->method != DS_METHOD_DIRECT) return DS_ERR_UNSUPPORTED;
  ds_view out{};
  out.dtype = h->dt;
  out.form = h->form;
  out.N = static_cast<int32_t>(h->N);
  out.jmin = static_cast<int32_t>(h->jmin);
  out.R = static_cast<int32_t>(h->R);
  out.H = h->H;
  out.W = h->W;
  out.X0 = h->X0;
  out.X = h->X;
  out.K = h->K;
  *v = out;
  return DS_OK;
}

ds_status ds_view_search(const ds_view* v, const void* z_dev, int64_t M, int32_t* out_dev, hipStream_t s) {
  if (!v || M < 0) return DS_ERR_ARG;
  if (M == 0) return DS_OK;
  if (!z_dev || !out_dev || !v->X || !v->K || v->N < 1 || (v->dtype != DS_F32 && v->dtype != DS_F64)) return DS_ERR_ARG;
  const int block = 256;
  const int64_t grid = std::min<int64_t>((M + block - 1) / block, int64_t(ds::num_cus()) * 64);
  if (v->dtype == DS_F32)
    hipLaunchKernelGGL(ds::view_search_kernel<float>, dim3((unsigned)grid), dim3(block), 0, s, *v,
                       static_cast<const float*>(z_dev), M, out_dev);
  else
    hipLaunchKernelGGL(ds::view_search_kernel<double>, dim3((unsigned)grid), dim3(block), 0, s, *v,
                       static_cast<const double*>(z_dev), M, out_dev);
  DS_HIP_CHECK(hipGetLastError());
  return DS_OK;
}

ds_status ds_histogram(ds_handle h, const void* z_dev, int64_t M, uint64_t* counts_dev, hipStream_t s) {
  ds_status st = ds::check_direct(h);
  if (st != DS_OK) return st;
  if (M < 0 || !counts_dev) return DS_ERR_ARG;
  if (M == 0) return DS_OK;
  if (!z_dev) return DS_ERR_ARG;
  const int64_t S = (h->dt == DS_F32) ? 4 : 8;
  const bool vec = (reinterpret_cast<uintptr_t>(z_dev) % (4 * S)) == 0;
  if (h->dt == DS_F32) {
    const auto a = ds::direct_args<float>(h, z_dev, M);
    return (h->form == DS_FORM_FMA) ? ds::hist_typed<float, DS_FORM_FMA>(h, a, vec, counts_dev, s)
                                    : ds::hist_typed<float, DS_FORM_SUB>(h, a, vec, counts_dev, s);
  }
  const auto a = ds::direct_args<double>(h, z_dev, M);
  return (h->form == DS_FORM_FMA) ? ds::hist_typed<double, DS_FORM_FMA>(h, a, vec, counts_dev, s)
                                  : ds::hist_typed<double, DS_FORM_SUB>(h, a, vec, counts_dev, s);
}

ds_status ds_interp_linear(ds_handle h, const void* Y_dev, const void* z_dev, int64_t M, void* y_dev, hipStream_t s) {
  ds_status st = ds::check_direct(h);
  if (st != DS_OK) return st;
  if (M < 0 || !Y_dev || !y_dev) return DS_ERR_ARG;
  if (M == 0) return DS_OK;
  if (!z_dev) return DS_ERR_ARG;
  const int64_t S = (h->dt == DS_F32) ? 4 : 8;
  const bool vec = (reinterpret_cast<uintptr_t>(z_dev) % (4 * S)) == 0;
  if (h->dt == DS_F32) {
    const auto a = ds::direct_args<float>(h, z_dev, M);
    return (h->form == DS_FORM_FMA)
               ? ds::interp_typed<float, DS_FORM_FMA>(h, a, vec, static_cast<const float*>(Y_dev), static_cast<float*>(y_dev), s)
               : ds::interp_typed<float, DS_FORM_SUB>(h, a, vec, static_cast<const float*>(Y_dev), static_cast<float*>(y_dev), s);
  }
  const auto a = ds::direct_args<double>(h, z_dev, M);
  return (h->form == DS_FORM_FMA)
             ? ds::interp_typed<double, DS_FORM_FMA>(h, a, vec, static_cast<const double*>(Y_dev), static_cast<double*>(y_dev), s)
             : ds::interp_typed<double, DS_FORM_SUB>(h, a, vec, static_cast<const double*>(Y_dev), static_cast<double*>(y_dev), s);
}

}  // extern "C"
