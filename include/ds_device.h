/*
 * ds_device.h -- scalar-problem device API of the interval-search library.
 *
 * The paper distinguishes the vectorial problem, where a block of queries is
 * searched in one call (ds_search), from the scalar problem, where queries
 * become known one at a time (Sec. 2, "scalar search problem").  On a GPU the
 * scalar problem is a query that some other kernel holds in a register: this
 * header lets such a kernel run the Direct search (Sec. 4.2, algorithm Direct)
 * itself, on the tables of an index built by ds_build.
 *
 * Use: on the host, ds_get_view(handle, &view) fills a ds_view (plain values
 * and device pointers into the handle, valid until ds_destroy); pass the view
 * to a kernel by value and call ds_find_f32 / ds_find_f64 there.  Results are
 * those of ds_search on the same handle, bit for bit, including the
 * out-of-domain convention (-1 below X_0 and for NaN, N at or above X_N).
 *
 * The functions read the PLAIN tables (K and X) through the caches; they are
 * self-contained (this header depends on nothing but HIP) and evaluate the
 * grid map with exactly the operations of the library's own kernels: no
 * contraction of the subtraction form (compile callers with
 * -ffp-contract=off or leave the explicit operations below alone), one fma in
 * the FMA form.
 */
#ifndef DS_DEVICE_H_
#define DS_DEVICE_H_

#include <stdint.h>

typedef struct ds_view {
  int32_t dtype;       /* ds_dtype: 0 = f32, 1 = f64 */
  int32_t form;        /* ds_form: 0 = H (x - X_0), 1 = fma(H, x, -W) */
  int32_t N;           /* intervals; X has N + 1 values */
  int32_t jmin;        /* first grid index f(X_0): 0, or -1 in the FMA form */
  int32_t R;           /* last grid index f(X_N) */
  int32_t pad_;
  double H;            /* grid scale (exactly a value of the dtype) */
  double W;            /* m(H X_0) in the FMA form, else 0 */
  double X0;           /* X_0 */
  const void* X;       /* N + 1 values of the dtype (device) */
  const int32_t* K;    /* R - jmin + 1 entries, K[e] = K_{jmin + e} (device) */
} ds_view;

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>

/* j = f(z) clamped to [jmin, R] in floating point (a NaN goes to jmin),
 * t = K_j, i = t - 1 + [z >= X_t] (Sec. 4.2). */
#define DS_DEVICE_FIND_BODY(T, FLOOR, FMA)                                      \
  const T H = (T)v.H, W = (T)v.W, X0 = (T)v.X0;                                 \
  T g;                                                                          \
  if (v.form == 1) {                                                            \
    g = FMA(H, z, -W);                                                          \
  } else {                                                                      \
    const T d = z - X0;                                                         \
    g = H * d;                                                                  \
  }                                                                             \
  g = fmin(fmax(g, (T)v.jmin), (T)v.R);                                         \
  const int32_t j = (int32_t)FLOOR(g);                                          \
  const int32_t t = v.K[j - v.jmin];                                            \
  const T x = ((const T*)v.X)[t];                                               \
  return t - 1 + (z >= x ? 1 : 0);

static __device__ __forceinline__ int32_t ds_find_f32(const ds_view v, float z) {
  DS_DEVICE_FIND_BODY(float, floorf, fmaf)
}

static __device__ __forceinline__ int32_t ds_find_f64(const ds_view v, double z) {
  DS_DEVICE_FIND_BODY(double, floor, fma)
}

#undef DS_DEVICE_FIND_BODY
#endif /* __HIPCC__ */

#endif /* DS_DEVICE_H_ */
