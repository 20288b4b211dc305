/*
 * Oracle for the interval search problem and for the Direct-search build.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links or calls it, and it shares no code, header or
 * constant with the product.
 *
 * Paper: F. Cannizzo, "A Fast and Vectorizable Alternative to Binary Search
 * in O(1) with Wide Applicability to Arrays of Floating Point Numbers".
 *
 * Contents
 *   oracle_search_*   the result itself (Sec. 2, Formal Problem Statement):
 *                     i with X_i <= z < X_{i+1}, computed with the classic
 *                     binary search (Sec. 3.1, algorithm "Classic"), extended
 *                     to out-of-domain z by i = #{k : X_k <= z} - 1.
 *   oracle_brute_*    the same count written as a linear scan (tiny N only).
 *   oracle_compute_hr_*  the choice of H and R (Sec. 4.4.3, algorithm
 *                     ComputeHR), in the subtraction form of eq. (function)
 *                     and in the FMA form of Sec. 4.9.
 *   oracle_init_k_*   the index table K (Sec. 4, eq. (indexdef), filled right
 *                     to left as in algorithm InitK).
 *   oracle_direct_*   the Direct search (Sec. 4.2, algorithm Direct) on the
 *                     oracle's own tables; used only to pin the build.
 *   oracle_eytzinger_layout_*, oracle_eytzinger_search_*
 *                     the cache-friendly binary search of Sec. 3.4: X padded
 *                     with X_N to 2^L - 1 values and stored in breadth-first
 *                     order of the complete search tree (the Eytzinger
 *                     layout), searched by descending L levels.
 *   oracle_refine_h_* the bisection of [last infeasible H, feasible H] that
 *                     the end of Sec. 4.4.3 proposes (not used by the paper's
 *                     own experiments); any q of the gap variant, q = 1 for
 *                     plain Direct.
 *   oracle_compute_hr_gap_*, oracle_init_k_gap_*, oracle_direct_gap_*
 *                     the relaxed variant of Sec. 4.7 ("Relaxing Limitations
 *                     and Reducing Memory Usage"): the grid only has to
 *                     satisfy f(X_{i+q}) > f(X_i) (eq. (f-monotonic-2) for
 *                     q = 2, eq. (f-monotonic-n) in general), K_j is
 *                     max{i : f(X_i) <= j} (eq. (kgeneral)), and the search
 *                     subtracts the q indicators [z < X_{t-k}], k < q
 *                     (eq. (index2), algorithm DirectGap2 for q = 2).
 *
 * Floating point: IEEE round-to-nearest-even, no contraction (the build file
 * passes -ffp-contract=off), denormals preserved, explicit fma() only in the
 * FMA form.  Comparisons are made in the array's own precision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* status codes (numerically equal to the product's, by the interface, not by
 * shared code) */
#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_NOT_SORTED 2
#define OR_ERR_NONFINITE 3
#define OR_ERR_INFEASIBLE 4

/* forms of the grid map f */
#define OR_FORM_SUB 0 /* f(x) = floor(m(H * m(x - X_0)))        eq. (function) */
#define OR_FORM_FMA 1 /* f(x) = floor(fma(H, x, -W)), W = m(H X_0)  Sec. 4.9   */

/* starting point of the H search */
#define OR_HSTART_PHI 0  /* H = phi(Hbar), as the text of Sec. 4.4.3 prints  */
#define OR_HSTART_HBAR 1 /* H = Hbar (reproduces the statistics of Table 101) */

/* Q = 31: grid indices and outputs are signed 32-bit integers. */
#define OR_TWO_POW_Q 2147483648.0

/*
 * The whole oracle is written once per precision through this macro; T is the
 * element type, S the symbol suffix, and FLOOR/FMA/NEXTUP the libm functions
 * of that precision.
 */
#define DEFINE_ORACLE(T, S, FLOOR, FMA, NEXTUP)                                  \
                                                                                 \
  /* Sec. 3.1, algorithm Classic: low = 0, high = N, halve until high-low=1. */ \
  static int64_t classic_##S(const T* X, int64_t N, T z) {                       \
    /* outside [X_0, X_N): the count #{k : X_k <= z} - 1 directly */             \
    if (!(z >= X[0])) return -1; /* also NaN: no X_k <= NaN */                   \
    if (z >= X[N]) return N;                                                     \
    int64_t low = 0, high = N;                                                   \
    while (high - low > 1) {                                                     \
      int64_t mid = (low + high) / 2;                                            \
      if (z < X[mid])                                                            \
        high = mid;                                                              \
      else                                                                       \
        low = mid;                                                               \
    }                                                                            \
    return low;                                                                  \
  }                                                                              \
                                                                                 \
  void oracle_search_##S(const T* X, int64_t N, const T* z, int64_t M,           \
                         int32_t* out, int nthreads) {                           \
    if (nthreads < 1) nthreads = 1;                                              \
    _Pragma("omp parallel for schedule(static) num_threads(nthreads)")           \
    for (int64_t k = 0; k < M; ++k) out[k] = (int32_t)classic_##S(X, N, z[k]);  \
  }                                                                              \
                                                                                 \
  /* i = #{k : X_k <= z} - 1, by a linear scan: the definition itself. */       \
  void oracle_brute_##S(const T* X, int64_t N, const T* z, int64_t M,            \
                        int32_t* out) {                                          \
    for (int64_t k = 0; k < M; ++k) {                                            \
      int64_t c = 0;                                                             \
      for (int64_t i = 0; i <= N; ++i) c += (X[i] <= z[k]) ? 1 : 0;              \
      out[k] = (int32_t)(c - 1);                                                 \
    }                                                                            \
  }                                                                              \
                                                                                 \
  /* the grid map f of eq. (function) or of Sec. 4.9, before the floor */       \
  static T grid_value_##S(int form, T H, T W, T X0, T x) {                       \
    if (form == OR_FORM_FMA) return FMA(H, x, -W);                               \
    T d = x - X0;                                                                \
    return H * d;                                                                \
  }                                                                              \
                                                                                 \
  /* Sec. 4.4.3, algorithm ComputeHR, with the readings listed in the design  \
   * notes: Q = 31, the overflow test is floor(m(H D_N)) >= 2^Q, the growth     \
   * term P is never reset, and after the pass over i = 1..N the whole pass is   \
   * repeated until it changes nothing (so every pair is verified under the     \
   * final H). */                                                                \
  int oracle_compute_hr_##S(const T* X, int64_t N, int form, int hstart,        \
                            T* H_out, T* W_out, int64_t* R_out,                  \
                            int64_t* jmin_out, int64_t* n_updates_out,           \
                            T* Hbad_out) {                                       \
    if (N < 1 || X == 0) return OR_ERR_ARG;                                      \
    for (int64_t i = 0; i <= N; ++i)                                             \
      if (!isfinite(X[i])) return OR_ERR_NONFINITE;                              \
    for (int64_t i = 0; i < N; ++i)                                              \
      if (!(X[i] < X[i + 1])) return OR_ERR_NOT_SORTED;                          \
    const T X0 = X[0];                                                           \
    /* eq. (distinguishable-exact): D_i = m(X_i - X_0) strictly increasing */    \
    T g = INFINITY;                                                              \
    for (int64_t i = 0; i < N; ++i) {                                            \
      T Di = X[i] - X0, Dn = X[i + 1] - X0;                                      \
      if (!(Di < Dn)) return OR_ERR_INFEASIBLE;                                  \
      T gap = Dn - Di; /* m(D_{i+1} - D_i) */                                    \
      if (gap < g) g = gap;                                                      \
    }                                                                            \
    /* eq. (minhnumeric): Hbar = m(1 / min gap) */                               \
    T one = 1;                                                                   \
    T Hbar = one / g;                                                            \
    if (isinf(Hbar)) return OR_ERR_INFEASIBLE;                                   \
    T H = (hstart == OR_HSTART_HBAR) ? Hbar : NEXTUP(Hbar, (T)INFINITY);         \
    T W = (form == OR_FORM_FMA) ? H * X0 : 0;                                    \
    if (FLOOR(grid_value_##S(form, H, W, X0, X[N])) >= (T)OR_TWO_POW_Q)          \
      return OR_ERR_INFEASIBLE;                                                  \
    T P = NEXTUP(H, (T)INFINITY) - H;                                            \
    int64_t n_updates = 0;                                                       \
    T Hbad = 0; /* last H seen to violate the condition; 0 = none */            \
    for (;;) {                                                                   \
      int changed = 0;                                                           \
      for (int64_t i = 1; i <= N; ++i) {                                         \
        /* eq. (cond2): floor(f(X_{i-1})) < floor(f(X_i)) must hold */           \
        while (FLOOR(grid_value_##S(form, H, W, X0, X[i - 1])) ==                \
               FLOOR(grid_value_##S(form, H, W, X0, X[i]))) {                    \
          Hbad = H;                                                              \
          H = H + P;                                                             \
          if (form == OR_FORM_FMA) W = H * X0;                                   \
          if (FLOOR(grid_value_##S(form, H, W, X0, X[N])) >= (T)OR_TWO_POW_Q)    \
            return OR_ERR_INFEASIBLE;                                            \
          P = P + P;                                                             \
          ++n_updates;                                                           \
          changed = 1;                                                           \
        }                                                                        \
      }                                                                          \
      if (!changed) break;                                                       \
    }                                                                            \
    *H_out = H;                                                                  \
    *W_out = W;                                                                  \
    *R_out = (int64_t)FLOOR(grid_value_##S(form, H, W, X0, X[N]));              \
    *jmin_out = (int64_t)FLOOR(grid_value_##S(form, H, W, X0, X[0]));           \
    *n_updates_out = n_updates;                                                  \
    if (Hbad_out) *Hbad_out = Hbad;                                              \
    return OR_OK;                                                                \
  }                                                                              \
                                                                                 \
  /* eq. (indexdef): K_j = i for f(X_{i-1}) < j <= f(X_i), K_{f(X_0)} = 0,     \
   * filled from the right as algorithm InitK does.  K has R - jmin + 1         \
   * entries; K[j - jmin] holds K_j. */                                          \
  int oracle_init_k_##S(const T* X, int64_t N, int form, T H, T W, int64_t jmin, \
                        int64_t R, int32_t* K) {                                 \
    const T X0 = X[0];                                                           \
    int64_t b = R;                                                               \
    for (int64_t i = N; i >= 0 && b >= jmin; --i) {                              \
      int64_t t = (int64_t)FLOOR(grid_value_##S(form, H, W, X0, X[i]));          \
      while (b > t) { /* cells strictly after f(X_i) and up to f(X_{i+1}) */     \
        K[b - jmin] = (int32_t)(i + 1);                                          \
        --b;                                                                     \
      }                                                                          \
      if (b != t) return OR_ERR_INFEASIBLE; /* f not strictly increasing */      \
      K[b - jmin] = (int32_t)i;                                                  \
      --b;                                                                       \
    }                                                                            \
    return (b == jmin - 1) ? OR_OK : OR_ERR_INFEASIBLE;                          \
  }                                                                              \
                                                                                 \
  /* Sec. 4.2, algorithm Direct: j = f(z), t = K_j, i = t - [z < X_t], with j  \
   * clamped to [jmin, R] in the floating-point domain first (fmax(NaN, a) = a  \
   * sends NaN to jmin), which leaves in-domain queries untouched and gives -1  \
   * below X_0 and N at or above X_N. */                                         \
  void oracle_direct_##S(const T* X, int64_t N, const int32_t* K, int form,     \
                         T H, T W, int64_t jmin, int64_t R, const T* z,          \
                         int64_t M, int32_t* out) {                              \
    (void)N;                                                                     \
    for (int64_t k = 0; k < M; ++k) {                                            \
      T v = grid_value_##S(form, H, W, X[0], z[k]);                              \
      if (!(v >= (T)jmin)) v = (T)jmin;                                          \
      if (v > (T)R) v = (T)R;                                                    \
      int64_t j = (int64_t)FLOOR(v);                                             \
      int64_t t = K[j - jmin];                                                   \
      /* [z >= X_t] is false for NaN, so NaN gives t - 1 = -1 */              \
      out[k] = (int32_t)(t - 1 + (z[k] >= X[t] ? 1 : 0));                        \
    }                                                                            \
  }

DEFINE_ORACLE(float, f32, floorf, fmaf, nextafterf)
DEFINE_ORACLE(double, f64, floor, fma, nextafter)

/*
 * The gap-q variant (Sec. 4.7), written once per precision like the above.
 */
#define DEFINE_ORACLE_GAP(T, S, FLOOR, FMA, NEXTUP)                              \
                                                                                 \
  /* ComputeHR with the condition of eq. (f-monotonic-n): the pairs checked   \
   * are (X_{i-q}, X_i) instead of neighbours, and the starting point is       \
   * Hbar = m(1 / min_i m(D_{i+q} - D_i)) (eq. (fcond11) in the rounded form of \
   * eq. (minhnumeric)); everything else (start phi(Hbar), growth term P never \
   * reset, passes repeated to a fixed point, overflow test) is as in          \
   * oracle_compute_hr.  q = 1 is plain Direct's condition. */                 \
  int oracle_compute_hr_gap_##S(const T* X, int64_t N, int64_t q, int form,     \
                                int hstart, T* H_out, T* W_out, int64_t* R_out,  \
                                int64_t* jmin_out, int64_t* n_updates_out,       \
                                T* Hbad_out) {                                   \
    if (N < 1 || X == 0 || q < 1 || q > N) return OR_ERR_ARG;                    \
    for (int64_t i = 0; i <= N; ++i)                                             \
      if (!isfinite(X[i])) return OR_ERR_NONFINITE;                              \
    for (int64_t i = 0; i < N; ++i)                                              \
      if (!(X[i] < X[i + 1])) return OR_ERR_NOT_SORTED;                          \
    const T X0 = X[0];                                                           \
    T g = INFINITY;                                                              \
    for (int64_t i = 0; i + q <= N; ++i) {                                       \
      T Di = X[i] - X0, Dq = X[i + q] - X0;                                      \
      if (!(Di < Dq)) return OR_ERR_INFEASIBLE;                                  \
      T gap = Dq - Di; /* m(D_{i+q} - D_i) */                                    \
      if (gap < g) g = gap;                                                      \
    }                                                                            \
    T one = 1;                                                                   \
    T Hbar = one / g;                                                            \
    if (isinf(Hbar)) return OR_ERR_INFEASIBLE;                                   \
    T H = (hstart == OR_HSTART_HBAR) ? Hbar : NEXTUP(Hbar, (T)INFINITY);         \
    T W = 0;                                                                     \
    if (form == OR_FORM_FMA) W = H * X0;                                         \
    if (FLOOR(grid_value_##S(form, H, W, X0, X[N])) >= (T)OR_TWO_POW_Q)          \
      return OR_ERR_INFEASIBLE;                                                  \
    T P = NEXTUP(H, (T)INFINITY) - H;                                            \
    int64_t n_updates = 0;                                                       \
    T Hbad = 0;                                                                  \
    for (;;) {                                                                   \
      int changed = 0;                                                           \
      for (int64_t i = q; i <= N; ++i) {                                         \
        while (FLOOR(grid_value_##S(form, H, W, X0, X[i - q])) ==                \
               FLOOR(grid_value_##S(form, H, W, X0, X[i]))) {                    \
          Hbad = H;                                                              \
          H = H + P;                                                             \
          if (form == OR_FORM_FMA) W = H * X0;                                   \
          if (FLOOR(grid_value_##S(form, H, W, X0, X[N])) >= (T)OR_TWO_POW_Q)    \
            return OR_ERR_INFEASIBLE;                                            \
          P = P + P;                                                             \
          ++n_updates;                                                           \
          changed = 1;                                                           \
        }                                                                        \
      }                                                                          \
      if (!changed) break;                                                       \
    }                                                                            \
    *H_out = H;                                                                  \
    *W_out = W;                                                                  \
    *R_out = (int64_t)FLOOR(grid_value_##S(form, H, W, X0, X[N]));              \
    *jmin_out = (int64_t)FLOOR(grid_value_##S(form, H, W, X0, X[0]));           \
    *n_updates_out = n_updates;                                                  \
    if (Hbad_out) *Hbad_out = Hbad;                                              \
    return OR_OK;                                                                \
  }                                                                              \
                                                                                 \
  /* Feasibility of one H: no overflow (eq. (overflowexact)) and              \
   * floor(f(X_{i-q})) < floor(f(X_i)) for every i in [q, N] (eq. (cond2) for \
   * q = 1, eq. (f-monotonic-n) otherwise). */                                  \
  static int feasible_##S(const T* X, int64_t N, int64_t q, int form, T H) {   \
    const T X0 = X[0];                                                           \
    const T W = (form == OR_FORM_FMA) ? H * X0 : 0;                              \
    if (FLOOR(grid_value_##S(form, H, W, X0, X[N])) >= (T)OR_TWO_POW_Q)          \
      return 0;                                                                  \
    for (int64_t i = q; i <= N; ++i)                                             \
      if (!(FLOOR(grid_value_##S(form, H, W, X0, X[i - q])) <                    \
            FLOOR(grid_value_##S(form, H, W, X0, X[i]))))                        \
        return 0;                                                                \
    return 1;                                                                    \
  }                                                                              \
                                                                                 \
  /* The refinement suggested at the end of Sec. 4.4.3: Hlo is known to be     \
   * infeasible and Hhi feasible; bisect [Hlo, Hhi] with the midpoint          \
   * Hlo + (Hhi - Hlo) / 2 rounded in the dtype, keeping an infeasible left    \
   * end and a feasible right end, until no float lies strictly between them.  \
   * Feasibility is not monotone in H, so the result is a feasible H whose     \
   * predecessor float is infeasible, not necessarily the smallest feasible H. \
   * Outputs the refined H with its W, R and jmin, the final left end and the  \
   * number of midpoints tested. */                                             \
  int oracle_refine_h_##S(const T* X, int64_t N, int64_t q, int form, T Hlo,    \
                          T Hhi, T* H_out, T* W_out, int64_t* R_out,             \
                          int64_t* jmin_out, T* Hlo_out, int64_t* steps_out) {   \
    if (N < 1 || X == 0 || q < 1 || q > N || !(Hlo > 0) || !(Hlo < Hhi))         \
      return OR_ERR_ARG;                                                         \
    if (feasible_##S(X, N, q, form, Hlo) || !feasible_##S(X, N, q, form, Hhi))   \
      return OR_ERR_ARG;                                                         \
    int64_t steps = 0;                                                           \
    for (;;) {                                                                   \
      T mid = Hlo + (Hhi - Hlo) / 2;                                             \
      if (!(Hlo < mid && mid < Hhi)) break;                                      \
      ++steps;                                                                   \
      if (feasible_##S(X, N, q, form, mid))                                      \
        Hhi = mid;                                                               \
      else                                                                       \
        Hlo = mid;                                                               \
    }                                                                            \
    const T X0 = X[0];                                                           \
    const T W = (form == OR_FORM_FMA) ? Hhi * X0 : 0;                            \
    *H_out = Hhi;                                                                \
    *W_out = W;                                                                  \
    *R_out = (int64_t)FLOOR(grid_value_##S(form, Hhi, W, X0, X[N]));            \
    *jmin_out = (int64_t)FLOOR(grid_value_##S(form, Hhi, W, X0, X[0]));         \
    *Hlo_out = Hlo;                                                              \
    *steps_out = steps;                                                          \
    return OR_OK;                                                                \
  }                                                                              \
                                                                                 \
  /* eq. (kgeneral): K_j = max{i : f(X_i) <= j} for j = jmin..R, by one scan  \
   * of the non-decreasing sequence f(X_i); K[j - jmin] holds K_j. */           \
  int oracle_init_k_gap_##S(const T* X, int64_t N, int form, T H, T W,           \
                            int64_t jmin, int64_t R, int32_t* K) {               \
    const T X0 = X[0];                                                           \
    int64_t i = 0;                                                               \
    for (int64_t j = jmin; j <= R; ++j) {                                        \
      while (i + 1 <= N &&                                                       \
             (int64_t)FLOOR(grid_value_##S(form, H, W, X0, X[i + 1])) <= j)      \
        ++i;                                                                     \
      if ((int64_t)FLOOR(grid_value_##S(form, H, W, X0, X[i])) > j)              \
        return OR_ERR_INFEASIBLE; /* only possible for j < f(X_0) */             \
      K[j - jmin] = (int32_t)i;                                                  \
    }                                                                            \
    return OR_OK;                                                                \
  }                                                                              \
                                                                                 \
  /* eq. (index2) for q compares: j = f(z) clamped to [jmin, R] in floating    \
   * point, t = K_j, i = t - sum_{k<q} [z < X_{t-k}], where X_{t-k} for        \
   * t - k < 0 is the left padding X_0 of the algorithm.  Below X_0 (and for   \
   * NaN) the result is -1, as everywhere else in this file. */                 \
  void oracle_direct_gap_##S(const T* X, int64_t N, int64_t q, const int32_t* K, \
                             int form, T H, T W, int64_t jmin, int64_t R,        \
                             const T* z, int64_t M, int32_t* out) {              \
    (void)N;                                                                     \
    for (int64_t k = 0; k < M; ++k) {                                            \
      if (!(z[k] >= X[0])) {                                                     \
        out[k] = -1;                                                             \
        continue;                                                                \
      }                                                                          \
      T v = grid_value_##S(form, H, W, X[0], z[k]);                              \
      if (!(v >= (T)jmin)) v = (T)jmin;                                          \
      if (v > (T)R) v = (T)R;                                                    \
      int64_t t = K[(int64_t)FLOOR(v) - jmin];                                   \
      int64_t i = t;                                                             \
      for (int64_t c = 0; c < q; ++c) {                                          \
        T x = (t - c >= 0) ? X[t - c] : X[0];                                    \
        if (z[k] < x) --i;                                                       \
      }                                                                          \
      out[k] = (int32_t)i;                                                       \
    }                                                                            \
  }

DEFINE_ORACLE_GAP(float, f32, floorf, fmaf, nextafterf)
DEFINE_ORACLE_GAP(double, f64, floor, fma, nextafter)

/*
 * Sec. 3.4, the Eytzinger layout: Y[1 .. 2^L - 1] holds the padded array
 * P_0 .. P_{2^L - 2} (P_i = X_i for i <= N, X_N after) in breadth-first order
 * of the complete binary search tree, node k having children 2k and 2k + 1
 * (Y[0] is unused).  L is the smallest height with 2^L - 1 >= N + 1.
 */
#define DEFINE_ORACLE_EYT(T, S)                                                  \
                                                                                 \
  /* in-order walk of the tree: the n-th node visited receives P_n */          \
  static void eyt_fill_##S(const T* X, int64_t N, int64_t nodes, int64_t k,     \
                           int64_t* next, T* Y) {                                \
    if (k > nodes) return;                                                       \
    eyt_fill_##S(X, N, nodes, 2 * k, next, Y);                                   \
    Y[k] = (*next <= N) ? X[*next] : X[N];                                       \
    ++*next;                                                                     \
    eyt_fill_##S(X, N, nodes, 2 * k + 1, next, Y);                               \
  }                                                                              \
                                                                                 \
  int oracle_eytzinger_layout_##S(const T* X, int64_t N, int64_t L, T* Y) {      \
    if (N < 1 || L < 1 || L > 40 || ((int64_t)1 << L) - 1 < N + 1) return OR_ERR_ARG; \
    const int64_t nodes = ((int64_t)1 << L) - 1;                                 \
    int64_t next = 0;                                                            \
    Y[0] = X[0];                                                                 \
    eyt_fill_##S(X, N, nodes, 1, &next, Y);                                      \
    return OR_OK;                                                                \
  }                                                                              \
                                                                                 \
  /* Descend L levels, k <- 2k + [z >= Y_k]; the leaf reached, k - 2^L, counts \
   * the padded values <= z (each step to the right passes a node and its left \
   * subtree).  i = min(count, N + 1) - 1: the pads equal X_N, so they only    \
   * count for z >= X_N, where the result is N; NaN counts nothing: -1. */     \
  void oracle_eytzinger_search_##S(const T* Y, int64_t N, int64_t L, const T* z, \
                                   int64_t M, int32_t* out) {                    \
    for (int64_t m = 0; m < M; ++m) {                                            \
      int64_t k = 1;                                                             \
      for (int64_t d = 0; d < L; ++d) k = 2 * k + (z[m] >= Y[k] ? 1 : 0);        \
      int64_t c = k - ((int64_t)1 << L);                                         \
      if (c > N + 1) c = N + 1;                                                  \
      out[m] = (int32_t)(c - 1);                                                 \
    }                                                                            \
  }

DEFINE_ORACLE_EYT(float, f32)
DEFINE_ORACLE_EYT(double, f64)
