"""CPU oracle for the interval search problem and the Direct-search build.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the GPU path.

The C part (``ds_oracle.c``) holds the result (classic binary search, Sec. 3.1),
the brute-force count, ComputeHR (Sec. 4.4.3), InitK (Sec. 4) and the Direct
search (Sec. 4.2); ``mlp`` holds the fp64 reference of the learned router.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ds_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_NOT_SORTED, ERR_NONFINITE, ERR_INFEASIBLE = 0, 1, 2, 3, 4
FORM_SUB, FORM_FMA = 0, 1
HSTART_PHI, HSTART_HBAR = 0, 1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-msse2", "-mfpmath=sse",
                               "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        for s, ct in (("f32", ctypes.c_float), ("f64", ctypes.c_double)):
            f = getattr(lib, f"oracle_search_{s}")
            f.argtypes, f.restype = [vp, i64, vp, i64, vp, i32], None
            f = getattr(lib, f"oracle_brute_{s}")
            f.argtypes, f.restype = [vp, i64, vp, i64, vp], None
            f = getattr(lib, f"oracle_compute_hr_{s}")
            f.argtypes = [vp, i64, i32, i32, ctypes.POINTER(ct), ctypes.POINTER(ct),
                          ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ct)]
            f.restype = i32
            f = getattr(lib, f"oracle_init_k_{s}")
            f.argtypes, f.restype = [vp, i64, i32, ct, ct, i64, i64, vp], i32
            f = getattr(lib, f"oracle_direct_{s}")
            f.argtypes, f.restype = [vp, i64, vp, i32, ct, ct, i64, i64, vp, i64, vp], None
            f = getattr(lib, f"oracle_eytzinger_layout_{s}")
            f.argtypes, f.restype = [vp, i64, i64, vp], i32
            f = getattr(lib, f"oracle_eytzinger_search_{s}")
            f.argtypes, f.restype = [vp, i64, i64, vp, i64, vp], None
            f = getattr(lib, f"oracle_compute_hr_gap_{s}")
            f.argtypes = [vp, i64, i64, i32, i32, ctypes.POINTER(ct), ctypes.POINTER(ct),
                          ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ct)]
            f.restype = i32
            f = getattr(lib, f"oracle_refine_h_{s}")
            f.argtypes = [vp, i64, i64, i32, ct, ct, ctypes.POINTER(ct), ctypes.POINTER(ct),
                          ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ct), ctypes.POINTER(i64)]
            f.restype = i32
            f = getattr(lib, f"oracle_init_k_gap_{s}")
            f.argtypes, f.restype = [vp, i64, i32, ct, ct, i64, i64, vp], i32
            f = getattr(lib, f"oracle_direct_gap_{s}")
            f.argtypes, f.restype = [vp, i64, i64, vp, i32, ct, ct, i64, i64, vp, i64, vp], None
        _lib = lib
    return _lib


def _suffix(dt) -> str:
    dt = np.dtype(dt)
    if dt == np.float32:
        return "f32"
    if dt == np.float64:
        return "f64"
    raise TypeError("float32 or float64 only")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def search(X: np.ndarray, z: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """i = #{k : X_k <= z} - 1 for each z (classic binary search, Sec. 3.1)."""
    X = np.ascontiguousarray(X)
    z = np.ascontiguousarray(z, dtype=X.dtype)
    out = np.empty(z.size, np.int32)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    getattr(_load(), f"oracle_search_{_suffix(X.dtype)}")(_ptr(X), X.size - 1, _ptr(z), z.size, _ptr(out), nthreads)
    return out


def brute(X: np.ndarray, z: np.ndarray) -> np.ndarray:
    """The same count by a linear scan over all of X (tiny inputs)."""
    X = np.ascontiguousarray(X)
    z = np.ascontiguousarray(z, dtype=X.dtype)
    out = np.empty(z.size, np.int32)
    getattr(_load(), f"oracle_brute_{_suffix(X.dtype)}")(_ptr(X), X.size - 1, _ptr(z), z.size, _ptr(out))
    return out


@dataclass
class DirectTables:
    status: int
    H: float = float("nan")
    W: float = float("nan")
    R: int = -1
    jmin: int = 0
    n_updates: int = 0
    K: np.ndarray | None = None   # K[j - jmin] = K_j, j in [jmin, R]
    form: int = FORM_SUB
    dtype: np.dtype = np.dtype(np.float32)
    q: int = 0                    # gap-q tables (Sec. 4.7); 0 for plain Direct
    H_bad: float = 0.0            # last H the growth loop found infeasible (0 = none)
    H_grown: float = float("nan")  # the H the growth loop ended with
    H_lo: float = 0.0             # refined: the infeasible float just below H
    n_refine: int = 0             # refined: midpoints tested by the bisection


def refine_h(X: np.ndarray, q: int, form: int, Hlo: float, Hhi: float):
    """Bisection of [Hlo (infeasible), Hhi (feasible)] (end of Sec. 4.4.3); q = 1 for plain
    Direct.  Returns (status, H, W, R, jmin, final Hlo, steps)."""
    X = np.ascontiguousarray(X)
    s = _suffix(X.dtype)
    ct = ctypes.c_float if s == "f32" else ctypes.c_double
    H, W, lo = ct(), ct(), ct()
    R, jmin, steps = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    st = getattr(_load(), f"oracle_refine_h_{s}")(_ptr(X), X.size - 1, q, form, Hlo, Hhi, ctypes.byref(H),
                                                    ctypes.byref(W), ctypes.byref(R), ctypes.byref(jmin),
                                                    ctypes.byref(lo), ctypes.byref(steps))
    return st, H.value, W.value, R.value, jmin.value, lo.value, steps.value


def _refined(X: np.ndarray, t: DirectTables, q: int) -> DirectTables:
    """t with H replaced by the bisection's result when the growth loop raised H."""
    if t.status != OK or t.n_updates == 0:
        return t
    st, H, W, R, jmin, lo, steps = refine_h(X, q, t.form, t.H_bad, t.H_grown)
    if st != OK:
        raise RuntimeError(f"refine_h rejected its interval: status {st}")
    t.H, t.W, t.R, t.jmin, t.H_lo, t.n_refine = H, W, R, jmin, lo, steps
    return t


def compute_hr(X: np.ndarray, form: int = FORM_SUB, hstart: int = HSTART_PHI,
               refine: bool = False) -> DirectTables:
    """ComputeHR (Sec. 4.4.3) in the chosen form; returns status, H, W, R, jmin, n_updates.
    refine: bisect between the last infeasible H and the grown one (end of Sec. 4.4.3)."""
    X = np.ascontiguousarray(X)
    s = _suffix(X.dtype)
    ct = ctypes.c_float if s == "f32" else ctypes.c_double
    H, W, Hb = ct(), ct(), ct()
    R, jmin, nu = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    st = getattr(_load(), f"oracle_compute_hr_{s}")(_ptr(X), X.size - 1, form, hstart, ctypes.byref(H),
                                                      ctypes.byref(W), ctypes.byref(R), ctypes.byref(jmin),
                                                      ctypes.byref(nu), ctypes.byref(Hb))
    if st != OK:
        return DirectTables(st, form=form, dtype=X.dtype)
    t = DirectTables(OK, H.value, W.value, R.value, jmin.value, nu.value, None, form, X.dtype,
                     H_bad=Hb.value, H_grown=H.value)
    return _refined(X, t, 1) if refine else t


def init_k(X: np.ndarray, H: float, W: float, R: int, jmin: int, form: int = FORM_SUB):
    """InitK (Sec. 4): K[j - jmin] = K_j for j in [jmin, R]; (status, K)."""
    X = np.ascontiguousarray(X)
    s = _suffix(X.dtype)
    K = np.empty(R - jmin + 1, np.int32)
    st = getattr(_load(), f"oracle_init_k_{s}")(_ptr(X), X.size - 1, form, H, W, jmin, R, _ptr(K))
    return st, K


def build_direct(X: np.ndarray, form: int = FORM_SUB, hstart: int = HSTART_PHI,
                 refine: bool = False) -> DirectTables:
    t = compute_hr(X, form, hstart, refine)
    if t.status != OK:
        return t
    st, K = init_k(X, t.H, t.W, t.R, t.jmin, form)
    t.status = st
    t.K = K
    return t


def direct(X: np.ndarray, t: DirectTables, z: np.ndarray) -> np.ndarray:
    """Direct search (Sec. 4.2) on the oracle's own tables; pins the build."""
    X = np.ascontiguousarray(X)
    z = np.ascontiguousarray(z, dtype=X.dtype)
    out = np.empty(z.size, np.int32)
    getattr(_load(), f"oracle_direct_{_suffix(X.dtype)}")(_ptr(X), X.size - 1, _ptr(t.K), t.form, t.H, t.W,
                                                           t.jmin, t.R, _ptr(z), z.size, _ptr(out))
    return out


# ---------------------------------------------------------------------------
# The gap-q variant (Sec. 4.7): f(X_{i+q}) > f(X_i), K_j = max{i : f(X_i) <= j},
# i = K_j - sum_{k<q} [z < X_{K_j - k}].

def compute_hr_gap(X: np.ndarray, q: int, form: int = FORM_SUB, hstart: int = HSTART_PHI,
                   refine: bool = False) -> DirectTables:
    """ComputeHR under eq. (f-monotonic-n); status, H, W, R, jmin, n_updates (1 <= q <= N)."""
    X = np.ascontiguousarray(X)
    s = _suffix(X.dtype)
    ct = ctypes.c_float if s == "f32" else ctypes.c_double
    H, W, Hb = ct(), ct(), ct()
    R, jmin, nu = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    st = getattr(_load(), f"oracle_compute_hr_gap_{s}")(_ptr(X), X.size - 1, q, form, hstart, ctypes.byref(H),
                                                          ctypes.byref(W), ctypes.byref(R), ctypes.byref(jmin),
                                                          ctypes.byref(nu), ctypes.byref(Hb))
    if st != OK:
        return DirectTables(st, form=form, dtype=X.dtype, q=q)
    t = DirectTables(OK, H.value, W.value, R.value, jmin.value, nu.value, None, form, X.dtype, q,
                     H_bad=Hb.value, H_grown=H.value)
    return _refined(X, t, q) if refine else t


def init_k_gap(X: np.ndarray, H: float, W: float, R: int, jmin: int, form: int = FORM_SUB):
    """eq. (kgeneral): K[j - jmin] = max{i : f(X_i) <= j}; (status, K)."""
    X = np.ascontiguousarray(X)
    K = np.empty(R - jmin + 1, np.int32)
    st = getattr(_load(), f"oracle_init_k_gap_{_suffix(X.dtype)}")(_ptr(X), X.size - 1, form, H, W, jmin, R, _ptr(K))
    return st, K


def build_direct_gap(X: np.ndarray, q: int, form: int = FORM_SUB, hstart: int = HSTART_PHI,
                     refine: bool = False) -> DirectTables:
    t = compute_hr_gap(X, q, form, hstart, refine)
    if t.status != OK:
        return t
    st, K = init_k_gap(X, t.H, t.W, t.R, t.jmin, form)
    t.status = st
    t.K = K
    return t


def direct_gap(X: np.ndarray, t: DirectTables, z: np.ndarray) -> np.ndarray:
    """eq. (index2) with q compares (algorithm DirectGap2 for q = 2) on the oracle's own tables."""
    X = np.ascontiguousarray(X)
    z = np.ascontiguousarray(z, dtype=X.dtype)
    out = np.empty(z.size, np.int32)
    getattr(_load(), f"oracle_direct_gap_{_suffix(X.dtype)}")(_ptr(X), X.size - 1, t.q, _ptr(t.K), t.form, t.H, t.W,
                                                               t.jmin, t.R, _ptr(z), z.size, _ptr(out))
    return out


# ---------------------------------------------------------------------------
# The Eytzinger layout and its search (Sec. 3.4).

def eytzinger_levels(N: int) -> int:
    """Smallest L with 2^L - 1 >= N + 1 (room for X_0..X_N)."""
    L = 1
    while (1 << L) - 1 < N + 1:
        L += 1
    return L


def eytzinger_layout(X: np.ndarray, L: int | None = None):
    """(status, Y): Y[1 .. 2^L - 1] the padded X in breadth-first tree order, Y[0] unused."""
    X = np.ascontiguousarray(X)
    N = X.size - 1
    L = eytzinger_levels(N) if L is None else L
    Y = np.empty(1 << L, X.dtype)
    st = getattr(_load(), f"oracle_eytzinger_layout_{_suffix(X.dtype)}")(_ptr(X), N, L, _ptr(Y))
    return st, Y


def eytzinger_search(Y: np.ndarray, N: int, L: int, z: np.ndarray) -> np.ndarray:
    """The L-level descent over Y; i = #{k : X_k <= z} - 1 like every search here."""
    Y = np.ascontiguousarray(Y)
    z = np.ascontiguousarray(z, dtype=Y.dtype)
    out = np.empty(z.size, np.int32)
    getattr(_load(), f"oracle_eytzinger_search_{_suffix(Y.dtype)}")(_ptr(Y), N, L, _ptr(z), z.size, _ptr(out))
    return out
