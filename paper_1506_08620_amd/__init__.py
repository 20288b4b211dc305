"""Interval search on AMD MI355X: the Direct method of Cannizzo (arXiv 1506.08620).

Thin ctypes binding over ``libds.so`` (declared in ``include/ds.h``).  The
functions here only marshal arguments: every step of the build and of the
search runs in the library's HIP kernels.  PyTorch provides device memory and
streams.

    import torch, paper_1506_08620_amd as ds
    idx = ds.build(x)                  # x: strictly increasing float32/float64 on the GPU
    out = ds.search(idx, z)            # int32 indices i with x[i] <= z < x[i+1]

The library must be built first (``python paper_1506_08620_amd/build_lib.py``);
importing this package without it raises ImportError rather than falling back
to anything else.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first: libds.so then binds to the HIP runtime torch already holds

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libds.so")

# ---- enums of ds.h --------------------------------------------------------
F32, F64 = 0, 1
(OK, ERR_ARG, ERR_NOT_SORTED, ERR_NONFINITE, ERR_INFEASIBLE, ERR_TABLE_CAP, ERR_OOM, ERR_HIP, ERR_UNSUPPORTED,
 ERR_SCRATCH_CAP) = range(10)
NOALLOC_SCRATCH_BYTES = 64 << 20  # DS_NOALLOC_SCRATCH_BYTES
FORM_SUB, FORM_FMA = 0, 1
HSTART_PHI, HSTART_HBAR = 0, 1
(METHOD_DIRECT, METHOD_BSEARCH_LEADBIT, METHOD_BSEARCH_OFFSET, METHOD_LEARNED, METHOD_AUTO, METHOD_DIRECT_GAP,
 METHOD_BSEARCH_EYTZINGER) = range(7)
MAX_GAP_Q = 16
FALLBACK_NONE, FALLBACK_BSEARCH, FALLBACK_LEARNED = range(3)
LAYOUT_RANKCODE, LAYOUT_PAIRS, LAYOUT_NIBBLE = 1, 2, 4
# ds_tune.stage values of the Direct method
STAGE_PLAIN_LDS, STAGE_PLAIN_L2, STAGE_RANKCODE_LDS, STAGE_PAIRS_L2, STAGE_RANKCODE_L2, STAGE_NIBBLE_L2 = 1, 2, 3, 4, 5, 6
STAGE_NIBBLE_LDS = 7
STAGE_GAPCODE_LDS = 8
_LAYOUTS = {"rankcode": LAYOUT_RANKCODE, "pairs": LAYOUT_PAIRS, "nibble": LAYOUT_NIBBLE}

_METHODS = {"direct": METHOD_DIRECT, "leadbit": METHOD_BSEARCH_LEADBIT, "offset": METHOD_BSEARCH_OFFSET,
            "learned": METHOD_LEARNED, "auto": METHOD_AUTO, "direct_gap": METHOD_DIRECT_GAP,
            "eytzinger": METHOD_BSEARCH_EYTZINGER}
_FORMS = {"sub": FORM_SUB, "fma": FORM_FMA}
_HSTARTS = {"phi": HSTART_PHI, "hbar": HSTART_HBAR}
_FALLBACKS = {"none": FALLBACK_NONE, "bsearch": FALLBACK_BSEARCH, "learned": FALLBACK_LEARNED}
LEARN_FP32_ROUTER, LEARN_EVAL_ROUTER = 1, 2
_LEARN_ROUTERS = {"table": 0, "fp16": LEARN_EVAL_ROUTER, "fp32": LEARN_FP32_ROUTER}
METHOD_NAMES = {v: k for k, v in _METHODS.items()}

# exported symbols of libds.so (every function ds.h declares)
SYMBOLS = ("ds_build", "ds_search", "ds_set_tune", "ds_autotune", "ds_info", "ds_copy_table", "ds_destroy", "ds_status_str",
           "ds_batch_workspace_bytes", "ds_search_batched", "ds_search_batched_noalloc", "ds_batch_autotune",
           "ds_batch_report",
           "ds_batch_fallbacks",
           "ds_learned_grad", "ds_learned_forward", "ds_learned_model", "ds_learned_route",
           "ds_get_view", "ds_view_search", "ds_histogram", "ds_interp_linear")
N_ROUTER_PARAMS = 1153


class BuildOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("form", ctypes.c_int32), ("hstart", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("table_cap_bytes", ctypes.c_int64),
                ("learn_epochs", ctypes.c_int32), ("learn_segments", ctypes.c_int32),
                ("learn_rate", ctypes.c_float), ("learn_batch", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("extra_layouts", ctypes.c_int32), ("learn_flags", ctypes.c_int32), ("gap_q", ctypes.c_int32),
                ("refine_h", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("dtype", ctypes.c_int32), ("form", ctypes.c_int32),
                ("staged", ctypes.c_int32), ("N", ctypes.c_int64), ("H", ctypes.c_double),
                ("W", ctypes.c_double), ("X0", ctypes.c_double), ("R", ctypes.c_int64),
                ("jmin", ctypes.c_int64), ("n_h_updates", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("model_bytes", ctypes.c_int64), ("max_err", ctypes.c_int64),
                ("mean_log2_window", ctypes.c_double), ("x_bytes", ctypes.c_int64),
                ("rankcode_bytes", ctypes.c_int64), ("pairs_bytes", ctypes.c_int64), ("build_ms", ctypes.c_double),
                ("nibble_bytes", ctypes.c_int64), ("gap_q", ctypes.c_int32), ("n_h_refine", ctypes.c_int32),
                ("gapcode_bytes", ctypes.c_int64), ("fallback_count", ctypes.c_uint64)]


class View(ctypes.Structure):
    """ds_view of ds_device.h: the Direct tables for the scalar-problem device API."""
    _fields_ = [("dtype", ctypes.c_int32), ("form", ctypes.c_int32), ("N", ctypes.c_int32), ("jmin", ctypes.c_int32),
                ("R", ctypes.c_int32), ("pad_", ctypes.c_int32), ("H", ctypes.c_double), ("W", ctypes.c_double),
                ("X0", ctypes.c_double), ("X", ctypes.c_void_p), ("K", ctypes.c_void_p)]


class Tune(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("unroll", ctypes.c_int32), ("stage", ctypes.c_int32),
                ("grid", ctypes.c_int32)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("num_arrays", ctypes.c_int32),
                ("x_off_dev", ctypes.c_void_p), ("X_dev", ctypes.c_void_p),
                ("q_off_dev", ctypes.c_void_p), ("z_dev", ctypes.c_void_p), ("out_dev", ctypes.c_void_p),
                ("workspace_dev", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("total_x", ctypes.c_int64), ("total_q", ctypes.c_int64), ("form", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("block", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("qpt", ctypes.c_int32), ("learn_segments", ctypes.c_int32), ("learn_steps", ctypes.c_int32),
                ("reserved_", ctypes.c_int32), ("direct_cap_bytes", ctypes.c_int64)]


class DsError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} (status {status})")


def _load_library():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_1506_08620_amd/build_lib.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.ds_build.argtypes = [vp, i64, i32, ctypes.POINTER(BuildOpts), vp, ctypes.POINTER(vp)]
    lib.ds_build.restype = i32
    lib.ds_search.argtypes = [vp, vp, i64, vp, vp]
    lib.ds_search.restype = i32
    lib.ds_set_tune.argtypes = [vp, ctypes.POINTER(Tune)]
    lib.ds_set_tune.restype = i32
    lib.ds_autotune.argtypes = [vp, vp, i64, vp, vp, ctypes.POINTER(Tune)]
    lib.ds_autotune.restype = i32
    lib.ds_info.argtypes = [vp, ctypes.POINTER(Info)]
    lib.ds_info.restype = i32
    lib.ds_copy_table.argtypes = [vp, vp, i64, vp]
    lib.ds_copy_table.restype = i32
    lib.ds_destroy.argtypes = [vp]
    lib.ds_destroy.restype = i32
    lib.ds_status_str.argtypes = [i32]
    lib.ds_status_str.restype = ctypes.c_char_p
    lib.ds_batch_workspace_bytes.argtypes = [i32, i64, i64, i32]
    lib.ds_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.ds_search_batched.argtypes = [ctypes.POINTER(BatchDesc), vp]
    lib.ds_search_batched.restype = i32
    lib.ds_search_batched_noalloc.argtypes = [ctypes.POINTER(BatchDesc), vp]
    lib.ds_search_batched_noalloc.restype = i32
    lib.ds_learned_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.ds_learned_grad.restype = i32
    lib.ds_learned_forward.argtypes = [vp, vp, i64, i32, vp, vp]
    lib.ds_learned_forward.restype = i32
    lib.ds_learned_model.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_uint64), vp]
    lib.ds_learned_model.restype = i32
    lib.ds_learned_route.argtypes = [vp, vp, i64, i32, vp, vp]
    lib.ds_learned_route.restype = i32
    lib.ds_batch_fallbacks.argtypes = [ctypes.POINTER(BatchDesc), ctypes.POINTER(ctypes.c_uint64), vp]
    lib.ds_batch_fallbacks.restype = i32
    lib.ds_batch_autotune.argtypes = [ctypes.POINTER(BatchDesc), vp]
    lib.ds_batch_autotune.restype = i32
    lib.ds_batch_report.argtypes = [ctypes.POINTER(BatchDesc), vp, vp, vp]
    lib.ds_batch_report.restype = i32
    lib.ds_get_view.argtypes = [vp, ctypes.POINTER(View)]
    lib.ds_get_view.restype = i32
    lib.ds_view_search.argtypes = [ctypes.POINTER(View), vp, i64, vp, vp]
    lib.ds_view_search.restype = i32
    lib.ds_histogram.argtypes = [vp, vp, i64, vp, vp]
    lib.ds_histogram.restype = i32
    lib.ds_interp_linear.argtypes = [vp, vp, vp, i64, vp, vp]
    lib.ds_interp_linear.restype = i32
    return lib


_lib = _load_library()


def status_str(status: int) -> str:
    return _lib.ds_status_str(int(status)).decode()


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("float32 or float64 tensors only")


def _check_device(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Index:
    """A built search index (wraps ds_handle)."""

    def __init__(self, handle: int, dtype: torch.dtype, device: torch.device):
        self._h = ctypes.c_void_p(handle)
        self.dtype = dtype
        self.device = device

    @property
    def handle(self) -> int:
        return self._h.value or 0

    def search(self, z: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        return search(self, z, out=out, stream=stream)

    def info(self) -> dict:
        return info(self)

    def table(self, stream=None) -> torch.Tensor:
        """The Direct table K (entry e holds K_{jmin+e}) as an int32 GPU tensor."""
        inf = self.info()
        n = inf["R"] - inf["jmin"] + 1
        dst = torch.empty(n, dtype=torch.int32, device=self.device)
        st = _lib.ds_copy_table(self._h, dst.data_ptr(), n, _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_copy_table")
        return dst

    def set_tune(self, block: int = 0, unroll: int = 0, stage: int = 0, grid: int = 0):
        t = Tune(block, unroll, stage, grid)
        st = _lib.ds_set_tune(self._h, ctypes.byref(t))
        if st != OK:
            raise DsError(st, "ds_set_tune")

    def autotune(self, z: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> dict:
        """ds_autotune on queries z; returns the chosen launch shape."""
        _check_device(z, "z")
        if out is None:
            out = torch.empty(z.numel(), dtype=torch.int32, device=z.device)
        t = Tune()
        st = _lib.ds_autotune(self._h, z.data_ptr(), z.numel(), out.data_ptr(), _stream_handle(stream),
                              ctypes.byref(t))
        if st != OK:
            raise DsError(st, "ds_autotune")
        return {name: getattr(t, name) for name, _ in Tune._fields_}

    def view(self) -> View:
        """ds_get_view: the Direct tables as a ds_view (valid while this index lives)."""
        v = View()
        st = _lib.ds_get_view(self._h, ctypes.byref(v))
        if st != OK:
            raise DsError(st, "ds_get_view")
        return v

    def histogram(self, z: torch.Tensor, counts: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """ds_histogram: adds the number of queries per interval to counts (N + 2 int64,
        bin i + 1 for result i; zeros if not given)."""
        _check_device(z, "z")
        if z.dtype != self.dtype or not z.is_contiguous():
            raise ValueError("z must be a contiguous tensor of the index dtype")
        n = self.info()["N"]
        if counts is None:
            counts = torch.zeros(n + 2, dtype=torch.int64, device=z.device)
        if counts.dtype != torch.int64 or counts.numel() != n + 2 or not counts.is_contiguous():
            raise ValueError("counts must be N + 2 contiguous int64")
        st = _lib.ds_histogram(self._h, z.data_ptr(), z.numel(), counts.data_ptr(), _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_histogram")
        return counts

    def interp_linear(self, Y: torch.Tensor, z: torch.Tensor, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
        """ds_interp_linear: piecewise-linear interpolation of the knots (X_i, Y_i) at z."""
        _check_device(z, "z")
        _check_device(Y, "Y")
        if z.dtype != self.dtype or Y.dtype != self.dtype or not z.is_contiguous() or not Y.is_contiguous():
            raise ValueError("Y and z must be contiguous tensors of the index dtype")
        if Y.numel() != self.info()["N"] + 1:
            raise ValueError("Y must hold N + 1 values")
        if out is None:
            out = torch.empty_like(z)
        st = _lib.ds_interp_linear(self._h, Y.data_ptr(), z.data_ptr(), z.numel(), out.data_ptr(),
                                   _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_interp_linear")
        return out

    def learned_model(self, stream=None):
        """(trained router parameters as a numpy float32 array, fallback count)."""
        import numpy as np

        p = np.empty(N_ROUTER_PARAMS, np.float32)
        fb = ctypes.c_uint64()
        st = _lib.ds_learned_model(self._h, p.ctypes.data, p.size, ctypes.byref(fb), _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_learned_model")
        return p, int(fb.value)

    def learned_route(self, u, mode: int = 0, stream=None):
        """Segments of the f32 features u (device tensor) by the handle's router:
        mode 0 as the search routes queries, 1 the network evaluated in FP32,
        2 as the build routed the keys."""
        u = u.contiguous()
        if u.dtype != torch.float32 or not u.is_cuda:
            raise ValueError("u must be a float32 device tensor")
        seg = torch.empty(u.numel(), dtype=torch.int32, device=u.device)
        st = _lib.ds_learned_route(self._h, u.data_ptr(), u.numel(), int(mode), seg.data_ptr(),
                                   _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_learned_route")
        return seg

    def clear_tune(self):
        st = _lib.ds_set_tune(self._h, None)
        if st != OK:
            raise DsError(st, "ds_set_tune")

    def destroy(self):
        if self._h.value:
            torch.cuda.synchronize(self.device)
            _lib.ds_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            if self._h.value:
                _lib.ds_destroy(self._h)
                self._h = ctypes.c_void_p(0)
        except Exception:
            pass


def build(x: torch.Tensor, *, method: str = "direct", form: str = "sub", hstart: str = "phi",
          fallback: str = "none", table_cap_bytes: int = 0, learn_epochs: int = 0, learn_segments: int = 0,
          learn_rate: float = 0.0, learn_batch: int = 0, seed: int = 0, layouts=(), learn_fp32_router: bool = False,
          learn_router: str = "table", gap_q: int = 0, refine_h: bool = False, stream=None) -> Index:
    """ds_build over the N+1 values of x (a strictly increasing GPU tensor).

    layouts: extra Direct layouts to build besides the automatic one
    ("rankcode", "pairs", "nibble"), so that set_tune(stage=...) can select them.
    gap_q: method "direct_gap" (Sec. 4.7): compares per query, 1..16, or 0 for the
    smallest q whose table fits table_cap_bytes.
    refine_h: when ComputeHR had to grow H, bisect between the last failing H and the
    grown one (end of Sec. 4.4.3); info()["n_h_refine"] counts the midpoints tested.
    learn_router: how the learned method routes keys and queries: "table" (the FP32
    network's exact step table, the default), "fp16" or "fp32" (the network evaluated per
    query on the matrix cores, 32x32 layer with FP16 or FP32 inputs);
    learn_fp32_router=True is "fp32".
    """
    _check_device(x, "x")
    if x.dim() != 1 or x.numel() < 2:
        raise ValueError("x must be 1-D with at least two values")
    router = "fp32" if learn_fp32_router else learn_router
    opts = BuildOpts(_METHODS[method], _FORMS[form], _HSTARTS[hstart], _FALLBACKS[fallback], int(table_cap_bytes),
                     int(learn_epochs), int(learn_segments), float(learn_rate), int(learn_batch), int(seed),
                     sum(_LAYOUTS[k] for k in set(layouts)), _LEARN_ROUTERS[router], int(gap_q),
                     1 if refine_h else 0)
    h = ctypes.c_void_p()
    with torch.cuda.device(x.device):
        st = _lib.ds_build(x.data_ptr(), x.numel() - 1, _dtype_code(x), ctypes.byref(opts), _stream_handle(stream),
                           ctypes.byref(h))
    if st != OK:
        raise DsError(st, "ds_build")
    return Index(h.value, x.dtype, x.device)


def view_search(view: View, z: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """ds_view_search: every query through the scalar device API of ds_device.h."""
    _check_device(z, "z")
    if out is None:
        out = torch.empty(z.numel(), dtype=torch.int32, device=z.device)
    st = _lib.ds_view_search(ctypes.byref(view), z.data_ptr(), z.numel(), out.data_ptr(), _stream_handle(stream))
    if st != OK:
        raise DsError(st, "ds_view_search")
    return out


def search(index: Index, z: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """ds_search: int32 i with X_i <= z < X_{i+1} for every z (asynchronous on the stream)."""
    _check_device(z, "z")
    if z.dtype != index.dtype:
        raise TypeError(f"z must be {index.dtype}")
    if out is None:
        out = torch.empty(z.numel(), dtype=torch.int32, device=z.device)
    else:
        _check_device(out, "out")
        if out.dtype != torch.int32 or out.numel() != z.numel():
            raise ValueError("out must be int32 with one entry per query")
    with torch.cuda.device(z.device):
        st = _lib.ds_search(index._h, z.data_ptr(), z.numel(), out.data_ptr(), _stream_handle(stream))
    if st != OK:
        raise DsError(st, "ds_search")
    return out


def info(index: Index) -> dict:
    i = Info()
    st = _lib.ds_info(index._h, ctypes.byref(i))
    if st != OK:
        raise DsError(st, "ds_info")
    d = {name: getattr(i, name) for name, _ in Info._fields_}
    d["method_name"] = METHOD_NAMES.get(d["method"], "?")
    return d


def destroy(index: Index):
    index.destroy()


# ---- learned router kernels ----------------------------------------------------

def learned_grad(params: torch.Tensor, u: torch.Tensor, t: torch.Tensor, stream=None):
    """(loss, gradient) of the router's mean squared error by the GPU training kernels."""
    for x, n in ((params, "params"), (u, "u"), (t, "t")):
        _check_device(x, n)
        if x.dtype != torch.float32:
            raise TypeError(f"{n} must be float32")
    g = torch.empty(N_ROUTER_PARAMS, dtype=torch.float32, device=params.device)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    st = _lib.ds_learned_grad(params.data_ptr(), u.data_ptr(), t.data_ptr(), u.numel(), g.data_ptr(),
                              loss.data_ptr(), _stream_handle(stream))
    if st != OK:
        raise DsError(st, "ds_learned_grad")
    return float(loss.item()), g


def learned_forward(params: torch.Tensor, u: torch.Tensor, fp16_router: bool = False, stream=None) -> torch.Tensor:
    """y(u) by the search-time router kernel (FP32 or FP16-input 32x32 layer)."""
    _check_device(params, "params")
    _check_device(u, "u")
    y = torch.empty(u.numel(), dtype=torch.float32, device=u.device)
    st = _lib.ds_learned_forward(params.data_ptr(), u.data_ptr(), u.numel(), int(bool(fp16_router)), y.data_ptr(),
                                 _stream_handle(stream))
    if st != OK:
        raise DsError(st, "ds_learned_forward")
    return y


# ---- batched ----------------------------------------------------------------

def batch_workspace_bytes(num_arrays: int, total_x: int, table_budget_entries: int = 0,
                          learn_segments: int = 0) -> int:
    return int(_lib.ds_batch_workspace_bytes(int(num_arrays), int(total_x), int(table_budget_entries),
                                             int(learn_segments)))


class Batch:
    """Device-side description of a batched ragged search (wraps ds_batch_desc)."""

    def __init__(self, x_off: torch.Tensor, X: torch.Tensor, q_off: torch.Tensor, z: torch.Tensor,
                 out: torch.Tensor | None = None, *, form: str = "sub", table_budget_entries: int | None = None,
                 tile: int = 0, block: int = 0, lds_bytes: int = 0, qpt: int = 0, total_x: int | None = None,
                 total_q: int | None = None, learn_segments: int = 0, learn_steps: int = 0,
                 direct_cap_bytes: int = 0):
        for t, n in ((x_off, "x_off"), (X, "X"), (q_off, "q_off"), (z, "z")):
            _check_device(t, n)
        if x_off.dtype != torch.int64 or q_off.dtype != torch.int64:
            raise TypeError("offsets must be int64")
        if X.dtype != z.dtype:
            raise TypeError("X and z must share a dtype")
        k = x_off.numel() - 1
        if q_off.numel() != k + 1:
            raise ValueError("x_off and q_off must both have num_arrays + 1 entries")
        self.num_arrays = k
        self.total_x = int(X.numel()) if total_x is None else int(total_x)
        self.total_q = int(z.numel()) if total_q is None else int(total_q)
        if out is None:
            out = torch.empty(self.total_q, dtype=torch.int32, device=z.device)
        if table_budget_entries is None:
            table_budget_entries = 8 * self.total_x + 64 * k
        ws = batch_workspace_bytes(k, self.total_x, table_budget_entries, learn_segments)
        self.workspace = torch.empty(max(ws, 1), dtype=torch.uint8, device=z.device)
        self.keep = (x_off, X, q_off, z, out)
        self.out = out
        self.desc = BatchDesc(_dtype_code(X), k, x_off.data_ptr(), X.data_ptr(), q_off.data_ptr(), z.data_ptr(),
                              out.data_ptr(), self.workspace.data_ptr(), ws, self.total_x, self.total_q,
                              _FORMS[form], int(tile), int(block), int(lds_bytes), int(qpt), int(learn_segments),
                              int(learn_steps), 0, int(direct_cap_bytes))
        self.device = z.device

    def run(self, stream=None) -> torch.Tensor:
        with torch.cuda.device(self.device):
            st = _lib.ds_search_batched(ctypes.byref(self.desc), _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_search_batched")
        return self.out

    def run_noalloc(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """The same build + search through ds_search_batched_noalloc: the library's fixed
        per-GPU scratch array serves as the workspace (this object's is not used).  Results
        go to out (int32, at least total_q entries), or to self.out."""
        d = BatchDesc.from_buffer_copy(self.desc)
        if out is None:
            out = self.out
        else:
            _check_device(out, "out")
            if out.dtype != torch.int32 or out.numel() < self.total_q or not out.is_contiguous():
                raise ValueError("out must be a contiguous int32 tensor of at least total_q entries")
            d.out_dev = out.data_ptr()
        with torch.cuda.device(self.device):
            st = _lib.ds_search_batched_noalloc(ctypes.byref(d), _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_search_batched_noalloc")
        return out

    def autotune(self, stream=None, cache: str | None = None) -> dict:
        """ds_batch_autotune; with cache (a JSON file path) the choice is stored under a key of
        the device and the batch's sizes, and reused instead of re-timed."""
        import json

        key = f"{torch.cuda.get_device_name(self.device)}|{self.desc.dtype}|{self.desc.form}|" \
              f"{self.num_arrays}|{self.total_x}|{self.total_q}"
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.set_shape(**table[key])
                return table[key]
        with torch.cuda.device(self.device):
            st = _lib.ds_batch_autotune(ctypes.byref(self.desc), _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_batch_autotune")
        best = dict(tile=self.desc.tile, block=self.desc.block, lds_bytes=self.desc.lds_bytes, qpt=self.desc.qpt)
        if cache:
            table[key] = best
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return best

    def fallbacks(self, stream=None) -> int:
        c = ctypes.c_uint64()
        st = _lib.ds_batch_fallbacks(ctypes.byref(self.desc), ctypes.byref(c), _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_batch_fallbacks")
        return int(c.value)

    def set_shape(self, tile: int = 0, block: int = 0, lds_bytes: int = 0, qpt: int = 0):
        self.desc.tile, self.desc.block, self.desc.lds_bytes, self.desc.qpt = int(tile), int(block), int(lds_bytes), int(qpt)

    def report(self, stream=None):
        import numpy as np

        meth = np.zeros(self.num_arrays, np.int32)
        R = np.zeros(self.num_arrays, np.int64)
        st = _lib.ds_batch_report(ctypes.byref(self.desc), meth.ctypes.data, R.ctypes.data, _stream_handle(stream))
        if st != OK:
            raise DsError(st, "ds_batch_report")
        return meth, R


def search_batched(x_off, X, q_off, z, out=None, stream=None, **kw) -> torch.Tensor:
    """ds_search_batched in one call (allocates its workspace)."""
    b = Batch(x_off, X, q_off, z, out, **kw)
    return b.run(stream)
