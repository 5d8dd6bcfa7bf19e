"""ctypes binding of libgammax (declared in include/gammax.h).

Argument marshalling only: every step of the gamma computation runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors' data pointers) and the current
HIP stream.  Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import threading
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libgammax.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libgammax.so is not built ({LIB_PATH}); run `python -m paper_1012_1900_amd._build` "
        "or __graft_entry__.build() first")

# PyTorch ships its own HIP runtime.  Loading torch first makes the library bind to that
# same runtime, so device pointers and streams from torch are valid in our calls (two
# runtimes in one process would not share streams or contexts).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

# ---- status codes (gammax_status_t) ------------------------------------------------------
OK = 0
E_NULL = -1
E_SHAPE = -2
E_PARAM = -3
E_NONFINITE = -4
E_NOMEM = -5
E_DEVICE = -6
E_RADIUS = -7
E_DOSE = -8
E_MODEL = -9

GLOBAL, LOCAL = 0, 1
SORT_NONE, SORT_DD, SORT_BOUND, SORT_PREDICTED, SORT_GIVEN = 0, 1, 2, 3, 4
PREC_FP32, PREC_GUARDED, PREC_FP64 = 0, 1, 2
RADIUS_PLAIN, RADIUS_LEARNED = 0, 1

_SORT = {"none": SORT_NONE, "dd": SORT_DD, "bound": SORT_BOUND, "predicted": SORT_PREDICTED, "given": SORT_GIVEN}
_RADIUS = {"plain": RADIUS_PLAIN, "learned": RADIUS_LEARNED}
_PREC = {"fp32": PREC_FP32, "guarded": PREC_GUARDED, "fp64": PREC_FP64}
_PROJ = {"faces": 0, "ju": 1}


class GammaxError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        msg = _lib.gammax_status_string(status).decode()
        super().__init__(f"gammax status {status}: {msg}" + (f" ({detail})" if detail else ""))


class Problem(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("norm", C.c_int32),
        ("shape", C.c_int64 * 3),
        ("spacing_mm", C.c_double * 3),
        ("dd", C.c_double),
        ("dta_mm", C.c_double),
        ("dose_threshold", C.c_double),
    ]


class Options(C.Structure):
    _fields_ = [
        ("sort_mode", C.c_int32),
        ("precision", C.c_int32),
        ("cond_threshold", C.c_double),
        ("timing", C.c_int32),
        ("tail_lanes", C.c_int32),
        ("cell_lanes", C.c_int32),
        ("radius_mode", C.c_int32),
        ("model", C.c_void_p),
        ("radius_factor", C.c_double),
        ("autotune", C.c_int32),
        ("cnn_pool", C.c_int32),
        ("projection", C.c_int32),
        ("reserved", C.c_int32 * 1),
        ("order_key", C.c_void_p),
    ]


class Result(C.Structure):
    _fields_ = [
        ("n_evaluated", C.c_uint64),
        ("n_pass", C.c_uint64),
        ("n_borderline", C.c_uint64),
        ("n_fp64_tets", C.c_uint64),
        ("n_cells", C.c_uint64),
        ("n_tail", C.c_uint64),
        ("n_guarded", C.c_uint64),
        ("pass_rate", C.c_double),
        ("max_gamma", C.c_float),
        ("dose_max", C.c_float),
        ("search_radius", C.c_float),
        ("table_len", C.c_int32),
        ("ms_prep", C.c_float),
        ("ms_table", C.c_float),
        ("ms_search", C.c_float),
        ("ms_sort", C.c_float),
        ("ms_tail", C.c_float),
        ("ms_guard", C.c_float),
        ("n_fallback", C.c_uint64),
        ("ms_cnn", C.c_float),
        ("ms_done", C.c_float),
        ("long_walk_rows", C.c_uint32),
    ]


_vp = C.c_void_p
_lib.gammax_options_default.restype = None
_lib.gammax_options_default.argtypes = [C.POINTER(Options)]
_lib.gammax_ctx_create.restype = C.c_int
_lib.gammax_ctx_create.argtypes = [C.c_int, C.POINTER(_vp)]
_lib.gammax_ctx_destroy.restype = C.c_int
_lib.gammax_ctx_destroy.argtypes = [_vp]
_lib.gammax_map.restype = C.c_int
_lib.gammax_map.argtypes = [_vp, C.POINTER(Problem), C.POINTER(Options), _vp, _vp, _vp,
                            C.POINTER(Result), _vp]
_lib.gammax_map_async.restype = C.c_int
_lib.gammax_map_async.argtypes = [_vp, C.POINTER(Problem), C.POINTER(Options), _vp, _vp, _vp,
                                  C.POINTER(C.c_uint64), _vp]
_lib.gammax_map_wait.restype = C.c_int
_lib.gammax_map_wait.argtypes = [_vp, C.c_uint64, C.POINTER(Result)]
ASYNC_SLOTS = 64
_lib.gamma_map.restype = C.c_int
_lib.gamma_map.argtypes = [_vp, _vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                           C.c_double, C.c_double, C.c_double, C.c_int32, _vp,
                           C.POINTER(C.c_double), _vp]
_lib.gammax_map_noalloc.restype = C.c_int
_lib.gammax_map_noalloc.argtypes = [C.POINTER(Problem), C.POINTER(Options), _vp, _vp, _vp, C.POINTER(Result), _vp]
_lib.gammax_sort_pairs.restype = C.c_int
_lib.gammax_sort_pairs.argtypes = [_vp, _vp, _vp, C.c_int64, _vp]
_lib.gammax_build_table.restype = C.c_int
_lib.gammax_build_table.argtypes = [_vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                    C.c_double, _vp, _vp, C.c_int64, C.POINTER(C.c_int64), _vp]
_lib.gammax_pass_count.restype = C.c_int
_lib.gammax_pass_count.argtypes = [_vp, _vp, C.c_int64, C.POINTER(C.c_uint64), _vp]
_lib.gammax_status_string.restype = C.c_char_p
_lib.gammax_status_string.argtypes = [C.c_int]
_lib.gammax_last_error.restype = C.c_char_p
_lib.gammax_last_error.argtypes = [_vp]


def status_string(status: int) -> str:
    return _lib.gammax_status_string(status).decode()


def default_options() -> Options:
    o = Options()
    _lib.gammax_options_default(C.byref(o))
    return o


class Context:
    """A library context on one HIP device (owns scratch memory and the table cache)."""

    def __init__(self, device: int = 0):
        h = _vp()
        st = _lib.gammax_ctx_create(int(device), C.byref(h))
        if st != OK:
            raise GammaxError(st, f"device {device}")
        self.handle = h
        self.device = int(device)

    def close(self):
        if self.handle:
            _lib.gammax_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int):
        if st != OK:
            raise GammaxError(st, _lib.gammax_last_error(self.handle).decode())


_ctx_lock = threading.Lock()
_contexts = {}


def context(device: int) -> Context:
    with _ctx_lock:
        c = _contexts.get(device)
        if c is None:
            c = _contexts[device] = Context(device)
        return c


@dataclass
class GammaResult:
    n_evaluated: int
    n_pass: int
    n_borderline: int
    n_fp64_tets: int
    n_cells: int
    n_tail: int
    n_guarded: int
    pass_rate: float
    max_gamma: float
    dose_max: float
    search_radius: float
    table_len: int
    ms_prep: float
    ms_table: float
    ms_search: float
    ms_sort: float
    ms_tail: float
    ms_guard: float
    n_fallback: int
    ms_cnn: float
    ms_done: float = 0.0
    long_walk_rows: int = 0


def _torch():
    import torch
    return torch


def _dev_tensor(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device (cuda/hip) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def make_problem(shape: Sequence[int], spacing: Sequence[float], dd: float, dta: float,
                 dose_threshold: float, local: bool) -> Problem:
    p = Problem()
    nd = len(shape)
    p.ndim = nd
    p.norm = LOCAL if local else GLOBAL
    for i in range(3):
        p.shape[i] = int(shape[i]) if i < nd else 0
        p.spacing_mm[i] = float(spacing[i]) if i < nd else 0.0
    p.dd, p.dta_mm, p.dose_threshold = float(dd), float(dta), float(dose_threshold)
    return p


def make_options(sort: str = "none", precision: str = "guarded", cond_threshold: float = 1e6,
                 timing: bool = False, tail_lanes: int = 0, cell_lanes: int = 0, radius: str = "plain",
                 model=None, radius_factor: float = 1.1, cnn_pool: int = 0, projection: str = "faces",
                 order_key: Optional[int] = None) -> Options:
    """Options of a map; ``order_key`` is the device address of the per-node key of
    ``sort="given"``."""
    o = default_options()
    o.order_key = order_key
    o.cnn_pool = int(cnn_pool)
    o.projection = _PROJ[projection]
    o.radius_mode = _RADIUS[radius]
    o.model = model.handle if model is not None else None
    o.radius_factor = float(radius_factor)
    o.sort_mode = _SORT[sort]
    o.precision = _PREC[precision]
    o.cond_threshold = float(cond_threshold)
    o.timing = 1 if timing else 0
    o.tail_lanes = int(tail_lanes)
    o.cell_lanes = int(cell_lanes)
    return o


def _order_key_ptr(order_key, ref):
    """Device address of the per-node key of the given order (checked against ``ref``)."""
    if order_key is None:
        return None
    _dev_tensor(order_key, "order_key")
    if order_key.shape != ref.shape or order_key.device != ref.device:
        raise ValueError("order_key must match ref in shape and device")
    return order_key.data_ptr()


def gammax_map(ref, ev, spacing: Sequence[float], dd: float, dta: float,
               dose_threshold: float = 0.1, local: bool = False, *, sort: str = "none",
               precision: str = "guarded", cond_threshold: float = 1e6, timing: bool = False,
               tail_lanes: int = 0, cell_lanes: int = 0, radius: str = "plain", model=None,
               radius_factor: float = 1.1, cnn_pool: int = 0, projection: str = "faces", order_key=None,
               out=None, ctx: Optional[Context] = None, stream=None):
    """Gamma map of a dose pair on the GPU.  Returns (gamma tensor, GammaResult).

    ``ref``/``ev``: float32 device tensors of shape (ny, nx) or (nz, ny, nx); ``spacing``
    in mm in the same axis order.  gamma is -1 where a node is not evaluated.
    ``order_key``: with ``sort="given"``, a float32 device tensor shaped like ``ref``.
    """
    torch = _torch()
    _dev_tensor(ref, "ref")
    _dev_tensor(ev, "ev")
    if ref.shape != ev.shape or ref.device != ev.device:
        raise ValueError("ref and ev must share shape and device")
    if len(spacing) != ref.dim():
        raise ValueError("spacing needs one entry per axis")
    if out is None:
        out = torch.empty_like(ref)
    else:
        _dev_tensor(out, "out")
        if out.shape != ref.shape or out.device != ref.device:
            raise ValueError("out must match ref")
    dev = ref.device.index if ref.device.index is not None else torch.cuda.current_device()
    ctx = ctx or context(dev)
    p = make_problem(tuple(ref.shape), spacing, dd, dta, dose_threshold, local)
    o = make_options(sort, precision, cond_threshold, timing, tail_lanes, cell_lanes, radius, model,
                     radius_factor, cnn_pool, projection, _order_key_ptr(order_key, ref))
    r = Result()
    s = stream if stream is not None else torch.cuda.current_stream(ref.device)
    with torch.cuda.device(ref.device):
        st = _lib.gammax_map(ctx.handle, C.byref(p), C.byref(o), ref.data_ptr(), ev.data_ptr(),
                             out.data_ptr(), C.byref(r), _vp(s.cuda_stream))
    ctx.check(st)
    res = GammaResult(**{f[0]: getattr(r, f[0]) for f in Result._fields_})
    return out, res


class MapTicket:
    """A map queued by :func:`gammax_map_async`.  ``wait()`` returns its GammaResult (once);
    ``gamma`` is the output tensor, complete after the wait."""

    def __init__(self, ctx, ticket: int, gamma, keep):
        self.ctx, self.ticket, self.gamma, self._keep = ctx, ticket, gamma, keep
        self._res = None

    def wait(self) -> "GammaResult":
        if self._res is None:
            r = Result()
            self.ctx.check(_lib.gammax_map_wait(self.ctx.handle, self.ticket, C.byref(r)))
            self._res = GammaResult(**{f[0]: getattr(r, f[0]) for f in Result._fields_})
            self._keep = None
        return self._res


def gammax_map_async(ref, ev, spacing: Sequence[float], dd: float, dta: float,
                     dose_threshold: float = 0.1, local: bool = False, *, sort: str = "none",
                     precision: str = "guarded", cond_threshold: float = 1e6, tail_lanes: int = 0,
                     cell_lanes: int = 0, radius: str = "plain", model=None, radius_factor: float = 1.1,
                     cnn_pool: int = 0, projection: str = "faces", order_key=None, out=None,
                     ctx: Optional[Context] = None, stream=None) -> MapTicket:
    """Queue a gamma map without waiting (``gammax_map_async``); the returned ticket's
    ``wait()`` gives the GammaResult.  The tensors are kept alive until then and must not
    be modified before it."""
    torch = _torch()
    _dev_tensor(ref, "ref")
    _dev_tensor(ev, "ev")
    if ref.shape != ev.shape or ref.device != ev.device:
        raise ValueError("ref and ev must share shape and device")
    if len(spacing) != ref.dim():
        raise ValueError("spacing needs one entry per axis")
    if out is None:
        out = torch.empty_like(ref)
    else:
        _dev_tensor(out, "out")
        if out.shape != ref.shape or out.device != ref.device:
            raise ValueError("out must match ref")
    dev = ref.device.index if ref.device.index is not None else torch.cuda.current_device()
    ctx = ctx or context(dev)
    p = make_problem(tuple(ref.shape), spacing, dd, dta, dose_threshold, local)
    o = make_options(sort, precision, cond_threshold, False, tail_lanes, cell_lanes, radius, model,
                     radius_factor, cnn_pool, projection, _order_key_ptr(order_key, ref))
    t = C.c_uint64(0)
    s = stream if stream is not None else torch.cuda.current_stream(ref.device)
    with torch.cuda.device(ref.device):
        st = _lib.gammax_map_async(ctx.handle, C.byref(p), C.byref(o), ref.data_ptr(), ev.data_ptr(),
                                   out.data_ptr(), C.byref(t), _vp(s.cuda_stream))
    ctx.check(st)
    return MapTicket(ctx, t.value, out, (ref, ev, model, order_key))


def gamma_map(ref_dose, eval_dose, spacing: Sequence[float], dd: float, dta: float,
              dose_threshold: float = 0.1, local: bool = False) -> Tuple[object, float]:
    """The paper's problem statement: (gamma tensor, pass rate) with default options,
    through the flat C entry point ``gamma_map``."""
    torch = _torch()
    _dev_tensor(ref_dose, "ref_dose")
    _dev_tensor(eval_dose, "eval_dose")
    if ref_dose.shape != eval_dose.shape:
        raise ValueError("ref_dose and eval_dose must share a shape")
    nd = ref_dose.dim()
    shape = (C.c_int64 * 3)(*(list(ref_dose.shape) + [0] * (3 - nd)))
    sp = (C.c_double * 3)(*(list(map(float, spacing)) + [0.0] * (3 - nd)))
    out = torch.empty_like(ref_dose)
    pr = C.c_double(float("nan"))
    s = torch.cuda.current_stream(ref_dose.device)
    with torch.cuda.device(ref_dose.device):
        st = _lib.gamma_map(ref_dose.data_ptr(), eval_dose.data_ptr(), nd, shape, sp, float(dd),
                            float(dta), float(dose_threshold), LOCAL if local else GLOBAL,
                            out.data_ptr(), C.byref(pr), _vp(s.cuda_stream))
    if st != OK:
        raise GammaxError(st)
    return out, pr.value


NOALLOC_MAX_NODES = 2097152   # GAMMAX_NOALLOC_MAX_NODES
NOALLOC_MAX_TABLE = 262144    # GAMMAX_NOALLOC_MAX_TABLE


def gammax_map_noalloc(ref, ev, spacing: Sequence[float], dd: float, dta: float,
                       dose_threshold: float = 0.1, local: bool = False, *, out, sort: str = "none",
                       precision: str = "guarded", cond_threshold: float = 1e6, tail_lanes: int = 0,
                       cell_lanes: int = 0, projection: str = "faces", stream=None) -> "GammaResult":
    """The map through ``gammax_map_noalloc``: no device allocation inside the call (its
    workspace is the library's fixed device array).  ``out`` (float32, shaped like ``ref``)
    receives gamma and must be given: the binding allocates nothing either.  Returns the
    GammaResult.  Calls that overlap on one GPU race."""
    torch = _torch()
    _dev_tensor(ref, "ref")
    _dev_tensor(ev, "ev")
    _dev_tensor(out, "out")
    if ref.shape != ev.shape or ref.device != ev.device or out.shape != ref.shape or out.device != ref.device:
        raise ValueError("ref, ev and out must share shape and device")
    if len(spacing) != ref.dim():
        raise ValueError("spacing needs one entry per axis")
    p = make_problem(tuple(ref.shape), spacing, dd, dta, dose_threshold, local)
    o = make_options(sort, precision, cond_threshold, False, tail_lanes, cell_lanes, "plain", None, 1.1, 0,
                     projection, None)
    r = Result()
    s = stream if stream is not None else torch.cuda.current_stream(ref.device)
    with torch.cuda.device(ref.device):
        st = _lib.gammax_map_noalloc(C.byref(p), C.byref(o), ref.data_ptr(), ev.data_ptr(), out.data_ptr(),
                                     C.byref(r), _vp(s.cuda_stream))
    if st != OK:
        raise GammaxError(st)
    return GammaResult(**{f[0]: getattr(r, f[0]) for f in Result._fields_})


def sort_pairs(keys, vals, ctx: Optional[Context] = None):
    """Stable ascending sort of uint32 (key, value) pairs in place (int32 tensors holding
    the uint32 bit patterns)."""
    torch = _torch()
    for t, nm in ((keys, "keys"), (vals, "vals")):
        if t.device.type != "cuda" or t.dtype != torch.int32 or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous int32 device tensor")
    if keys.numel() != vals.numel():
        raise ValueError("keys and vals differ in length")
    ctx = ctx or context(keys.device.index or 0)
    s = torch.cuda.current_stream(keys.device)
    with torch.cuda.device(keys.device):
        st = _lib.gammax_sort_pairs(ctx.handle, keys.data_ptr(), vals.data_ptr(), keys.numel(),
                                    _vp(s.cuda_stream))
    ctx.check(st)
    return keys, vals


def build_table(shape: Sequence[int], spacing_over_dta: Sequence[float], radius: float,
                cap: Optional[int] = None, device: int = 0, ctx: Optional[Context] = None):
    """Sorted cell table: (key2 float32 tensor [T], offsets int32 tensor [T, 3])."""
    torch = _torch()
    nd = len(shape)
    if cap is None:
        cap = 1
        for i in range(nd):
            r = int(math.ceil(radius / spacing_over_dta[i])) + 1
            cap *= min(2 * r + 2, 2 * int(shape[i]) - 1)
    dev = torch.device("cuda", device)
    key2 = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    offs = torch.empty((max(cap, 1), 3), dtype=torch.int32, device=dev)
    n = C.c_int64(0)
    shp = (C.c_int64 * 3)(*(list(shape) + [0] * (3 - nd)))
    sp = (C.c_double * 3)(*(list(map(float, spacing_over_dta)) + [0.0] * (3 - nd)))
    ctx = ctx or context(device)
    s = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        st = _lib.gammax_build_table(ctx.handle, nd, shp, sp, float(radius), key2.data_ptr(),
                                     offs.data_ptr(), int(cap), C.byref(n), _vp(s.cuda_stream))
    ctx.check(st)
    return key2[: n.value], offs[: n.value]


def pass_count(gamma, ctx: Optional[Context] = None) -> Tuple[int, int, int]:
    """(evaluated, pass, borderline) counts of a gamma map on the device."""
    torch = _torch()
    _dev_tensor(gamma, "gamma")
    ctx = ctx or context(gamma.device.index or 0)
    counts = (C.c_uint64 * 3)()
    s = torch.cuda.current_stream(gamma.device)
    with torch.cuda.device(gamma.device):
        st = _lib.gammax_pass_count(ctx.handle, gamma.data_ptr(), gamma.numel(), counts,
                                    _vp(s.cuda_stream))
    ctx.check(st)
    return int(counts[0]), int(counts[1]), int(counts[2])


# ---- learned search radius ---------------------------------------------------------------

MODEL_NPARAM = 15169


class Adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


_lib.gammax_model_create.restype = C.c_int
_lib.gammax_model_create.argtypes = [C.c_int, C.POINTER(C.c_float), C.POINTER(_vp)]
_lib.gammax_model_destroy.restype = C.c_int
_lib.gammax_model_destroy.argtypes = [_vp]
_lib.gammax_model_get_params.restype = C.c_int
_lib.gammax_model_get_params.argtypes = [_vp, _vp, _vp]
_lib.gammax_model_last_error.restype = C.c_char_p
_lib.gammax_model_last_error.argtypes = [_vp]
_lib.gammax_model_save.restype = C.c_int
_lib.gammax_model_save.argtypes = [_vp, C.c_char_p]
_lib.gammax_model_load.restype = C.c_int
_lib.gammax_model_load.argtypes = [C.c_int, C.c_char_p, C.POINTER(_vp)]
_lib.gammax_model_features.restype = C.c_int
_lib.gammax_model_features.argtypes = [_vp, C.POINTER(Problem), _vp, _vp, _vp, _vp]
_lib.gammax_model_predict.restype = C.c_int
_lib.gammax_model_predict.argtypes = [_vp, _vp, C.POINTER(Problem), _vp, _vp, _vp, _vp]
_lib.gammax_model_predict_nodes.restype = C.c_int
_lib.gammax_model_predict_nodes.argtypes = [_vp, _vp, C.POINTER(Problem), _vp, _vp, _vp, C.c_int64, _vp, _vp]
_lib.gammax_model_predict_nodes_pooled.restype = C.c_int
_lib.gammax_model_predict_nodes_pooled.argtypes = [_vp, _vp, C.POINTER(Problem), _vp, _vp, _vp, C.c_int64, _vp, _vp]
_lib.gammax_model_forward.restype = C.c_int
_lib.gammax_model_forward.argtypes = [_vp, C.c_int32, C.POINTER(C.c_int64), _vp, _vp, _vp]
_lib.gammax_model_train_step.restype = C.c_int
_lib.gammax_model_train_step.argtypes = [_vp, C.c_int32, C.POINTER(C.c_int64), _vp, _vp,
                                         C.POINTER(Adam), C.POINTER(C.c_double), _vp]


class Model:
    """The learned-radius CNN on one device (``gammax_model_*``)."""

    def __init__(self, params, device: int = 0):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        if p.size != MODEL_NPARAM:
            raise ValueError(f"expected {MODEL_NPARAM} parameters, got {p.size}")
        h = _vp()
        st = _lib.gammax_model_create(int(device), p.ctypes.data_as(C.POINTER(C.c_float)), C.byref(h))
        if st != 0:
            raise GammaxError(st)
        self.handle = h
        self.device = int(device)

    def close(self):
        if getattr(self, "handle", None):
            _lib.gammax_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int):
        if st != 0:
            raise GammaxError(st, _lib.gammax_model_last_error(self.handle).decode(errors="replace"))

    def params(self):
        import numpy as np
        out = np.empty(MODEL_NPARAM, dtype=np.float32)
        self.check(_lib.gammax_model_get_params(self.handle, out.ctypes.data, None))
        return out

    def grad(self):
        import numpy as np
        out = np.empty(MODEL_NPARAM, dtype=np.float32)
        self.check(_lib.gammax_model_get_params(self.handle, None, out.ctypes.data))
        return out

    def save(self, path: str):
        """Checkpoint: the parameters and the Adam state (``gammax_model_save``), so that
        training resumes where it stopped."""
        self.check(_lib.gammax_model_save(self.handle, os.fsencode(path)))

    def save_params(self, path: str):
        """Only the parameters, as one flat float32 ``.npy`` array (the shipped weights)."""
        import numpy as np
        np.save(path, self.params(), allow_pickle=False)

    @classmethod
    def load(cls, path: str, device: int = 0) -> "Model":
        """A model from a checkpoint written by :meth:`save` (``gammax_model_load``: parameters
        and Adam state), or from a ``.npy`` parameter file (parameters only, fresh Adam state)."""
        import numpy as np
        if str(path).endswith(".npy"):
            return cls(np.load(path, allow_pickle=False), device)
        h = _vp()
        st = _lib.gammax_model_load(int(device), os.fsencode(path), C.byref(h))
        if st != 0:
            raise GammaxError(st, f"cannot load a model from {path}")
        m = cls.__new__(cls)
        m.handle = h
        m.device = int(device)
        return m

    def forward(self, feats):
        """y for a batch of feature crops: int16/uint16 tensor (B, c0+8, c1+8, c2+8, 2)."""
        torch = _torch()
        if feats.dim() != 5 or feats.shape[-1] != 2 or feats.dtype not in (torch.int16, torch.uint16):
            raise ValueError("features must be a (B, z, y, x, 2) 16-bit tensor")
        if not feats.is_contiguous() or feats.device.type != "cuda":
            raise ValueError("features must be a contiguous device tensor")
        b = feats.shape[0]
        crop = (C.c_int64 * 3)(*[int(n) - 8 for n in feats.shape[1:4]])
        y = torch.empty((b, crop[0], crop[1], crop[2]), dtype=torch.float32, device=feats.device)
        s = torch.cuda.current_stream(feats.device)
        with torch.cuda.device(feats.device):
            st = _lib.gammax_model_forward(self.handle, b, crop, feats.data_ptr(), y.data_ptr(), _vp(s.cuda_stream))
        self.check(st)
        return y

    def train_step(self, feats, gamma, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                   eps: float = 1e-8) -> float:
        """One Adam step on a batch of crops; returns the loss before the step."""
        torch = _torch()
        if feats.dim() != 5 or feats.shape[-1] != 2 or feats.dtype not in (torch.int16, torch.uint16):
            raise ValueError("features must be a (B, z, y, x, 2) 16-bit tensor")
        _dev_tensor(gamma, "gamma")
        b = feats.shape[0]
        crop = (C.c_int64 * 3)(*[int(n) - 8 for n in feats.shape[1:4]])
        if tuple(gamma.shape) != (b, crop[0], crop[1], crop[2]):
            raise ValueError("gamma must have shape (B, c0, c1, c2)")
        hp = Adam(lr, beta1, beta2, eps)
        loss = C.c_double()
        s = torch.cuda.current_stream(feats.device)
        with torch.cuda.device(feats.device):
            st = _lib.gammax_model_train_step(self.handle, b, crop, feats.data_ptr(), gamma.data_ptr(),
                                              C.byref(hp), C.byref(loss), _vp(s.cuda_stream))
        self.check(st)
        return loss.value

    def predict(self, ref, ev, spacing: Sequence[float], dd: float, dta: float = 3.0,
                ctx: Optional[Context] = None):
        """y = log(gamma_hat + 0.01) on the grid of a 3D dose pair (float32 tensor)."""
        torch = _torch()
        _dev_tensor(ref, "ref")
        _dev_tensor(ev, "ev")
        ctx = ctx or context(ref.device.index or 0)
        prob = make_problem(ref.shape, spacing, dd, dta, 0.1, False)
        y = torch.empty_like(ref)
        s = torch.cuda.current_stream(ref.device)
        with torch.cuda.device(ref.device):
            st = _lib.gammax_model_predict(ctx.handle, self.handle, C.byref(prob), ref.data_ptr(),
                                           ev.data_ptr(), y.data_ptr(), _vp(s.cuda_stream))
        ctx.check(st)
        return y


def predict_nodes(model, ref, ev, spacing: Sequence[float], dd: float, nodes, dta: float = 3.0,
                  ctx: Optional[Context] = None, pool: int = 0):
    """y = log(gamma_hat + 0.01) at flat node indices ``nodes`` (int32 device tensor).
    ``pool=2``: from the pair average-pooled 2x2x2 (``gammax_model_predict_nodes_pooled``)."""
    if pool not in (0, 2):
        raise ValueError("pool must be 0 or 2")
    torch = _torch()
    _dev_tensor(ref, "ref")
    _dev_tensor(ev, "ev")
    if nodes.dtype != torch.int32 or nodes.device != ref.device or not nodes.is_contiguous():
        raise ValueError("nodes must be a contiguous int32 tensor on the doses' device")
    ctx = ctx or context(ref.device.index or 0)
    prob = make_problem(ref.shape, spacing, dd, dta, 0.1, False)
    y = torch.empty(nodes.numel(), dtype=torch.float32, device=ref.device)
    s = torch.cuda.current_stream(ref.device)
    with torch.cuda.device(ref.device):
        fn = _lib.gammax_model_predict_nodes_pooled if pool == 2 else _lib.gammax_model_predict_nodes
        st = fn(ctx.handle, model.handle, C.byref(prob), ref.data_ptr(), ev.data_ptr(), nodes.data_ptr(),
                nodes.numel(), y.data_ptr(), _vp(s.cuda_stream))
    ctx.check(st)
    return y


def model_features(ref, ev, spacing: Sequence[float], dd: float, dta: float = 3.0,
                   ctx: Optional[Context] = None):
    """Input features of a 3D pair on the grid padded by 4: int16 tensor (z+8, y+8, x+8, 2)
    holding bf16 bit patterns."""
    torch = _torch()
    _dev_tensor(ref, "ref")
    _dev_tensor(ev, "ev")
    if ref.dim() != 3:
        raise ValueError("the learned radius is 3D only")
    ctx = ctx or context(ref.device.index or 0)
    prob = make_problem(ref.shape, spacing, dd, dta, 0.1, False)
    feat = torch.empty((ref.shape[0] + 8, ref.shape[1] + 8, ref.shape[2] + 8, 2), dtype=torch.int16,
                       device=ref.device)
    s = torch.cuda.current_stream(ref.device)
    with torch.cuda.device(ref.device):
        st = _lib.gammax_model_features(ctx.handle, C.byref(prob), ref.data_ptr(), ev.data_ptr(),
                                        feat.data_ptr(), _vp(s.cuda_stream))
    ctx.check(st)
    return feat


# ---- batches -----------------------------------------------------------------------------

_lib.gammax_batch.restype = C.c_int
_lib.gammax_batch.argtypes = [_vp, C.c_int32, C.POINTER(Problem), C.POINTER(_vp), C.POINTER(_vp),
                              C.POINTER(_vp), C.POINTER(Options), C.POINTER(Result), _vp]
_lib.gammax_tune_save.restype = C.c_int
_lib.gammax_tune_save.argtypes = [_vp, C.c_char_p]
_lib.gammax_tune_load.restype = C.c_int
_lib.gammax_tune_load.argtypes = [_vp, C.c_char_p]


def gammax_batch(pairs, *, precision: str = "guarded", cond_threshold: float = 1e6, tail_lanes: int = 0,
                 radius: str = "plain", model=None, radius_factor: float = 1.1, autotune: bool = False,
                 cnn_pool: int = 0, sort: str = "none", projection: str = "faces", outs=None,
                 ctx: Optional[Context] = None, stream=None):
    """Gamma maps of a batch of pairs (``gammax_batch``): one captured HIP graph per batch
    (every pair's compaction, one key-0 launch over all pairs' nodes in cost order, every
    pair's tail, guard and counts), replayed when the batch comes again; each pair's
    completion time in ``ms_done``.

    ``pairs``: sequence of dicts with ``ref``, ``ev`` (float32 device tensors), ``spacing``,
    ``dd``, ``dta`` and optionally ``threshold`` (default 0.1) and ``local`` (default False).
    Returns (list of gamma tensors, list of GammaResult).
    """
    torch = _torch()
    n = len(pairs)
    if n == 0:
        return [], []
    dev = pairs[0]["ref"].device
    probs = (Problem * n)()
    refs, evs, gams = (_vp * n)(), (_vp * n)(), (_vp * n)()
    out_list = []
    for i, q in enumerate(pairs):
        _dev_tensor(q["ref"], "ref")
        _dev_tensor(q["ev"], "ev")
        if q["ref"].shape != q["ev"].shape or q["ref"].device != dev or q["ev"].device != dev:
            raise ValueError(f"pair {i}: ref and ev must share shape and device")
        if len(q["spacing"]) != q["ref"].dim():
            raise ValueError(f"pair {i}: spacing needs one entry per axis")
        probs[i] = make_problem(tuple(q["ref"].shape), q["spacing"], q["dd"], q["dta"],
                                q.get("threshold", 0.1), q.get("local", False))
        g = outs[i] if outs is not None else torch.empty_like(q["ref"])
        out_list.append(g)
        refs[i], evs[i], gams[i] = q["ref"].data_ptr(), q["ev"].data_ptr(), g.data_ptr()
    ctx = ctx or context(dev.index or 0)
    o = make_options(sort, precision, cond_threshold, False, tail_lanes, 0, radius, model, radius_factor,
                     cnn_pool, projection)
    o.autotune = 1 if autotune else 0
    res = (Result * n)()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        st = _lib.gammax_batch(ctx.handle, n, probs, refs, evs, gams, C.byref(o), res, _vp(s.cuda_stream))
    ctx.check(st)
    results = [GammaResult(**{f[0]: getattr(r, f[0]) for f in Result._fields_}) for r in res]
    return out_list, results


class Grid(C.Structure):
    _fields_ = [("shape", C.c_int64 * 3), ("spacing_mm", C.c_double * 3), ("origin_mm", C.c_double * 3)]


_lib.gammax_map_grids.restype = C.c_int
_lib.gammax_map_grids.argtypes = [_vp, C.POINTER(Problem), C.POINTER(Grid), _vp, _vp, _vp, C.POINTER(Options),
                                  C.POINTER(Result), _vp]


def gammax_map_grids(ref, ev, ref_spacing: Sequence[float], ev_spacing: Sequence[float],
                     ev_origin: Sequence[float], dd: float, dta: float, dose_threshold: float = 0.1,
                     local: bool = False, *, precision: str = "guarded", cond_threshold: float = 1e6,
                     tail_lanes: int = 0, out=None, ctx: Optional[Context] = None, stream=None):
    """Gamma map with the evaluation dose on a grid of its own (``gammax_map_grids``, 2D or
    3D): ``ev`` (float32 device tensor) sampled at ``ev_origin + j * ev_spacing`` mm in the
    frame where reference node k sits at ``k * ref_spacing``.  Returns (gamma on the
    reference grid, GammaResult); gamma is -1 where a node is not evaluated."""
    torch = _torch()
    _dev_tensor(ref, "ref")
    _dev_tensor(ev, "ev")
    if ref.dim() not in (2, 3) or ev.dim() != ref.dim() or ref.device != ev.device:
        raise ValueError("ref and ev must both be 2D or both 3D tensors on one device")
    nd = ref.dim()
    if len(ref_spacing) != nd or len(ev_spacing) != nd or len(ev_origin) != nd:
        raise ValueError("spacings and origin need one entry per axis")
    if out is None:
        out = torch.empty_like(ref)
    dev = ref.device.index if ref.device.index is not None else torch.cuda.current_device()
    ctx = ctx or context(dev)
    p = make_problem(tuple(ref.shape), ref_spacing, dd, dta, dose_threshold, local)
    g = Grid()
    for i in range(nd):
        g.shape[i] = int(ev.shape[i])
        g.spacing_mm[i] = float(ev_spacing[i])
        g.origin_mm[i] = float(ev_origin[i])
    o = make_options("none", precision, cond_threshold, False, tail_lanes, 0)
    r = Result()
    s = stream if stream is not None else torch.cuda.current_stream(ref.device)
    with torch.cuda.device(ref.device):
        st = _lib.gammax_map_grids(ctx.handle, C.byref(p), C.byref(g), ref.data_ptr(), ev.data_ptr(), out.data_ptr(),
                                   C.byref(o), C.byref(r), _vp(s.cuda_stream))
    ctx.check(st)
    return out, GammaResult(**{f[0]: getattr(r, f[0]) for f in Result._fields_})


_lib.gammax_map_many.restype = C.c_int
_lib.gammax_map_many.argtypes = [_vp, C.c_int32, C.POINTER(Problem), C.POINTER(_vp), C.POINTER(_vp),
                                 C.POINTER(_vp), C.POINTER(Options), C.POINTER(Result), _vp]


def gammax_map_many(pairs, *, sort: str = "none", precision: str = "guarded", cond_threshold: float = 1e6,
                    tail_lanes: int = 0, radius: str = "plain", model=None, radius_factor: float = 1.1,
                    cnn_pool: int = 0, outs=None, ctx: Optional[Context] = None, stream=None):
    """Gamma maps of several pairs in one call (``gammax_map_many``): each pair index keeps
    a context of its own inside ``ctx``, the pairs run on the stream and three internal ones.

    ``pairs``: sequence of dicts with ``ref``, ``ev`` (float32 device tensors), ``spacing``,
    ``dd``, ``dta`` and optionally ``threshold`` (default 0.1) and ``local`` (default False).
    Returns (list of gamma tensors, list of GammaResult).
    """
    torch = _torch()
    n = len(pairs)
    if n == 0:
        return [], []
    dev = pairs[0]["ref"].device
    probs = (Problem * n)()
    refs, evs, gams = (_vp * n)(), (_vp * n)(), (_vp * n)()
    out_list = []
    for i, q in enumerate(pairs):
        _dev_tensor(q["ref"], "ref")
        _dev_tensor(q["ev"], "ev")
        if q["ref"].shape != q["ev"].shape or q["ref"].device != dev or q["ev"].device != dev:
            raise ValueError(f"pair {i}: ref and ev must share shape and device")
        if len(q["spacing"]) != q["ref"].dim():
            raise ValueError(f"pair {i}: spacing needs one entry per axis")
        probs[i] = make_problem(tuple(q["ref"].shape), q["spacing"], q["dd"], q["dta"],
                                q.get("threshold", 0.1), q.get("local", False))
        g = outs[i] if outs is not None else torch.empty_like(q["ref"])
        out_list.append(g)
        refs[i], evs[i], gams[i] = q["ref"].data_ptr(), q["ev"].data_ptr(), g.data_ptr()
    ctx = ctx or context(dev.index or 0)
    o = make_options(sort, precision, cond_threshold, False, tail_lanes, 0, radius, model, radius_factor, cnn_pool)
    res = (Result * n)()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        st = _lib.gammax_map_many(ctx.handle, n, probs, refs, evs, gams, C.byref(o), res, _vp(s.cuda_stream))
    ctx.check(st)
    return out_list, [GammaResult(**{f[0]: getattr(r, f[0]) for f in Result._fields_}) for r in res]


def tune_save(path: str, ctx: Context):
    ctx.check(_lib.gammax_tune_save(ctx.handle, path.encode()))


def tune_load(path: str, ctx: Context):
    ctx.check(_lib.gammax_tune_load(ctx.handle, path.encode()))


def raw_library() -> C.CDLL:
    """The loaded shared library (for symbol checks)."""
    return _lib
