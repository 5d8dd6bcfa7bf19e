"""ctypes front end of the C oracle (``gamma_oracle.c``).  Test infrastructure only.

The shared object is compiled with gcc on first use (or by ``build()``), in place,
next to its source.  No fast-math: the oracle relies on IEEE double arithmetic.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gamma_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Problem(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("local", C.c_int32),
        ("shape", C.c_int64 * 3),
        ("spacing", C.c_double * 3),
        ("dd", C.c_double),
        ("dta", C.c_double),
        ("thr", C.c_double),
    ]


class _Stats(C.Structure):
    _fields_ = [
        ("n_evaluated", C.c_int64),
        ("n_pass", C.c_int64),
        ("n_borderline", C.c_int64),
        ("cells_visited", C.c_int64),
        ("cells_key0", C.c_int64),
        ("table_len", C.c_int64),
        ("n_masked", C.c_int64),
        ("dose_max", C.c_double),
        ("threshold", C.c_double),
        ("radius", C.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def configure(lib):
    """Declare the C signatures of the oracle's entry points on a loaded library (this
    oracle's, or a variant compiled from an edited copy of its source by a test)."""
    lib.oracle_gamma.restype = C.c_int
    lib.oracle_gamma.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(_Stats), C.c_int]
    lib.oracle_gamma_grids.restype = C.c_int
    lib.oracle_gamma_grids.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.POINTER(_Stats), C.c_int]
    lib.oracle_simplex_dist.restype = C.c_double
    lib.oracle_simplex_dist.argtypes = [C.c_int, C.c_int, C.c_void_p]
    lib.oracle_max_threads.restype = C.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = configure(C.CDLL(_LIB))
    return _lib


@dataclass
class OracleResult:
    gamma: np.ndarray          # float64; -1 where not evaluated
    cells: np.ndarray          # int32 visited cells per computed node
    n_evaluated: int
    n_pass: int
    n_borderline: int
    cells_visited: int
    cells_key0: int
    table_len: int
    n_masked: int
    dose_max: float
    threshold: float
    radius: float

    @property
    def pass_rate(self) -> float:
        return self.n_pass / self.n_evaluated if self.n_evaluated else float("nan")


def gamma(ref: np.ndarray, ev: np.ndarray, spacing: Sequence[float], dd: float, dta: float,
          threshold: float = 0.1, local: bool = False, subset: Optional[np.ndarray] = None,
          nthreads: int = 0) -> OracleResult:
    """Gamma index of every masked node of ``ref`` against ``ev`` (same grid).

    ``ref``/``ev`` may be float32 (converted exactly) or float64.  ``subset`` (flat node
    indices) restricts the search to those nodes; the search radius is still the maximum
    gamma0 over the whole grid, as in Algorithm A1 step 1.
    """
    ref64 = np.ascontiguousarray(ref, dtype=np.float64)
    ev64 = np.ascontiguousarray(ev, dtype=np.float64)
    if ref64.shape != ev64.shape or ref64.ndim not in (2, 3):
        raise ValueError("ref and eval must share a 2D or 3D shape")
    nd = ref64.ndim
    pb = _Problem()
    pb.ndim = nd
    pb.local = 1 if local else 0
    for i in range(3):
        pb.shape[i] = ref64.shape[i] if i < nd else 1
        pb.spacing[i] = float(spacing[i]) if i < nd else 1.0
    pb.dd, pb.dta, pb.thr = float(dd), float(dta), float(threshold)
    if subset is not None:
        sub = np.ascontiguousarray(subset, dtype=np.int64).ravel()
        count = sub.size
        sub_ptr = sub.ctypes.data
    else:
        sub = None
        count = ref64.size
        sub_ptr = None
    out = np.empty(count, dtype=np.float64)
    cells = np.zeros(count, dtype=np.int32)
    st = _Stats()
    rc = _load().oracle_gamma(C.byref(pb), ref64.ctypes.data, ev64.ctypes.data, sub_ptr,
                              C.c_int64(count if sub is not None else 0), out.ctypes.data,
                              cells.ctypes.data, C.byref(st), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    if sub is None:
        out = out.reshape(ref64.shape)
        cells = cells.reshape(ref64.shape)
    return OracleResult(out, cells, st.n_evaluated, st.n_pass, st.n_borderline, st.cells_visited,
                        st.cells_key0, st.table_len, st.n_masked, st.dose_max, st.threshold, st.radius)


def gamma_grids(ref: np.ndarray, ev: np.ndarray, ref_spacing: Sequence[float], ev_spacing: Sequence[float],
                ev_origin: Sequence[float], dd: float, dta: float, threshold: float = 0.1, local: bool = False,
                nthreads: int = 0) -> OracleResult:
    """Gamma index with the evaluation dose on a grid of its own: ``ev`` sampled at
    ``ev_origin + j * ev_spacing`` (mm, slowest axis first), the reference node k at
    ``k * ref_spacing``.  Reference nodes outside the evaluation grid's box get -1.  Only
    gamma and the counts are filled (cells, table and radius are 0)."""
    ref64 = np.ascontiguousarray(ref, dtype=np.float64)
    ev64 = np.ascontiguousarray(ev, dtype=np.float64)
    nd = ref64.ndim
    if nd not in (2, 3) or ev64.ndim != nd:
        raise ValueError("ref and eval must both be 2D or both 3D")
    pb = _Problem()
    pb.ndim = nd
    pb.local = 1 if local else 0
    for i in range(3):
        pb.shape[i] = ref64.shape[i] if i < nd else 1
        pb.spacing[i] = float(ref_spacing[i]) if i < nd else 1.0
    pb.dd, pb.dta, pb.thr = float(dd), float(dta), float(threshold)
    es = np.array([ev64.shape[i] if i < nd else 1 for i in range(3)], dtype=np.int64)
    eh = np.array([float(ev_spacing[i]) if i < nd else 1.0 for i in range(3)])
    eo = np.array([float(ev_origin[i]) if i < nd else 0.0 for i in range(3)])
    out = np.empty(ref64.size, dtype=np.float64)
    st = _Stats()
    rc = _load().oracle_gamma_grids(C.byref(pb), es.ctypes.data, eh.ctypes.data, eo.ctypes.data,
                                    ref64.ctypes.data, ev64.ctypes.data, out.ctypes.data, C.byref(st),
                                    int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    return OracleResult(out.reshape(ref64.shape), np.zeros(ref64.shape, dtype=np.int32), st.n_evaluated,
                        st.n_pass, st.n_borderline, 0, 0, 0, st.n_masked, st.dose_max, st.threshold, 0.0)


def simplex_dist(verts: np.ndarray) -> float:
    """Distance from the origin to the simplex with the given vertices (rows)."""
    v = np.ascontiguousarray(verts, dtype=np.float64)
    m = v.shape[0] - 1
    amb = v.shape[1]
    if not (1 <= amb <= 4 and 0 <= m <= 3 and m < amb + 1):
        raise ValueError("unsupported simplex")
    return float(_load().oracle_simplex_dist(amb, m, v.ctypes.data))


def max_threads() -> int:
    return int(_load().oracle_max_threads())
