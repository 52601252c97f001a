"""ctypes wrapper of the FP64 C oracle in ``fredopt_oracle.c``.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU-baseline
leg of the benchmark.  It promotes the FP32 input arrays to FP64 and forwards them
to the C functions, each of which cites the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses
import os
import subprocess
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fredopt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KIND_BITS = {"DOSE_LO": 1, "DOSE_HI": 2, "CDL_LO": 4, "CDL_HI": 8, "LETD_HI": 16,
             "OBJ_DOSE": 32, "OBJ_CDL": 64}


def lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Mat(ct.Structure):
    _fields_ = [("R", ct.c_int64), ("C", ct.c_int64),
                ("row_ptr", ct.c_void_p), ("col", ct.c_void_p),
                ("dv", ct.c_void_p), ("lv", ct.c_void_p),
                ("col_ptr", ct.c_void_p), ("row", ct.c_void_p),
                ("cdv", ct.c_void_p), ("clv", ct.c_void_p)]


class _Problem(ct.Structure):
    _fields_ = [("kind", ct.c_void_p), ("dose_lo", ct.c_void_p), ("dose_hi", ct.c_void_p),
                ("cdl_lo", ct.c_void_p), ("cdl_hi", ct.c_void_p), ("letd_max", ct.c_void_p),
                ("w_feas", ct.c_void_p), ("w_obj", ct.c_void_p),
                ("dose_target", ct.c_void_p), ("cdl_target", ct.c_void_p),
                ("c", ct.c_double), ("objective", ct.c_int32)]


class _Params(ct.Structure):
    _fields_ = [("lambda_", ct.c_double), ("alpha", ct.c_double), ("eta", ct.c_double),
                ("reductions_n", ct.c_int32), ("normalization", ct.c_int32),
                ("line_search", ct.c_int32), ("unit_direction", ct.c_int32)]


class _Info(ct.Structure):
    _fields_ = [("n_accepted", ct.c_int64), ("n_trials", ct.c_int64),
                ("n_violated", ct.c_int64), ("beta_last", ct.c_double),
                ("cost_before", ct.c_double), ("cost_after_perturb", ct.c_double),
                ("proximity", ct.c_double), ("grad_sq", ct.c_double),
                ("q_last", ct.c_double), ("capped", ct.c_int32)]


@dataclasses.dataclass
class OracleParams:
    lam: float = 1.0
    alpha: float = 0.99
    eta: float = 0.999
    reductions_n: int = 1
    normalization: int = 0     # 0 convex over all, 1 convex over violated, 2 raw
    line_search: int = 1       # 0 literal (Fig. 3), 1 exact quadratic identity
    unit_direction: int = 0    # 0 perturb along the gradient, 1 along gradient / norm


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle(force=False)
        lib = ct.CDLL(_LIB)
        P = ct.c_void_p
        lib.orc_mat_init.argtypes = [ct.POINTER(_Mat), ct.c_int64, ct.c_int64, P, P, P, P]
        lib.orc_mat_init.restype = ct.c_int
        lib.orc_mat_free.argtypes = [ct.POINTER(_Mat)]
        lib.orc_forward.argtypes = [ct.POINTER(_Mat), P, P, P]
        lib.orc_forward_rows.argtypes = [ct.POINTER(_Mat), P, P, ct.c_int64, P, P]
        lib.orc_transposed.argtypes = [ct.POINTER(_Mat), P, P, P]
        lib.orc_dose_let.argtypes = [ct.POINTER(_Mat), P, ct.c_double, P, P, P, P]
        lib.orc_cost.argtypes = [ct.POINTER(_Mat), ct.POINTER(_Problem), P]
        lib.orc_cost.restype = ct.c_double
        lib.orc_gradient.argtypes = [ct.POINTER(_Mat), ct.POINTER(_Problem), P, P]
        lib.orc_proximity.argtypes = [ct.POINTER(_Mat), ct.POINTER(_Problem), P,
                                      ct.POINTER(ct.c_int64)]
        lib.orc_proximity.restype = ct.c_double
        lib.orc_ams_simultaneous.argtypes = [ct.POINTER(_Mat), ct.POINTER(_Problem),
                                             ct.c_double, ct.c_double, ct.c_int, P, P,
                                             ct.POINTER(ct.c_int64)]
        lib.orc_ams_simultaneous.restype = ct.c_double
        lib.orc_ams_blocks.argtypes = [ct.POINTER(_Mat), ct.POINTER(_Problem), ct.c_double,
                                       ct.c_double, ct.c_int, ct.c_int64, P, P]
        lib.orc_ams_sequential.argtypes = [ct.POINTER(_Mat), ct.POINTER(_Problem),
                                           ct.c_double, ct.c_double, P, ct.c_int64, P,
                                           ct.c_int64, P]
        lib.orc_sa_iteration.argtypes = [ct.POINTER(_Mat), ct.POINTER(_Problem),
                                         ct.POINTER(_Params), ct.POINTER(ct.c_int64),
                                         ct.POINTER(ct.c_int64), P, ct.POINTER(_Info)]
        lib.orc_solve.argtypes = [ct.POINTER(_Mat), ct.POINTER(_Problem), ct.POINTER(_Params),
                                  ct.c_int64, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64),
                                  P, ct.POINTER(_Info)]
        lib.orc_num_threads.restype = ct.c_int
        lib.orc_set_threads.argtypes = [ct.c_int]
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (n >= 1)."""
    _load().orc_set_threads(int(n))


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """FP64 oracle bound to one pair of influence matrices and one problem.

    ``values`` may override D and L (e.g. dequantised reduced-precision values).
    ``objective``: 0 Eq. (2) as printed, 1 the OAR term one-sided (counted only where
    cDL exceeds its target)."""

    def __init__(self, ph, d_val: Optional[np.ndarray] = None,
                 l_val: Optional[np.ndarray] = None, problem: Optional[Dict] = None,
                 objective: int = 0):
        lib = _load()
        self.R, self.C = int(ph.n_rows), int(ph.n_cols)
        self._row_ptr = np.ascontiguousarray(ph.row_ptr, dtype=np.int64)
        self._col = np.ascontiguousarray(ph.col_idx, dtype=np.int32)
        self._dv = _f64(ph.d_val if d_val is None else d_val)
        self._lv = _f64(ph.l_val if l_val is None else l_val)
        self._mat = _Mat()
        rc = lib.orc_mat_init(ct.byref(self._mat), self.R, self.C, _p(self._row_ptr),
                              _p(self._col), _p(self._dv), _p(self._lv))
        if rc != 0:
            raise MemoryError("oracle matrix allocation failed")
        pa = problem if problem is not None else ph.problem_arrays()
        self.c = float(ph.c)
        self._prob_arrays = {"kind": np.ascontiguousarray(pa["kind"], dtype=np.uint16)}
        for k in ("dose_lo", "dose_hi", "cdl_lo", "cdl_hi", "letd_max", "w_feas", "w_obj",
                  "dose_target", "cdl_target"):
            self._prob_arrays[k] = _f64(pa[k])
        self._prob = _Problem(**{k: _p(v) for k, v in self._prob_arrays.items()}, c=self.c,
                              objective=int(objective))

    def __del__(self):
        try:
            if _lib is not None and getattr(self, "_mat", None) is not None:
                _lib.orc_mat_free(ct.byref(self._mat))
        except Exception:
            pass

    # --- products -----------------------------------------------------------------
    def forward(self, x) -> Tuple[np.ndarray, np.ndarray]:
        x = _f64(x)
        d = np.empty(self.R)
        l = np.empty(self.R)
        _load().orc_forward(ct.byref(self._mat), _p(x), _p(d), _p(l))
        return d, l

    def forward_rows(self, x, rows) -> Tuple[np.ndarray, np.ndarray]:
        x = _f64(x)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        d = np.empty(rows.size)
        l = np.empty(rows.size)
        _load().orc_forward_rows(ct.byref(self._mat), _p(x), _p(rows), rows.size, _p(d), _p(l))
        return d, l

    def transposed(self, ud, ul) -> np.ndarray:
        ud, ul = _f64(ud), _f64(ul)
        out = np.empty(self.C)
        _load().orc_transposed(ct.byref(self._mat), _p(ud), _p(ul), _p(out))
        return out

    def dose_let(self, x):
        x = _f64(x)
        d, l, letd, cdl = (np.empty(self.R) for _ in range(4))
        _load().orc_dose_let(ct.byref(self._mat), _p(x), self.c, _p(d), _p(l), _p(letd), _p(cdl))
        return d, l, letd, cdl

    # --- objective ----------------------------------------------------------------
    def cost(self, x) -> float:
        x = _f64(x)
        return float(_load().orc_cost(ct.byref(self._mat), ct.byref(self._prob), _p(x)))

    def gradient(self, x) -> np.ndarray:
        x = _f64(x)
        g = np.empty(self.C)
        _load().orc_gradient(ct.byref(self._mat), ct.byref(self._prob), _p(x), _p(g))
        return g

    def proximity(self, x) -> Tuple[float, int]:
        x = _f64(x)
        nv = ct.c_int64(0)
        p = _load().orc_proximity(ct.byref(self._mat), ct.byref(self._prob), _p(x), ct.byref(nv))
        return float(p), int(nv.value)

    # --- feasibility seeking ------------------------------------------------------
    def ams_simultaneous(self, y, lam: float = 1.0, weight_scale: float = 1.0,
                         normalization: int = 0):
        y = _f64(y)
        out = np.empty(self.C)
        nv = ct.c_int64(0)
        prox = _load().orc_ams_simultaneous(ct.byref(self._mat), ct.byref(self._prob),
                                            lam, weight_scale, normalization, _p(y), _p(out),
                                            ct.byref(nv))
        return out, float(prox), int(nv.value)

    def ams_blocks(self, y, block_rows: int, lam: float = 1.0, weight_scale: float = 1.0,
                   normalization: int = 0) -> np.ndarray:
        """Block-sequential sweep: consecutive blocks of block_rows rows in ascending
        order, each a simultaneous projection at the current point; clamp at the end."""
        y = _f64(y)
        out = np.empty(self.C)
        _load().orc_ams_blocks(ct.byref(self._mat), ct.byref(self._prob), lam, weight_scale,
                               normalization, int(block_rows), _p(y), _p(out))
        return out

    def ams_sequential(self, x, dose_order: Sequence[int], cdl_order: Sequence[int],
                       lam: float = 1.0, weight_scale: float = 1.0) -> np.ndarray:
        x = _f64(x).copy()
        do = np.ascontiguousarray(dose_order, dtype=np.int64)
        co = np.ascontiguousarray(cdl_order, dtype=np.int64)
        _load().orc_ams_sequential(ct.byref(self._mat), ct.byref(self._prob), lam,
                                   weight_scale, _p(do), do.size, _p(co), co.size, _p(x))
        return x

    # --- superiorization ----------------------------------------------------------
    @staticmethod
    def _params(q: OracleParams) -> _Params:
        return _Params(lambda_=q.lam, alpha=q.alpha, eta=q.eta, reductions_n=q.reductions_n,
                       normalization=q.normalization, line_search=q.line_search,
                       unit_direction=q.unit_direction)

    def sa_iteration(self, x, k: int, s: int, q: OracleParams):
        x = _f64(x).copy()
        kk, ss = ct.c_int64(k), ct.c_int64(s)
        info = _Info()
        prm = self._params(q)
        _load().orc_sa_iteration(ct.byref(self._mat), ct.byref(self._prob), ct.byref(prm),
                                 ct.byref(kk), ct.byref(ss), _p(x), ct.byref(info))
        return x, int(kk.value), int(ss.value), _info_dict(info)

    def solve(self, x, iter_max: int, q: OracleParams, k: int = 0, s: int = -1):
        x = _f64(x).copy()
        kk, ss = ct.c_int64(k), ct.c_int64(s)
        info = _Info()
        prm = self._params(q)
        _load().orc_solve(ct.byref(self._mat), ct.byref(self._prob), ct.byref(prm), iter_max,
                          ct.byref(kk), ct.byref(ss), _p(x), ct.byref(info))
        return x, int(kk.value), int(ss.value), _info_dict(info)


def _info_dict(info: _Info) -> Dict[str, float]:
    return {f: getattr(info, f) for f, _ in _Info._fields_}
