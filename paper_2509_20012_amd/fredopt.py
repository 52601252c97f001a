"""Thin Python binding of the fredopt C ABI (include/fredopt.h).

Argument marshalling only: every step of the optimizer runs in the HIP kernels of
``libfredopt.so``.  PyTorch provides device memory (the workspace and the
problem arrays) and the current HIP stream.  If the library is missing the import
of a function fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses
import os
from typing import Dict, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfredopt.so")

F32, F16, BF16, F16_IDX16, BF16_IDX16 = 0, 1, 2, 3, 4
STORAGE = {"f32": F32, "fp32": F32, "f16": F16, "fp16": F16, "bf16": BF16,
           "f16i16": F16_IDX16, "bf16i16": BF16_IDX16}
NORM_CONVEX_ALL, NORM_CONVEX_VIOLATED, NORM_RAW = 0, 1, 2
OBJECTIVE_PRINTED, OBJECTIVE_ONE_SIDED = 0, 1
KERNEL_NAMES = ("fwd_obj", "tr_grad", "fwd_dir", "rows", "tr_proj", "fwd_resid", "col",
                "finalize", "active_list", "scatter", "scatter_sum", "line_search")

STATUS = {0: "OK", -1: "E_ARG", -2: "E_SHAPE", -3: "E_INDEX", -4: "E_NONFINITE",
          -5: "E_WORKSPACE", -6: "E_DEVICE", -7: "E_STATE", -8: "E_NOT_IMPLEMENTED"}


class FredoptError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Matrices(ct.Structure):
    _fields_ = [("n_rows", ct.c_int64), ("n_cols", ct.c_int64), ("nnz", ct.c_int64),
                ("row_ptr", ct.c_void_p), ("col_idx", ct.c_void_p),
                ("d_val", ct.c_void_p), ("l_val", ct.c_void_p),
                ("storage", ct.c_int32), ("on_device", ct.c_int32),
                ("lanes_per_row", ct.c_int32), ("gradient_reserve_pct", ct.c_int32)]


class Problem(ct.Structure):
    _fields_ = [("kind", ct.c_void_p), ("dose_lo", ct.c_void_p), ("dose_hi", ct.c_void_p),
                ("cdl_lo", ct.c_void_p), ("cdl_hi", ct.c_void_p), ("letd_max", ct.c_void_p),
                ("w_feas", ct.c_void_p), ("w_obj", ct.c_void_p),
                ("dose_target", ct.c_void_p), ("cdl_target", ct.c_void_p),
                ("c", ct.c_double)]


class Params(ct.Structure):
    _fields_ = [("lambda_", ct.c_double), ("alpha", ct.c_double), ("eta", ct.c_double),
                ("reductions_n", ct.c_int32), ("iter_max", ct.c_int32),
                ("normalization", ct.c_int32), ("objective", ct.c_int32),
                ("unit_direction", ct.c_int32), ("reserved", ct.c_int32)]


class State(ct.Structure):
    _fields_ = [("k", ct.c_int64), ("s", ct.c_int64), ("n_violated", ct.c_int64),
                ("beta", ct.c_double), ("cost", ct.c_double), ("cost_perturbed", ct.c_double),
                ("proximity", ct.c_double), ("grad_sq", ct.c_double), ("q", ct.c_double),
                ("n_active", ct.c_int64), ("projection_path", ct.c_int32),
                ("reserved", ct.c_int32), ("active_entries", ct.c_int64)]

    def as_dict(self) -> Dict[str, float]:
        return {f: getattr(self, f) for f, _ in self._fields_}


class PlanInfo(ct.Structure):
    _fields_ = [("n_rows", ct.c_int64), ("n_cols", ct.c_int64), ("nnz", ct.c_int64),
                ("sell_slots", ct.c_int64), ("csc_slots", ct.c_int64),
                ("bytes_per_sell_slot", ct.c_int64), ("bytes_per_csc_slot", ct.c_int64),
                ("n_slices", ct.c_int64), ("tr_items", ct.c_int64), ("row_items", ct.c_int64),
                ("workspace_bytes", ct.c_int64), ("grad_entries", ct.c_int64),
                ("obj_entries", ct.c_int64),
                ("storage", ct.c_int32), ("lanes_per_row", ct.c_int32),
                ("fwd_grid", ct.c_int32), ("tr_chunk", ct.c_int32), ("lds_x", ct.c_int32),
                ("schedule", ct.c_int32), ("scatter_wgs", ct.c_int32),
                ("scatter_max_rows", ct.c_int64), ("obj_lanes_per_row", ct.c_int32),
                ("fwd_schedule", ct.c_int32), ("scatter_lanes", ct.c_int32),
                ("row_copy_slots", ct.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTED = ("fredopt_workspace_bytes", "fredopt_workspace_bytes_csr",
            "fredopt_load_matrices", "fredopt_load_matrices_noalloc", "fredopt_free_plan",
            "fredopt_dose_let", "fredopt_project_sweep", "fredopt_superiorize_step",
            "fredopt_solve", "fredopt_last_error", "fredopt_get_plan_info",
            "fredopt_profile_kernels", "fredopt_autotune", "fredopt_set_tuning",
            "fredopt_set_scatter", "fredopt_batch_workspace_bytes", "fredopt_batch_create",
            "fredopt_batch_solve", "fredopt_batch_free", "fredopt_scenario_workspace_bytes",
            "fredopt_scenario_dose_let", "fredopt_volume_histogram", "fredopt_roi_quantiles",
            "fredopt_project_sweep_blocks")

_lib = None


def lib():
    """The loaded HIP library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(the optimizer has no CPU fallback)")
        L = ct.CDLL(LIB_PATH)
        P, PP = ct.c_void_p, ct.POINTER(ct.c_void_p)
        L.fredopt_workspace_bytes.argtypes = [ct.c_int64, ct.c_int64, ct.c_int64, ct.c_int32]
        L.fredopt_workspace_bytes.restype = ct.c_size_t
        L.fredopt_workspace_bytes_csr.argtypes = [ct.c_int64, ct.c_int64, P, ct.c_int32,
                                                  ct.c_int32, ct.c_int32]
        L.fredopt_workspace_bytes_csr.restype = ct.c_size_t
        L.fredopt_load_matrices.argtypes = [ct.POINTER(Matrices), P, ct.c_size_t, P, PP]
        L.fredopt_load_matrices_noalloc.argtypes = [ct.POINTER(Matrices), P, ct.c_size_t, P,
                                                    PP]
        L.fredopt_free_plan.argtypes = [P]
        L.fredopt_dose_let.argtypes = [P, P, ct.c_double, P, P, P, P]
        L.fredopt_project_sweep.argtypes = [P, ct.POINTER(Problem), ct.POINTER(Params),
                                            ct.c_double, P, ct.POINTER(ct.c_double), P]
        L.fredopt_superiorize_step.argtypes = [P, ct.POINTER(Problem), ct.POINTER(Params),
                                               ct.POINTER(State), P, P]
        L.fredopt_solve.argtypes = [P, ct.POINTER(Problem), ct.POINTER(Params),
                                    ct.POINTER(State), P, P]
        L.fredopt_last_error.restype = ct.c_char_p
        L.fredopt_get_plan_info.argtypes = [P, ct.POINTER(PlanInfo)]
        L.fredopt_profile_kernels.argtypes = [P, ct.POINTER(Problem), ct.POINTER(Params),
                                              ct.POINTER(State), P, ct.c_int32, P,
                                              ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)]
        L.fredopt_autotune.argtypes = [P, P, P]
        L.fredopt_set_tuning.argtypes = [P, ct.c_int32, ct.c_int32, ct.c_int32]
        L.fredopt_set_scatter.argtypes = [P, ct.c_int32, ct.c_int64]
        L.fredopt_batch_workspace_bytes.argtypes = [ct.POINTER(ct.c_void_p), ct.c_int32]
        L.fredopt_batch_workspace_bytes.restype = ct.c_size_t
        L.fredopt_batch_create.argtypes = [ct.POINTER(ct.c_void_p), ct.c_int32,
                                           ct.POINTER(Problem), P, ct.c_size_t, P, PP]
        L.fredopt_batch_solve.argtypes = [P, ct.POINTER(Params), ct.POINTER(State),
                                          ct.POINTER(ct.c_void_p), ct.c_int32, P]
        L.fredopt_batch_free.argtypes = [P]
        L.fredopt_project_sweep_blocks.argtypes = [P, ct.POINTER(Problem), ct.POINTER(Params),
                                                   ct.c_double, ct.c_int64, P, P]
        L.fredopt_volume_histogram.argtypes = [P, ct.c_int64, P, ct.c_int64, ct.c_double,
                                               ct.c_int32, P, P]
        L.fredopt_roi_quantiles.argtypes = [P, ct.c_int64, P, ct.c_int64,
                                            ct.POINTER(ct.c_double), ct.c_int32, P, P]
        L.fredopt_scenario_workspace_bytes.argtypes = [ct.POINTER(ct.c_void_p), ct.c_int32]
        L.fredopt_scenario_workspace_bytes.restype = ct.c_size_t
        L.fredopt_scenario_dose_let.argtypes = [ct.POINTER(ct.c_void_p), ct.c_int32, P,
                                                ct.c_double, P, P, P, P, P, P, P, P,
                                                ct.c_size_t, P]
        for name in EXPORTED:
            if name not in ("fredopt_workspace_bytes", "fredopt_workspace_bytes_csr",
                            "fredopt_last_error", "fredopt_batch_workspace_bytes"):
                getattr(L, name).restype = ct.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().fredopt_last_error().decode()


def _check(status: int):
    if status != 0:
        raise FredoptError(status, last_error())


def _torch():
    import torch  # noqa: WPS433  (device memory and streams only)
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _dev(t, n: int, name: str, dtype=None) -> int:
    """Device address of tensor t after checking what the C ABI assumes of it: a
    contiguous device tensor of n elements of the given dtype (float32 by default).
    The library cannot check a raw pointer, and a host address or a short buffer
    would make its kernels read out of bounds, so a mismatch raises here."""
    torch = _torch()
    dtype = torch.float32 if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise FredoptError(-1, f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise FredoptError(-1, f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise FredoptError(-1, f"{name} must have dtype {dtype}, not {t.dtype}")
    if not t.is_contiguous():
        raise FredoptError(-1, f"{name} must be contiguous")
    if t.numel() != n:
        raise FredoptError(-2, f"{name} has {t.numel()} elements, expected {n}")
    return int(t.data_ptr())


def workspace_bytes(n_rows: int, n_cols: int, nnz: int, storage: int = F32) -> int:
    """Pattern-free upper bound of the workspace."""
    return int(lib().fredopt_workspace_bytes(n_rows, n_cols, nnz, storage))


def workspace_bytes_csr(row_ptr, n_cols: int, storage: int = F32, lanes_per_row: int = 0,
                        gradient_reserve_pct: int = 0) -> int:
    """Exact workspace for one sparsity pattern (host row pointers)."""
    rp = np.ascontiguousarray(row_ptr, np.int64)
    return int(lib().fredopt_workspace_bytes_csr(rp.size - 1, n_cols, rp.ctypes.data, storage,
                                                 lanes_per_row, gradient_reserve_pct))


@dataclasses.dataclass
class SolverParams:
    """Parameters of Figs. 2-3.  The paper gives no values; these defaults are the
    library's (relaxation 1, alpha 0.99, eta 0.999, one perturbation per iteration,
    convex weights over all constraints)."""
    lam: float = 1.0
    alpha: float = 0.99
    eta: float = 0.999
    reductions_n: int = 1
    iter_max: int = 100
    normalization: int = NORM_CONVEX_ALL
    objective: int = OBJECTIVE_PRINTED
    unit_direction: int = 0

    def struct(self) -> Params:
        return Params(lambda_=self.lam, alpha=self.alpha, eta=self.eta,
                      reductions_n=self.reductions_n, iter_max=self.iter_max,
                      normalization=self.normalization, objective=self.objective,
                      unit_direction=self.unit_direction, reserved=0)


class DeviceProblem:
    """Per-row problem arrays resident on the device."""

    def __init__(self, arrays: Dict[str, np.ndarray], c: float, device="cuda"):
        torch = _torch()
        self.c = float(c)
        self.t = {}
        for k in ("dose_lo", "dose_hi", "cdl_lo", "cdl_hi", "letd_max", "w_feas", "w_obj",
                  "dose_target", "cdl_target"):
            self.t[k] = torch.from_numpy(np.ascontiguousarray(arrays[k], np.float32)).to(device)
        kind = np.ascontiguousarray(arrays["kind"], np.uint16).view(np.int16)
        self.t["kind"] = torch.from_numpy(kind).to(device)

    def struct(self, n_rows: Optional[int] = None) -> Problem:
        """The C struct; with n_rows, every array is first checked to be a contiguous
        device array of n_rows elements (kind int16/uint16 bits, the rest float32)."""
        if n_rows is not None:
            torch = _torch()
            for k, v in self.t.items():
                _dev(v, n_rows, f"problem.{k}", torch.int16 if k == "kind" else None)
        return Problem(**{k: _ptr(v) for k, v in self.t.items()}, c=self.c)


class Plan:
    """A loaded pair of influence matrices (owns its device workspace)."""

    def __init__(self, handle: ct.c_void_p, ws, n_rows: int, n_cols: int, nnz: int,
                 storage: int, keep=()):
        self._h = handle
        self.ws = ws
        self.n_rows, self.n_cols, self.nnz, self.storage = n_rows, n_cols, nnz, storage
        self._keep = keep

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h:
            _check(lib().fredopt_free_plan(self._h))
            self._h = None

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.fredopt_free_plan(self._h)
                self._h = None
        except Exception:
            pass

    def info(self) -> Dict[str, int]:
        inf = PlanInfo()
        _check(lib().fredopt_get_plan_info(self._h, ct.byref(inf)))
        return inf.as_dict()


def load_matrices(row_ptr, col_idx, d_val, l_val, n_cols: int, storage: int = F32,
                  device="cuda", stream=None, on_device: bool = True,
                  lanes_per_row: int = 0, gradient_reserve_pct: int = 0,
                  noalloc: bool = False) -> Plan:
    """Loads CSR influence matrices.  With on_device=True the arrays are copied to
    the device with torch first (the library then reads device pointers); with
    on_device=False host arrays are handed to the library, which stages them.
    noalloc: the library's load that allocates no device memory (host matrices are
    staged in its fixed per-device area; the workspace is still allocated here)."""
    torch = _torch()
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col_idx = np.ascontiguousarray(col_idx, np.int32)
    d_val = np.ascontiguousarray(d_val, np.float32)
    l_val = np.ascontiguousarray(l_val, np.float32)
    R = row_ptr.size - 1
    nnz = int(row_ptr[-1]) if row_ptr.size else 0
    nbytes = workspace_bytes_csr(row_ptr, n_cols, storage, lanes_per_row, gradient_reserve_pct)
    if nbytes == 0:
        nbytes = 256  # invalid sizes: let the library report the error
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    keep = ()
    if on_device:
        tens = [torch.from_numpy(a).to(device) for a in (row_ptr, col_idx, d_val, l_val)]
        m = Matrices(R, n_cols, nnz, *[_ptr(t) for t in tens], storage, 1, lanes_per_row,
                     gradient_reserve_pct)
        keep = tens
    else:
        m = Matrices(R, n_cols, nnz, row_ptr.ctypes.data, col_idx.ctypes.data,
                     d_val.ctypes.data, l_val.ctypes.data, storage, 0, lanes_per_row,
                     gradient_reserve_pct)
    h = ct.c_void_p()
    load = lib().fredopt_load_matrices_noalloc if noalloc else lib().fredopt_load_matrices
    _check(load(ct.byref(m), _ptr(ws), nbytes, _stream(stream), ct.byref(h)))
    del keep  # input arrays are no longer referenced after the load
    return Plan(h, ws, R, n_cols, nnz, storage)


def free_plan(plan: Plan):
    plan.free()


def dose_let(plan: Plan, x, c: float = 0.04, stream=None, want=("dose", "letd", "cdl")):
    """(dose, LETd, cDL) device tensors for the device fluence x."""
    torch = _torch()
    outs = {k: (torch.empty(plan.n_rows, dtype=torch.float32, device=x.device)
                if k in want else None) for k in ("dose", "letd", "cdl")}
    _check(lib().fredopt_dose_let(plan.handle, _dev(x, plan.n_cols, "x"), float(c),
                                  _ptr(outs["dose"]),
                                  _ptr(outs["letd"]), _ptr(outs["cdl"]), _stream(stream)))
    return outs["dose"], outs["letd"], outs["cdl"]


def scenario_dose_let(plans, x, c: float = 0.04, stream=None,
                      want=("dose", "letd", "cdl"), bands: bool = True):
    """Robustness evaluation of one fluence x under n scenario plans (same voxels and
    beamlets): a dict with the per-scenario "dose", "letd", "cdl" device tensors of
    shape (n, n_rows) named in want, and, with bands, the per-voxel "dose_min",
    "dose_max", "letd_min", "letd_max" over the scenarios."""
    torch = _torch()
    n = len(plans)
    if n < 1:
        raise FredoptError(-1, "at least one scenario plan")
    R, C = plans[0].n_rows, plans[0].n_cols
    hp = (ct.c_void_p * n)(*[p.handle for p in plans])
    nbytes = int(lib().fredopt_scenario_workspace_bytes(hp, n))
    if nbytes == 0:
        raise FredoptError(-1, "scenario workspace size: a plan is invalid")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    out = {k: torch.empty((n, R), dtype=torch.float32, device=x.device)
           for k in ("dose", "letd", "cdl") if k in want}
    if bands:
        for k in ("dose_min", "dose_max", "letd_min", "letd_max"):
            out[k] = torch.empty(R, dtype=torch.float32, device=x.device)
    _check(lib().fredopt_scenario_dose_let(
        hp, n, _dev(x, C, "x"), float(c), _ptr(out.get("dose")), _ptr(out.get("letd")),
        _ptr(out.get("cdl")), _ptr(out.get("dose_min")), _ptr(out.get("dose_max")),
        _ptr(out.get("letd_min")), _ptr(out.get("letd_max")), _ptr(ws), nbytes,
        _stream(stream)))
    return out


def _roi_rows(rows, n_rows: int, device):
    """A region's row indices as a device int32 tensor, checked against n_rows."""
    torch = _torch()
    if isinstance(rows, torch.Tensor):
        rows = rows.detach().cpu().numpy()
    r = np.ascontiguousarray(rows, np.int64)
    if r.size and (r.min() < 0 or r.max() >= n_rows):
        raise FredoptError(-3, f"region rows must lie in [0, {n_rows})")
    return torch.from_numpy(r.astype(np.int32)).to(device)


def volume_histogram(values, rows, vmax: float, n_bins: int, stream=None):
    """Cumulative volume histogram of a region (DVH / LVH / cDLVH): a device uint32
    tensor cum[0..n_bins], cum[b] = rows with value >= b vmax / n_bins."""
    torch = _torch()
    n_rows = int(values.numel())
    rt = _roi_rows(rows, n_rows, values.device)
    cum = torch.empty(n_bins + 1, dtype=torch.int32, device=values.device)
    _check(lib().fredopt_volume_histogram(_dev(values, n_rows, "values"), n_rows, _ptr(rt),
                                          int(rt.numel()), float(vmax), int(n_bins), _ptr(cum),
                                          _stream(stream)))
    return cum


def roi_quantiles(values, rows, qs, stream=None):
    """Nearest-rank quantiles (value at rank ceil(q n)) of a region's values: a device
    float tensor, one entry per q (D95: q = 0.05 of dose, cDL30: q = 0.70 of cDL)."""
    torch = _torch()
    n_rows = int(values.numel())
    rt = _roi_rows(rows, n_rows, values.device)
    qa = (ct.c_double * len(qs))(*[float(q) for q in qs])
    out = torch.empty(len(qs), dtype=torch.float32, device=values.device)
    _check(lib().fredopt_roi_quantiles(_dev(values, n_rows, "values"), n_rows, _ptr(rt),
                                       int(rt.numel()), qa, len(qs), _ptr(out),
                                       _stream(stream)))
    return out


def percentile_target(plan: Plan, x, rows, c: float = 0.04, q: float = 0.70) -> float:
    """A percentile constraint from a forward calculation (Section 2.4.1): the cDL of
    fluence x over a region, and its nearest-rank q quantile (cDL30 for q = 0.70)."""
    _, _, cdl = dose_let(plan, x, c, want=("cdl",))
    return float(roi_quantiles(cdl, rows, [q])[0].item())


def project_sweep_blocks(plan: Plan, problem: DeviceProblem, params: SolverParams, x,
                         block_rows: int, weight_scale: float = 1.0, stream=None):
    """One block-sequential sweep in place on x (blocks of block_rows rows, a multiple
    of 8192, or every row)."""
    pr, q = problem.struct(plan.n_rows), params.struct()
    _check(lib().fredopt_project_sweep_blocks(plan.handle, ct.byref(pr), ct.byref(q),
                                              float(weight_scale), int(block_rows),
                                              _dev(x, plan.n_cols, "x"), _stream(stream)))


def project_sweep(plan: Plan, problem: DeviceProblem, params: SolverParams, x,
                  weight_scale: float = 1.0, stream=None) -> float:
    """One simultaneous AMS sweep in place on x; returns the input proximity."""
    prox = ct.c_double(0.0)
    pr, q = problem.struct(plan.n_rows), params.struct()
    _check(lib().fredopt_project_sweep(plan.handle, ct.byref(pr), ct.byref(q),
                                       float(weight_scale), _dev(x, plan.n_cols, "x"),
                                       ct.byref(prox),
                                       _stream(stream)))
    return float(prox.value)


def superiorize_step(plan: Plan, problem: DeviceProblem, params: SolverParams, state: State,
                     x, stream=None) -> State:
    pr, q = problem.struct(plan.n_rows), params.struct()
    _check(lib().fredopt_superiorize_step(plan.handle, ct.byref(pr), ct.byref(q),
                                          ct.byref(state), _dev(x, plan.n_cols, "x"),
                                          _stream(stream)))
    return state


def solve(plan: Plan, problem: DeviceProblem, params: SolverParams, state: State, x,
          stream=None) -> State:
    pr, q = problem.struct(plan.n_rows), params.struct()
    _check(lib().fredopt_solve(plan.handle, ct.byref(pr), ct.byref(q), ct.byref(state),
                               _dev(x, plan.n_cols, "x"), _stream(stream)))
    return state


class Batch:
    """Several plans iterated by the same kernel launches (fredopt_batch_*)."""

    def __init__(self, plans, problems, stream=None):
        torch = _torch()
        n = len(plans)
        assert n == len(problems) and n > 0
        hp = (ct.c_void_p * n)(*[p.handle for p in plans])
        nbytes = int(lib().fredopt_batch_workspace_bytes(hp, n))
        if nbytes == 0:
            raise FredoptError(-1, "batch workspace size: a plan is invalid")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        prs = (Problem * n)(*[pr.struct(pl.n_rows) for pr, pl in zip(problems, plans)])
        h = ct.c_void_p()
        _check(lib().fredopt_batch_create(hp, n, prs, _ptr(self.ws), nbytes, _stream(stream),
                                          ct.byref(h)))
        self._h = h
        self.plans, self.problems, self.n = list(plans), list(problems), n

    def solve(self, params: "SolverParams", states, xs, n_iters: int, stream=None):
        assert len(states) == self.n and len(xs) == self.n
        sts = (State * self.n)(*states)
        xp = (ct.c_void_p * self.n)(*[_dev(x, pl.n_cols, f"x[{i}]")
                                      for i, (x, pl) in enumerate(zip(xs, self.plans))])
        q = params.struct()
        _check(lib().fredopt_batch_solve(self._h, ct.byref(q), sts, xp, int(n_iters),
                                         _stream(stream)))
        for i in range(self.n):
            ct.memmove(ct.byref(states[i]), ct.byref(sts[i]), ct.sizeof(State))
        return states

    def free(self):
        if self._h:
            _check(lib().fredopt_batch_free(self._h))
            self._h = None

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.fredopt_batch_free(self._h)
                self._h = None
        except Exception:
            pass


def new_state(k: int = 0, s: int = -1) -> State:
    st = State()
    st.k, st.s = k, s
    return st


def profile_kernels(plan: Plan, problem: DeviceProblem, params: SolverParams, state: State,
                    x, n_iters: int, stream=None):
    nk = len(KERNEL_NAMES)
    ms = (ct.c_double * nk)()
    cnt = (ct.c_int64 * nk)()
    pr, q = problem.struct(plan.n_rows), params.struct()
    _check(lib().fredopt_profile_kernels(plan.handle, ct.byref(pr), ct.byref(q),
                                         ct.byref(state), _dev(x, plan.n_cols, "x"),
                                         int(n_iters),
                                         _stream(stream), ms, cnt))
    return {KERNEL_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(nk)}


def autotune(plan: Plan, x, stream=None):
    _check(lib().fredopt_autotune(plan.handle, _dev(x, plan.n_cols, "x"), _stream(stream)))
    return plan.info()


def set_tuning(plan: Plan, fwd_wgs_per_cu: int = 0, tr_chunk: int = 0, fwd_schedule: int = 0):
    """0 keeps a value; fwd_schedule 1 = groups from a counter, 2 = round robin."""
    _check(lib().fredopt_set_tuning(plan.handle, int(fwd_wgs_per_cu), int(tr_chunk),
                                    int(fwd_schedule)))


def set_scatter(plan: Plan, n_workgroups: int = 0, max_active_rows: int = -1):
    """Active-row projection path: ``n_workgroups`` 0 default, -1 off;
    ``max_active_rows`` -1 default (a quarter of the rows)."""
    _check(lib().fredopt_set_scatter(plan.handle, int(n_workgroups), int(max_active_rows)))


# ----------------------------------------------------------------------- phantoms

def load_phantom(ph, storage: int = F32, device="cuda", on_device: bool = True,
                 lanes_per_row: int = 0, gradient_reserve_pct: int = 0):
    """(Plan, DeviceProblem, x0 device tensor) for a ``phantom.Phantom``."""
    torch = _torch()
    plan = load_matrices(ph.row_ptr, ph.col_idx, ph.d_val, ph.l_val, ph.n_cols, storage,
                         device=device, on_device=on_device, lanes_per_row=lanes_per_row,
                         gradient_reserve_pct=gradient_reserve_pct)
    prob = DeviceProblem(ph.problem_arrays(), ph.c, device=device)
    x0 = torch.from_numpy(np.ascontiguousarray(ph.x0, np.float32)).to(device)
    return plan, prob, x0
