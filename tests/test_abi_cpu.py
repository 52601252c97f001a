"""C ABI checks that need no GPU: the library loads, exports every function that
include/fredopt.h declares, sizes its workspace, and rejects bad arguments before
touching the device."""
import ctypes as ct
import os
import re

import pytest

from paper_2509_20012_amd import fredopt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fredopt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fredopt_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = fredopt.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(fredopt.EXPORTED)


def test_workspace_bytes_exact_within_bound():
    import numpy as np
    from paper_2509_20012_amd import phantom as ph
    for args in ((48, 12, 0.3, 1), (300, 37, 0.2, 2), (1000, 130, 0.05, 3)):
        p = ph.tiny_problem(*args[:3], seed=args[3])
        exact = fredopt.workspace_bytes_csr(p.row_ptr, p.n_cols)
        bound = fredopt.workspace_bytes(p.n_rows, p.n_cols, p.nnz)
        assert 0 < exact <= bound
        for lpr in (1, 2, 4, 8, 16):
            assert fredopt.workspace_bytes_csr(p.row_ptr, p.n_cols, lanes_per_row=lpr) > 0
        assert fredopt.workspace_bytes_csr(p.row_ptr, p.n_cols, lanes_per_row=3) == 0
    bad = np.array([0, 3, 2], np.int64)
    assert fredopt.workspace_bytes_csr(bad, 4) == 0


def test_workspace_bytes():
    assert fredopt.workspace_bytes(0, 0, 0) == 0          # no columns
    assert fredopt.workspace_bytes(-1, 4, 0) == 0
    assert fredopt.workspace_bytes(10, 4, 5, storage=7) == 0
    a = fredopt.workspace_bytes(1000, 100, 10_000)
    b = fredopt.workspace_bytes(1000, 100, 20_000)
    h = fredopt.workspace_bytes(1000, 100, 20_000, fredopt.F16)
    assert 0 < a < b and h < b
    # the matrices alone: two copies of 4-byte indices + two FP32 values per slot
    assert b >= 2 * 12 * 20_000
    assert b % 256 == 0
    # 16-bit column indices: smaller than 16-bit values alone; only up to 65,536 columns
    h16 = fredopt.workspace_bytes(1000, 100, 20_000, fredopt.F16_IDX16)
    assert 0 < h16 < h
    assert fredopt.workspace_bytes(1000, 65_536, 20_000, fredopt.BF16_IDX16) > 0
    assert fredopt.workspace_bytes(1000, 65_537, 20_000, fredopt.BF16_IDX16) == 0


def test_null_arguments_rejected_without_device():
    L = fredopt.lib()
    assert L.fredopt_load_matrices(None, None, 0, None, None) == -1
    assert L.fredopt_load_matrices_noalloc(None, None, 0, None, None) == -1
    assert L.fredopt_free_plan(None) == -1
    assert L.fredopt_dose_let(None, None, 0.04, None, None, None, None) == -1
    q = fredopt.SolverParams().struct()
    pr = fredopt.Problem()
    st = fredopt.State()
    assert L.fredopt_project_sweep(None, ct.byref(pr), ct.byref(q), 1.0, None, None, None) == -1
    assert L.fredopt_superiorize_step(None, ct.byref(pr), ct.byref(q), ct.byref(st), None,
                                      None) == -1
    assert L.fredopt_solve(None, ct.byref(pr), ct.byref(q), ct.byref(st), None, None) == -1
    assert L.fredopt_set_tuning(None, 0, 0, 0) == -1
    assert L.fredopt_profile_kernels(None, None, None, None, None, 1, None, None, None) == -1
    assert L.fredopt_autotune(None, None, None) == -1
    assert L.fredopt_get_plan_info(None, None) == -1
    assert "NULL" in fredopt.last_error() or "non-NULL" in fredopt.last_error()


def test_load_rejects_bad_workspace_before_device_work():
    import numpy as np
    L = fredopt.lib()
    rp = np.array([0, 1], np.int64)
    ci = np.array([0], np.int32)
    v = np.array([1.0], np.float32)
    m = fredopt.Matrices(1, 1, 1, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                         v.ctypes.data, 0, 0, 0, 0)
    h = ct.c_void_p()
    assert L.fredopt_load_matrices(ct.byref(m), None, 1 << 20, None, ct.byref(h)) == -5
    assert L.fredopt_load_matrices(ct.byref(m), ct.c_void_p(256), 16, None, ct.byref(h)) == -5
    assert L.fredopt_load_matrices_noalloc(ct.byref(m), None, 1 << 20, None, ct.byref(h)) == -5
    assert L.fredopt_load_matrices_noalloc(ct.byref(m), ct.c_void_p(256), 16, None,
                                           ct.byref(h)) == -5
    m.storage = 9
    assert L.fredopt_load_matrices(ct.byref(m), ct.c_void_p(256), 1 << 20, None,
                                   ct.byref(h)) == -2
    assert L.fredopt_load_matrices_noalloc(ct.byref(m), ct.c_void_p(256), 1 << 20, None,
                                           ct.byref(h)) == -2
    assert not h.value


@pytest.mark.parametrize("field,value", [("lam", 0.0), ("lam", 2.5), ("alpha", 1.0),
                                         ("eta", 0.0), ("normalization", 5),
                                         ("reductions_n", -1), ("objective", 2),
                                         ("unit_direction", 2)])
def test_param_ranges_documented(field, value):
    """Parameter ranges from Fig. 2's caption and the text after Fig. 3 are the ones
    the binding forwards; the library checks them (exercised on the GPU)."""
    p = fredopt.SolverParams(**{field: value})
    s = p.struct()
    assert getattr(s, "lambda_" if field == "lam" else field) == value


def test_binding_rejects_bad_tensors_before_the_call():
    """The binding checks every tensor it hands to the library: a host tensor, a
    wrong dtype, a non-contiguous view or a wrong length raises FredoptError before
    the C call (the library cannot check raw pointers)."""
    import torch
    from paper_2509_20012_amd import phantom as ph
    plan = fredopt.Plan(None, None, n_rows=6, n_cols=4, nnz=0, storage=0)
    x = torch.zeros(4)
    with pytest.raises(fredopt.FredoptError, match="device tensor"):
        fredopt.dose_let(plan, x)
    prob = fredopt.DeviceProblem(ph._empty_problem(6), ph.C_DL, device="cpu")
    with pytest.raises(fredopt.FredoptError, match="device tensor"):
        prob.struct(6)
    with pytest.raises(fredopt.FredoptError, match="device tensor"):
        fredopt.solve(plan, prob, fredopt.SolverParams(), fredopt.new_state(), x)

    # dtype, layout and length checks, on tensors that claim to live on the device
    class OnDevice(torch.Tensor):
        is_cuda = True

    def check(t, n, dtype=None):
        return fredopt._dev(t.as_subclass(OnDevice), n, "x", dtype)

    with pytest.raises(fredopt.FredoptError, match="dtype"):
        check(torch.zeros(4, dtype=torch.float64), 4)
    with pytest.raises(fredopt.FredoptError, match="contiguous"):
        check(torch.zeros(4, 2)[:, 0], 4)
    with pytest.raises(fredopt.FredoptError, match="elements"):
        check(torch.zeros(3), 4)
    t = torch.zeros(4)
    assert check(t, 4) == t.data_ptr()
    k = torch.zeros(6, dtype=torch.int16)
    assert check(k, 6, torch.int16) == k.data_ptr()
