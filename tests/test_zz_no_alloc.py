"""The load that allocates no device memory (fredopt_load_matrices_noalloc) against
the ordinary load (fredopt_load_matrices), both through the C ABI with host-resident
matrices, so that the first stages them in the library's fixed per-device area and
the second in a buffer it allocates.  Two calls in a row, the second with a smaller
plan: each plan must give the same plan description, the same dose / LETd / cDL and
the same solve, bit for bit, as the ordinary load of the same matrices."""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2509_20012_amd import phantom as ph

pytestmark = pytest.mark.gpu

STAGING_MAX = 128 << 20  # FREDOPT_NOALLOC_STAGING_BYTES


@pytest.fixture(scope="module")
def fo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_20012_amd import fredopt
    fredopt.lib()
    return fredopt


def _staged_bytes(p):
    a = lambda n: (n + 255) // 256 * 256  # noqa: E731
    return a(8 * (p.n_rows + 1)) + 3 * a(4 * p.nnz)


def _outputs(fo, plan, p, iters):
    import torch
    x = torch.from_numpy(np.random.default_rng(7).uniform(0.2, 1.8, p.n_cols)
                         .astype(np.float32)).cuda()
    dose, letd, cdl = fo.dose_let(plan, x, p.c)
    prob = fo.DeviceProblem(p.problem_arrays(), p.c)
    xs = torch.from_numpy(np.ascontiguousarray(p.x0, np.float32)).cuda()
    st = fo.new_state()
    fo.solve(plan, prob, fo.SolverParams(iter_max=iters), st, xs)
    torch.cuda.synchronize()
    return ([t.cpu().numpy() for t in (dose, letd, cdl, xs)],
            (st.k, st.s, st.n_violated, st.cost, st.proximity))


def _same(a, b):
    (arrs_a, st_a), (arrs_b, st_b) = a, b
    for u, v in zip(arrs_a, arrs_b):
        assert u.tobytes() == v.tobytes()
    assert st_a == st_b


def test_noalloc_load_equals_load_twice(fo):
    cases = [ph.tiny_problem(6000, 420, 0.04, seed=11),   # larger first
             ph.tiny_problem(900, 70, 0.1, seed=12)]      # then a smaller plan
    first = None
    for i, p in enumerate(cases):
        print(f"noalloc load call {i}: {p.n_rows} x {p.n_cols}, nnz {p.nnz}, "
              f"staged {_staged_bytes(p)} bytes", flush=True)
        assert _staged_bytes(p) <= STAGING_MAX
        ref = fo.load_matrices(p.row_ptr, p.col_idx, p.d_val, p.l_val, p.n_cols,
                               on_device=False)
        got = fo.load_matrices(p.row_ptr, p.col_idx, p.d_val, p.l_val, p.n_cols,
                               on_device=False, noalloc=True)
        assert got.info() == ref.info()
        out_ref = _outputs(fo, ref, p, 12)
        out_got = _outputs(fo, got, p, 12)
        _same(out_got, out_ref)
        if first is None:
            first = (got, p, out_got)
        ref.free()
    # the first plan does not depend on what the area held afterwards
    got0, p0, out0 = first
    _same(_outputs(fo, got0, p0, 12), out0)
    got0.free()


def test_noalloc_load_refuses_what_the_area_cannot_hold(fo):
    import torch
    # 1,400 rows x 8,192 columns, full rows: 11.5M entries, ~137 MB staged
    R, C = 1400, 8192
    rp = np.arange(R + 1, dtype=np.int64) * C
    ci = np.tile(np.arange(C, dtype=np.int32), R)
    v = np.full(R * C, 0.5, np.float32)
    staged = _staged_bytes(SimpleNamespace(n_rows=R, nnz=R * C))
    assert staged > STAGING_MAX
    print(f"noalloc load refusal: staged {staged} bytes", flush=True)
    with pytest.raises(fo.FredoptError) as e:
        fo.load_matrices(rp, ci, v, v, C, on_device=False, noalloc=True)
    assert e.value.status == -5 and "staging" in str(e.value)
    # device-resident matrices need no staging: the same matrices load
    plan = fo.load_matrices(rp, ci, v, v, C, on_device=True, noalloc=True)
    x = torch.ones(C, dtype=torch.float32, device="cuda")
    dose, _, _ = fo.dose_let(plan, x, ph.C_DL)
    torch.cuda.synchronize()
    assert np.all(dose.cpu().numpy() == np.float32(0.5 * C))
    plan.free()
