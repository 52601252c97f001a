"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tiers (tolerances of the FP32 path):
  T1  dose_let with identical inputs: max relative error <= 1e-5 over rows with
      dose > 0, structurally empty rows exactly 0.
  T2  one sweep / one outer iteration from the same state: ||x_gpu - x_ref|| /
      ||x_ref|| <= 1e-5 and the same integer step exponent s.
  T3  a full solve: PTV D95 and OAR mean LETd within 0.5 %.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from paper_2509_20012_amd import metrics
from paper_2509_20012_amd import phantom as ph
from tests.helpers import load_filled

pytestmark = pytest.mark.gpu

T1 = 1e-5
T2 = 1e-5
T3 = 5e-3


@pytest.fixture(scope="module")
def fo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_20012_amd import fredopt
    fredopt.lib()  # raises if the library was not built
    return fredopt


@pytest.fixture(scope="module")
def w32():
    return ph.water32()


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel_rows(gpu, ref, mask=None):
    ref = np.asarray(ref, np.float64)
    m = (ref > 0) if mask is None else mask
    if not m.any():
        return 0.0
    return float(np.max(np.abs(gpu[m] - ref[m]) / np.abs(ref[m])))


def _params(fo, **kw):
    return fo.SolverParams(**kw)


def _oparams(p):
    return OracleParams(lam=p.lam, alpha=p.alpha, eta=p.eta, reductions_n=p.reductions_n,
                        normalization=p.normalization, line_search=1)


TINY = [dict(R=1, C=1, density=1.0, seed=1), dict(R=7, C=3, density=0.5, seed=2),
        dict(R=48, C=12, density=0.3, seed=3), dict(R=300, C=37, density=0.2, seed=4),
        dict(R=1000, C=130, density=0.05, seed=5),
        dict(R=64, C=16, density=0.3, seed=6, empty_rows=[0, 5, 63], empty_cols=[3, 15])]


@pytest.mark.parametrize("case", TINY, ids=lambda c: f"R{c['R']}C{c['C']}s{c['seed']}")
@pytest.mark.parametrize("on_device", [True, False])
def test_dose_let_tiny(fo, case, on_device):
    import torch
    p = ph.tiny_problem(**case)
    print(f"dose_let tiny {case} on_device={on_device}", flush=True)
    plan, prob, _ = fo.load_phantom(p, on_device=on_device)
    x = np.random.default_rng(case["seed"]).uniform(0.1, 2.0, p.n_cols).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    dose, letd, cdl = fo.dose_let(plan, xt, p.c)
    torch.cuda.synchronize()
    d_ref, l_ref, letd_ref, cdl_ref = Oracle(p).dose_let(x)
    dg, lg, cg = _np(dose), _np(letd), _np(cdl)
    assert _rel_rows(dg, d_ref) <= T1
    assert _rel_rows(lg, letd_ref, d_ref > 0) <= T1
    assert _rel_rows(cg, cdl_ref) <= T1
    empty = np.diff(p.row_ptr) == 0
    assert np.all(dg[empty] == 0.0) and np.all(lg[empty] == 0.0) and np.all(cg[empty] == 0.0)


@pytest.mark.parametrize("lpr", [1, 2, 4, 8, 16])
def test_dose_let_every_layout_width(fo, lpr):
    """Every lanes-per-row width of the sliced-ELL layout gives T1 results, on rows
    of very uneven length (ragged slices and windows)."""
    import torch
    p = ph.tiny_problem(2500, 300, 0.08, seed=40 + lpr, empty_rows=[0, 17, 2499])
    plan, _, _ = fo.load_phantom(p, lanes_per_row=lpr)
    assert plan.info()["lanes_per_row"] == lpr
    x = np.random.default_rng(lpr).uniform(0.0, 2.0, p.n_cols).astype(np.float32)
    dose, letd, _ = fo.dose_let(plan, torch.from_numpy(x).cuda(), p.c)
    torch.cuda.synchronize()
    d_ref, _, letd_ref, _ = Oracle(p).dose_let(x)
    assert _rel_rows(_np(dose), d_ref) <= T1
    assert _rel_rows(_np(letd), letd_ref, d_ref > 0) <= T1
    assert np.all(_np(dose)[np.diff(p.row_ptr) == 0] == 0.0)


def test_dose_let_water32(fo, w32):
    import torch
    plan, prob, x0 = fo.load_phantom(w32)
    x = np.random.default_rng(0).uniform(0.0, 2.0, w32.n_cols).astype(np.float32)
    dose, letd, cdl = fo.dose_let(plan, torch.from_numpy(x).cuda(), w32.c)
    torch.cuda.synchronize()
    d_ref, l_ref, letd_ref, cdl_ref = Oracle(w32).dose_let(x)
    assert _rel_rows(_np(dose), d_ref) <= T1
    assert _rel_rows(_np(letd), letd_ref, d_ref > 0) <= T1
    assert _rel_rows(_np(cdl), cdl_ref) <= T1
    # LETd lies within the LET range of the contributing beamlets (0.5 .. 10 keV/um)
    lg = _np(letd)[d_ref > 0]
    assert lg.min() >= 0.5 * (1 - 1e-6) and lg.max() <= 10.0 * (1 + 1e-6)


def test_dose_linearity_gpu(fo, w32):
    import torch
    plan, _, _ = fo.load_phantom(w32)
    rng = np.random.default_rng(1)
    x1 = rng.uniform(0, 1, w32.n_cols).astype(np.float32)
    x2 = rng.uniform(0, 1, w32.n_cols).astype(np.float32)
    d1 = _np(fo.dose_let(plan, torch.from_numpy(x1).cuda(), want=("dose",))[0])
    d2 = _np(fo.dose_let(plan, torch.from_numpy(x2).cuda(), want=("dose",))[0])
    d12 = _np(fo.dose_let(plan, torch.from_numpy(x1 + x2).cuda(), want=("dose",))[0])
    m = d12 > 0
    assert np.max(np.abs(d12[m] - d1[m] - d2[m]) / d12[m]) <= 1e-6 * 4


# projection paths: the column-major copy for every row ("csc"), the active-row
# scatter whenever rows are violated ("scatter", with the default and with an odd
# workgroup count), and the plan's own choice ("auto")
PATHS = {"csc": (-1, -1), "scatter": (0, 1 << 40), "scatter7": (7, 1 << 40), "auto": (0, -1)}


def _set_path(fo, plan, path):
    n_wg, max_rows = PATHS[path]
    fo.set_scatter(plan, n_wg, max_rows)
    info = plan.info()
    if path == "csc":
        assert info["scatter_wgs"] == 0
    elif path == "scatter7":
        assert info["scatter_wgs"] == 7
    else:
        assert info["scatter_wgs"] > 0


@pytest.mark.parametrize("path", ["csc", "scatter", "scatter7"])
@pytest.mark.parametrize("norm", [0, 1, 2])
@pytest.mark.parametrize("seed", [11, 12])
def test_project_sweep_tiny(fo, norm, seed, path):
    import torch
    p = ph.tiny_problem(200, 24, 0.2, seed=seed)
    print(f"project_sweep tiny seed={seed} norm={norm} path={path}", flush=True)
    plan, prob, _ = fo.load_phantom(p)
    _set_path(fo, plan, path)
    x = np.random.default_rng(seed).uniform(0.5, 1.5, p.n_cols).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    q = _params(fo, lam=1.3, normalization=norm)
    prox = fo.project_sweep(plan, prob, q, xt, weight_scale=0.9)
    xr, prox_ref, _ = Oracle(p).ams_simultaneous(x, lam=1.3, weight_scale=0.9, normalization=norm)
    xg = _np(xt)
    assert np.linalg.norm(xg - xr) <= T2 * max(np.linalg.norm(xr), 1e-30)
    assert prox == pytest.approx(prox_ref, rel=1e-4)


@pytest.mark.parametrize("path", ["csc", "scatter", "auto"])
def test_project_sweep_water32(fo, w32, path):
    import torch
    print(f"project_sweep water32 path={path}", flush=True)
    plan, prob, x0 = fo.load_phantom(w32)
    _set_path(fo, plan, path)
    q = _params(fo)
    o = Oracle(w32)
    x = x0.clone()
    xr = w32.x0.astype(np.float64)
    for it in range(3):
        prox = fo.project_sweep(plan, prob, q, x, weight_scale=0.999 ** it)
        xr, prox_ref, nv = o.ams_simultaneous(xr, lam=1.0, weight_scale=0.999 ** it,
                                              normalization=0)
        assert prox == pytest.approx(prox_ref, rel=1e-4)
    xg = _np(x)
    assert np.linalg.norm(xg - xr) <= T2 * np.linalg.norm(xr)


@pytest.mark.parametrize("path", ["csc", "scatter"])
@pytest.mark.parametrize("reserve", [0, 100])
@pytest.mark.parametrize("lpr", [1, 4])
@pytest.mark.parametrize("r", [0, 1, 2])
def test_superiorize_step_tiny(fo, r, lpr, reserve, path):
    """Both iteration schedules (objective-row view with a 100 % reserve, two
    all-row forward products with the default reserve on this 2/3-objective
    problem) and both projection paths against the oracle."""
    import torch
    p = ph.tiny_problem(300, 30, 0.15, seed=21)
    print(f"superiorize_step tiny r={r} lpr={lpr} reserve={reserve} path={path}", flush=True)
    plan, prob, x0 = fo.load_phantom(p, lanes_per_row=lpr, gradient_reserve_pct=reserve)
    _set_path(fo, plan, path)
    q = _params(fo, alpha=0.9, reductions_n=r)
    st = fo.new_state()
    o = Oracle(p)
    x = x0.clone()
    xr = p.x0.astype(np.float64)
    k, s = 0, -1
    for it in range(5):
        fo.superiorize_step(plan, prob, q, st, x)
        xr, k, s, info = o.sa_iteration(xr, k, s, _oparams(q))
        assert (st.k, st.s) == (k, s), f"iteration {it}"
        xg = _np(x)
        assert np.linalg.norm(xg - xr) <= T2 * np.linalg.norm(xr), f"iteration {it}"
        assert st.proximity == pytest.approx(info["proximity"], rel=1e-3, abs=1e-12)
        if r:
            assert st.cost_perturbed < st.cost


@pytest.mark.parametrize("path", ["csc", "scatter", "auto"])
def test_superiorize_step_water32(fo, w32, path):
    print(f"superiorize_step water32 path={path}", flush=True)
    plan, prob, x0 = fo.load_phantom(w32)
    _set_path(fo, plan, path)
    q = _params(fo)
    st = fo.new_state()
    o = Oracle(w32)
    x = x0.clone()
    xr = w32.x0.astype(np.float64)
    k, s = 0, -1
    for it in range(3):
        fo.superiorize_step(plan, prob, q, st, x)
        xr, k, s, info = o.sa_iteration(xr, k, s, _oparams(q))
        assert (st.k, st.s) == (k, s)
        xg = _np(x)
        assert np.linalg.norm(xg - xr) <= T2 * np.linalg.norm(xr)
        assert st.cost == pytest.approx(info["cost_before"], rel=1e-5)
        assert st.grad_sq == pytest.approx(info["grad_sq"], rel=1e-4)


def test_solve_water32_plan_quality(fo, w32):
    """T3: 100 superiorized iterations on the 32^3 phantom."""
    import torch
    plan, prob, x0 = fo.load_phantom(w32)
    q = _params(fo, iter_max=100)
    st = fo.new_state()
    x = x0.clone()
    fo.solve(plan, prob, q, st, x)
    xr, k, s, info = Oracle(w32).solve(w32.x0, 100, _oparams(q))
    assert st.k == k == 100
    print(f"gpu s={st.s} oracle s={s} cost={st.cost:.6g}/{info['cost_before']:.6g}", flush=True)
    dose, letd, _ = fo.dose_let(plan, x, w32.c)
    torch.cuda.synchronize()
    d_ref, _, letd_ref, _ = Oracle(w32).dose_let(xr)
    rg = metrics.plan_report(_np(dose), _np(letd), w32.roi)
    rr = metrics.plan_report(d_ref, letd_ref, w32.roi)
    print("gpu", rg, "\noracle", rr, flush=True)
    assert rg["PTV_D95"] == pytest.approx(rr["PTV_D95"], rel=T3)
    assert rg["OAR_cyl_mean_LETd"] == pytest.approx(rr["OAR_cyl_mean_LETd"], rel=T3)
    xg = _np(x)
    print("normwise x error", np.linalg.norm(xg - xr) / np.linalg.norm(xr), flush=True)


@pytest.mark.parametrize("r", [0, 1])
def test_dose_only_problem_water32(fo, w32, r):
    """The paper's dose-only arm (dose bounds and the PTV dose objective, no cDL or
    LETd terms): three outer iterations at T2 with the same step exponent, then D95
    within T3 after 100 iterations (r = 0: the feasibility sweep alone)."""
    import torch
    p = w32.dose_only()
    print(f"dose-only water32 r={r}", flush=True)
    plan, prob, x0 = fo.load_phantom(p)
    q = _params(fo, reductions_n=r)
    o = Oracle(p)
    st = fo.new_state()
    x = x0.clone()
    xr = p.x0.astype(np.float64)
    k, s = 0, -1
    for it in range(3):
        fo.superiorize_step(plan, prob, q, st, x)
        xr, k, s, _ = o.sa_iteration(xr, k, s, _oparams(q))
        assert (st.k, st.s) == (k, s)
        assert np.linalg.norm(_np(x) - xr) <= T2 * np.linalg.norm(xr)
    q.iter_max = 100
    st = fo.new_state()
    x = x0.clone()
    fo.solve(plan, prob, q, st, x)
    xr, _, _, _ = o.solve(p.x0, 100, _oparams(q))
    dose, letd, _ = fo.dose_let(plan, x, p.c)
    torch.cuda.synchronize()
    d_ref, _, letd_ref, _ = o.dose_let(xr)
    rg = metrics.plan_report(_np(dose), _np(letd), p.roi)
    rr = metrics.plan_report(d_ref, letd_ref, p.roi)
    print("gpu", rg, "\noracle", rr, flush=True)
    assert rg["PTV_D95"] == pytest.approx(rr["PTV_D95"], rel=T3)


@pytest.mark.parametrize("path", ["csc", "scatter"])
def test_solve_deterministic_and_resumable(fo, w32, path):
    print(f"determinism water32 path={path}", flush=True)
    plan, prob, x0 = fo.load_phantom(w32)
    _set_path(fo, plan, path)
    q = _params(fo, iter_max=20)
    xa = x0.clone()
    sa = fo.new_state()
    fo.solve(plan, prob, q, sa, xa)
    xb = x0.clone()
    sb = fo.new_state()
    fo.solve(plan, prob, q, sb, xb)
    assert np.array_equal(_np(xa), _np(xb)) and (sa.k, sa.s) == (sb.k, sb.s)
    xc = x0.clone()
    sc = fo.new_state()
    q10 = _params(fo, iter_max=10)
    fo.solve(plan, prob, q10, sc, xc)
    fo.solve(plan, prob, q10, sc, xc)
    assert np.array_equal(_np(xa), _np(xc)) and (sa.k, sa.s) == (sc.k, sc.s)
    # graph replay and direct launches agree bit for bit
    xd = x0.clone()
    sd = fo.new_state()
    for _ in range(20):
        fo.superiorize_step(plan, prob, q, sd, xd)
    assert np.array_equal(_np(xa), _np(xd))


@pytest.mark.parametrize("reserve", [0, -1])
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16i16"])
@pytest.mark.parametrize("path", ["csc", "scatter"])
def test_result_independent_of_workspace_contents(fo, w32, path, storage, reserve):
    """A solve reads nothing of the workspace that it has not written: workspaces
    that start as zeros, as NaNs (0xFF bytes) or as large finite values (0x7F) give
    the same iterates bit for bit (with the objective-row view, reserve 0, and
    without it, reserve -1), and in FP32 they match the oracle."""
    print(f"workspace contents water32 path={path} storage={storage} reserve={reserve}",
          flush=True)
    st_code = {"f32": fo.F32, "f16": fo.F16, "bf16i16": fo.BF16_IDX16}[storage]
    q = _params(fo, iter_max=20)
    runs = []
    for fill in (0x00, 0xFF, 0x7F):
        plan, prob, x0 = load_filled(fo, w32, fill, storage=st_code, reserve=reserve)
        _set_path(fo, plan, path)
        st = fo.new_state()
        x = x0.clone()
        fo.solve(plan, prob, q, st, x)
        runs.append((_np(x), st.k, st.s))
        plan.free()
    assert np.all(np.isfinite(runs[0][0]))
    for xr_, k_, s_ in runs[1:]:
        assert np.array_equal(runs[0][0], xr_) and (runs[0][1], runs[0][2]) == (k_, s_)
    if storage == "f32":
        xr, k, s, _ = Oracle(w32).solve(w32.x0, 20, _oparams(q))
        assert (runs[0][1], runs[0][2]) == (k, s)
        assert np.linalg.norm(runs[0][0] - xr) / np.linalg.norm(xr) <= T2


@pytest.mark.parametrize("storage", ["f32", "bf16i16"])
def test_entry_points_independent_of_workspace_contents(fo, w32, storage):
    """The first call on a freshly loaded plan, for each entry point (dose / LETd,
    one sweep on both projection paths, one superiorized step), gives the same
    result bit for bit whatever the workspace held before the load."""
    import torch
    print(f"entry points, workspace contents water32 storage={storage}", flush=True)
    st_code = {"f32": fo.F32, "bf16i16": fo.BF16_IDX16}[storage]
    x = torch.from_numpy(np.random.default_rng(4).uniform(0.5, 1.5, w32.n_cols)
                         .astype(np.float32)).cuda()
    q = _params(fo)
    out = {}
    for fill in (0x00, 0xFF, 0x7F):
        res = []
        plan, prob, _ = load_filled(fo, w32, fill, storage=st_code)
        res += [_np(t) for t in fo.dose_let(plan, x, w32.c)]
        plan.free()
        for path in ("csc", "scatter"):
            plan, prob, _ = load_filled(fo, w32, fill, storage=st_code)
            _set_path(fo, plan, path)
            xs = x.clone()
            prox = fo.project_sweep(plan, prob, q, xs)
            res += [_np(xs), np.array([prox])]
            plan.free()
        plan, prob, _ = load_filled(fo, w32, fill, storage=st_code)
        st = fo.new_state()
        xs = x.clone()
        fo.superiorize_step(plan, prob, q, st, xs)
        res += [_np(xs), np.array([st.k, st.s, st.cost])]
        plan.free()
        out[fill] = res
    for a in out[0x00]:
        assert np.all(np.isfinite(a))
    for fill in (0xFF, 0x7F):
        for a, b in zip(out[0x00], out[fill]):
            assert np.array_equal(a, b), hex(fill)


def test_wide_plan_without_lds_staging(fo):
    """70,000 beamlets: the input vector does not fit in LDS, so the forward passes
    gather it from global memory; the active-row scatter's column sums do not fit
    either and live in global memory; 16-bit column indices are refused.  T1 for
    dose / LETd / cDL, T2 for a sweep and a superiorized step on both projection
    paths."""
    import torch
    print("wide plan R=600 C=70000", flush=True)
    p = ph.tiny_problem(600, 70000, 0.001, seed=31)
    plan, prob, x0 = fo.load_phantom(p)
    info = plan.info()
    assert info["lds_x"] == 0 and info["scatter_wgs"] > 0
    x = torch.from_numpy(np.random.default_rng(8).uniform(0.5, 1.5, p.n_cols)
                         .astype(np.float32)).cuda()
    dose, letd, cdl = fo.dose_let(plan, x, p.c)
    d_r, l_r, t_r, c_r = Oracle(p).dose_let(_np(x))
    assert _rel_rows(_np(dose), d_r) <= T1
    assert _rel_rows(_np(letd), t_r, d_r > 0) <= T1
    assert _rel_rows(_np(cdl), c_r, d_r > 0) <= T1
    q = _params(fo)
    xr = Oracle(p).ams_simultaneous(p.x0, lam=q.lam, weight_scale=1.0,
                                    normalization=q.normalization)[0]
    xo, k, s, _ = Oracle(p).sa_iteration(p.x0.astype(np.float64), 0, -1, _oparams(q))
    for path in ("csc", "scatter"):
        _set_path(fo, plan, path)
        xs = x0.clone()
        fo.project_sweep(plan, prob, q, xs)
        assert np.linalg.norm(_np(xs) - xr) / np.linalg.norm(xr) <= T2, path
        st = fo.new_state()
        xs = x0.clone()
        fo.superiorize_step(plan, prob, q, st, xs)
        assert (st.k, st.s) == (k, s), path
        assert np.linalg.norm(_np(xs) - xo) / np.linalg.norm(xo) <= T2, path
    with pytest.raises(fo.FredoptError):
        fo.load_phantom(p, storage=fo.F16_IDX16)


@pytest.mark.parametrize("path", ["csc", "scatter"])
def test_wide_plan_independent_of_workspace_contents(fo, path):
    """The 70,000-beamlet plan (the scatter's column sums in global memory) gives the
    same sweep and solve bit for bit whatever its workspace held."""
    print(f"wide plan, workspace contents, path={path}", flush=True)
    p = ph.tiny_problem(600, 70000, 0.001, seed=31)
    q = _params(fo, iter_max=5)
    out = []
    for fill in (0x00, 0xFF, 0x7F):
        plan, prob, x0 = load_filled(fo, p, fill)
        _set_path(fo, plan, path)
        xs = x0.clone()
        fo.project_sweep(plan, prob, q, xs)
        st = fo.new_state()
        xg = x0.clone()
        fo.solve(plan, prob, q, st, xg)
        out.append((_np(xs), _np(xg), st.k, st.s))
        plan.free()
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0]) and np.array_equal(out[0][1], o[1])
        assert out[0][2:] == o[2:]


@pytest.mark.parametrize("case", ["no_entries", "no_rows"])
def test_empty_plans(fo, case):
    """Degenerate plans: rows without entries (every constraint row has a zero
    normal, so nothing moves and the gradient is zero) and a plan without rows
    (its problem arrays have length 0).  Every call succeeds; dose, LETd and cDL
    are 0; the fluence stays x0 (already >= 0); s stays -1; the oracle agrees."""
    import torch
    print(f"empty plan {case}", flush=True)
    R = 40 if case == "no_entries" else 0
    p = ph.tiny_problem(R, 6, 0.3, seed=9, empty_rows=list(range(R)))
    assert p.nnz == 0
    plan, prob, x0 = fo.load_phantom(p)
    x = torch.from_numpy(np.linspace(0.5, 1.5, p.n_cols).astype(np.float32)).cuda()
    dose, letd, cdl = fo.dose_let(plan, x, p.c)
    for t in (dose, letd, cdl):
        assert t.numel() == R and np.all(_np(t) == 0.0)
    q = _params(fo, iter_max=4)
    xs = x.clone()
    fo.project_sweep(plan, prob, q, xs)
    assert np.array_equal(_np(xs), _np(x))
    st = fo.new_state()
    xs = x0.clone()
    fo.superiorize_step(plan, prob, q, st, xs)
    assert (st.k, st.s) == (1, -1) and np.array_equal(_np(xs), _np(x0))
    st = fo.new_state()
    fo.solve(plan, prob, q, st, xs)
    assert (st.k, st.s) == (4, -1) and np.array_equal(_np(xs), _np(x0))
    if R > 0:
        xr, k, s, _ = Oracle(p).solve(p.x0, 4, _oparams(q))
        assert (k, s) == (4, -1) and np.array_equal(xr, p.x0.astype(np.float64))


def test_nonfinite_halts_the_solve(fo):
    """An iterate that overflows FP32 mid-solve (raw weights, lambda = 2, large
    priorities: the sweep overshoots and grows until d = D x is infinite) sets the
    device's non-finite flag; every later kernel of the call skips the plan, so a
    300-iteration solve stops where the step-by-step run first reports the error,
    with the same state and the same x."""
    import torch
    p = ph.tiny_problem(300, 30, 0.15, seed=21)
    p.w_feas[:] = 50.0
    q = _params(fo, lam=2.0, normalization=2, eta=1.0, iter_max=300)
    print("non-finite halt: step by step", flush=True)
    plan, prob, x0 = fo.load_phantom(p)
    st1 = fo.new_state()
    x1 = x0.clone()
    for it in range(300):
        try:
            fo.superiorize_step(plan, prob, q, st1, x1)
        except fo.FredoptError as e:
            assert e.name == "E_NONFINITE"
            break
    else:
        pytest.fail("the iterate did not overflow")
    assert 10 < it < 299, it
    print(f"non-finite halt: detected in outer iteration {it}; solve", flush=True)
    st2 = fo.new_state()
    x2 = x0.clone()
    with pytest.raises(fo.FredoptError) as e:
        fo.solve(plan, prob, q, st2, x2)
    assert e.value.name == "E_NONFINITE"
    torch.cuda.synchronize()
    assert (st2.k, st2.s) == (st1.k, st1.s)
    assert np.array_equal(_np(x2), _np(x1), equal_nan=True)
    # a NaN in the input is caught by the first pass and nothing moves
    x3 = x0.clone()
    x3[5] = float("nan")
    st3 = fo.new_state()
    with pytest.raises(fo.FredoptError):
        fo.solve(plan, prob, q, st3, x3)
    assert st3.k == 0
    xs = _np(x3)
    assert np.isnan(xs[5]) and np.array_equal(np.delete(xs, 5), np.delete(_np(x0), 5))


def test_load_errors(fo):
    import torch
    p = ph.tiny_problem(10, 4, 0.5, seed=3)
    bad_col = p.col_idx.copy()
    bad_col[0] = 4
    with pytest.raises(fo.FredoptError) as e:
        fo.load_matrices(p.row_ptr, bad_col, p.d_val, p.l_val, p.n_cols)
    assert e.value.name == "E_INDEX"
    bad_d = p.d_val.copy()
    bad_d[1] = -1.0
    with pytest.raises(fo.FredoptError) as e:
        fo.load_matrices(p.row_ptr, p.col_idx, bad_d, p.l_val, p.n_cols)
    assert e.value.name == "E_NONFINITE"
    bad_d[1] = np.nan
    with pytest.raises(fo.FredoptError) as e:
        fo.load_matrices(p.row_ptr, p.col_idx, bad_d, p.l_val, p.n_cols, on_device=False)
    assert e.value.name == "E_NONFINITE"
    bad_rp = p.row_ptr.copy()
    bad_rp[3], bad_rp[4] = bad_rp[4], bad_rp[3] - 1
    with pytest.raises(fo.FredoptError) as e:
        fo.load_matrices(bad_rp, p.col_idx, p.d_val, p.l_val, p.n_cols)
    assert e.value.name in ("E_SHAPE", "E_INDEX")
    plan, prob, x0 = fo.load_phantom(p)
    x_before = x0.clone()
    with pytest.raises(fo.FredoptError) as e:
        fo.project_sweep(plan, prob, fo.SolverParams(lam=2.5), x0)
    assert e.value.name == "E_ARG"
    arr = {k: v.copy() for k, v in p.problem_arrays().items()}
    arr["kind"][:] = ph.DOSE_LO | ph.DOSE_HI
    arr["dose_lo"][:] = 2.0
    arr["dose_hi"][:] = 1.0
    with pytest.raises(fo.FredoptError) as e:
        fo.project_sweep(plan, fo.DeviceProblem(arr, p.c), fo.SolverParams(), x0)
    assert e.value.name == "E_ARG"
    st = fo.new_state(k=-1)
    with pytest.raises(fo.FredoptError) as e:
        fo.solve(plan, prob, fo.SolverParams(iter_max=2), st, x0)
    assert e.value.name == "E_STATE"
    torch.cuda.synchronize()
    assert torch.equal(x0, x_before)


@pytest.mark.parametrize("reserve", [-1, 0, 100])
def test_gradient_copy_and_fallback(fo, reserve):
    """The objective-row CSC used by the gradient (default reserve), the full CSC
    (no reserve) and a reserve of the whole CSC give the oracle's iterates."""
    p = ph.tiny_problem(600, 50, 0.1, seed=77)
    plan, prob, x0 = fo.load_phantom(p, gradient_reserve_pct=reserve)
    q = _params(fo, alpha=0.9, reductions_n=2)
    st = fo.new_state()
    x = x0.clone()
    o = Oracle(p)
    xr, k, s = p.x0.astype(np.float64), 0, -1
    for it in range(4):
        fo.superiorize_step(plan, prob, q, st, x)
        info = plan.info()
        # two thirds of the rows carry objective terms: the 100 % reserve holds them
        assert info["schedule"] == (1 if reserve == 100 else 0)
        xr, k, s, info = o.sa_iteration(xr, k, s, _oparams(q))
        assert (st.k, st.s) == (k, s)
        assert st.grad_sq == pytest.approx(info["grad_sq"], rel=1e-4)
        assert np.linalg.norm(_np(x) - xr) <= T2 * np.linalg.norm(xr)


def test_gradient_copy_follows_kind_changes(fo):
    """Changing the kind array in place (same device address) is detected."""
    import torch
    p = ph.tiny_problem(400, 40, 0.12, seed=78)
    plan, prob, x0 = fo.load_phantom(p)
    q = _params(fo, alpha=0.9, iter_max=3)
    st = fo.new_state()
    x = x0.clone()
    fo.solve(plan, prob, q, st, x)
    # drop the objective terms of every other row, in place
    arr = {k: v.copy() for k, v in p.problem_arrays().items()}
    arr["kind"][::2] &= ~np.uint16(ph.OBJ_DOSE | ph.OBJ_CDL)
    prob.t["kind"].copy_(torch.from_numpy(arr["kind"].view(np.int16)).cuda())
    st2 = fo.new_state()
    x2 = x0.clone()
    fo.solve(plan, prob, q, st2, x2)
    xr, k, s, _ = Oracle(p, problem=arr).solve(p.x0, 3, _oparams(q))
    assert (st2.k, st2.s) == (k, s)
    assert np.linalg.norm(_np(x2) - xr) <= T2 * np.linalg.norm(xr)


def test_scatter_and_csc_paths_agree(fo, w32):
    """The two projection paths differ only by the rounding of the column sums."""
    import torch
    xs = {}
    for path in ("csc", "scatter"):
        plan, prob, x0 = fo.load_phantom(w32)
        _set_path(fo, plan, path)
        x = x0.clone()
        st = fo.new_state()
        for _ in range(3):
            fo.superiorize_step(plan, prob, _params(fo), st, x)
        xs[path] = (_np(x), (st.k, st.s))
    assert xs["csc"][1] == xs["scatter"][1]
    a, b = xs["csc"][0], xs["scatter"][0]
    assert np.linalg.norm(a - b) <= 2e-6 * np.linalg.norm(a)


def test_set_scatter_arguments(fo):
    p = ph.tiny_problem(20, 5, 0.5, seed=4)
    plan, _, _ = fo.load_phantom(p)
    for bad in [(-2, -1), (257, -1), (0, -2)]:
        with pytest.raises(fo.FredoptError):
            fo.set_scatter(plan, *bad)


@pytest.mark.parametrize("norm", [0, 1, 2])
@pytest.mark.parametrize("block", [8192, 16384, 32768])
def test_block_sequential_sweep_water32(fo, w32, block, norm):
    """Block-sequential sweeps (4, 2 and 1 blocks of the 32,768 rows) against the
    oracle's, three in a row at T2; one block equals the simultaneous sweep on the
    active-row path bit for bit."""
    import torch
    print(f"block sweep water32 block={block} norm={norm}", flush=True)
    plan, prob, x0 = fo.load_phantom(w32)
    q = _params(fo, lam=1.2, normalization=norm)
    o = Oracle(w32)
    x = x0.clone()
    xr = w32.x0.astype(np.float64)
    for it in range(3):
        fo.project_sweep_blocks(plan, prob, q, x, block, weight_scale=0.9)
        xr = o.ams_blocks(xr, block, lam=1.2, weight_scale=0.9, normalization=norm)
        assert np.linalg.norm(_np(x) - xr) <= T2 * np.linalg.norm(xr), it
    if block == 32768:
        _set_path(fo, plan, "scatter")
        xa, xb = x0.clone(), x0.clone()
        fo.project_sweep(plan, prob, q, xa, weight_scale=0.9)
        fo.project_sweep_blocks(plan, prob, q, xb, block, weight_scale=0.9)
        torch.cuda.synchronize()
        assert np.array_equal(_np(xa), _np(xb))


def test_block_sequential_sweep_ragged(fo):
    """20,000 random rows (windows of 8,192, 8,192 and 3,616 rows; lanes per row 1 and
    4), against the oracle; a block size that is not a multiple of 8,192 is refused."""
    p = ph.tiny_problem(20000, 300, 0.01, seed=97)
    o = Oracle(p)
    for lpr in (1, 4):
        print(f"block sweep ragged lpr={lpr}", flush=True)
        plan, prob, x0 = fo.load_phantom(p, lanes_per_row=lpr)
        q = _params(fo, lam=1.0, normalization=0)
        x = x0.clone()
        fo.project_sweep_blocks(plan, prob, q, x, 8192)
        xr = o.ams_blocks(p.x0, 8192, lam=1.0, weight_scale=1.0, normalization=0)
        assert np.linalg.norm(_np(x) - xr) <= T2 * np.linalg.norm(xr)
        with pytest.raises(fo.FredoptError) as e:
            fo.project_sweep_blocks(plan, prob, q, x, 5000)
        assert e.value.name == "E_ARG"
