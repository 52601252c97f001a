"""The boundary's two options against the FP64 oracle, through the C ABI.

objective = ONE_SIDED: Eq. (2)'s OAR term counted only where cDL exceeds its target
(the device then searches the step by evaluating the cost for windows of candidate
exponents); unit_direction = 1: the perturbation moves along g / ||g||.  Both
iteration schedules (with and without the objective-row view) and both projection
paths; T2 with the same integer step exponent, T3 on the 32^3 water plan, a batch
equal to its plans alone, and the option values the library refuses.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from paper_2509_20012_amd import metrics
from paper_2509_20012_amd import phantom as ph

pytestmark = pytest.mark.gpu

T2 = 1e-5
T3 = 5e-3


@pytest.fixture(scope="module")
def fo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_20012_amd import fredopt
    fredopt.lib()
    return fredopt


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _split_targets(p):
    """OAR targets at the median of c l at x0, so the one-sided term is off for
    about half the OAR rows (the printed term would push them up)."""
    _, l0, _, _ = Oracle(p).dose_let(p.x0.astype(np.float64))
    oar = (p.kind & ph.OBJ_CDL) > 0
    if oar.any():
        p.cdl_target[oar] = np.float32(np.median(p.c * l0[oar]))
    return p


def _oparams(q):
    return OracleParams(lam=q.lam, alpha=q.alpha, eta=q.eta, reductions_n=q.reductions_n,
                        normalization=q.normalization, line_search=1,
                        unit_direction=q.unit_direction)


@pytest.mark.parametrize("path", ["csc", "scatter"])
@pytest.mark.parametrize("reserve", [0, 100])
@pytest.mark.parametrize("r", [1, 2])
@pytest.mark.parametrize("objective,unit", [(1, 0), (0, 1), (1, 1)])
def test_options_steps_tiny(fo, objective, unit, r, reserve, path):
    """Reserve 100: the objective-row view; default reserve on this 2/3-objective
    problem: the schedule with two all-row products."""
    p = _split_targets(ph.tiny_problem(300, 30, 0.15, seed=21))
    print(f"options tiny objective={objective} unit={unit} r={r} reserve={reserve} "
          f"path={path}", flush=True)
    plan, prob, x0 = fo.load_phantom(p, gradient_reserve_pct=reserve)
    fo.set_scatter(plan, *((-1, -1) if path == "csc" else (0, 1 << 40)))
    q = fo.SolverParams(alpha=0.9, reductions_n=r, objective=objective, unit_direction=unit)
    o = Oracle(p, objective=objective)
    st = fo.new_state()
    x = x0.clone()
    xr = p.x0.astype(np.float64)
    k, s = 0, -1
    for it in range(5):
        fo.superiorize_step(plan, prob, q, st, x)
        xr, k, s, info = o.sa_iteration(xr, k, s, _oparams(q))
        assert (st.k, st.s) == (k, s), f"iteration {it}"
        assert np.linalg.norm(_np(x) - xr) <= T2 * np.linalg.norm(xr), f"iteration {it}"
        assert st.cost == pytest.approx(info["cost_before"], rel=1e-5)
        assert st.grad_sq == pytest.approx(info["grad_sq"], rel=1e-4)
        assert st.beta == pytest.approx(info["beta_last"], rel=1e-12)
        assert st.cost_perturbed < st.cost


@pytest.mark.parametrize("objective,unit", [(1, 0), (0, 1), (1, 1)])
def test_options_water32(fo, objective, unit):
    """Three outer iterations at T2 with the same step exponent, then T3 after 100."""
    import torch
    w32 = _split_targets(ph.water32())
    print(f"options water32 objective={objective} unit={unit}", flush=True)
    plan, prob, x0 = fo.load_phantom(w32)
    q = fo.SolverParams(objective=objective, unit_direction=unit)
    o = Oracle(w32, objective=objective)
    st = fo.new_state()
    x = x0.clone()
    xr = w32.x0.astype(np.float64)
    k, s = 0, -1
    for it in range(3):
        fo.superiorize_step(plan, prob, q, st, x)
        xr, k, s, info = o.sa_iteration(xr, k, s, _oparams(q))
        assert (st.k, st.s) == (k, s), f"iteration {it}"
        assert np.linalg.norm(_np(x) - xr) <= T2 * np.linalg.norm(xr)
    q.iter_max = 100
    st = fo.new_state()
    x = x0.clone()
    fo.solve(plan, prob, q, st, x)
    xr, k, s, _ = o.solve(w32.x0, 100, _oparams(q))
    dose, letd, _ = fo.dose_let(plan, x, w32.c)
    torch.cuda.synchronize()
    d_ref, _, letd_ref, _ = o.dose_let(xr)
    rg = metrics.plan_report(_np(dose), _np(letd), w32.roi)
    rr = metrics.plan_report(d_ref, letd_ref, w32.roi)
    print(f"s {st.s}/{s}\ngpu {rg}\noracle {rr}", flush=True)
    assert st.k == k == 100
    assert rg["PTV_D95"] == pytest.approx(rr["PTV_D95"], rel=T3)
    assert rg["OAR_cyl_mean_LETd"] == pytest.approx(rr["OAR_cyl_mean_LETd"], rel=T3)


def test_one_sided_batch_equals_alone(fo):
    """The step search runs one workgroup per plan; a batch of uneven plans gives
    every plan its solo iterates bit for bit."""
    phs = [_split_targets(ph.tiny_problem(300, 30, 0.15, seed=21)),
           _split_targets(ph.tiny_problem(1000, 130, 0.05, seed=5)),
           _split_targets(ph.small_plan(3001, 5000, 200))]
    q = fo.SolverParams(alpha=0.9, reductions_n=2, objective=1, unit_direction=1, iter_max=6)
    print("one-sided batch vs alone", flush=True)
    ref = []
    for p in phs:
        plan, prob, x0 = fo.load_phantom(p, gradient_reserve_pct=100)
        x = x0.clone()
        st = fo.new_state()
        fo.solve(plan, prob, q, st, x)
        ref.append((_np(x), st.k, st.s))
    loaded = [fo.load_phantom(p, gradient_reserve_pct=100) for p in phs]
    xs = [x0.clone() for _, _, x0 in loaded]
    states = [fo.new_state() for _ in phs]
    batch = fo.Batch([pl for pl, _, _ in loaded], [pr for _, pr, _ in loaded])
    batch.solve(q, states, xs, 6)
    for i in range(len(phs)):
        assert (states[i].k, states[i].s) == ref[i][1:]
        assert np.array_equal(_np(xs[i]), ref[i][0])
    batch.free()


def test_option_values_refused(fo):
    p = ph.tiny_problem(48, 12, 0.3, seed=3)
    plan, prob, x0 = fo.load_phantom(p)
    for kw in ({"objective": 2}, {"unit_direction": 2}, {"objective": -1}):
        with pytest.raises(fo.FredoptError) as e:
            fo.superiorize_step(plan, prob, fo.SolverParams(**kw), fo.new_state(), x0.clone())
        assert e.value.name == "E_ARG"
