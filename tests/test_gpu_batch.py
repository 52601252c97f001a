"""Batched form: several plans of uneven size iterated by the same launches.

A plan's iterates in a batch must equal, bit for bit, its iterates alone (the
active-row projection sums in exact fixed point, so sharing its rows among a
different number of workgroups changes nothing); and they must match the oracle to
the T2 tier.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from paper_2509_20012_amd import phantom as ph
from tests.helpers import load_filled

pytestmark = pytest.mark.gpu

T2 = 1e-5


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


def _mix():
    """Plans of uneven size and shape, with empty rows and columns in one."""
    return [ph.tiny_problem(300, 30, 0.15, seed=21),
            ph.tiny_problem(1000, 130, 0.05, seed=5),
            ph.tiny_problem(64, 16, 0.3, seed=6, empty_rows=[0, 5, 63], empty_cols=[3, 15]),
            ph.small_plan(3001, 5000, 200),
            ph.tiny_problem(1, 1, 1.0, seed=1)]


def _alone(fo, p, q, iters, reserve):
    plan, prob, x0 = fo.load_phantom(p, gradient_reserve_pct=reserve)
    x = x0.clone()
    st = fo.new_state()
    q.iter_max = iters
    fo.solve(plan, prob, q, st, x)
    return _np(x), (st.k, st.s), plan.info()["schedule"]


@pytest.mark.parametrize("r", [0, 1, 2])
@pytest.mark.parametrize("reserve", [100, -1, 0])
def test_batch_equals_alone_bitwise(fo, r, reserve):
    """reserve 100: every plan has the objective-row view (schedule with one all-row
    product); reserve -1: none has (two all-row products); default reserve: the
    random problems (two thirds objective rows) have none, the water plan has it, so
    the batch holds both schedules."""
    print(f"batch vs alone r={r} reserve={reserve}", flush=True)
    phs = _mix()
    q = fo.SolverParams(alpha=0.9, reductions_n=r)
    iters = 6
    ref = [_alone(fo, p, q, iters, reserve) for p in phs]
    loaded = [fo.load_phantom(p, gradient_reserve_pct=reserve) for p in phs]
    plans = [pl for pl, _, _ in loaded]
    probs = [pr for _, pr, _ in loaded]
    xs = [x0.clone() for _, _, x0 in loaded]
    states = [fo.new_state() for _ in phs]
    batch = fo.Batch(plans, probs)
    # two calls of 3 iterations: a batch resumes like a single plan
    batch.solve(q, states, xs, 3)
    batch.solve(q, states, xs, iters - 3)
    for i, p in enumerate(phs):
        xr, ks, sched = ref[i]
        if r > 0 and reserve != 0:
            assert sched == (1 if reserve == 100 else 0), p.name
        assert (states[i].k, states[i].s) == ks, p.name
        assert np.array_equal(_np(xs[i]), xr), p.name
    if r > 0 and reserve == 0:
        assert sorted({x[2] for x in ref}) == [0, 1]   # both schedules present
    batch.free()


def test_batch_mixed_projection_paths(fo):
    """One launch serves both projection paths: in the same batched iteration one plan
    takes the active-row scatter (allowed for any number of active rows), one the
    column-major walk (scatter off) and one whichever its device state picks.  Each
    plan's iterates equal its run alone with the same setting, bit for bit."""
    print("batch with mixed projection paths", flush=True)
    phs = [ph.small_plan(3001, 5000, 200), ph.tiny_problem(1000, 130, 0.05, seed=5),
           ph.tiny_problem(300, 30, 0.15, seed=21)]
    settings = [("scatter", lambda pl: fo.set_scatter(pl, 0, pl.n_rows)),
                ("column-major", lambda pl: fo.set_scatter(pl, -1)),
                ("device", lambda pl: None)]
    q = fo.SolverParams(alpha=0.9, reductions_n=1)
    iters = 5
    ref = []
    for p, (_, setup) in zip(phs, settings):
        plan, prob, x0 = fo.load_phantom(p, gradient_reserve_pct=100)
        setup(plan)
        x = x0.clone()
        st = fo.new_state()
        q.iter_max = iters
        fo.solve(plan, prob, q, st, x)
        ref.append((_np(x), (st.k, st.s), st.projection_path))
        plan.free()
    loaded = [fo.load_phantom(p, gradient_reserve_pct=100) for p in phs]
    for (pl, _, _), (_, setup) in zip(loaded, settings):
        setup(pl)
    states = [fo.new_state() for _ in phs]
    xs = [x0.clone() for _, _, x0 in loaded]
    batch = fo.Batch([pl for pl, _, _ in loaded], [pr for _, pr, _ in loaded])
    batch.solve(q, states, xs, iters)
    assert ref[0][2] == 1 and ref[1][2] == 0  # the two forced paths were taken
    for i, (p, (name, _)) in enumerate(zip(phs, settings)):
        assert states[i].projection_path == ref[i][2], name
        assert (states[i].k, states[i].s) == ref[i][1], name
        assert np.array_equal(_np(xs[i]), ref[i][0]), name
    batch.free()
    for pl, _, _ in loaded:
        pl.free()


def test_batch_independent_of_workspace_contents(fo):
    """Plans whose workspaces start as NaN bytes give, in a batch, the iterates of
    the same plans alone (every plan with the objective-row view, r = 1)."""
    print("batch with NaN-filled plan workspaces", flush=True)
    phs = _mix()
    q = fo.SolverParams(alpha=0.9, reductions_n=1)
    iters = 6
    ref = [_alone(fo, p, q, iters, 100) for p in phs]
    loaded = [load_filled(fo, p, 0xFF, reserve=100) for p in phs]
    xs = [x0.clone() for _, _, x0 in loaded]
    states = [fo.new_state() for _ in phs]
    batch = fo.Batch([pl for pl, _, _ in loaded], [pr for _, pr, _ in loaded])
    batch.solve(q, states, xs, iters)
    for i, p in enumerate(phs):
        xr, ks, _ = ref[i]
        assert (states[i].k, states[i].s) == ks, p.name
        assert np.array_equal(_np(xs[i]), xr), p.name
    batch.free()


def test_batch_matches_oracle(fo):
    phs = _mix()[:3]
    q = fo.SolverParams(alpha=0.9, reductions_n=1)
    loaded = [fo.load_phantom(p, gradient_reserve_pct=100) for p in phs]
    batch = fo.Batch([l[0] for l in loaded], [l[1] for l in loaded])
    xs = [l[2].clone() for l in loaded]
    states = [fo.new_state() for _ in phs]
    oq = OracleParams(lam=q.lam, alpha=q.alpha, eta=q.eta, reductions_n=q.reductions_n,
                      normalization=q.normalization, line_search=1)
    refs = [(p.x0.astype(np.float64), 0, -1) for p in phs]
    orcs = [Oracle(p) for p in phs]
    for it in range(4):
        batch.solve(q, states, xs, 1)
        for i, p in enumerate(phs):
            xr, k, s = refs[i]
            xr, k, s, _ = orcs[i].sa_iteration(xr, k, s, oq)
            refs[i] = (xr, k, s)
            assert (states[i].k, states[i].s) == (k, s), (p.name, it)
            assert np.linalg.norm(_np(xs[i]) - xr) <= T2 * np.linalg.norm(xr), (p.name, it)


def test_batch_arguments(fo):
    p = ph.tiny_problem(20, 5, 0.5, seed=4)
    plan, prob, x0 = fo.load_phantom(p)
    with pytest.raises(fo.FredoptError):
        fo.Batch([plan, plan], [prob, prob])   # the same plan twice
    plan16, prob16, _ = fo.load_phantom(p, storage=fo.F16)
    with pytest.raises(fo.FredoptError):
        fo.Batch([plan, plan16], [prob, prob16])  # mixed storage


def test_lane_autotuner_picks_a_timed_candidate(fo):
    from paper_2509_20012_amd import autotune
    p = ph.small_plan(3001, 5000, 200)
    best, times = autotune.choose_lanes(p, candidates=(1, 2, 4), reps=2)
    assert set(times) == {1, 2, 4} and best in times
    assert all(t > 0 for t in times.values())
    assert times[best] == min(times.values())


def test_batch_autotuner_picks_the_fastest_timed_width(fo):
    from paper_2509_20012_amd import autotune
    phs = [ph.small_plan(3001, 5000, 200), ph.small_plan(3002, 8000, 300),
           ph.tiny_problem(300, 30, 0.15, seed=21)]
    best, rates = autotune.choose_batch_lanes(phs, candidates=(1, 2), iters=4)
    assert set(rates) == {1, 2} and best in rates
    assert all(r > 0 for r in rates.values())
    assert rates[best] == max(rates.values())


def test_scenario_batch_equals_alone(fo):
    """Robustness scenarios of one plan iterated together equal their solo runs."""
    phs = ph.scenario_plans(1, seed=3)
    q = fo.SolverParams(alpha=0.9)
    ref = [_alone(fo, p, q, 4, 0) for p in phs]
    loaded = [fo.load_phantom(p) for p in phs]
    batch = fo.Batch([l[0] for l in loaded], [l[1] for l in loaded])
    xs = [l[2].clone() for l in loaded]
    states = [fo.new_state() for _ in phs]
    batch.solve(q, states, xs, 4)
    for i, p in enumerate(phs):
        assert (states[i].k, states[i].s) == ref[i][1], p.name
        assert np.array_equal(_np(xs[i]), ref[i][0]), p.name
