"""Robustness evaluation (Section 2.5: the final plan recomputed under setup and range
scenarios, the spread shown in Figs. 4-5) through the C ABI, against the FP64 oracle
scenario by scenario.

Nine scenarios of one water plan: nominal, ranges x (1 -+ 3.5 %), +-2 mm beam shifts
along each axis, all with the nominal plan's voxels, beamlets and dose scale.  One
fluence, one launch: every scenario's dose, LETd and cDL element-wise at T1, and the
per-voxel min / max bands equal to the min / max of the GPU's own per-scenario
values (exact) and within T1 of the oracle's.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2509_20012_amd import phantom as ph

pytestmark = pytest.mark.gpu

T1 = 1e-5
T1_16 = 1e-3


@pytest.fixture(scope="module")
def fo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_20012_amd import fredopt
    fredopt.lib()
    return fredopt


@pytest.fixture(scope="module")
def scen():
    return ph.robustness_scenarios(3005, 20000, 800)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(gpu, ref, mask):
    if not mask.any():
        return 0.0
    return float(np.max(np.abs(gpu[mask] - ref[mask]) / np.abs(ref[mask])))


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_nine_scenarios_against_the_oracle(fo, scen, storage):
    import torch
    st = {"f32": fo.F32, "f16": fo.F16}[storage]
    tol = T1 if storage == "f32" else T1_16
    print(f"robustness: 9 scenarios, storage {storage}", flush=True)
    plans = [fo.load_matrices(p.row_ptr, p.col_idx, p.d_val, p.l_val, p.n_cols, st)
             for p in scen]
    x = np.random.default_rng(12).uniform(0.5, 1.5, scen[0].n_cols).astype(np.float32)
    out = fo.scenario_dose_let(plans, torch.from_numpy(x).cuda(), scen[0].c)
    torch.cuda.synchronize()
    dose, letd, cdl = _np(out["dose"]), _np(out["letd"]), _np(out["cdl"])
    ref_d, ref_t = [], []
    for i, p in enumerate(scen):
        d_r, _, t_r, c_r = Oracle(p).dose_let(x)
        m = d_r > 0
        assert _rel(dose[i], d_r, m) <= tol, i
        assert _rel(letd[i], t_r, m) <= tol, i
        assert _rel(cdl[i], c_r, m) <= tol, i
        assert np.all(dose[i][~m] == 0.0) and np.all(letd[i][~m] == 0.0)
        ref_d.append(d_r)
        ref_t.append(t_r)
    # bands: exactly the extremes of the GPU's own values, and T1 of the oracle's
    assert np.array_equal(_np(out["dose_min"]), dose.min(axis=0))
    assert np.array_equal(_np(out["dose_max"]), dose.max(axis=0))
    assert np.array_equal(_np(out["letd_min"]), letd.min(axis=0))
    assert np.array_equal(_np(out["letd_max"]), letd.max(axis=0))
    rd, rt = np.array(ref_d), np.array(ref_t)
    for got, ref in ((out["dose_min"], rd.min(0)), (out["dose_max"], rd.max(0)),
                     (out["letd_min"], rt.min(0)), (out["letd_max"], rt.max(0))):
        assert _rel(_np(got), ref, ref > 0) <= tol
    # the scenarios differ: shifts and range errors move the dose
    spread = _np(out["dose_max"]) - _np(out["dose_min"])
    assert np.max(spread) > 0.05 * np.max(dose)
    for pl in plans:
        pl.free()


def test_one_scenario_and_bands_only(fo, scen):
    """n = 1: the bands are the scenario's own values; bands without per-scenario
    outputs; per-scenario outputs without bands."""
    import torch
    p = scen[0]
    plan = fo.load_matrices(p.row_ptr, p.col_idx, p.d_val, p.l_val, p.n_cols)
    x = torch.from_numpy(np.random.default_rng(3).uniform(0.5, 1.5, p.n_cols)
                         .astype(np.float32)).cuda()
    d1, l1, _ = fo.dose_let(plan, x, p.c)
    out = fo.scenario_dose_let([plan], x, p.c)
    b = fo.scenario_dose_let([plan], x, p.c, want=())
    nb = fo.scenario_dose_let([plan], x, p.c, bands=False)
    torch.cuda.synchronize()
    for o in (out, b):
        assert np.array_equal(_np(o["dose_min"]), _np(d1))
        assert np.array_equal(_np(o["dose_max"]), _np(d1))
        assert np.array_equal(_np(o["letd_min"]), _np(l1))
        assert np.array_equal(_np(o["letd_max"]), _np(l1))
    assert np.array_equal(_np(nb["dose"][0]), _np(d1)) and "dose_min" not in nb
    plan.free()


def test_mismatched_scenarios_refused(fo, scen):
    import torch
    a = scen[0]
    other = ph.small_plan(3006, 8000, 400)
    pa = fo.load_matrices(a.row_ptr, a.col_idx, a.d_val, a.l_val, a.n_cols)
    pb = fo.load_matrices(other.row_ptr, other.col_idx, other.d_val, other.l_val,
                          other.n_cols)
    x = torch.ones(a.n_cols, dtype=torch.float32, device="cuda")
    with pytest.raises(fo.FredoptError) as e:
        fo.scenario_dose_let([pa, pb], x, a.c)
    assert e.value.name == "E_SHAPE"
    pc = fo.load_matrices(a.row_ptr, a.col_idx, a.d_val, a.l_val, a.n_cols, fo.F16)
    with pytest.raises(fo.FredoptError) as e:
        fo.scenario_dose_let([pa, pc], x, a.c)
    assert e.value.name == "E_ARG"
    for pl in (pa, pb, pc):
        pl.free()
