"""Volume histograms (DVH / LVH / cDLVH, Figs. 4-5) and nearest-rank quantiles (D95,
D98, cDL30: Sections 2.4.1 and 2.5) on the GPU, through the C ABI.

Both are exact: the histogram counts are integers, bin decisions are taken in FP64
on both sides from the same FP32 values; the quantiles are selected, not
interpolated, so they equal the sorted values bit for bit.  On a solved plan the GPU
evaluation of its own dose agrees exactly with the host's, and within T1 with the
evaluation of the oracle's dose at the same fluence.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2509_20012_amd import metrics
from paper_2509_20012_amd import phantom as ph

pytestmark = pytest.mark.gpu

T1 = 1e-5


@pytest.fixture(scope="module")
def fo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_20012_amd import fredopt
    fredopt.lib()
    return fredopt


def _values(n, seed):
    """Doses with zeros, ties, values past vmax and a few negatives."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.0, 2.5, n).astype(np.float32)
    v[rng.integers(0, n, n // 10)] = 0.0
    v[rng.integers(0, n, n // 20)] = np.float32(1.25)
    v[rng.integers(0, n, n // 50)] = -rng.uniform(0.0, 1.0, n // 50).astype(np.float32)
    return v


def _cum_ref(v, rows, vmax, n_bins):
    x = v[rows].astype(np.float64)
    ok = x >= 0.0
    b = np.floor(x[ok] * n_bins / vmax)
    b = np.minimum(b, n_bins).astype(np.int64)
    counts = np.bincount(b, minlength=n_bins + 1)
    return np.cumsum(counts[::-1])[::-1]


@pytest.mark.parametrize("n_bins", [1, 7, 100, 32768])
def test_volume_histogram_exact(fo, n_bins):
    import torch
    v = _values(100_000, n_bins)
    v[5] = np.nan
    rows = np.random.default_rng(1).integers(0, v.size, 60_000)  # duplicates count twice
    cum = fo.volume_histogram(torch.from_numpy(v).cuda(), rows, 2.0, n_bins)
    torch.cuda.synchronize()
    got = cum.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(got, _cum_ref(v, rows, 2.0, n_bins))


@pytest.mark.parametrize("n", [1, 2, 1000, 100_000])
def test_quantiles_exact(fo, n):
    import torch
    v = _values(100_000, 7 + n)
    rows = np.random.default_rng(n).permutation(v.size)[:n]
    qs = [0.05, 0.02, 0.70, 1.0, 1e-9, 0.5]
    out = fo.roi_quantiles(torch.from_numpy(v).cuda(), rows, qs)
    torch.cuda.synchronize()
    srt = np.sort(v[rows])
    for k, q in enumerate(qs):
        rank = min(max(1, int(np.ceil(q * n - 1e-12))), n)
        assert out[k].item() == srt[rank - 1], (q, n)
        assert out[k].item() == ph.percentile_nearest_rank(v[rows], q)


def test_empty_region_and_bad_rows(fo):
    import torch
    v = torch.ones(10, dtype=torch.float32, device="cuda")
    out = fo.roi_quantiles(v, np.zeros(0, np.int64), [0.5, 0.05])
    cum = fo.volume_histogram(v, np.zeros(0, np.int64), 1.0, 4)
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 0.0) and np.all(cum.cpu().numpy() == 0)
    with pytest.raises(fo.FredoptError):
        fo.roi_quantiles(v, np.array([3, 10]), [0.5])


def test_solved_plan_evaluation(fo):
    """The 32^3 water plan after 100 iterations: PTV D95 / D98 and the PTV DVH and OAR
    LVH from the GPU's dose equal the host's evaluation of the same arrays, and the
    oracle's dose at the same fluence gives the same D95 within T1."""
    import torch
    w = ph.water32()
    plan, prob, x0 = fo.load_phantom(w)
    st = fo.new_state()
    x = x0.clone()
    fo.solve(plan, prob, fo.SolverParams(iter_max=100), st, x)
    dose, letd, cdl = fo.dose_let(plan, x, w.c)
    ptv, oar = w.roi["PTV"], w.roi["OAR_cyl"]
    q = fo.roi_quantiles(dose, ptv, [0.05, 0.02])
    dvh = fo.volume_histogram(dose, ptv, 2.5, 250)
    lvh = fo.volume_histogram(letd, oar, 10.0, 200)
    torch.cuda.synchronize()
    d = dose.cpu().numpy()
    t = letd.cpu().numpy()
    assert q[0].item() == metrics.d_percent(d[ptv], 0.95)
    assert q[1].item() == metrics.d_percent(d[ptv], 0.98)
    np.testing.assert_array_equal(dvh.cpu().numpy().astype(np.int64),
                                  _cum_ref(d, ptv, 2.5, 250))
    np.testing.assert_array_equal(lvh.cpu().numpy().astype(np.int64),
                                  _cum_ref(t, oar, 10.0, 200))
    d_ref, _, _, _ = Oracle(w).dose_let(x.cpu().numpy().astype(np.float64))
    assert q[0].item() == pytest.approx(metrics.d_percent(d_ref[ptv], 0.95), rel=T1)


def test_percentile_constraint_from_forward_calculation(fo):
    """cDL30 of the OAR at unit fluence, computed on the GPU, against the target the
    phantom placed from the host's row sums (the same nearest-rank definition)."""
    import torch
    w = ph.water32()
    plan, _, x0 = fo.load_phantom(w)
    oar = w.roi["OAR_cyl"]
    got = fo.percentile_target(plan, x0, oar, w.c, 0.70)
    want = float(w.cdl_target[oar][0])
    assert got == pytest.approx(want, rel=T1)
    _, _, _, c_ref = Oracle(w).dose_let(w.x0.astype(np.float64))
    assert got == pytest.approx(ph.percentile_nearest_rank(c_ref[oar], 0.70), rel=T1)
    torch.cuda.synchronize()
