"""Host-side pieces of the serving loop (no GPU needed)."""
import numpy as np

from paper_2509_20012_amd import phantom as ph
from paper_2509_20012_amd import serve


def test_percentile_nearest_rank():
    v = [5.0, 1.0, 4.0, 2.0, 3.0]
    assert serve.percentile(v, 50) == 3.0
    assert serve.percentile(v, 99) == 5.0
    assert serve.percentile(v, 0) == 1.0
    assert np.isnan(serve.percentile([], 50))


def test_poisson_trace_rate_and_order():
    t = serve.poisson_trace(4000, 4.0, seed=4)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 4.0) < 0.25


def test_batch_sizes_log_uniform_and_correlated():
    sizes = ph.batch_sizes(48, seed=3)
    rows = np.array([r for _, r, _ in sizes])
    cols = np.array([c for _, _, c in sizes])
    assert rows.min() >= 5000 and rows.max() <= 120000
    assert cols.min() >= 200 and cols.max() <= 4000
    # one draw per plan sets both sizes: their logarithms are linearly related
    assert np.corrcoef(np.log(rows), np.log(cols))[0, 1] > 0.999


def test_scenarios_shift_and_range():
    """Setup shifts move the dose with the beams; range scaling moves the Bragg
    peaks; the nominal structures and bounds stay put."""
    base = ph.small_plan(3001, 5000, 200)
    sx = ph.small_plan(3001, 5000, 200, shift_mm=(0.0, 3.0, 0.0))
    lr = ph.small_plan(3001, 5000, 200, range_scale=1.035)
    assert np.array_equal(base.kind, sx.kind) and np.array_equal(base.dose_hi, sx.dose_hi)
    n = round(base.n_rows ** (1 / 3))
    centres = (np.indices((n, n, n)).reshape(3, -1)[::-1].T + 0.5) * 3.0  # x, y, z in mm
    def centroid(p):
        rid = np.repeat(np.arange(p.n_rows), np.diff(p.row_ptr))
        dose = np.bincount(rid, weights=p.d_val.astype(np.float64), minlength=p.n_rows)
        return (dose[:, None] * centres).sum(0) / dose.sum()
    c0, c1 = centroid(base), centroid(sx)
    # the beams travel along x: a shift along y moves the dose by the shift
    assert abs((c1 - c0)[1] - 3.0) < 0.6
    assert abs((c1 - c0)[2]) < 0.6
    # longer ranges deposit dose deeper: more entries, same beamlets
    assert lr.n_cols == base.n_cols and lr.nnz > base.nnz
    assert len(ph.scenario_plans(1)) == 8


class _FakePlan:
    def __init__(self, name, log):
        self.name, self.log = name, log

    def free(self):
        self.log.append(self.name)


def test_resident_plans_lru_order():
    """Idle resident plans: take() hands back the newest kept plan of the phantom and
    counts a hit; phantoms are ordered by their latest use (kept or taken), and
    evict() frees the oldest plan of the least recently used phantom and returns its
    bytes; clear() frees the rest without counting them as evictions."""
    freed = []
    res = serve._Resident()

    class _A:  # what put() reads of a finished request
        def __init__(self, phantom, name, nbytes):
            self.req = serve.Request(0, phantom, 1, 0.0)
            self.plan, self.prob, self.x0, self.bytes = _FakePlan(name, freed), None, None, nbytes

    pa, pb, pc = object(), object(), object()
    res.put(_A(pa, "a1", 10))
    res.put(_A(pb, "b1", 20))
    res.put(_A(pa, "a2", 11))        # order by latest use: b, a
    assert res.take(pc) is None and res.hits == 0
    k = res.take(pa)                 # the newest plan of a; a stays the newest phantom
    assert k is not None and k.bytes == 11 and res.hits == 1
    res.put(_A(pc, "c1", 5))         # order: b, a, c
    assert res.evict() == 20 and freed == ["b1"]
    assert res.evict() == 10 and freed == ["b1", "a1"]
    assert res.take(pa) is None      # a has no idle plan left
    assert res.evictions == 2
    assert res.clear() == 5 and res.evictions == 2 and freed == ["b1", "a1", "c1"]
    assert res.evict() == 0
