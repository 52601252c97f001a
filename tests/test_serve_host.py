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
