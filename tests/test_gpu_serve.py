"""Serving form: requests admitted by a memory budget and iterated together while
the batch changes around them.  Each result must equal the request served alone
(bit for bit, same k and s) and the memory budget must hold at every moment.
"""
import numpy as np
import pytest

from paper_2509_20012_amd import phantom as ph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2509_20012_amd import fredopt
    fredopt.lib()
    return fredopt


def _alone(fo, p, q, iters):
    plan, prob, x0 = fo.load_phantom(p)
    x = x0.clone()
    st = fo.new_state()
    q.iter_max = iters
    fo.solve(plan, prob, q, st, x)
    return x.cpu().numpy(), (st.k, st.s)


def test_served_results_equal_alone(fo):
    from paper_2509_20012_amd import serve
    phs = [ph.tiny_problem(300, 30, 0.15, seed=21), ph.small_plan(3002, 6000, 300),
           ph.tiny_problem(1000, 130, 0.05, seed=5), ph.small_plan(3003, 9000, 400),
           ph.tiny_problem(64, 16, 0.3, seed=6, empty_rows=[0, 5, 63], empty_cols=[3, 15]),
           ph.small_plan(3004, 5000, 220)]
    iters = [160, 12, 120, 20, 140, 3]
    # the three small requests (one lane) arrive together; the first to finish its
    # load starts alone, the others join it as their loads complete (a batch), they
    # leave at different times and the longest finishes alone; the water plans (the
    # other lane) queue on the budget
    arrivals = [0.0, 0.0, 0.0, 0.0, 0.0, 0.05]
    reqs = [serve.Request(i, p, n, t) for i, (p, n, t) in enumerate(zip(phs, iters, arrivals))]
    sizes = [serve.plan_bytes(p) for p in phs]
    budget = sorted(sizes)[-1] + sorted(sizes)[-2]   # forces queueing
    q = fo.SolverParams(alpha=0.9)
    # the water plans (> 100k entries) form the second lane
    srv = serve.Server(budget, q, quantum=4, big_nnz=100_000)
    done = srv.run(reqs)
    print(f"batches built {srv.batches_built}, solo quanta {srv.solo_quanta}, peak active "
          f"{srv.peak_active}, peak bytes {srv.peak_bytes} of {budget}", flush=True)
    assert len(done) == len(reqs)
    assert srv.peak_bytes <= budget
    assert srv.batches_built >= 1 and srv.solo_quanta >= 1 and srv.peak_active >= 3
    for r in done:
        x_ref, ks = _alone(fo, r.phantom, fo.SolverParams(alpha=0.9), r.iters)
        assert (r.k, r.s) == ks, r.rid
        assert np.array_equal(r.x, x_ref), r.rid
        assert r.finished >= r.loaded >= r.admitted >= r.arrival


def test_one_at_a_time_baseline_runs(fo):
    from paper_2509_20012_amd import serve
    reqs = [serve.Request(i, ph.tiny_problem(200, 24, 0.2, seed=40 + i), 5, 0.0)
            for i in range(3)]
    done = serve.serve_one_at_a_time(reqs, fo.SolverParams())
    assert all(r.k == 5 for r in done)
    assert serve.percentile([r.latency for r in done], 50) > 0
