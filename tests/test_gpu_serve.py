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
    params = fo.SolverParams()
    iter_max = params.iter_max
    done = serve.serve_one_at_a_time(reqs, params)
    assert all(r.k == 5 for r in done)
    assert params.iter_max == iter_max   # the caller's parameters are left as they were
    assert serve.percentile([r.latency for r in done], 50) > 0


def test_plan_cache_reuses_and_evicts(fo):
    """With plan_cache, a later request of a finished plan takes its resident matrices
    (no load); an admission that needs room frees idle plans, least recently used
    first; every result equals the request served alone, bit for bit, and the budget
    holds throughout."""
    from paper_2509_20012_amd import serve
    A = ph.tiny_problem(300, 30, 0.15, seed=21)
    B = ph.tiny_problem(1000, 130, 0.05, seed=5)
    C = ph.tiny_problem(800, 90, 0.08, seed=8)
    size = {id(p): serve.plan_bytes(p) for p in (A, B, C)}
    assert size[id(C)] <= size[id(B)]
    # room for A and B: C's admission evicts the idle B (A was used after it); B's
    # return evicts the idle C; both later A requests find A resident
    seq = [(A, 0.0, 6), (B, 0.0, 9), (A, 0.3, 7), (C, 0.6, 5), (A, 0.9, 8), (B, 1.2, 4)]
    reqs = [serve.Request(i, p, n, t) for i, (p, t, n) in enumerate(seq)]
    budget = size[id(A)] + size[id(B)] + 1
    srv = serve.Server(budget, fo.SolverParams(alpha=0.9), quantum=4, plan_cache=True)
    done = srv.run(reqs)
    print(f"cache hits {srv.cache_hits}, evictions {srv.resident.evictions}, peak bytes "
          f"{srv.peak_bytes} of {budget}", flush=True)
    assert len(done) == len(reqs)
    assert srv.peak_bytes <= budget
    assert srv.cache_hits == 2 and srv.resident.evictions == 2
    for r in done:
        x_ref, ks = _alone(fo, r.phantom, fo.SolverParams(alpha=0.9), r.iters)
        assert (r.k, r.s) == ks, r.rid
        assert np.array_equal(r.x, x_ref), r.rid
        assert r.finished >= r.loaded >= r.admitted >= r.arrival
    # the one-at-a-time form with resident plans gives the same results
    base = serve.serve_one_at_a_time([serve.Request(i, p, n, t) for i, (p, t, n) in
                                      enumerate(seq)], fo.SolverParams(alpha=0.9),
                                     plan_cache=True)
    for r, b in zip(done, base):
        assert np.array_equal(r.x, b.x) and (r.k, r.s) == (b.k, b.s)
