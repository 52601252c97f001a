"""Slice-width autotuners: pick lanes per row by timing what the width is for.

The sliced-ELL copy spreads each row over `lanes_per_row` lanes (a slice holds
64 / lanes_per_row rows); the width is fixed when the matrices are loaded.  The
default rule takes the largest power of two not above (mean row length) / 64.

* choose_lanes: a plan solved alone.  Each candidate width is loaded and the plan's
  dose/LETd pass (the all-row forward product, timed with HIP events on the current
  stream) is timed; the fastest wins.  Alone, a small plan is bound by latency, so
  wider slices (more lanes per row, more rows in flight) tend to win.
* choose_batch_lanes: plans iterated together.  A full batch keeps the GPU busy
  with other plans' work, so what counts is the batched iteration itself: every
  plan is loaded at each candidate width, the batch is built and a few outer
  iterations are timed; the fastest width is used for all plans.

Host logic only: every measurement goes through the C ABI.
"""
from __future__ import annotations

from typing import Dict, Sequence, Tuple

from . import fredopt


def time_forward(plan: "fredopt.Plan", x, c: float, reps: int = 5) -> float:
    """Mean milliseconds of one dose/LETd pass of `plan` at fluence x."""
    import torch
    fredopt.dose_let(plan, x, c)  # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fredopt.dose_let(plan, x, c)
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def choose_lanes(ph, storage: int = fredopt.F32, candidates: Sequence[int] = (1, 2, 4, 8, 16),
                 reps: int = 5) -> Tuple[int, Dict[int, float]]:
    """(fastest lanes per row, {lanes: ms}) for a phantom's matrices."""
    times: Dict[int, float] = {}
    for lanes in candidates:
        plan, _, x0 = fredopt.load_phantom(ph, storage=storage, lanes_per_row=lanes)
        times[lanes] = time_forward(plan, x0, ph.c, reps)
        plan.free()
    best = min(times, key=lambda k: (times[k], k))
    return best, times


def choose_batch_lanes(phantoms, storage: int = fredopt.F32, candidates: Sequence[int] = (1, 2, 4),
                       iters: int = 20, reductions_n: int = 1,
                       gradient_reserve_pct: int = 0) -> Tuple[int, Dict[int, float]]:
    """(fastest lanes per row for the whole batch, {lanes: plan-iterations/s})."""
    import time
    import torch
    rates: Dict[int, float] = {}
    q = fredopt.SolverParams(reductions_n=reductions_n)
    for lanes in candidates:
        loaded = [fredopt.load_phantom(p, storage=storage, lanes_per_row=lanes,
                                       gradient_reserve_pct=gradient_reserve_pct)
                  for p in phantoms]
        batch = fredopt.Batch([l[0] for l in loaded], [l[1] for l in loaded])
        xs = [l[2].clone() for l in loaded]
        states = [fredopt.new_state() for _ in loaded]
        batch.solve(q, states, xs, 2)  # graph capture and warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.solve(q, states, xs, iters)
        torch.cuda.synchronize()
        rates[lanes] = len(loaded) * iters / (time.perf_counter() - t0)
        batch.free()
        for plan, _, _ in loaded:
            plan.free()
    best = max(rates, key=lambda k: (rates[k], -k))
    return best, rates
