"""Slice-width autotuner: picks a plan's lanes per row by timing the forward pass.

The sliced-ELL copy spreads each row over `lanes_per_row` lanes (a slice holds
64 / lanes_per_row rows); the width is fixed when the matrices are loaded.  The
default rule takes the largest power of two not above (mean row length) / 64; this
module instead loads the plan with each candidate width and keeps the one whose
dose/LETd pass (the all-row forward product, timed with HIP events on the current
stream) is fastest.  Host logic only: every measurement goes through the C ABI.
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
