#!/usr/bin/env python3
"""Throughput of the superiorized dose/LETd iteration on one MI355X.

A step is one outer iteration of the superiorization algorithm (Fig. 3 of Borys et
al., arXiv 2509.20012): the objective and its gradient (Eq. 2), the direction
products and the device-side step decision, the perturbation, the constraint
residuals and one simultaneous projection sweep (Fig. 2) with the x >= 0 clamp.
The default workload is the clinical-scale phantom (160 x 160 x 120 grid at 2 mm,
three fields of 80 x 50 spots = 12,000 beamlets, ~458k voxel rows, ~155M nonzeros
in each of D and L), synthetic and seeded, resident in HBM before timing starts.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "superiorized iters/s + achieved HBM GB/s vs plain FP32; p50/p99 plan latency"
HBM_PEAK_GBPS = 8000.0
KERNEL_SYMBOLS = {  # fredopt kernel id -> device symbol in profiler output (vt: storage)
    "fwd_obj": "fo::k_forward<{vt}, 1, {sub}>", "fwd_dir": "fo::k_forward<{vt}, 2, {sub}>",
    "fwd_resid": "fo::k_forward<{vt}, 3, 0>", "tr_grad": "fo::k_tr_chunks<{vt}, 0>",
    "tr_proj": "fo::k_tr_chunks<{vt}, 1>", "rows": "fo::k_rows<1>", "col": "fo::k_tcol",
    "finalize": "fo::k_finalize", "active_list": "fo::k_active_list",
    "scatter": "fo::k_project<{vt}, ...>", "scatter_sum": "fo::k_scatter_sum",
    "line_search": "fo::k_linesearch<{sub}>"}


def device_info() -> dict:
    """The GPU the line was measured on, as the runtime reports it (the roofline's
    peak is the published 8 TB/s of HBM3E, not a measured figure)."""
    import torch
    pr = torch.cuda.get_device_properties(0)
    info = {"name": pr.name, "compute_units": pr.multi_processor_count,
            "memory_gib": round(pr.total_memory / 2**30, 1)}
    arch = getattr(pr, "gcnArchName", None)
    if arch:
        info["arch"] = arch
    lds = getattr(pr, "shared_memory_per_multiprocessor", None)
    if lds:
        info["lds_kib_per_cu"] = round(lds / 1024)
    return info


def dtype_of(storage: str) -> str:
    """The arithmetic type of the path with the storage form it reads.  BF16 values
    (8-bit mantissa) miss the 1e-3 tolerance of the reduced-precision form against
    the original values; FP16 meets it."""
    if storage == "f32":
        return "f32"
    if storage.startswith("bf16"):
        return f"f32 (values stored {storage}; outside the 1e-3 tolerance of the 16-bit form)"
    return f"f32 (values stored {storage})"


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sources that define the iteration kernels (the counters in
    profiles/ are valid only for the kernels they were taken on)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2509_20012_amd", "csrc")
    for f in ("fredopt_device.h", "kernels_iter.hip"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(kernel: str, R: int, C: int, nnz: int, vb: int, n_tr_items: int,
                      grad_entries: int, n_obj_rows: int, obj_entries: int, ib: int = 4) -> int:
    """Bytes a kernel launch must move: the unpadded matrix entries (shared index, D
    and L values), the input vector once, per-row problem data and outputs.  Padding
    and re-reads are not counted.  vb: bytes per stored value; ib: bytes per column
    index of the row-major copy (the column-major copy keeps 4-byte row indices)."""
    b = ib + 2 * vb      # row-major entry
    bt = 4 + 2 * vb      # column-major entry
    if kernel == "fwd_obj" and obj_entries:   # objective rows only
        return obj_entries * b + 4 * C + n_obj_rows * (8 + 8 + 2 + 12)
    if kernel == "fwd_dir" and obj_entries:   # objective rows only; Q
        return obj_entries * b + 4 * C + n_obj_rows * (2 + 4)
    if kernel == "fwd_obj":     # x in; d, l, coef out; kind, w_obj, targets in
        return nnz * b + 4 * C + R * (8 + 8 + 2 + 12)
    if kernel == "fwd_dir":     # g in; Dg, Lg out; kind, w_obj in
        return nnz * b + 4 * C + R * (8 + 2 + 4)
    if kernel == "fwd_resid":   # x in; d, l, coef out; kind, bounds, weights, moments in
        return nnz * b + 4 * C + R * (8 + 8 + 2 + 20 + 4 + 24 + 12)
    if kernel == "tr_grad":     # entries of rows with objective terms only
        return grad_entries * bt + 8 * n_obj_rows + C * (32 + 4)
    if kernel == "tr_proj":     # coefficient pair per row once; chunk sums
        return nnz * bt + 8 * R + n_tr_items * (32 + 4)
    if kernel == "col":         # chunk sums in; x, g in and out
        return n_tr_items * 4 + C * 16
    if kernel == "rows":        # d, l, Dg, Lg in; d, l, coef out; problem data in
        return R * (16 + 8 + 8 + 2 + 20 + 4 + 24 + 12)
    if kernel == "line_search":  # one window: kind, weight, targets, d, l, D g, L g per row
        return (n_obj_rows if obj_entries else R) * (2 + 12 + 16)
    if kernel in ("finalize", "active_list", "scatter", "scatter_sum"):
        return 0  # scalars; the active-row work depends on the iterate (not priced)
    raise KeyError(kernel)


def make_workload(name: str):
    from paper_2509_20012_amd import phantom as ph
    if name == "clinical":
        return ph.clinical(progress=log)
    if name == "water32":
        return ph.water32()
    if name.startswith("clinical_x"):
        return ph.clinical(scale=float(name[len("clinical_x"):]), progress=log)
    raise SystemExit(f"unknown workload {name}")


def _oracle_run(o, p, prm, n_iters: int):
    """n_iters outer iterations of the oracle from x0: seconds, the iterate and the
    mean number of step sizes tried per iteration."""
    x = p.x0.astype(np.float64)
    k, s = 0, -1
    trials = 0
    t0 = time.perf_counter()
    for _ in range(n_iters):
        x, k, s, info = o.sa_iteration(x, k, s, prm)
        trials += info["n_trials"]
    return time.perf_counter() - t0, (x, k, s), trials / max(n_iters, 1)


def cpu_baseline(p, q, n_iters: int, n_literal: int, n_single: int):
    """The FP64 oracle, as it stands, on the host cores: n_iters outer iterations with
    the closed-form step search on every thread (the reported value), then two
    variants beside it: Fig. 3's literal backtracking search (each trial step
    recomputes Eq. (2) with a full forward product) on every thread, and the
    closed form on one thread.  Matrix passes per iteration count the forward
    (D x, L x) and transposed (D^T u, L^T u) products over every row the oracle
    makes: 1 for the starting cost, per perturbation 2 for the gradient plus 2
    (closed form: direction product and new cost) or one per trial (literal), and 2
    for the feasibility sweep."""
    from oracle import Oracle, OracleParams, num_threads, set_threads
    t0 = time.perf_counter()
    o = Oracle(p, objective=q.objective)
    t_load = time.perf_counter() - t0
    cores = num_threads()
    # (with the one-sided objective the oracle's closed form falls back to the literal
    # comparison, as the identity it rests on does not hold)
    base = dict(lam=q.lam, alpha=q.alpha, eta=q.eta, reductions_n=q.reductions_n,
                normalization=q.normalization, unit_direction=q.unit_direction)
    r = q.reductions_n
    dt, state, _ = _oracle_run(o, p, OracleParams(line_search=1, **base), n_iters)
    variants = []
    if n_literal > 0:
        dl, _, trials = _oracle_run(o, p, OracleParams(line_search=0, **base), n_literal)
        variants.append({"line_search": "literal (Fig. 3 backtracking)", "cores": cores,
                         "iters_per_s": n_literal / dl, "sample": f"{n_literal} outer "
                         f"iterations from x0", "trials_per_iteration": round(trials, 2),
                         "matrix_passes_per_iteration": round(3 + r * 2 + trials, 2)})
    if n_single > 0:
        set_threads(1)
        try:
            ds, _, _ = _oracle_run(o, p, OracleParams(line_search=1, **base), n_single)
        finally:
            set_threads(cores)
        variants.append({"line_search": "closed form", "cores": 1,
                         "iters_per_s": n_single / ds,
                         "sample": f"{n_single} outer iterations from x0",
                         "matrix_passes_per_iteration": 3 + 4 * r})
    return {"value": n_iters / dt, "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_iters} outer iterations (reductions_n={r}, closed-form step "
                      f"search, {3 + 4 * r} matrix passes each) of the same workload from "
                      f"x0; oracle load (FP64 promotion + CSC) {t_load:.1f} s not timed",
            "variants": variants, "seconds": dt}, state


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def bench_batch(args):
    """48 plans iterated by batched launches, against the same plans solved one at a
    time.  batch48: uneven sizes (5k-120k rows, 200-4,000 beamlets, one draw per
    plan); scenarios48: 6 of those plans under 8 robustness scenarios each."""
    import torch
    from paper_2509_20012_amd import autotune, fredopt, phantom as ph
    t0 = time.perf_counter()
    if args.workload == "scenarios48":
        phs = ph.scenario_plans(6, seed=3)
        desc = "scenarios48: 6 water plans x 8 robustness scenarios (range +-3.5 %, +-3 mm shifts)"
    else:
        phs = [ph.small_plan(sd, r, c) for sd, r, c in ph.batch_sizes(48, seed=3)]
        desc = "batch48: 48 water plans, 5k-120k rows, 200-4000 beamlets"
    nnz = sum(p.nnz for p in phs)
    log(f"{len(phs)} plans: rows {sum(p.n_rows for p in phs)}, nnz {nnz} in "
        f"{time.perf_counter() - t0:.1f} s")
    storage = fredopt.STORAGE[args.storage]
    lanes = [0] * len(phs)
    if args.autotune:
        # the batch autotuner: the batched iteration timed at each candidate width
        t0 = time.perf_counter()
        best, rates = autotune.choose_batch_lanes(phs, storage, reductions_n=args.reductions,
                                                  gradient_reserve_pct=args.reserve)
        lanes = [best] * len(phs)
        log(f"autotuned lanes per row in {time.perf_counter() - t0:.1f} s: {best} "
            f"(plan-iterations/s by width: { {k: round(v) for k, v in rates.items()} })")
    loaded = [fredopt.load_phantom(p, storage=storage, lanes_per_row=lw,
                                   gradient_reserve_pct=args.reserve)
              for p, lw in zip(phs, lanes)]
    q = fredopt.SolverParams(reductions_n=args.reductions)
    # one at a time (the plain single-plan form, default projection path)
    k_alone = max(1, args.steps // 4)
    t_alone = 0.0
    for plan, prob, x0 in loaded:
        x = x0.clone()
        st = fredopt.new_state()
        q.iter_max = args.warmup
        fredopt.solve(plan, prob, q, st, x)
        q.iter_max = k_alone
        t_alone += _timed(lambda: fredopt.solve(plan, prob, q, st, x))
    alone_rate = len(loaded) * k_alone / t_alone
    log(f"one at a time: {alone_rate:.1f} plan-iterations/s ({k_alone} iterations per plan)")
    batch = fredopt.Batch([l[0] for l in loaded], [l[1] for l in loaded])
    xs = [l[2].clone() for l in loaded]
    states = [fredopt.new_state() for _ in loaded]
    batch.solve(q, states, xs, args.warmup)
    dt = _timed(lambda: batch.solve(q, states, xs, args.steps))
    rate = len(loaded) * args.steps / dt
    log(f"batched: {rate:.1f} plan-iterations/s ({args.steps} iterations, {dt:.3f} s)")
    return {
        "metric": METRIC, "value": round(rate, 2), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_of(args.storage),
        "data": "synthetic",
        "config": {"workload": desc, "plans": len(loaded), "nnz_total": nnz,
                   "storage": args.storage, "reductions_n": args.reductions,
                   "gradient_reserve_pct": args.reserve,
                   "lanes_per_row": f"autotuned ({lanes[0]})" if args.autotune else "rule"},
        "value_meaning": "plan-iterations per second summed over the plans",
        "one_at_a_time_iters_per_s": round(alone_rate, 2),
        "speedup_vs_one_at_a_time": round(rate / alone_rate, 3),
    }


def bench_robust(args):
    """Robustness evaluation: one fluence under the nominal plan and its 8 scenario
    recalculations (+-2 mm shifts along each axis, ranges x (1 -+ 3.5 %)), dose, LETd
    and cDL per scenario plus per-voxel bands, in one launch.  The plan is the largest
    of the batched workload (110k voxels, 3,694 beamlets)."""
    import torch
    from paper_2509_20012_amd import fredopt, phantom as ph
    t0 = time.perf_counter()
    sd, r, c = max(ph.batch_sizes(48, seed=3), key=lambda t: t[1] * t[2])
    scen = ph.robustness_scenarios(sd, r, c)
    nnz = sum(p.nnz for p in scen)
    R = scen[0].n_rows
    log(f"{len(scen)} scenarios of {R} voxels x {scen[0].n_cols} beamlets, {nnz} entries "
        f"in {time.perf_counter() - t0:.1f} s")
    storage = fredopt.STORAGE[args.storage]
    plans = [fredopt.load_matrices(p.row_ptr, p.col_idx, p.d_val, p.l_val, p.n_cols, storage)
             for p in scen]
    x = torch.from_numpy(np.random.default_rng(1).uniform(0.5, 1.5, scen[0].n_cols)
                         .astype(np.float32)).cuda()
    for _ in range(max(1, args.warmup)):
        fredopt.scenario_dose_let(plans, x, scen[0].c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fredopt.scenario_dose_let(plans, x, scen[0].c)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rate = args.steps / dt
    vb = 4 if storage == fredopt.F32 else 2
    ib = 2 if storage in (fredopt.F16_IDX16, fredopt.BF16_IDX16) else 4
    # per evaluation: every scenario's entries once, x per scenario, three outputs per
    # scenario row, and the four bands (filled, updated, decoded)
    alg = nnz * (ib + 2 * vb) + len(scen) * (4 * scen[0].n_cols + 12 * R) + 4 * 4 * R * 3
    log(f"robustness evaluation: {rate:.1f} evaluations/s ({dt / args.steps * 1e3:.3f} ms "
        f"each, host call included), {alg * rate / 1e9:.0f} GB/s of algorithmic bytes")
    for pl in plans:
        pl.free()
    return {
        "metric": METRIC, "value": round(rate, 2), "unit": "evaluations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_of(args.storage),
        "data": "synthetic",
        "config": {"workload": f"robust9: {scen[0].name} and 8 scenarios, {R} voxels, "
                               f"{nnz} entries in all", "storage": args.storage},
        "value_meaning": "robustness evaluations per second (9 scenarios: dose, LETd, cDL "
                         "and per-voxel bands), host call and synchronisation included",
        "hbm_gbps": round(alg * rate / 1e9, 1), "alg_bytes_per_evaluation": alg,
    }


def bench_sweeps(args):
    """Feasibility seeking alone, simultaneous against block-sequential: sweeps from x0
    with weights w_i (no decay), the proximity of every iterate and the time per
    sweep.  One sweep streams every row once in every form; the blocks add launches."""
    import torch
    from paper_2509_20012_amd import fredopt
    wl = args.sweep_plan
    p = make_workload(wl)
    plan, prob, x0 = fredopt.load_phantom(p)
    q = fredopt.SolverParams()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    forms = {"simultaneous": None}
    for b in (8192, 65536):
        if b < p.n_rows:
            forms[f"blocks of {b} rows"] = b
    out = {}
    for name, block in forms.items():
        x = x0.clone()
        prox = [fredopt.project_sweep(plan, prob, q, x.clone())]
        ms = 0.0
        for _ in range(args.steps):
            torch.cuda.synchronize()
            ev0.record(stream)
            if block is None:
                fredopt.project_sweep(plan, prob, q, x)
            else:
                fredopt.project_sweep_blocks(plan, prob, q, x, block)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms += ev0.elapsed_time(ev1)
            prox.append(fredopt.project_sweep(plan, prob, q, x.clone()))
        out[name] = {"ms_per_sweep": round(ms / args.steps, 4),
                     "proximity": [float(f"{v:.6g}") for v in prox]}
        log(f"{name}: {ms / args.steps:.3f} ms per sweep, proximity {prox[0]:.4g} -> "
            f"{prox[-1]:.4g}")
    sim = out["simultaneous"]
    return {
        "metric": METRIC, "value": round(1e3 / sim["ms_per_sweep"], 2), "unit": "sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 0, "ms_per_step": sim["ms_per_sweep"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"sweeps: {p.name}, {p.n_rows} x {p.n_cols}, {p.nnz} entries",
                   "weights": "w_i, no decay, convex over all constraints, lambda 1"},
        "value_meaning": "simultaneous feasibility sweeps per second (each host-synchronised)",
        "forms": out,
    }


def bench_serve(args):
    """Poisson stream of re-optimisation requests (4/s), sizes as the batched plans
    plus 10 % at clinical scale, 200-1,000 iterations each, memory budget 200 GB;
    continuous batching against first-come-first-served single-plan solves."""
    from paper_2509_20012_amd import fredopt, phantom as ph, serve
    rng = np.random.default_rng(4)
    n_req = args.requests
    arrivals = serve.poisson_trace(n_req, args.rate, seed=4)
    pool = [ph.small_plan(sd, r, c) for sd, r, c in ph.batch_sizes(48, seed=3)]
    big = ph.clinical(progress=log) if not args.serve_small_only else None
    reqs = []
    for i in range(n_req):
        p = big if (big is not None and rng.random() < 0.10) else pool[rng.integers(len(pool))]
        reqs.append(serve.Request(i, p, int(rng.integers(200, 1001)), float(arrivals[i])))
    n_big = sum(r.phantom is big for r in reqs)
    log(f"{n_req} requests over {arrivals[-1]:.1f} s ({args.rate:g}/s), {n_big} at clinical scale")
    q = fredopt.SolverParams(reductions_n=args.reductions)
    srv = serve.Server(200 * 10**9, q, quantum=args.quantum, log=log,
                       gradient_reserve_pct=args.reserve, plan_cache=args.plan_cache)
    t0 = time.perf_counter()
    done = srv.run([dataclasses.replace(r) for r in reqs])
    wall = time.perf_counter() - t0
    lat = [r.latency for r in done]
    iters = sum(r.iters for r in done)
    log(f"continuous batching: p50 {serve.percentile(lat, 50):.3f} s, p99 "
        f"{serve.percentile(lat, 99):.3f} s, {iters / wall:.1f} plan-iterations/s, "
        f"{srv.batches_built} batches, peak {srv.peak_active} resident")
    t0 = time.perf_counter()
    base = serve.serve_one_at_a_time([dataclasses.replace(r) for r in reqs], q, log=log,
                                     gradient_reserve_pct=args.reserve,
                                     plan_cache=args.plan_cache)
    wall_b = time.perf_counter() - t0
    lat_b = [r.latency for r in base]
    log(f"one at a time: p50 {serve.percentile(lat_b, 50):.3f} s, p99 "
        f"{serve.percentile(lat_b, 99):.3f} s, {iters / wall_b:.1f} plan-iterations/s")

    def breakdown(rs):
        """Latency percentiles per request class, and the mean wait for admission,
        load time and time from load to result."""
        out = {}
        for name, sel in (("clinical", lambda r: r.phantom is big),
                          ("small", lambda r: r.phantom is not big)):
            sub = [r for r in rs if sel(r)]
            if not sub:
                continue
            lt = [r.latency for r in sub]
            out[name] = {
                "requests": len(sub),
                "latency_p50_s": round(serve.percentile(lt, 50), 4),
                "latency_p99_s": round(serve.percentile(lt, 99), 4),
                "latency_max_s": round(max(lt), 4),
                "mean_admit_wait_s": round(float(np.mean([r.admitted - r.arrival for r in sub])), 4),
                "mean_load_s": round(float(np.mean([r.loaded - r.admitted for r in sub])), 4),
                "mean_solve_s": round(float(np.mean([r.finished - r.loaded for r in sub])), 4),
            }
        return out

    by_b, by_o = breakdown(done), breakdown(base)
    for name in by_b:
        log(f"  {name}: batching {by_b[name]}")
        log(f"  {name}: one at a time {by_o[name]}")
    return {
        "metric": METRIC, "value": round(iters / wall, 2), "unit": "iters/s", "n_gpus": 1,
        "steps": iters, "warmup": 0, "ms_per_step": round(wall / iters * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serve: {n_req} Poisson requests at {args.rate:g}/s, {n_big} at "
                               f"clinical scale, 200-1000 iterations, 200 GB budget",
                   "quantum": args.quantum, "reductions_n": args.reductions,
                   "plan_cache": args.plan_cache},
        "value_meaning": "plan-iterations per second over the whole trace (wall clock)",
        "latency_p50_s": round(serve.percentile(lat, 50), 4),
        "latency_p99_s": round(serve.percentile(lat, 99), 4),
        "by_class": by_b,
        "one_at_a_time": {"latency_p50_s": round(serve.percentile(lat_b, 50), 4),
                          "latency_p99_s": round(serve.percentile(lat_b, 99), 4),
                          "iters_per_s": round(iters / wall_b, 2),
                          "by_class": by_o},
        "peak_resident_plans": srv.peak_active, "batches_built": srv.batches_built,
        "plan_cache_hits": srv.cache_hits,
    }


def bench_small_plan(args, steps: int = 1000, warmup: int = 50):
    """The 32^3 water plan (400 beamlets): small enough to stay in cache, so its rate
    is set by launch and synchronisation latency.  Steady-state iterations/s after
    warm-up, and its 100-iteration solve from x0."""
    import torch
    from paper_2509_20012_amd import fredopt, phantom as ph
    p = ph.water32()
    plan, prob, x0 = fredopt.load_phantom(p)
    q = fredopt.SolverParams(reductions_n=args.reductions, iter_max=warmup)
    x = x0.clone()
    st = fredopt.new_state()
    fredopt.solve(plan, prob, q, st, x)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    q.iter_max = steps
    torch.cuda.synchronize()
    ev0.record(stream)
    fredopt.solve(plan, prob, q, st, x)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    n_full = int(p.meta.get("iterations", 100))
    q.iter_max = n_full
    xf = x0.clone()
    sf = fredopt.new_state()
    torch.cuda.synchronize()
    ev0.record(stream)
    fredopt.solve(plan, prob, q, sf, xf)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_full = ev0.elapsed_time(ev1)
    plan.free()
    log(f"water32: {steps / ms * 1e3:.1f} it/s steady, {n_full} from x0 in {ms_full:.2f} ms")
    return {"workload": f"water32: {p.name}, {p.n_rows} x {p.n_cols}, {p.nnz} entries",
            "iters_per_s": round(steps / ms * 1e3, 1), "ms_per_step": round(ms / steps, 5),
            "steps": steps, "warmup": warmup,
            "full_solve": {"iterations": n_full, "ms": round(ms_full, 3),
                           "iters_per_s": round(n_full / ms_full * 1e3, 1)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="clinical",
                    help="clinical (160x160x120 grid, 12k beamlets), water32 (32^3, 400 "
                         "beamlets), clinical_x<scale>, batch48 (48 plans in batched "
                         "launches), scenarios48 (6 plans x 8 robustness scenarios), "
                         "robust9 (robustness evaluation of one fluence under 9 "
                         "scenarios), sweeps (simultaneous against block-sequential "
                         "feasibility sweeps) or serve (request stream, continuous "
                         "batching)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "f16i16", "bf16i16"],
                    help="matrix values in FP32, FP16 or BF16 (per-beamlet FP32 scale); the "
                         "i16 forms also keep column indices in 16 bits")
    ap.add_argument("--reductions", type=int, default=1)
    ap.add_argument("--problem", default="full", choices=["full", "dose_only"],
                    help="full: dose and LETd terms; dose_only: the paper's dose-only arm "
                         "(dose bounds and the PTV dose objective only)")
    ap.add_argument("--objective", type=int, default=0, choices=[0, 1],
                    help="0 Eq. (2) as printed, 1 the OAR term one-sided (device step search)")
    ap.add_argument("--unit-direction", type=int, default=0, choices=[0, 1],
                    help="1 perturbs along the normalised gradient")
    ap.add_argument("--reserve", type=int, default=None,
                    help="gradient reserve of each plan in %% of its CSC (batch and serve "
                         "workloads: 100, so that every plan has the objective-row view; "
                         "0 library default)")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=100)
    ap.add_argument("--cpu-literal-iters", type=int, default=10,
                    help="cpu baseline: iterations with the literal step search")
    ap.add_argument("--cpu-single-iters", type=int, default=5,
                    help="cpu baseline: iterations on one host thread")
    ap.add_argument("--full-solve", type=int, default=None,
                    help="iterations of the whole-trajectory solve from x0 (default: the "
                         "workload's iteration count; 0 skips it)")
    ap.add_argument("--no-config0", action="store_true",
                    help="skip the 32^3 water plan's rate in the clinical line")
    ap.add_argument("--profile-iters", type=int, default=5)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for PMC scaling)")
    ap.add_argument("--sweep-plan", default="clinical",
                    help="sweeps: the plan (clinical or water32)")
    ap.add_argument("--requests", type=int, default=120, help="serve: trace length")
    ap.add_argument("--quantum", type=int, default=50, help="serve: iterations per round")
    ap.add_argument("--rate", type=float, default=4.0, help="serve: requests per second")
    ap.add_argument("--plan-cache", action="store_true",
                    help="serve: plans stay resident between requests of the same plan "
                         "(both forms)")
    ap.add_argument("--serve-small-only", action="store_true",
                    help="serve: no clinical-scale requests")
    args = ap.parse_args()
    if args.reserve is None:
        args.reserve = 100 if args.workload in ("batch48", "scenarios48", "serve") else 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a plan would "
              "be split by rows across GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_20012_amd import fredopt

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    torch.cuda.set_device(0)
    fredopt.lib()
    if args.workload in ("batch48", "scenarios48", "serve", "robust9", "sweeps"):
        if args.workload == "serve":
            res = bench_serve(args)
        elif args.workload == "sweeps":
            res = bench_sweeps(args)
        elif args.workload == "robust9":
            res = bench_robust(args)
        else:
            res = bench_batch(args)
        res["device"] = device_info()
        print(json.dumps(res), flush=True)
        return
    log(f"generating workload {args.workload}")
    t0 = time.perf_counter()
    p = make_workload(args.workload)
    if args.problem == "dose_only":
        p = p.dose_only()
    log(f"workload {p.summary()} in {time.perf_counter() - t0:.1f} s")

    storage = fredopt.STORAGE[args.storage]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan, prob, x0 = fredopt.load_phantom(p, storage=storage)
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t0
    log(f"loaded in {t_load:.2f} s: {plan.info()}")
    if args.autotune:
        info = fredopt.autotune(plan, x0)
        log(f"autotuned: lanes {info['lanes_per_row']} chunk {info['tr_chunk']}")
    info = plan.info()

    q = fredopt.SolverParams(reductions_n=args.reductions, iter_max=args.warmup,
                             objective=args.objective, unit_direction=args.unit_direction)
    x = x0.clone()
    st = fredopt.new_state()
    if args.warmup:
        fredopt.solve(plan, prob, q, st, x)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} iterations done (k={st.k}, s={st.s})")

    q.iter_max = args.steps
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    fredopt.solve(plan, prob, q, st, x)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    its = 1000.0 / ms_per_step
    log(f"timed {args.steps} iterations: {ms_per_step:.4f} ms/iter ({its:.1f} it/s), "
        f"wall {wall:.3f} s, state k={st.k} s={st.s} cost={st.cost:.6g} prox={st.proximity:.3g} "
        f"violated={st.n_violated}")

    # per-kernel durations with HIP events on the launch stream
    xp = x.clone()
    sp = fredopt.State()
    sp.k, sp.s = st.k, st.s
    prof = fredopt.profile_kernels(plan, prob, q, sp, xp, args.profile_iters)
    info = plan.info()
    from paper_2509_20012_amd import phantom as ph_mod
    n_obj_rows = int(np.count_nonzero(p.kind & (ph_mod.OBJ_DOSE | ph_mod.OBJ_CDL)))
    R, C, nnz = p.n_rows, p.n_cols, p.nnz
    vb = 4 if storage == fredopt.F32 else 2
    ib = 2 if storage in (fredopt.F16_IDX16, fredopt.BF16_IDX16) else 4
    per_kernel = {}
    scatter_path = sp.projection_path == 1
    log(f"projection: {'active rows' if scatter_path else 'column-major'}, "
        f"{sp.n_active} active rows")
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        ab = algorithmic_bytes(name, R, C, nnz, vb, info["tr_items"], info["grad_entries"],
                               n_obj_rows, info["obj_entries"], ib)
        if name == "tr_proj" and scatter_path:
            ab = 0  # its workgroups see the active-row path and return at once
        if name == "scatter":
            # one launch takes the path the device chose: the active rows' stored
            # entries (counted on the device by the residual pass that listed them)
            # and their 32-byte list records, or the column-major pass
            ab = (int(sp.active_entries * (ib + 2 * vb) + 32 * sp.n_active) if scatter_path
                  else algorithmic_bytes("tr_proj", R, C, nnz, vb, info["tr_items"],
                                         info["grad_entries"], n_obj_rows,
                                         info["obj_entries"], ib))
        per_kernel[name] = {"ms": ms, "launches_per_iter": cnt / args.profile_iters,
                            "alg_bytes": ab, "gbps": ab / (ms * 1e-3) / 1e9 if ms > 0 else 0.0}
    dom = max((k for k in per_kernel if per_kernel[k]["alg_bytes"] > 0),
              key=lambda k: per_kernel[k]["ms"] * per_kernel[k]["launches_per_iter"])
    b_iter = sum(v["alg_bytes"] * v["launches_per_iter"] for v in per_kernel.values())
    log("kernels: " + ", ".join(f"{k} {v['ms']:.4f} ms {v['gbps']:.0f} GB/s"
                                for k, v in per_kernel.items()))
    log(f"plan: {info}")

    traffic = None
    src_hash = kernel_source_hash()
    tpath = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if os.path.exists(tpath):
        try:
            with open(tpath) as fh:
                tr = json.load(fh)
            ent = tr.get(args.workload, {}).get(args.storage, {}).get(dom)
            if ent and ent.get("kernel_source_hash") == src_hash:
                traffic = ent["bytes_per_launch"]
        except (OSError, ValueError, KeyError):
            traffic = None

    if args.copy_calibration:
        n = 256 * 1024 * 1024
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {n} bytes")

    roofline = {"bound": "hbm", "kernel": dom,
                "symbol": KERNEL_SYMBOLS[dom].format(vt=storage, sub=info["schedule"]),
                "achieved": round(per_kernel[dom]["gbps"], 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(per_kernel[dom]["gbps"] / HBM_PEAK_GBPS, 4),
                "traffic": traffic,
                "alg_bytes_per_launch": per_kernel[dom]["alg_bytes"],
                "ms_per_launch": round(per_kernel[dom]["ms"], 5)}

    result = {
        "metric": METRIC, "value": round(its, 3), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_of(args.storage),
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {p.name}", "rows": R, "cols": C, "nnz": nnz,
                   "storage": args.storage, "reductions_n": args.reductions,
                   "problem": args.problem, "normalization": "convex_all",
                   "objective": "one-sided OAR" if args.objective else "Eq. (2) as printed",
                   "unit_direction": args.unit_direction,
                   "lanes_per_row": info["lanes_per_row"],
                   "tr_chunk": info["tr_chunk"]},
        "hbm_gbps_iteration": round(b_iter * its / 1e9, 1),
        "hbm_frac_iteration": round(b_iter * its / 1e9 / HBM_PEAK_GBPS, 4),
        "alg_bytes_per_iteration": b_iter,
        "roofline": roofline,
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in per_kernel.items()},
        "load_seconds": round(t_load, 3),
        "kernel_source_hash": src_hash,
        "paper_context": "Table 2 stage (iv): 200 SA iterations in 2091 s / 1508 s "
                         "(0.096 / 0.133 it/s) on an NVIDIA P100, private patient matrices",
    }
    # the whole trajectory: the workload's full iteration count from x0 (the timed
    # window above samples iterations warmup+1 .. warmup+steps)
    n_full = args.full_solve if args.full_solve is not None else int(p.meta.get("iterations", 0))
    if n_full > 0:
        qf = fredopt.SolverParams(reductions_n=args.reductions, iter_max=n_full,
                                  objective=args.objective, unit_direction=args.unit_direction)
        xf = x0.clone()
        sf = fredopt.new_state()
        torch.cuda.synchronize()
        ev0.record(stream)
        fredopt.solve(plan, prob, qf, sf, xf)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_full = ev0.elapsed_time(ev1)
        result["full_solve"] = {"iterations": n_full, "from": "x0", "ms": round(ms_full, 3),
                                "iters_per_s": round(n_full / ms_full * 1e3, 2),
                                "final": {"k": sf.k, "s": sf.s, "violated": sf.n_violated,
                                          "active_rows": sf.n_active,
                                          "projection_path": sf.projection_path}}
        log(f"full solve: {n_full} iterations from x0 in {ms_full:.1f} ms "
            f"({n_full / ms_full * 1e3:.1f} it/s)")
    if args.workload == "clinical" and not args.no_config0:
        result["config0"] = bench_small_plan(args)
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_iters} iterations (+ {args.cpu_literal_iters} "
            f"literal, {args.cpu_single_iters} on one thread)")
        cb, _ = cpu_baseline(p, q, args.cpu_iters, args.cpu_literal_iters,
                             args.cpu_single_iters)
        log(f"cpu baseline {cb['value']:.4f} it/s on {cb['cores']} threads ({cb['seconds']:.1f} s); "
            f"variants {cb['variants']}")
        cb.pop("seconds")
        result["cpu_baseline"] = cb
    result["device"] = device_info()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
