"""Serving loop for re-optimisation requests (host logic over the fredopt C ABI).

Requests (a plan's influence matrices and problem, an iteration count, an arrival
time) are admitted while the device memory they need fits a budget; admitted plans
stay resident and are iterated together by batched launches (fredopt_batch_*):
continuous batching, where the batch is rebuilt whenever a request joins or
leaves, between quanta of outer iterations.  A lane with a single active request
runs the plain single-plan solve instead (no batch to build).  Loads run on a
loader thread per lane, on a stream of their own: the lane keeps iterating its
resident plans while the next plan's matrices are copied and laid out, and a
request joins the batch when its load has completed.  A request's latency runs from
its arrival to its result (the fluence) being on the host, and includes the load.

With plan_cache, a finished request's plan stays resident (its bytes still counted
in the budget) for the next request of the same plan, a re-optimisation of the same
patient's matrices: that request starts without a load, and idle plans are freed,
least recently used first, when an admission needs their room.

Every batched iteration of a plan equals its single-plan iteration bit for bit,
and quanta resume exactly, so a request's result does not depend on what else was
served with it.

The comparison form ("one at a time") serves the same trace first come, first
served, each request solved alone with the plain single-plan call.
"""
from __future__ import annotations

import collections
import dataclasses
import queue as _queue
import threading
import time
from typing import Callable, List, Optional

import numpy as np

from . import fredopt


@dataclasses.dataclass
class Request:
    rid: int
    phantom: object            # phantom.Phantom
    iters: int
    arrival: float             # seconds after the start of the trace
    admitted: Optional[float] = None
    loaded: Optional[float] = None     # load complete (matrices resident)
    finished: Optional[float] = None
    x: Optional[np.ndarray] = None
    k: int = 0
    s: int = -1

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def plan_bytes(ph, storage: int = fredopt.F32, gradient_reserve_pct: int = 0) -> int:
    """Device bytes a request holds while resident: the plan workspace, the input
    CSR copies used during the load, the problem arrays and the fluence."""
    ws = fredopt.workspace_bytes_csr(ph.row_ptr, ph.n_cols, storage, 0, gradient_reserve_pct)
    csr = ph.row_ptr.nbytes + ph.col_idx.nbytes + ph.d_val.nbytes + ph.l_val.nbytes
    return int(ws + csr + ph.n_rows * 38 + ph.n_cols * 4)


class _Active:
    def __init__(self, req: Request, storage: int, reserve: int, keep_x0: bool = False):
        self.req = req
        self.plan, self.prob, self.x = fredopt.load_phantom(req.phantom, storage=storage,
                                                            gradient_reserve_pct=reserve)
        # the starting fluence, kept for the next request of the plan when plans stay
        self.x0 = self.x.clone() if keep_x0 else None
        self.state = fredopt.new_state()
        self.left = req.iters
        self.bytes = plan_bytes(req.phantom, storage, reserve)
        self.loaded: Optional[float] = None

    @classmethod
    def reuse(cls, req: Request, kept: "_Kept", at: float) -> "_Active":
        """A request served by a resident plan: no load, a fresh state and x0."""
        a = cls.__new__(cls)
        a.req = req
        a.plan, a.prob, a.x0, a.bytes = kept.plan, kept.prob, kept.x0, kept.bytes
        a.x = kept.x0.clone()
        a.state = fredopt.new_state()
        a.left = req.iters
        a.loaded = at
        return a


@dataclasses.dataclass
class _Kept:
    plan: object
    prob: object
    x0: object
    bytes: int
    phantom: object   # keeps the key's object alive while the plan stays


class _Resident:
    """Plans kept on the device after their request finished, by phantom (one
    patient's matrices and problem), for the next request of the same plan.  Idle
    plans only: a plan in use by a request is not here.  Phantoms are ordered by
    their latest use (a plan kept or taken); eviction frees the oldest kept plan of
    the least recently used phantom.  The caller holds the serving lock around every
    call."""

    def __init__(self):
        self.idle: "collections.OrderedDict[int, List[_Kept]]" = collections.OrderedDict()
        self.hits = 0
        self.evictions = 0

    def take(self, phantom) -> Optional[_Kept]:
        got = self.idle.get(id(phantom))
        if not got:
            return None
        k = got.pop()
        if got:
            self.idle.move_to_end(id(phantom))   # a use: the phantom is the newest
        else:
            del self.idle[id(phantom)]
        self.hits += 1
        return k

    def put(self, a: _Active):
        self.idle.setdefault(id(a.req.phantom), []).append(
            _Kept(a.plan, a.prob, a.x0, a.bytes, a.req.phantom))
        self.idle.move_to_end(id(a.req.phantom))

    def evict(self, counted: bool = True) -> int:
        """Frees the least recently kept idle plan; its bytes (0 if none is idle)."""
        if not self.idle:
            return 0
        key, lst = next(iter(self.idle.items()))
        k = lst.pop(0)
        if not lst:
            del self.idle[key]
        k.plan.free()
        if counted:
            self.evictions += 1
        return k.bytes

    def clear(self) -> int:
        """Frees every kept plan (not counted as evictions); their bytes."""
        freed = 0
        while self.idle:
            freed += self.evict(counted=False)
        return freed


class _Loader:
    """Loads admitted requests in order on a host thread with its own stream.  A load
    is handed over only after its stream has drained, so the lane's stream sees
    complete matrices without any cross-stream event.  An exception in a load is
    handed over in place of the request and raised by the lane."""

    def __init__(self, storage: int, reserve: int, now: Callable[[], float],
                 keep_x0: bool = False):
        self.storage, self.reserve, self.now, self.keep_x0 = storage, reserve, now, keep_x0
        self.inbox: _queue.Queue = _queue.Queue()
        self.ready: _queue.Queue = _queue.Queue()
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def _run(self):
        import torch
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            while True:
                req = self.inbox.get()
                if req is None:
                    return
                try:
                    a = _Active(req, self.storage, self.reserve, self.keep_x0)
                    stream.synchronize()
                    a.loaded = self.now()
                    self.ready.put(a)
                except BaseException as e:  # raised by the lane that asked for it
                    self.ready.put(e)

    def submit(self, req: Request):
        self.inbox.put(req)

    def take(self, timeout: Optional[float]):
        """The next finished load, or None when none finishes within timeout
        (0: do not wait)."""
        try:
            got = self.ready.get(block=timeout != 0, timeout=timeout or None)
        except _queue.Empty:
            return None
        if isinstance(got, BaseException):
            raise got
        return got

    def close(self):
        self.inbox.put(None)
        self.thread.join()


class Server:
    """Continuous batching under a device-memory budget.

    Requests are split into lanes by size (plans above `big_nnz` entries form their
    own lane): each lane is a host thread with its own stream and its own batch, so
    the small plans' launch-bound iterations overlap on the device with the large
    plans' bandwidth-bound passes instead of waiting for them.  Within a lane,
    requests are admitted in arrival order while the shared budget allows."""

    def __init__(self, budget_bytes: int, params: fredopt.SolverParams, quantum: int = 50,
                 storage: int = fredopt.F32, big_nnz: int = 20_000_000,
                 log: Optional[Callable[[str], None]] = None, gradient_reserve_pct: int = 0,
                 plan_cache: bool = False):
        fredopt.lib()
        self.reserve = int(gradient_reserve_pct)   # per plan, % of its CSC (0 default)
        self.plan_cache = bool(plan_cache)
        self.resident = _Resident()
        self.budget = int(budget_bytes)
        self.params = params
        self.quantum = int(quantum)
        self.storage = storage
        self.big_nnz = int(big_nnz)
        self.log = log or (lambda m: None)
        self.progress_every = 100   # a log line every this many finished requests
        self.batches_built = 0
        self.solo_quanta = 0        # quanta run by a lane's single active request
        self.peak_active = 0
        self.peak_bytes = 0

    @property
    def cache_hits(self) -> int:
        return self.resident.hits

    def run(self, requests: List[Request]) -> List[Request]:
        queue = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in queue:
            if plan_bytes(r.phantom, self.storage, self.reserve) > self.budget:
                raise ValueError(f"request {r.rid} alone exceeds the memory budget")
        lanes = [[r for r in queue if r.phantom.nnz <= self.big_nnz],
                 [r for r in queue if r.phantom.nnz > self.big_nnz]]
        lock = threading.Lock()
        state = {"used": 0, "active": 0}
        done: List[Request] = []
        errors: List[BaseException] = []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731

        def lane_loop(reqs: List[Request]):
            import torch
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                self._lane(reqs, lock, state, done, now)

        def guarded(reqs):
            try:
                lane_loop(reqs)
            except BaseException as e:  # surfaced after the join
                errors.append(e)

        threads = [threading.Thread(target=guarded, args=(l,)) for l in lanes if l]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        state["used"] -= self.resident.clear()   # resident plans end with the run
        if errors:
            raise errors[0]
        return sorted(done, key=lambda r: r.rid)

    def _lane(self, queue, lock, state, done, now):
        loader = _Loader(self.storage, self.reserve, now, keep_x0=self.plan_cache)
        try:
            self._lane_loop(queue, lock, state, done, now, loader)
        finally:
            loader.close()

    def _lane_loop(self, queue, lock, state, done, now, loader):
        import torch
        params = dataclasses.replace(self.params)
        active: List[_Active] = []
        batch = None
        qi = 0
        loading = 0     # admitted requests whose load has not been handed over yet
        while qi < len(queue) or active or loading:
            changed = False
            # admission: arrival order, while the shared budget allows; the memory
            # is counted from the moment the load starts.  A request whose plan is
            # resident and idle takes it and joins at once; otherwise idle resident
            # plans make room, least recently used first
            while qi < len(queue) and queue[qi].arrival <= now():
                req = queue[qi]
                need = plan_bytes(req.phantom, self.storage, self.reserve)
                with lock:
                    kept = self.resident.take(req.phantom) if self.plan_cache else None
                    if kept is None:
                        while state["used"] + need > self.budget:
                            freed = self.resident.evict()
                            if freed == 0:
                                break
                            state["used"] -= freed
                        if state["used"] + need > self.budget:
                            break
                        state["used"] += need
                    state["active"] += 1
                    self.peak_bytes = max(self.peak_bytes, state["used"])
                    self.peak_active = max(self.peak_active, state["active"])
                qi += 1
                req.admitted = now()
                if kept is not None:
                    active.append(_Active.reuse(req, kept, req.admitted))
                    changed = True
                else:
                    loader.submit(req)
                    loading += 1
            # completed loads join; with nothing resident, wait for one (or for the
            # next arrival)
            wait = 0.0
            if not active:
                nxt = queue[qi].arrival - now() if qi < len(queue) else 0.05
                wait = min(max(nxt, 0.0005), 0.05) if loading else None
            if wait is None:  # nothing resident or loading: sleep to the next arrival
                nxt = queue[qi].arrival - now() if qi < len(queue) else 0.0
                time.sleep(nxt if nxt > 0 else 0.001)  # next arrival, or budget freed
                continue
            while loading:
                a = loader.take(wait)
                if a is None:
                    break
                active.append(a)
                loading -= 1
                changed = True
                wait = 0.0
            if not active:
                continue
            n = min(self.quantum, min(a.left for a in active))
            if len(active) == 1:
                # alone in its lane: the plain single-plan solve (its own cached graph);
                # it resumes from the same state, so the iterates are those of a batch
                if batch is not None:
                    batch.free()
                    batch = None
                a = active[0]
                params.iter_max = n
                fredopt.solve(a.plan, a.prob, params, a.state, a.x)
                with lock:
                    self.solo_quanta += 1
            else:
                if changed or batch is None:
                    if batch is not None:
                        batch.free()
                    batch = fredopt.Batch([a.plan for a in active], [a.prob for a in active])
                    with lock:
                        self.batches_built += 1
                batch.solve(params, [a.state for a in active], [a.x for a in active], n)
            for a in active:
                a.left -= n
            finished = [a for a in active if a.left == 0]
            if finished:
                for a in finished:
                    req = a.req
                    req.x = a.x.cpu().numpy()
                    req.k, req.s = a.state.k, a.state.s
                    req.finished = now()
                    req.loaded = a.loaded
                # every launch that reads the finished plans has completed before
                # their memory goes back to the allocator
                torch.cuda.current_stream().synchronize()
                if batch is not None:
                    batch.free()
                    batch = None
                active = [a for a in active if a.left > 0]
                if not self.plan_cache:
                    for a in finished:
                        a.plan.free()
                with lock:
                    for a in finished:
                        done.append(a.req)
                        if self.plan_cache:
                            self.resident.put(a)   # its bytes stay counted
                        else:
                            state["used"] -= a.bytes
                        state["active"] -= 1
                        if len(done) % self.progress_every == 0:
                            self.log(f"served {len(done)} requests")
                del finished
        if batch is not None:
            batch.free()


def serve_one_at_a_time(requests: List[Request], params: fredopt.SolverParams,
                        storage: int = fredopt.F32,
                        log: Optional[Callable[[str], None]] = None,
                        gradient_reserve_pct: int = 0,
                        plan_cache: bool = False) -> List[Request]:
    """First come, first served; each request solved alone by fredopt_solve.  With
    plan_cache, plans stay resident between requests of the same plan (no budget)."""
    import torch
    params = dataclasses.replace(params)   # iter_max is set per request on this copy
    queue = sorted(requests, key=lambda r: (r.arrival, r.rid))
    kept = {}
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0  # noqa: E731
    for i, req in enumerate(queue):
        wait = req.arrival - now()
        if wait > 0:
            time.sleep(wait)
        req.admitted = now()
        if plan_cache and id(req.phantom) in kept:
            plan, prob, x0, _ = kept[id(req.phantom)]
            x = x0.clone()
        else:
            plan, prob, x = fredopt.load_phantom(req.phantom, storage=storage,
                                                 gradient_reserve_pct=gradient_reserve_pct)
            if plan_cache:
                kept[id(req.phantom)] = (plan, prob, x.clone(), req.phantom)
        torch.cuda.current_stream().synchronize()
        req.loaded = now()
        st = fredopt.new_state()
        params.iter_max = req.iters
        fredopt.solve(plan, prob, params, st, x)
        req.x = x.cpu().numpy()
        req.k, req.s = st.k, st.s
        req.finished = now()
        if not plan_cache:
            plan.free()
        if log and (i + 1) % 100 == 0:
            log(f"served {i + 1} requests one at a time")
    for plan, _, _, _ in kept.values():
        plan.free()
    return queue


def percentile(values, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = np.sort(np.asarray(values, np.float64))
    if v.size == 0:
        return float("nan")
    rank = max(1, int(np.ceil(q / 100.0 * v.size)))
    return float(v[rank - 1])


def poisson_trace(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of n requests of a Poisson process of the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
