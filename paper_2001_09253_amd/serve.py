"""Open-loop replay of a request trace through the request API.

A submitter thread calls solve_submit at each request's scheduled arrival
time; a request submitted late is charged for it, since latency runs from the
scheduled arrival.  A reaper thread waits for the tickets in order and reads
the completion time the library stamps once the result is in the caller's
buffer (solve_ticket_info), then reaps the ticket (solve_poll).  Results go to
a ring of caller-owned host buffers; a buffer is reused only after the
request that held it has completed.

With plain=True the same trace runs through SOLVE_PLAIN contexts (one request
per synchronous launch sequence), the single-instance comparison path.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import api, workloads


@dataclass
class Request:
    x: np.ndarray
    y: np.ndarray
    sd: float
    ed: float
    m: int

    @property
    def n(self) -> int:
        return len(self.x)


@dataclass
class ReplayResult:
    latency_s: np.ndarray          # per measured request, scheduled arrival -> result delivered
    submit_lag_s: np.ndarray       # per measured request, scheduled arrival -> submit call
    steps: int                     # sum of n + m over measured requests
    window_s: float                # first measured arrival -> last measured completion
    requests: int
    errors: int
    stats: dict = field(default_factory=dict)
    sizes: np.ndarray = field(default_factory=lambda: np.zeros(0))  # per measured request, n + m

    def summary(self) -> dict:
        lat = self.latency_s * 1e3
        return {"requests": self.requests, "errors": self.errors,
                "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
                "mean_ms": float(lat.mean()) if len(lat) else None,
                "max_ms": float(lat.max()) if len(lat) else None,
                "submit_lag_p99_ms": float(np.percentile(self.submit_lag_s * 1e3, 99)) if len(lat) else None,
                "steps_per_s": self.steps / self.window_s if self.window_s > 0 else None,
                "requests_per_s": self.requests / self.window_s if self.window_s > 0 else None}


def make_requests(trace: workloads.Trace, seed: int) -> list[Request]:
    """Inputs of every request of the trace, drawn once up front (the
    paper's generator; the ends cycle natural / flat / twist)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(len(trace.t)):
        x, y = workloads.paper_curve(rng, int(trace.n[r]))
        _, sd, ed = workloads.bc_for(r)
        out.append(Request(x, y, sd, ed, int(trace.m[r])))
    return out


def _sleep_until(clock, target):
    while True:
        d = target - clock()
        if d <= 0:
            return
        if d > 2e-4:
            time.sleep(d - 1e-4)


def replay(trace: workloads.Trace, reqs: list[Request], *, plain: bool = False, budget: int = 200 << 30,
           max_slots: int = 65536, max_inflight: int = 2, flags: int = 0, warmup_s: float = 0.0,
           pool: int = 512, keep_outputs: bool = False, device: int = 0, pinned: bool = True):
    """Run the trace; returns (ReplayResult, outputs or None).  outputs[r] is
    request r's result copy when keep_outputs.  pinned: the result buffers are
    pinned host memory (the device writes them directly), else pageable."""
    count = len(reqs)
    mmax = max((q.m for q in reqs), default=1)
    pool = max(1, min(pool, count))
    if pinned:
        import torch
        bufs = [torch.empty(mmax, dtype=torch.float64, pin_memory=True).numpy() for _ in range(pool)]
    else:
        bufs = [np.empty(mmax, dtype=np.float64) for _ in range(pool)]
    ctx = api.solve_create(device=device, hbm_budget_bytes=budget, max_slots=max_slots,
                           flags=flags | (api.PLAIN if plain else 0), max_inflight=max_inflight)
    tickets = [None] * count
    sub_t = np.zeros(count)
    done_t = np.zeros(count)
    codes = np.zeros(count, dtype=np.int64)
    status = np.zeros(count, dtype=np.int64)
    outputs = [None] * count if keep_outputs else None
    slot_free = [threading.Event() for _ in range(pool)]
    for e in slot_free:
        e.set()
    posted = threading.Semaphore(0)
    failure = []
    clock = api.solve_clock
    t0 = clock() + 0.05

    def submitter():
        try:
            for r, q in enumerate(reqs):
                b = r % pool
                slot_free[b].wait()
                slot_free[b].clear()
                _sleep_until(clock, t0 + trace.t[r])
                sub_t[r] = clock()
                tickets[r] = api.solve_submit(ctx, q.x, q.y, q.sd, q.ed, None, q.m, bufs[b][:q.m])
                posted.release()
        except Exception as e:  # surfaced by the caller
            failure.append(e)
            posted.release()

    def reaper():
        try:
            for r in range(count):
                posted.acquire()
                if failure:
                    return
                t = tickets[r]
                st = api.solve_wait(ctx, t)
                times, code = api.solve_ticket_info(ctx, t)
                done_t[r] = times[3]
                codes[r] = code
                status[r] = api.solve_poll(ctx, t)
                if keep_outputs:
                    outputs[r] = bufs[r % pool][:reqs[r].m].copy()
                slot_free[r % pool].set()
                assert st != api.PENDING
        except Exception as e:
            failure.append(e)
            for ev in slot_free:
                ev.set()

    th = [threading.Thread(target=submitter, daemon=True), threading.Thread(target=reaper, daemon=True)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    stats = api.solve_stats(ctx)
    stats.update(api.solve_memory(ctx))
    api.solve_destroy(ctx)
    if failure:
        raise failure[0]
    arrive = t0 + trace.t[:count]
    sel = trace.t[:count] >= warmup_s
    lat = (done_t - arrive)[sel]
    lag = (sub_t - arrive)[sel]
    steps = int(sum(reqs[r].n + reqs[r].m for r in np.nonzero(sel)[0]))
    window = float(done_t[sel].max() - arrive[sel].min()) if sel.any() else 0.0
    errors = int(np.sum(status[sel] != api.DONE))
    sizes = np.array([reqs[r].n + reqs[r].m for r in np.nonzero(sel)[0]], dtype=np.float64)
    res = ReplayResult(lat, lag, steps, window, int(sel.sum()), errors, stats, sizes)
    return res, outputs
