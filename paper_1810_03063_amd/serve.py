"""Request loop of the serving form: continuous batching of endgame solves.

Requests arrive over time (a trace of arrival times and instances).  The loop
admits waiting requests in arrival order while the batch engine accepts them
(device-memory budget and free slots), advances every live solve with one
engine tick at a time, retires finished solves as soon as they complete and
admits new requests into the freed memory.  Latency is completion minus
arrival.  The sequential baseline serves the same trace one request at a
time, first come first served.

The engine is any object with admit(request) -> slot | None, tick(),
poll(slot) -> None | (status, result), retire(slot) and live(); LibEngine
drives the library's egt_batch_* interface, and tests drive the loop with a
CPU stand-in.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the run
    payload: object  # instance (or anything the engine understands)
    admitted: float = float("nan")
    done: float = float("nan")
    status: str = ""
    result: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def summarize(reqs, wall):
    lat = [r.latency for r in reqs]
    return dict(
        requests=len(reqs),
        solves_per_sec=len(reqs) / wall if wall > 0 else float("nan"),
        p50_ms=percentile(lat, 50) * 1e3,
        p99_ms=percentile(lat, 99) * 1e3,
        mean_ms=sum(lat) / len(lat) * 1e3 if lat else float("nan"),
        wall_s=wall,
        converged=sum(1 for r in reqs if r.status == "EGT_OK"),
    )


def serve(engine, requests, clock=time.perf_counter, sleep=time.sleep, max_idle=None):
    """Continuous batching of `requests` (sorted by arrival) on `engine`.
    Returns (requests with times and results filled in, wall seconds)."""
    pending = sorted(requests, key=lambda r: r.arrival)
    waiting = []
    live = {}  # slot -> request
    t0 = clock()
    i = 0
    finished = []
    while len(finished) < len(requests):
        now = clock() - t0
        while i < len(pending) and pending[i].arrival <= now:
            waiting.append(pending[i])
            i += 1
        while waiting:
            slot = engine.admit(waiting[0])
            if slot is None:
                break
            r = waiting.pop(0)
            r.admitted = clock() - t0
            live[slot] = r
        if not live:
            if i < len(pending):
                wait = pending[i].arrival - (clock() - t0)
                if wait > 0:
                    sleep(min(wait, max_idle) if max_idle else wait)
                continue
            if waiting:
                raise RuntimeError("a request can never be admitted (larger than the whole budget)")
        engine.tick()
        for slot in list(live):
            out = engine.poll(slot)
            if out is None:
                continue
            r = live.pop(slot)
            r.status, r.result = out
            r.done = clock() - t0
            engine.retire(slot)
            finished.append(r)
    return requests, clock() - t0


def serve_sequential(solve_one, requests, clock=time.perf_counter, sleep=time.sleep):
    """First come, first served, one request at a time: solve_one(request) ->
    (status, result)."""
    t0 = clock()
    for r in sorted(requests, key=lambda q: q.arrival):
        now = clock() - t0
        if r.arrival > now:
            sleep(r.arrival - now)
        r.admitted = clock() - t0
        r.status, r.result = solve_one(r)
        r.done = clock() - t0
    return requests, clock() - t0


class LibEngine:
    """egt_batch_* engine: each request is admitted by its description; the
    batch builds the game's tables into its own arena (charged to the budget
    with the solve's state), so admission and retirement allocate and
    synchronise nothing on the device."""

    def __init__(self, egt_module, budget_bytes, max_slots=64, **solve_opts):
        self.egt = egt_module
        self.batch = egt_module.Batch(budget_bytes, max_slots)
        self.opts = solve_opts

    def admit(self, req):
        return self.batch.admit_desc(req.payload, **self.opts)

    def tick(self):
        return self.batch.tick()

    def poll(self, slot):
        return self.batch.poll(slot)

    def retire(self, slot):
        self.batch.retire(slot)

    def live(self):
        return self.batch.usage()[1]

    def close(self):
        self.batch.close()
