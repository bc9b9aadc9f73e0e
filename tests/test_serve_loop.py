"""The serving loop's scheduling logic on the CPU, with a stand-in engine:
FCFS admission under a memory budget, continuous admission as memory frees
up, latency accounting, and the sequential baseline."""
import pytest

from paper_1810_03063_amd.serve import Request, percentile, serve, serve_sequential, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, d):
        self.t += max(d, 0.0)


class FakeEngine:
    """Each request needs payload['mem'] bytes and payload['ticks'] ticks;
    a tick costs 1 ms of fake time."""

    def __init__(self, budget, clock, max_slots=8):
        self.budget = budget
        self.used = 0
        self.clock = clock
        self.slots = {}
        self.max_slots = max_slots
        self.peak = 0
        self.admit_order = []

    def admit(self, req):
        need = req.payload["mem"]
        if self.used + need > self.budget or len(self.slots) >= self.max_slots:
            return None
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = [req, req.payload["ticks"]]
        self.used += need
        self.peak = max(self.peak, self.used)
        self.admit_order.append(req.rid)
        return slot

    def tick(self):
        self.clock.t += 1e-3
        for s in self.slots.values():
            s[1] -= 1
        return len(self.slots), 0

    def poll(self, slot):
        req, left = self.slots[slot]
        return None if left > 0 else ("EGT_OK", {"iters": req.payload["ticks"]})

    def retire(self, slot):
        req, _ = self.slots.pop(slot)
        self.used -= req.payload["mem"]

    def live(self):
        return len(self.slots)


def make_reqs(specs):
    return [Request(i, a, {"mem": m, "ticks": t}) for i, (a, m, t) in enumerate(specs)]


def test_budget_is_respected_and_admission_is_fcfs():
    clk = FakeClock()
    eng = FakeEngine(budget=100, clock=clk)
    reqs = make_reqs([(0.0, 60, 5), (0.0, 60, 5), (0.0, 30, 2), (0.0, 10, 1)])
    out, wall = serve(eng, reqs, clock=clk, sleep=clk.sleep)
    assert eng.peak <= 100
    # request 1 does not fit next to request 0; FCFS keeps 2 and 3 behind it
    assert eng.admit_order == [0, 1, 2, 3]
    assert all(r.status == "EGT_OK" for r in out)
    assert out[1].admitted >= out[0].done - 1e-12


def test_requests_join_while_others_run():
    clk = FakeClock()
    eng = FakeEngine(budget=100, clock=clk)
    reqs = make_reqs([(0.0, 40, 50), (0.010, 40, 5), (0.020, 40, 5)])
    out, _ = serve(eng, reqs, clock=clk, sleep=clk.sleep)
    # request 1 arrives during request 0's run and is admitted without waiting for it
    assert out[1].admitted < out[0].done
    assert out[1].done < out[0].done
    assert out[2].admitted >= out[1].done - 1e-12 or out[2].admitted < out[0].done


def test_latency_accounting_and_summary():
    clk = FakeClock()
    eng = FakeEngine(budget=1000, clock=clk)
    reqs = make_reqs([(0.0, 1, 3), (0.5, 1, 3)])
    out, wall = serve(eng, reqs, clock=clk, sleep=clk.sleep)
    for r in out:
        assert r.latency == pytest.approx(3e-3, abs=1e-9)
    s = summarize(out, wall)
    assert s["requests"] == 2 and s["converged"] == 2
    assert s["p50_ms"] == pytest.approx(3.0, abs=1e-6)


def test_oversized_request_is_reported():
    clk = FakeClock()
    eng = FakeEngine(budget=10, clock=clk)
    with pytest.raises(RuntimeError):
        serve(eng, make_reqs([(0.0, 11, 1)]), clock=clk, sleep=clk.sleep)


def test_sequential_baseline_is_fcfs():
    clk = FakeClock()

    def solve_one(r):
        clk.t += r.payload["ticks"] * 1e-3
        return "EGT_OK", {}

    reqs = make_reqs([(0.0, 1, 10), (0.001, 1, 10), (0.5, 1, 10)])
    out, wall = serve_sequential(solve_one, reqs, clock=clk, sleep=clk.sleep)
    assert out[1].admitted == pytest.approx(0.010)
    assert out[1].latency == pytest.approx(0.019)
    assert out[2].admitted == pytest.approx(0.5)


def test_percentile():
    assert percentile([1, 2, 3, 4, 5], 50) == 3
    assert percentile([1, 2], 99) == pytest.approx(1.99)
