"""Host logic of the serving loop (no GPU): slot limit, admission in arrival
order, HBM budget, latency accounting and per-request errors, with a
stand-in solve that sleeps."""
import threading
import time

import pytest

from paper_2306_00632_amd import serve


class Probe:
    def __init__(self, durations, fail=()):
        self.durations = durations
        self.fail = set(fail)
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.bytes = 0
        self.max_bytes = 0
        self.order = []

    def solve(self, slot, req, keep):
        with self.lock:
            self.active += 1
            self.bytes += serve.estimate_bytes(req)
            self.max_active = max(self.max_active, self.active)
            self.max_bytes = max(self.max_bytes, self.bytes)
            self.order.append(req.rid)
        time.sleep(self.durations[req.rid])
        with self.lock:
            self.active -= 1
            self.bytes -= serve.estimate_bytes(req)
        if req.rid in self.fail:
            raise RuntimeError("planted failure")
        return {"iters": 3, "relres": 1e-7, "converged": True, "rank": (1, 1, 1)}


def make_server(probe, slots, budget=1e15):
    return serve.Server(slots=slots, hbm_budget=budget, solve=probe.solve, make_slot=lambda: object())


def test_slot_limit_and_arrival_order():
    reqs = serve.poisson_arrivals(serve.mixed_requests(12, 7), rate=0.0, seed=1)
    probe = Probe({r.rid: 0.05 for r in reqs})
    res = make_server(probe, 3).run(reqs)
    assert probe.max_active == 3
    assert probe.order == sorted(probe.order)          # admitted in arrival (= id) order
    assert [r.rid for r in res] == list(range(12))
    s = serve.summarize(res)
    assert s["completed"] == 12 and s["errors"] == 0
    # 12 jobs of 50 ms on 3 slots take at least 4 rounds
    assert s["makespan_s"] >= 0.2 - 1e-3


def test_arrivals_respected_and_latency():
    reqs = serve.poisson_arrivals(serve.mixed_requests(6, 3), rate=20.0, seed=4)
    probe = Probe({r.rid: 0.02 for r in reqs})
    res = make_server(probe, 8).run(reqs)
    for r in res:
        assert r.start >= r.arrival - 1e-3
        assert r.latency >= 0.02 - 1e-3
    # the arrival times are increasing and the solves are admitted in that order
    assert probe.order == [r.rid for r in sorted(reqs, key=lambda q: q.arrival)]


def test_budget_limits_concurrency():
    reqs = serve.mixed_requests(8, 11, n_els=(64,), ps=(3,), Rs=(9,))
    one = serve.estimate_bytes(reqs[0])
    probe = Probe({r.rid: 0.03 for r in reqs})
    res = make_server(probe, 8, budget=2.5 * one).run(reqs)
    assert probe.max_bytes <= 2.5 * one
    assert probe.max_active == 2
    assert serve.summarize(res)["completed"] == 8


def test_request_larger_than_budget_is_rejected():
    reqs = serve.mixed_requests(2, 5)
    probe = Probe({r.rid: 0.0 for r in reqs})
    with pytest.raises(ValueError):
        make_server(probe, 2, budget=1.0).run(reqs)


def test_failure_is_reported_per_request():
    reqs = serve.mixed_requests(5, 9)
    probe = Probe({r.rid: 0.01 for r in reqs}, fail={2})
    res = make_server(probe, 2).run(reqs)
    assert [r.error is not None for r in res] == [False, False, True, False, False]
    s = serve.summarize(res)
    assert s["completed"] == 4 and s["errors"] == 1
