"""Serving-loop scheduling and admission on the CPU (fake executor, no GPU)."""
import threading
import time

import numpy as np

from paper_2008_11480_amd import inputs
from paper_2008_11480_amd.serve import Admission, Request, Server


class FakeExecutor:
    """Sleeps in proportion to n^3 and records what ran concurrently."""

    def __init__(self):
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.batches = []

    def footprint(self, r):
        return r.n * r.n * 8

    def _enter(self):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)

    def _leave(self):
        with self.lock:
            self.running -= 1

    def solve_single(self, r, wid):
        self._enter()
        time.sleep(2e-4 + (r.n / 2048.0) ** 3 * 5e-3)
        r.status, r.precision = "ok", 2
        self._leave()

    def solve_batch(self, batch):
        self._enter()
        self.batches.append(len(batch))
        time.sleep(5e-4)
        for r in batch:
            r.status, r.precision = "ok", 1
        self._leave()


def make(trace):
    return [Request(rid=i, arrival_s=q.arrival_s, n=q.n) for i, q in enumerate(trace)]


def test_admission_accounting():
    a = Admission(100)
    assert a.fits_at_all(100) and not a.fits_at_all(101)
    assert a.try_admit(60) and not a.try_admit(50) and a.try_admit(40)
    assert a.in_use == 100 and a.peak == 100
    a.release(60)
    assert a.try_admit(50) and a.in_use == 90


def test_server_serves_all_and_respects_budget():
    trace = inputs.serving_trace(2000.0, 0.25, seed=5)
    reqs = make(trace)
    ex = FakeExecutor()
    budget = 64 << 20                      # 64 MiB: several large requests at most
    srv = Server(ex, budget, workers=3, small_max_n=256, batch_max=64, batch_window_s=0.002)
    st = srv.run(reqs)
    big = [r for r in reqs if r.n * r.n * 8 > budget]
    assert st["rejected"] == len(big)
    assert st["served"] == len(reqs) - len(big)
    assert st["ok"] == st["served"]
    assert st["hbm_peak_in_service_bytes"] <= budget
    assert st["batched"] == sum(1 for r in reqs if r.n <= 256 and r.status == "ok")
    assert max(ex.batches) <= 64
    for r in reqs:
        if r.status == "ok":
            assert r.end_s >= r.admitted_s >= r.arrival_s - 1e-3
    # FIFO admission: admitted in arrival order
    adm = [r.admitted_s for r in sorted(reqs, key=lambda r: r.arrival_s) if r.status == "ok"]
    assert all(x <= y + 1e-9 for x, y in zip(adm, adm[1:]))
    assert st["latency_ms_p99"] >= st["latency_ms_p50"] > 0


def test_tight_budget_serializes():
    """A budget that holds one request at a time: requests still all finish
    and never overlap in service."""
    reqs = [Request(rid=i, arrival_s=0.0005 * i, n=400) for i in range(20)]
    ex = FakeExecutor()
    srv = Server(ex, 400 * 400 * 8, workers=4)
    st = srv.run(reqs)
    assert st["served"] == 20 and st["ok"] == 20
    assert ex.max_running == 1
    assert st["hbm_peak_in_service_bytes"] == 400 * 400 * 8


def test_trace_distribution():
    trace = inputs.serving_trace(2000.0, 2.0, seed=5)
    n = np.array([q.n for q in trace])
    k = np.array([q.kappa for q in trace])
    assert 3500 < len(trace) < 4500                      # Poisson, rate 2000/s
    assert n.min() >= 32 and n.max() <= 2048
    assert 10 <= k.min() and k.max() <= 1e6
    # log-uniform: the median of log n sits at the middle of [ln 32, ln 2048]
    assert abs(np.median(np.log(n)) - 0.5 * (np.log(32) + np.log(2048))) < 0.15
