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

    def release(self, r):
        assert r.payload == ("system", r.n)
        r.payload = None

    def _enter(self):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)

    def _leave(self):
        with self.lock:
            self.running -= 1

    def solve_single(self, r, wid):
        r.payload = ("system", r.n)            # the system is made when its solve starts
        self._enter()
        time.sleep(2e-4 + (r.n / 2048.0) ** 3 * 5e-3)
        r.status, r.precision = "ok", 2
        self._leave()

    def solve_batch(self, batch):
        for r in batch:
            r.payload = ("system", r.n)
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
            assert r.payload is None          # freed on completion
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


def test_admission_refuses_over_budget_through_the_library_ledger():
    """The ledger behind Admission: refusals are counted, a footprint above
    the whole budget is an error, and releases cannot go below zero."""
    import pytest
    from paper_2008_11480_amd import nsr
    L = nsr.Ledger(1000)
    assert L.admit(600) and not L.admit(500) and L.admit(400)
    q = L.query()
    assert q["in_use"] == 1000 and q["peak"] == 1000 and q["refused"] == 1 and q["admitted"] == 2
    with pytest.raises(nsr.NSError):
        L.admit(1001)
    L.release(1000)
    with pytest.raises(nsr.NSError):
        L.release(1)
    assert nsr.solve_footprint(100, nsr.PREC_FP64, 0) == (nsr.workspace_bytes(100) +
                                                          (100 * 100 + 200) * 8)
    assert nsr.solve_footprint(0) == 0


def test_householder_factors_wy_form():
    """The serving inputs' compact WY form: diag(lam) + Z C Z^T equals
    Q diag(lam) Q^T with Q the product of the explicit reflections, and the
    draws are those of the seeded recipe (lam pinned at 1 and kappa)."""
    lam, vs, b = inputs.householder_factors(70, 1e5, 11)
    assert lam.min() == 1.0 and lam.max() == 1e5 and vs.shape == (4, 70) and b.shape == (70,)
    z, c = inputs._wy_core(lam, vs)
    q = np.eye(70)
    for v in vs:
        q = q @ (np.eye(70) - 2.0 * np.outer(v, v) / (v @ v))
    ref = q @ np.diag(lam) @ q.T
    np.testing.assert_allclose(np.diag(lam) + z @ c @ z.T, ref, rtol=0, atol=1e-15 * 1e5 * 10)
    np.testing.assert_allclose(c, c.T, rtol=0, atol=0)
    # the packed host array: (Z C) Z^T + diag(lam) is the same matrix
    pk = inputs.householder_pack(lam, vs, b)
    zc, z2 = pk[:70 * 8].reshape(70, 8), pk[70 * 8:2 * 70 * 8].reshape(70, 8)
    np.testing.assert_allclose(zc @ z2.T + np.diag(lam), ref, rtol=0, atol=1e-15 * 1e5 * 10)
    tail = pk[2 * 70 * 8:]
    np.testing.assert_array_equal(tail[:70], lam)
    np.testing.assert_array_equal(tail[70:140], b)
    np.testing.assert_array_equal(tail[140:210], 0.0)
    np.testing.assert_array_equal(tail[210:].reshape(4, 70), vs)
