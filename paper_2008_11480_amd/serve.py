"""Serving loop: a stream of SPD solve requests of different sizes on one GPU.

Requests arrive on a clock (a replayed Poisson trace).  An admission stage
lets a request into service only while the HBM footprint of all requests in
service (inputs + solver workspace) stays within a budget; a request larger
than the whole budget is rejected.  Admitted requests are routed by size:

* ``n <= small_max_n``: coalesced into one persistent batch launch
  (``ns_batch_*``: one workgroup per system, float32 products with float64
  refinement and float64 re-solve), flushed when ``batch_max`` requests are
  waiting or the oldest has waited ``batch_window_s``;
* larger: solved one by one by worker threads, each on its own HIP stream
  with its own device-resident solver state (``richardson_ns_solve``, mixed
  precision by default: bf16 powers, float32 residual / G-side, float64
  Richardson; from ``split_min_n`` on, the residual and G-side products are
  float32-class products of split half-precision operands, which are faster
  there).

Latency = completion - arrival.  The scheduling and admission logic is plain
host code driven through an executor object, so it runs on the CPU with a
fake executor in the tests; :class:`GpuExecutor` is the real one.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    payload: object = None          # executor-specific (device tensors)
    footprint: int = 0
    admitted_s: float = float("nan")
    end_s: float = float("nan")
    status: str = "pending"         # pending | ok | noconv | diverged | rejected | error
    path: str = ""                  # "batch" | "single"
    precision: int = -1
    ns_steps: int = 0


class Admission:
    """HBM-footprint admission control (host logic, thread-safe)."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.in_use = 0
        self.peak = 0
        self._lock = threading.Lock()

    def fits_at_all(self, footprint: int) -> bool:
        return footprint <= self.budget

    def try_admit(self, footprint: int) -> bool:
        with self._lock:
            if self.in_use + footprint > self.budget:
                return False
            self.in_use += footprint
            self.peak = max(self.peak, self.in_use)
            return True

    def release(self, footprint: int):
        with self._lock:
            self.in_use -= footprint
            assert self.in_use >= 0


class Server:
    def __init__(self, executor, budget_bytes: int, workers: int = 4, small_max_n: int = 256,
                 batch_max: int = 256, batch_window_s: float = 0.002):
        self.ex = executor
        self.adm = Admission(budget_bytes)
        self.workers = int(workers)
        self.small_max_n = int(small_max_n)
        self.batch_max = int(batch_max)
        self.batch_window_s = float(batch_window_s)

    def run(self, requests: list[Request], time_scale: float = 1.0) -> dict:
        """Replay ``requests`` (sorted by arrival) and serve them; returns stats."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        for r in reqs:
            r.footprint = int(self.ex.footprint(r))
        cv = threading.Condition()
        arrived = collections.deque()
        small_q = collections.deque()
        large_q = collections.deque()
        state = {"done": 0, "arrivals_done": False}
        total = len(reqs)
        t0 = time.perf_counter() + 0.05

        def now():
            return time.perf_counter() - t0

        def finish(batch):
            with cv:
                for r in batch:
                    r.end_s = now()
                    self.adm.release(r.footprint)
                state["done"] += len(batch)
                cv.notify_all()

        def arrivals():
            for r in reqs:
                delay = r.arrival_s / time_scale - now()
                if delay > 0:
                    time.sleep(delay)
                with cv:
                    arrived.append(r)
                    cv.notify_all()
            with cv:
                state["arrivals_done"] = True
                cv.notify_all()

        def large_worker(wid):
            while True:
                with cv:
                    while not large_q and state["done"] < total:
                        cv.wait(0.05)
                    if not large_q:
                        return
                    r = large_q.popleft()
                try:
                    self.ex.solve_single(r, wid)
                    r.path = "single"
                except Exception as e:  # keep serving; the request reports the error
                    r.status = f"error: {e}"
                finish([r])

        def batch_worker():
            while True:
                with cv:
                    while not small_q and state["done"] < total:
                        cv.wait(0.05)
                    if not small_q:
                        return
                    # wait for a full batch or the window of the oldest request
                    while (len(small_q) < self.batch_max
                           and now() - small_q[0].admitted_s < self.batch_window_s
                           and not (state["arrivals_done"] and not arrived)):
                        cv.wait(max(1e-4, self.batch_window_s - (now() - small_q[0].admitted_s)))
                    batch = [small_q.popleft() for _ in range(min(len(small_q), self.batch_max))]
                try:
                    self.ex.solve_batch(batch)
                    for r in batch:
                        r.path = "batch"
                except Exception as e:
                    for r in batch:
                        r.status = f"error: {e}"
                finish(batch)

        threads = [threading.Thread(target=arrivals, daemon=True)]
        threads += [threading.Thread(target=large_worker, args=(w,), daemon=True)
                    for w in range(self.workers)]
        threads += [threading.Thread(target=batch_worker, daemon=True)]
        for t in threads:
            t.start()
        # Admission / dispatch (this thread): FIFO, head of line waits for room.
        with cv:
            while state["done"] < total:
                while arrived:
                    r = arrived[0]
                    if not self.adm.fits_at_all(r.footprint):
                        arrived.popleft()
                        r.status = "rejected"
                        r.end_s = now()
                        state["done"] += 1
                        continue
                    if not self.adm.try_admit(r.footprint):
                        break
                    arrived.popleft()
                    r.admitted_s = now()
                    (small_q if r.n <= self.small_max_n else large_q).append(r)
                    cv.notify_all()
                cv.wait(0.01)
        for t in threads:
            t.join(timeout=5.0)
        return self.stats(reqs, time_scale)

    def stats(self, reqs, time_scale):
        served = [r for r in reqs if r.status not in ("rejected",)]
        lat = np.array([r.end_s - r.arrival_s / time_scale for r in served]) * 1e3
        wait = np.array([r.admitted_s - r.arrival_s / time_scale for r in served]) * 1e3
        span = max((r.end_s for r in reqs), default=0.0)
        out = {
            "requests": len(reqs),
            "served": len(served),
            "rejected": sum(1 for r in reqs if r.status == "rejected"),
            "ok": sum(1 for r in reqs if r.status == "ok"),
            "not_ok": [r.rid for r in served if r.status != "ok"][:20],
            "offered_per_s": len(reqs) / (reqs[-1].arrival_s / time_scale) if reqs else 0.0,
            "solves_per_s": len(served) / span if span > 0 else 0.0,
            "span_s": span,
            "latency_ms_p50": float(np.percentile(lat, 50)) if len(lat) else None,
            "latency_ms_p99": float(np.percentile(lat, 99)) if len(lat) else None,
            "latency_ms_max": float(lat.max()) if len(lat) else None,
            "admission_wait_ms_p99": float(np.percentile(wait, 99)) if len(wait) else None,
            "hbm_budget_bytes": self.adm.budget,
            "hbm_peak_in_service_bytes": self.adm.peak,
            "batched": sum(1 for r in served if r.path == "batch"),
            "single": sum(1 for r in served if r.path == "single"),
            "escalated_to_fp64": sum(1 for r in served if r.precision == 0 and r.path == "batch"),
            "single_split": sum(1 for r in served if r.precision == 3 and r.path == "single"),
        }
        return out


class GpuExecutor:
    """Runs requests through libnsr: batches for small systems, one solver per
    worker thread and HIP stream for the rest."""

    def __init__(self, workers: int, precision: int, order: int = 8, resid_tol: float = 1e-10,
                 small_max_n: int = 256, batch_max: int = 256, refine_max: int = 100,
                 split_min_n: int = 1536):
        import torch
        from . import nsr
        self.torch, self.nsr = torch, nsr
        self.precision, self.order, self.resid_tol = precision, order, resid_tol
        self.split_min_n = split_min_n
        self.refine_max = refine_max
        self.streams = [torch.cuda.Stream() for _ in range(workers)]
        self.batch_stream = torch.cuda.Stream()
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        # float64 executor: batched systems in float64 too; otherwise float32
        # with float64 re-solves where float32 cannot reach the tolerance
        bprec = nsr.PREC_FP64 if precision == nsr.PREC_FP64 else nsr.PREC_FP32
        with torch.cuda.stream(self.batch_stream):
            self.batch = nsr.Batch(max_n=small_max_n, max_count=batch_max,
                                   slots=min(batch_max, 4 * cus), precision=bprec,
                                   stream=self.batch_stream)

    def precision_for(self, n: int) -> int:
        """Precision of a single solve of size n: the split mode from
        split_min_n on when the executor runs the mixed mode."""
        if self.precision == self.nsr.PREC_MIXED_BF16 and n >= self.split_min_n:
            return self.nsr.PREC_MIXED_SPLIT
        return self.precision

    def footprint(self, r: Request) -> int:
        n = r.n
        ws = self.nsr.workspace_bytes(n, self.precision_for(n), False)
        return ws + (n * n + 2 * n) * 8

    def solve_single(self, r: Request, wid: int):
        torch, nsr = self.torch, self.nsr
        st = self.streams[wid]
        A, b, th = r.payload[:3]
        with torch.cuda.stream(st):
            s = nsr.Solver(r.n, precision=self.precision_for(r.n), composite=False, stream=st)
            s.bind(A)
            rep = s.solve(b, th, order=self.order, form="squaring", k_max=64,
                          resid_tol=self.resid_tol, refine_max=self.refine_max,
                          raise_on_error=False)
            s.close()
            del s
        r.status = {nsr.NS_OK: "ok", nsr.NS_ENOCONV: "noconv"}.get(rep.status, "diverged")
        r.precision = rep.precision
        r.ns_steps = rep.ns_steps

    def solve_batch(self, batch: list[Request]):
        torch, nsr = self.torch, self.nsr
        As = [r.payload[0] for r in batch]
        bs = [r.payload[1] for r in batch]
        ths = [r.payload[2] for r in batch]
        with torch.cuda.stream(self.batch_stream):
            t = self.batch.submit(As, bs, ths, order=4, resid_tol=self.resid_tol,
                                  refine_max=self.refine_max)
            cols = self.batch.poll_arrays(t, wait=True)
        names = {nsr.NS_OK: "ok", nsr.NS_ENOCONV: "noconv"}
        for r, st, prec, steps in zip(batch, cols["status"].tolist(), cols["precision"].tolist(),
                                      cols["ns_steps"].tolist()):
            r.status = names.get(st, "diverged")
            r.precision = prec
            r.ns_steps = steps


def make_requests(trace, device="cuda") -> list[Request]:
    """Device-resident requests for a trace of ``inputs.Request`` records
    (generated before the serving clock starts)."""
    import torch
    from . import inputs
    out = []
    for i, q in enumerate(trace):
        A, b, lam, V = inputs.spd_householder_device(q.n, q.kappa, q.seed % (2 ** 31),
                                                     device=device)
        out.append(Request(rid=i, arrival_s=q.arrival_s, n=q.n,
                           payload=(A, b, torch.zeros_like(b), lam, V)))
    return out
