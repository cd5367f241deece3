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

A request's system is made on the device when it is admitted (its inputs
count in the ledger from then on) and freed when it completes, so only the
requests in service occupy HBM, whatever the length of the trace.  The
admission ledger is the library's (``ns_ledger_*``: thread-safe, host only).
Single solves take their Newton-Schulz program from an autotuned
:class:`autotune.ProgramTable` per (precision, N bucket), tuned before the
clock starts (``GpuExecutor.prepare``).

Latency = completion - arrival (making the request's system on the device is
part of it).  The scheduling and admission logic is plain host code driven
through an executor object, so it runs on the CPU with a fake executor in the
tests; :class:`GpuExecutor` is the real one.
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
    kappa: float = 0.0              # of the request's seeded system (not used to solve)
    seed: int = 0
    payload: object = None          # executor-specific (device tensors while in service)
    host: object = None             # host draws of the system, until it is made
    footprint: int = 0
    admitted_s: float = float("nan")
    ready_s: float = float("nan")   # its system made on the device
    start_s: float = float("nan")   # its solve started
    end_s: float = float("nan")
    status: str = "pending"         # pending | ok | noconv | diverged | rejected | error
    path: str = ""                  # "batch" | "single"
    precision: int = -1
    ns_steps: int = 0
    rel_resid: float = float("nan")  # the library's report of the returned theta


class Admission:
    """HBM-footprint admission control through the library's ledger
    (``ns_ledger_*``, thread-safe)."""

    def __init__(self, budget_bytes: int):
        from . import nsr
        self.budget = int(budget_bytes)
        self._ledger = nsr.Ledger(self.budget)

    @property
    def in_use(self) -> int:
        return self._ledger.query()["in_use"]

    @property
    def peak(self) -> int:
        return self._ledger.query()["peak"]

    def fits_at_all(self, footprint: int) -> bool:
        return footprint <= self.budget

    def try_admit(self, footprint: int) -> bool:
        return self._ledger.admit(footprint)

    def release(self, footprint: int):
        self._ledger.release(footprint)


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
        self.ex._now = now

        def finish(batch):
            end = now()
            for r in batch:
                self.ex.release(r)          # the request's device memory
            with cv:
                for r in batch:
                    r.end_s = end
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
                r.start_s = now()
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
                t_start = now()
                for r in batch:
                    r.start_s = t_start
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

        def pct(vals, q):
            v = np.array([x for x in vals if np.isfinite(x)]) * 1e3
            return float(np.percentile(v, q)) if len(v) else None
        stages = {
            "queue_ms": [r.start_s - r.admitted_s for r in served],
            "make_system_ms": [r.ready_s - r.start_s for r in served],
            "solve_single_ms": [r.end_s - r.start_s for r in served if r.path == "single"],
            "solve_batch_ms": [r.end_s - r.start_s for r in served if r.path == "batch"],
        }
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
            "rel_resid_max_reported": max((r.rel_resid for r in served if r.status == "ok"),
                                          default=None),
            "stages": {k: {"p50": pct(v, 50), "p99": pct(v, 99)} for k, v in stages.items()},
        }
        return out


class GpuExecutor:
    """Runs requests through libnsr: batches for small systems, one solver per
    worker thread and HIP stream for the rest.  ``order="auto"``: single
    solves take their program from ``self.table`` (an autotuned
    :class:`autotune.ProgramTable`, kappa unknown to the server: the table's
    ``kappa_hint``); an integer order runs the squaring form of that order."""

    def __init__(self, workers: int, precision: int, order="auto", resid_tol: float = 1e-10,
                 small_max_n: int = 256, batch_max: int = 256, refine_max: int = 100,
                 split_min_n: int = 1536, kappa_hint: float = 1e4):
        import torch
        from . import autotune, nsr
        self.torch, self.nsr = torch, nsr
        self.precision, self.order, self.resid_tol = precision, order, resid_tol
        self.split_min_n = split_min_n
        self.small_max_n = small_max_n
        self.refine_max = refine_max
        self.table = autotune.ProgramTable(resid_tol=resid_tol, kappa_hint=kappa_hint,
                                           refine_max=refine_max)
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
        if n <= self.small_max_n:   # batched: inputs only (the batch workspace is resident)
            return (n * n + 2 * n) * 8
        return self.nsr.solve_footprint(n, self.precision_for(n), 0)

    def prepare(self, sizes):
        """Tune the program table for the single-solve sizes in ``sizes``
        (one lookup per (precision, N bucket)) before the clock starts."""
        if self.order != "auto":
            return []
        seen = set()
        for n in sorted(set(int(x) for x in sizes)):
            if n <= self.small_max_n:
                continue
            from .autotune import bucket
            key = bucket(n, self.table.kappa_hint, self.precision_for(n))
            if key in seen:
                continue
            seen.add(key)
            self.table.lookup(n, None, self.precision_for(n))
        return self.table.choices()

    def host_draws(self, r: Request):
        """The request's host data (before the clock): small systems whole
        (``inputs.householder_dense_pack``, uploaded with their batch), larger
        ones as O(n) factors (``inputs.householder_pack``, made on the device
        by the worker that solves them)."""
        from . import inputs
        f = inputs.householder_factors(r.n, r.kappa, r.seed % (2 ** 31))
        return (inputs.householder_dense_pack(*f) if r.n <= self.small_max_n
                else inputs.householder_pack(*f))

    def _make_single(self, r: Request):
        """Make a single-path request's system on the current stream."""
        from . import inputs
        host = r.host if r.host is not None else self.host_draws(r)
        r.payload = inputs.householder_unpack_device(host, r.n)
        r.host = None

    def _make_batch(self, batch: list[Request]):
        """Upload a batch of small requests' systems with one copy on the
        current stream."""
        import numpy as np
        from . import inputs
        hosts = [r.host if r.host is not None else self.host_draws(r) for r in batch]
        dev = self.torch.from_numpy(np.concatenate(hosts)).to("cuda", non_blocking=False)
        o = 0
        for r, h in zip(batch, hosts):
            r.payload = inputs.dense_unpack(dev[o:o + h.size], r.n)
            r.host = None
            o += h.size

    def release(self, r: Request):
        """Drop the request's device tensors, keeping theta and what checks it
        (lam, V, b) unless ``keep_results`` is off."""
        if r.payload is not None and not getattr(self, "keep_results", False):
            r.payload = None

    def solve_single(self, r: Request, wid: int):
        torch, nsr = self.torch, self.nsr
        st = self.streams[wid]
        with torch.cuda.stream(st):
            self._make_single(r)
            r.ready_s = self._now() if hasattr(self, "_now") else float("nan")
            A, b, th = r.payload[:3]
            s = nsr.Solver(r.n, precision=self.precision_for(r.n), composite=False, stream=st)
            s.bind(A)
            prog = dict(order="auto", table=self.table) if self.order == "auto" else dict(
                order=self.order, form="squaring")
            rep = s.solve(b, th, k_max=64, resid_tol=self.resid_tol,
                          refine_max=self.refine_max, raise_on_error=False, **prog)
            s.close()
            del s
        r.status = {nsr.NS_OK: "ok", nsr.NS_ENOCONV: "noconv"}.get(rep.status, "diverged")
        r.precision = rep.precision
        r.ns_steps = rep.ns_steps
        r.rel_resid = rep.rel_resid

    def solve_batch(self, batch: list[Request]):
        torch, nsr = self.torch, self.nsr
        with torch.cuda.stream(self.batch_stream):
            self._make_batch(batch)
            ready = self._now() if hasattr(self, "_now") else float("nan")
            for r in batch:
                r.ready_s = ready
            As = [r.payload[0] for r in batch]
            bs = [r.payload[1] for r in batch]
            ths = [r.payload[2] for r in batch]
            t = self.batch.submit(As, bs, ths, order=4, resid_tol=self.resid_tol,
                                  refine_max=self.refine_max)
            cols = self.batch.poll_arrays(t, wait=True)
        names = {nsr.NS_OK: "ok", nsr.NS_ENOCONV: "noconv"}
        for r, st, prec, steps, rel in zip(batch, cols["status"].tolist(),
                                           cols["precision"].tolist(), cols["ns_steps"].tolist(),
                                           cols["rel_resid"].tolist()):
            r.status = names.get(st, "diverged")
            r.precision = prec
            r.ns_steps = steps
            r.rel_resid = rel


def make_requests(trace, draw=None) -> list[Request]:
    """Requests for a trace of ``inputs.Request`` records.  ``draw`` (an
    executor): make each request's host data now, before the serving clock
    (``GpuExecutor.host_draws``); otherwise the executor makes it when the
    request starts.  The system reaches the device only when its solve
    starts, and is freed when it completes."""
    out = []
    for i, q in enumerate(trace):
        r = Request(rid=i, arrival_s=q.arrival_s, n=q.n, kappa=q.kappa, seed=q.seed)
        if draw is not None and draw is not False:
            r.host = draw.host_draws(r)
        out.append(r)
    return out
