"""Choice of the Newton-Schulz program per (N, kappa, precision).

The paper compares evaluation programs of one step by their efficiency index
``order ** (1 / mmm)`` (eq. ei): the order reached per matrix product.  On
one GPU the products are not equal in cost -- in float64 the products among
powers of the residual run with a symmetric output (about half the flop),
the nested table programs add element-wise sums, and whole steps are
discrete (the iteration stops at the rounding floor, one step after reaching
it) -- so the program is chosen by measurement: every candidate solves the
same system (the caller's, or a seeded stand-in with the requested N and
kappa) and the fastest one that reaches the residual tolerance wins.  Results
are cached per bucket (precision, round(log2 N), round(log10 kappa)).

:func:`predicted_steps` gives the step count the eigen closed form of eq. fk1
predicts, ``rho(F_k) = rho(F_0)^(order^k)``, for the report.

Host logic only: every solve runs through ``richardson_ns_solve``.
"""
from __future__ import annotations

import dataclasses
import math
import time


@dataclasses.dataclass(frozen=True)
class Program:
    order: int
    form: str
    p: int = 0
    w: int = 0

    @property
    def name(self) -> str:
        if self.form.startswith("unified"):
            return f"{self.form}(p={self.p},w={self.w}) order {self.order}"
        return f"{self.form} order {self.order}"


# Programs with the best efficiency index of each family (Tables 1-3,
# eqs. ex1-ex3, ztab2), plus order 4 for ill-conditioned float32 work.
CANDIDATES = (
    Program(8, "squaring"),
    Program(16, "squaring"),
    Program(4, "squaring"),
    Program(11, "table"),
    Program(15, "table"),
    Program(45, "table"),
    Program(9, "unified", 2, 3),
    Program(7, "unified_plus1", 2, 2),
)


# Margin of the stop rule's error-law floor test (the library's value).
LAW_MARGIN = 1e3


def _stop_step(exact, order: int, floor: float, k_max: int) -> int:
    """Step at which the stop rule fires on the modelled history
    ``f_k = max(exact(k), floor)``: the error-law test (``f_{k-1} < 1`` and
    ``f_k > LAW_MARGIN f_{k-1}^order``) or, once at the floor, the ratio test
    (``f_k > f_{k-1} / 2``)."""
    prev = max(exact(0), floor)
    for k in range(1, k_max + 1):
        ex = exact(k)
        cur = max(ex, floor)
        if prev < 1.0 and cur > LAW_MARGIN * prev ** order:
            return k
        if cur > 0.5 * prev and ex <= floor:
            return k
        prev = cur
    return k_max


def predicted_steps(order: int, rho0: float, floor: float, k_max: int = 64) -> int:
    """Stop step predicted by ``||F_k|| = rho0 ** (order ** k)`` (eq. fk1)
    with a rounding floor ``floor`` (see :func:`_stop_step`)."""
    if not 0.0 < rho0 < 1.0:
        raise ValueError("rho(F_0) must lie in (0, 1)")

    def exact(k):
        e = float(order) ** k
        return 0.0 if e > 1e300 else rho0 ** e
    return _stop_step(exact, order, floor, k_max)


def predicted_steps_spectrum(order: int, mu, floor: float, k_max: int = 64) -> int:
    """Stop step predicted by the closed form ``||F_k||_F = sqrt(sum
    mu_i^(2 order^k))`` (eq. fk1, ``mu_i = 1 - lambda_i / alpha``) with a
    Frobenius-norm rounding floor ``floor`` (see :func:`_stop_step`)."""
    import numpy as np
    mu = np.abs(np.asarray(mu, dtype=np.float64))

    def exact(k):
        e = float(order) ** k
        return 0.0 if e > 1e300 else math.sqrt(float(np.sum(mu ** (2.0 * e))))
    return _stop_step(exact, order, floor, k_max)


@dataclasses.dataclass
class Trial:
    program: Program
    ms: float
    ns_steps: int
    refine_steps: int
    mmm: int
    rel_resid: float
    ok: bool


def time_programs(solver, b, theta, programs=CANDIDATES, reps: int = 1, resid_tol: float = 1e-12,
                  k_max: int = 64, refine_max: int = 64) -> list[Trial]:
    """Solve ``solver``'s bound system with every program (one untimed warm-up
    each, then ``reps`` timed solves); returns the trials fastest first."""
    import torch
    out = []
    for prog in programs:
        kw = dict(order=prog.order, form=prog.form, p=prog.p, w=prog.w, k_max=k_max,
                  refine_max=refine_max, resid_tol=resid_tol, raise_on_error=False)
        rep = solver.solve(b, theta, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rep = solver.solve(b, theta, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        ok = rep.status == 0 and rep.rel_resid <= resid_tol
        out.append(Trial(prog, ms, rep.ns_steps, rep.refine_steps, rep.mmm, rep.rel_resid, ok))
    out.sort(key=lambda t: (not t.ok, t.ms))
    return out


def bucket(n: int, kappa: float, precision: int) -> tuple:
    return (int(precision), int(round(math.log2(max(n, 1)))),
            int(round(math.log10(max(kappa, 1.0)))))


class ProgramTable:
    """Best program per (precision, N bucket, kappa bucket), tuned on first use
    with a seeded stand-in system (Householder-product SPD matrix with a
    log-uniform spectrum of condition number kappa).  Callers that do not
    know their system's kappa (a serving loop) look up with ``kappa=None``,
    which uses ``kappa_hint``.  Thread-safe: concurrent lookups of a bucket
    that is not tuned yet tune it once."""

    def __init__(self, programs=CANDIDATES, resid_tol: float = 1e-12, seed: int = 7,
                 kappa_hint: float = 1e4, refine_max: int = 64):
        import threading
        self.programs = tuple(programs)
        self.resid_tol = resid_tol
        self.seed = seed
        self.kappa_hint = float(kappa_hint)
        self.refine_max = int(refine_max)
        self.table: dict[tuple, list[Trial]] = {}
        self._lock = threading.Lock()

    def lookup(self, n: int, kappa: float | None, precision: int) -> Program:
        kappa = self.kappa_hint if kappa is None else kappa
        key = bucket(n, kappa, precision)
        with self._lock:
            if key not in self.table:
                self.table[key] = self._tune(n, kappa, precision)
            return self.table[key][0].program

    def choices(self) -> list[dict]:
        """The tuned buckets and their winners (for reports)."""
        with self._lock:
            return [{"precision": k[0], "log2_n": k[1], "log10_kappa": k[2],
                     "program": v[0].program.name, "ms": v[0].ms,
                     "runner_up": v[1].program.name if len(v) > 1 else None,
                     "runner_up_ms": v[1].ms if len(v) > 1 else None}
                    for k, v in sorted(self.table.items())]

    def _tune(self, n, kappa, precision):
        import torch
        from . import inputs, nsr
        A, b, _, _ = inputs.spd_householder_device(n, kappa, self.seed)
        theta = torch.zeros_like(b)
        s = nsr.Solver(n, precision=precision, composite=False)
        try:
            s.bind(A)
            return time_programs(s, b, theta, self.programs, resid_tol=self.resid_tol,
                                 refine_max=self.refine_max)
        finally:
            s.close()


_DEFAULT_TABLE: ProgramTable | None = None


def default_table() -> ProgramTable:
    """Process-wide table behind ``Solver.solve(order="auto")``."""
    global _DEFAULT_TABLE
    if _DEFAULT_TABLE is None:
        _DEFAULT_TABLE = ProgramTable()
    return _DEFAULT_TABLE


# ---------------------------------------------------------------------------
# Tile autotuner: the GEMM tile per family and size bucket, by measurement.
# ---------------------------------------------------------------------------

def _family_gemm(family: int, n: int, torch, nsr):
    """A representative product of the family at n x n x n (the solver's
    shapes): returns a zero-argument callable that enqueues it."""
    g = torch.Generator(device="cpu").manual_seed(n)
    if family == nsr.TILE_F64:
        X = torch.randn(n, n, generator=g, dtype=torch.float64).cuda()
        D = torch.empty_like(X)
        return lambda: nsr.gemm_f64(X, X, D=D)
    X = torch.randn(n, n, generator=g, dtype=torch.float32).cuda()
    D = torch.empty_like(X)
    if family == nsr.TILE_F32:
        return lambda: nsr.gemm_lp(X, X, nt=False, D=D)
    if family == nsr.TILE_BF16:
        Xb = X.to(torch.bfloat16)
        return lambda: nsr.gemm_lp(Xb, Xb, nt=True, D=D)
    scratch = torch.empty(int(nsr.lib().ns_gemm_f32_split_scratch_bytes(n, n, n)),
                          dtype=torch.uint8, device="cuda")
    return lambda: nsr.gemm_f32_split(X, X, D=D, scratch=scratch)


def tune_tiles(families=None, sizes=(256, 512, 1024, 2048, 4096, 8192), reps: int = 3,
               trials: int = 3, min_ms: float = 4.0, install: bool = True) -> list[dict]:
    """Time every tile of each GEMM family at each size (n x n x n) and, with
    ``install``, set the fastest for that size's bucket (``ns_tile_set``).

    Each candidate (the rule's own choice, tile 0, and every explicit tile)
    is warmed up once; then ``trials`` rounds go over the candidates in turn,
    each timing a run of at least ``reps`` launches and ``min_ms``
    milliseconds between HIP events on the current stream, and a candidate's
    time is its fastest round (interleaving the rounds keeps clock and
    cache drift from favouring the candidates timed last).  Returns one
    record per (family, size) with every candidate's time and the rule's."""
    import torch
    from . import nsr
    families = tuple(nsr.TILE_OPTIONS) if families is None else tuple(families)
    out = []

    def timed(run, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            run()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / k

    for fam in families:
        for n in sizes:
            b = int(math.ceil(math.log2(n)))
            run = _family_gemm(fam, n, torch, nsr)
            cands = (0,) + tuple(nsr.TILE_OPTIONS[fam])
            k = max(1, int(reps))
            for tile in cands:
                nsr.tile_set(fam, b, tile)
                run()
                est = timed(run, 1)
                k = max(k, min(200, int(math.ceil(min_ms / max(est, 1e-3)))))
            times = {t: float("inf") for t in cands}
            for _ in range(max(1, int(trials))):
                for tile in cands:
                    nsr.tile_set(fam, b, tile)
                    times[tile] = min(times[tile], timed(run, k))
            best = min((t for t in times if t), key=lambda t: times[t])
            nsr.tile_set(fam, b, best if install else 0)
            out.append({"family": fam, "n": n, "log2_dim": b, "best_tile": best,
                        "launches_per_round": k,
                        "ms": {str(t): v for t, v in times.items()},
                        "speedup_vs_rule": times[0] / times[best]})
            del run
        torch.cuda.empty_cache()
    return out
