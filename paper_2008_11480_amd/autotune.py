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
    log-uniform spectrum of condition number kappa)."""

    def __init__(self, programs=CANDIDATES, resid_tol: float = 1e-12, seed: int = 7):
        self.programs = tuple(programs)
        self.resid_tol = resid_tol
        self.seed = seed
        self.table: dict[tuple, list[Trial]] = {}

    def lookup(self, n: int, kappa: float, precision: int) -> Program:
        key = bucket(n, kappa, precision)
        if key not in self.table:
            self.table[key] = self._tune(n, kappa, precision)
        return self.table[key][0].program

    def _tune(self, n, kappa, precision):
        import torch
        from . import inputs, nsr
        A, b, _, _ = inputs.spd_householder_device(n, kappa, self.seed)
        theta = torch.zeros_like(b)
        s = nsr.Solver(n, precision=precision, composite=False)
        try:
            s.bind(A)
            return time_programs(s, b, theta, self.programs, resid_tol=self.resid_tol)
        finally:
            s.close()
