"""Plain float64 oracle of the paper's method (test infrastructure only).

Notation follows the paper: ``A`` is the SPD matrix of ``A theta* = b``
(eq. ae1), ``X = G_{k-1}`` the current inverse estimate, ``Y = F_{k-1}`` its
residual, ``Z = G_k`` the next estimate, ``h`` / ``n`` the order of the power
series, ``p, w`` the unified-factorization parameters (eq. h1).

Orientation.  The paper writes the residual on the left, ``Y = I - X A`` and
``Z = P(Y) X``.  This oracle uses the mirrored (right) orientation everywhere,
``Y = I - A X`` and ``Z = X P(Y)``.  For the right pairing
``A Z = (I - Y) P(Y)`` holds without any commutation, so every identity of
Sections 3-5 holds verbatim with left and right exchanged (and every iterate is
a polynomial in ``A`` in exact arithmetic, so the two orientations produce the
same iterates up to rounding).

Every matrix-matrix product goes through ``_mm``, which counts it: the paper
measures cost in matrix-matrix multiplications ("mmm", Section 4), and those
printed counts pin the evaluation orders below.

parity pins: every function here is pinned by a test in ``tests/`` against
exact integer identities (nilpotent shift operands), printed mmm counts, the
eigen-decomposition closed forms of eqs. (fk1)/(ermoex1), diagonal closed
forms, the same iteration in exact rational arithmetic on tiny systems, and
an independent Cholesky solve.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "MMCounter", "alpha_frobenius", "alpha_inf_half", "splitting_condition",
    "residual", "z_horner", "z_unified", "z_unified_plus1", "z_squaring",
    "diag_preconditioner", "initial_series", "gc_init", "gc_step", "gc_exponent",
    "sri_init", "sri_step", "sri_exponent",
    "z_table", "TABLE_ORDERS", "z_form", "form_mmm", "ns_step",
    "dns_init", "dns_step", "dns_step_recursive", "accelerator_matrix",
    "richardson_update", "accelerator_apply", "SolveOptions",
    "SolveReport", "riem6_gamma",
    "solve", "stop_check", "floor_probe_needed", "STOP", "LAW_MARGIN", "efficiency_index",
]


class MMCounter:
    """Counts matrix-matrix multiplications (mmm)."""

    def __init__(self) -> None:
        self.n = 0

    def __call__(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        self.n += 1
        return x @ y


def _mm(ctr: MMCounter | None, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    if ctr is None:
        return x @ y
    return ctr(x, y)


def _eye_like(a: np.ndarray) -> np.ndarray:
    return np.eye(a.shape[0], dtype=np.float64)


# ---------------------------------------------------------------------------
# Section 2: splitting and the scalar preconditioner S^{-1} = I / alpha
# ---------------------------------------------------------------------------

def alpha_frobenius(a: np.ndarray) -> float:
    """``alpha = ||A||_F``, summed with correct rounding (math.fsum).

    With ``S = alpha I``, ``2S - A`` is positive definite because
    ``lambda_max(A) <= ||A||_F``, which is the convergence condition of the
    splitting (eqs. minus, sp1, spro).
    """
    return math.sqrt(math.fsum(np.square(np.asarray(a, dtype=np.float64)).ravel()))


def alpha_inf_half(a: np.ndarray, eps: float) -> float:
    """``alpha = ||A||_inf / 2 + eps`` (maximum row sum; Section 2)."""
    return float(np.max(np.sum(np.abs(a), axis=1))) / 2.0 + float(eps)


def diag_preconditioner(a: np.ndarray) -> np.ndarray:
    """``S = diag(a_11, ..., a_NN)`` of an SDD positive definite ``A``
    (Section 2); returned as the vector of diagonal entries."""
    d = np.diag(np.asarray(a, dtype=np.float64)).copy()
    if not np.all(d > 0.0) or not np.all(np.isfinite(d)):
        raise ValueError("the diagonal preconditioner needs a positive diagonal")
    return d


def initial_series(a: np.ndarray, s_inv: np.ndarray, h: int, p: int, w: int,
                   ctr=None) -> np.ndarray:
    """Initial series of eq. (g01)-(g02), right orientation: with
    ``Y = I - A S^-1``, ``G_0 = S^-1 sum_{j<w} Y^{(p+1) j} sum_{d<=p} Y^d``
    ``= S^-1 sum_{j<h} Y^j`` for ``h = w (p + 1)``, so that
    ``F_0 = I - A G_0 = Y^h`` (eq. g03)."""
    if h != w * (p + 1):
        raise ValueError("initial series needs h = w (p + 1)")
    if h == 1:
        return s_inv.copy()
    return z_unified(a, s_inv, p, w, ctr)


def splitting_condition(a: np.ndarray, alpha: float) -> bool:
    """True iff ``2S - A`` is positive definite for ``S = alpha I`` (Section 2)."""
    m = 2.0 * alpha * _eye_like(a) - a
    try:
        np.linalg.cholesky(0.5 * (m + m.T))
        return True
    except np.linalg.LinAlgError:
        return False


# ---------------------------------------------------------------------------
# Sections 3-4 and the Appendix: Z = X * sum_{j<h} Y^j, Y = I - A X
# ---------------------------------------------------------------------------

def residual(a: np.ndarray, x: np.ndarray, ctr: MMCounter | None = None) -> np.ndarray:
    """``Y = I - A X`` (eq. xa1 / xa2, right orientation): one mmm."""
    return _eye_like(a) - _mm(ctr, a, x)


def z_horner(a, x, h, ctr=None, y=None):
    """Horner's scheme for eq. (z1): ``Z_0 = X``, ``Z_i = X + Z_{i-1} Y``.

    ``h`` mmm including the residual (Section 4).
    """
    if y is None:
        y = residual(a, x, ctr)
    z = x
    for _ in range(h - 1):
        z = x + _mm(ctr, z, y)
    return z


def z_unified(a, x, p, w, ctr=None, y=None):
    """Unified factorization, eqs. (xa2)-(zi1), order ``h = w (p + 1)``.

    ``U = X sum_{d<=p} Y^d`` (u1, by Horner), ``Y^{p+1} = I - A U`` (ua1),
    ``Z = U sum_{j<w} (Y^{p+1})^j`` via ``Z_i = Z_{i-1} Y^{p+1} + U`` (zi1).
    ``p + w + 1`` mmm; ``p + 1`` when ``w = 1`` and ``w`` when ``p = 0``
    (eq. np1 and the note after it).
    """
    if y is None:
        y = residual(a, x, ctr)
    u = x
    for _ in range(p):
        u = x + _mm(ctr, u, y)
    if w == 1:
        return u
    yp1 = y if p == 0 else residual(a, u, ctr)
    z = u
    for _ in range(w - 1):
        z = _mm(ctr, z, yp1) + u
    return z


def z_unified_plus1(a, x, p, w, ctr=None, y=None):
    """Eq. (ztab2): ``Z_1 = X (I + Y Q(Y))`` with ``Q`` the (ztab1) product.

    Order ``h_1 = w (p + 1) + 1`` (eq. hape1), evaluated as ``Z_1 = X + Z Y``
    with ``Z = X Q(Y)`` from :func:`z_unified`: one mmm more than (ztab1).
    """
    if y is None:
        y = residual(a, x, ctr)
    z = z_unified(a, x, p, w, ctr, y=y)
    return x + _mm(ctr, z, y)


def z_squaring(a, x, n, ctr=None, y=None):
    """Factorized form ``Z = X (I + Y)(I + Y^2)(I + Y^4)...`` for ``n = 2^s``.

    Tables 1-2, orders 2, 4, 8 (``(I+Y^2)(I+Y)X``, ``(I+Y^4)(I+Y^2)(I+Y)X``):
    the powers come from repeated squaring, the factors are multiplied out,
    then applied to ``X``.  ``2 s`` mmm: 2, 4 and 6 for orders 2, 4, 8
    (the Appendix's remark that two / three second-order steps cost 4 / 6 mmm).
    """
    s = int(round(math.log2(n)))
    if n < 2 or (1 << s) != n:
        raise ValueError("squaring form needs n = 2^s >= 2")
    if y is None:
        y = residual(a, x, ctr)
    eye = _eye_like(a)
    p = eye + y
    ypow = y
    for _ in range(s - 1):
        ypow = _mm(ctr, ypow, ypow)
        p = _mm(ctr, p, eye + ypow)
    return _mm(ctr, x, p)


TABLE_ORDERS = (11, 15, 45)


def z_table(a, x, h, ctr=None, y=None):
    """Nested factorizations printed in the paper, right orientation.

    * ``h = 11``: Table 2, second form, ``(I + Y (I + (Y^2+Y^4)(I+Y^4))(I+Y)) X``;
      the polynomial is formed first and applied to ``X`` last: 6 mmm.
    * ``h = 15``: Table 3, nested form
      ``(I + (I + (Y^3)^2)((Y^3)^2 + Y^3)) (I + Y + Y^2) X`` with ``Y^3`` from
      the residual of ``U = (I + Y + Y^2) X`` (eq. ua1): 7 mmm.
    * ``h = 45``: eqs. (ex1)-(ex3): ``U3 = X [3I + (AX)(-3I + AX)]`` with
      ``AX = I - Y`` taken from the residual,
      ``Y^3 = I - A U3``, ``U9 = U3 (I + Y^3 + Y^6)``, ``Y^9 = I - A U9``,
      ``Z = U9 (I + (I + (Y^9)^2)(Y^9 + (Y^9)^2))``: 10 mmm.
    """
    eye = _eye_like(a)
    if h == 11:
        if y is None:
            y = residual(a, x, ctr)
        y2 = _mm(ctr, y, y)
        y4 = _mm(ctr, y2, y2)
        v = y2 + y4
        v = v + _mm(ctr, v, y4)                 # (Y^2+Y^4)(I+Y^4)
        r = eye + _mm(ctr, y + y2, eye + v)     # I + Y(I+Y)(I + ...)
        return _mm(ctr, x, r)
    if h == 15:
        if y is None:
            y = residual(a, x, ctr)
        u = x + _mm(ctr, x + _mm(ctr, x, y), y)  # X (I + Y + Y^2)
        y3 = residual(a, u, ctr)                  # Y^3 = I - A U
        y6 = _mm(ctr, y3, y3)
        s = y6 + y3
        wpoly = s + _mm(ctr, y6, s)               # (I + Y^6)(Y^6 + Y^3)
        return u + _mm(ctr, u, wpoly)
    if h == 45:
        if y is None:
            y = residual(a, x, ctr)
        ax = eye - y                              # A X, from the residual
        u3 = _mm(ctr, x, 3.0 * eye + _mm(ctr, ax, ax - 3.0 * eye))
        y3 = residual(a, u3, ctr)
        y6 = _mm(ctr, y3, y3)
        u9 = _mm(ctr, u3, eye + y3 + y6)
        y9 = residual(a, u9, ctr)
        y18 = _mm(ctr, y9, y9)
        s = y9 + y18
        wpoly = s + _mm(ctr, y18, s)              # (I + (Y^9)^2)(Y^9 + (Y^9)^2)
        return u9 + _mm(ctr, u9, wpoly)
    raise ValueError(f"no nested table form for order {h}")


FORMS = ("horner", "squaring", "unified", "unified_plus1", "table")


def z_form(a, x, order, form, p=None, w=None, ctr=None, y=None):
    """One step ``Z = X sum_{j<order} Y^j`` by the named evaluation form."""
    if form == "horner":
        return z_horner(a, x, order, ctr, y)
    if form == "squaring":
        return z_squaring(a, x, order, ctr, y)
    if form == "unified":
        if p is None or w is None or w * (p + 1) != order:
            raise ValueError("unified form needs order = w (p + 1)")
        return z_unified(a, x, p, w, ctr, y)
    if form == "unified_plus1":
        if p is None or w is None or w * (p + 1) + 1 != order:
            raise ValueError("unified_plus1 form needs order = w (p + 1) + 1")
        return z_unified_plus1(a, x, p, w, ctr, y)
    if form == "table":
        return z_table(a, x, order, ctr, y)
    raise ValueError(f"unknown form {form!r}")


def form_mmm(order, form, p=None, w=None) -> int:
    """mmm of one step, counted by running the form on a 1x1 operand."""
    ctr = MMCounter()
    z_form(np.eye(1) * 0.5, np.eye(1), order, form, p, w, ctr)
    return ctr.n


def riem6_gamma(k: int, n: int, h: int = 1) -> int:
    """Eq. (riem6): exponent of ``S^{-1} D`` in the parameter error after k
    accelerated steps with q = n, ``theta~_k = (S^{-1}D)^{gamma_k} theta~_0``."""
    num = k * n ** (k + 2) - (k - 1) * n ** (k + 1) - 2 * n ** k - n + 2
    g, rem = divmod(h * n * n * num, (n - 1) ** 2)
    assert rem == 0
    return g


def efficiency_index(order: int, mmm: int) -> float:
    """Efficiency index ``order^(1/mmm)`` (eq. ei)."""
    return float(order) ** (1.0 / float(mmm))


def ns_step(a, g, order, form="squaring", p=None, w=None, ctr=None, f=None):
    """Classical high-order Newton-Schulz step, eq. (ns): ``G_k = G_{k-1} P(F_{k-1})``
    with ``F_{k-1} = I - A G_{k-1}`` (passed in as ``f`` when already known)."""
    return z_form(a, g, order, form, p, w, ctr, y=f)


# ---------------------------------------------------------------------------
# Section 5.1: double Newton-Schulz (composite expansion with T = L_k)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class DNSState:
    L: np.ndarray      # L_{k-1}
    Gam: np.ndarray    # Gamma_k = I - A L_{k-1}
    G: np.ndarray      # G_{k-1}
    F: np.ndarray      # F_{k-1} = I - A G_{k-1}


def dns_init(a, t0, order, form="squaring", p=None, w=None, ctr=None) -> DNSState:
    """Precalculation of Section 5.1: ``T_0 = G_0``, ``Gamma_0 = I - A T_0``,
    ``L_0 = T_0 P(Gamma_0)``, ``Gamma_1 = I - A L_0``; ``F_0 = Gamma_0``."""
    gam0 = residual(a, t0, ctr)
    l0 = z_form(a, t0, order, form, p, w, ctr, y=gam0)
    gam1 = residual(a, l0, ctr)
    return DNSState(L=l0, Gam=gam1, G=t0, F=gam0)


def dns_step(a, st: DNSState, order, form="squaring", p=None, w=None, ctr=None) -> DNSState:
    """One step of eqs. (gamk11)-(fks1), right orientation.

    ``L_k = L_{k-1} P(Gamma_k)`` (lkk1); ``Gamma_k^n = I - A L_k`` (gamk21),
    which is also ``Gamma_{k+1}``; the ordinary loop ``H = G_{k-1} P(F_{k-1})``;
    the merge ``G_k = L_k + H Gamma_k^n`` (gkgen21); ``F_k = I - A G_k``, which
    equals ``F_{k-1}^n Gamma_k^n`` (fks1).
    """
    l_k = z_form(a, st.L, order, form, p, w, ctr, y=st.Gam)
    gam_n = residual(a, l_k, ctr)
    hmat = z_form(a, st.G, order, form, p, w, ctr, y=st.F)
    g_k = l_k + _mm(ctr, hmat, gam_n)
    f_k = residual(a, g_k, ctr)
    return DNSState(L=l_k, Gam=gam_n, G=g_k, F=f_k)


def accelerator_matrix(a, st: DNSState, q, ctr=None):
    """Eq. (redttk2)'s ``omega_k`` formed as a matrix, right orientation:
    ``omega_k = L_k + G_k {sum_{j<q} F_k^j} Gamma_k^n`` (the sum by Horner's
    scheme, eq. z1), for the state after step k."""
    w = st.G
    for _ in range(q - 1):
        w = st.G + _mm(ctr, w, st.F)
    return st.L + _mm(ctr, w, st.Gam)


def dns_step_recursive(a, st: DNSState, omega_prev, order, form="squaring", p=None, w=None,
                       ctr=None) -> DNSState:
    """One double Newton-Schulz step with ``G_k`` from the recursion of
    eq. (gkrecu1) (Section 6.2), right orientation.

    Both parts start from the sum ``P(Gamma_k) = sum_{j<n} Gamma_k^j`` with
    ``Gamma_k = Gamma_{k-1}^n``.  Part 1: the ordinary loop
    ``H = G_{k-1} P(F_{k-1})`` and ``G_k = (omega_{k-1} - H) P(Gamma_k) + H``,
    one product given ``omega_{k-1}`` (eq. redttk2 with q = n, of the previous
    step, as a matrix).  Part 2: ``L_k = L_{k-1} P(Gamma_k)`` (lkk1) and
    ``Gamma_k^n = I - A L_k`` (gamk21).  Then ``F_k = I - A G_k``.  In exact
    arithmetic ``G_k`` equals eq. (gkgen21)'s ``L_k + H Gamma_k^n``."""
    eye = _eye_like(a)
    p_gam = z_form(a, eye, order, form, p, w, ctr, y=st.Gam)
    l_k = _mm(ctr, st.L, p_gam)
    gam_n = residual(a, l_k, ctr)
    hmat = z_form(a, st.G, order, form, p, w, ctr, y=st.F)
    g_k = _mm(ctr, omega_prev - hmat, p_gam) + hmat
    f_k = residual(a, g_k, ctr)
    return DNSState(L=l_k, Gam=gam_n, G=g_k, F=f_k)


# ---------------------------------------------------------------------------
# Section 5: general composite expansion, eqs. (gkgen1)-(ga1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class GCState:
    T: list            # T_i = S^-1 sum_{j < x_i} (S^-1 D)^j, x_i = m_i^(k-1)
    Gam: list          # Gamma_i = I - A T_i = (S^-1 D)^(x_i)   (eq. ga1, mirrored)
    G: np.ndarray      # G_{k-1}
    F: np.ndarray      # F_{k-1} = I - A G_{k-1}


def _loop_step(a, t, gam, m, form, ctr):
    """One order-m Newton-Schulz step of a composite loop: ``T P_m(Gamma)``;
    order 1 leaves ``T`` unchanged (``x_i = 1^k = 1``)."""
    if m == 1:
        return t
    return z_form(a, t, m, form, None, None, ctr, y=gam)


def gc_init(a, g0, rates, ctr=None) -> GCState:
    """Step 0 of the composite: every ``T_i = G_0 = S^-1`` (``x_i = m_i^0 = 1``),
    ``Gamma_i = F_0``."""
    f0 = residual(a, g0, ctr)
    return GCState(T=[g0.copy() for _ in rates], Gam=[f0.copy() for _ in rates], G=g0, F=f0)


def gc_step(a, st: GCState, order, rates, form="squaring", ctr=None) -> GCState:
    """One step of the composite expansion with w = len(rates) parallel power
    series, right orientation.

    Each loop advances its series to ``x_i = m_i^k`` (``T_i <- T_i P_{m_i}(Gamma_i)``,
    ``Gamma_i = I - A T_i``, eqs. ti / ga1); the composite polynomial and residual
    are ``T_c = T_1 + T_2 Gamma_1 + T_3 Gamma_2 Gamma_1 + ...`` and
    ``Gamma_c = Gamma_w ... Gamma_1`` (eqs. tc / gc, mirrored so that
    ``A T_c = I - Gamma_c``, eq. rel1); then
    ``G_k = T_c + G_{k-1} P_n(F_{k-1}) Gamma_c`` (eq. gkgen1) and
    ``F_k = I - A G_k = F_{k-1}^n Gamma_c`` (eq. gem1).
    """
    ts, gams = [], []
    for t, gam, m in zip(st.T, st.Gam, rates):
        t_new = _loop_step(a, t, gam, m, form, ctr)
        ts.append(t_new)
        gams.append(gam if m == 1 else residual(a, t_new, ctr))
    tc, gc = ts[0], gams[0]
    for t_i, g_i in zip(ts[1:], gams[1:]):
        tc = tc + _mm(ctr, t_i, gc)          # + T_i Gamma_{i-1} ... Gamma_1
        gc = _mm(ctr, g_i, gc)               # Gamma_i ... Gamma_1
    if order == 1:
        hmat = st.G
    else:
        hmat = z_form(a, st.G, order, form, None, None, ctr, y=st.F)
    g_k = tc + _mm(ctr, hmat, gc)
    f_k = residual(a, g_k, ctr)
    return GCState(T=ts, Gam=gams, G=g_k, F=f_k)


def gc_exponent(k: int, order: int, rates) -> int:
    """Exponent e_k of ``F_k = F_0^(e_k)`` for :func:`gc_step`:
    ``e_0 = 1``, ``e_k = n e_{k-1} + sum_i m_i^k`` (eq. gem1 with
    ``Gamma_c = F_0^(sum x_i)``)."""
    e = 1
    for j in range(1, k + 1):
        e = order * e + sum(m ** j for m in rates)
    return e


# ---------------------------------------------------------------------------
# Remark 2: the two-loop algorithm of [sri], for comparison
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SRIState:
    Z: np.ndarray      # Z_{k-1}
    L: np.ndarray      # L_{k-1} = I - A Z_{k-1}
    G: np.ndarray      # G_{k-1}
    F: np.ndarray      # F_{k-1} = I - A G_{k-1}


def sri_init(a, g0, ctr=None) -> SRIState:
    f0 = residual(a, g0, ctr)
    return SRIState(Z=g0, L=f0, G=g0, F=f0)


def sri_step(a, st: SRIState, order, form="squaring", ctr=None) -> SRIState:
    """Eqs. (sri1)-(sri2) in the right orientation: ``Z_k = Z_{k-1} P_p(L_{k-1})``,
    ``G_k = G_{k-1} + Z_k F_{k-1}``; then ``L_k = I - A Z_k = L_{k-1}^p``
    (srilk) and ``F_k = I - A G_k = L_k F_{k-1}`` (srifk1, mirrored)."""
    z_k = z_form(a, st.Z, order, form, None, None, ctr, y=st.L)
    l_k = residual(a, z_k, ctr)
    g_k = st.G + _mm(ctr, z_k, st.F)
    f_k = residual(a, g_k, ctr)
    return SRIState(Z=z_k, L=l_k, G=g_k, F=f_k)


def sri_exponent(k: int, order: int) -> int:
    """``F_k = F_0^(E_k)`` with ``E_k = 1 + p + ... + p^k`` (from srilk / srifk1
    with ``Z_0 = G_0``, so ``L_0 = F_0``)."""
    return sum(order ** j for j in range(k + 1))


# ---------------------------------------------------------------------------
# Section 6: Richardson iteration coupled with the inverse estimate
# ---------------------------------------------------------------------------

def richardson_update(a, b, theta, g):
    """``theta_k = theta_{k-1} - G_k (A theta_{k-1} - b)``: eq. (redttk1) with
    ``omega_k = G_k``.  Returns ``(theta_k, r)`` where ``r = b - A theta_{k-1}``."""
    r = b - a @ theta
    return theta + g @ r, r


def accelerator_apply(a, st: DNSState, r, q):
    """Eq. (ttk1)'s operator on a vector, right orientation:
    ``omega r = L_k r + G_k {sum_{j<q} F_k^j} Gamma_k^n r``, with ``L_k``,
    ``Gamma_k^n = I - A L_k``, ``G_k`` and ``F_k = I - A G_k`` of the double
    Newton-Schulz step (Section 5.1).  Then ``I - A omega = F_k^q Gamma_k^n``
    (eq. riem1 mirrored), so the parameter error contracts by
    ``F_k^q Gamma_k^n`` per step."""
    t = st.Gam @ r
    w = t
    for _ in range(q - 1):
        w = t + st.F @ w
    return st.L @ r + st.G @ w


# Stop reasons (shared meaning with the solver's report; values are the
# oracle's own).
STOP = {
    "none": 0, "f_tol": 1, "floor": 2, "k_max": 3, "diverged": 4,
    "resid_tol": 5, "refine_max": 6, "refine_stall": 7,
}


# Margin of the error-law floor test (see stop_check).
LAW_MARGIN = 1e3


def stop_check(fhist, f_tol, k, k_max, floor_detect=True, f_sq=None, order=None):
    """Stop rule for the Newton-Schulz phase; the paper gives none.

    ``fhist[j] = ||F_j||_F`` for ``j = 0..k``; ``f_sq = ||F_k^2||_F`` (needed
    only when ``||F_k|| > ||F_{k-1}|| / 2``); ``order`` is the step's order n
    for the programs whose ``F_k`` is ``F_{k-1}^m`` with ``m >= n`` in exact
    arithmetic (None: not used).  Stop when
    (i) ``||F_k|| <= f_tol``;
    (ii-a) the error law says rounding dominates: ``F_k = F_{k-1}^n``
    (eq. fk1) gives ``||F_k||_F <= ||F_{k-1}||_2^{n-1} ||F_{k-1}||_F
    <= ||F_{k-1}||_F^n`` in exact arithmetic, so with ``||F_{k-1}|| < 1`` a
    measured ``||F_k|| > LAW_MARGIN ||F_{k-1}||^n`` is rounding error, which
    another step reproduces: floor, found on the step that reaches it;
    (ii) the rounding floor is reached.  In exact arithmetic
    ``F_k = F_{k-1}^n`` gives ``||F_k|| / ||F_{k-1}|| <= ||F_k||_2^{(n-1)/n}``.
    ``s = ||F_k^2||_F / ||F_k||_F`` estimates ``||F_k||_2`` (it is a lower
    bound that is close whenever the dominant eigenvalues carry the
    Frobenius sum).  A ratio above 1/2 together with ``s <= 1/4`` contradicts
    exact arithmetic, so rounding dominates: floor.  A ratio above 1/2 with
    ``s`` near 1 is a slow mode that is still converging: continue;
    (iii) ``k = k_max``;
    (iv) divergence: a non-finite norm or ``||F_k|| > ||F_0||``.
    Returns the reason name or ``None``.
    """
    fk = fhist[k]
    if not math.isfinite(fk) or fk > fhist[0]:
        return "diverged"
    if fk <= f_tol:
        return "f_tol"
    if (floor_detect and order and k >= 1 and fhist[k - 1] < 1.0
            and fk > LAW_MARGIN * fhist[k - 1] ** order):
        return "floor"
    if floor_detect and k >= 1 and fk > 0.5 * fhist[k - 1]:
        if f_sq is None:
            raise ValueError("||F_k^2|| is needed to test the floor")
        if f_sq <= 0.25 * fk:
            return "floor"
    if k >= k_max:
        return "k_max"
    return None


def floor_probe_needed(fhist, k, floor_detect=True, order=None):
    """True when :func:`stop_check` needs ``||F_k^2||``."""
    if not (floor_detect and k >= 1 and math.isfinite(fhist[k])):
        return False
    if order and fhist[k - 1] < 1.0 and fhist[k] > LAW_MARGIN * fhist[k - 1] ** order:
        return False                       # the error-law test decides
    return fhist[k] > 0.5 * fhist[k - 1]


@dataclasses.dataclass
class SolveOptions:
    order: int = 8
    form: str = "squaring"
    p: int | None = None
    w: int | None = None
    composite: bool = False        # double Newton-Schulz (Section 5.1)
    k_max: int = 64
    f_tol: float = 0.0
    floor_detect: bool = True
    refine_max: int = 64
    resid_tol: float = 1e-12
    scale: str = "frobenius"       # or "inf_half", or "diag" (S = diag(A), SDD case)
    eps: float = 0.0               # for "inf_half"
    init_order: int = 1            # h of the initial series, eq. (g01)
    init_p: int | None = None      # its factorization, h = init_w (init_p + 1)
    init_w: int | None = None
    theta0: str = "g0b"            # "g0b": theta_0 = G_0 b;  "zero";  "l0b": L_0 b
    accel_q: int = 0               # >0: Richardson with the accelerator of eq. (ttk1),
                                   # Neumann order q (composite form only)
    rates: tuple | None = None     # general composite (eqs. gkgen1-ga1): loop orders m_i
    sri: bool = False              # the two-loop algorithm of Remark 2 ([sri])


@dataclasses.dataclass
class SolveReport:
    alpha: float
    theta: np.ndarray
    G: np.ndarray
    fnorm_hist: list        # ||F_k||_F, k = 0..ns_steps
    resid_hist: list        # ||b - A theta_j|| / ||b|| for every theta_j formed
    ns_steps: int
    refine_steps: int
    ns_stop: str            # why the Newton-Schulz phase ended
    refine_stop: str        # why the refinement phase ended
    rel_resid: float        # of the returned theta
    mmm: int


def solve(a, b, opts: SolveOptions = SolveOptions()) -> SolveReport:
    """Coupled Newton-Schulz / Richardson solve of ``A theta = b``.

    1. ``G_0 = I / alpha`` (Section 2; ``alpha = ||A||_F`` or ``||A||_inf/2+eps``)
       and ``theta_0 = G_0 b``.
    2. Step ``k``: ``G_k`` from eq. (ns) (or eqs. (gamk11)-(fks1) for the
       composite form), then the Richardson update with the new ``G_k``
       (eq. redttk1 with ``omega_k = G_k``; its residual ``b - A theta_{k-1}``
       is recorded), then ``F_k = I - A G_k`` and the stop rule of
       :func:`stop_check`.
    3. Refinement-only Richardson steps with the final ``G`` until
       ``||b - A theta|| / ||b|| <= resid_tol``, ``refine_max`` steps, or a
       stall (less than a factor 2 of progress over 3 steps).
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ctr = MMCounter()
    eye = _eye_like(a)
    if opts.scale == "frobenius":
        alpha = alpha_frobenius(a)
        g0 = eye / alpha
    elif opts.scale == "inf_half":
        alpha = alpha_inf_half(a, opts.eps)
        g0 = eye / alpha
    elif opts.scale == "diag":
        sd = diag_preconditioner(a)
        alpha = float(np.max(sd))         # reported only
        g0 = np.diag(1.0 / sd)
    else:
        raise ValueError(opts.scale)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        bnorm = 1.0
    if opts.init_order > 1:
        if opts.composite:
            raise ValueError("the initial series is used with the classical forms")
        ip = opts.init_p if opts.init_p is not None else opts.init_order - 1
        iw = opts.init_w if opts.init_w is not None else 1
        g0 = initial_series(a, g0, opts.init_order, ip, iw, ctr)
    theta = g0 @ b if opts.theta0 == "g0b" else np.zeros_like(b)
    if opts.accel_q and not opts.composite:
        raise ValueError("the accelerator of eq. (ttk1) needs the composite form")

    if sum([bool(opts.composite), opts.rates is not None, bool(opts.sri)]) > 1:
        raise ValueError("composite, rates and sri are exclusive")
    if opts.composite:
        st = dns_init(a, g0, opts.order, opts.form, opts.p, opts.w, ctr)
        g, f = st.G, st.F
        if opts.theta0 == "l0b" or opts.accel_q:
            theta = st.L @ b              # theta_0 = L_0 b (Section 6, below eq. riem6)
    elif opts.rates is not None:
        st = gc_init(a, g0, opts.rates, ctr)
        g, f = st.G, st.F
    elif opts.sri:
        st = sri_init(a, g0, ctr)
        g, f = st.G, st.F
    else:
        g = g0
        f = residual(a, g, ctr)
    fhist = [float(np.linalg.norm(f))]
    rhist: list[float] = []
    ns_stop = "diverged" if not math.isfinite(fhist[0]) else None
    k = 0
    while ns_stop is None:
        k += 1
        if opts.composite:
            st = dns_step(a, st, opts.order, opts.form, opts.p, opts.w, ctr)
            g, f = st.G, st.F
            if opts.accel_q:
                r = b - a @ theta                      # eq. (ttk1)
                theta = theta + accelerator_apply(a, st, r, opts.accel_q)
            else:
                theta, r = richardson_update(a, b, theta, g)
        elif opts.rates is not None or opts.sri:
            if opts.sri:
                st = sri_step(a, st, opts.order, opts.form, ctr)
            else:
                st = gc_step(a, st, opts.order, opts.rates, opts.form, ctr)
            g, f = st.G, st.F
            theta, r = richardson_update(a, b, theta, g)
        else:
            g = ns_step(a, g, opts.order, opts.form, opts.p, opts.w, ctr, f=f)
            theta, r = richardson_update(a, b, theta, g)
            f = residual(a, g, ctr)          # also the next step's residual
        rhist.append(float(np.linalg.norm(r)) / bnorm)
        fhist.append(float(np.linalg.norm(f)))
        f_sq = None
        # the error-law floor test: classical programs (F_k = F_{k-1}^n) and
        # the double Newton-Schulz, whose F_k = F_0^(k n^(k+1) + n^k)
        # (Section 5.1) has an exponent at least n times the previous one
        law = None if (opts.rates is not None or opts.sri) else opts.order
        if floor_probe_needed(fhist, k, opts.floor_detect, law):
            f_sq = float(np.linalg.norm(_mm(ctr, f, f)))
        ns_stop = stop_check(fhist, opts.f_tol, k, opts.k_max, opts.floor_detect, f_sq, law)

    refine = 0
    rel = float("nan")
    refine_stop = "diverged"
    if ns_stop != "diverged":
        while True:
            r = b - a @ theta
            rel = float(np.linalg.norm(r)) / bnorm
            rhist.append(rel)
            if not math.isfinite(rel):
                refine_stop = "diverged"
                break
            if rel <= opts.resid_tol:
                refine_stop = "resid_tol"
                break
            if refine >= opts.refine_max:
                refine_stop = "refine_max"
                break
            if refine >= 3 and rel > 0.5 * rhist[-4]:
                refine_stop = "refine_stall"
                break
            if opts.composite and opts.accel_q:
                theta = theta + accelerator_apply(a, st, r, opts.accel_q)
            else:
                theta = theta + g @ r
            refine += 1
    return SolveReport(alpha=alpha, theta=theta, G=g, fnorm_hist=fhist, resid_hist=rhist,
                       ns_steps=k, refine_steps=refine, ns_stop=ns_stop,
                       refine_stop=refine_stop, rel_resid=rel, mmm=ctr.n)
