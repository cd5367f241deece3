"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: the expected values are
exact integer identities (nilpotent shift operands, for which every power is
exact in floating point), counts printed in the paper, eigen-decomposition and
diagonal closed forms, an independent Cholesky solve (LAPACK through scipy),
and ``numpy.linalg.matrix_power`` for the error law.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2008_11480_amd import inputs


def band_ones(m, h):
    """sum_{j<h} J^j for the m x m upper shift J: ones on diagonals 0..h-1."""
    out = np.zeros((m, m))
    for j in range(min(h, m)):
        out += np.eye(m, k=j)
    return out


def shift_power(m, e):
    return np.eye(m, k=e) if e < m else np.zeros((m, m))


# Evaluation forms and the order each one produces.
FORM_CASES = (
    [("horner", h, None, None) for h in range(2, 20)]
    + [("squaring", n, None, None) for n in (2, 4, 8, 16, 32)]
    + [("unified", w * (p + 1), p, w) for p in range(0, 8) for w in range(1, 7)]
    + [("unified_plus1", w * (p + 1) + 1, p, w) for p in range(0, 8) for w in range(1, 7)]
    + [("table", h, None, None) for h in oracle.TABLE_ORDERS]
)


@pytest.mark.parametrize("form,order,p,w", FORM_CASES)
def test_forms_are_exact_power_series(form, order, p, w):
    """Each factorized evaluation equals X sum_{j<order} Y^j exactly (eq. z1).

    With A = c (I - J) and X = I / c (c a power of two), Y = I - A X = J
    exactly, so Z must be the band of ones of width ``order``.  A dropped term,
    a wrong power or a sign error changes an integer entry.
    """
    if form == "unified" and order < 2:
        pytest.skip("order 1 is the identity step")
    m = 64
    c = 4.0
    a = c * (np.eye(m) - inputs.shift_matrix(m))
    x = np.eye(m) / c
    z = oracle.z_form(a, x, order, form, p, w)
    np.testing.assert_array_equal(z * c, band_ones(m, order))


def test_ns_step_error_law_exact():
    """eq. (fk1): after k steps F_k = F_0^{n^k}; exact on the shift operand."""
    m = 80
    a = np.eye(m) - inputs.shift_matrix(m)
    for n, form in ((2, "squaring"), (3, "horner"), (4, "squaring")):
        g = np.eye(m)
        for k in range(1, 4):
            g = oracle.ns_step(a, g, n, form)
            f = oracle.residual(a, g)
            np.testing.assert_array_equal(f, shift_power(m, n ** k))


def test_printed_mmm_counts(golden_dir):
    with open(os.path.join(golden_dir, "mmm_counts.json")) as fh:
        gold = json.load(fh)
    for e in gold["counts"]:
        got = oracle.form_mmm(e["order"], e["form"], e.get("p"), e.get("w"))
        assert got == e["mmm"], e
    for e in gold["efficiency_index"]:
        ei = oracle.efficiency_index(e["order"], e["mmm"])
        assert round(ei, e["digits"]) == e["ei"], e


@pytest.mark.parametrize("p", range(0, 8))
@pytest.mark.parametrize("w", range(1, 7))
def test_unified_mmm_formula(p, w):
    """eq. (np1): p + w + 1 mmm, p + 1 when w = 1, w when p = 0."""
    if w * (p + 1) < 2:
        pytest.skip("order 1")
    expected = p + w + 1
    if w == 1:
        expected = p + 1
    elif p == 0:
        expected = w
    assert oracle.form_mmm(w * (p + 1), "unified", p, w) == expected
    assert oracle.form_mmm(w * (p + 1), "horner") == w * (p + 1)   # Section 4: h mmm


def test_error_law_matrix_identity():
    """F_{k+1} = F_k^n as matrices (eq. fk1) on a random SPD system, above the
    rounding floor; the power comes from numpy.linalg.matrix_power."""
    s = inputs.spd_qlq(48, 50.0, seed=11)
    a = s.A
    alpha = oracle.alpha_frobenius(a)
    for n, form in ((2, "squaring"), (4, "squaring"), (8, "squaring"), (3, "horner"),
                    (6, "unified"), (7, "unified_plus1"), (11, "table"), (15, "table")):
        p = w = None
        if form == "unified":
            p, w = 2, 2
        if form == "unified_plus1":
            p, w = 2, 2
        g = np.eye(48) / alpha
        f = oracle.residual(a, g)
        for _ in range(3):
            g = oracle.ns_step(a, g, n, form, p, w)
            f_next = oracle.residual(a, g)
            fpow = np.linalg.matrix_power(f, n)
            err = np.linalg.norm(f_next - fpow)
            assert err <= 1e-13 * max(1.0, np.linalg.norm(f)) * 48, (n, form, err)
            f = f_next
            if np.linalg.norm(f) < 1e-6:
                break


def eigen_fnorm(lam, alpha, e):
    mu = 1.0 - lam / alpha
    return math.sqrt(float(np.sum(mu ** (2 * e))))


@pytest.mark.parametrize("order", [2, 4, 8])
def test_eigen_closed_form_fnorm_and_theta(order):
    """On A = Q diag(lam) Q^T: ||F_k||_F = sqrt(sum mu_i^{2 n^k}) with
    mu = 1 - lam / alpha (eq. fk1 with h = 1, S = alpha I), and the coupled
    Richardson iterate theta_K = theta* - Q diag(mu^{E_K}) Q^T theta* with
    E_K = (n^{K+1} - 1)/(n - 1) while above the rounding floor."""
    s = inputs.spd_qlq(64, 100.0, seed=1)
    opts = oracle.SolveOptions(order=order, form="squaring", k_max=3, floor_detect=False,
                               refine_max=0, resid_tol=0.0)
    rep = oracle.solve(s.A, s.b, opts)
    alpha = rep.alpha
    for k, fk in enumerate(rep.fnorm_hist):
        ref = eigen_fnorm(s.lam, alpha, order ** k)
        if ref > 1e-9:
            assert abs(fk - ref) <= 1e-9 * ref + 1e-12, (k, fk, ref)
    theta_star = s.Q @ ((s.Q.T @ s.b) / s.lam)
    mu = 1.0 - s.lam / alpha
    kk = rep.ns_steps
    e_k = (order ** (kk + 1) - 1) // (order - 1)
    theta_ref = theta_star - s.Q @ ((mu ** e_k) * (s.Q.T @ theta_star))
    assert np.linalg.norm(rep.theta - theta_ref) <= 1e-12 * np.linalg.norm(theta_star)


def test_diagonal_closed_form():
    """Diagonal A: G_K = diag((1 - (1 - lam/alpha)^{n^K}) / lam) (eqs. g02, fk1)."""
    lam = np.array([1.0, 2.0, 3.5, 10.0, 40.0, 100.0])
    s = inputs.spd_diag(lam, seed=3)
    alpha = oracle.alpha_frobenius(s.A)
    assert alpha == pytest.approx(math.sqrt(float(np.sum(lam ** 2))), rel=1e-15)
    for n in (2, 4, 8):
        g = np.eye(6) / alpha
        for k in range(1, 4):
            g = oracle.ns_step(s.A, g, n, "squaring")
            ref = (1.0 - (1.0 - lam / alpha) ** (n ** k)) / lam
            np.testing.assert_allclose(np.diag(g), ref, rtol=2e-15, atol=0)
            assert np.max(np.abs(g - np.diag(np.diag(g)))) == 0.0


@pytest.mark.parametrize("n,kappa,order,composite",
                         [(64, 1e2, 4, False), (64, 1e2, 8, False), (200, 1e4, 8, False),
                          (96, 1e3, 8, True), (64, 1e2, 4, True)])
def test_solution_matches_cholesky(n, kappa, order, composite):
    """theta agrees with LAPACK's Cholesky solve to ~kappa * u (the limit
    of theta itself is A^{-1} b, eq. ae1)."""
    s = inputs.spd_qlq(n, kappa, seed=7)
    rep = oracle.solve(s.A, s.b, oracle.SolveOptions(order=order, composite=composite,
                                                     resid_tol=1e-13))
    chol = scipy.linalg.cho_solve(scipy.linalg.cho_factor(s.A), s.b)
    rel = np.linalg.norm(rep.theta - chol) / np.linalg.norm(chol)
    assert rel <= 20 * kappa * np.finfo(float).eps, rel
    assert rep.rel_resid <= max(1e-12, 4 * np.linalg.norm(s.b - s.A @ chol) / np.linalg.norm(s.b))


@pytest.mark.parametrize("n,ks", [(2, (1, 2, 3)), (3, (1, 2)), (4, (1,))])
def test_double_ns_exponent_exact(n, ks):
    """eq. (ermoex1) with h = 1: F_k = J^{k n^{k+1} + n^k} and
    G_k = sum_{j < e_k} J^j exactly on the shift operand."""
    m = 64 if n != 3 else 72
    a = np.eye(m) - inputs.shift_matrix(m)
    st = oracle.dns_init(a, np.eye(m), n, "horner")
    np.testing.assert_array_equal(st.F, shift_power(m, 1))          # F_0 = Gamma_0
    np.testing.assert_array_equal(st.Gam, shift_power(m, n))        # Gamma_1 = Gamma_0^n
    for k in range(1, max(ks) + 1):
        st = oracle.dns_step(a, st, n, "horner")
        e_k = k * n ** (k + 1) + n ** k
        if k in ks:
            np.testing.assert_array_equal(st.F, shift_power(m, e_k))
            np.testing.assert_array_equal(st.G, band_ones(m, e_k))
            np.testing.assert_array_equal(st.Gam, shift_power(m, n ** (k + 1)))


@pytest.mark.parametrize("n,q,ks", [(2, 2, (1, 2, 3)), (3, 3, (1, 2)), (2, 1, (1, 2)),
                                    (4, 2, (1,))])
def test_accelerator_matrix_exact(n, q, ks):
    """eq. (redttk2) / (riem1) mirrored: I - A omega_k = F_k^q Gamma_k^n, so on
    the shift operand omega_k = sum_{j < q e_k + n^(k+1)} J^j exactly, and the
    operator applied to a vector (the solver's form) equals the matrix."""
    m = 72
    a = np.eye(m) - inputs.shift_matrix(m)
    st = oracle.dns_init(a, np.eye(m), n, "horner")
    r = np.arange(1.0, m + 1.0)
    for k in range(1, max(ks) + 1):
        st = oracle.dns_step(a, st, n, "horner")
        if k in ks:
            om = oracle.accelerator_matrix(a, st, q)
            e_k = k * n ** (k + 1) + n ** k
            np.testing.assert_array_equal(om, band_ones(m, q * e_k + n ** (k + 1)))
            np.testing.assert_array_equal(oracle.accelerator_apply(a, st, r, q), om @ r)


@pytest.mark.parametrize("n,ks", [(2, (1, 2, 3)), (3, (1, 2)), (4, (1,))])
def test_gkrecu1_recursion_exact(n, ks):
    """eq. (gkrecu1): G_k rebuilt from omega_{k-1} (eq. redttk2, q = n) with
    one product equals the double Newton-Schulz iterate of eq. (gkgen21):
    exactly on the shift operand (G_k = sum_{j < e_k} J^j), and the whole
    state (L_k, Gamma_k^n, G_k, F_k) of both steps agrees."""
    m = 64 if n != 3 else 72
    a = np.eye(m) - inputs.shift_matrix(m)
    st = oracle.dns_init(a, np.eye(m), n, "horner")
    rec = st
    for k in range(1, max(ks) + 1):
        om = oracle.accelerator_matrix(a, rec, n)
        rec = oracle.dns_step_recursive(a, rec, om, n, "horner")
        st = oracle.dns_step(a, st, n, "horner")
        e_k = k * n ** (k + 1) + n ** k
        if k in ks:
            np.testing.assert_array_equal(rec.G, band_ones(m, e_k))
            np.testing.assert_array_equal(rec.F, shift_power(m, e_k))
        for x, y in ((rec.L, st.L), (rec.Gam, st.Gam), (rec.G, st.G), (rec.F, st.F)):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("order,form", [(4, "squaring"), (8, "squaring"), (3, "horner")])
def test_gkrecu1_recursion_matches_merge_on_spd(order, form):
    """On a seeded SPD system the recursion of eq. (gkrecu1) and the merge of
    eq. (gkgen21) give the same G_k to rounding over four steps, and
    I - A omega_k = F_k^n Gamma_k^n (eq. riem3 mirrored) holds as matrices."""
    s = inputs.spd_qlq(96, 1e3, seed=17)
    g0 = np.eye(96) / oracle.alpha_frobenius(s.A)
    st = oracle.dns_init(s.A, g0, order, form)
    rec = st
    for _ in range(4):
        om = oracle.accelerator_matrix(s.A, rec, order)
        rec = oracle.dns_step_recursive(s.A, rec, om, order, form)
        st = oracle.dns_step(s.A, st, order, form)
        assert np.linalg.norm(rec.G - st.G) <= 1e-12 * np.linalg.norm(st.G)
        om = oracle.accelerator_matrix(s.A, st, order)
        lhs = np.eye(96) - s.A @ om
        rhs = np.linalg.matrix_power(st.F, order) @ st.Gam
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * max(1.0, np.linalg.norm(rhs))


def test_double_ns_eigen_closed_form():
    """||F_k||_F = sqrt(sum mu^{2 e_k}), e_k = k n^{k+1} + n^k (eq. ermoex1)."""
    s = inputs.spd_qlq(64, 1e3, seed=5)
    n = 2
    rep = oracle.solve(s.A, s.b, oracle.SolveOptions(order=n, form="squaring", composite=True,
                                                     k_max=3, floor_detect=False,
                                                     refine_max=0, resid_tol=0))
    for k, fk in enumerate(rep.fnorm_hist):
        e_k = k * n ** (k + 1) + n ** k
        ref = eigen_fnorm(s.lam, rep.alpha, e_k)
        if ref > 1e-9:
            assert abs(fk - ref) <= 1e-9 * ref, (k, fk, ref)


@pytest.mark.parametrize("composite", [False, True])
def test_richardson_mismatch_exact(composite):
    """theta_K - theta* = -(prod_k F_k) theta*: with theta_0 = G_0 b the
    mismatch is -J^{E} theta* on the shift operand, E the summed exponents
    (E = sum_{k<=K} n^k classically; sum_{k<=K} (k n^{k+1} + n^k) for the
    composite form, eqs. redttk1 and ermoex1)."""
    m, n, K = 80, 2, 3
    a = np.eye(m) - inputs.shift_matrix(m)
    rng = np.random.default_rng(0)
    b = rng.integers(-3, 4, size=m).astype(float)
    theta_star = np.linalg.solve(a, b)          # exact: unit upper triangular
    assert np.array_equal(a @ theta_star, b)
    opts = oracle.SolveOptions(order=n, form="squaring", composite=composite, k_max=K,
                               floor_detect=False, refine_max=0, resid_tol=0, scale="inf_half",
                               eps=0.0)
    # ||A||_inf / 2 = 1 here, so G_0 = I and F_0 = J exactly.
    rep = oracle.solve(a, b, opts)
    assert rep.alpha == 1.0
    if composite:
        e = sum(k * n ** (k + 1) + n ** k for k in range(0, K + 1))
    else:
        e = sum(n ** k for k in range(0, K + 1))
    np.testing.assert_array_equal(rep.theta - theta_star, -(shift_power(m, e) @ theta_star))


def test_order2_twice_equals_order4():
    """Appendix: two second-order steps equal one fourth-order step."""
    s = inputs.spd_qlq(40, 30.0, seed=9)
    alpha = oracle.alpha_frobenius(s.A)
    g0 = np.eye(40) / alpha
    g2 = oracle.ns_step(s.A, oracle.ns_step(s.A, g0, 2, "squaring"), 2, "squaring")
    g4 = oracle.ns_step(s.A, g0, 4, "squaring")
    assert np.linalg.norm(g2 - g4) <= 1e-13 * np.linalg.norm(g4)


def test_splitting_condition_and_divergence():
    """rho(I - A/alpha) < 1 iff 2 alpha I - A is positive definite (Section 2);
    a violated condition is reported as divergence."""
    s = inputs.spd_qlq(32, 10.0, seed=4)
    lmax = float(s.lam.max())
    for alpha in (0.4 * lmax, 0.6 * lmax, lmax, oracle.alpha_frobenius(s.A)):
        rho = np.max(np.abs(1.0 - s.lam / alpha))
        assert (rho < 1.0) == oracle.splitting_condition(s.A, alpha)
    assert oracle.alpha_frobenius(s.A) >= lmax
    # alpha = 0.4 lambda_max < lambda_max / 2: diverges.
    eps = 0.4 * lmax - float(np.max(np.sum(np.abs(s.A), axis=1))) / 2.0
    rep = oracle.solve(s.A, s.b, oracle.SolveOptions(order=4, scale="inf_half", eps=eps))
    assert rep.ns_stop == "diverged"
    # Indefinite matrix: diverges under the Frobenius scaling too.
    a_bad = s.A - 2.0 * np.eye(32) * s.lam.min() - np.outer(s.Q[:, 0], s.Q[:, 0]) * 5.0
    rep = oracle.solve(a_bad, s.b, oracle.SolveOptions(order=4))
    assert rep.ns_stop == "diverged"


def test_iterates_symmetric():
    """Every G_k is a polynomial in A, hence symmetric to rounding."""
    s = inputs.spd_qlq(128, 1e3, seed=12)
    alpha = oracle.alpha_frobenius(s.A)
    g = np.eye(128) / alpha
    for _ in range(4):
        g = oracle.ns_step(s.A, g, 8, "squaring")
        assert np.linalg.norm(g - g.T) <= 1e-13 * np.linalg.norm(g)


def test_stop_rule():
    chk = oracle.stop_check
    # fast contraction: continue, no probe needed
    f = [64.0, 20.0, 1.0]
    assert not oracle.floor_probe_needed(f, 2)
    assert chk(f, 0.0, 2, 64) is None
    # ratio > 1/2 and F^2 as large as F (slow mode): continue
    f = [64.0, 50.0, 10.0, 8.0]
    assert oracle.floor_probe_needed(f, 3)
    assert chk(f, 0.0, 3, 64, f_sq=7.9) is None
    # ratio > 1/2 but ||F^2|| << ||F||: rounding floor
    f = [64.0, 50.0, 10.0, 1e-3, 4e-11, 3.9e-11]
    assert chk(f, 0.0, 5, 64, f_sq=1e-20) == "floor"
    assert chk(f, 0.0, 5, 64, floor_detect=False) is None
    assert chk(f, 1e-10, 4, 64) == "f_tol"
    assert chk([1.0, 2.0], 0.0, 1, 64) == "diverged"
    assert chk([1.0, float("nan")], 0.0, 1, 64) == "diverged"
    assert chk([1.0, 0.9], 0.0, 1, 1, f_sq=0.8) == "k_max"
    with pytest.raises(ValueError):
        chk([1.0, 0.9], 0.0, 1, 64)


@pytest.mark.parametrize("c3,stalls", [(0.614, True), (0.52, True), (0.48, False),
                                       (0.343, False)])
def test_refinement_stall_rule_closed_form(c3, stalls):
    """The refinement phase's stall stop on an input whose residual history is
    known in closed form.  A = diag(1, x), b = e_2, order 2, one fixed
    Newton-Schulz step.  With mu = 1 - x/alpha, theta_0 = b/alpha leaves
    r_0 = mu e_2; the coupled update with G_1 leaves r_1 = F_1 r_0 =
    mu^3 e_2 (eq. fk1: F_1 = F_0^2), and every refinement step multiplies
    the residual by c = mu^2.  So the recorded history is mu, mu^3, mu^5, ...,
    and progress over three steps is c^3: the stall stop (less than a factor
    2 over 3 steps) fires at exactly the third refinement step when
    c^3 > 1/2, and never otherwise (then the step budget ends the run)."""
    c = c3 ** (1.0 / 3.0)
    mu = math.sqrt(c)
    d = 1.0 - mu                          # x / alpha with alpha = sqrt(1 + x^2)
    x = d / math.sqrt(1.0 - d * d)
    a = np.diag([1.0, x])
    b = np.array([0.0, 1.0])
    rep = oracle.solve(a, b, oracle.SolveOptions(order=2, k_max=1, floor_detect=False,
                                                 resid_tol=0.0, refine_max=12))
    assert rep.alpha == pytest.approx(math.sqrt(1.0 + x * x), rel=1e-15)
    want = [mu ** (2 * j + 1) for j in range(len(rep.resid_hist))]
    np.testing.assert_allclose(rep.resid_hist, want, rtol=1e-12)
    if stalls:
        assert rep.refine_stop == "refine_stall" and rep.refine_steps == 3
    else:
        assert rep.refine_stop == "refine_max" and rep.refine_steps == 12


def test_error_law_floor_rule():
    """The error-law floor test (eq. fk1: ||F_k|| <= ||F_{k-1}||^n exactly):
    fires on a norm far above ||F_{k-1}||^n, never while ||F_{k-1}|| >= 1,
    never on a composite program (order None), and needs no F^2 probe."""
    chk = oracle.stop_check
    f = [64.0, 20.0, 1.0, 4e-6, 8.8e-11]                 # 8.8e-11 >> 1e3 (4e-6)^8
    assert chk(f, 0.0, 4, 64, order=8) == "floor"
    assert not oracle.floor_probe_needed(f, 4, order=8)
    assert chk(f, 0.0, 4, 64, f_sq=1e-30) is None        # ratio test alone: continue
    assert chk(f, 0.0, 4, 64, floor_detect=False, order=8) is None
    # converging exactly: ||F_k|| at the bound is no floor
    f = [64.0, 20.0, 0.5, 0.5 ** 8]
    assert chk(f, 0.0, 3, 64, order=8) is None
    # ||F_{k-1}|| >= 1: the bound says nothing
    f = [64.0, 1.5, 1.2]
    assert chk(f, 0.0, 2, 64, f_sq=1.0, order=8) is None


def test_error_law_never_fires_on_exact_iterates():
    """On exact iterates F_k = F_{k-1}^n of symmetric F with eigenvalues in
    (-1, 1), ||F_k||_F <= ||F_{k-1}||_F^n always, so the error-law test (which
    needs a norm LAW_MARGIN times above that) cannot stop an exact iteration."""
    rng = np.random.default_rng(7)
    for _ in range(300):
        m = int(rng.integers(2, 60))
        mu = rng.uniform(-1, 1, size=m) ** int(rng.integers(1, 6))
        n = int(rng.choice([2, 3, 4, 8, 11, 45]))
        prev = float(np.sqrt(np.sum(mu ** 2)))
        cur = float(np.sqrt(np.sum((mu ** n) ** 2)))
        assert cur <= prev ** n * (1 + 1e-12) + 1e-300, (n, prev, cur)
        if prev < 1.0:
            assert not cur > oracle.LAW_MARGIN * prev ** n


def test_floor_rule_is_sound_in_exact_arithmetic():
    """For symmetric F with eigenvalues in (-1, 1) and F_k = F_{k-1}^n:
    ||F_k|| > ||F_{k-1}|| / 2 never happens together with ||F_k^2|| <= ||F_k|| / 4
    when the ratio bound of the stop rule holds, i.e. the floor test cannot
    fire on an exact iteration.  Checked on random spectra in exact-ish
    float64 (no rounding floor at these sizes)."""
    rng = np.random.default_rng(3)
    for trial in range(300):
        m = int(rng.integers(2, 40))
        mu = rng.uniform(-1, 1, size=m) ** int(rng.integers(1, 6))
        n = int(rng.choice([2, 3, 4, 8]))
        prev = np.sqrt(np.sum(mu ** 2))
        cur_mu = mu ** n
        cur = np.sqrt(np.sum(cur_mu ** 2))
        if cur < 1e-100 or prev < 1e-100:
            continue
        sq = np.sqrt(np.sum(cur_mu ** 4))
        assert not (cur > 0.5 * prev and sq <= 0.25 * cur), (mu, n)


def test_harmonic_slow_tail_not_a_floor():
    """A harmonic-regressor Gram matrix whose ||F|| ratio exceeds 1/2 while a
    slow mode persists: the solve must not stop there (it reaches 1e-10)."""
    rng = np.random.default_rng(11)
    ms = rng.integers(8, 41, size=24)
    seeds = [int(rng.integers(1 << 30)) for _ in ms]
    s = inputs.harmonic_gram(int(ms[6]), seed=seeds[6])
    rep = oracle.solve(s.A, s.b, oracle.SolveOptions(order=4, resid_tol=1e-10))
    assert rep.rel_resid <= 1e-10, (rep.ns_stop, rep.refine_stop, rep.fnorm_hist)


def test_spd64_trace_and_floor():
    """N=64, kappa=100, order 4, 12 steps: the relative residual reaches the
    1e-13 target and the ||F|| trace follows the closed form until the floor."""
    s = inputs.spd_qlq(64, 100.0, seed=1)
    rep = oracle.solve(s.A, s.b, oracle.SolveOptions(order=4, k_max=12, floor_detect=False,
                                                     resid_tol=1e-13))
    assert rep.ns_steps == 12
    assert rep.rel_resid <= 1e-13
    assert rep.mmm == 1 + 12 * 4          # F_0, then 4 mmm per step (Table 1, h=4)
    for k in range(1, 7):
        ref = eigen_fnorm(s.lam, rep.alpha, 4 ** k)
        if ref > 1e-9:
            assert rep.fnorm_hist[k] == pytest.approx(ref, rel=1e-9)
    assert max(rep.fnorm_hist[8:]) < 1e-12


@pytest.mark.parametrize("n,K,q", [(2, 1, 2), (2, 2, 2), (3, 1, 3), (2, 2, 1), (2, 1, 3)])
def test_accelerated_richardson_exponent_exact(n, K, q):
    """Eqs. (ttk1), (riem1)-(riem6): with theta_0 = L_0 b the mismatch after K
    accelerated steps is -J^{n + E} theta*, E = sum_k (q e_k + n^{k+1}),
    e_k = k n^{k+1} + n^k; for q = n, E is gamma_K of eq. (riem6)."""
    e = [k * n ** (k + 1) + n ** k for k in range(K + 1)]
    E = sum(q * e[k] + n ** (k + 1) for k in range(1, K + 1))
    if q == n:
        assert E == oracle.riem6_gamma(K, n)
    m = n + E + 8
    a = np.eye(m) - inputs.shift_matrix(m)
    rng = np.random.default_rng(1)
    b = rng.integers(-2, 3, size=m).astype(float)
    theta_star = np.linalg.solve(a, b)
    opts = oracle.SolveOptions(order=n, form="horner", composite=True, accel_q=q, k_max=K,
                               floor_detect=False, refine_max=0, resid_tol=0,
                               scale="inf_half", eps=0.0)
    rep = oracle.solve(a, b, opts)
    np.testing.assert_array_equal(rep.theta - theta_star,
                                  -(shift_power(m, n + E) @ theta_star))


def test_riem6_closed_form_values():
    """gamma_k of eq. (riem6) equals the summed per-step exponents of eq. (riem4)."""
    for n in (2, 3, 4, 8):
        for k in range(1, 6):
            direct = sum(j * n ** (j + 2) + 2 * n ** (j + 1) for j in range(1, k + 1))
            assert oracle.riem6_gamma(k, n) == direct


def test_accelerated_richardson_eigen_closed_form():
    """On A = Q diag(lam) Q^T: theta_K = theta* - Q diag(mu^{n + gamma_K}) Q^T theta*."""
    s = inputs.spd_qlq(64, 50.0, seed=3)
    n, K = 2, 2
    rep = oracle.solve(s.A, s.b, oracle.SolveOptions(order=n, composite=True, accel_q=n,
                                                     k_max=K, floor_detect=False,
                                                     refine_max=0, resid_tol=0))
    mu = 1.0 - s.lam / rep.alpha
    theta_star = s.Q @ ((s.Q.T @ s.b) / s.lam)
    ex = n + oracle.riem6_gamma(K, n)
    ref = theta_star - s.Q @ ((mu ** ex) * (s.Q.T @ theta_star))
    assert np.linalg.norm(rep.theta - ref) <= 1e-12 * np.linalg.norm(theta_star)


# --------------------------------------------------------------------------
# Section 2 diagonal preconditioner and the initial series of eq. (g01)-(g03)
# --------------------------------------------------------------------------

def test_diag_preconditioner_on_diagonal_matrix_is_exact():
    """For a diagonal A the diagonal preconditioner is A^-1: F_0 = 0 up to one
    rounding per entry and theta_0 = b / a_ii."""
    rng = np.random.default_rng(3)
    d = 10.0 ** rng.uniform(-2, 3, size=40)
    a = np.diag(d)
    b = rng.standard_normal(40)
    rep = oracle.solve(a, b, oracle.SolveOptions(order=4, scale="diag", resid_tol=1e-15))
    assert rep.fnorm_hist[0] <= 40 * np.finfo(float).eps
    assert np.allclose(rep.theta, b / d, rtol=4 * np.finfo(float).eps, atol=0)


@pytest.mark.parametrize("order", [2, 4, 8])
def test_diag_preconditioner_closed_form(order):
    """G_0 = S^-1 with S = diag(A): F_0 = I - A S^-1 is not symmetric, yet
    F_{k+1} = F_k^n holds as matrices (right orientation), and with
    A~ = S^-1/2 A S^-1/2 = Q diag(lam) Q^T the iterates are
    F_k = S^1/2 Q diag((1 - lam)^(n^k)) Q^T S^-1/2 (eq. fk1 after the
    similarity)."""
    sysm = inputs.spd_jacobi(60, seed=order)
    a = sysm.A
    s = oracle.diag_preconditioner(a)
    sh = np.sqrt(s)
    lam, q = np.linalg.eigh(a / np.outer(sh, sh))
    assert np.all(np.abs(1.0 - lam) < 1.0)              # 2S - A > 0
    g = np.diag(1.0 / s)
    f_prev = oracle.residual(a, g)
    for k in range(1, 4):
        g = oracle.ns_step(a, g, order, "squaring")
        f = oracle.residual(a, g)
        closed = (sh[:, None] * (q * (1.0 - lam) ** (order ** k)) @ q.T) / sh[None, :]
        scale = max(1.0, np.linalg.norm(closed))
        assert np.linalg.norm(f - closed) <= 1e-12 * scale * 60, k
        pw = np.linalg.matrix_power(f_prev, order)
        assert np.linalg.norm(f - pw) <= 1e-12 * max(1.0, np.linalg.norm(pw)) * 60, k
        f_prev = f


@pytest.mark.parametrize("h,p,w", [(4, 1, 2), (6, 2, 2), (3, 2, 1), (4, 0, 4), (9, 2, 3)])
def test_initial_series_power(h, p, w):
    """Eq. (g02)-(g03): G_0 = S^-1 sum_{j<h} Y^j with Y = I - A S^-1, so
    F_0 = Y^h exactly; the factorized evaluation (p, w) of eq. (g01) equals
    the plain sum."""
    sysm = inputs.spd_qlq(50, 1e2, seed=h + p)
    a = sysm.A
    alpha = oracle.alpha_frobenius(a)
    s_inv = np.eye(50) / alpha
    y = np.eye(50) - a / alpha
    g0 = oracle.initial_series(a, s_inv, h, p, w)
    plain = s_inv @ sum(np.linalg.matrix_power(y, j) for j in range(h))
    assert np.linalg.norm(g0 - plain) <= 1e-13 * np.linalg.norm(plain)
    f0 = oracle.residual(a, g0)
    yh = np.linalg.matrix_power(y, h)
    assert np.linalg.norm(f0 - yh) <= 1e-13 * max(1.0, np.linalg.norm(yh)) * 50


@pytest.mark.parametrize("h,order", [(2, 4), (3, 4), (4, 8)])
def test_initial_series_solve_exponent(h, order):
    """With the initial series of order h the iterates follow
    ||F_k||_F = sqrt(sum mu_i^(2 h n^k)) (eq. f10 and the steps after it)."""
    sysm = inputs.spd_qlq(64, 1e3, seed=11 + h)
    rep = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=order, init_order=h,
                                                           resid_tol=1e-13))
    mu = 1.0 - sysm.lam / rep.alpha
    for k, fk in enumerate(rep.fnorm_hist):
        ref = math.sqrt(float(np.sum(mu ** (2 * h * order ** k))))
        if ref > 1e-8:
            assert fk == pytest.approx(ref, rel=1e-9), k
    assert rep.rel_resid <= 1e-13


# --------------------------------------------------------------------------
# General composite expansion (eqs. gkgen1-ga1) and the [sri] algorithm of
# Remark 2
# --------------------------------------------------------------------------

@pytest.mark.parametrize("order,rates", [(2, (2,)), (4, (2, 4)), (2, (4, 2, 2)), (4, (1, 2))])
def test_general_composite_exponent(order, rates):
    """F_k = F_{k-1}^n Gamma_c as matrices (eq. gem1, mirrored) and
    ||F_k||_F = sqrt(sum mu^(2 e_k)) with e_k = n e_{k-1} + sum_i m_i^k."""
    sysm = inputs.spd_qlq(48, 1e4, seed=len(rates) * 7 + order)
    a = sysm.A
    alpha = oracle.alpha_frobenius(a)
    mu = 1.0 - sysm.lam / alpha
    st = oracle.gc_init(a, np.eye(48) / alpha, rates)
    for k in range(1, 4):
        f_prev = st.F
        st = oracle.gc_step(a, st, order, rates)
        gc = np.eye(48)
        for g_i in st.Gam:
            gc = g_i @ gc
        ref_mat = np.linalg.matrix_power(f_prev, order) @ gc
        assert np.linalg.norm(st.F - ref_mat) <= 1e-12 * max(1.0, np.linalg.norm(ref_mat)) * 48
        e = oracle.gc_exponent(k, order, rates)
        ref = math.sqrt(float(np.sum(mu ** (2 * e))))
        if ref > 1e-8:
            assert np.linalg.norm(st.F) == pytest.approx(ref, rel=1e-9), k


def test_general_composite_n_w_m_one_is_the_splitting_iteration():
    """n = w = m = 1 reduces eq. (gkgen1) to G_k = S^-1 + G_{k-1} (S^-1 D)
    (right orientation of the splitting iteration quoted after eq. ga1)."""
    sysm = inputs.spd_qlq(20, 10.0, seed=2)
    a = sysm.A
    alpha = oracle.alpha_frobenius(a)
    s_inv = np.eye(20) / alpha
    y = np.eye(20) - a / alpha
    st = oracle.gc_init(a, s_inv, (1,))
    g = s_inv.copy()
    for k in range(1, 6):
        st = oracle.gc_step(a, st, 1, (1,))
        g = s_inv + g @ y
        assert np.allclose(st.G, g, rtol=1e-14, atol=1e-18)
        assert oracle.gc_exponent(k, 1, (1,)) == k + 1


@pytest.mark.parametrize("order", [2, 4, 8])
def test_sri_error_model(order):
    """Remark 2: L_k = L_{k-1}^p and F_k = L_k F_{k-1} (mirrored), so with
    Z_0 = G_0 the exponent is E_k = 1 + p + ... + p^k."""
    sysm = inputs.spd_qlq(40, 1e4, seed=order)
    a = sysm.A
    alpha = oracle.alpha_frobenius(a)
    mu = 1.0 - sysm.lam / alpha
    st = oracle.sri_init(a, np.eye(40) / alpha)
    for k in range(1, 4):
        prev = st
        st = oracle.sri_step(a, st, order)
        lp = np.linalg.matrix_power(prev.L, order)
        assert np.linalg.norm(st.L - lp) <= 1e-12 * max(1.0, np.linalg.norm(lp)) * 40
        lf = st.L @ prev.F
        assert np.linalg.norm(st.F - lf) <= 1e-12 * max(1.0, np.linalg.norm(lf)) * 40
        e = oracle.sri_exponent(k, order)
        assert e == (order ** (k + 1) - 1) // (order - 1)
        ref = math.sqrt(float(np.sum(mu ** (2 * e))))
        if ref > 1e-8:
            assert np.linalg.norm(st.F) == pytest.approx(ref, rel=1e-9), k


@pytest.mark.parametrize("n", [2, 3, 4, 8])
def test_remark2_double_ns_exponent_exceeds_sri(n):
    """Remark 2: the double Newton-Schulz error exponent k n^(k+1) + n^k
    (eq. ermoex1) exceeds the [sri] exponent (n^(k+1) - 1) / (n - 1) from
    the first step on (the F_{k-1}^n versus F_{k-1} factor)."""
    for k in range(1, 8):
        assert k * n ** (k + 1) + n ** k > oracle.sri_exponent(k, n)


# ---------------------------------------------------------------------------
# P6: exact rational arithmetic on tiny systems
# ---------------------------------------------------------------------------

def _q_mat(rows):
    from fractions import Fraction
    return [[Fraction(v) for v in r] for r in rows]


def _q_mul(x, y):
    from fractions import Fraction
    n, m, k = len(x), len(y[0]), len(y)
    return [[sum((x[i][t] * y[t][j] for t in range(k)), Fraction(0)) for j in range(m)]
            for i in range(n)]


def _q_add(x, y):
    return [[a + b for a, b in zip(r, s)] for r, s in zip(x, y)]


def _q_eye(n):
    from fractions import Fraction
    return [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]


@pytest.mark.parametrize("rows,bvec,order,steps", [
    ([[4, 1, 0], [1, 3, 1], [0, 1, 2]], [1, -2, 3], 4, 4),
    ([[2, 1], [1, 2]], [3, 1], 8, 3),
    ([[5, 2, 1], [2, 4, 0], [1, 0, 3]], [0, 1, 1], 2, 6),
])
def test_iterates_match_exact_rationals(rows, bvec, order, steps):
    """P6: G_k and theta_k of the float64 oracle (squaring form, Richardson
    with the new G_k, theta_0 = G_0 b) against the same iteration in exact
    rational arithmetic, where P(F) is the plain sum I + F + ... + F^(n-1)
    (eq. ns) and alpha = ||A||_inf / 2 + 1/4 is rational (Section 2)."""
    from fractions import Fraction
    n = len(rows)
    Aq = _q_mat(rows)
    bq = [Fraction(v) for v in bvec]
    alpha_q = Fraction(max(sum(abs(v) for v in r) for r in rows), 2) + Fraction(1, 4)
    A = np.array(rows, dtype=np.float64)
    b = np.array(bvec, dtype=np.float64)
    alpha = oracle.alpha_inf_half(A, 0.25)
    assert alpha == float(alpha_q)
    Gq = [[Fraction(int(i == j)) / alpha_q for j in range(n)] for i in range(n)]
    thq = [v / alpha_q for v in bq]
    G = np.eye(n) / alpha
    th = G @ b
    for _ in range(steps):
        # exact: F = I - A G, P = sum_{j<order} F^j, G <- G P
        F = _q_add(_q_eye(n), [[-v for v in r] for r in _q_mul(Aq, Gq)])
        Pq, Fj = _q_eye(n), _q_eye(n)
        for _j in range(1, order):
            Fj = _q_mul(Fj, F)
            Pq = _q_add(Pq, Fj)
        Gq = _q_mul(Gq, Pq)
        rq = [bq[i] - sum(Aq[i][t] * thq[t] for t in range(n)) for i in range(n)]
        thq = [thq[i] + sum(Gq[i][t] * rq[t] for t in range(n)) for i in range(n)]
        # oracle
        G = oracle.ns_step(A, G, order, "squaring")
        th, _ = oracle.richardson_update(A, b, th, G)
        Ge = np.array([[float(v) for v in r] for r in Gq])
        te = np.array([float(v) for v in thq])
        assert np.max(np.abs(G - Ge)) <= 1e-13 * np.max(np.abs(Ge))
        assert np.max(np.abs(th - te)) <= 1e-13 * np.max(np.abs(te))
