"""Host logic of the program chooser: step predictions from the eigen closed
form (eq. fk1) and the bucket key."""
import math

import numpy as np
import pytest

import oracle
from paper_2008_11480_amd import autotune, inputs


def test_predicted_steps_rho0():
    # rho0 = 1/2, floor 2^-53 (f_k = max(rho0^(n^k), floor)).  Order 8:
    # f_1 = 2^-8, f_2 = floor > 1e3 f_1^8 = 1e3 2^-64: the error law fires at 2.
    assert autotune.predicted_steps(8, 0.5, 2.0 ** -53) == 2
    assert autotune.predicted_steps(2, 0.5, 2.0 ** -53) == 6      # 2^6 = 64 >= 53
    # order 53 reaches the floor exactly at step 1, where the law cannot tell
    # (f_1 = 2^-53 = f_0^53): found at step 2
    assert autotune.predicted_steps(53, 0.5, 2.0 ** -53) == 2
    assert autotune.predicted_steps(4, 0.5, 0.75) == 1            # already below
    with pytest.raises(ValueError):
        autotune.predicted_steps(4, 1.0, 1e-16)


@pytest.mark.parametrize("order", [4, 8, 11, 15, 45])
def test_predicted_steps_spectrum_matches_oracle_stop(order):
    """The closed-form prediction (eq. fk1, with the oracle's own float64
    floor as the floor level) equals the step at which the oracle's stop rule
    ends the iteration."""
    sysm = inputs.spd_qlq(48, 1e3, seed=5)
    form = "table" if order in (11, 15, 45) else "squaring"
    rep = oracle.solve(sysm.A, sysm.b, oracle.SolveOptions(order=order, form=form,
                                                           resid_tol=1e-13))
    assert rep.ns_stop == "floor"
    mu = 1.0 - sysm.lam / rep.alpha
    assert autotune.predicted_steps_spectrum(order, mu, min(rep.fnorm_hist)) == rep.ns_steps


def test_bucket_and_names():
    assert autotune.bucket(4096, 1e4, 0) == (0, 12, 4)
    assert autotune.bucket(3000, 3e5, 2) == (2, 12, 5)
    assert autotune.Program(9, "unified", 2, 3).name == "unified(p=2,w=3) order 9"
    for p in autotune.CANDIDATES:
        if p.form == "unified":
            assert p.w * (p.p + 1) == p.order
        if p.form == "unified_plus1":
            assert p.w * (p.p + 1) + 1 == p.order
        if p.form == "squaring":
            assert p.order & (p.order - 1) == 0
        if p.form == "table":
            assert p.order in oracle.TABLE_ORDERS
    # efficiency index of the candidates (eq. ei) with the oracle's mmm counts
    ei = {p.name: p.order ** (1.0 / oracle.form_mmm(p.order, p.form, p.p or None, p.w or None))
          for p in autotune.CANDIDATES if p.form != "unified_plus1"}
    assert ei["table order 11"] == pytest.approx(11 ** (1 / 6))
    assert max(ei, key=ei.get) == "table order 11"
