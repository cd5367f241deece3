"""Host logic of the program chooser: step predictions from the eigen closed
form (eq. fk1) and the bucket key."""
import math

import numpy as np
import pytest

import oracle
from paper_2008_11480_amd import autotune, inputs


def test_predicted_steps_rho0():
    # rho0 = 1/2, floor 2^-53: order^k >= 53 -> order 8: k = 2 (64 >= 53), +1 detect
    assert autotune.predicted_steps(8, 0.5, 2.0 ** -53) == 3
    assert autotune.predicted_steps(2, 0.5, 2.0 ** -53) == 7      # 2^6 = 64
    assert autotune.predicted_steps(53, 0.5, 2.0 ** -53) == 2     # exactly 53
    assert autotune.predicted_steps(4, 0.5, 0.75) == 1            # already below
    with pytest.raises(ValueError):
        autotune.predicted_steps(4, 1.0, 1e-16)


@pytest.mark.parametrize("order", [4, 8, 11, 15, 45])
def test_predicted_steps_spectrum_matches_oracle_iterates(order):
    """The closed-form prediction equals the step at which the oracle's
    float64 iterates first fall below the same Frobenius level (plus one)."""
    sysm = inputs.spd_qlq(48, 1e3, seed=5)
    alpha = oracle.alpha_frobenius(sysm.A)
    mu = 1.0 - sysm.lam / alpha
    level = 1e-6
    form = "table" if order in (11, 15, 45) else "squaring"
    g = np.eye(48) / alpha
    k = 0
    while np.linalg.norm(oracle.residual(sysm.A, g)) > level:
        g = oracle.ns_step(sysm.A, g, order, form)
        k += 1
    assert autotune.predicted_steps_spectrum(order, mu, level) == k + 1


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
