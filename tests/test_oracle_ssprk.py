"""Pins of the oracle's SSPRK(5,4) integrator (Sec. 3, eqs. SSPRK54_1-SSPRK54_5).

The paper prints the Shu-Osher coefficients; what fixes them independently of
any implementation is (i) consistency (each stage is a convex combination),
(ii) the eight classical fourth-order conditions, (iii) the stability
polynomial agreeing with exp(z) through z^4, and (iv) observed order four on
y' = lambda y.
"""
import os

import numpy as np
import pytest
from numpy.polynomial import Polynomial

from oracle.cavity_oracle import SSPRK54, SSPRK54_PRINTED, ssprk54_step

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ssprk54_printed.txt")


def _read_golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


def _butcher(c):
    """Butcher tableau (A, b) of the Shu-Osher form, built stage by stage.

    Stage k is y_k = y_0 + dt * sum_m A[k-1, m] F(y_m) (m < k) where F(y_m) is
    the slope evaluated at stage value m (m = 0..4).  The coefficient vector of
    a combination sum_l a_kl y_l + dt sum_l b_kl F(y_l) is
    sum_l a_kl coef(y_l) + sum_l b_kl e_l.
    """
    coef = [np.zeros(5)]                  # y_0 = y_n

    def stage(alphas, betas):
        v = np.zeros(5)
        for a, l in alphas:
            v += a * coef[l]
        for b, l in betas:
            v[l] += b
        return v

    coef.append(stage([(1.0, 0)], [(c["c10"], 0)]))
    coef.append(stage([(c["a20"], 0), (c["a21"], 1)], [(c["b21"], 1)]))
    coef.append(stage([(c["a30"], 0), (c["a32"], 2)], [(c["b32"], 2)]))
    coef.append(stage([(c["a40"], 0), (c["a43"], 3)], [(c["b43"], 3)]))
    bvec = stage([(c["a52"], 2), (c["a53"], 3), (c["a54"], 4)], [(c["b53"], 3), (c["b54"], 4)])
    A = np.array(coef[:5])                # row m: slope-weights of stage value m
    return A, bvec


def _order_defects(c):
    A, b = _butcher(c)
    cc = A.sum(axis=1)
    one = np.ones(5)
    return np.array([
        b @ one - 1.0,
        b @ cc - 1.0 / 2,
        b @ cc**2 - 1.0 / 3,
        b @ (A @ cc) - 1.0 / 6,
        b @ cc**3 - 1.0 / 4,
        b @ (cc * (A @ cc)) - 1.0 / 8,
        b @ (A @ cc**2) - 1.0 / 12,
        b @ (A @ (A @ cc)) - 1.0 / 24,
    ])


def test_printed_table_matches_golden_fixture():
    g = _read_golden()
    assert g == SSPRK54_PRINTED


def test_printed_alpha21_is_inconsistent_and_reading_fixes_it():
    p = SSPRK54_PRINTED
    assert abs(p["a20"] + p["a21"] - 1.0) == pytest.approx(3e-6, rel=1e-6)
    c = SSPRK54
    assert c["a21"] == pytest.approx(1.0 - c["a20"], abs=2e-16)
    # every other coefficient is used exactly as printed
    for k in p:
        if k not in ("a21", "c10"):
            assert c[k] == p[k]
    assert abs(c["c10"] - p["c10"]) < 5e-12


@pytest.mark.parametrize("stage_keys", [["a20", "a21"], ["a30", "a32"], ["a40", "a43"],
                                        ["a52", "a53", "a54"]])
def test_stage_consistency(stage_keys):
    assert abs(sum(SSPRK54[k] for k in stage_keys) - 1.0) < 2e-15


def test_fourth_order_conditions_hold_with_readings():
    d = _order_defects(SSPRK54)
    assert np.max(np.abs(d)) < 5e-15, d


def test_fourth_order_conditions_fail_as_printed():
    d = _order_defects(SSPRK54_PRINTED)
    assert np.max(np.abs(d)) > 1e-7


def test_nonnegative_coefficients_and_ssp_ratio():
    # strong-stability preservation needs alpha, beta >= 0; the ratios
    # alpha_kl / beta_kl bound the SSP step-size coefficient from below.
    assert all(v >= 0 for v in SSPRK54.values())
    ratios = [1.0 / SSPRK54["c10"], SSPRK54["a21"] / SSPRK54["b21"],
              SSPRK54["a32"] / SSPRK54["b32"], SSPRK54["a43"] / SSPRK54["b43"],
              SSPRK54["a53"] / SSPRK54["b53"], SSPRK54["a54"] / SSPRK54["b54"]]
    assert min(ratios) > 1.5


def _poly_step():
    z = Polynomial([0.0, 1.0])
    return ssprk54_step(
        Polynomial([1.0]), lambda y: z * y, 1.0,
        lambda ys, ks: sum((a * y for a, y in ys), Polynomial([0.0]))
        + sum((b * k for b, k in ks), Polynomial([0.0])),
        lambda y, yin: y)


def test_stability_polynomial_matches_exp_through_z4():
    R = _poly_step()
    coef = R.coef
    assert len(coef) == 6
    np.testing.assert_allclose(coef[:5], [1.0, 1.0, 0.5, 1.0 / 6, 1.0 / 24], rtol=0, atol=2e-15)
    # degree-5 term exists and is not exp's 1/120 (a 5-stage, order-4 method)
    assert 0.0 < coef[5] < 1.0 / 120


@pytest.mark.parametrize("lam", [-1.0, 1j, -1.0 + 2j])
def test_observed_order_four_on_linear_ode(lam):
    T = 1.0

    def solve(nsteps):
        y = complex(1.0)
        dt = T / nsteps
        for _ in range(nsteps):
            y = ssprk54_step(y, lambda v: lam * v, dt,
                             lambda ys, ks: sum(a * v for a, v in ys) + sum(b * k for b, k in ks),
                             lambda v, vin: v)
        return abs(y - np.exp(lam * T))

    errs = [solve(n) for n in (10, 20, 40)]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    for p in orders:
        assert 3.8 < p < 4.3, (errs, orders)
