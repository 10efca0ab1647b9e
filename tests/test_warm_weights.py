"""The warm-start weights (host logic of the library, no device): the start of
a stage solve is sum_q w_q psi(step - q), the value at the current step of the
polynomial of degree d through the same stage's solutions of the last L steps.

Pinned by what fixes them independently of the library's QR factorisation:
the interpolating weights are the alternating binomials (Lagrange weights at
0 for the nodes -1 ... -L); every weight set reproduces polynomials of degree
<= d exactly; the least-squares weights are the minimum-norm weights with that
property (numpy's SVD-based lstsq of the underdetermined system), which is
what evaluating a least-squares fit amounts to."""
import math
import os
import re

import numpy as np
import pytest

# The largest number of levels, read from the header: the library itself is
# loaded only by the fixture below, so that collecting this module (also in a
# GPU run, which deselects it) does not load the HIP runtime before torch.
_HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "include", "cavity.h")
LEVELS_MAX = int(re.search(r"CAVITY_WARM_LEVELS_MAX\s*=\s*(\d+)", open(_HEADER).read()).group(1))


@pytest.fixture(scope="module")
def cav():
    from paper_0809_3098_amd import cavity
    assert cavity.CAVITY_WARM_LEVELS_MAX == LEVELS_MAX
    return cavity


@pytest.mark.parametrize("levels", range(2, LEVELS_MAX + 1))
def test_interpolating_weights_are_alternating_binomials(cav, levels):
    w = cav.cavity_warm_weights(levels, levels - 1)
    expect = [(-1) ** (q + 1) * math.comb(levels, q) for q in range(1, levels + 1)]
    assert w.tolist() == [float(e) for e in expect]


def _all_cases():
    return [(L, d) for L in range(2, LEVELS_MAX + 1) for d in range(1, L)]


@pytest.mark.parametrize("levels,degree", _all_cases())
def test_weights_reproduce_polynomials_of_their_degree(cav, levels, degree):
    w = cav.cavity_warm_weights(levels, degree)
    q = np.arange(1, levels + 1, dtype=np.float64)
    rng = np.random.default_rng(1000 * levels + degree)
    for k in range(degree + 1):
        # the monomial t^k at t = -q extrapolated to t = 0 (1 for k = 0, else 0)
        got = float(np.dot(w, (-q) ** k))
        scale = float(np.dot(np.abs(w), q ** k))
        assert abs(got - (1.0 if k == 0 else 0.0)) <= 1e-13 * scale, (k, got)
    c = rng.standard_normal(degree + 1)
    vals = np.polynomial.polynomial.polyval(-q, c)
    assert abs(np.dot(w, vals) - c[0]) <= 1e-13 * np.dot(np.abs(w), np.abs(vals)) + 1e-15


@pytest.mark.parametrize("levels,degree", [c for c in _all_cases() if c[1] < c[0] - 1])
def test_least_squares_weights_are_the_minimum_norm_exact_weights(cav, levels, degree):
    w = cav.cavity_warm_weights(levels, degree)
    q = np.arange(1, levels + 1, dtype=np.float64)
    # constraints sum_q w_q (-q)^k = delta_k0, k = 0 ... degree, in a scaled
    # abscissa for conditioning (the solution set does not depend on it)
    t = -q / levels
    a = np.vstack([t ** k for k in range(degree + 1)])
    b = np.zeros(degree + 1)
    b[0] = 1.0
    w_min, *_ = np.linalg.lstsq(a, b, rcond=None)
    assert np.max(np.abs(w - w_min)) <= 1e-12 * np.max(np.abs(w_min)), (w, w_min)


def test_noise_gain_of_the_default_fits(cav):
    """sqrt(sum w^2), the factor by which the fit passes on independent
    tolerance-level differences of the solutions on file."""
    gain = lambda L, d: float(np.sqrt(np.sum(cav.cavity_warm_weights(L, d) ** 2)))
    assert gain(7, 6) == pytest.approx(math.sqrt(math.comb(14, 7) - 1))  # 58.6
    assert gain(6, 5) == pytest.approx(math.sqrt(math.comb(12, 6) - 1))  # 30.4
    assert 2.0 < gain(8, 3) < 3.0
    assert 9.0 < gain(8, 5) < 11.0
    assert gain(8, 5) < gain(8, 7)


@pytest.mark.parametrize("levels,degree", [(1, 1), (LEVELS_MAX + 1, 2), (5, 0), (5, 5)])
def test_out_of_range_levels_and_degrees_are_rejected(cav, levels, degree):
    with pytest.raises(cav.CavityError):
        cav.cavity_warm_weights(levels, degree)
