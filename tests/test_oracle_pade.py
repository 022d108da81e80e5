"""Pins of the oracle's Pade approximant (Sec. 2.1 end, Sec. 2.4)."""
import math

import numpy as np
import pytest

import oracle


def test_rational_reproduced_exactly():
    """A rational function of degree (2, 2) is its own [2/2] (and [3/3]) approximant."""
    # f = (1 + 2z - z^2) / (1 - 0.5 z + 0.25 z^2): Taylor coefficients by long division
    num = [1.0, 2.0, -1.0]
    den = [1.0, -0.5, 0.25]
    a = np.zeros(9)
    for n in range(9):
        v = num[n] if n < 3 else 0.0
        for j in range(1, 3):
            if n - j >= 0:
                v -= den[j] * a[n - j]
        a[n] = v
    for z in (0.3, 1.0, -0.7):
        exact = (1 + 2 * z - z * z) / (1 - 0.5 * z + 0.25 * z * z)
        assert abs(oracle.pade_value(a, 2, 2, z)[0] - exact) < 1e-13
    p, q = oracle.pade_coeffs(a, 2, 2)
    np.testing.assert_allclose(q, den, atol=1e-13)
    np.testing.assert_allclose(p, num, atol=1e-13)


def test_geometric_series_beyond_radius():
    """Sum r^n with |r| > 1 (divergent) is summed exactly by any [L/M], M >= 1."""
    r = -3.7
    a = np.array([r ** n for n in range(13)])
    for L, M in [(6, 6), (5, 1), (1, 1)]:
        assert abs(oracle.pade_value(a, L, M)[0] - 1 / (1 - r)) < 1e-10


def test_exponential_closed_form():
    """[2/2] of e^z is (1 + z/2 + z^2/12)/(1 - z/2 + z^2/12): 19/7 at z = 1."""
    a = np.array([1 / math.factorial(n) for n in range(5)])
    assert abs(oracle.pade_value(a, 2, 2)[0] - 19 / 7) < 1e-14


def test_against_scipy():
    scipy_interp = pytest.importorskip("scipy.interpolate")
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = rng.normal(size=13)
        p, q = scipy_interp.pade(a, 6, 6)
        ref = p(1.0) / q(1.0)
        assert abs(oracle.pade_value(a, 6, 6)[0] - ref) < 1e-8 * max(1.0, abs(ref))


def test_singular_system_lowers_denominator():
    """A polynomial (all higher coefficients zero) gives a singular system: the rule falls to M = 0."""
    a = np.array([1.0, 2.0, 3.0] + [0.0] * 10)
    val, used, _ = oracle.pade_value(a, 6, 6)
    assert used[1] == 0 and abs(val - 6.0) < 1e-14


def test_delta_method_se_linear_case():
    """With M = 0 the value is the partial sum, so its SE is sqrt(1' C 1)."""
    rng = np.random.default_rng(1)
    a = rng.normal(size=5)
    A = rng.normal(size=(5, 5))
    cov = A @ A.T * 1e-4
    se = oracle.pade_se(a, cov, 4, 0)
    assert abs(se - math.sqrt(cov.sum())) < 1e-9
