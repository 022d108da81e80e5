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


def _taylor(num, den, n):
    """Taylor coefficients of num(z)/den(z) (den[0] = 1) by long division."""
    a = np.zeros(n)
    for k in range(n):
        v = num[k] if k < len(num) else 0.0
        for j in range(1, len(den)):
            if k - j >= 0:
                v -= den[j] * a[k - j]
        a[k] = v
    return a


def test_polynomial_keeps_a_trivial_denominator():
    """A polynomial (coefficients zero beyond degree 2) at [6/6]: the conditions have rank 2, the
    degrees drop to [2/2], whose denominator is 1 (q_1 = q_2 = 0), and the value is the sum."""
    a = np.array([1.0, 2.0, 3.0] + [0.0] * 10)
    val, used, q = oracle.pade_value(a, 6, 6)
    assert used == (2, 2) and abs(val - 6.0) < 1e-14
    np.testing.assert_array_equal(q, [1.0, 0.0, 0.0])


def test_rank_deficient_geometric_series():
    """sum r^n is the rational 1/(1 - r z) of type (0, 1): at [6/6] the 6 x 7 conditions have rank 1, so
    the degrees drop by 5 to [1/1] (the plain square solve of [6/6] would be singular) and the value is
    exact even far outside the radius of convergence."""
    for r in (-3.7, 0.4, 2.0):
        a = np.array([r ** n for n in range(13)])
        L, M, margin = oracle.pade_order(a, 6, 6)
        assert (L, M) == (1, 1) and margin > 1e3
        val, used, q = oracle.pade_value(a, 6, 6)
        assert abs(val - 1 / (1 - r)) < 1e-12 * max(1.0, abs(1 / (1 - r)))
        np.testing.assert_allclose(q, [1.0, -r], rtol=1e-13)


@pytest.mark.parametrize("L,M", [(3, 3), (4, 2), (2, 4), (6, 6)])
def test_rational_of_lower_degree_is_recovered(L, M):
    """A rational of exact type (L-1, M-1) asked at [L/M]: the conditions lose one rank, the degrees
    drop to (L-1, M-1), and numerator and denominator come back exactly."""
    rng = np.random.default_rng(10 * L + M)
    num = np.concatenate([[1.0], rng.uniform(-1, 1, L - 1)])
    roots = rng.uniform(1.6, 3.0, M - 1) * rng.choice([-1.0, 1.0], M - 1)  # poles outside |z| <= 1.5
    den = np.array([1.0])
    for rt in roots:
        den = np.convolve(den, [1.0, -1.0 / rt])
    a = _taylor(num, den, L + M + 1)
    assert oracle.pade_order(a, L, M)[:2] == (L - 1, M - 1)
    val, used, q = oracle.pade_value(a, L, M)
    exact = np.polyval(num[::-1], 1.0) / np.polyval(den[::-1], 1.0)
    assert used == (L - 1, M - 1) and abs(val - exact) < 1e-11 * max(1.0, abs(exact))
    np.testing.assert_allclose(q, den, atol=1e-11)
    # every pole is real with |z| >= 1.6: its distance from [0, 1] is |z| - 1 (z > 0) or |z| (z < 0)
    dist = min(r - 1.0 if r > 0 else -r for r in roots)
    assert oracle.pole_distance(q) == pytest.approx(dist, rel=1e-9)


def test_near_degenerate_data_decided_by_the_singular_values():
    """The same rational of type (2, 2) at [3/3] with one coefficient perturbed by delta times the
    coefficients' norm: above the rank tolerance (delta = 1e-6) the conditions have full rank and [3/3]
    stays; below it (delta = 1e-15) the degrees drop to [2/2] as for exact data."""
    num, den = [1.0, 0.5, -0.3], np.convolve([1.0, -1 / 2.0], [1.0, 1 / 2.5])
    a = _taylor(num, den, 7)
    s = np.linalg.norm(a)
    exact = sum(num) / sum(den)
    for delta, order in ((1e-6, (3, 3)), (1e-15, (2, 2))):
        b = a.copy()
        b[5] += delta * s
        L, M, margin = oracle.pade_order(b, 3, 3)
        assert (L, M) == order, (delta, L, M)
        assert margin > 10.0  # both decisions are far from the threshold 1e-12 s
        assert abs(oracle.pade_value(b, 3, 3)[0] - exact) < (1e-3 if delta > 1e-12 else 1e-12)


def test_missing_normalised_denominator_moves_along_the_antidiagonal():
    """sum z^{2k} = 1/(1 - z^2) at [1/1]: the condition a_2 q_0 + a_1 q_1 = 0 reads q_0 = 0, so no
    approximant with Q(0) = 1 exists; the rule takes [2/0], the partial sum 1 + 0 + 1."""
    a = np.array([1.0, 0.0, 1.0, 0.0, 1.0])
    val, used, _ = oracle.pade_value(a, 1, 1)
    assert used == (2, 0) and val == 2.0


def test_zero_series():
    val, used, _ = oracle.pade_value(np.zeros(13), 6, 6)
    assert used == (0, 0) and val == 0.0


def test_neighbour_orders_of_a_rational():
    """Both neighbours of [3/3] for a rational of type (2, 2) reproduce it ([2/3] and [3/2] contain
    type (2, 2)); for e^z they are the [1/2] and [2/1] closed forms at z = 1: 8/3 and 11/4."""
    num, den = [1.0, 2.0, -1.0], [1.0, -0.5, 0.25]
    a = _taylor(num, den, 7)
    exact = sum(num) / sum(den)
    lo, mo = oracle.pade_neighbours(a, 3, 3)
    assert abs(lo - exact) < 1e-12 and abs(mo - exact) < 1e-12
    e = np.array([1 / math.factorial(n) for n in range(5)])
    lo, mo = oracle.pade_neighbours(e, 2, 2)
    # [1/2] of e^z: (1 + z/3)/(1 - 2z/3 + z^2/6) -> 8/3 at z = 1; [2/1]: (1 + 2z/3 + z^2/6)/(1 - z/3) -> 11/4
    assert abs(lo - 8 / 3) < 1e-14 and abs(mo - 11 / 4) < 1e-14
    assert all(math.isnan(v) for v in oracle.pade_neighbours(e, 0, 0))


def test_pole_distance_and_flag():
    """The pole distance is the distance from [0, 1] to the nearest zero of Q; the summary flags a pole
    within 0.5 of the segment and not one on the far side of z = 0."""
    q = np.convolve([1.0, -1 / 1.2], [1.0, 1 / 4.0])  # zeros 1.2 and -4
    assert oracle.pole_distance(q) == pytest.approx(0.2, rel=1e-12)
    assert oracle.pole_distance(np.array([1.0, 0.0])) == math.inf
    qc = np.array([1.0, -1.0, 0.5])  # zeros 1 +- i: distance 1 from the segment
    assert oracle.pole_distance(qc) == pytest.approx(1.0, rel=1e-12)
    num = [1.0, 0.3]
    a = _taylor(num, q, 5)
    summ = oracle.pade_summary(a, None, 2, 2)
    # type (1, 2) lies inside [2/2] (only a drop of both degrees reduces the rank): [2/2] is exact
    assert summ["pade_order"] == (2, 2) and summ["pole"] and summ["pole_distance"] == pytest.approx(0.2, rel=1e-9)
    a = _taylor(num, np.convolve([1.0, 1 / 0.8], [1.0, 1 / 4.0]), 5)  # zeros -0.8 and -4
    summ = oracle.pade_summary(a, None, 2, 2)
    assert not summ["pole"] and summ["pole_distance"] == pytest.approx(0.8, rel=1e-9)


def test_sensitivity_is_the_gradient_weighted_by_the_coefficients():
    """kappa = sum_k |du/da_k| |a_k|; for M = 0 (the partial sum) du/da_k = 1, so kappa = sum |a_k|."""
    a = np.array([1.0, -0.5, 0.25, -0.125])
    summ = oracle.pade_summary(a, None, 3, 0)
    assert summ["kappa"] == pytest.approx(1.875, rel=1e-9) and not summ["sensitive"]


def test_delta_method_se_linear_case():
    """With M = 0 the value is the partial sum, so its SE is sqrt(1' C 1)."""
    rng = np.random.default_rng(1)
    a = rng.normal(size=5)
    A = rng.normal(size=(5, 5))
    cov = A @ A.T * 1e-4
    se = oracle.pade_se(a, cov, 4, 0)
    assert abs(se - math.sqrt(cov.sum())) < 1e-9
