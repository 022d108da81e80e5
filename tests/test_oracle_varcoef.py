"""Pins of the oracle's variable coefficients c_j(x, t) (the paper's Example 5 family).

A vertex scales its constant coefficient by exp(-beta x^2) (t + t0)^(-pow) at the split position and
the PDE time left after the split.  Pinned by (1) the closed-form epsilon-series of the spatially
constant problem u_t = eps c u^2 / (t + t0), whose coefficients are g0 (c g0 ln(1 + t/t0))^n, and (2) the
first-order coefficient of the Gaussian problem, an integral over the split time of products of heat
kernels evaluated by quadrature; a wrong evaluation point (the time before the split, or the start of
the edge instead of the split position) fails them.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import pure
from paper_2402_06491_amd import inputs

Z = 4.5


def _coefs(prob, mc, x, t, n):
    r = oracle.walk_point(prob, mc, x, t, 0, n)
    nz = oracle.normalize(prob, mc)
    m = oracle.moments(r, mc)
    a, cov = oracle.coefficients(m, nz.mu, t)
    return a, np.sqrt(np.maximum(np.diag(cov), 0.0))


@pytest.mark.parametrize("strategy", [0, 1])
def test_time_only_coefficient_series(oracle_mod, strategy):
    g0, c, t0, t = 0.8, -1.3, 0.1, 0.6
    prob = inputs.problem(1, 1.0, [0.0, 0.0, c], inputs.const(g0), coef_mod={"beta": (0.0, 0.0), "t0": t0, "pow": 1})
    mc = inputs.mc_params(seed=4, max_order=8, prune=1, precision=64, strategy=strategy, q=0.45)
    a, se = _coefs(prob, mc, [0.3], t, 400_000)
    L = math.log(1.0 + t / t0)
    for k in range(5):
        exact = g0 * (c * g0 * L) ** k
        assert abs(a[k] - exact) <= Z * se[k] + 1e-12, (k, a[k], exact, se[k])


def _a1_gaussian(A, s, a, c, beta, t0, x, t):
    """First-order coefficient of u_t = a u_xx + eps c e^{-beta x^2}/(t + t0) u^2, u0 = A e^{-x^2/(2 s^2)}."""
    def integrand(tau):
        S2 = s * s + 2.0 * a * tau                  # variance of the heat-evolved data at PDE time tau
        k = 1.0 / S2 + beta                          # w(y, tau)^2 e^{-beta y^2} = A^2 s^2/S2 e^{-k y^2}
        v = 2.0 * a * (t - tau)                      # variance of the path from the root to the split
        return (A * A * s * s / S2) / (tau + t0) / math.sqrt(1.0 + 2.0 * k * v) * math.exp(-k * x * x / (1.0 + 2.0 * k * v))
    val, _ = integrate.quad(integrand, 0.0, t, epsabs=1e-13, epsrel=1e-11)
    return c * val


@pytest.mark.parametrize("strategy", [0, 1])
@pytest.mark.parametrize("x", [0.0, 0.9, -1.7])
def test_first_order_coefficient_gaussian(oracle_mod, strategy, x):
    A, s, a, c, beta, t0, t = 0.9, 1.1, 0.7, -1.0, 0.8, 0.1, 0.5
    prob = inputs.problem(1, a, [0.0, 0.0, c], inputs.gauss_sum([(A, 0.0, 0.0, s)]),
                          coef_mod={"beta": (beta, 0.0), "t0": t0, "pow": 1})
    mc = inputs.mc_params(seed=7, max_order=6, prune=1, precision=64, strategy=strategy, q=0.5)
    a_hat, se = _coefs(prob, mc, [x], t, 400_000)
    S2 = s * s + 2.0 * a * t
    a0 = A * s / math.sqrt(S2) * math.exp(-x * x / (2.0 * S2))
    assert abs(a_hat[0] - a0) <= Z * se[0] + 1e-12
    a1 = _a1_gaussian(A, s, a, c, beta, t0, x, t)
    assert abs(a_hat[1] - a1) <= Z * se[1] + 1e-12, (a_hat[1], a1, se[1])


def test_space_only_modulation_without_time_factor(oracle_mod):
    """pow = 0: the coefficient has no time factor; the first-order coefficient is the same integral
    without 1/(tau + t0)."""
    A, s, a, c, beta, t = 0.7, 0.9, 1.0, 1.2, 0.5, 0.4
    prob = inputs.problem(1, a, [0.0, 0.0, c], inputs.gauss_sum([(A, 0.0, 0.0, s)]),
                          coef_mod={"beta": (beta, 0.0), "t0": 0.0, "pow": 0})
    mc = inputs.mc_params(seed=9, max_order=6, prune=1, precision=64)
    a_hat, se = _coefs(prob, mc, [0.4], t, 300_000)

    def integrand(tau):
        S2 = s * s + 2.0 * a * tau
        k = 1.0 / S2 + beta
        v = 2.0 * a * (t - tau)
        return (A * A * s * s / S2) / math.sqrt(1.0 + 2.0 * k * v) * math.exp(-k * 0.16 / (1.0 + 2.0 * k * v))
    a1 = c * integrate.quad(integrand, 0.0, t, epsabs=1e-13)[0]
    assert abs(a_hat[1] - a1) <= Z * se[1] + 1e-12


@pytest.mark.parametrize("strategy", [0, 1])
def test_recursive_and_explicit_stack_walkers_agree_2d(oracle_mod, strategy):
    prob = inputs.problem(2, 0.8, [0.1, -0.4, 0.6, -0.5], inputs.cubic_2d_u0(3),
                          coef_mod={"beta": (0.3, 0.7), "t0": 0.2, "pow": 1})
    mc = inputs.mc_params(seed=11, max_order=10, prune=1, precision=64, strategy=strategy, q=0.55)
    nz = oracle.normalize(prob, mc)
    x = np.array([[0.4, -1.2]])
    r = oracle.walk_point(prob, mc, x, 0.9, 5, 300)
    for tr in range(300):
        F, ne, nodes, flags = pure.walk_tree(nz, mc, [0.4, -1.2], 0.9, 5, tr)
        assert (ne, nodes, flags) == (int(r["ne"][tr]), int(r["nodes"][tr]), int(r["flags"][tr]))
        assert abs(F - r["F"][tr]) <= 1e-12 * max(1.0, abs(F))


# ---- c_1 modulated too (coef_mod "linear"): c_1(x, t) u is an arity-1 branching -------------------

@pytest.mark.parametrize("strategy", [0, 1])
def test_modulated_linear_term_time_only_series(oracle_mod, strategy):
    """u_t = a u_xx + c (t + t0)^-1 u with constant data: u = g0 exp(c L), L = ln(1 + t/t0), and the
    coefficient of n splits is the n-th term of that exponential, g0 (c L)^n / n!."""
    g0, c, t0, t = 0.8, -0.9, 0.2, 0.7
    prob = inputs.problem(1, 1.0, [0.0, c], inputs.const(g0),
                          coef_mod={"beta": (0.0, 0.0), "t0": t0, "pow": 1, "linear": True})
    mc = inputs.mc_params(seed=5, max_order=8, prune=1, precision=64, strategy=strategy, q=0.45)
    a, se = _coefs(prob, mc, [0.3], t, 400_000)
    L = math.log(1.0 + t / t0)
    for k in range(5):
        exact = g0 * (c * L) ** k / math.factorial(k)
        assert abs(a[k] - exact) <= Z * se[k] + 1e-12, (k, a[k], exact, se[k])


def _a1_linear_gaussian(A, s, a, c, beta, t0, pw, x, t):
    """First-order coefficient of u_t = a u_xx + c e^{-beta x^2} (t + t0)^-pw u, u0 = A e^{-x^2/(2 s^2)}:
    the integral over the split's PDE time tau of the heat kernel applied to c e^{-beta y^2} times the
    heat-evolved data at tau."""
    def integrand(tau):
        S2 = s * s + 2.0 * a * tau          # variance of the heat-evolved data at PDE time tau
        k = beta + 1.0 / (2.0 * S2)         # e^{-beta y^2} w(y, tau) = A s/sqrt(S2) e^{-k y^2}
        v = 2.0 * a * (t - tau)             # variance of the path from the root to the split
        time = (tau + t0) ** -pw if pw else 1.0
        return A * s / math.sqrt(S2) * time / math.sqrt(1.0 + 2.0 * k * v) * math.exp(-k * x * x / (1.0 + 2.0 * k * v))
    val, _ = integrate.quad(integrand, 0.0, t, epsabs=1e-13, epsrel=1e-11)
    return c * val


@pytest.mark.parametrize("strategy,pw", [(0, 1), (1, 0)])
@pytest.mark.parametrize("x", [0.0, 1.1])
def test_modulated_linear_term_first_order_gaussian(oracle_mod, strategy, pw, x):
    A, s, a, c, beta, t0, t = 0.9, 1.0, 0.6, 1.3, 0.7, 0.15, 0.6
    prob = inputs.problem(1, a, [0.0, c], inputs.gauss_sum([(A, 0.0, 0.0, s)]),
                          coef_mod={"beta": (beta, 0.0), "t0": t0, "pow": pw, "linear": True})
    mc = inputs.mc_params(seed=8, max_order=6, prune=1, precision=64, strategy=strategy, q=0.5)
    a_hat, se = _coefs(prob, mc, [x], t, 400_000)
    S2 = s * s + 2.0 * a * t
    assert abs(a_hat[0] - A * s / math.sqrt(S2) * math.exp(-x * x / (2.0 * S2))) <= Z * se[0] + 1e-12
    a1 = _a1_linear_gaussian(A, s, a, c, beta, t0, pw, x, t)
    assert abs(a_hat[1] - a1) <= Z * se[1] + 1e-12, (a_hat[1], a1, se[1])


@pytest.mark.parametrize("strategy", [0, 1])
def test_walkers_agree_with_modulated_linear_term_2d(oracle_mod, strategy):
    prob = inputs.problem(2, 0.8, [0.1, -0.7, 0.6, -0.5], inputs.cubic_2d_u0(2),
                          coef_mod={"beta": (0.3, 0.7), "t0": 0.2, "pow": 1, "linear": True})
    mc = inputs.mc_params(seed=19, max_order=10, prune=1, precision=64, strategy=strategy, q=0.55)
    nz = oracle.normalize(prob, mc)
    assert 1 in nz.J
    r = oracle.walk_point(prob, mc, np.array([[-0.6, 0.8]]), 0.8, 2, 300)
    for tr in range(300):
        F, ne, nodes, flags = pure.walk_tree(nz, mc, [-0.6, 0.8], 0.8, 2, tr)
        assert (ne, nodes, flags) == (int(r["ne"][tr]), int(r["nodes"][tr]), int(r["flags"][tr]))
        assert abs(F - r["F"][tr]) <= 1e-12 * max(1.0, abs(F))
