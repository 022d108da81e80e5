"""Pins of the oracle's Euler-Maruyama paths for a general L = sigma(x)^2/2 Lap + b(x).grad with
b(x) = b + B x and sigma(x) = sqrt(2a) (1 + A exp(-|x|^2/(2 w^2))): an edge of duration s takes
ceil(s/h) equal steps, step k drawing its normals from the Philox block (node, tree, point, k).

(1) When one step covers every edge the scheme is the exact increment with the coefficients frozen at
the edge's start: with constant coefficients every tree equals the exact-path tree, and with a
variable sigma and drift a single-edge problem (no non-linearity) has the closed form of a Gaussian of
mean x + b(x) t and variance sigma(x)^2 t.  (2) For an Ornstein-Uhlenbeck drift and constant sigma the
n-step scheme is linear, so its end point is exactly Gaussian with mean x (1 + Bh)^n + b h sum (1+Bh)^i
and variance sigma^2 h sum (1+Bh)^{2i}: the estimate must match that at every step size, and it tends
to the exact OU value as h -> 0.  A wrong step count, step size, normal stream or coefficient
evaluation point fails one of these.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import pure
from paper_2402_06491_amd import inputs

Z = 4.5


def _coef0(prob, mc, x, t, n):
    r = oracle.walk_point(prob, mc, x, t, 0, n)
    nz = oracle.normalize(prob, mc)
    a, cov = oracle.coefficients(oracle.moments(r, mc), nz.mu, t)
    return a[0], math.sqrt(max(cov[0, 0], 0.0))


def _gauss_expect(A, c, s, mean, var):
    """E[A exp(-(X - c)^2 / (2 s^2))] for X ~ N(mean, var)."""
    return A * s / math.sqrt(s * s + var) * math.exp(-(mean - c) ** 2 / (2.0 * (s * s + var)))


@pytest.mark.parametrize("strategy", [0, 1])
@pytest.mark.parametrize("dim", [1, 2])
def test_one_step_edges_equal_the_exact_path(oracle_mod, strategy, dim):
    u0 = inputs.logistic(1.0, 1.0 / math.sqrt(6.0), 0.0, 2) if dim == 1 else inputs.cubic_2d_u0(1)
    coef = [0.0, 1.0, -1.0] if dim == 1 else [0.0, 1.0, 0.0, -1.0]
    b = (0.6, -0.3)[:dim]
    mc = inputs.mc_params(seed=23, max_order=10, prune=1, precision=64, strategy=strategy, q=0.55)
    x = np.array([0.4, -0.2][:dim])
    exact = oracle.walk_point(inputs.problem(dim, 1.0, coef, u0, drift=b), mc, x, 0.9, 4, 1500)
    euler = oracle.walk_point(inputs.problem(dim, 1.0, coef, u0, drift=b, euler={"dt": 5.0}), mc, x, 0.9, 4, 1500)
    for k in ("ne", "nodes", "flags"):
        np.testing.assert_array_equal(exact[k], euler[k])
    np.testing.assert_allclose(euler["F"], exact["F"], rtol=1e-13, atol=1e-300)


def test_one_step_with_variable_coefficients_closed_form(oracle_mod):
    a, t, A, c, s = 0.5, 0.7, 1.1, 0.4, 0.8
    B, b0, amp, w = -0.9, 0.3, 0.6, 1.3
    x = 0.5
    prob = inputs.problem(1, a, [0.0, 0.0, 0.0], inputs.gauss_sum([(A, c, 0.0, s)]), drift=(b0,),
                          euler={"dt": 10.0, "drift_lin": (B,), "sigma_amp": amp, "sigma_width": w})
    mc = inputs.mc_params(seed=29, max_order=4, prune=0, precision=64)
    est, se = _coef0(prob, mc, [x], t, 300_000)
    sig = math.sqrt(2.0 * a) * (1.0 + amp * math.exp(-x * x / (2.0 * w * w)))
    exact = _gauss_expect(A, c, s, x + (b0 + B * x) * t, sig * sig * t)
    assert abs(est - exact) <= Z * se + 1e-12, (est, exact, se)


@pytest.mark.parametrize("steps", [3, 8, 40])
def test_ou_scheme_law_at_every_step_size(oracle_mod, steps):
    a, t, A, c, s = 0.4, 1.0, 1.0, 0.2, 0.6
    B, b0 = -1.5, 0.4
    x = 0.9
    h = t / steps
    prob = inputs.problem(1, a, [0.0, 0.0, 0.0], inputs.gauss_sum([(A, c, 0.0, s)]), drift=(b0,),
                          euler={"dt": h * (1.0 + 1e-9), "drift_lin": (B,)})
    mc = inputs.mc_params(seed=37, max_order=4, prune=0, precision=64)
    est, se = _coef0(prob, mc, [x], t, 300_000)
    g = 1.0 + B * h
    mean = x * g ** steps + b0 * h * sum(g ** i for i in range(steps))
    var = 2.0 * a * h * sum(g ** (2 * i) for i in range(steps))
    scheme = _gauss_expect(A, c, s, mean, var)
    assert abs(est - scheme) <= Z * se + 1e-12, (steps, est, scheme, se)
    # the scheme's law tends to the exact Ornstein-Uhlenbeck law at first order in h
    m_ou = x * math.exp(B * t) + b0 / B * (math.exp(B * t) - 1.0)
    v_ou = 2.0 * a * (math.exp(2.0 * B * t) - 1.0) / (2.0 * B)
    exact = _gauss_expect(A, c, s, m_ou, v_ou)
    assert abs(scheme - exact) <= 2.0 * h, (steps, scheme, exact)


@pytest.mark.parametrize("strategy", [0, 1])
def test_recursive_and_explicit_stack_walkers_agree_with_euler(oracle_mod, strategy):
    prob = inputs.problem(2, 0.8, [0.1, -0.7, 0.6, -0.5], inputs.cubic_2d_u0(2), drift=(0.3, -0.2),
                          coef_mod={"beta": (0.3, 0.7), "t0": 0.2, "pow": 1, "linear": True},
                          euler={"dt": 0.07, "drift_lin": (-0.5, 0.8), "sigma_amp": 0.4, "sigma_width": 1.5})
    mc = inputs.mc_params(seed=13, max_order=10, prune=1, precision=64, strategy=strategy, q=0.55)
    nz = oracle.normalize(prob, mc)
    r = oracle.walk_point(prob, mc, np.array([[-0.6, 0.8]]), 0.8, 2, 200)
    for tr in range(200):
        F, ne, nodes, flags = pure.walk_tree(nz, mc, [-0.6, 0.8], 0.8, 2, tr)
        assert (ne, nodes, flags) == (int(r["ne"][tr]), int(r["nodes"][tr]), int(r["flags"][tr]))
        assert abs(F - r["F"][tr]) <= 1e-12 * max(1.0, abs(F))
