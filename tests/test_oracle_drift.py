"""Pins of the oracle's constant drift b (L = a Lap + b.grad; an edge of duration s moves its path by
b s + sigma W_s).

(1) The heat equation with drift and Gaussian data has a closed form: the heat-evolved Gaussian moved
by -b t.  (2) With constant coefficients the value of a tree depends on the paths only at its leaves,
and every root-to-leaf path lasts exactly t, so a tree walked with drift b from x equals, node for node,
the same tree (same Philox streams) walked without drift from x + b t.  A drift applied with the wrong
sign, scaled by sqrt(s), taken from the time left instead of the edge's duration, or missing at the
leaves fails one of these.
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


@pytest.mark.parametrize("dim", [1, 2])
def test_heat_with_drift_closed_form(oracle_mod, dim):
    a, t, A, s = 0.6, 0.8, 0.9, 0.7
    c = (0.3, -0.5)[:dim]
    b = (1.3, -0.8)[:dim]
    x = (-0.4, 0.9)[:dim]
    u0 = inputs.gauss_sum([(A, c[0], c[1] if dim == 2 else 0.0, s)])
    prob = inputs.problem(dim, a, [0.0, 0.0, 0.0], u0, drift=b)
    mc = inputs.mc_params(seed=21, max_order=4, prune=0, precision=64)
    est, se = _coef0(prob, mc, list(x), t, 200_000)
    var = s * s + 2.0 * a * t
    exact = A
    for d in range(dim):
        exact *= s / math.sqrt(var) * math.exp(-(x[d] + b[d] * t - c[d]) ** 2 / (2.0 * var))
    assert abs(est - exact) <= Z * se + 1e-12, (est, exact, se)


@pytest.mark.parametrize("strategy", [0, 1])
@pytest.mark.parametrize("dim", [1, 2])
def test_drift_is_a_shift_of_the_query_point(oracle_mod, strategy, dim):
    if dim == 1:
        u0 = inputs.logistic(1.0, 1.0 / math.sqrt(6.0), 0.0, 2)
        coef = [0.0, 1.0, -1.0]
    else:
        u0 = inputs.cubic_2d_u0(4)
        coef = [0.0, 1.0, 0.0, -1.0]
    b = (0.7, -1.1)[:dim]
    t = 0.9
    x = np.array([0.35, -0.6][:dim])
    mc = inputs.mc_params(seed=17, max_order=10, prune=1, precision=64, strategy=strategy, q=0.55)
    with_drift = oracle.walk_point(inputs.problem(dim, 1.0, coef, u0, drift=b), mc, x, t, 3, 2000)
    shifted = oracle.walk_point(inputs.problem(dim, 1.0, coef, u0), mc, x + np.array(b) * t, t, 3, 2000)
    for k in ("ne", "nodes", "flags"):
        np.testing.assert_array_equal(with_drift[k], shifted[k])
    F0, F1 = np.asarray(with_drift["F"]), np.asarray(shifted["F"])
    np.testing.assert_allclose(F0, F1, rtol=1e-12, atol=1e-300)
    # and the drift does change the trees' values (it is not ignored)
    plain = oracle.walk_point(inputs.problem(dim, 1.0, coef, u0), mc, x, t, 3, 2000)
    assert np.abs(np.asarray(plain["F"]) - F0).max() > 1e-3


@pytest.mark.parametrize("strategy", [0, 1])
def test_recursive_and_explicit_stack_walkers_agree_with_drift(oracle_mod, strategy):
    prob = inputs.problem(2, 0.8, [0.1, -0.4, 0.6, -0.5], inputs.cubic_2d_u0(3), drift=(0.9, -0.4),
                          coef_mod={"beta": (0.3, 0.7), "t0": 0.2, "pow": 1})
    mc = inputs.mc_params(seed=11, max_order=10, prune=1, precision=64, strategy=strategy, q=0.55)
    nz = oracle.normalize(prob, mc)
    r = oracle.walk_point(prob, mc, np.array([[0.4, -1.2]]), 0.9, 5, 300)
    for tr in range(300):
        F, ne, nodes, flags = pure.walk_tree(nz, mc, [0.4, -1.2], 0.9, 5, tr)
        assert (ne, nodes, flags) == (int(r["ne"][tr]), int(r["nodes"][tr]), int(r["flags"][tr]))
        assert abs(F - r["F"][tr]) <= 1e-12 * max(1.0, abs(F))
