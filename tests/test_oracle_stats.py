"""Pins of the oracle's statistics and of the cos^2 initial-data family (no GPU).

* The covariance of the coefficient estimates (oracle.coefficients) and the delta-method standard error
  of the Pade value (oracle.pade_se, M > 0) are checked against the spread of independent replicas: the
  same point estimated again and again with different Philox keys (Sec. 2.4: the statistical error of
  the sample mean propagates into the Pade coefficients and the value).
* The cos^2 bump of Example 4 is checked at f = 0, where every tree is one leaf and u = E[g(x + sigma W_t)],
  against numerical integration over the Gaussian law.

Replica counts are fixed and the seeds too, so every check is deterministic; the bands are 4.5 standard
errors of the compared statistic.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2402_06491_amd import inputs

Z = 4.5


def _replicas(oracle_mod, prob, mc, x, t, n, reps, seed0=1000):
    out = []
    for r in range(reps):
        m = dict(mc, seed=seed0 + r)
        out.append(oracle_mod.solve(prob, m, np.atleast_2d(x), [t], [n])[0])
    return out


def _fisher():
    return inputs.problem(1, 1.0, [0.0, 1.0, -1.0], inputs.logistic(A=1.0, s=1 / math.sqrt(6), p=2))


def test_coefficient_covariance_against_replicas(oracle_mod):
    """The predicted Cov(a_n, a_m) = e^{2 mu t} (delta_nm S2_n/N - m_n m_m)/(N - 1), averaged over 400
    replicas of 2000 trees, against the empirical covariance of the 400 coefficient vectors.

    The problem is u_t = u_xx/2 + u^2 - u with constant g: a tree's value g^{n+1} depends on its bin n
    only, so the bins compete for the same trees and their estimates are strongly anti-correlated.
    Catches: a dropped cross term -m_n m_m, a missing e^{2 mu t} or 1/N, S2 taken as (sum F)^2, a variance
    of the trees instead of their mean."""
    mc = inputs.mc_params(max_order=6, prune=0, pade=(3, 3), precision=64)
    prob = inputs.problem(1, 0.5, [0.0, -1.0, 1.0], inputs.const(0.7))
    reps = _replicas(oracle_mod, prob, mc, [0.0], 0.3, 2000, 400)
    A = np.array([r["a"][:7] for r in reps])
    pred = np.mean([r["cov"][:7, :7] for r in reps], axis=0)
    emp = np.cov(A, rowvar=False)
    R = len(reps)
    for n in range(4):  # bins with enough trees for a Gaussian sample mean
        rel = emp[n, n] / pred[n, n]
        assert abs(rel - 1.0) < Z * math.sqrt(2.0 / (R - 1)), (n, rel)
    for n, m in ((0, 1), (0, 2), (1, 2)):
        rp = pred[n, m] / math.sqrt(pred[n, n] * pred[m, m])
        re = emp[n, m] / math.sqrt(emp[n, n] * emp[m, m])
        assert rp < -0.1, (n, m, rp)  # the cross term matters at this point
        assert abs(re - rp) < Z * (1 - rp * rp) / math.sqrt(R), (n, m, re, rp)
    # the partial sum's variance needs every cross term
    s_pred = float(np.ones(7) @ pred @ np.ones(7))
    s_emp = float(np.var(A.sum(axis=1), ddof=1))
    assert abs(s_emp / s_pred - 1.0) < Z * math.sqrt(2.0 / (R - 1)), (s_emp, s_pred)


@pytest.mark.parametrize("L,M,t", [(2, 1, 1.0), (1, 1, 1.5)])
def test_pade_se_against_replicas(oracle_mod, L, M, t):
    """The delta-method SE of the [L/M] value (M > 0), averaged over 200 replicas of 20000 trees,
    against the standard deviation of the 200 values.  The orders are ones whose denominator the data
    determine well at this point (the pole stays far from [0, 1] in every replica), the regime where a
    first-order propagation of the coefficients' noise holds.

    Catches: a wrong or incomplete gradient of the approximant (its dependence through the denominator),
    the covariance slips above, an SE of the partial sum instead of the Pade value."""
    mc = inputs.mc_params(max_order=L + M, prune=1, pade=(L, M), precision=64)
    reps = _replicas(oracle_mod, _fisher(), mc, [0.0], t, 20000, 200)
    vals = np.array([r["pade"] for r in reps])
    ses = np.array([r["pade_se"] for r in reps])
    assert all(r["pade_order"] == (L, M) for r in reps)
    assert not any(r["pole"] or r["sensitive"] for r in reps)  # the delta method's regime
    R = len(vals)
    ratio = np.std(vals, ddof=1) / np.mean(ses)
    assert abs(ratio - 1.0) < Z * math.sqrt(1.0 / (2 * (R - 1))), ratio
    # and the SE of the value is not the SE of the partial sum at this point
    psum_se = np.mean([math.sqrt(np.ones(L + M + 1) @ r["cov"][:L + M + 1, :L + M + 1] @ np.ones(L + M + 1))
                       for r in reps])
    assert abs(psum_se / np.mean(ses) - 1.0) > 0.05


def _cos2_mean_1d(x, s, A_half):
    """E[cos^2(pi (x + s Z) / (2 A_half)) 1{|x + s Z| <= A_half}] by adaptive quadrature over the support."""
    k = math.pi / (2 * A_half)

    def f(y):
        return math.cos(k * y) ** 2 * math.exp(-0.5 * ((y - x) / s) ** 2) / (s * math.sqrt(2 * math.pi))

    return integrate.quad(f, -A_half, A_half, epsabs=1e-13, epsrel=1e-12, limit=200)[0]


@pytest.mark.parametrize("dim", [1, 2])
def test_cos2_bump_at_f_zero(oracle_mod, dim):
    """f = 0: u(x, t) = E[g(x + sqrt(2a) W_t)] with g the cos^2 bump of Example 4 (separable in 2-D).

    Catches: cos instead of cos^2, a wrong half-width scaling (pi x / (2 A_x)), a missing cut-off outside
    the box, the y factor using A_x."""
    amp, ax, ay, a, t = 0.8, 1.5, 2.5, 0.7, 0.6
    u0 = {"u0_kind": "cos2_bump", "u0_params": [amp, ax, ay]}
    prob = inputs.problem(dim, a, [0.0], u0)
    mc = inputs.mc_params(seed=9, max_order=0, prune=0, pade=(0, 0), precision=64)
    s = math.sqrt(2 * a * t)
    pts = [(0.0, 0.0), (1.1, -1.9), (-1.8, 2.2)] if dim == 2 else [(0.0,), (1.2,), (-1.9,), (2.4,)]
    for x in pts:
        exact = amp * _cos2_mean_1d(x[0], s, ax) * (_cos2_mean_1d(x[1], s, ay) if dim == 2 else 1.0)
        res = oracle_mod.solve(prob, mc, np.atleast_2d(x), [t], [100_000])[0]
        est = res["a"][0]
        se = math.sqrt(res["cov"][0, 0])
        assert abs(est - exact) < Z * se + 1e-12, (x, est, exact, se)
        assert se < 0.02 * max(exact, 0.05)  # the check has teeth
