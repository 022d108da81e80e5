"""Pins of the oracle's Strategy B (Sec. 2.2): coin with P(leaf) = q, uniform split times."""
import math
from math import comb

import numpy as np
import pytest
from scipy import stats

from oracle import cn, pure
from paper_2402_06491_amd import inputs

Z = 4.5


def _mc(q, **kw):
    mc = inputs.mc_params(**kw)
    mc.update(strategy=1, q=q)
    return mc


def fuss_catalan(ne, m):
    """Number of m-ary trees with ne internal nodes (the paper's diagram count N_D(Ne, m))."""
    return comb(m * ne + 1, ne) // (m * ne + 1)


def count_mary_trees(ne, m):
    """Brute-force count: an m-ary tree with ne internal nodes is a root with m subtrees whose internal
    node counts sum to ne - 1."""
    memo = {0: 1}

    def c(n):
        if n in memo:
            return memo[n]
        # number of ordered m-tuples of trees with n - 1 internal nodes in total
        ways = [1] + [0] * (n - 1)
        for _ in range(m):
            new = [0] * n
            for a in range(n):
                if ways[a]:
                    for b in range(n - a):
                        new[a + b] += ways[a] * c(b) if b < n else 0
            ways = new
        memo[n] = ways[n - 1]
        return memo[n]

    return c(ne)


@pytest.mark.parametrize("m", [2, 3, 4])
def test_fuss_catalan_counts_by_enumeration(m):
    """The paper's closed form for the number of diagrams against direct enumeration."""
    for ne in range(7):
        assert count_mary_trees(ne, m) == fuss_catalan(ne, m)


@pytest.mark.parametrize("m,q", [(2, 0.6), (3, 0.8)])
def test_tree_size_law(oracle_mod, m, q):
    """g = 1, one arity m: P(Ne = n) = q^k (1-q)^n N_D(n, m) with k = (m-1) n + 1 leaves (eq. pfinal),
    and the mean number of leaves q / (1 - m (1 - q)).  Catches the coin rule and the children count."""
    coef = [0.0] * 8
    coef[m] = 1.0
    prob = inputs.problem(1, 0.5, coef, inputs.const(1.0))
    N = 200_000
    rec = oracle_mod.walk_point(prob, _mc(q, seed=31, max_order=250, prune=0), [0.0], 1.0, 0, N)
    assert np.all(rec["flags"] == 0)
    pmf = [q ** ((m - 1) * n + 1) * (1 - q) ** n * fuss_catalan(n, m) for n in range(200)]
    kmax = max(n for n in range(200) if pmf[n] * N > 5)
    obs = np.bincount(np.minimum(rec["ne"], kmax + 1), minlength=kmax + 2)
    exp = np.array(pmf[: kmax + 1] + [max(1.0 - sum(pmf[: kmax + 1]), 0.0)]) * N
    assert stats.chisquare(obs, exp).pvalue > 1e-4
    leaves = (m - 1) * rec["ne"].astype(float) + 1
    assert abs(leaves.mean() - q / (1 - m * (1 - q))) < Z * leaves.std() / math.sqrt(N)
    assert np.array_equal(rec["nodes"], 1 + m * rec["ne"])


def _est(oracle_mod, prob, mc, x, t, n):
    res = oracle_mod.solve(prob, mc, np.atleast_2d(x), [t], [n])[0]
    return res["a"], np.sqrt(np.maximum(np.diag(res["cov"]), 0.0)), res


@pytest.mark.parametrize("t", [0.5, 1.0])
def test_fisher_series_closed_form_b(oracle_mod, t):
    """Strategy B estimates the same eps-coefficients: Fisher with constant g0 (mu = c_1, eta = t)."""
    g0 = 0.4
    prob = inputs.problem(1, 1.0, [0, 1, -1], inputs.const(g0))
    a, se, _ = _est(oracle_mod, prob, _mc(0.55, seed=32, max_order=12, prune=1), [0.0], t, 400_000)
    for n in range(7):
        ex = g0 * math.exp(t) * (-g0 * (math.exp(t) - 1)) ** n
        assert abs(a[n] - ex) < Z * se[n], n


def test_mixed_arity_b_vs_ode(oracle_mod):
    coef = [0.3, -0.4, 0.8, -0.6]
    g0, t = 0.6, 0.8
    prob = inputs.problem(1, 1.0, coef, inputs.const(g0))
    a, se, _ = _est(oracle_mod, prob, _mc(0.7, seed=33, max_order=12, prune=1), [0.0], t, 400_000)
    ex = cn.ode_hierarchy(g0, coef, [t], 6)[:, 0]
    for n in range(7):
        assert abs(a[n] - ex[n]) < Z * se[n] + 1e-14, n


def test_strategy_b_agrees_with_a(oracle_mod):
    """Both strategies estimate the same coefficients at spatially varying data (logistic, 1-D)."""
    prob = inputs.problem(1, 1.0, [0, 0.5, -1.0, 0.0, 0.5], inputs.logistic(0.8, 1.0, 0.0, 1))
    aA, sA, _ = _est(oracle_mod, prob, inputs.mc_params(seed=34), [0.5], 0.7, 300_000)
    aB, sB, _ = _est(oracle_mod, prob, _mc(0.75, seed=35), [0.5], 0.7, 300_000)
    for n in range(6):
        assert abs(aA[n] - aB[n]) < Z * math.hypot(sA[n], sB[n]), n


def test_heat_kernel_b(oracle_mod):
    """No non-linear term: every node is a leaf (q is 1), so B reduces to the heat kernel."""
    g = inputs.gauss_sum([(1 / math.sqrt(4 * math.pi), 0.0, 0.0, math.sqrt(2.0))])
    prob = inputs.problem(1, 1.0, [0, 0, 0], g)
    a, se, res = _est(oracle_mod, prob, _mc(0.5, seed=36), [1.0], 0.5, 100_000)
    exact = math.exp(-1.0 / (4 * 1.5)) / math.sqrt(4 * math.pi * 1.5)
    assert res["moments"]["nodes"] == 100_000
    assert abs(a[0] - exact) < Z * se[0]


@pytest.mark.parametrize("case", range(3))
def test_recursive_vs_explicit_stack_b(oracle_mod, case):
    probs = [
        (inputs.problem(1, 1.0, [0, 1, -1], inputs.logistic(1, 1 / math.sqrt(6), 0, 2)), 0.55, dict(max_order=6)),
        (inputs.problem(2, 1.0, [0, 1, 0, -1], inputs.cubic_2d_u0(0)), 0.75, dict(max_order=12, prune=0)),
        (inputs.problem(1, 1.0, [0.3, -0.2, 0.5, 0.0, -0.7, 0.2], inputs.logistic(0.5, 1, 0, 1)), 0.8,
         dict(max_order=12, node_cap=9)),
    ]
    prob, q, extra = probs[case]
    mc = _mc(q, seed=200 + case, **extra)
    nz = oracle_mod.normalize(prob, mc)
    rng = np.random.default_rng(case)
    n = 300
    x = rng.uniform(-2, 2, size=(n, prob["dim"]))
    t = rng.uniform(0.0, 1.5, size=n)
    pid = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    tid = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    rec = oracle_mod.walk(prob, mc, x, t, pid, tid)
    for i in range(n):
        F, ne, nodes, flags = pure.walk_tree(nz, mc, list(x[i]), float(t[i]), int(pid[i]), int(tid[i]))
        assert (rec["ne"][i], rec["nodes"][i], rec["flags"][i]) == (ne, nodes, flags), i
        assert abs(rec["F"][i] - F) <= 1e-13 * max(abs(F), 1e-300), i
