"""Pins of the oracle's domain-decomposition tail (Sec. 3): not-a-knot splines and the ADI solver.

The spline is pinned by exact reproduction of cubics (which the not-a-knot condition guarantees) and
by scipy's own not-a-knot spline; the solver by closed-form solutions of the heat equation, of a
linear reaction and of the Fisher equation's planar travelling wave, and by its second-order
convergence under refinement (a wrong boundary or mid-step treatment drops it to first order).
"""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import pdd
from paper_2402_06491_amd import inputs


# ---------------------------------------------------------------------------------- splines ----
@pytest.mark.parametrize("m", [4, 5, 9, 33])
def test_spline_reproduces_cubics(m):
    rng = np.random.default_rng(m)
    h = 0.37
    c = rng.normal(size=4)
    s_nodes = np.arange(m) * h
    y = c[0] + c[1] * s_nodes + c[2] * s_nodes ** 2 + c[3] * s_nodes ** 3
    C = pdd.spline_coefficients(y, h)
    s = rng.uniform(0, (m - 1) * h, size=200)
    exact = c[0] + c[1] * s + c[2] * s ** 2 + c[3] * s ** 3
    np.testing.assert_allclose(pdd.spline_eval(C, h, s), exact, rtol=0, atol=1e-11 * np.abs(exact).max())


@pytest.mark.parametrize("m", [4, 6, 17, 33])
def test_spline_matches_scipy_not_a_knot(m):
    rng = np.random.default_rng(100 + m)
    h = 0.5
    y = rng.normal(size=m)
    C = pdd.spline_coefficients(y, h)
    ref = CubicSpline(np.arange(m) * h, y, bc_type="not-a-knot")
    s = np.concatenate([np.arange(m) * h, rng.uniform(0, (m - 1) * h, size=300)])
    np.testing.assert_allclose(pdd.spline_eval(C, h, s), ref(s), rtol=0, atol=1e-12)


def test_spline_columns_are_independent():
    rng = np.random.default_rng(5)
    Y = rng.normal(size=(9, 3))
    C = pdd.spline_coefficients(Y, 0.25)
    s = rng.uniform(0, 2.0, size=50)
    for j in range(3):
        Cj = pdd.spline_coefficients(Y[:, j], 0.25)
        np.testing.assert_allclose(pdd.spline_eval(C, 0.25, s)[:, j], pdd.spline_eval(Cj, 0.25, s), atol=1e-14)


def test_tensor_interpolation_reproduces_bicubics_and_commutes():
    rng = np.random.default_rng(9)
    hs, ht = 0.5, 0.125
    s_nodes = np.arange(33) * hs
    t_nodes = np.arange(9) * ht
    p = rng.normal(size=4)
    q = rng.normal(size=4)
    P = lambda s: p[0] + p[1] * s + p[2] * s ** 2 + p[3] * s ** 3
    Q = lambda t: q[0] + q[1] * t + q[2] * t ** 2 + q[3] * t ** 3
    V = Q(t_nodes)[:, None] * P(s_nodes)[None, :]
    s = rng.uniform(0, 16.0, size=40)
    t = rng.uniform(0, 1.0, size=30)
    W = pdd.tensor_interpolate(V, hs, ht, s, t)
    exact = Q(t)[:, None] * P(s)[None, :]
    np.testing.assert_allclose(W, exact, rtol=0, atol=1e-10 * np.abs(exact).max())
    # arbitrary data: interpolating along t first gives the same values (the operators commute)
    V = rng.normal(size=(9, 33))
    W1 = pdd.tensor_interpolate(V, hs, ht, s, t)
    Ct = pdd.spline_coefficients(V, ht)
    cols = pdd.spline_eval(Ct, ht, t)                      # (len t, 33)
    Cs = pdd.spline_coefficients(cols.T, hs)
    W2 = pdd.spline_eval(Cs, hs, s).T
    np.testing.assert_allclose(W1, W2, rtol=0, atol=1e-12)


# ----------------------------------------------------------------------------------- solver ----
def _heat_problem(a=1.0, c1=0.0):
    return inputs.problem(2, a, [0.0, c1], inputs.const(0.0))


def _max_err(grid, prob, fn, n_steps=None):
    bd = pdd.boundary_from_function(grid, fn)
    xs, ys = pdd.grid_coords(grid)
    U0 = fn(xs[None, :], ys[:, None], 0.0)
    U = pdd.adi_solve(grid, prob, bd, U0=U0)
    return float(np.abs(U - fn(xs[None, :], ys[:, None], grid.T)).max())


def _grid(c, steps, px=2, py=2, L=4.0, T=0.5):
    return pdd.Grid(x_lo=-L, x_hi=L, y_lo=-L, y_hi=L, px=px, py=py, cx=c, cy=c, T=T, n_steps=steps,
                    ns_x=9, ns_y=9, nt=4)


def test_heat_gaussian_second_order():
    prob = _heat_problem(a=0.7)
    fn = pdd.heat_gaussian(0.7, 0.6, cx=0.4, cy=-0.3)
    e = [_max_err(_grid(c, s), prob, fn) for c, s in ((16, 8), (32, 16), (64, 32))]
    assert e[2] < 2e-3
    for a, b in zip(e, e[1:]):
        assert 3.0 < a / b < 5.5, e


def test_linear_reaction_second_order():
    prob = _heat_problem(a=1.0, c1=-0.8)
    fn = pdd.heat_gaussian(1.0, 0.8, c1=-0.8)
    e = [_max_err(_grid(c, s), prob, fn) for c, s in ((16, 8), (32, 16), (64, 32))]
    for a, b in zip(e, e[1:]):
        assert 3.0 < a / b < 5.5, e


def test_fisher_plane_wave_second_order_across_interfaces():
    """Non-linear f with a front crossing the interfaces (time-dependent data on every line)."""
    prob = inputs.problem(2, 1.0, [0.0, 1.0, -1.0], inputs.const(0.0))
    fn = pdd.fisher_plane_wave(0.5)
    e = [_max_err(_grid(c, s, px=3, py=2, L=6.0, T=0.6), prob, fn) for c, s in ((12, 12), (24, 24), (48, 48))]
    assert e[2] < 2e-3
    for a, b in zip(e, e[1:]):
        assert 3.0 < a / b < 5.5, e


def test_decomposition_only_moves_the_solution_at_discretisation_order():
    """With exact data on every line, the decomposed and the undecomposed solves approximate the same
    solution: their difference shrinks at second order too."""
    prob = inputs.problem(2, 1.0, [0.0, 1.0, -1.0], inputs.const(0.0))
    fn = pdd.fisher_plane_wave(1.1)
    diffs = []
    for c, s in ((8, 10), (16, 20), (32, 40)):
        g4 = _grid(c, s, px=2, py=2, L=4.0, T=0.4)
        g1 = _grid(2 * c, s, px=1, py=1, L=4.0, T=0.4)
        xs, ys = pdd.grid_coords(g4)
        U0 = fn(xs[None, :], ys[:, None], 0.0)
        U4 = pdd.adi_solve(g4, prob, pdd.boundary_from_function(g4, fn), U0=U0)
        U1 = pdd.adi_solve(g1, prob, pdd.boundary_from_function(g1, fn), U0=U0)
        diffs.append(float(np.abs(U4 - U1).max()))
    assert diffs[0] > 0
    for a, b in zip(diffs, diffs[1:]):
        assert a / b > 2.5, diffs


def test_node_points_layout():
    g = pdd.Grid(px=4, py=4, cx=8, cy=8, ns_x=33, ns_y=33, nt=8)
    xy, t = pdd.node_points(g)
    assert len(g.lines()) == 10 and xy.shape == (10 * 8 * 33, 2)
    # first line: x = -8, times 1/8 .. 1, nodes along y
    assert np.all(xy[:33, 0] == -8.0) and np.allclose(xy[:33, 1], np.linspace(-8, 8, 33))
    assert np.allclose(np.unique(t), np.arange(1, 9) / 8)
    gz = pdd.Grid(px=4, py=4, cx=8, cy=8, outer="zero")
    assert [c for _, _, c in gz.lines()] == [-4.0, 0.0, 4.0, -4.0, 0.0, 4.0]


def test_pdd_with_exact_node_values_is_limited_by_interpolation():
    """Node values taken from the exact Fisher wave: against the same solve fed the exact boundary data,
    the tail differs only by the interpolation error of the data, which falls with denser nodes (at
    the spline's fourth order, damped by the solve)."""
    prob = inputs.problem(2, 1.0, [0.0, 1.0, -1.0], inputs.logistic(1.0, 1.0 / math.sqrt(6.0), 0.0, 2,
                                                                  (math.cos(0.3), math.sin(0.3))))
    fn = pdd.fisher_plane_wave(0.3)
    errs = []
    for ns, nt in ((9, 4), (17, 8), (33, 16)):
        g = pdd.Grid(x_lo=-4, x_hi=4, y_lo=-4, y_hi=4, px=2, py=2, cx=32, cy=32, T=0.5, n_steps=40,
                     ns_x=ns, ns_y=ns, nt=nt)
        xy, t = pdd.node_points(g)
        vals = fn(xy[:, 0], xy[:, 1], t)
        U = pdd.pdd_solve(g, prob, vals)
        Uex = pdd.adi_solve(g, prob, pdd.boundary_from_function(g, fn))
        errs.append(float(np.abs(U - Uex).max()))
    assert errs[0] > 4 * errs[1] > 16 * errs[2], errs
    assert errs[2] < 1e-6, errs


def _second_difference(nx, ny, axis):
    """Dense second-difference operator over all (ny+1) x (nx+1) nodes (row-major, x fastest); rows
    where the difference is undefined (the first and last node along `axis`) are zero."""
    N = (nx + 1) * (ny + 1)
    D = np.zeros((N, N))
    for j in range(ny + 1):
        for i in range(nx + 1):
            k = j * (nx + 1) + i
            if axis == 0 and 0 < i < nx:
                D[k, k - 1], D[k, k], D[k, k + 1] = 1.0, -2.0, 1.0
            if axis == 1 and 0 < j < ny:
                D[k, k - (nx + 1)], D[k, k], D[k, k + (nx + 1)] = 1.0, -2.0, 1.0
    return D


@pytest.mark.parametrize("px,py", [(1, 1), (2, 2)])
def test_adi_equals_factored_crank_nicolson(px, py):
    """Adding the two half-steps gives the factored Crank-Nicolson scheme
    (I - rx/2 Dxx)(I - ry/2 Dyy) u^{n+1} = (I + rx/2 Dxx)(I + ry/2 Dyy) u^n + dt F on every subdomain,
    which holds exactly only with the intermediate boundary values derived from it.  Solved here as
    one dense system per subdomain and step, from arbitrary data on the lines."""
    rng = np.random.default_rng(7 + px)
    cx, cy, steps = 5, 4, 3
    g = pdd.Grid(x_lo=0.0, x_hi=1.0 * px, y_lo=0.0, y_hi=0.8 * py, px=px, py=py, cx=cx, cy=cy, T=0.03,
                 n_steps=steps, ns_x=4, ns_y=4, nt=1)
    prob = inputs.problem(2, 0.9, [0.3, -0.5, 0.8, -1.1], inputs.const(0.0))
    coef = [0.3, -0.5, 0.8, -1.1]
    bd = {li: rng.normal(size=(steps + 1, (g.NY if o == "v" else g.NX) + 1)) for li, (o, _, _) in enumerate(g.lines())}
    U0 = rng.normal(size=(g.NY + 1, g.NX + 1))
    got = pdd.adi_solve(g, prob, bd, U0=U0.copy())

    rx = 0.9 * g.dt / g.hx ** 2
    ry = 0.9 * g.dt / g.hy ** 2
    Dxx = _second_difference(cx, cy, 0)
    Dyy = _second_difference(cx, cy, 1)
    I = np.eye(Dxx.shape[0])
    Mnew = (I - rx / 2 * Dxx) @ (I - ry / 2 * Dyy)
    Mold = (I + rx / 2 * Dxx) @ (I + ry / 2 * Dyy)
    inner = np.array([j * (cx + 1) + i for j in range(1, cy) for i in range(1, cx)])
    outer = np.setdiff1d(np.arange(Dxx.shape[0]), inner)

    def with_lines(U, n):
        U = U.copy()
        for li, (o, k, _) in enumerate(g.lines()):
            if o == "h":
                U[k * cy, :] = bd[li][n]
        for li, (o, k, _) in enumerate(g.lines()):
            if o == "v":
                U[:, k * cx] = bd[li][n]
        return U

    U = with_lines(U0, 0)
    Uold = U.copy()
    for n in range(steps):
        F = sum(c * (1.5 * U - 0.5 * Uold) ** j for j, c in enumerate(coef))
        Unew = with_lines(np.zeros_like(U), n + 1)
        for sx in range(px):
            for sy in range(py):
                ys, xs_ = slice(sy * cy, (sy + 1) * cy + 1), slice(sx * cx, (sx + 1) * cx + 1)
                u = U[ys, xs_].ravel()
                b = Unew[ys, xs_].ravel()
                rhs = (Mold @ u + g.dt * F[ys, xs_].ravel())[inner] - (Mnew[:, outer] @ b[outer])[inner]
                sol = b.copy()
                sol[inner] = np.linalg.solve(Mnew[np.ix_(inner, inner)], rhs)
                Unew[ys, xs_] = sol.reshape(cy + 1, cx + 1)
        Uold, U = U, Unew
    np.testing.assert_allclose(got, U, rtol=0, atol=1e-12 * np.abs(U).max())


def test_time_varying_coefficient_second_order():
    """u_t = Lap u + c u^2/(t + t0) with constant data stays constant in space; the ADI then integrates the
    ODE, whose solution is 1/(1/g0 - c ln(1 + t/t0)), at second order (the coefficient is taken at the
    mid-step time)."""
    g0, c, t0 = 0.7, -1.5, 0.1
    prob = inputs.problem(2, 1.0, [0.0, 0.0, c], inputs.const(g0), coef_mod={"beta": (0.0, 0.0), "t0": t0, "pow": 1})

    def fn(X, Y, t):
        return np.full(np.broadcast(X, Y).shape, 1.0 / (1.0 / g0 - c * math.log(1.0 + t / t0)))
    # 1/(t + t0) varies on the scale t0 = 0.1, so the asymptotic ratio 4 is reached from above
    e = [_max_err(_grid(8, s, T=0.5), prob, fn) for s in (80, 160, 320)]
    for a, b in zip(e, e[1:]):
        assert 3.5 < a / b < 5.0, e


def test_space_varying_coefficient_is_applied_at_the_node():
    """beta_x > 0, beta_y = 0: against the constant coefficient, the damping u^2 term is weaker away from
    x = 0, so the field grows there, more off-centre along x than along y (a coordinate mix-up would
    reverse that), symmetrically in both axes."""
    base = {"beta": (0.0, 0.0), "t0": 0.0, "pow": 0}
    var = {"beta": (0.6, 0.0), "t0": 0.0, "pow": 0}
    g = _grid(32, 20, px=1, py=1, T=0.4)  # one subdomain: the middle row is not a line
    og = g
    u0 = inputs.gauss_sum([(0.8, 0.0, 0.0, 1.5)])
    p0 = inputs.problem(2, 1.0, [0.0, 0.0, -2.0], u0, coef_mod=base)
    p1 = inputs.problem(2, 1.0, [0.0, 0.0, -2.0], u0, coef_mod=var)
    xs, ys = pdd.grid_coords(og)
    fn = lambda X, Y, t: np.zeros(np.broadcast(X, Y).shape)
    bd = pdd.boundary_from_function(og, fn)
    U0 = pdd.g_grid(p0, xs[None, :], ys[:, None])
    d = pdd.adi_solve(og, p1, bd, U0=U0) - pdd.adi_solve(og, p0, bd, U0=U0)
    i0, j0 = len(xs) // 2, len(ys) // 2
    assert d.min() >= -1e-14
    assert d[j0, i0 + 6] > 2.0 * d[j0 + 6, i0] > 1e-3
    np.testing.assert_allclose(d, d[::-1, :], atol=1e-12)
    np.testing.assert_allclose(d, d[:, ::-1], atol=1e-12)


def test_time_varying_linear_coefficient_second_order():
    """c_1 modulated too: u_t = Lap u + c u/(t + t0) with constant data is the ODE u' = c u/(t + t0),
    u = g0 (1 + t/t0)^c; the ADI integrates it at second order (the modulation multiplies c_1 u)."""
    g0, c, t0 = 0.6, 1.4, 0.1
    prob = inputs.problem(2, 1.0, [0.0, c], inputs.const(g0),
                          coef_mod={"beta": (0.0, 0.0), "t0": t0, "pow": 1, "linear": True})

    def fn(X, Y, t):
        return np.full(np.broadcast(X, Y).shape, g0 * (1.0 + t / t0) ** c)
    e = [_max_err(_grid(8, s, T=0.5), prob, fn) for s in (80, 160, 320)]
    for a, b in zip(e, e[1:]):
        assert 3.5 < a / b < 5.0, e
