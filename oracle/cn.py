"""ORACLE — test infrastructure, not product code.

Deterministic reference solutions on a fine grid, the way the paper validates
its probabilistic values: an implicit (Crank-Nicolson) finite-difference
scheme whose banded systems are solved directly (Sec. 2.4, before Example 1).

* :func:`cn_hierarchy` solves, in 1D, the linear hierarchy satisfied by the
  series coefficients that the trees estimate: writing the non-linearity as
  c_1 u + eps * sum_{j != 1} c_j u^j and expanding u = sum_n eps^n a_n,

      d a_n / dt = a a_n'' + c_1 a_n + sum_{j != 1} c_j [u^j]_{n-1},
      a_0(x, 0) = g(x),  a_n(x, 0) = 0  (n >= 1),

  where [u^j]_m is the eps^m coefficient of (sum_k a_k eps^k)^j.  Each vertex of
  a tree carries one factor c_j, so the trees with n splits estimate a_n
  (the partial contributions of the recursion of Sec. 2.1).
* :func:`cn_full` solves u_t = a u'' + sum_j c_j u^j itself with Newton
  iterations per Crank-Nicolson step.
* :func:`ode_hierarchy` is the same hierarchy without diffusion (constant g),
  integrated with scipy's adaptive Runge-Kutta at tight tolerance.

Boundary values are taken from :func:`ode_hierarchy` at g(+-L): far from the
query points the solution is spatially constant to within the Gaussian tails.
All results are Richardson-extrapolated in (h, dt) jointly (CN is second order
in both).
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp
from scipy.linalg import solve_banded


def _power_coeff(a_levels, j: int, m: int):
    """eps^m coefficient of (sum_k a_k eps^k)^j for arrays a_k (k <= m)."""
    if j == 0:
        return np.ones_like(a_levels[0]) if m == 0 else np.zeros_like(a_levels[0])
    # repeated truncated convolution
    cur = [a_levels[k] for k in range(m + 1)]
    for _ in range(j - 1):
        nxt = []
        for mm in range(m + 1):
            acc = np.zeros_like(a_levels[0])
            for k in range(mm + 1):
                acc = acc + cur[k] * a_levels[mm - k]
            nxt.append(acc)
        cur = nxt
    return cur[m]


def _source(levels, coef, n):
    """sum_{j != 1} c_j [u^j]_{n-1}."""
    if n == 0:
        return np.zeros_like(levels[0])
    src = np.zeros_like(levels[0])
    for j, c in enumerate(coef):
        if j == 1 or c == 0.0:
            continue
        src = src + c * _power_coeff(levels, j, n - 1)
    return src


def ode_hierarchy(g0: float, coef, t_eval, nmax: int):
    """Coefficients a_0..a_nmax(t) of the eps-expansion of u' = c_1 u + eps sum c_j u^j."""
    coef = list(coef) + [0.0] * (8 - len(coef))

    def rhs(_t, y):
        lv = [np.array([v]) for v in y]
        out = np.empty(nmax + 1)
        for n in range(nmax + 1):
            out[n] = coef[1] * y[n] + _source(lv, coef, n)[0]
        return out

    y0 = np.zeros(nmax + 1)
    y0[0] = g0
    t_eval = np.atleast_1d(np.asarray(t_eval, dtype=np.float64))
    if np.all(t_eval == 0):
        return np.repeat(y0[:, None], len(t_eval), axis=1)
    sol = solve_ivp(rhs, (0.0, float(t_eval.max())), y0, t_eval=t_eval, rtol=1e-12, atol=1e-14, method="DOP853")
    return sol.y  # (nmax+1, len(t_eval))


def _grid(xq, L, h):
    n = int(round(2 * L / h))
    xs = np.linspace(-L, L, n + 1)
    idx = np.rint((np.asarray(xq) + L) / h).astype(int)
    assert np.allclose(xs[idx], xq, atol=1e-12), "query points must lie on the grid"
    return xs, idx


def _lap_band(nint, r):
    """Banded form of I - r*D2 (D2 = second difference / h^2 folded into r)."""
    ab = np.zeros((3, nint))
    ab[0, 1:] = -r
    ab[1, :] = 1 + 2 * r
    ab[2, :-1] = -r
    return ab


def _cn_hierarchy_once(g, a_diff, coef, xq, t, nmax, L, h, dt):
    coef = list(coef) + [0.0] * (8 - len(coef))
    xs, idx = _grid(xq, L, h)
    nsteps = int(round(t / dt))
    dt = t / nsteps
    u = [g(xs)] + [np.zeros_like(xs) for _ in range(nmax)]
    times = np.linspace(0.0, t, nsteps + 1)
    bl = ode_hierarchy(float(g(np.array([-L]))[0]), coef, times, nmax)
    br = ode_hierarchy(float(g(np.array([L]))[0]), coef, times, nmax)
    r = a_diff * dt / (2 * h * h)
    c1 = coef[1]
    ab = _lap_band(len(xs) - 2, r)
    ab[1, :] -= dt / 2 * c1
    for k in range(nsteps):
        src_old = [_source(u, coef, n) for n in range(nmax + 1)]
        new = []
        for n in range(nmax + 1):
            un = u[n]
            rhs = un[1:-1] + r * (un[2:] - 2 * un[1:-1] + un[:-2]) + dt / 2 * c1 * un[1:-1]
            src_new = _source(new + [np.zeros_like(xs)] * (nmax + 1 - len(new)), coef, n) if n > 0 else 0.0
            rhs = rhs + dt / 2 * (src_old[n][1:-1] + (src_new[1:-1] if n > 0 else 0.0))
            lo, hi = bl[n, k + 1], br[n, k + 1]
            rhs[0] += r * lo
            rhs[-1] += r * hi
            sol = solve_banded((1, 1), ab, rhs)
            full = np.concatenate([[lo], sol, [hi]])
            new.append(full)
        u = new
    return np.array([lv[idx] for lv in u])  # (nmax+1, len(xq))


def cn_hierarchy(g, a_diff, coef, xq, t, nmax, L=20.0, h=1 / 32, dt=1 / 400):
    """Richardson-extrapolated CN values of a_0..a_nmax at the query points."""
    coarse = _cn_hierarchy_once(g, a_diff, coef, xq, t, nmax, L, h, dt)
    fine = _cn_hierarchy_once(g, a_diff, coef, xq, t, nmax, L, h / 2, dt / 2)
    return (4 * fine - coarse) / 3


def _cn_full_once(g, a_diff, coef, xq, t, L, h, dt):
    coef = list(coef) + [0.0] * (8 - len(coef))
    xs, idx = _grid(xq, L, h)
    nsteps = int(round(t / dt))
    dt = t / nsteps
    times = np.linspace(0.0, t, nsteps + 1)

    def f(u):
        return sum(c * u ** j for j, c in enumerate(coef) if c != 0.0)

    def fp(u):
        return sum(j * c * u ** (j - 1) for j, c in enumerate(coef) if c != 0.0 and j > 0)

    def ode_bc(g0):
        sol = solve_ivp(lambda _t, y: [f(y[0])], (0, t), [g0], t_eval=times, rtol=1e-12, atol=1e-14,
                        method="DOP853")
        return sol.y[0]

    bl = ode_bc(float(g(np.array([-L]))[0]))
    br = ode_bc(float(g(np.array([L]))[0]))
    u = g(xs)
    r = a_diff * dt / (2 * h * h)
    n = len(xs) - 2
    for k in range(nsteps):
        ui = u[1:-1]
        expl = ui + r * (u[2:] - 2 * ui + u[:-2]) + dt / 2 * f(ui)
        lo, hi = bl[k + 1], br[k + 1]
        v = ui.copy()
        for _ in range(30):
            full = np.concatenate([[lo], v, [hi]])
            res = v - r * (full[2:] - 2 * v + full[:-2]) - dt / 2 * f(v) - expl
            ab = _lap_band(n, r)
            ab[1, :] -= dt / 2 * fp(v)
            dv = solve_banded((1, 1), ab, -res)
            v = v + dv
            if np.max(np.abs(dv)) < 1e-14 * max(1.0, np.max(np.abs(v))):
                break
        u = np.concatenate([[lo], v, [hi]])
    return u[idx]


def cn_full(g, a_diff, coef, xq, t, L=20.0, h=1 / 32, dt=1 / 400):
    """Richardson-extrapolated CN solution of the full semilinear PDE."""
    coarse = _cn_full_once(g, a_diff, coef, xq, t, L, h, dt)
    fine = _cn_full_once(g, a_diff, coef, xq, t, L, h / 2, dt / 2)
    return (4 * fine - coarse) / 3
