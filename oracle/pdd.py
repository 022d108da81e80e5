"""Oracle for the domain-decomposition tail (Sec. 3): interface interpolation and subdomain solves.

TEST INFRASTRUCTURE.  Plain FP64 CPU reference; only tests/, the smoke check and the bench's CPU
baseline use it.  It shares nothing with the HIP path.

The probabilistic part gives u at a few nodes on lines of the space-time domain; the tail turns those
values into boundary data and solves the decoupled subdomain problems (Sec. 3, "Interpolation" and
"Local solver").  Readings taken here (the paper names the ingredients, not the formulas):

* Lines.  The domain [x_lo, x_hi] x [y_lo, y_hi] is cut into px x py equal subdomains.  Every cut and
  every outer edge is a line: vertical lines x = x_lo + k Lx/px (k = 0..px) carry nodes uniform in y,
  horizontal lines y = y_lo + k Ly/py carry nodes uniform in x, at the times t_k = k T / nt
  (k = 1..nt); at t = 0 the node values are u0.  Outer edges may instead be held at zero.
* Interpolation.  On each line, the tensor product of 1-D not-a-knot cubic splines over the uniform
  nodes in s (the coordinate along the line) and in t: first along s for every time row, then along
  t (the two 1-D operators commute in exact arithmetic).  A node shared by a vertical and a
  horizontal line takes the vertical line's value.
* Local solver.  Crank-Nicolson in its Peaceman-Rachford ADI form on the fine grid (cell sizes hx, hy,
  step dt), for u_t = a (u_xx + u_yy) + f(u), f(u) = sum_j c_j u^j.  f is taken at the extrapolated
  mid-step value (3 u^n - u^{n-1}) / 2 (u^{-1} = u^0), which keeps second order:
      (I - rx/2 dxx) u*      = (I + ry/2 dyy) u^n + dt/2 F
      (I - ry/2 dyy) u^{n+1} = (I + rx/2 dxx) u*  + dt/2 F,      rx = a dt/hx^2, ry = a dt/hy^2,
  with dxx, dyy the second differences.  Boundary nodes hold the interpolated data at every time
  level; the intermediate level's boundary values on the lines that bound the x-sweeps follow from
  adding the two half-steps:  u*_b = (I + ry/2 dyy) g^n / 2 + (I - ry/2 dyy) g^{n+1} / 2.
  With variable coefficients c_j(x, t) = c_j exp(-bx x^2 - by y^2) (t + t0)^-pow the non-linear part of f
  is taken at the node and at the mid-step time (n + 1/2) dt: F = c_1 u~ + (e^{-bx x^2} e^{-by y^2})
  (t_mid + t0)^-pow sum_{j != 1} c_j u~^j.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.linalg import solve_banded


# ------------------------------------------------------------------------------- splines -------
def spline_matrix(m, h):
    """The defining linear system of the not-a-knot cubic spline through m >= 4 uniform nodes.

    Unknowns: per interval k (k = 0..m-2) the coefficients (a, b, c, d) of
    S_k(s) = a + b (s - s_k) + c (s - s_k)^2 + d (s - s_k)^3.  Rows: S_k matches the data at both
    ends of its interval; S' and S'' are continuous at the m-2 interior knots; S''' is continuous at
    the second and the second-to-last knot (not-a-knot).  Returns (A, rows_of_data) where the data
    vector y enters the right-hand side as r[rows_of_data[i]] = y[i] (twice for interior nodes).
    """
    if m < 4:
        raise ValueError("the not-a-knot spline needs at least 4 nodes")
    n = m - 1
    A = np.zeros((4 * n, 4 * n))
    data_rows = [[] for _ in range(m)]
    row = 0
    for k in range(n):
        A[row, 4 * k] = 1.0
        data_rows[k].append(row)
        row += 1
        A[row, 4 * k: 4 * k + 4] = [1.0, h, h * h, h * h * h]
        data_rows[k + 1].append(row)
        row += 1
    for k in range(1, n):
        A[row, 4 * (k - 1): 4 * k] = [0.0, 1.0, 2.0 * h, 3.0 * h * h]
        A[row, 4 * k + 1] = -1.0
        row += 1
        A[row, 4 * (k - 1): 4 * k] = [0.0, 0.0, 2.0, 6.0 * h]
        A[row, 4 * k + 2] = -2.0
        row += 1
    A[row, 3] = 1.0
    A[row, 7] = -1.0
    row += 1
    A[row, 4 * (n - 2) + 3] = 1.0
    A[row, 4 * (n - 1) + 3] = -1.0
    row += 1
    assert row == 4 * n
    return A, data_rows


def spline_coefficients(Y, h):
    """Not-a-knot spline coefficients for data Y of shape (m, ...) at nodes s_i = i h.

    Returns C of shape (m-1, 4, ...): C[k] = (a, b, c, d) of interval k, for every trailing column.
    """
    Y = np.asarray(Y, dtype=np.float64)
    m = Y.shape[0]
    A, data_rows = spline_matrix(m, h)
    R = np.zeros((A.shape[0],) + Y.shape[1:])
    for i, rows in enumerate(data_rows):
        for r in rows:
            R[r] = Y[i]
    C = np.linalg.solve(A, R.reshape(A.shape[0], -1))
    return C.reshape((m - 1, 4) + Y.shape[1:])


def spline_eval(C, h, s):
    """Evaluate the spline with coefficients C (from spline_coefficients) at positions s (relative
    to the first node); positions outside [0, (m-1) h] use the end intervals' cubics."""
    s = np.asarray(s, dtype=np.float64)
    n = C.shape[0]
    k = np.clip(np.floor(s / h).astype(np.int64), 0, n - 1)
    ds = s - k * h
    a, b, c, d = (C[k, j] for j in range(4))
    if C.ndim > 2:  # trailing data columns: broadcast the positions over them
        ds = ds.reshape(ds.shape + (1,) * (C.ndim - 2))
    return a + ds * (b + ds * (c + ds * d))


def tensor_interpolate(V, hs, ht, s, t):
    """Tensor-product not-a-knot interpolation of V[k_t, i_s] (time rows k_t = 0..nt at k_t ht,
    nodes i_s at i_s hs) at all pairs of positions s (relative to the first node) and times t:
    returns W[len(t), len(s)].  First along s for every time row, then along t."""
    V = np.asarray(V, dtype=np.float64)
    Cs = spline_coefficients(V.T, hs)              # (ns-1, 4, nt+1): one spline per time row
    rows = spline_eval(Cs, hs, s)                  # (len(s), nt+1)
    Ct = spline_coefficients(rows.T, ht)           # (nt, 4, len(s)): one spline per position
    return spline_eval(Ct, ht, t)                  # (len(t), len(s))


# ------------------------------------------------------------------------------- geometry ------
@dataclass
class Grid:
    x_lo: float = -8.0
    x_hi: float = 8.0
    y_lo: float = -8.0
    y_hi: float = 8.0
    px: int = 4           # subdomains along x
    py: int = 4           # subdomains along y
    cx: int = 512         # fine cells per subdomain along x
    cy: int = 512         # fine cells per subdomain along y
    T: float = 1.0
    n_steps: int = 1000
    ns_x: int = 33        # nodes on a horizontal line (uniform in x over [x_lo, x_hi])
    ns_y: int = 33        # nodes on a vertical line (uniform in y)
    nt: int = 8           # node time levels k T / nt, k = 1..nt
    outer: str = "mc"     # "mc": outer edges are lines with nodes; "zero": held at 0

    @property
    def NX(self):
        return self.px * self.cx

    @property
    def NY(self):
        return self.py * self.cy

    @property
    def hx(self):
        return (self.x_hi - self.x_lo) / self.NX

    @property
    def hy(self):
        return (self.y_hi - self.y_lo) / self.NY

    @property
    def dt(self):
        return self.T / self.n_steps

    def lines(self):
        """[(orientation, k, coordinate)]: vertical lines first ('v', k, x_k), then horizontal."""
        ks_x = range(self.px + 1) if self.outer == "mc" else range(1, self.px)
        ks_y = range(self.py + 1) if self.outer == "mc" else range(1, self.py)
        out = [("v", k, self.x_lo + k * (self.x_hi - self.x_lo) / self.px) for k in ks_x]
        out += [("h", k, self.y_lo + k * (self.y_hi - self.y_lo) / self.py) for k in ks_y]
        return out

    def line_nodes(self, orient):
        """Nodes s_lo + i h_s, h_s = (line length) / (ns - 1): the uniform nodes at spacing h_s."""
        if orient == "v":
            return self.y_lo + np.arange(self.ns_y) * ((self.y_hi - self.y_lo) / (self.ns_y - 1))
        return self.x_lo + np.arange(self.ns_x) * ((self.x_hi - self.x_lo) / (self.ns_x - 1))


def node_points(grid: Grid):
    """The Monte Carlo query points: line by line, time level k = 1..nt, node along the line.
    Returns (xy[n, 2], t[n])."""
    xy, ts = [], []
    for orient, _, c in grid.lines():
        s = grid.line_nodes(orient)
        for k in range(1, grid.nt + 1):
            tk = k * grid.T / grid.nt
            for si in s:
                xy.append((c, si) if orient == "v" else (si, c))
                ts.append(tk)
    return np.array(xy, dtype=np.float64).reshape(-1, 2), np.array(ts, dtype=np.float64)


# ---------------------------------------------------------------------------- initial data -----
def g_grid(problem, X, Y):
    """u0 of a problem dict (2-D) at arrays of positions, FP64 (same families as the walker's)."""
    kind = problem["u0_kind"]
    p = [float(v) for v in problem["u0_params"]]
    if kind in ("const", 0):
        return np.full(np.broadcast(X, Y).shape, p[0])
    if kind in ("logistic", 1):
        nx = X * p[4] + Y * p[5]
        return p[0] * (1.0 / (1.0 + np.exp(p[1] * (nx - p[2])))) ** int(p[3])
    if kind in ("gauss_sum", 2):
        out = np.zeros(np.broadcast(X, Y).shape)
        for k in range(int(problem["u0_nterms"])):
            A, cx, cy, s = p[4 * k: 4 * k + 4]
            out += A * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * s * s))
        return out
    if kind in ("cos2_bump", 3):
        inside = (np.abs(X) <= p[1]) & (np.abs(Y) <= p[2])
        v = p[0] * np.cos(np.pi * X / (2 * p[1])) ** 2 * np.cos(np.pi * Y / (2 * p[2])) ** 2
        return np.where(inside, v, 0.0)
    raise ValueError(kind)


# ---------------------------------------------------------------------------- boundary data ----
def boundary_data(grid: Grid, problem, node_values):
    """Interpolated Dirichlet data on every line at every fine time level.

    node_values: Monte Carlo values in the order of node_points.  Returns {line index:
    W[n_steps+1, fine nodes along the line]} in the order of grid.lines().
    """
    node_values = np.asarray(node_values, dtype=np.float64)
    out = {}
    pos = 0
    t_fine = np.arange(grid.n_steps + 1) * grid.dt
    ht = grid.T / grid.nt
    for li, (orient, _, c) in enumerate(grid.lines()):
        s = grid.line_nodes(orient)
        ns = len(s)
        V = np.empty((grid.nt + 1, ns))
        V[0] = g_grid(problem, np.full(ns, c), s) if orient == "v" else g_grid(problem, s, np.full(ns, c))
        V[1:] = node_values[pos: pos + grid.nt * ns].reshape(grid.nt, ns)
        pos += grid.nt * ns
        if orient == "v":
            fine = np.arange(grid.NY + 1) * grid.hy
            hs = (grid.y_hi - grid.y_lo) / (grid.ns_y - 1)
        else:
            fine = np.arange(grid.NX + 1) * grid.hx
            hs = (grid.x_hi - grid.x_lo) / (grid.ns_x - 1)
        out[li] = tensor_interpolate(V, hs, ht, fine, t_fine)
    assert pos == len(node_values)
    return out


def boundary_from_function(grid: Grid, fn):
    """Exact Dirichlet data fn(x, y, t) on every line (for pins with a known solution)."""
    out = {}
    for li, (orient, _, c) in enumerate(grid.lines()):
        W = np.empty((grid.n_steps + 1, (grid.NY if orient == "v" else grid.NX) + 1))
        for n in range(grid.n_steps + 1):
            tn = n * grid.dt
            if orient == "v":
                ys = grid.y_lo + np.arange(grid.NY + 1) * grid.hy
                W[n] = fn(np.full_like(ys, c), ys, tn)
            else:
                xs = grid.x_lo + np.arange(grid.NX + 1) * grid.hx
                W[n] = fn(xs, np.full_like(xs, c), tn)
        out[li] = W
    return out


def _set_boundary(grid: Grid, U, bd, n):
    """Write time level n of the boundary data into the field U[NY+1, NX+1] (vertical lines last, so
    they win at shared nodes); outer edges without lines are held at zero."""
    lines = grid.lines()
    if grid.outer == "zero":
        U[0, :] = 0.0
        U[-1, :] = 0.0
        U[:, 0] = 0.0
        U[:, -1] = 0.0
    for li, (orient, k, _) in enumerate(lines):
        if orient == "h":
            U[k * grid.cy, :] = bd[li][n]
    for li, (orient, k, _) in enumerate(lines):
        if orient == "v":
            U[:, k * grid.cx] = bd[li][n]


# ---------------------------------------------------------------------------------- solver -----
def f_poly(coef, u):
    out = np.zeros_like(u)
    for j in range(len(coef) - 1, -1, -1):
        out = out * u + coef[j]
    return out


def adi_solve(grid: Grid, problem, bd, U0=None, n_steps=None):
    """Peaceman-Rachford ADI (the CN form stated in the module docstring) on every subdomain.

    bd: boundary data as returned by boundary_data / boundary_from_function.  U0: initial field
    (default u0 at the grid nodes).  Returns the field at step n_steps (default grid.n_steps).
    """
    n_steps = grid.n_steps if n_steps is None else n_steps
    if any(float(b) != 0.0 for b in problem.get("drift", (0.0, 0.0))):
        raise ValueError("the subdomain solver is for L = a Lap (no drift)")
    a = float(problem["diffusion"])
    coef = [float(c) for c in problem["coef"]]
    dt = grid.dt
    rx = a * dt / grid.hx ** 2
    ry = a * dt / grid.hy ** 2
    xs = grid.x_lo + np.arange(grid.NX + 1) * grid.hx
    ys = grid.y_lo + np.arange(grid.NY + 1) * grid.hy
    if U0 is None:
        U0 = g_grid(problem, xs[None, :], ys[:, None])
    U = np.array(U0, dtype=np.float64)
    _set_boundary(grid, U, bd, 0)
    Uold = U.copy()
    vlines = {k: li for li, (o, k, _) in enumerate(grid.lines()) if o == "v"}

    def band(r, n):
        ab = np.zeros((3, n))
        ab[0, 1:] = -r / 2.0
        ab[1, :] = 1.0 + r
        ab[2, :-1] = -r / 2.0
        return ab

    abx = band(rx, grid.cx - 1)
    aby = band(ry, grid.cy - 1)
    from oracle import cmod_of, linear_modulated

    cm = cmod_of(problem)
    if cm:
        bx, by, t0, pw = cm
        exy = np.exp(-by * ys * ys)[:, None] * np.exp(-bx * xs * xs)[None, :]
        pcoef = list(coef)
        lin_c = coef[1]  # the unmodulated linear coefficient
        if linear_modulated(problem):
            lin_c = 0.0  # the modulation multiplies c_1 u as well
        else:
            pcoef[1] = 0.0
    for n in range(n_steps):
        ut = 1.5 * U - 0.5 * Uold
        if cm:
            T = 1.0 / ((n + 0.5) * dt + t0) if pw == 1 else 1.0
            F = lin_c * ut + (exy * T) * f_poly(pcoef, ut)
        else:
            F = f_poly(coef, ut)
        Unew = np.zeros_like(U)
        _set_boundary(grid, Unew, bd, n + 1)
        # intermediate level: interior rows from the x-sweeps; on the vertical lines from the data
        Ustar = np.zeros_like(U)
        for kx in range(grid.px + 1):
            col = kx * grid.cx
            if kx in vlines:
                g0 = bd[vlines[kx]][n]
                g1 = bd[vlines[kx]][n + 1]
            else:  # outer edge held at zero
                g0 = np.zeros(grid.NY + 1)
                g1 = g0
            d0 = np.zeros_like(g0)
            d1 = np.zeros_like(g1)
            d0[1:-1] = g0[:-2] - 2.0 * g0[1:-1] + g0[2:]
            d1[1:-1] = g1[:-2] - 2.0 * g1[1:-1] + g1[2:]
            Ustar[:, col] = 0.5 * (g0 + ry / 2.0 * d0) + 0.5 * (g1 - ry / 2.0 * d1)
        for sx in range(grid.px):
            c0, c1 = sx * grid.cx, (sx + 1) * grid.cx
            for sy in range(grid.py):
                r0, r1 = sy * grid.cy, (sy + 1) * grid.cy
                rows = slice(r0 + 1, r1)
                cols = slice(c0 + 1, c1)
                # x-sweep: one tridiagonal system per interior row (right-hand sides as columns)
                rhs = (U[rows, cols] + ry / 2.0 * (U[r0:r1 - 1, cols] - 2.0 * U[rows, cols] + U[r0 + 2:r1 + 1, cols])
                       + dt / 2.0 * F[rows, cols])
                rhs[:, 0] += rx / 2.0 * Ustar[rows, c0]
                rhs[:, -1] += rx / 2.0 * Ustar[rows, c1]
                Ustar[rows, cols] = solve_banded((1, 1), abx, rhs.T).T
        for sx in range(grid.px):
            c0, c1 = sx * grid.cx, (sx + 1) * grid.cx
            for sy in range(grid.py):
                r0, r1 = sy * grid.cy, (sy + 1) * grid.cy
                rows = slice(r0 + 1, r1)
                cols = slice(c0 + 1, c1)
                # y-sweep: one tridiagonal system per interior column
                rhs = (Ustar[rows, cols] + rx / 2.0 * (Ustar[rows, c0:c1 - 1] - 2.0 * Ustar[rows, cols]
                                                        + Ustar[rows, c0 + 2:c1 + 1])
                       + dt / 2.0 * F[rows, cols])
                rhs[0, :] += ry / 2.0 * Unew[r0, cols]
                rhs[-1, :] += ry / 2.0 * Unew[r1, cols]
                Unew[rows, cols] = solve_banded((1, 1), aby, rhs)
        Uold, U = U, Unew
    return U


def pdd_solve(grid: Grid, problem, node_values, n_steps=None):
    """The whole tail: interpolate the node values, then solve every subdomain."""
    bd = boundary_data(grid, problem, node_values)
    return adi_solve(grid, problem, bd, n_steps=n_steps)


def grid_coords(grid: Grid):
    xs = grid.x_lo + np.arange(grid.NX + 1) * grid.hx
    ys = grid.y_lo + np.arange(grid.NY + 1) * grid.hy
    return xs, ys


def heat_gaussian(a, s0, cx=0.0, cy=0.0, c1=0.0):
    """Exact solution of u_t = a lap u + c1 u with u0 a unit-amplitude Gaussian of width s0."""
    def fn(X, Y, t):
        s2 = s0 * s0 + 2.0 * a * t
        return (s0 * s0 / s2) * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * s2) + c1 * t)
    return fn


def fisher_plane_wave(angle):
    """Exact planar travelling wave of u_t = lap u + u - u^2 along the unit vector at `angle`."""
    n0, n1 = math.cos(angle), math.sin(angle)
    s6 = math.sqrt(6.0)

    def fn(X, Y, t):
        z = X * n0 + Y * n1
        return (1.0 + np.exp((z - 5.0 * t / s6) / s6)) ** -2
    return fn
