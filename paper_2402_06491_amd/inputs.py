"""Seeded synthetic workloads (inputs only: no arithmetic of the method).

Both the HIP path and the CPU oracle receive these arrays; neither generates
its own inputs.  Problems are plain dicts:

  problem = {"dim": 1|2, "diffusion": a, "coef": [c_0, ..., c_7],
             "u0_kind": "const"|"logistic"|"gauss_sum"|"cos2_bump",
             "u0_params": [...], "u0_nterms": k}
  mc      = {"seed", "lambda", "max_order", "prune", "node_cap",
             "pade_L", "pade_M", "precision"}

u0 parameter layouts:
  const      (g0,)
  logistic   (A, s, x0, p, n0, n1):  A * (1 + exp(s * (n.x - x0)))^(-p), p integer 1..4
  gauss_sum  k terms (A, cx, cy, s):  sum A exp(-|x - c|^2 / (2 s^2))
  cos2_bump  (A, Ax, Ay):  A cos^2(pi x / 2Ax) cos^2(pi y / 2Ay) inside the box, else 0

The workloads follow the paper's examples: the KPP equation of McKean's
representation (Sec. 1), the Fisher equation with its travelling-wave initial
data, the 2-D cubic problem on the interfaces of a domain decomposition
(Sec. 3), a batch of random polynomial non-linearities, and a served stream.
"""
from __future__ import annotations

import math

import numpy as np


def logistic(A=1.0, s=1.0, x0=0.0, p=1, n=(1.0, 0.0)):
    return {"u0_kind": "logistic", "u0_params": [float(A), float(s), float(x0), float(p), float(n[0]), float(n[1])],
            "u0_nterms": 0}


def const(g0):
    return {"u0_kind": "const", "u0_params": [float(g0)], "u0_nterms": 0}


def gauss_sum(terms):
    params = []
    for (A, cx, cy, s) in terms:
        params += [float(A), float(cx), float(cy), float(s)]
    return {"u0_kind": "gauss_sum", "u0_params": params, "u0_nterms": len(terms)}


def problem(dim, diffusion, coef, u0, coef_mod=None, drift=None, euler=None):
    """coef_mod (optional): {"beta": (bx, by), "t0": t0, "pow": 0|1[, "linear": True]} makes every non-linear
    coefficient (and with "linear" c_1 too) c_j exp(-bx x^2 - by y^2) (t + t0)^(-pow).  drift (optional):
    the constant b of L = a Lap + b.grad.  euler (optional): {"dt": h, "drift_lin": (B_x, B_y),
    "sigma_amp": A, "sigma_width": w} integrates the paths by Euler-Maruyama steps of at most h for
    b(x) = drift + B x and sigma(x) = sqrt(2a) (1 + A exp(-|x|^2/(2 w^2)))."""
    coef = [float(c) for c in coef] + [0.0] * (8 - len(coef))
    d = {"dim": int(dim), "diffusion": float(diffusion), "coef": coef}
    d.update(u0)
    if coef_mod:
        d["coef_mod"] = {"beta": [float(b) for b in coef_mod.get("beta", (0.0, 0.0))],
                         "t0": float(coef_mod.get("t0", 0.0)), "pow": int(coef_mod.get("pow", 0)),
                         "linear": bool(coef_mod.get("linear", False))}
    if drift is not None:
        d["drift"] = [float(b) for b in drift]
    if euler is not None:
        d["euler"] = {"dt": float(euler["dt"]), "drift_lin": [float(b) for b in euler.get("drift_lin", (0.0, 0.0))],
                      "sigma_amp": float(euler.get("sigma_amp", 0.0)),
                      "sigma_width": float(euler.get("sigma_width", 1.0))}
    return d


def mc_params(seed=0, lam=1.0, max_order=12, prune=1, node_cap=1 << 16, pade=(6, 6), precision=32, strategy=0,
              q=0.5):
    return {"seed": int(seed), "lambda": float(lam), "max_order": int(max_order), "prune": int(prune),
            "node_cap": int(node_cap), "pade_L": int(pade[0]), "pade_M": int(pade[1]),
            "precision": int(precision), "strategy": int(strategy), "q": float(q)}


# ---------------------------------------------------------------------------
# The five workloads.  ``scale`` shrinks the number of trees per point for the
# small parity cases; the point sets are always the full ones unless
# ``points`` is given.
# ---------------------------------------------------------------------------
def kpp(n_trees=100_000):
    """1-D KPP  u_t = 0.5 u_xx + u^2 - u,  u0 = 1/(1+e^x): binary branching at rate 1.

    16 points uniform in [-4, 4], t = 1, FP64 paths, no pruning (bins 0..63
    plus a tail bin), tree size capped at 2^16 nodes.
    """
    prob = problem(1, 0.5, [0.0, -1.0, 1.0], logistic(1.0, 1.0, 0.0, 1))
    x = np.linspace(-4.0, 4.0, 16).reshape(-1, 1)
    t = np.full(16, 1.0)
    mc = mc_params(seed=0, max_order=63, prune=0, node_cap=1 << 16, precision=64)
    return {"name": "kpp_1d", "problems": [prob], "mc": mc, "x": x, "t": t,
            "n_trees": np.full(16, n_trees, np.int64), "problem_id": np.zeros(16, np.uint32)}


def fisher(n_trees=1_000_000, n_x=64, times=(0.5, 1.0, 2.0)):
    """1-D Fisher  u_t = u_xx + u - u^2  with u0 = (1 + e^{x/sqrt6})^-2 (exact travelling wave).

    64 points in [-10, 10] times t in {0.5, 1, 2}: 192 queries, order-12 series
    with pruning, Pade [6/6], FP32 paths with FP64 moments.
    """
    prob = problem(1, 1.0, [0.0, 1.0, -1.0], logistic(1.0, 1.0 / math.sqrt(6.0), 0.0, 2))
    xs = np.linspace(-10.0, 10.0, n_x)
    x = np.concatenate([xs for _ in times]).reshape(-1, 1)
    t = np.concatenate([np.full(n_x, tt) for tt in times])
    n = x.shape[0]
    mc = mc_params(seed=0, max_order=12, prune=1, node_cap=1 << 16, precision=32)
    return {"name": "fisher_1d", "problems": [prob], "mc": mc, "x": x, "t": t,
            "n_trees": np.full(n, n_trees, np.int64), "problem_id": np.zeros(n, np.uint32)}


def fisher_exact(x, t):
    """Travelling-wave solution of the Fisher equation above (speed 5/sqrt6)."""
    s6 = math.sqrt(6.0)
    return (1.0 + np.exp((np.asarray(x) - 5.0 * np.asarray(t) / s6) / s6)) ** -2


def cubic_2d_u0(seed=0):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-6.0, 6.0, size=(4, 2))
    widths = rng.uniform(0.5, 2.0, size=4)
    amps = rng.uniform(0.2, 1.0, size=4)
    return gauss_sum([(amps[k], centres[k, 0], centres[k, 1], widths[k]) for k in range(4)])


def interface_points(n_per_line=256):
    """Points on the interfaces x in {-4,0,4} and y in {-4,0,4} of [-8,8]^2."""
    s = np.linspace(-8.0, 8.0, n_per_line)
    pts = []
    for xi in (-4.0, 0.0, 4.0):
        pts.append(np.stack([np.full_like(s, xi), s], axis=1))
    for yi in (-4.0, 0.0, 4.0):
        pts.append(np.stack([s, np.full_like(s, yi)], axis=1))
    return np.concatenate(pts, axis=0)


def cubic_2d(n_trees=100_000, n_per_line=256, u0_seed=0):
    """2-D  u_t = Lap u + u - u^3,  u0 = sum of 4 seeded Gaussians: ternary trees.

    3 x 3 interfaces x 256 points = 1536 Monte Carlo points at t = 1.
    """
    prob = problem(2, 1.0, [0.0, 1.0, 0.0, -1.0], cubic_2d_u0(u0_seed))
    x = interface_points(n_per_line)
    n = x.shape[0]
    mc = mc_params(seed=0, max_order=12, prune=1, node_cap=1 << 16, precision=32)
    return {"name": "cubic_2d_interfaces", "problems": [prob], "mc": mc, "x": x, "t": np.full(n, 1.0),
            "n_trees": np.full(n, n_trees, np.int64), "problem_id": np.zeros(n, np.uint32)}


def pdd_cubic_2d(n_trees=100_000, cells=512, n_steps=1000, ns=33, nt=8, outer="mc", u0_seed=0, precision=32):
    """Domain decomposition of the 2-D cubic problem on [-8, 8]^2 into 4 x 4 subdomains.

    Lines: the interfaces x, y in {-4, 0, 4} and (outer="mc") the edges x, y = +-8, each with ns nodes
    uniform over [-8, 8] at the times k/nt, k = 1..nt (t = 1); 33 x 8 = 264 Monte Carlo points per
    line.  Subdomains: cells x cells fine cells (h = 4/cells), n_steps Crank-Nicolson ADI steps, FP64.
    """
    grid = {"x_lo": -8.0, "x_hi": 8.0, "y_lo": -8.0, "y_hi": 8.0, "px": 4, "py": 4, "cx": int(cells),
            "cy": int(cells), "T": 1.0, "n_steps": int(n_steps), "ns_x": int(ns), "ns_y": int(ns),
            "nt": int(nt), "outer": outer}
    mc = mc_params(seed=0, max_order=12, prune=1, node_cap=1 << 16, precision=precision)
    return {"name": "pdd_cubic_2d", "problem": problem(2, 1.0, [0.0, 1.0, 0.0, -1.0], cubic_2d_u0(u0_seed)),
            "mc": mc, "grid": grid, "n_trees": int(n_trees)}


def example5(n_trees=100_000, n_x=64, t=0.5, precision=32, strategy=0, q=0.5):
    """A single non-linear term with a coefficient varying in space and time (the paper's Example 5):
    u_t = Lap u - e^{-x^2} / (t + 0.1) u^2, u0 = e^{-x^2/4} / sqrt(4 pi).  Neither the data nor the
    coefficient depend on y, so the solution does not either and the 2-D problem is the 1-D problem
    u_t = u_xx - e^{-x^2} / (t + 0.1) u^2 exactly; it is posed in 1-D here.  64 points in [-6, 6] at t."""
    prob = problem(1, 1.0, [0.0, 0.0, -1.0], gauss_sum([(1.0 / math.sqrt(4 * math.pi), 0.0, 0.0, math.sqrt(2.0))]),
                   coef_mod={"beta": (1.0, 0.0), "t0": 0.1, "pow": 1})
    x = np.linspace(-6.0, 6.0, n_x).reshape(-1, 1)
    mc = mc_params(seed=0, max_order=12, prune=1, node_cap=1 << 16, precision=precision, strategy=strategy, q=q)
    return {"name": "example5", "problems": [prob], "mc": mc, "x": x, "t": np.full(n_x, float(t)),
            "n_trees": np.full(n_x, n_trees, np.int64), "problem_id": np.zeros(n_x, np.uint32)}


def poly_batch(n_points=4096, n_min=10_000, n_max=1_000_000, seed=1234, precision=32):
    """8 PDEs with polynomial f of degree 2,2,3,3,4,4,5,5 (coefficients U[-1,1]).

    Points: PDE id uniform, x ~ U[-4, 4], t log-uniform in [0.25, 4], trees per
    point log-uniform in [n_min, n_max] rounded to a multiple of 64.
    """
    degrees = [2, 2, 3, 3, 4, 4, 5, 5]
    probs = []
    for p, dg in enumerate(degrees):
        rng = np.random.default_rng(p)
        c = rng.uniform(-1.0, 1.0, size=dg + 1)
        probs.append(problem(1, 1.0, list(c), logistic(0.5, 1.0, 0.0, 1)))
    rng = np.random.default_rng(seed)
    pid = rng.integers(0, 8, size=n_points).astype(np.uint32)
    x = rng.uniform(-4.0, 4.0, size=(n_points, 1))
    t = np.exp(rng.uniform(math.log(0.25), math.log(4.0), size=n_points))
    nt = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_points))
    nt = np.maximum(64, (np.rint(nt / 64) * 64)).astype(np.int64)
    mc = mc_params(seed=0, max_order=12, prune=1, node_cap=1 << 16, precision=precision)
    return {"name": "poly_batch", "problems": probs, "mc": mc, "x": x, "t": t, "n_trees": nt,
            "problem_id": pid}


def served_stream(rate=200.0, duration=60.0, seed=7):
    """Poisson arrivals of point queries on the 2-D cubic family.

    Each request: arrival time, 1..1024 points (log-uniform integer), its own u0
    seed, x ~ U([-8, 8]^2), t log-uniform in [0.25, 2].
    """
    rng = np.random.default_rng(seed)
    reqs = []
    now = 0.0
    rid = 0
    while True:
        now += rng.exponential(1.0 / rate)
        if now > duration:
            break
        npts = int(min(1024, max(1, math.floor(math.exp(rng.uniform(0.0, math.log(1025.0)))))))
        u0_seed = int(rng.integers(0, 2 ** 31))
        x = rng.uniform(-8.0, 8.0, size=(npts, 2))
        t = np.exp(rng.uniform(math.log(0.25), math.log(2.0), size=npts))
        reqs.append({"id": rid, "arrival": now, "u0_seed": u0_seed, "x": x, "t": t,
                     "problem": problem(2, 1.0, [0.0, 1.0, 0.0, -1.0], cubic_2d_u0(u0_seed))})
        rid += 1
    return reqs
