"""ORACLE — test infrastructure, not product code.

A plain, slow, obviously-correct FP64 CPU implementation of what the random-tree
Monte Carlo of Strategy A computes (Acebron & Rodriguez-Rozas, Sec. 2.1 and the
Pade summation of Sec. 2.4).  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the HIP path (``paper_2402_06491_amd``) and does not import it.

Pieces:
  * ``walker.c`` (compiled to ``liboracle.so``): one recursive FP64 walk per
    tree, with its own Philox4x32-10 (see the header of ``walker.c`` for the
    documented assignment of random words to nodes);
  * :func:`normalize`: the change of variables of Strategy A generalised to a
    clock of rate lambda (u = v e^{mu t}, mu = c_1 + lambda, vertex weight
    K c_alpha / lambda * e^{(alpha-1) mu tau'});
  * :func:`moments`: exact (``math.fsum``) per-bin sums of F and F^2, binned by
    the number of splits Ne (the partial contributions whose sum is the series);
  * :func:`coefficients`: a_n = e^{mu t} S1_n / N and their covariance
    (the sample mean of the multiplicative functional, Sec. 2.4);
  * :func:`pade`: the [L/M] Pade approximant of the series evaluated at z = 1
    (Sec. 2.1 end, Sec. 2.4), plain dense solve of the M x M linear system;
  * :func:`solve`: everything above for a set of points.

Parity pins for all of this live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "walker.c")

FLAG_OVERFLOW = 1
FLAG_CAPPED = 2

U0_KINDS = {"const": 0, "logistic": 1, "gauss_sum": 2, "cos2_bump": 3}


def build(force: bool = True) -> str:
    """Compile walker.c with gcc (plain FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("u0_kind", ctypes.c_int32),
        ("u0_nterms", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("J", ctypes.c_int32 * 8),
        ("omega", ctypes.c_double * 8),
        ("sigma", ctypes.c_double),
        ("lam", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("u0p", ctypes.c_double * 40),
        ("key", ctypes.c_uint32 * 2),
        ("max_order", ctypes.c_int32),
        ("prune", ctypes.c_int32),
        ("node_cap", ctypes.c_uint32),
        ("strategy", ctypes.c_int32),
        ("Q", ctypes.c_uint64),
        ("q", ctypes.c_double),
        ("cmod", ctypes.c_int32),
        ("cmod_pow", ctypes.c_int32),
        ("cmod_bx", ctypes.c_double),
        ("cmod_by", ctypes.c_double),
        ("cmod_t0", ctypes.c_double),
        ("drift", ctypes.c_double * 2),
        ("sde", ctypes.c_int32),
        ("sde_pad", ctypes.c_int32),
        ("dlin", ctypes.c_double * 2),
        ("sig_amp", ctypes.c_double),
        ("sig_k", ctypes.c_double),
        ("inv_h", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.or_walk.restype = ctypes.c_int
        lib.or_walk.argtypes = [
            ctypes.POINTER(_Problem), ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
        ]
        lib.or_philox4x32_10.restype = None
        lib.or_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


# ---------------------------------------------------------------------------
# Problem normalisation (Strategy A change of variables, Sec. 2.1)
# ---------------------------------------------------------------------------
@dataclass
class Normalized:
    dim: int
    sigma: float          # sqrt(2 a): generator of sigma*W is (sigma^2/2) Lap = a Lap
    lam: float            # clock rate (0 when there is no non-linear term)
    mu: float             # u = v exp(mu t)
    J: list               # powers j != 1 with c_j != 0, ascending
    omega: list           # K c_j / lam for each j in J
    u0_kind: int
    u0_params: list
    u0_nterms: int
    strategy: int = 0     # 0: Strategy A (Sec. 2.1), 1: Strategy B (Sec. 2.2)
    q: float = 1.0        # Strategy B: probability that a node is a leaf
    cmod: tuple = None    # variable coefficients (bx, by, t0, pow): c_j exp(-bx x^2 - by y^2) (t + t0)^-pow
    drift: tuple = (0.0, 0.0)  # constant drift b of L = a Lap + b.grad (the paths are x + b s + sigma W_s)
    euler: tuple = None   # general L by Euler-Maruyama: (B_x, B_y, A, 1/(2 w^2), 1/h) for b(x) = drift + B x,
                          # sigma(x) = sigma (1 + A e^{-|x|^2/(2 w^2)}), steps of at most h


def normalize(problem: dict, mc: dict) -> Normalized:
    """Strategy A normalisation.

    With u = v e^{mu t} and mu = c_1 + lam the equation for v has the
    potential -lam v, so the killing time is Exp(lam); the non-linear part
    sum_{j != 1} c_j e^{(j-1) mu t} v^j is sampled by picking one of its K terms
    uniformly, which gives the vertex weight K c_j / lam * e^{(j-1) mu tau'}.
    For lam = 1, c_1 = 0 this is the paper's u = v e^t with weight (m-1) c_j
    e^{(j-1) tau'}.  With no non-linear term there is no clock at all.
    """
    coef = [float(c) for c in problem["coef"]] + [0.0] * (8 - len(problem["coef"]))
    lam = float(mc.get("lambda", 1.0))
    strategy = strategy_of(mc)
    # with c_1 itself modulated (c_1(x, t) u) the linear term cannot be absorbed into the prefactor: it
    # joins the terms chosen at a split as an arity-1 branching (one child, weight K c_1 m / lam)
    lin = linear_modulated(problem)
    J = [j for j in range(8) if (j != 1 or lin) and coef[j] != 0.0]
    c1 = 0.0 if lin else coef[1]  # the part of c_1 absorbed into the prefactor e^{mu t}
    K = len(J)
    q = 1.0
    if K == 0:
        lam_eff, mu, omega = 0.0, c1, []
    elif strategy == 1:
        # Strategy B: u = v e^{c_1 t}; a vertex carries t K c_j / (1 - q) e^{(j-1) c_1 tau'}
        # the coin is w0 < floor(q 2^32) for a uniform 32-bit w0: its leaf probability is exactly
        # floor(q 2^32) / 2^32, and that is the q of the weights g/q and c/(1-q)
        q = math.floor(float(mc.get("q", 0.5)) * 4294967296.0) / 4294967296.0
        lam_eff = 0.0
        mu = c1
        omega = [K * coef[j] / (1.0 - q) for j in J]
    else:
        lam_eff = lam
        mu = c1 + lam
        omega = [K * coef[j] / lam for j in J]
    kind = problem["u0_kind"]
    kind = U0_KINDS[kind] if isinstance(kind, str) else int(kind)
    params = list(problem.get("u0_params", []))
    nterms = int(problem.get("u0_nterms", 0))
    if kind == 1 and len(params) != 6:
        raise ValueError("logistic u0 takes (A, s, x0, pow, n0, n1)")
    return Normalized(dim=int(problem["dim"]), sigma=math.sqrt(2.0 * float(problem["diffusion"])),
                      lam=lam_eff, mu=mu, J=J, omega=omega, u0_kind=kind,
                      u0_params=params, u0_nterms=nterms, strategy=strategy, q=q, cmod=cmod_of(problem),
                      drift=drift_of(problem), euler=euler_of(problem))


def euler_of(problem: dict):
    """(B_x, B_y, A, 1/(2 w^2), 1/h) of a problem whose paths are integrated by Euler-Maruyama, else None."""
    e = problem.get("euler")
    if not e:
        return None
    bl = [float(v) for v in e.get("drift_lin", (0.0, 0.0))] + [0.0, 0.0]
    amp = float(e.get("sigma_amp", 0.0))
    w = float(e.get("sigma_width", 1.0))
    return (bl[0], bl[1] if int(problem["dim"]) == 2 else 0.0, amp, 1.0 / (2.0 * w * w) if amp != 0.0 else 0.0,
            1.0 / float(e["dt"]))


def drift_of(problem: dict):
    """The constant drift b (x and y components; y is 0 in 1-D)."""
    b = [float(v) for v in problem.get("drift", (0.0, 0.0))] + [0.0, 0.0]
    return (b[0], b[1] if int(problem["dim"]) == 2 else 0.0)


def linear_modulated(problem: dict) -> bool:
    """True when the coefficient modulation also applies to c_1 (coef_mod "linear")."""
    cm = problem.get("coef_mod")
    return bool(cm) and bool(cm.get("linear", False))


def cmod_of(problem: dict):
    """(bx, by, t0, pow) of a problem with variable coefficients, else None."""
    cm = problem.get("coef_mod")
    if not cm:
        return None
    beta = list(cm.get("beta", (0.0, 0.0))) + [0.0]
    by = float(beta[1]) if int(problem["dim"]) == 2 else 0.0
    return (float(beta[0]), by, float(cm.get("t0", 0.0)), int(cm.get("pow", 0)))


def strategy_of(mc: dict) -> int:
    s = mc.get("strategy", 0)
    return {"A": 0, "B": 1}[s] if isinstance(s, str) else int(s)


def _make_struct(nz: Normalized, mc: dict) -> _Problem:
    pb = _Problem()
    pb.dim = nz.dim
    pb.u0_kind = nz.u0_kind
    pb.u0_nterms = nz.u0_nterms
    pb.K = len(nz.J)
    for i, j in enumerate(nz.J):
        pb.J[i] = j
        pb.omega[i] = nz.omega[i]
    pb.sigma = nz.sigma
    pb.lam = nz.lam if nz.lam > 0 else 1.0
    pb.mu = nz.mu
    for i, v in enumerate(nz.u0_params):
        pb.u0p[i] = v
    seed = int(mc.get("seed", 0))
    pb.key[0] = seed & 0xFFFFFFFF
    pb.key[1] = (seed >> 32) & 0xFFFFFFFF
    pb.max_order = int(mc.get("max_order", 12))
    pb.prune = int(mc.get("prune", 1))
    pb.node_cap = int(mc.get("node_cap", 1 << 16))
    pb.strategy = nz.strategy
    pb.drift[0], pb.drift[1] = nz.drift
    if nz.euler:
        pb.sde = 1
        pb.dlin[0], pb.dlin[1], pb.sig_amp, pb.sig_k, pb.inv_h = nz.euler
    if nz.cmod:
        pb.cmod = 1
        pb.cmod_bx, pb.cmod_by, pb.cmod_t0, pb.cmod_pow = nz.cmod
    pb.q = nz.q
    pb.Q = int(math.floor(nz.q * 4294967296.0))
    return pb


# ---------------------------------------------------------------------------
# Walking trees
# ---------------------------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 block (from walker.c) for one counter/key pair."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.or_philox4x32_10(ctypes.addressof(c), ctypes.addressof(k), ctypes.addressof(o))
    return [o[0], o[1], o[2], o[3]]


def walk(problem: dict, mc: dict, x, t, point_id, tree_idx, nthreads: int = 0):
    """Walk one tree per item.  Returns dict of per-tree F, ne, nodes, flags."""
    lib = _load()
    nz = normalize(problem, mc)
    pb = _make_struct(nz, mc)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, nz.dim))
    n = x.shape[0]
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), (n,)))
    pid = np.ascontiguousarray(np.broadcast_to(np.asarray(point_id, dtype=np.uint32), (n,)))
    tid = np.ascontiguousarray(np.asarray(tree_idx, dtype=np.uint32).reshape(n))
    F = np.empty(n, np.float64)
    ne = np.empty(n, np.uint32)
    nodes = np.empty(n, np.uint32)
    flags = np.empty(n, np.uint32)
    lib.or_walk(ctypes.byref(pb), n, x.ctypes.data, t.ctypes.data, pid.ctypes.data, tid.ctypes.data,
                F.ctypes.data, ne.ctypes.data, nodes.ctypes.data, flags.ctypes.data, int(nthreads))
    return {"F": F, "ne": ne, "nodes": nodes, "flags": flags}


def walk_point(problem, mc, x, t, point_id, n_trees, first_tree=0, nthreads=0):
    """All trees [first_tree, first_tree + n_trees) of one point."""
    dim = int(problem["dim"])
    x = np.asarray(x, dtype=np.float64).reshape(1, dim)
    xs = np.repeat(x, n_trees, axis=0)
    return walk(problem, mc, xs, t, point_id, np.arange(first_tree, first_tree + n_trees, dtype=np.uint64), nthreads)


# ---------------------------------------------------------------------------
# Binned moments and coefficients (Sec. 2.4: u ~ (1/N) sum of the functional)
# ---------------------------------------------------------------------------
def n_bins(mc: dict) -> int:
    """Bins 0..max_order, plus one tail bin for Ne > max_order (prune off)."""
    return int(mc.get("max_order", 12)) + 2


def moments(rec: dict, mc: dict):
    """Exact per-bin count, sum F, sum F^2 (math.fsum), plus overflow/capped counts."""
    B = n_bins(mc)
    F, ne, flags = rec["F"], rec["ne"], rec["flags"]
    ok = flags == 0
    b = np.minimum(ne, B - 1)
    count = np.zeros(B, np.int64)
    s1 = np.zeros(B, np.float64)
    s2 = np.zeros(B, np.float64)
    for k in range(B):
        sel = ok & (b == k)
        count[k] = int(sel.sum())
        vals = F[sel]
        s1[k] = math.fsum(vals.tolist())
        s2[k] = math.fsum((vals * vals).tolist())
    overflow = int(((flags & FLAG_OVERFLOW) != 0).sum())
    capped = int(((flags & FLAG_CAPPED) != 0).sum())
    return {"count": count, "s1": s1, "s2": s2, "overflow": overflow, "capped": capped,
            "nodes": int(rec["nodes"].astype(np.int64).sum()), "n": int(F.shape[0])}


def coefficients(mom: dict, mu: float, t: float):
    """a_n = e^{mu t} S1_n / N for every bin and the covariance of the estimates.

    Each tree falls in exactly one bin, so E[F_n F_m] = 0 for n != m and
    Cov(a_n, a_m) = e^{2 mu t} (delta_nm S2_n/N - (S1_n/N)(S1_m/N)) / (N - 1).
    """
    N = mom["n"]
    scale = math.exp(mu * t)
    if N == 0:
        B = len(mom["s1"])
        return np.zeros(B), np.zeros((B, B))
    m1 = mom["s1"] / N
    a = scale * m1
    cov = np.diag(mom["s2"] / N) - np.outer(m1, m1)
    cov = cov * (scale * scale) / max(N - 1, 1)
    return a, cov


# ---------------------------------------------------------------------------
# Pade approximant (Sec. 2.1 end; robustness discussion of Sec. 2.4)
# ---------------------------------------------------------------------------
def pade_coeffs(a, L: int, M: int):
    """Numerator p_0..p_L and denominator q_0..q_M (q_0 = 1) of the [L/M] approximant.

    Defined by P(z) - Q(z) F(z) = O(z^{L+M+1}): for k = L+1..L+M,
    sum_{j=0}^{M} q_j a_{k-j} = 0 (a_i = 0 for i < 0); then
    p_i = sum_{j=0}^{min(i,M)} q_j a_{i-j}.  The M x M system is solved by LU with
    partial pivoting; it counts as singular (numpy.linalg.LinAlgError) when an
    entry is not finite or the smallest pivot is below 1e-13 times the largest.
    """
    from scipy.linalg import lu_factor, lu_solve

    a = np.asarray(a, dtype=np.float64)
    coef = lambda i: a[i] if i >= 0 else 0.0  # noqa: E731
    q = np.ones(M + 1)
    if M > 0:
        T = np.array([[coef(L + i - j) for j in range(1, M + 1)] for i in range(1, M + 1)])
        rhs = -np.array([coef(L + i) for i in range(1, M + 1)])
        if not (np.all(np.isfinite(T)) and np.all(np.isfinite(rhs))):
            raise np.linalg.LinAlgError("non-finite Pade system")
        piv = np.abs(np.diag(lu_factor(T, check_finite=False)[0])) if np.any(T) else np.zeros(M)
        if piv.max() == 0.0 or piv.min() <= 1e-13 * piv.max():
            raise np.linalg.LinAlgError("singular Pade system")
        q[1:] = lu_solve(lu_factor(T, check_finite=False), rhs, check_finite=False)
    p = np.array([sum(q[j] * coef(i - j) for j in range(0, min(i, M) + 1)) for i in range(L + 1)])
    return p, q


def pade_value(a, L: int, M: int, z: float = 1.0):
    """[L/M](z); if the system is singular, lower M by one and raise L by one (same order)."""
    while True:
        try:
            p, q = pade_coeffs(a, L, M)
            break
        except np.linalg.LinAlgError:
            if M == 0:
                raise
            L, M = L + 1, M - 1
    num = sum(p[i] * z ** i for i in range(len(p)))
    den = sum(q[j] * z ** j for j in range(len(q)))
    return num / den, (L, M), q


def pade_se(a, cov, L: int, M: int):
    """Delta-method standard error of [L/M](1) with central-difference gradient."""
    a = np.asarray(a, dtype=np.float64)
    n = L + M + 1
    grad = np.zeros(len(a))
    for k in range(n):
        h = 1e-6 * max(abs(a[k]), 1e-300) if a[k] != 0 else 1e-12
        ap = a.copy(); ap[k] += h
        am = a.copy(); am[k] -= h
        grad[k] = (pade_value(ap, L, M)[0] - pade_value(am, L, M)[0]) / (2 * h)
    var = float(grad @ cov @ grad)
    return math.sqrt(max(var, 0.0))


def solve(problem: dict, mc: dict, x, t, n_trees, point_ids=None, nthreads: int = 0):
    """Full oracle pipeline for a set of points: walk, bin, coefficients, Pade.

    Returns one dict per point with the moments, coefficients (a[0..max_order]
    plus the tail), the Pade value at z = 1, its delta-method SE and the plain
    partial sum.
    """
    nz = normalize(problem, mc)
    dim = nz.dim
    x = np.asarray(x, dtype=np.float64).reshape(-1, dim)
    npts = x.shape[0]
    t = np.broadcast_to(np.asarray(t, dtype=np.float64), (npts,))
    n_trees = np.broadcast_to(np.asarray(n_trees, dtype=np.int64), (npts,))
    if point_ids is None:
        point_ids = np.arange(npts, dtype=np.uint32)
    L = int(mc.get("pade_L", 6))
    M = int(mc.get("pade_M", 6))
    no = int(mc.get("max_order", 12))
    out = []
    for i in range(npts):
        rec = walk_point(problem, mc, x[i], float(t[i]), int(point_ids[i]), int(n_trees[i]), nthreads=nthreads)
        mom = moments(rec, mc)
        a, cov = coefficients(mom, nz.mu, float(t[i]))
        series = a[: no + 1]
        try:
            val, used, q = pade_value(series, L, M)
            se = pade_se(series, cov[: no + 1, : no + 1], L, M)
        except np.linalg.LinAlgError:
            val, used, q, se = float("nan"), (L, 0), np.ones(1), float("nan")
        out.append({"moments": mom, "a": a, "cov": cov, "pade": val, "pade_order": used, "pade_q": q,
                    "pade_se": se, "partial_sum": math.fsum(a.tolist()), "records": rec})
    return out
