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
  * :func:`pade_value`: the [L/M] Pade approximant of the series evaluated at z = 1
    (Sec. 2.1 end, Sec. 2.4), with the degrees chosen by an SVD rank test of the
    denominator's linear conditions (:func:`pade_order`, reading R13), plus the
    neighbouring orders and the poles (:func:`pade_summary`);
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
# Relative rank tolerance of the order selection (reading R13): a singular value of the linear
# conditions on the denominator counts as zero when it is at most PADE_TOL times the 2-norm of the
# coefficients a_0..a_{L+M}.
PADE_TOL = 1e-12
# A pole of the approximant within POLE_DIST of the segment [0, 1] (the path along which the series is
# continued to z = 1) is flagged: the value there is then unreliable.
POLE_DIST = 0.5
# A value whose sensitivity sum_k |du/da_k| |a_k| exceeds SENSITIVE_KAPPA is flagged: a relative change of
# 1e-5 in every coefficient (the accuracy of coefficients summed from FP32 paths) can move it by 1e-3.
SENSITIVE_KAPPA = 100.0


def _coef(a, i):
    return float(a[i]) if 0 <= i < len(a) else 0.0


def denominator_conditions(a, L: int, M: int):
    """The M x (M+1) matrix C with C[i, j] = a_{L+1+i-j} (i = 0..M-1, j = 0..M; a_k = 0 for k < 0).

    The [L/M] approximant P/Q of F(z) = sum a_n z^n satisfies Q F - P = O(z^{L+M+1}); the coefficients of
    z^{L+1}..z^{L+M} of Q F involve q alone, so C q = 0 for q = (q_0..q_M)."""
    return np.array([[_coef(a, L + 1 + i - j) for j in range(M + 1)] for i in range(M)], dtype=np.float64)


def pade_order(a, L: int, M: int, tol: float = PADE_TOL):
    """The degrees actually used for a requested [L/M] (reading R13).

    After Gonnet, Guettel and Trefethen, "Robust Pade approximation via SVD" (SIAM Review 55, 2013):
    with s = ||a_0..a_{L+M}||_2, count rho = the singular values of C (denominator_conditions) above
    tol * s.  If rho < M the conditions have a null space of dimension M + 1 - rho > 1 (the data come from
    a rational of lower degree, or carry no information at that order): lower both degrees by M - rho
    (L stays >= 0) and look again.  Once C has full rank its null vector is unique up to scale; if the
    square block C[:, 1:] is itself rank deficient (smallest singular value at most tol * s) that vector
    has q_0 = 0 and no approximant with Q(0) = 1 exists: take [L+1/M-1], the next entry on the same
    antidiagonal of the Pade table.  All-zero data give [0/0].  Returns (L, M, margin), where margin is
    the smallest ratio, over every rank decision taken, of the deciding singular value to the threshold
    tol * s or its reciprocal (how far the decisions are from flipping; inf when none was taken)."""
    a = np.asarray(a, dtype=np.float64)
    s = float(np.linalg.norm(a[: L + M + 1]))
    if s == 0.0 or not np.isfinite(s):
        return 0, 0, math.inf
    thr = tol * s
    margin = math.inf

    def note(sv):
        nonlocal margin
        if sv > 0.0:
            margin = min(margin, sv / thr if sv > thr else thr / sv)

    while M > 0:
        sv = np.linalg.svd(denominator_conditions(a, L, M), compute_uv=False)
        rho = int(np.sum(sv > thr))
        if rho < M:
            note(sv[rho])  # the largest singular value counted as zero
            if rho > 0:
                note(sv[rho - 1])
            L, M = max(L - (M - rho), 0), rho
            continue
        note(sv[M - 1])
        svT = np.linalg.svd(denominator_conditions(a, L, M)[:, 1:], compute_uv=False)
        note(svT[-1])
        if svT[-1] <= thr:
            L, M = L + 1, M - 1
            continue
        break
    return L, M, margin


def pade_coeffs(a, L: int, M: int):
    """Numerator p_0..p_L and denominator q_0..q_M (q_0 = 1) of the [L/M] approximant of sum a_n z^n.

    Defined by Q(z) F(z) - P(z) = O(z^{L+M+1}): C q = 0 with q_0 = 1 (denominator_conditions), i.e. the
    M x M system C[:, 1:] (q_1..q_M) = -C[:, 0], solved by numpy's LU; then p_i = sum_{j<=min(i,M)} q_j a_{i-j}.
    No degree selection here: pade_order chooses (L, M)."""
    a = np.asarray(a, dtype=np.float64)
    q = np.ones(M + 1)
    if M > 0:
        C = denominator_conditions(a, L, M)
        q[1:] = np.linalg.solve(C[:, 1:], -C[:, 0])
    p = np.array([sum(q[j] * _coef(a, i - j) for j in range(0, min(i, M) + 1)) for i in range(L + 1)])
    return p, q


def pade_value(a, L: int, M: int, z: float = 1.0, tol: float = PADE_TOL):
    """The approximant at z for a requested [L/M]: degrees from pade_order, then P(z)/Q(z).

    Returns (value, (L', M') used, q)."""
    Lu, Mu, _ = pade_order(a, L, M, tol)
    p, q = pade_coeffs(a, Lu, Mu)
    num = sum(p[i] * z ** i for i in range(len(p)))
    den = sum(q[j] * z ** j for j in range(len(q)))
    return num / den, (Lu, Mu), q


def pade_neighbours(a, L: int, M: int, tol: float = PADE_TOL):
    """The [L-1/M] and [L/M-1] values at z = 1 (each with its own degree selection; NaN where the order
    does not exist).  Sec. 2.4 judges an approximant by comparing it across numbers of coefficients: a
    value that moves a lot when one coefficient is dropped is not yet converged."""
    lo = pade_value(a, L - 1, M, tol=tol)[0] if L >= 1 else float("nan")
    mo = pade_value(a, L, M - 1, tol=tol)[0] if M >= 1 else float("nan")
    return lo, mo


def pole_distance(q):
    """Distance from the segment [0, 1] to the nearest zero of Q(z) = sum q_j z^j (a pole of the
    approximant; inf if Q is constant), the zeros from numpy.roots (eigenvalues of the companion matrix)."""
    q = np.trim_zeros(np.asarray(q, dtype=np.float64), "b")
    if len(q) <= 1:
        return math.inf
    r = np.roots(q[::-1])
    return float(min(abs(z - min(max(z.real, 0.0), 1.0)) for z in r)) if len(r) else math.inf


def pade_gradient(a, L: int, M: int, tol: float = PADE_TOL):
    """Gradient of [L'/M'](1) with respect to a_0..a_{L'+M'} at the degrees (L', M') that pade_order
    chooses for a, by central differences (step 1e-6 |a_k|, or 1e-12 for a zero coefficient); zero for
    the coefficients the approximant does not use."""
    a = np.asarray(a, dtype=np.float64)
    Lu, Mu, _ = pade_order(a, L, M, tol)

    def val(b):
        p, q = pade_coeffs(b, Lu, Mu)
        return sum(p) / sum(q)

    grad = np.zeros(len(a))
    for k in range(min(len(a), Lu + Mu + 1)):
        h = 1e-6 * abs(a[k]) if a[k] != 0 else 1e-12
        ap = a.copy(); ap[k] += h
        am = a.copy(); am[k] -= h
        grad[k] = (val(ap) - val(am)) / (2 * h)
    return grad


def pade_se(a, cov, L: int, M: int, tol: float = PADE_TOL):
    """Delta-method standard error of the approximant at z = 1: sqrt(g' Cov g) with g = pade_gradient."""
    g = pade_gradient(a, L, M, tol)
    var = float(g @ cov @ g)
    return math.sqrt(max(var, 0.0))


def pade_summary(a, cov, L: int, M: int, tol: float = PADE_TOL):
    """Everything the finalize reports about the approximant of one point: value, degrees used and the
    margin of their selection, SE, the two neighbour values, the sensitivity kappa = sum_k |du/da_k| |a_k|,
    the pole distance from [0, 1] and the flags (pole, sensitive, lowered)."""
    a = np.asarray(a, dtype=np.float64)
    val, used, q = pade_value(a, L, M, tol=tol)
    margin = pade_order(a, L, M, tol)[2]
    lo, mo = pade_neighbours(a, L, M, tol)
    g = pade_gradient(a, L, M, tol)
    kappa = float(np.abs(g) @ np.abs(a))
    dist = pole_distance(q)
    se = math.sqrt(max(float(g @ cov @ g), 0.0)) if cov is not None else float("nan")
    return {"pade": val, "pade_order": used, "pade_q": q, "order_margin": margin, "pade_se": se,
            "pade_lo": lo, "pade_mo": mo, "kappa": kappa, "pole_distance": dist,
            "pole": dist <= POLE_DIST, "sensitive": kappa > SENSITIVE_KAPPA, "lowered": used != (L, M)}


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
        if np.all(np.isfinite(series)):
            pd = pade_summary(series, cov[: no + 1, : no + 1], L, M)
        else:
            pd = {"pade": float("nan"), "pade_order": None, "pade_q": np.ones(1), "pade_se": float("nan")}
        out.append({"moments": mom, "a": a, "cov": cov, **pd, "partial_sum": math.fsum(a.tolist()),
                    "records": rec})
    return out
