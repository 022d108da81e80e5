"""Helpers for GPU-vs-oracle parity tests (test code only).

Tolerances (stated per result):
  * tree shape (splits Ne, nodes visited, overflow/capped flags), per-bin counts: bit-exact.  Both
    sides decide vertex vs leaf with the same FP64 product of Philox uniforms against the same
    host-computed theta, and the arity from the same integer product.
  * tree value F, FP64 paths: |dF| <= 1e-12 |F|.  Differences come only from the device math
    library's log/exp/sin/cos (a few ulp) along at most a few hundred operations.
  * tree value F, FP32 paths: |dF| <= 2e-4 |F| + 1e-6 max_point |F| (see compare_trees).  Each node rounds to 2^-24 in a handful of
    operations; exp arguments reach |(alpha-1) mu tau| <= 10 (relative error ~10 ulp) and the initial
    data amplifies position errors by |g'/g| <= 1/sqrt6..2; trees here have at most ~60 nodes.
  * per-bin sums S1 (S2): |dS| <= tolF * sum|F| (2 tolF * sum F^2) + 1e-13 * sum|F| (summation order).
  * Pade value: |du| <= 1e-3 absolute (the target), and the observed difference is reported.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

FP64_TOL = 1e-12
FP32_TOL = 2e-4


def gpu_run(ctx, wl, records=True, launch=None):
    """Run a workload through Plan.execute on the current stream; return numpy outputs."""
    import torch

    from paper_2402_06491_amd import Plan

    if launch:
        ctx.set_launch(**launch)
    plan = Plan(ctx, wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"],
                problem_id=wl.get("problem_id"), point_id=wl.get("point_id"))
    out = plan.outputs(records=records)
    plan.execute(out)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["plan"] = plan
    return res


def tree_items(wl, point_idx=None, tree_idx=None):
    """Expand (point, tree) pairs: all trees of all points, or the given pairs."""
    n_trees = np.asarray(wl["n_trees"], dtype=np.int64)
    base = np.concatenate([[0], np.cumsum(n_trees)])
    if point_idx is None:
        point_idx = np.repeat(np.arange(len(n_trees)), n_trees)
        tree_idx = np.concatenate([np.arange(n) for n in n_trees]) if len(n_trees) else np.zeros(0, np.int64)
    rec_idx = base[point_idx] + tree_idx
    return np.asarray(point_idx), np.asarray(tree_idx), rec_idx


def oracle_trees(wl, point_idx, tree_idx):
    """Oracle records for the given (point, tree) pairs, grouped by problem."""
    x = np.asarray(wl["x"], dtype=np.float64)
    t = np.asarray(wl["t"], dtype=np.float64)
    pids = wl.get("point_id")
    pids = np.arange(len(t), dtype=np.uint32) if pids is None else np.asarray(pids, np.uint32)
    prob_of = np.asarray(wl.get("problem_id", np.zeros(len(t), np.uint32)))
    n = len(point_idx)
    F = np.zeros(n)
    ne = np.zeros(n, np.uint32)
    nodes = np.zeros(n, np.uint32)
    flags = np.zeros(n, np.uint32)
    for k, prob in enumerate(wl["problems"]):
        sel = np.nonzero(prob_of[point_idx] == k)[0]
        if len(sel) == 0:
            continue
        pi = point_idx[sel]
        r = oracle.walk(prob, wl["mc"], x[pi], t[pi], pids[pi], tree_idx[sel])
        F[sel], ne[sel], nodes[sel], flags[sel] = r["F"], r["ne"], r["nodes"], r["flags"]
    return {"F": F, "ne": ne, "nodes": nodes, "flags": flags}


def decode_meta(meta):
    m = meta.astype(np.uint32)
    ne = m & 0xFF
    flags = ((m >> 8) & 1) * 1 + ((m >> 9) & 1) * 2
    depth = (m >> 10) & 1
    nodes = m >> 11
    return ne, flags, depth, nodes


def compare_trees(gpu, rec_idx, orc, tol, point_idx=None):
    """Per-tree comparison; returns the max relative F difference.

    FP32 paths also get an absolute floor of 1e-6 times the largest |F| among the point's trees: near
    a zero of g (the edge of the cos^2 bump, a Gaussian tail) FP32 evaluation is accurate to about
    1e-7 max|g| in absolute terms, not relative to g itself.
    """
    ne, flags, depth, nodes = decode_meta(gpu["tree_meta"][rec_idx])
    assert not depth.any(), "stack depth exceeded"
    np.testing.assert_array_equal(ne, np.minimum(orc["ne"], 255))
    np.testing.assert_array_equal(flags, orc["flags"])
    np.testing.assert_array_equal(nodes, orc["nodes"])
    Fg = gpu["tree_f"][rec_idx].astype(np.float64)
    Fo = orc["F"]
    err = np.abs(Fg - Fo)
    bound = tol * np.abs(Fo) + (1e-30 if tol > FP64_TOL else 1e-300)
    if tol > FP64_TOL and point_idx is not None and len(Fo):
        scale = np.zeros(int(point_idx.max()) + 1)
        np.maximum.at(scale, point_idx, np.abs(Fo))
        bound = bound + 1e-6 * scale[point_idx]
    bad = np.nonzero(err > bound)[0]
    assert len(bad) == 0, f"{len(bad)} trees off; first {bad[:5]}: gpu {Fg[bad[:5]]} oracle {Fo[bad[:5]]}"
    rel = err / np.maximum(np.abs(Fo), 1e-300)
    return float(rel.max()) if len(rel) else 0.0


def oracle_moments(wl, orc, point_idx):
    """Exact per-point, per-bin moments from oracle records (all trees of every point present)."""
    mc = wl["mc"]
    B = oracle.n_bins(mc)
    npts = len(wl["t"])
    out = []
    for p in range(npts):
        sel = point_idx == p
        rec = {k: v[sel] for k, v in orc.items()}
        m = oracle.moments(rec, mc)
        ok = rec["flags"] == 0
        b = np.minimum(rec["ne"], B - 1)
        m["abs1"] = np.array([math.fsum(np.abs(rec["F"][ok & (b == k)]).tolist()) for k in range(B)])
        out.append(m)
    return out


def compare_moments(wl, gpu, omom, tol):
    B = oracle.n_bins(wl["mc"])
    for p, m in enumerate(omom):
        h = gpu["hist"][p]
        np.testing.assert_array_equal(h[:B], m["count"], err_msg=f"point {p} hist")
        assert h[B] == m["overflow"] and h[B + 1] == m["capped"] and h[B + 2] == 0, p
        assert gpu["nodes"][p] == m["nodes"], p
        d1 = np.abs(gpu["s1"][p] - m["s1"])
        assert np.all(d1 <= (tol + 1e-13) * m["abs1"] + 1e-300), (p, d1, m["abs1"])
        d2 = np.abs(gpu["s2"][p] - m["s2"])
        assert np.all(d2 <= (2 * tol + 1e-13) * m["s2"] + 1e-300), (p, d2, m["s2"])


def oracle_pade(wl, omom):
    """Oracle coefficients and Pade value per point from exact moments."""
    mc = wl["mc"]
    L, M = int(mc["pade_L"]), int(mc["pade_M"])
    no = int(mc["max_order"])
    prob_of = np.asarray(wl.get("problem_id", np.zeros(len(wl["t"]), np.uint32)))
    res = []
    for p, m in enumerate(omom):
        nz = oracle.normalize(wl["problems"][prob_of[p]], mc)
        a, cov = oracle.coefficients(m, nz.mu, float(wl["t"][p]))
        try:
            val, used, _ = oracle.pade_value(a[: no + 1], L, M)
            se = oracle.pade_se(a[: no + 1], cov[: no + 1, : no + 1], L, M)
        except np.linalg.LinAlgError:
            val, used, se = float("nan"), None, float("nan")
        res.append({"a": a, "cov": cov, "pade": val, "used": used, "se": se, "psum": math.fsum(a.tolist())})
    return res


def pade_grad(a, L, M):
    """Central-difference gradient of the oracle's Pade value with respect to the coefficients."""
    a = np.asarray(a, dtype=np.float64)
    g = np.zeros(len(a))
    for k in range(min(len(a), L + M + 1)):
        h = 1e-6 * abs(a[k]) if a[k] != 0 else 1e-12
        ap, am = a.copy(), a.copy()
        ap[k] += h
        am[k] -= h
        g[k] = (oracle.pade_value(ap, L, M)[0] - oracle.pade_value(am, L, M)[0]) / (2 * h)
    return g


def compare_pade(wl, gpu, opade, pade_tol=1e-3):
    """Pade parity, two ways.

    (a) the Pade step itself: the oracle's [L/M] on the GPU's own coefficients equals the GPU's value
        to 1e-9 relative (skipped when the two sides lower a near-singular system differently);
    (b) end to end: |u_gpu - u_oracle| <= pade_tol + 4 * sum_k |du/da_k| |a_gpu,k - a_oracle,k|, i.e.
        the target tolerance plus the first-order propagation of the coefficient differences (which are
        within the stated per-tree tolerance) through the approximant.
    Returns (max |du|, number of points within pade_tol, number of points compared).
    """
    mc = wl["mc"]
    L, M = int(mc["pade_L"]), int(mc["pade_M"])
    no = int(mc["max_order"])
    worst, strict, n = 0.0, 0, 0
    for p, r in enumerate(opade):
        ag = gpu["coef"][p][: no + 1]
        if not np.all(np.isfinite(ag)) or r["used"] is None or not np.isfinite(r["pade"]):
            continue
        v, used, _ = oracle.pade_value(ag, L, M)
        if used == r["used"]:
            assert abs(gpu["u"][p] - v) <= 1e-9 * max(1.0, abs(v)), (p, gpu["u"][p], v)
            # delta-method SE: the device's exact gradient against the oracle's central differences
            se_tol = 1e-4 if mc["precision"] == 64 else 1e-2
            if np.isfinite(r["se"]) and abs(r["pade"]) < 1e3:
                # absolute floor: sqrt of the rounding of m2 - m1^2 (exact cancellation at t = 0)
                floor = 1e-7 * float(np.abs(r["a"]).max())
                assert abs(gpu["se"][p] - r["se"]) <= se_tol * r["se"] + floor, (p, gpu["se"][p], r["se"])
        du = abs(gpu["u"][p] - r["pade"])
        prop = float(np.abs(pade_grad(r["a"][: no + 1], L, M)) @ np.abs(ag - r["a"][: no + 1]))
        if not np.isfinite(prop):  # the finite-difference gradient failed (near-singular perturbed system):
            prop = 0.0             # no propagation allowance, the strict tolerance alone applies
        assert du <= pade_tol + 4 * prop, (p, gpu["u"][p], r["pade"], prop)
        worst = max(worst, du)
        strict += du <= pade_tol
        n += 1
    return worst, strict, n
