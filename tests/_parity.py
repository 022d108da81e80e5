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
  * Pade value: |du| <= 1e-3 absolute (the target) at every point that the device and the oracle do not
    both flag as having a pole near [0, 1] or a sensitivity kappa > 100 (compare_pade).
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


def _ulps(a, b):
    """Distance in units in the last place between two finite doubles of the same sign (0 if equal)."""
    if a == b:
        return 0
    ia = np.array([a], np.float64).view(np.int64)[0]
    ib = np.array([b], np.float64).view(np.int64)[0]
    return abs(int(ia) - int(ib)) if (a > 0) == (b > 0) else 1 << 62


def check_exact_sums(wl, gpu, rec_idx, point_idx):
    """The device's per-bin sums against the exactly rounded sums of its own tree values (math.fsum).
    S1 within 1 ulp: the device sums each segment in double-double (error at most about 2^-100 sum|F|) and
    joins the segments exactly, so it differs from the exactly rounded sum only where that sum lies within
    its error of a rounding midpoint (FP32-path values have short significands, and sums of a few of them
    can sit exactly on a midpoint).  S2 (sum of F*F, positive terms, plain FP64 per lane in a fixed order,
    segments joined exactly) within 1e-13 relative."""
    B = oracle.n_bins(wl["mc"])
    ne, flags, depth, _ = decode_meta(gpu["tree_meta"][rec_idx])
    F = gpu["tree_f"][rec_idx].astype(np.float64)
    ok = (flags == 0) & (depth == 0)
    b = np.minimum(ne, B - 1)
    for p in range(len(wl["t"])):
        sel = ok & (point_idx == p)
        for k in range(B):
            v = F[sel & (b == k)]
            s1 = math.fsum(v.tolist())
            s2 = math.fsum((v * v).tolist())
            assert _ulps(gpu["s1"][p][k], s1) <= 1, (p, k, gpu["s1"][p][k], s1)
            assert abs(gpu["s2"][p][k] - s2) <= 1e-13 * s2, (p, k, gpu["s2"][p][k], s2)


def oracle_pade(wl, omom):
    """Oracle coefficients and Pade summary (value, degrees, SE, neighbours, kappa, pole) per point from
    exact moments."""
    mc = wl["mc"]
    L, M = int(mc["pade_L"]), int(mc["pade_M"])
    no = int(mc["max_order"])
    prob_of = np.asarray(wl.get("problem_id", np.zeros(len(wl["t"]), np.uint32)))
    res = []
    for p, m in enumerate(omom):
        nz = oracle.normalize(wl["problems"][prob_of[p]], mc)
        a, cov = oracle.coefficients(m, nz.mu, float(wl["t"][p]))
        if np.all(np.isfinite(a[: no + 1])):
            summ = oracle.pade_summary(a[: no + 1], cov[: no + 1, : no + 1], L, M)
        else:
            summ = {"pade": float("nan"), "pade_order": None, "pade_se": float("nan")}
        res.append({"a": a, "cov": cov, **summ, "used": summ["pade_order"], "se": summ["pade_se"],
                    "psum": math.fsum(a.tolist())})
    return res


# A degree selection whose margin (ratio of a deciding singular value to the threshold 1e-12 s, or its
# reciprocal) is below this band may go either way between two sets of coefficients that differ by the
# path precision's rounding: FP64 coefficients agree to ~1e-13 s, FP32 ones to ~1e-5 s.
MARGIN_BAND = {64: 1e4, 32: 1e8}
FLAGGED = 1 | 32  # BRT_FLAG_POLE | BRT_FLAG_SENSITIVE


def _pole_kappa_flags(summ):
    return (1 if summ["pole"] else 0) | (32 if summ["sensitive"] else 0)


def compare_pade(wl, gpu, opade, pade_tol=1e-3):
    """Pade parity (reading R13), point by point.

    (a) Degrees: the device's degrees used (pade_diag columns 0, 1) equal the oracle's, except where the
        device's or the oracle's selection margin is inside MARGIN_BAND of the path precision (counted).
    (b) The Pade step itself, on the device's own coefficients: the oracle's summary of them gives the
        same degrees, value and neighbour values (1e-9 relative), sensitivity kappa (1e-3 relative: the
        oracle's gradient is a central difference) and LOWERED / POLE / SENSITIVE flags, the pole flag
        except where the oracle's pole distance from [0, 1] is within 0.01 of 0.5 (the device counts
        poles on a sampled contour) and the sensitivity flag except where kappa is within 1 % of 100.
    (c) End to end against the oracle's own Monte Carlo: |u_gpu - u_oracle| <= pade_tol at every point,
        except a point that the device flags POLE or SENSITIVE and that the oracle, on its own
        coefficients, flags POLE or SENSITIVE too.  There is no other allowance.
    (d) SE: the device's delta-method SE (exact gradient) against the oracle's (central differences) at
        unflagged points with equal degrees: 1e-4 (FP64) or 1e-2 (FP32) relative, plus a floor of
        1e-7 max|a| for zero-variance points.
    Returns (max |du| over unflagged points, points within pade_tol, points compared, points flagged on
    both sides, degree mismatches near the threshold)."""
    mc = wl["mc"]
    prec = int(mc["precision"])
    L, M = int(mc["pade_L"]), int(mc["pade_M"])
    no = int(mc["max_order"])
    band = MARGIN_BAND[prec]
    worst, strict, n, flagged, near = 0.0, 0, 0, 0, 0
    for p, r in enumerate(opade):
        ag = gpu["coef"][p][: no + 1]
        diag = gpu["pade_diag"][p]
        fl = int(gpu["flags"][p])
        if not np.all(np.isfinite(ag)) or r["used"] is None:
            continue
        dev_used = (int(diag[0]), int(diag[1]))
        # (b) the device's Pade step against the oracle's on the same coefficients
        o = oracle.pade_summary(ag, None, L, M)
        if o["order_margin"] >= 1e4 or diag[5] >= 1e4:
            assert o["pade_order"] == dev_used, (p, o["pade_order"], dev_used, o["order_margin"], diag[5])
        if o["pade_order"] == dev_used:
            v = o["pade"]
            assert abs(gpu["u"][p] - v) <= 1e-9 * max(1.0, abs(v)), (p, gpu["u"][p], v)
            for k, key in ((2, "pade_lo"), (3, "pade_mo")):
                ref = o[key]
                assert (math.isnan(ref) and math.isnan(diag[k])) or abs(diag[k] - ref) <= 1e-9 * max(1.0, abs(ref)), \
                    (p, key, diag[k], ref)
            assert abs(diag[4] - o["kappa"]) <= 1e-3 * o["kappa"] + 1e-12, (p, diag[4], o["kappa"])
            assert bool(fl & 2) == (dev_used != (L, M)), (p, fl)
            if abs(o["pole_distance"] - oracle.POLE_DIST) > 0.01:
                assert bool(fl & 1) == o["pole"], (p, fl, o["pole_distance"])
            if abs(o["kappa"] / oracle.SENSITIVE_KAPPA - 1.0) > 0.01:
                assert bool(fl & 32) == o["sensitive"], (p, fl, o["kappa"])
        # (a) degrees against the oracle's own coefficients
        if dev_used != r["used"]:
            assert min(diag[5], r["order_margin"]) < band, (p, dev_used, r["used"], diag[5], r["order_margin"])
            near += 1
        # (c) end to end
        du = abs(gpu["u"][p] - r["pade"])
        both = bool(fl & FLAGGED) and bool(_pole_kappa_flags(r) & FLAGGED)
        if both:
            flagged += 1
        else:
            assert du <= pade_tol, (p, gpu["u"][p], r["pade"], fl, r["pole_distance"], r["kappa"])
            worst = max(worst, du)
            strict += 1
            # (d) SE
            if dev_used == r["used"] and np.isfinite(r["se"]):
                se_tol = 1e-4 if prec == 64 else 1e-2
                floor = 1e-7 * float(np.abs(r["a"]).max())
                assert abs(gpu["se"][p] - r["se"]) <= se_tol * r["se"] + floor, (p, gpu["se"][p], r["se"])
        n += 1
    return worst, strict, n, flagged, near
