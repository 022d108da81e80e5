"""GPU-vs-oracle parity through the C ABI (needs an MI355X).

Every case prints its name, shape and seed before touching the GPU.  Tolerances are stated in
tests/_parity.py.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2402_06491_amd import inputs

from . import _parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "no GPU"
    import paper_2402_06491_amd as brt

    c = brt.Context(0)
    yield c
    c.close()


def _announce(name, wl):
    print(f"\n[case] {name}: points={len(wl['t'])} trees={int(np.sum(wl['n_trees']))} "
          f"precision={wl['mc']['precision']} seed={wl['mc']['seed']}", flush=True)


def _full_parity(ctx, name, wl, launch=None, pade_tol=1e-3):
    _announce(name, wl)
    tol = P.FP64_TOL if wl["mc"]["precision"] == 64 else P.FP32_TOL
    gpu = P.gpu_run(ctx, wl, launch=launch)
    pi, ti, ri = P.tree_items(wl)
    orc = P.oracle_trees(wl, pi, ti)
    worst = P.compare_trees(gpu, ri, orc, tol, pi)
    omom = P.oracle_moments(wl, orc, pi)
    P.compare_moments(wl, gpu, omom, tol)
    P.check_exact_sums(wl, gpu, ri, pi)
    opade = P.oracle_pade(wl, omom)
    B = oracle.n_bins(wl["mc"])
    for p, r in enumerate(opade):
        a = r["a"]
        np.testing.assert_allclose(gpu["coef"][p], a, rtol=0, atol=(tol + 1e-12) * np.abs(a).max() + 1e-300)
        assert abs(gpu["psum"][p] - r["psum"]) <= (tol + 1e-12) * np.abs(a).sum() + 1e-300
    du, strict, n, flagged, near = P.compare_pade(wl, gpu, opade, pade_tol)
    print(f"[case] {name}: max rel tree diff {worst:.3e}, max |du| {du:.3e} over {strict} unflagged points "
          f"(all within {pade_tol}), {flagged}/{n} flagged on both sides, {near} degree choices near the "
          f"threshold, bins {B}", flush=True)
    return gpu, orc


def test_kpp_small_fp64(ctx):
    wl = inputs.kpp(n_trees=3000)
    _full_parity(ctx, "kpp_small_fp64", wl)


def test_kpp_full_fp64(ctx):
    """The KPP workload at its full size (16 points x 1e5 trees): every tree against the oracle."""
    wl = inputs.kpp(n_trees=100_000)
    gpu, _ = _full_parity(ctx, "kpp_full_fp64", wl)
    assert np.all(gpu["flags"] & 24 == 0)


def test_fisher_small_fp32(ctx):
    wl = inputs.fisher(n_trees=1000)  # ragged: not a multiple of 64
    _full_parity(ctx, "fisher_small_fp32", wl)


def test_fisher_small_fp64(ctx):
    wl = inputs.fisher(n_trees=1000)
    wl["mc"] = dict(wl["mc"], precision=64)
    _full_parity(ctx, "fisher_small_fp64", wl)


def test_cubic_2d_small_fp32(ctx):
    wl = inputs.cubic_2d(n_trees=200, n_per_line=64)
    _full_parity(ctx, "cubic_2d_small_fp32", wl)


def test_poly_batch_small(ctx):
    for prec in (32, 64):
        wl = inputs.poly_batch(n_points=512, n_min=64, n_max=2000, precision=prec)
        _full_parity(ctx, f"poly_batch_small_fp{prec}", wl, pade_tol=1e-3)


def test_fisher_full_sampled(ctx):
    """Fisher at full size (192 points x 1e6 trees): sampled trees against the oracle; the reduction
    against an independent FP64 sum of the tree records; histogram totals."""
    import torch

    wl = inputs.fisher(n_trees=1_000_000)
    _announce("fisher_full_sampled", wl)
    gpu = P.gpu_run(ctx, wl)
    rng = np.random.default_rng(2024)
    pi = rng.integers(0, len(wl["t"]), size=4000)
    ti = rng.integers(0, 1_000_000, size=4000)
    _, _, ri = P.tree_items(wl, pi, ti)
    orc = P.oracle_trees(wl, pi, ti)
    worst = P.compare_trees(gpu, ri, orc, P.FP32_TOL, pi)
    B = oracle.n_bins(wl["mc"])
    assert np.all(gpu["hist"].sum(axis=1) == 1_000_000)
    # per-bin sums from the records with torch on the GPU (a different summation order)
    f = torch.from_numpy(gpu["tree_f"]).cuda().view(len(wl["t"]), -1)
    meta = torch.from_numpy(gpu["tree_meta"]).cuda().long().view(len(wl["t"]), -1)
    ne = (meta & 255).clamp(max=B - 1)
    ok = (meta & (7 << 8)) == 0
    for b in range(B):
        sel = ok & (ne == b)
        s1 = torch.where(sel, f, torch.zeros_like(f)).sum(dim=1).cpu().numpy()
        sa = torch.where(sel, f.abs(), torch.zeros_like(f)).sum(dim=1).cpu().numpy()
        assert np.all(np.abs(gpu["s1"][:, b] - s1) <= 1e-12 * sa + 1e-300), b
    print(f"[case] fisher_full_sampled: max rel tree diff {worst:.3e}", flush=True)


def _subset(wl, pts):
    """The workload restricted to the given points, keeping their Philox point ids."""
    pid = wl.get("point_id")
    pid = np.arange(len(wl["t"]), dtype=np.uint32) if pid is None else np.asarray(pid, np.uint32)
    return dict(wl, x=np.asarray(wl["x"])[pts], t=np.asarray(wl["t"])[pts], n_trees=np.asarray(wl["n_trees"])[pts],
                problem_id=np.asarray(wl["problem_id"])[pts], point_id=pid[pts])


@pytest.mark.parametrize("prec", [32, 64])
def test_poly_batch_full_size_sampled(ctx, prec):
    """The uneven batch at its full size (4096 points of 8 PDEs, 1e4..1e6 trees per point, about 8.8e8
    trees) in one launch, as the bench runs it: 16 sampled trees at each of 512 sampled points against
    the oracle tree by tree; and every tree of the 8 points with the fewest trees against the oracle's
    walk of them, through the moments (exact sums), coefficients and the Pade value (1e-3 unless both
    sides flag the point)."""
    import torch

    from paper_2402_06491_amd import Plan

    wl = inputs.poly_batch(precision=prec)
    _announce(f"poly_batch_full_size_sampled_fp{prec}", wl)
    tol = P.FP64_TOL if prec == 64 else P.FP32_TOL
    plan = Plan(ctx, wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"], problem_id=wl["problem_id"])
    out = plan.outputs(records=True)
    plan.execute(out)
    torch.cuda.synchronize()
    n_trees = np.asarray(wl["n_trees"], np.int64)
    base = np.concatenate([[0], np.cumsum(n_trees)])
    assert np.array_equal(out["hist"].sum(dim=1).cpu().numpy(), n_trees)

    rng = np.random.default_rng(77 + prec)
    pts = rng.choice(len(n_trees), size=512, replace=False)
    pi = np.repeat(pts, 16)
    ti = np.concatenate([rng.integers(0, n_trees[p], 16) for p in pts])
    rec = torch.as_tensor(base[pi] + ti, device="cuda")
    g = {"tree_f": out["tree_f"][rec].cpu().numpy(), "tree_meta": out["tree_meta"][rec].cpu().numpy()}
    orc = P.oracle_trees(wl, pi, ti)
    worst = P.compare_trees(g, np.arange(len(pi)), orc, tol, pi)

    full = np.sort(np.argsort(n_trees, kind="stable")[:8])
    sub = _subset(wl, full)
    rows = torch.as_tensor(full, device="cuda")
    g2 = {k: out[k][rows].cpu().numpy() for k in ("u", "se", "psum", "coef", "coef_var", "hist", "s1", "s2",
                                                  "nodes", "flags", "pade_diag")}
    recs = torch.cat([torch.arange(int(base[p]), int(base[p + 1]), device="cuda") for p in full])
    g2["tree_f"] = out["tree_f"][recs].cpu().numpy()
    g2["tree_meta"] = out["tree_meta"][recs].cpu().numpy()
    plan.close()
    del out
    spi, sti, sri = P.tree_items(sub)
    sorc = P.oracle_trees(sub, spi, sti)
    P.compare_trees(g2, sri, sorc, tol, spi)
    omom = P.oracle_moments(sub, sorc, spi)
    P.compare_moments(sub, g2, omom, tol)
    P.check_exact_sums(sub, g2, sri, spi)
    opade = P.oracle_pade(sub, omom)
    du, strict, n, flagged, near = P.compare_pade(sub, g2, opade, 1e-3)
    print(f"[case] poly_batch_full_size_sampled_fp{prec}: {len(pi)} sampled trees, max rel diff {worst:.3e}; "
          f"{int(n_trees[full].sum())} trees of {len(full)} points in full: max |du| {du:.3e} over {strict} "
          f"unflagged points, {flagged} flagged on both sides, {near} degree choices near the threshold", flush=True)


# ---------------------------------------------------------------- edge cases --------------------
def test_edge_empty_and_ragged_points(ctx):
    wl = inputs.fisher(n_trees=1, n_x=6, times=(0.5,))
    wl["n_trees"] = np.array([0, 1, 63, 64, 65, 1500], np.int64)
    gpu, _ = _full_parity(ctx, "edge_empty_ragged", wl)
    assert gpu["hist"][0].sum() == 0 and gpu["u"][0] == 0.0


def test_edge_zero_points(ctx):
    """A plan, brt_solve and brt_solve_noalloc with no points at all run (their kernels find no work)
    and return empty outputs."""
    import torch

    import paper_2402_06491_amd as brt
    from paper_2402_06491_amd import Plan

    wl = inputs.fisher(n_trees=10, n_x=1, times=(0.5,))
    x, t, nt = np.zeros((0, 1)), np.zeros(0), np.zeros(0, np.int64)
    _announce("edge_zero_points", dict(wl, x=x, t=t, n_trees=nt))
    plan = Plan(ctx, wl["problems"], wl["mc"], x, t, nt)
    try:
        out = plan.outputs(records=True)
        plan.execute(out)
        s = torch.cuda.Stream()  # a created stream: the step is captured into a graph, then replayed
        plan.execute(out, stream=s)
        plan.execute(out, stream=s)
        torch.cuda.synchronize()
        assert out["u"].numel() == 0 and out["hist"].shape[0] == 0
    finally:
        plan.close()
    for na in (False, True):
        o = brt.solve(ctx, wl["problems"], wl["mc"], x, t, nt, noalloc=na)
        torch.cuda.synchronize()
        assert o["u"].numel() == 0 and o["se"].numel() == 0


def test_edge_time_zero_and_no_nonlinearity(ctx):
    wl = inputs.fisher(n_trees=500, n_x=8, times=(0.0,))
    _full_parity(ctx, "edge_t0", wl)
    g = inputs.gauss_sum([(1 / math.sqrt(4 * math.pi), 0.0, 0.0, math.sqrt(2.0))])
    wl = {"problems": [inputs.problem(1, 1.0, [0, 0, 0], g)], "mc": inputs.mc_params(seed=3, precision=64),
          "x": np.linspace(-2, 2, 5).reshape(-1, 1), "t": np.full(5, 1.0), "n_trees": np.full(5, 700)}
    gpu, _ = _full_parity(ctx, "edge_heat_kernel", wl)
    assert np.all(gpu["nodes"] == 700)


def test_edge_node_cap_and_order_zero(ctx):
    wl = inputs.kpp(n_trees=800)
    wl["mc"] = dict(wl["mc"], node_cap=5)
    gpu, _ = _full_parity(ctx, "edge_node_cap", wl)
    assert np.all(gpu["flags"] & 8)
    wl = inputs.fisher(n_trees=800, n_x=4, times=(1.0,))
    wl["mc"] = dict(wl["mc"], max_order=0, pade_L=0, pade_M=0)
    _full_parity(ctx, "edge_order_zero", wl)


def test_edge_max_order_and_mixed_problems(ctx):
    wl = inputs.kpp(n_trees=600)
    wl["mc"] = dict(wl["mc"], max_order=62, prune=1, pade_L=8, pade_M=8)
    _full_parity(ctx, "edge_max_order_62", wl)
    probs = []
    for k in range(16):
        rng = np.random.default_rng(100 + k)
        probs.append(inputs.problem(1, rng.uniform(0.3, 1.5), list(rng.uniform(-1, 1, size=4)),
                                    inputs.logistic(0.6, 1.0, rng.uniform(-1, 1), 1)))
    rng = np.random.default_rng(9)
    n = 64
    wl = {"problems": probs, "mc": inputs.mc_params(seed=77, precision=32),
          "x": rng.uniform(-3, 3, size=(n, 1)), "t": rng.uniform(0.1, 1.5, size=n),
          "n_trees": rng.integers(0, 900, size=n), "problem_id": rng.integers(0, 16, size=n).astype(np.uint32),
          "point_id": rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)}
    _full_parity(ctx, "edge_16_problems", wl, pade_tol=1e-3)


def test_edge_max_trees_per_point(ctx):
    """One point with the largest tree count a plan takes (2^32 - 1 trees: 51.5 GB of tree records) and
    no non-linear term (every tree is one leaf), FP32 paths: every tree is counted exactly once, by a
    reduction whose last segments end next to 2^32; the value matches the heat-kernel mean within its
    Monte Carlo error; trees at both ends of the Philox tree counter agree with the oracle."""
    import torch

    from paper_2402_06491_amd import Plan

    nt = (1 << 32) - 1
    g = inputs.gauss_sum([(1.0, 0.0, 0.0, 1.0)])
    wl = {"problems": [inputs.problem(1, 1.0, [0, 0, 0], g)], "mc": inputs.mc_params(seed=11, precision=32),
          "x": np.array([[0.3]]), "t": np.array([1.0]), "n_trees": np.array([nt], np.int64)}
    _announce("edge_max_trees_per_point", wl)
    plan = Plan(ctx, wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"])
    out = plan.outputs(records=True)
    try:
        plan.execute(out)
        torch.cuda.synchronize()
        B = oracle.n_bins(wl["mc"])
        hist = out["hist"].cpu().numpy()[0]
        assert int(hist[0]) == nt and int(hist[:B].sum()) == nt and int(hist[B:].sum()) == 0, hist
        assert int(out["nodes"].cpu().numpy()[0]) == nt
        ti = np.array([0, 1, 2, 777, 65535, 65536, nt - 65537, nt - 3, nt - 2, nt - 1], np.int64)
        pi = np.zeros(len(ti), np.int64)
        rec = torch.as_tensor(ti, device="cuda")
        gt = {"tree_f": out["tree_f"][rec].cpu().numpy(), "tree_meta": out["tree_meta"][rec].cpu().numpy()}
        orc = P.oracle_trees(wl, pi, ti)
        P.compare_trees(gt, np.arange(len(ti)), orc, P.FP32_TOL, pi)
        # u_t = u_xx from a Gaussian of width 1: the width grows to sqrt(1 + 2t)
        exact = math.exp(-0.3 ** 2 / (2 * 3.0)) / math.sqrt(3.0)
        u = float(out["u"].cpu().numpy()[0])
        se = float(out["se"].cpu().numpy()[0])
        print(f"[case] edge_max_trees_per_point: u {u:.9f} exact {exact:.9f} se {se:.2e}", flush=True)
        assert abs(u - exact) <= 6 * se + 1e-6, (u, exact, se)
    finally:
        plan.close()
        del out
        torch.cuda.empty_cache()


def test_edge_cos2_bump_2d(ctx):
    prob = inputs.problem(2, 1.0, [0, 0, -1.25, -1.0], {"u0_kind": "cos2_bump", "u0_params": [-2.0, 10.0, 40.0],
                                                         "u0_nterms": 0})
    rng = np.random.default_rng(4)
    wl = {"problems": [prob], "mc": inputs.mc_params(seed=5, precision=32),
          "x": rng.uniform(-12, 12, size=(40, 2)), "t": np.full(40, 0.5), "n_trees": np.full(40, 300)}
    _full_parity(ctx, "edge_cos2_bump_2d", wl, pade_tol=1e-3)


def test_edge_small_chunks_and_stack_depth(ctx):
    """Tiny chunks (one wave's worth) and the smallest stack that the workload needs."""
    wl = inputs.fisher(n_trees=700, n_x=8)
    _full_parity(ctx, "edge_chunk64", wl, launch={"chunk_trees": 64, "waves_per_block": 1})
    ctx.set_launch()


def test_graph_replay_matches_direct_enqueue_and_oracle(ctx):
    """A plan run on a created stream is captured once into a HIP graph and replayed; its outputs are
    bit-identical to the same plan enqueued kernel by kernel and to a fresh plan, and they match the
    oracle tree by tree."""
    import torch

    from paper_2402_06491_amd import Plan

    wl = inputs.fisher(n_trees=5000, n_x=16)
    _announce("graph_replay", wl)
    stream = torch.cuda.Stream()
    plan = Plan(ctx, wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"])
    out = plan.outputs()
    results = []
    with torch.cuda.stream(stream):
        for _ in range(3):
            plan.execute(out, stream=stream)
            stream.synchronize()
            results.append({k: v.cpu().numpy().copy() for k, v in out.items()})
            for v in out.values():
                v.zero_()
            stream.synchronize()
    st = plan.graph_stats()
    assert st == {"captures": 1, "replays": 3, "direct": 0}, st
    # the same plan, kernel by kernel on the same stream
    plan.set_graph(False)
    with torch.cuda.stream(stream):
        plan.execute(out, stream=stream)
        stream.synchronize()
    results.append({k: v.cpu().numpy().copy() for k, v in out.items()})
    assert plan.graph_stats()["direct"] == 1
    plan2 = Plan(ctx, wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"])
    out2 = plan2.outputs()
    plan2.execute(out2)  # torch's default stream (NULL): enqueued directly
    torch.cuda.synchronize()
    assert plan2.graph_stats() == {"captures": 0, "replays": 0, "direct": 1}
    results.append({k: v.cpu().numpy() for k, v in out2.items()})
    for r in results[1:]:
        for k in r:
            np.testing.assert_array_equal(r[k], results[0][k], err_msg=k)
    # and the replayed results are the oracle's trees
    pi, ti, ri = P.tree_items(wl)
    orc = P.oracle_trees(wl, pi, ti)
    P.compare_trees(results[2], ri, orc, P.FP32_TOL, pi)
    plan.close()
    plan2.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_strategy_b_fisher(ctx, prec):
    wl = inputs.fisher(n_trees=1000)
    wl["mc"] = dict(wl["mc"], precision=prec, strategy=1, q=0.55)
    _full_parity(ctx, f"strategy_b_fisher_fp{prec}", wl)


def test_strategy_b_cubic_2d_and_batch(ctx):
    wl = inputs.cubic_2d(n_trees=200, n_per_line=64)
    wl["mc"] = dict(wl["mc"], strategy=1, q=0.7)
    _full_parity(ctx, "strategy_b_cubic_2d", wl)
    wl = inputs.poly_batch(n_points=256, n_min=64, n_max=1500, precision=32)
    wl["mc"] = dict(wl["mc"], strategy=1, q=0.8)
    _full_parity(ctx, "strategy_b_poly_batch", wl)


def test_strategy_b_unpruned_and_heat(ctx):
    """Subcritical Galton-Watson trees without pruning (tail bin), and q forced to 1 at f = 0."""
    wl = inputs.kpp(n_trees=2000)
    wl["mc"] = dict(wl["mc"], strategy=1, q=0.6)
    _full_parity(ctx, "strategy_b_kpp_unpruned", wl)
    g = inputs.gauss_sum([(1 / math.sqrt(4 * math.pi), 0.0, 0.0, math.sqrt(2.0))])
    wl = {"problems": [inputs.problem(1, 1.0, [0, 0, 0], g)],
          "mc": inputs.mc_params(seed=3, precision=64, strategy=1, q=0.5),
          "x": np.linspace(-2, 2, 5).reshape(-1, 1), "t": np.full(5, 1.0), "n_trees": np.full(5, 700)}
    gpu, _ = _full_parity(ctx, "strategy_b_heat_kernel", wl)
    assert np.all(gpu["nodes"] == 700)


@pytest.mark.parametrize("prec", [32, 64])
def test_variable_coefficients_example5(ctx, prec):
    """The paper's Example 5 coefficient -e^{-x^2}/(t + 0.1), evaluated at every split."""
    wl = inputs.example5(n_trees=1500, n_x=24, precision=prec)
    _full_parity(ctx, f"example5_fp{prec}", wl)


def test_variable_coefficients_2d_strategy_b_and_mixed(ctx):
    prob = inputs.problem(2, 0.8, [0.1, -0.4, 0.6, -0.5], inputs.cubic_2d_u0(3),
                          coef_mod={"beta": (0.3, 0.7), "t0": 0.2, "pow": 1})
    x = inputs.interface_points(16)[::3]
    n = len(x)
    wl = {"problems": [prob], "mc": inputs.mc_params(seed=12, precision=32, strategy=1, q=0.55), "x": x,
          "t": np.full(n, 0.9), "n_trees": np.full(n, 700)}
    _full_parity(ctx, "varcoef_2d_strategy_b", wl)
    # constant and variable coefficients in one launch (per-lane problem tables)
    plain = inputs.problem(2, 0.8, [0.1, -0.4, 0.6, -0.5], inputs.cubic_2d_u0(3))
    space = inputs.problem(2, 0.8, [0.1, -0.4, 0.6, -0.5], inputs.cubic_2d_u0(3),
                           coef_mod={"beta": (0.5, 0.0), "t0": 0.0, "pow": 0})
    wl = {"problems": [plain, prob, space], "mc": inputs.mc_params(seed=13, precision=64), "x": x,
          "t": np.full(n, 0.7), "n_trees": np.full(n, 500), "problem_id": (np.arange(n) % 3).astype(np.uint32)}
    _full_parity(ctx, "varcoef_mixed_problems", wl)


@pytest.mark.parametrize("prec", [32, 64])
def test_drift_fisher_moving_frame(ctx, prec):
    """Fisher with a constant drift b = 0.8 (L = Lap + b d/dx): the paths gain b times each edge's
    duration; Strategy A, pruned order 10."""
    prob = inputs.problem(1, 1.0, [0.0, 1.0, -1.0], inputs.logistic(1.0, 1.0 / math.sqrt(6.0), 0.0, 2), drift=(0.8,))
    x = np.linspace(-6.0, 6.0, 20).reshape(-1, 1)
    wl = {"problems": [prob], "mc": inputs.mc_params(seed=31, max_order=10, pade=(5, 5), precision=prec), "x": x,
          "t": np.full(20, 1.0), "n_trees": np.full(20, 1500)}
    _full_parity(ctx, f"drift_fisher_fp{prec}", wl)


def test_drift_2d_strategy_b_with_variable_coefficients_and_mixed(ctx):
    """2-D cubic with drift (0.9, -0.4) under Strategy B, with and without variable coefficients, and
    a drift-free problem in the same launch."""
    x = inputs.interface_points(16)[::3]
    n = len(x)
    drifted = inputs.problem(2, 0.8, [0.1, -0.4, 0.6, -0.5], inputs.cubic_2d_u0(3), drift=(0.9, -0.4))
    both = inputs.problem(2, 0.8, [0.1, -0.4, 0.6, -0.5], inputs.cubic_2d_u0(3), drift=(0.9, -0.4),
                          coef_mod={"beta": (0.3, 0.7), "t0": 0.2, "pow": 1})
    plain = inputs.problem(2, 0.8, [0.1, -0.4, 0.6, -0.5], inputs.cubic_2d_u0(3))
    wl = {"problems": [drifted], "mc": inputs.mc_params(seed=32, precision=64, strategy=1, q=0.55), "x": x,
          "t": np.full(n, 0.9), "n_trees": np.full(n, 600)}
    _full_parity(ctx, "drift_2d_strategy_b", wl)
    wl = {"problems": [plain, drifted, both], "mc": inputs.mc_params(seed=33, precision=32), "x": x,
          "t": np.full(n, 0.7), "n_trees": np.full(n, 500), "problem_id": (np.arange(n) % 3).astype(np.uint32)}
    _full_parity(ctx, "drift_mixed_problems", wl)


@pytest.mark.parametrize("prec", [32, 64])
def test_modulated_linear_term(ctx, prec):
    """c_1 modulated too (coef_mod "linear"): c_1(x, t) u is sampled as a branching with one child;
    1-D Strategy A and 2-D Strategy B."""
    p1 = inputs.problem(1, 1.0, [0.0, 0.9, -1.0], inputs.logistic(1.0, 1.0 / math.sqrt(6.0), 0.0, 2),
                        coef_mod={"beta": (0.4, 0.0), "t0": 0.1, "pow": 1, "linear": True})
    x = np.linspace(-5.0, 5.0, 16).reshape(-1, 1)
    wl = {"problems": [p1], "mc": inputs.mc_params(seed=41, max_order=10, pade=(5, 5), precision=prec), "x": x,
          "t": np.full(16, 0.8), "n_trees": np.full(16, 1200)}
    _full_parity(ctx, f"linear_modulated_1d_fp{prec}", wl)
    p2 = inputs.problem(2, 0.8, [0.1, -0.7, 0.6, -0.5], inputs.cubic_2d_u0(2),
                        coef_mod={"beta": (0.3, 0.7), "t0": 0.2, "pow": 1, "linear": True})
    x2 = inputs.interface_points(16)[::4]
    wl = {"problems": [p2], "mc": inputs.mc_params(seed=42, precision=prec, strategy=1, q=0.55), "x": x2,
          "t": np.full(len(x2), 0.8), "n_trees": np.full(len(x2), 600)}
    _full_parity(ctx, f"linear_modulated_2d_b_fp{prec}", wl)


def test_euler_maruyama_general_operator(ctx):
    """A general L (b(x) = b + B x, sigma(x) with a Gaussian bump) integrated by Euler-Maruyama steps of at
    most h: FP64 paths tree by tree (on FP32 paths a step count ceil(s/h) may round differently from
    the oracle's FP64 one at an exact step boundary).  The linear drifts contract (an expanding one
    sends paths far out, where e^{-beta x^2} of the variable coefficients magnifies last-bit
    differences past the FP64 tree bound).  1-D Fisher under Strategy A with 10+ steps per
    unit time, and a 2-D Strategy B problem with variable coefficients and c_1(x, t) as well."""
    p1 = inputs.problem(1, 1.0, [0.0, 1.0, -1.0], inputs.logistic(1.0, 1.0 / math.sqrt(6.0), 0.0, 2), drift=(0.4,),
                        euler={"dt": 0.09, "drift_lin": (-0.6,), "sigma_amp": 0.5, "sigma_width": 2.0})
    x = np.linspace(-5.0, 5.0, 12).reshape(-1, 1)
    wl = {"problems": [p1], "mc": inputs.mc_params(seed=51, max_order=10, pade=(5, 5), precision=64), "x": x,
          "t": np.full(12, 1.0), "n_trees": np.full(12, 800)}
    _full_parity(ctx, "euler_fisher_fp64", wl)
    p2 = inputs.problem(2, 0.8, [0.1, -0.7, 0.6, -0.5], inputs.cubic_2d_u0(2), drift=(0.3, -0.2),
                        coef_mod={"beta": (0.3, 0.7), "t0": 0.2, "pow": 1, "linear": True},
                        euler={"dt": 0.07, "drift_lin": (-0.5, -0.3), "sigma_amp": 0.4, "sigma_width": 1.5})
    x2 = inputs.interface_points(16)[::5]
    wl = {"problems": [p2], "mc": inputs.mc_params(seed=52, precision=64, strategy=1, q=0.55), "x": x2,
          "t": np.full(len(x2), 0.8), "n_trees": np.full(len(x2), 400)}
    _full_parity(ctx, "euler_2d_strategy_b_fp64", wl)


def test_launch_settings_do_not_change_results(ctx):
    """Every tree is computed by one lane from its own counters and segments are fixed, so launch
    settings (block size, LDS stack levels, chunk size) change nothing in the outputs."""
    wl = inputs.fisher(n_trees=3000, n_x=8)
    _announce("launch_settings", wl)
    ref = None
    for launch in ({"waves_per_block": 4, "chunk_trees": 1024, "stack_depth": 8},
                   {"waves_per_block": 1, "chunk_trees": 256, "stack_depth": 2},
                   {"waves_per_block": 2, "chunk_trees": 4096, "stack_depth": 12}):
        res = P.gpu_run(ctx, wl, launch=launch)
        res.pop("plan")
        if ref is None:
            ref = res
        else:
            for k in ref:
                np.testing.assert_array_equal(res[k], ref[k], err_msg=f"{k} {launch}")
    ctx.set_launch()


def test_autotune_and_cache(ctx, tmp_path):
    wl = inputs.fisher(n_trees=20000, n_x=16)
    _announce("autotune", wl)
    path = str(tmp_path / "tune.jsonl")
    best = ctx.autotune(wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"], cache_path=path)
    assert best["waves_per_block"] in (1, 2, 4) and best["chunk_trees"] in (256, 1024, 4096)
    assert ctx.get_launch()["stack_depth"] == best["stack_depth"]
    lines = open(path).read().strip().split("\n")
    assert len(lines) == 1 and '"key": "' in lines[0]
    ctx.set_launch()
    again = ctx.autotune(wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"], cache_path=path)
    assert again == best and len(open(path).read().strip().split("\n")) == 1
    _full_parity(ctx, "after_autotune", inputs.fisher(n_trees=500, n_x=8))
    ctx.set_launch()


def test_alone_equals_in_batch(ctx):
    """A point's results alone equal its results inside a larger mixed batch (bit-identical)."""
    wl = inputs.poly_batch(n_points=256, n_min=64, n_max=3000, precision=32)
    wl["point_id"] = np.arange(256, dtype=np.uint32)
    _announce("alone_vs_batch", wl)
    batch = P.gpu_run(ctx, wl, records=False)
    for p in (0, 17, 255):
        one = {"problems": wl["problems"], "mc": wl["mc"], "x": wl["x"][p:p + 1], "t": wl["t"][p:p + 1],
               "n_trees": wl["n_trees"][p:p + 1], "problem_id": wl["problem_id"][p:p + 1],
               "point_id": wl["point_id"][p:p + 1]}
        alone = P.gpu_run(ctx, one, records=False)
        for k in ("u", "se", "coef", "hist", "s1", "s2", "nodes"):
            np.testing.assert_array_equal(alone[k][0], batch[k][p], err_msg=f"{k} point {p}")


@pytest.mark.parametrize("prec", [32, 64])
def test_family_batch(ctx, prec):
    """Problems that differ only in their initial data (Gaussian sums of 1, 3 and 8 terms, the same
    coefficients) form a family: one launch keeps only their initial data per problem.  Against the
    oracle, and every sampled point bit-identical to the same point solved with its problem alone."""
    probs = []
    for k, nterms in enumerate((1, 3, 8)):
        r = np.random.default_rng(300 + k)
        probs.append(inputs.problem(2, 1.0, [0.0, 1.0, 0.0, -1.0], inputs.gauss_sum(
            [(r.uniform(0.2, 1.0), r.uniform(-3, 3), r.uniform(-3, 3), r.uniform(0.5, 2.0)) for _ in range(nterms)])))
    rng = np.random.default_rng(12)
    n = 48
    wl = {"problems": probs, "mc": inputs.mc_params(seed=5, precision=prec),
          "x": rng.uniform(-4, 4, size=(n, 2)), "t": rng.uniform(0.2, 1.0, size=n),
          "n_trees": rng.integers(1, 700, size=n), "problem_id": (np.arange(n) % 3).astype(np.uint32),
          "point_id": np.arange(n, dtype=np.uint32)}
    gpu, _ = _full_parity(ctx, f"family_batch_fp{prec}", wl)
    for p in (0, 1, 2, 47):
        k = int(wl["problem_id"][p])
        one = {"problems": [probs[k]], "mc": wl["mc"], "x": wl["x"][p:p + 1], "t": wl["t"][p:p + 1],
               "n_trees": wl["n_trees"][p:p + 1], "problem_id": np.zeros(1, np.uint32),
               "point_id": wl["point_id"][p:p + 1]}
        alone = P.gpu_run(ctx, one, records=False)
        for key in ("u", "se", "coef", "hist", "s1", "s2", "nodes"):
            np.testing.assert_array_equal(alone[key][0], gpu[key][p], err_msg=f"{key} point {p}")
