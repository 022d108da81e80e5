"""Domain-decomposition tail on the GPU against the oracle (needs an MI355X).

Node values given to both sides are synthetic (seeded) or computed by each side's own Monte Carlo;
nothing the GPU computes is fed to the oracle.  Tolerances: the spline and the solver are FP64 with the
same operations in a different order (Thomas recurrence vs banded LU, fused multiply-adds), so
boundary data agree to 1e-12 and fields to 1e-11 of their largest magnitude.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import pdd as opdd
from paper_2402_06491_amd import inputs

from . import _parity as P

pytestmark = pytest.mark.gpu

BD_TOL = 1e-12
FIELD_TOL = 1e-11


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "no GPU"
    import paper_2402_06491_amd as brt

    c = brt.Context(0)
    yield c
    c.close()


def _announce(name, grid):
    print(f"\n[case] {name}: px={grid['px']} py={grid['py']} cx={grid['cx']} cy={grid['cy']} "
          f"steps={grid['n_steps']} ns={grid['ns_x']}x{grid['ns_y']} nt={grid['nt']} outer={grid['outer']}",
          flush=True)


def _grid(**kw):
    g = {"x_lo": -4.0, "x_hi": 4.0, "y_lo": -4.0, "y_hi": 4.0, "px": 2, "py": 2, "cx": 16, "cy": 16, "T": 0.5,
         "n_steps": 40, "ns_x": 9, "ns_y": 9, "nt": 4, "outer": "mc"}
    g.update(kw)
    return g


def _cubic(seed=0):
    return inputs.problem(2, 1.0, [0.0, 1.0, 0.0, -1.0], inputs.cubic_2d_u0(seed))


def _tail_parity(ctx, name, problem, grid, node_values, steps=None, groups=None):
    import torch

    import paper_2402_06491_amd as brt

    _announce(name, grid)
    og = opdd.Grid(**grid)
    pd = brt.Pdd(ctx, problem, grid)
    try:
        xy, t = pd.nodes()
        oxy, ot = opdd.node_points(og)
        np.testing.assert_array_equal(xy, oxy)
        np.testing.assert_array_equal(t, ot)
        o, c, f = pd.lines()
        assert [(int(a), float(b)) for a, b in zip(o, c)] == [(0 if s == "v" else 1, cc) for s, _, cc in og.lines()]
        pd.interpolate(torch.tensor(node_values, dtype=torch.float64, device="cuda"))
        obd = opdd.boundary_data(og, problem, node_values)
        scale = max(float(np.abs(v).max()) for v in obd.values())
        for li in range(len(o)):
            gb = pd.boundary(li).cpu().numpy()
            np.testing.assert_allclose(gb, obd[li], rtol=0, atol=BD_TOL * scale, err_msg=f"line {li}")
        steps = grid["n_steps"] if steps is None else steps
        field = pd.solve(steps).cpu().numpy()
        ms = pd.timing()
        n_groups, die_local = pd.barrier()
        print(f"[case] {name}: {n_groups} barrier groups, {die_local} on one die", flush=True)
        if groups is not None:
            # blocks are dealt to the dies round-robin and every group is formed from the blocks of one
            # die, so its barriers take the die-local fences
            assert (n_groups, die_local) == (groups, groups)
        ofield = opdd.adi_solve(og, problem, obd, n_steps=steps)
        err = float(np.abs(field - ofield).max())
        print(f"[case] {name}: max |dU| {err:.3e} of max |U| {np.abs(ofield).max():.3e}; "
              f"interp {ms[1]:.3f} ms, solve {ms[2]:.3f} ms", flush=True)
        np.testing.assert_allclose(field, ofield, rtol=0, atol=FIELD_TOL * max(1.0, float(np.abs(ofield).max())))
        return field, ofield
    finally:
        pd.close()


def test_tail_small_synthetic_nodes(ctx):
    grid = _grid()
    og = opdd.Grid(**grid)
    rng = np.random.default_rng(11)
    xy, t = opdd.node_points(og)
    vals = 0.5 * np.exp(-(xy[:, 0] ** 2 + xy[:, 1] ** 2) / 8.0) * (1 + t) + 0.01 * rng.normal(size=len(t))
    _tail_parity(ctx, "tail_small_synthetic", _cubic(), grid, vals)


def test_tail_ragged_zero_outer_fisher(ctx):
    """3 x 2 subdomains of 20 x 70 cells (x blocks ragged against 64 lanes, y items span two blocks),
    outer edges held at zero, Fisher reaction, logistic initial data."""
    grid = _grid(x_lo=-6.0, x_hi=6.0, px=3, py=2, cx=20, cy=70, n_steps=30, ns_x=13, ns_y=5, nt=3, outer="zero",
                 T=0.3)
    prob = inputs.problem(2, 1.0, [0.0, 1.0, -1.0], inputs.logistic(1.0, 1.0 / math.sqrt(6.0), 0.0, 2,
                                                                  (math.cos(0.4), math.sin(0.4))))
    og = opdd.Grid(**grid)
    xy, t = opdd.node_points(og)
    vals = opdd.fisher_plane_wave(0.4)(xy[:, 0], xy[:, 1], t)
    _tail_parity(ctx, "tail_ragged_zero_outer", prob, grid, vals)


def test_tail_single_subdomain_and_cos2(ctx):
    grid = _grid(px=1, py=1, cx=37, cy=29, n_steps=25, ns_x=4, ns_y=6, nt=5)
    prob = inputs.problem(2, 0.5, [0.1, -0.3, 0.0, -0.2], {"u0_kind": "cos2_bump", "u0_params": [-2.0, 3.0, 3.5],
                                                               "u0_nterms": 0})
    og = opdd.Grid(**grid)
    rng = np.random.default_rng(3)
    vals = rng.uniform(-0.1, 0.1, size=len(opdd.node_points(og)[1]))
    _tail_parity(ctx, "tail_single_cos2", prob, grid, vals)


def test_tail_odd_subdomain_width(ctx):
    """3 x 2 subdomains of 21 x 19 cells: with an odd width the y sweep's column pairs of the middle
    subdomain start on 8-byte (not 16-byte) boundaries, and the last pair of each strip is ragged."""
    grid = _grid(px=3, py=2, cx=21, cy=19, n_steps=20, ns_x=11, ns_y=7, nt=4)
    og = opdd.Grid(**grid)
    rng = np.random.default_rng(23)
    xy, t = opdd.node_points(og)
    vals = 0.3 * np.cos(0.4 * xy[:, 0]) * np.exp(-xy[:, 1] ** 2 / 10.0) * (1 + 0.5 * t) + 0.01 * rng.normal(size=len(t))
    _tail_parity(ctx, "tail_odd_width", _cubic(1), grid, vals)


@pytest.mark.parametrize("px,py", [(4, 2), (4, 4), (6, 4)])
def test_tail_die_barrier_groups(ctx, px, py):
    """8, 16 and 24 small subdomains: the solver launches one block per subdomain and, with the subdomains
    split evenly over the dies, synchronises each subdomain's blocks among themselves (one group per
    subdomain) through their die's L2; the subdomains then never read each other's field values."""
    grid = _grid(x_lo=-6.0, x_hi=6.0, px=px, py=py, cx=16, cy=12, n_steps=30, ns_x=13, ns_y=9, nt=3, T=0.3)
    og = opdd.Grid(**grid)
    rng = np.random.default_rng(px * 10 + py)
    xy, t = opdd.node_points(og)
    vals = 0.5 * np.exp(-(xy[:, 0] ** 2 + xy[:, 1] ** 2) / 12.0) * (1 + t) + 0.02 * rng.normal(size=len(t))
    _tail_parity(ctx, f"tail_groups_{px}x{py}", _cubic(3), grid, vals, groups=px * py)


def test_tail_die_groups_of_several_subdomains(ctx):
    """8 x 5 subdomains of 16 x 224 cells: 280 x items over 144 blocks, which do not split evenly over
    the 40 subdomains, so each die's 18 blocks form one barrier group for its 5 subdomains (two rounds
    of x items, most blocks idle in the y phase)."""
    grid = _grid(x_lo=-6.0, x_hi=6.0, y_lo=-6.0, y_hi=6.0, px=8, py=5, cx=16, cy=224, n_steps=12, ns_x=17, ns_y=57,
                 nt=3, T=0.2)
    og = opdd.Grid(**grid)
    rng = np.random.default_rng(85)
    xy, t = opdd.node_points(og)
    vals = 0.5 * np.exp(-(xy[:, 0] ** 2 + xy[:, 1] ** 2) / 15.0) * (1 + 0.5 * t) + 0.02 * rng.normal(size=len(t))
    _tail_parity(ctx, "tail_die_groups_8x5", _cubic(4), grid, vals, groups=8)


def test_tail_long_lines_in_subdomain_groups(ctx):
    """4 x 2 subdomains of 600 x 20 cells: the 32-unknown segment shape (16 lines per item) under one
    barrier group per subdomain (152 blocks, 19 per subdomain)."""
    grid = _grid(x_lo=-6.0, x_hi=6.0, px=4, py=2, cx=600, cy=20, n_steps=10, ns_x=65, ns_y=7, nt=3, T=0.2)
    og = opdd.Grid(**grid)
    xy, t = opdd.node_points(og)
    vals = 0.4 * np.exp(-(xy[:, 0] ** 2 + 2.0 * xy[:, 1] ** 2) / 8.0) * (1.0 + t)
    _tail_parity(ctx, "tail_long_lines_groups", _cubic(5), grid, vals, groups=8)


def test_tail_long_lines_32_unknown_segments(ctx):
    """2 x 1 subdomains of 600 x 30 cells: lines of 599 unknowns take the solver's 32-unknown segments
    (the ragged last segment holds 23), and the short y lines leave most segments empty."""
    grid = _grid(x_lo=-6.0, x_hi=6.0, px=2, py=1, cx=600, cy=30, n_steps=12, ns_x=41, ns_y=7, nt=3, T=0.2,
                 outer="zero")
    og = opdd.Grid(**grid)
    xy, t = opdd.node_points(og)
    vals = 0.4 * np.exp(-(xy[:, 0] ** 2 + 2.0 * xy[:, 1] ** 2) / 6.0) * (1.0 - t)
    _tail_parity(ctx, "tail_long_lines", _cubic(2), grid, vals)


def test_tail_modulated_linear_term(ctx):
    """c_1 modulated with the other coefficients: f = m(x, y, t) (c_1 u + c_3 u^3) in the subdomain solves."""
    grid = _grid(n_steps=30)
    prob = inputs.problem(2, 1.0, [0.0, 1.0, 0.0, -1.0], inputs.cubic_2d_u0(0),
                          coef_mod={"beta": (0.05, 0.08), "t0": 0.3, "pow": 1, "linear": True})
    og = opdd.Grid(**grid)
    xy, t = opdd.node_points(og)
    vals = opdd.g_grid(prob, xy[:, 0], xy[:, 1]) * np.exp(-0.2 * t)
    _tail_parity(ctx, "tail_linear_modulated", prob, grid, vals)


def test_tail_rejects_a_drift(ctx):
    import paper_2402_06491_amd as brt

    prob = inputs.problem(2, 1.0, [0.0, 1.0, 0.0, -1.0], inputs.cubic_2d_u0(0), drift=(0.5, 0.0))
    with pytest.raises(brt.BrtError, match="drift"):
        brt.Pdd(ctx, prob, _grid())
    prob = inputs.problem(2, 1.0, [0.0, 1.0, 0.0, -1.0], inputs.cubic_2d_u0(0), euler={"dt": 0.01})
    with pytest.raises(brt.BrtError, match="constant sigma"):
        brt.Pdd(ctx, prob, _grid())


def test_tail_full_size_first_steps(ctx):
    """The decomposition of the 2-D cubic workload at its full size (4 x 4 subdomains of 512^2 cells,
    264 nodes per line on 10 lines, 1000 steps of boundary data), solved through its first 100 steps in
    the benchmark's launch (256 blocks, one die-local barrier group of 16 blocks per subdomain)."""
    wl = inputs.pdd_cubic_2d()
    grid = wl["grid"]
    og = opdd.Grid(**grid)
    xy, t = opdd.node_points(og)
    # stand-in node values: u0 carried along by the heat kernel's widening (smooth, the workload's scale)
    vals = opdd.g_grid(wl["problem"], xy[:, 0], xy[:, 1]) * np.exp(-0.3 * t)
    _tail_parity(ctx, "tail_full_size_100_steps", wl["problem"], grid, vals, steps=100, groups=16)


def test_tail_full_step_count(ctx):
    """The workload's full step count (1000 steps to t = 1, boundary data at 8 node times on lines of 33
    nodes, outer edges from Monte Carlo nodes) on 2 x 2 subdomains of 128^2 cells over [-8, 8]^2: the
    field after every one of the 1000 steps' accumulation against the oracle's solve."""
    prob = _cubic(0)
    grid = _grid(x_lo=-8.0, x_hi=8.0, y_lo=-8.0, y_hi=8.0, px=2, py=2, cx=128, cy=128, T=1.0, n_steps=1000,
                 ns_x=33, ns_y=33, nt=8)
    og = opdd.Grid(**grid)
    xy, t = opdd.node_points(og)
    vals = opdd.g_grid(prob, xy[:, 0], xy[:, 1]) * np.exp(-0.3 * t)
    _tail_parity(ctx, "tail_full_step_count_2x2x128", prob, grid, vals)


def test_pdd_end_to_end_against_oracle_monte_carlo(ctx):
    """Monte Carlo at the nodes (FP64 paths) then the tail, against the oracle's own Monte Carlo values
    fed to the oracle's tail.  The node values agree to the Pade parity bound; the fields then agree to
    a small multiple of the largest node difference (interpolation and the solve do not amplify it)."""
    import torch

    import paper_2402_06491_amd as brt

    grid = _grid(cx=32, cy=32, n_steps=50)
    prob = _cubic(seed=2)
    mc = inputs.mc_params(seed=5, max_order=12, prune=1, node_cap=1 << 16, precision=64)
    n_trees = 2000
    _announce("pdd_end_to_end", grid)
    og = opdd.Grid(**grid)
    xy, t = opdd.node_points(og)
    n = len(t)
    wl = {"problems": [prob], "mc": mc, "x": xy, "t": t, "n_trees": np.full(n, n_trees, np.int64)}
    pi, ti, _ = P.tree_items(wl)
    orc = P.oracle_trees(wl, pi, ti)
    omom = P.oracle_moments(wl, orc, pi)
    opade = P.oracle_pade(wl, omom)
    onode = np.array([r["pade"] for r in opade])
    pd = brt.Pdd(ctx, prob, grid)
    try:
        node_u = torch.empty(n, dtype=torch.float64, device="cuda")
        field = pd.run(mc, n_trees, node_u=node_u).cpu().numpy()
        ms = pd.timing()
        gnode = node_u.cpu().numpy()
    finally:
        pd.close()
    dnode = float(np.abs(gnode - onode).max())
    assert dnode <= 1e-9 * max(1.0, float(np.abs(onode).max())), dnode
    ofield = opdd.pdd_solve(og, prob, onode)
    dfield = float(np.abs(field - ofield).max())
    print(f"[case] pdd_end_to_end: max |d node| {dnode:.3e}, max |dU| {dfield:.3e}; MC {ms[0]:.2f} ms, "
          f"interp {ms[1]:.3f} ms, solve {ms[2]:.3f} ms", flush=True)
    assert dfield <= 4.0 * dnode + FIELD_TOL * max(1.0, float(np.abs(ofield).max()))


def test_pdd_monte_carlo_leg_full_size(ctx):
    """The tail workload's Monte Carlo leg at its full size, as the bench runs it (2640 line nodes x 1e5
    trees, FP32 paths; paper Sec. 3, the values that the interpolation turns into boundary data):
    the node values brt_pdd_run produces equal, bit for bit, those of a plan over the same nodes; 4000
    of that plan's trees, sampled over all nodes, agree with the oracle tree by tree; and every tree of
    two sampled nodes goes through the oracle's moments and Pade value (1e-3 unless both sides flag)."""
    import torch

    import paper_2402_06491_amd as brt
    from paper_2402_06491_amd import Plan

    wl = inputs.pdd_cubic_2d()
    prob, grid, mc, nt = wl["problem"], wl["grid"], wl["mc"], wl["n_trees"]
    _announce("pdd_monte_carlo_leg_full_size", grid)
    pd = brt.Pdd(ctx, prob, grid)
    try:
        xy, t = pd.nodes()
        n = len(t)
        node_u = torch.empty(n, dtype=torch.float64, device="cuda")
        pd.run(mc, nt, node_u=node_u)
        torch.cuda.synchronize()
        u_pdd = node_u.cpu().numpy()
    finally:
        pd.close()
    pw = {"problems": [prob], "mc": mc, "x": np.asarray(xy), "t": np.asarray(t),
          "n_trees": np.full(n, nt, np.int64), "problem_id": np.zeros(n, np.uint32)}
    plan = Plan(ctx, [prob], mc, pw["x"], pw["t"], pw["n_trees"], problem_id=pw["problem_id"])
    out = plan.outputs(records=True)
    plan.execute(out)
    torch.cuda.synchronize()
    assert np.array_equal(out["u"].cpu().numpy(), u_pdd, equal_nan=True)
    assert np.all(out["hist"].sum(dim=1).cpu().numpy() == nt)

    rng = np.random.default_rng(2640)
    pi = rng.integers(0, n, size=4000)
    ti = rng.integers(0, nt, size=4000)
    rec = torch.as_tensor(pi * nt + ti, device="cuda")
    g = {"tree_f": out["tree_f"][rec].cpu().numpy(), "tree_meta": out["tree_meta"][rec].cpu().numpy()}
    orc = P.oracle_trees(pw, pi, ti)
    worst = P.compare_trees(g, np.arange(len(pi)), orc, P.FP32_TOL, pi)

    full = np.sort(rng.choice(n, size=2, replace=False))
    sub = dict(pw, x=pw["x"][full], t=pw["t"][full], n_trees=pw["n_trees"][full],
               problem_id=pw["problem_id"][full], point_id=full.astype(np.uint32))
    rows = torch.as_tensor(full, device="cuda")
    g2 = {k: out[k][rows].cpu().numpy() for k in ("u", "se", "psum", "coef", "coef_var", "hist", "s1", "s2",
                                                  "nodes", "flags", "pade_diag")}
    recs = torch.cat([torch.arange(int(p) * nt, (int(p) + 1) * nt, device="cuda") for p in full])
    g2["tree_f"] = out["tree_f"][recs].cpu().numpy()
    g2["tree_meta"] = out["tree_meta"][recs].cpu().numpy()
    plan.close()
    del out
    spi, sti, sri = P.tree_items(sub)
    sorc = P.oracle_trees(sub, spi, sti)
    P.compare_trees(g2, sri, sorc, P.FP32_TOL, spi)
    omom = P.oracle_moments(sub, sorc, spi)
    P.compare_moments(sub, g2, omom, P.FP32_TOL)
    P.check_exact_sums(sub, g2, sri, spi)
    opade = P.oracle_pade(sub, omom)
    du, strict, _, flagged, near = P.compare_pade(sub, g2, opade, 1e-3)
    print(f"[case] pdd_monte_carlo_leg_full_size: {n} nodes x {nt} trees; {len(pi)} sampled trees, max rel diff "
          f"{worst:.3e}; nodes {full.tolist()} in full: max |du| {du:.3e} over {strict} unflagged, {flagged} "
          f"flagged on both sides, {near} degree choices near the threshold", flush=True)


@pytest.mark.parametrize("pw", [0, 1])
def test_tail_variable_coefficients(ctx, pw):
    """Reaction with c_j(x, t) = c_j e^{-bx x^2 - by y^2} (t + t0)^-pow at the node and the mid-step time."""
    grid = _grid(px=2, py=3, cx=24, cy=20, n_steps=30, ns_x=9, ns_y=13, nt=4, T=0.4)
    prob = inputs.problem(2, 0.9, [0.05, 0.6, -1.0, -0.3], inputs.cubic_2d_u0(4),
                          coef_mod={"beta": (0.3, 0.5), "t0": 0.1, "pow": pw})
    og = opdd.Grid(**grid)
    rng = np.random.default_rng(21 + pw)
    xy, t = opdd.node_points(og)
    vals = opdd.g_grid(prob, xy[:, 0], xy[:, 1]) * np.exp(-0.5 * t) + 0.01 * rng.normal(size=len(t))
    _tail_parity(ctx, f"tail_varcoef_pow{pw}", prob, grid, vals)
