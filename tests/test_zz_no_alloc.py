"""brt_solve_noalloc (the allocation-free one-shot solve) against brt_solve, through the C ABI.

Both entry points run the same kernels, so their outputs must agree bit for bit.  Each case makes two
calls in a row, the second with a smaller input, so that whatever the first call left in the library's
scratch array cannot leak into the second.  Every case prints its name and shape before touching the GPU.
"""
import numpy as np
import pytest

from paper_2402_06491_amd import inputs

pytestmark = pytest.mark.gpu

_OUT_KEYS = ("u", "se", "psum", "coef", "coef_var", "hist", "s1", "s2", "nodes", "flags", "pade_diag")


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "no GPU"
    import paper_2402_06491_amd as brt

    c = brt.Context(0)
    yield c
    c.close()


def _bits(v):
    import torch

    v = v.detach().cpu()
    if v.dtype == torch.float64:
        v = v.view(torch.int64)
    return v.numpy()


def _run_both(ctx, name, wl, records):
    import torch

    import paper_2402_06491_amd as brt

    n = len(wl["t"])
    total = int(np.sum(wl["n_trees"]))
    print(f"\n[case] {name}: points={n} trees={total} precision={wl['mc']['precision']} "
          f"max_order={wl['mc']['max_order']} records={records}", flush=True)
    args = (ctx, wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"])
    kw = dict(problem_id=wl.get("problem_id"), records=records)
    ref = brt.solve(*args, **kw)
    got = brt.solve(*args, noalloc=True, **kw)
    torch.cuda.synchronize()
    keys = _OUT_KEYS + (("tree_f", "tree_meta") if records else ())
    for k in keys:
        a, b = _bits(ref[k]), _bits(got[k])
        assert a.shape == b.shape, k
        bad = np.flatnonzero(a.reshape(-1) != b.reshape(-1))
        assert bad.size == 0, f"{name}: {k} differs at {bad.size} entries (first flat index {bad[0]})"
    u = ref["u"].cpu().numpy()
    print(f"[case] {name}: bit-identical over {len(keys)} outputs; u in [{u.min():.4f}, {u.max():.4f}]", flush=True)
    return ref


def _ragged(wl, seed):
    """Trees per point made ragged (not multiples of 64) without exceeding the original counts."""
    rng = np.random.default_rng(seed)
    nt = np.asarray(wl["n_trees"], np.int64)
    wl["n_trees"] = np.maximum(1, nt - rng.integers(0, 64, size=nt.shape))
    return wl


def test_noalloc_fp32_multi_problem_two_calls(ctx):
    """8 polynomial PDEs, FP32 paths, tree records in the library's scratch: 400 points then 37."""
    big = _ragged(inputs.poly_batch(n_points=400, n_min=1_000, n_max=20_000, seed=11), 1)
    assert int(np.sum(big["n_trees"])) <= (1 << 22)
    _run_both(ctx, "noalloc_poly_fp32_400", big, records=False)
    small = _ragged(inputs.poly_batch(n_points=37, n_min=64, n_max=3_000, seed=12), 2)
    _run_both(ctx, "noalloc_poly_fp32_37", small, records=False)


def test_noalloc_fp64_2d_two_calls(ctx):
    """The 2-D cubic problem in FP64 with caller-owned tree records: 384 points then 24."""
    big = inputs.cubic_2d(n_trees=4_000, n_per_line=64)
    big["mc"] = dict(big["mc"], precision=64)
    big = _ragged(big, 3)
    _run_both(ctx, "noalloc_cubic2d_fp64_384", big, records=True)
    small = inputs.cubic_2d(n_trees=700, n_per_line=4)
    small["mc"] = dict(small["mc"], precision=64, seed=5)
    small = _ragged(small, 4)
    _run_both(ctx, "noalloc_cubic2d_fp64_24", small, records=True)


def test_noalloc_limits_rejected(ctx):
    """Sizes beyond the scratch array and settings the LDS-only stack cannot hold are refused on the
    host with a message, before any launch."""
    import paper_2402_06491_amd as brt

    wl = inputs.fisher(n_trees=64, n_x=8, times=(1.0,))
    args = (ctx, wl["problems"])
    print("\n[case] noalloc_limits: host-side rejections", flush=True)
    cases = [
        ("points", wl["mc"], np.zeros((4097, 1)), np.ones(4097), np.full(4097, 64), "POINTS"),
        ("trees", wl["mc"], wl["x"], wl["t"], np.full(8, (1 << 22) // 8 + 1), "TREES"),
        ("order", dict(wl["mc"], max_order=17, pade_L=6, pade_M=6), wl["x"], wl["t"], wl["n_trees"], "ORDER"),
        ("prune", dict(wl["mc"], prune=0), wl["x"], wl["t"], wl["n_trees"], "ORDER"),
    ]
    for name, mc, x, t, nt, word in cases:
        with pytest.raises(brt.BrtError) as e:
            brt.solve(*args, mc, x, t, nt, records=False, noalloc=True)
        assert e.value.code == -1 and word in str(e.value), (name, str(e.value))
    # the library still works after the rejections
    _run_both(ctx, "noalloc_after_rejections", wl, records=False)
