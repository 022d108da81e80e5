"""The C-ABI library loads and exports every entry point declared in include/brt.h (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2402_06491_amd", "libbrt.so")


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(brt_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_symbols()
    assert "brt_solve" in names and "brt_plan_execute" in names and len(names) >= 12


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbrt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbrt.so not built")
def test_binding_signatures_cover_header():
    import paper_2402_06491_amd as brt

    bound = {name for name, _, _ in brt._SIGS}
    assert set(declared_symbols()) <= bound


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbrt.so not built")
def test_problem_check_host_only():
    """Argument validation is host code: it runs (and rejects bad input) without a GPU."""
    import paper_2402_06491_amd as brt
    from paper_2402_06491_amd import inputs

    L = brt.lib()
    wl = inputs.fisher(n_trees=1)
    p = brt.make_problem(wl["problems"][0])
    m = brt.make_mc(wl["mc"])
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(m)) == 0
    bad = brt.make_mc(dict(wl["mc"], max_order=127))
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(bad)) == -1
    assert b"max_order" in L.brt_last_error()
    bad = brt.make_mc(dict(wl["mc"], pade_L=7, pade_M=6))
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(bad)) == -1
    q = brt.make_problem(dict(wl["problems"][0], diffusion=0.0))
    assert L.brt_problem_check(ctypes.byref(q), ctypes.byref(m)) == -1
    q = brt.make_problem(dict(wl["problems"][0], u0_params=[1, 1, 0, 2.5, 1, 0]))
    assert L.brt_problem_check(ctypes.byref(q), ctypes.byref(m)) == -1
    q = brt.make_problem(dict(wl["problems"][0], u0_kind=9))
    assert L.brt_problem_check(ctypes.byref(q), ctypes.byref(m)) == -1
    p.struct_size = 8
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(m)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbrt.so not built")
def test_strategy_b_validation_host_only():
    import paper_2402_06491_amd as brt
    from paper_2402_06491_amd import inputs

    L = brt.lib()
    wl = inputs.kpp(n_trees=1)
    p = brt.make_problem(wl["problems"][0])
    ok = brt.make_mc(dict(wl["mc"], strategy=1, q=0.6))
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(ok)) == 0
    # binary trees without pruning are critical or supercritical for q <= 1/2
    bad = brt.make_mc(dict(wl["mc"], strategy=1, q=0.5))
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(bad)) == -1
    assert b"subcritical" in L.brt_last_error()
    bad = brt.make_mc(dict(wl["mc"], strategy=2))
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(bad)) == -1
    bad = brt.make_mc(dict(wl["mc"], strategy=1, q=1.0))
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(bad)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbrt.so not built")
def test_coef_mod_validation_host_only():
    import paper_2402_06491_amd as brt
    from paper_2402_06491_amd import inputs

    L = brt.lib()
    mc = brt.make_mc(inputs.mc_params())
    good = brt.make_problem(inputs.example5()["problems"][0])
    assert L.brt_problem_check(ctypes.byref(good), ctypes.byref(mc)) == 0
    for bad_mod in ({"beta": (-1.0, 0.0), "t0": 0.1, "pow": 1}, {"beta": (1.0, 0.0), "t0": 0.0, "pow": 1},
                    {"beta": (1.0, 0.0), "t0": 0.1, "pow": 2}):
        d = inputs.problem(1, 1.0, [0.0, 0.0, -1.0], inputs.const(1.0), coef_mod=bad_mod)
        p = brt.make_problem(d)
        assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(mc)) == -1, bad_mod
    p = brt.make_problem(inputs.problem(1, 1.0, [0.0, 0.0, -1.0], inputs.const(1.0)))
    p.coef_mod = 7
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(mc)) == -1
    lin = brt.make_problem(inputs.problem(1, 1.0, [0.0, 0.5, -1.0], inputs.const(1.0),
                                          coef_mod={"beta": (1.0, 0.0), "t0": 0.1, "pow": 1, "linear": True}))
    assert lin.coef_mod == 2
    assert L.brt_problem_check(ctypes.byref(lin), ctypes.byref(mc)) == 0
    lin.coef_mod = 3
    assert L.brt_problem_check(ctypes.byref(lin), ctypes.byref(mc)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbrt.so not built")
def test_drift_validation_host_only():
    import paper_2402_06491_amd as brt
    from paper_2402_06491_amd import inputs

    L = brt.lib()
    mc = brt.make_mc(inputs.mc_params())
    ok1 = brt.make_problem(inputs.problem(1, 1.0, [0.0, 1.0, -1.0], inputs.const(1.0), drift=(0.5,)))
    ok2 = brt.make_problem(inputs.problem(2, 1.0, [0.0, 1.0, -1.0], inputs.const(1.0), drift=(0.5, -2.0)))
    assert L.brt_problem_check(ctypes.byref(ok1), ctypes.byref(mc)) == 0
    assert L.brt_problem_check(ctypes.byref(ok2), ctypes.byref(mc)) == 0
    bad_1d = brt.make_problem(inputs.problem(1, 1.0, [0.0, 1.0, -1.0], inputs.const(1.0), drift=(0.5, 1.0)))
    assert L.brt_problem_check(ctypes.byref(bad_1d), ctypes.byref(mc)) == -1
    bad_inf = brt.make_problem(inputs.problem(2, 1.0, [0.0, 1.0, -1.0], inputs.const(1.0), drift=(float("inf"), 0.0)))
    assert L.brt_problem_check(ctypes.byref(bad_inf), ctypes.byref(mc)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbrt.so not built")
def test_euler_validation_host_only():
    import paper_2402_06491_amd as brt
    from paper_2402_06491_amd import inputs

    L = brt.lib()
    mc = brt.make_mc(inputs.mc_params(precision=64))
    mc32 = brt.make_mc(inputs.mc_params(precision=32))

    def check(m=mc, **kw):
        d = inputs.problem(2, 1.0, [0.0, 1.0, -1.0], inputs.const(1.0), **kw)
        return L.brt_problem_check(ctypes.byref(brt.make_problem(d)), ctypes.byref(m))

    assert check(euler={"dt": 0.01, "drift_lin": (0.5, -1.0), "sigma_amp": 0.3, "sigma_width": 1.0}) == 0
    # FP32 paths do not step (the step count ceil(s/h) of an FP32 edge can differ from the FP64 one)
    assert check(mc32, euler={"dt": 0.01, "drift_lin": (0.5, -1.0), "sigma_amp": 0.3, "sigma_width": 1.0}) == -1
    assert "precision 64" in L.brt_last_error().decode()
    assert check(euler={"dt": 0.0}) == -1
    assert check(euler={"dt": 0.01, "sigma_amp": -1.0, "sigma_width": 1.0}) == -1
    assert check(euler={"dt": 0.01, "sigma_amp": 0.5, "sigma_width": 0.0}) == -1
    p = brt.make_problem(inputs.problem(2, 1.0, [0.0, 1.0, -1.0], inputs.const(1.0)))
    p.sigma_amp = 0.5  # needs the Euler scheme
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(mc)) == -1
    p.sigma_amp = 0.0
    p.sde = 5
    assert L.brt_problem_check(ctypes.byref(p), ctypes.byref(mc)) == -1
    one_d = brt.make_problem(inputs.problem(1, 1.0, [0.0, 1.0, -1.0], inputs.const(1.0),
                                            euler={"dt": 0.01, "drift_lin": (0.5, 1.0)}))
    assert L.brt_problem_check(ctypes.byref(one_d), ctypes.byref(mc)) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbrt.so not built")
def test_pdd_queries_reject_null_arguments_host_only():
    """The tail's query entry points check their arguments on the host before any device call."""
    import paper_2402_06491_amd as brt

    L = brt.lib()
    g, d = ctypes.c_uint32(7), ctypes.c_uint32(7)
    assert L.brt_pdd_get_barrier(None, ctypes.byref(g), ctypes.byref(d)) == -1
    assert b"brt_pdd_get_barrier" in L.brt_last_error()
    ms = (ctypes.c_double * 3)()
    assert L.brt_pdd_get_timing(None, ms) == -1
