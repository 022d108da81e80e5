"""Random-tree Monte Carlo solver for semilinear parabolic PDEs on MI355X (gfx950).

Thin ctypes binding over ``libbrt.so`` (the C ABI of ``include/brt.h``): argument marshalling only.
Every step of the method (tree walk, moment reduction, coefficients, Pade) runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  If the library is missing, every entry point
raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbrt.so")

BRT_OK = 0
ERRORS = {-1: "BRT_E_ARG", -2: "BRT_E_DEVICE", -3: "BRT_E_NOMEM", -4: "BRT_E_BUSY", -5: "BRT_E_RANGE",
          -6: "BRT_E_STATE"}
U0_KINDS = {"const": 0, "logistic": 1, "gauss_sum": 2, "cos2_bump": 3}
FLAG_POLE, FLAG_LOWERED, FLAG_OVERFLOW, FLAG_CAPPED, FLAG_DEPTH, FLAG_SENSITIVE = 1, 2, 4, 8, 16, 32
PADE_DIAG = 6  # columns of the pade_diag output: L used, M used, [L-1/M], [L/M-1], kappa, selection margin
META_OVERFLOW, META_CAPPED, META_DEPTH, META_NODES_SHIFT = 1 << 8, 1 << 9, 1 << 10, 11


class BrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("dim", ctypes.c_uint32), ("diffusion", ctypes.c_double),
                ("coef", ctypes.c_double * 8), ("u0_kind", ctypes.c_uint32), ("u0_nterms", ctypes.c_uint32),
                ("u0_params", ctypes.c_double * 40), ("coef_mod", ctypes.c_uint32), ("coef_mod_pow", ctypes.c_uint32),
                ("coef_mod_beta", ctypes.c_double * 2), ("coef_mod_t0", ctypes.c_double),
                ("drift", ctypes.c_double * 2), ("sde", ctypes.c_uint32), ("sde_pad", ctypes.c_uint32),
                ("drift_lin", ctypes.c_double * 2), ("sigma_amp", ctypes.c_double), ("sigma_width", ctypes.c_double),
                ("sde_dt", ctypes.c_double)]


class MC(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("lambda_", ctypes.c_double), ("max_order", ctypes.c_uint32), ("prune", ctypes.c_uint32),
                ("node_cap", ctypes.c_uint32), ("pade_L", ctypes.c_uint32), ("pade_M", ctypes.c_uint32),
                ("strategy", ctypes.c_uint32), ("q", ctypes.c_double)]


class Points(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n", ctypes.c_uint32), ("x", ctypes.c_void_p),
                ("t", ctypes.c_void_p), ("n_trees", ctypes.c_void_p), ("problem_id", ctypes.c_void_p),
                ("point_id", ctypes.c_void_p), ("tree_first", ctypes.c_void_p)]


class Out(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32)] + [
        (name, ctypes.c_void_p) for name in
        ("u", "se", "psum", "coef", "coef_var", "hist", "s1", "s2", "nodes", "flags", "tree_f", "tree_meta",
         "pade_diag")]


class Launch(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("waves_per_block", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32), ("chunk_trees", ctypes.c_uint32),
                ("stack_depth", ctypes.c_uint32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("dim", ctypes.c_uint32), ("u0_kind", ctypes.c_uint32),
                ("mc", MC), ("max_points", ctypes.c_uint32), ("round_trees", ctypes.c_uint32),
                ("max_trees", ctypes.c_uint32), ("target_se", ctypes.c_double), ("queue_cap", ctypes.c_uint32),
                ("max_active_requests", ctypes.c_uint32)]


class Request(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n", ctypes.c_uint32), ("problem", ctypes.POINTER(Problem)),
                ("x", ctypes.c_void_p), ("t", ctypes.c_void_p), ("stream_id", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("u", ctypes.c_void_p), ("se", ctypes.c_void_p),
                ("coef", ctypes.c_void_p), ("trees", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("latency_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32)] + [
        (n, ctypes.c_uint64) for n in ("submitted", "completed", "rejected", "ticks", "trees", "nodes")] + [
        (n, ctypes.c_double) for n in ("p50_latency_s", "p99_latency_s", "mean_latency_s", "busy_s", "span_s",
                                       "trees_per_s")]


class PddGrid(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double),
                ("y_lo", ctypes.c_double), ("y_hi", ctypes.c_double), ("px", ctypes.c_uint32),
                ("py", ctypes.c_uint32), ("cx", ctypes.c_uint32), ("cy", ctypes.c_uint32), ("T", ctypes.c_double),
                ("n_steps", ctypes.c_uint32), ("ns_x", ctypes.c_uint32), ("ns_y", ctypes.c_uint32),
                ("nt", ctypes.c_uint32), ("outer", ctypes.c_uint32)]


_lib = None

# (name, restype, argtypes) for every entry point of include/brt.h
_SIGS = [
    ("brt_version", ctypes.c_int, []),
    ("brt_last_error", ctypes.c_char_p, []),
    ("brt_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    ("brt_destroy", None, [ctypes.c_void_p]),
    ("brt_problem_check", ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(MC)]),
    ("brt_set_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Launch)]),
    ("brt_get_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Launch)]),
    ("brt_plan_create", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(Problem), ctypes.POINTER(MC),
                                       ctypes.POINTER(Points), ctypes.POINTER(ctypes.c_void_p)]),
    ("brt_plan_execute", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Out), ctypes.c_void_p]),
    ("brt_plan_info", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                     ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32),
                                     ctypes.POINTER(ctypes.c_uint32)]),
    ("brt_plan_depth_exceeded", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    ("brt_plan_set_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("brt_plan_get_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_uint64)]),
    ("brt_plan_set_graph", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("brt_plan_graph_stats", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                            ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    ("brt_plan_destroy", None, [ctypes.c_void_p]),
    ("brt_solve", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(Problem), ctypes.POINTER(MC),
                                 ctypes.POINTER(Points), ctypes.POINTER(Out), ctypes.c_void_p]),
    ("brt_solve_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(Problem),
                                         ctypes.POINTER(MC), ctypes.POINTER(Points), ctypes.POINTER(Out),
                                         ctypes.c_void_p]),
    ("brt_autotune", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(Problem), ctypes.POINTER(MC),
                                    ctypes.POINTER(Points), ctypes.c_char_p, ctypes.POINTER(Launch)]),
    ("brt_server_create", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerOpts), ctypes.POINTER(ctypes.c_void_p)]),
    ("brt_server_submit", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    ("brt_server_poll", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Result),
                                       ctypes.POINTER(ctypes.c_int)]),
    ("brt_server_drain", ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    ("brt_server_stats_get", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    ("brt_server_destroy", None, [ctypes.c_void_p]),
    ("brt_pdd_create", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(PddGrid),
                                      ctypes.POINTER(ctypes.c_void_p)]),
    ("brt_pdd_nodes", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_uint64)]),
    ("brt_pdd_lines", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    ("brt_pdd_interpolate", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("brt_pdd_boundary", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]),
    ("brt_pdd_solve", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]),
    ("brt_pdd_run", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MC), ctypes.c_uint64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    ("brt_pdd_get_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    ("brt_pdd_get_barrier", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                            ctypes.POINTER(ctypes.c_uint32)]),
    ("brt_pdd_destroy", None, [ctypes.c_void_p]),
]


def lib():
    """Load libbrt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2402_06491_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != BRT_OK:
        raise BrtError(rc, lib().brt_last_error().decode())
    return rc


def make_problem(d: dict) -> Problem:
    p = Problem()
    p.struct_size = ctypes.sizeof(Problem)
    p.dim = int(d["dim"])
    p.diffusion = float(d["diffusion"])
    coef = list(d["coef"]) + [0.0] * (8 - len(d["coef"]))
    for j in range(8):
        p.coef[j] = float(coef[j])
    kind = d["u0_kind"]
    p.u0_kind = U0_KINDS[kind] if isinstance(kind, str) else int(kind)
    p.u0_nterms = int(d.get("u0_nterms", 0))
    for i, v in enumerate(d.get("u0_params", [])):
        p.u0_params[i] = float(v)
    cm = d.get("coef_mod")
    if cm:
        p.coef_mod = 2 if cm.get("linear", False) else 1
        beta = list(cm.get("beta", (0.0, 0.0))) + [0.0]
        p.coef_mod_beta[0] = float(beta[0])
        p.coef_mod_beta[1] = float(beta[1])
        p.coef_mod_pow = int(cm.get("pow", 0))
        p.coef_mod_t0 = float(cm.get("t0", 0.0))
    b = list(d.get("drift", (0.0, 0.0))) + [0.0, 0.0]
    p.drift[0] = float(b[0])
    p.drift[1] = float(b[1])
    e = d.get("euler")
    if e:
        p.sde = 1
        bl = list(e.get("drift_lin", (0.0, 0.0))) + [0.0, 0.0]
        p.drift_lin[0] = float(bl[0])
        p.drift_lin[1] = float(bl[1])
        p.sigma_amp = float(e.get("sigma_amp", 0.0))
        p.sigma_width = float(e.get("sigma_width", 1.0))
        p.sde_dt = float(e["dt"])
    return p


def make_mc(d: dict) -> MC:
    m = MC()
    m.struct_size = ctypes.sizeof(MC)
    m.precision = int(d.get("precision", 32))
    m.seed = int(d.get("seed", 0))
    m.lambda_ = float(d.get("lambda", 1.0))
    m.max_order = int(d.get("max_order", 12))
    m.prune = int(d.get("prune", 1))
    m.node_cap = int(d.get("node_cap", 1 << 16))
    m.pade_L = int(d.get("pade_L", 6))
    m.pade_M = int(d.get("pade_M", 6))
    s = d.get("strategy", 0)
    m.strategy = {"A": 0, "B": 1}[s] if isinstance(s, str) else int(s)
    m.q = float(d.get("q", 0.5))
    return m


class Context:
    """A brt_ctx on one HIP device."""

    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().brt_create(ctypes.byref(self._h), int(device)))
        self.device = device

    def set_launch(self, waves_per_block=4, blocks_per_cu=0, chunk_trees=1024, stack_depth=0):
        l = Launch(ctypes.sizeof(Launch), waves_per_block, blocks_per_cu, chunk_trees, stack_depth)
        _check(lib().brt_set_launch(self._h, ctypes.byref(l)))

    def autotune(self, problems, mc: dict, x, t, n_trees, problem_id=None, cache_path=None) -> dict:
        """brt_autotune on these points; returns the chosen launch settings (now set on the context)."""
        if isinstance(problems, dict):
            problems = [problems]
        arr = (Problem * len(problems))(*[make_problem(p) for p in problems])
        m = make_mc(mc)
        keep = []
        pts, _, _ = _points(x, t, n_trees, problem_id, None, int(problems[0]["dim"]), keep)
        best = Launch()
        best.struct_size = ctypes.sizeof(Launch)
        path = cache_path.encode() if cache_path else None
        _check(lib().brt_autotune(self._h, len(problems), arr, ctypes.byref(m), ctypes.byref(pts), path,
                                  ctypes.byref(best)))
        return {"waves_per_block": best.waves_per_block, "blocks_per_cu": best.blocks_per_cu,
                "chunk_trees": best.chunk_trees, "stack_depth": best.stack_depth}

    def get_launch(self) -> dict:
        l = Launch()
        _check(lib().brt_get_launch(self._h, ctypes.byref(l)))
        return {"waves_per_block": l.waves_per_block, "blocks_per_cu": l.blocks_per_cu,
                "chunk_trees": l.chunk_trees, "stack_depth": l.stack_depth}

    def close(self):
        if self._h:
            lib().brt_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _points(x, t, n_trees, problem_id, point_id, dim, keep, tree_first=None):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, dim))
    n = x.shape[0]
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), (n,)))
    nt = np.ascontiguousarray(np.broadcast_to(np.asarray(n_trees, dtype=np.uint64), (n,)))
    pts = Points()
    pts.struct_size = ctypes.sizeof(Points)
    pts.n = n
    pts.x, pts.t, pts.n_trees = x.ctypes.data, t.ctypes.data, nt.ctypes.data
    keep += [x, t, nt]
    if problem_id is not None:
        pid = np.ascontiguousarray(np.asarray(problem_id, dtype=np.uint32).reshape(n))
        pts.problem_id = pid.ctypes.data
        keep.append(pid)
    if point_id is not None:
        qid = np.ascontiguousarray(np.asarray(point_id, dtype=np.uint32).reshape(n))
        pts.point_id = qid.ctypes.data
        keep.append(qid)
    if tree_first is not None:
        tf = np.ascontiguousarray(np.broadcast_to(np.asarray(tree_first, dtype=np.uint32), (n,)))
        pts.tree_first = tf.ctypes.data
        keep.append(tf)
    return pts, n, int(nt.sum())


def alloc_outputs(n_points, n_bins, total_trees, precision, records=True, device="cuda"):
    """Device tensors for every output of brt_out (torch supplies the memory)."""
    import torch

    o = {
        "u": torch.empty(n_points, dtype=torch.float64, device=device),
        "se": torch.empty(n_points, dtype=torch.float64, device=device),
        "psum": torch.empty(n_points, dtype=torch.float64, device=device),
        "coef": torch.empty((n_points, n_bins), dtype=torch.float64, device=device),
        "coef_var": torch.empty((n_points, n_bins), dtype=torch.float64, device=device),
        "hist": torch.empty((n_points, n_bins + 3), dtype=torch.int64, device=device),
        "s1": torch.empty((n_points, n_bins), dtype=torch.float64, device=device),
        "s2": torch.empty((n_points, n_bins), dtype=torch.float64, device=device),
        "nodes": torch.empty(n_points, dtype=torch.int64, device=device),
        "flags": torch.empty(n_points, dtype=torch.int32, device=device),
        "pade_diag": torch.empty((n_points, PADE_DIAG), dtype=torch.float64, device=device),
    }
    if records:
        o["tree_f"] = torch.empty(max(total_trees, 1), dtype=torch.float64, device=device)
        o["tree_meta"] = torch.empty(max(total_trees, 1), dtype=torch.int32, device=device)
    return o


def make_out(tensors: dict) -> Out:
    o = Out()
    o.struct_size = ctypes.sizeof(Out)
    for name, _ in Out._fields_[1:]:
        v = tensors.get(name)
        setattr(o, name, v.data_ptr() if v is not None else None)
    return o


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """brt_plan: normalised problems, uploaded points and work chunks, replayable on a stream."""

    def __init__(self, ctx: Context, problems, mc: dict, x, t, n_trees, problem_id=None, point_id=None,
                 tree_first=None):
        if isinstance(problems, dict):
            problems = [problems]
        self.ctx = ctx
        self.mc = dict(mc)
        self.dim = int(problems[0]["dim"])
        arr = (Problem * len(problems))(*[make_problem(p) for p in problems])
        m = make_mc(mc)
        keep = []
        pts, self.n_points, self.total_trees = _points(x, t, n_trees, problem_id, point_id, self.dim, keep,
                                                       tree_first)
        self._h = ctypes.c_void_p()
        _check(lib().brt_plan_create(ctx._h, len(problems), arr, ctypes.byref(m), ctypes.byref(pts),
                                     ctypes.byref(self._h)))
        npnt, ntr, nb, nch = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().brt_plan_info(self._h, ctypes.byref(npnt), ctypes.byref(ntr), ctypes.byref(nb), ctypes.byref(nch)))
        self.n_bins, self.n_chunks = nb.value, nch.value
        self.precision = int(mc.get("precision", 32))
        self._out_cache = None

    def outputs(self, records=True):
        return alloc_outputs(self.n_points, self.n_bins, self.total_trees, self.precision, records)

    def execute(self, tensors: dict, stream=None):
        """Enqueue the whole path on `stream` (torch's current stream by default)."""
        o = make_out(tensors)
        _check(lib().brt_plan_execute(self._h, ctypes.byref(o), _stream_handle(stream)))

    def set_graph(self, enable: bool):
        _check(lib().brt_plan_set_graph(self._h, int(bool(enable))))

    def graph_stats(self) -> dict:
        """Graphs instantiated, graph launches and kernel-by-kernel runs of this plan so far."""
        c, r, d = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().brt_plan_graph_stats(self._h, ctypes.byref(c), ctypes.byref(r), ctypes.byref(d)))
        return {"captures": c.value, "replays": r.value, "direct": d.value}

    def depth_exceeded(self) -> int:
        v = ctypes.c_uint64()
        _check(lib().brt_plan_depth_exceeded(self._h, ctypes.byref(v)))
        return v.value

    def set_timing(self, enable: bool):
        _check(lib().brt_plan_set_timing(self._h, int(bool(enable))))

    def get_timing(self):
        """Summed (walk, reduce, finalize) kernel milliseconds and run count since the last call."""
        ms = (ctypes.c_double * 3)()
        runs = ctypes.c_uint64()
        _check(lib().brt_plan_get_timing(self._h, ms, ctypes.byref(runs)))
        return (ms[0], ms[1], ms[2]), runs.value

    def close(self):
        if self._h:
            lib().brt_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(ctx: Context, problems, mc: dict, x, t, n_trees, problem_id=None, point_id=None, records=True,
          stream=None, noalloc=False):
    """One-shot brt_solve (brt_solve_noalloc with noalloc=True); returns the output tensors (on the GPU)."""
    if isinstance(problems, dict):
        problems = [problems]
    arr = (Problem * len(problems))(*[make_problem(p) for p in problems])
    m = make_mc(mc)
    keep = []
    pts, n, total = _points(x, t, n_trees, problem_id, point_id, int(problems[0]["dim"]), keep)
    nb = int(mc.get("max_order", 12)) + 2
    tensors = alloc_outputs(n, nb, total, int(mc.get("precision", 32)), records)
    o = make_out(tensors)
    fn = lib().brt_solve_noalloc if noalloc else lib().brt_solve
    _check(fn(ctx._h, len(problems), arr, ctypes.byref(m), ctypes.byref(pts), ctypes.byref(o), _stream_handle(stream)))
    return tensors


class Server:
    """brt_server: continuous batching of point-query requests (see include/brt.h)."""

    def __init__(self, ctx: Context, dim: int, u0_kind, mc: dict, max_points=4096, round_trees=16384,
                 max_trees=1 << 20, target_se=1e-3, queue_cap=100_000, max_active_requests=0):
        o = ServerOpts()
        o.struct_size = ctypes.sizeof(ServerOpts)
        o.dim = int(dim)
        o.u0_kind = U0_KINDS[u0_kind] if isinstance(u0_kind, str) else int(u0_kind)
        o.mc = make_mc(mc)
        o.max_points, o.round_trees, o.max_trees = int(max_points), int(round_trees), int(max_trees)
        o.target_se, o.queue_cap, o.max_active_requests = float(target_se), int(queue_cap), int(max_active_requests)
        self.B = int(mc.get("max_order", 12)) + 2
        self.dim = int(dim)
        self._h = ctypes.c_void_p()
        _check(lib().brt_server_create(ctx._h, ctypes.byref(o), ctypes.byref(self._h)))

    def submit(self, problem: dict, x, t, stream_id: int) -> int:
        """Queue one request; returns its ticket (raises BrtError with code -4 when the queue is full)."""
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, self.dim))
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), (x.shape[0],)))
        p = make_problem(problem)
        q = Request(ctypes.sizeof(Request), x.shape[0], ctypes.pointer(p), x.ctypes.data, t.ctypes.data,
                    int(stream_id))
        ticket = ctypes.c_uint64()
        _check(lib().brt_server_submit(self._h, ctypes.byref(q), ctypes.byref(ticket)))
        return ticket.value

    def poll(self, ticket: int, n: int):
        """None while running; when complete, a dict of host arrays (and the ticket is released)."""
        u, se = np.zeros(n), np.zeros(n)
        coef = np.zeros((n, self.B))
        trees = np.zeros(n, np.uint64)
        flags = np.zeros(n, np.uint32)
        r = Result(ctypes.sizeof(Result), u.ctypes.data, se.ctypes.data, coef.ctypes.data, trees.ctypes.data,
                   flags.ctypes.data, 0.0)
        done = ctypes.c_int()
        _check(lib().brt_server_poll(self._h, int(ticket), ctypes.byref(r), ctypes.byref(done)))
        if not done.value:
            return None
        return {"u": u, "se": se, "coef": coef, "trees": trees, "flags": flags, "latency_s": r.latency_s}

    def drain(self, timeout_s=600.0):
        _check(lib().brt_server_drain(self._h, float(timeout_s)))

    def stats(self) -> dict:
        s = ServerStats()
        s.struct_size = ctypes.sizeof(ServerStats)
        _check(lib().brt_server_stats_get(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in ServerStats._fields_[1:]}

    def close(self):
        if self._h:
            lib().brt_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PDD_OUTER = {"mc": 0, "lines": 0, "zero": 1}


def make_pdd_grid(d: dict) -> PddGrid:
    g = PddGrid()
    g.struct_size = ctypes.sizeof(PddGrid)
    for k in ("x_lo", "x_hi", "y_lo", "y_hi", "T"):
        setattr(g, k, float(d[k]))
    for k in ("px", "py", "cx", "cy", "n_steps", "ns_x", "ns_y", "nt"):
        setattr(g, k, int(d[k]))
    o = d.get("outer", "mc")
    g.outer = PDD_OUTER[o] if isinstance(o, str) else int(o)
    return g


class Pdd:
    """The domain-decomposition tail (brt_pdd_*) for one 2-D problem on one grid."""

    def __init__(self, ctx: Context, problem: dict, grid: dict):
        import torch

        self._torch = torch
        self.ctx = ctx
        self.grid = dict(grid)
        self._prob = make_problem(problem)
        self._grid = make_pdd_grid(grid)
        self._h = ctypes.c_void_p()
        _check(lib().brt_pdd_create(ctx._h, ctypes.byref(self._prob), ctypes.byref(self._grid),
                                    ctypes.byref(self._h)))
        self.NX = self._grid.px * self._grid.cx
        self.NY = self._grid.py * self._grid.cy

    def nodes(self):
        """(xy[n, 2], t[n]) host arrays of the Monte Carlo query points."""
        n = ctypes.c_uint64()
        _check(lib().brt_pdd_nodes(self._h, None, None, ctypes.byref(n)))
        xy = np.empty((n.value, 2), np.float64)
        t = np.empty(n.value, np.float64)
        _check(lib().brt_pdd_nodes(self._h, xy.ctypes.data, t.ctypes.data, ctypes.byref(n)))
        return xy, t

    def lines(self):
        n = ctypes.c_uint32()
        _check(lib().brt_pdd_lines(self._h, ctypes.byref(n), None, None, None))
        o = np.empty(n.value, np.uint32)
        c = np.empty(n.value, np.float64)
        f = np.empty(n.value, np.uint32)
        _check(lib().brt_pdd_lines(self._h, ctypes.byref(n), o.ctypes.data, c.ctypes.data, f.ctypes.data))
        return o, c, f

    def _stream(self):
        return ctypes.c_void_p(self._torch.cuda.current_stream().cuda_stream)

    def interpolate(self, node_values):
        """node_values: a float64 CUDA tensor in node order."""
        v = node_values.contiguous()
        _check(lib().brt_pdd_interpolate(self._h, ctypes.c_void_p(v.data_ptr()), self._stream()))
        self._keep = v

    def boundary(self, line):
        _, _, f = self.lines()
        out = self._torch.empty((self._grid.n_steps + 1, int(f[line])), dtype=self._torch.float64, device="cuda")
        _check(lib().brt_pdd_boundary(self._h, int(line), ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def solve(self, steps=None, field=None):
        steps = self._grid.n_steps if steps is None else int(steps)
        if field is None:
            field = self._torch.empty((self.NY + 1, self.NX + 1), dtype=self._torch.float64, device="cuda")
        _check(lib().brt_pdd_solve(self._h, steps, ctypes.c_void_p(field.data_ptr()), self._stream()))
        return field

    def run(self, mc: dict, trees_per_node: int, node_u=None, field=None):
        m = make_mc(mc)
        if field is None:
            field = self._torch.empty((self.NY + 1, self.NX + 1), dtype=self._torch.float64, device="cuda")
        nu = ctypes.c_void_p(node_u.data_ptr()) if node_u is not None else None
        _check(lib().brt_pdd_run(self._h, ctypes.byref(m), int(trees_per_node), nu,
                                 ctypes.c_void_p(field.data_ptr()), self._stream()))
        return field

    def timing(self):
        """(Monte Carlo, interpolation, solve) in ms of the last run; waits for it."""
        ms = (ctypes.c_double * 3)()
        _check(lib().brt_pdd_get_timing(self._h, ms))
        return tuple(ms)

    def barrier(self):
        """(barrier groups, groups whose blocks all ran on one die) of the last solve; waits for it."""
        g, d = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().brt_pdd_get_barrier(self._h, ctypes.byref(g), ctypes.byref(d)))
        return int(g.value), int(d.value)

    def close(self):
        if self._h:
            lib().brt_pdd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
