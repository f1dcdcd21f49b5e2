"""MI355X (gfx950) HIP implementation of the P-GVIMP hot path.

Thin Python binding over the C ABI of include/pgvimp.h.  Every function
only marshals arguments and calls the library of the same name; all steps
of the method run in the HIP kernels of libpgvimp.so.  PyTorch provides the
device arena and the stream the library works on.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import _abi
from ._abi import (ARM_DOF, COLL_ARM3D, COLL_NONE, COLL_POINT2D, COLL_POINT3D, EBUSY, EDEVICE, EINVAL,  # noqa: F401
                   ENOCONV, ENOMEM, ENOTPD, FP64, MIXED, MODEL_QUAD2D, OK)

__all__ = [
    "PgvimpError", "Context", "pgvimp_create", "pgvimp_destroy", "pgvimp_add_plan", "pgvimp_remove_plan",
    "pgvimp_marginals", "pgvimp_factor_expectations", "pgvimp_prox_step", "pgvimp_solve", "pgvimp_slr_linearize",
    "pgvimp_get_state", "pgvimp_set_state", "pgvimp_set_budget", "pgvimp_kernel_times", "pgvimp_profile",
    "pgvimp_launch_shape", "pgvimp_arena_bytes", "problem_struct", "library_path", "ipgvimp_begin",
    "ipgvimp_next_round", "pgvimp_expect_all", "pgvimp_slr_round",
]

_KIND = {"none": COLL_NONE, "point2d": COLL_POINT2D, "point3d": COLL_POINT3D, "arm3d": COLL_ARM3D}


class PgvimpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pgvimp error {code}: {msg}")
        self.code = code


def library_path():
    return _abi.LIB_PATH


def _check(rc, ctx_handle=None):
    if rc != OK:
        lib = _abi.load()
        msg = lib.pgvimp_last_error(ctx_handle)
        raise PgvimpError(rc, msg.decode() if msg else "")


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def problem_struct(prob, mu_init=None):
    """Marshal a problem dictionary (see workloads.py) into the C struct.
    Returns (struct, keepalive) - keep the second alive during the call."""
    keep = []

    def arr(x, dt=np.float64):
        a = np.ascontiguousarray(np.asarray(x, dtype=dt))
        keep.append(a)
        return a

    s = _abi.Problem()
    n, N = int(prob["n"]), int(prob["N"])
    s.n, s.m, s.N = n, int(prob["m"]), N
    s.dt = float(prob["dt"])
    s.ltv = 1 if prob.get("ltv", False) else 0
    s.A = _dptr(arr(prob["A"]))
    s.a = _dptr(arr(prob["a"]))
    s.B = _dptr(arr(prob["B"]))
    s.Qc = _dptr(arr(prob["Qc"]))
    s.mu_start = _dptr(arr(prob["mu_start"]))
    s.Sig_start = _dptr(arr(prob["Sig_start"]))
    s.mu_goal = _dptr(arr(prob["mu_goal"]))
    s.Sig_goal = _dptr(arr(prob["Sig_goal"]))
    s.temperature = float(prob["temperature"])
    s.beta_max = float(prob["beta_max"])
    s.kl_bound = float(prob["kl_bound"])
    s.max_bisect = int(prob["max_bisect"])
    s.n_iters = int(prob.get("n_iters", 0))
    kind = _KIND[prob.get("coll_kind", "none")]
    s.coll_kind = kind
    ci = np.asarray(prob.get("coll_index", []), dtype=np.int32)
    s.coll_dim = int(ci.size)
    for k in range(ci.size):
        s.coll_index[k] = int(ci[k])
    s.gh_points = int(prob.get("gh_points", 1))
    s.coll_states = 1 if prob.get("coll_states", "all") == "interior" else 0
    if kind != COLL_NONE:
        g = arr(prob["sdf"], np.float32)
        s.sdf = g.ctypes.data_as(C.POINTER(C.c_float))
        if g.ndim == 2:
            s.gz, s.gy, s.gx = 1, g.shape[0], g.shape[1]
        else:
            s.gz, s.gy, s.gx = g.shape
        for k in range(3):
            s.origin[k] = float(prob["origin"][k])
        s.cell = float(prob["cell"])
        s.hinge_eps = float(prob["hinge_eps"])
        s.obs_weight = float(prob["obs_weight"])
        r = arr(prob["sphere_radius"])
        s.n_spheres = int(r.size)
        s.sphere_radius = _dptr(r)
        if kind == COLL_ARM3D:
            fk = prob["fk"]
            s.fk_base = _dptr(arr(fk["base"]))
            s.fk_link_len = _dptr(arr(fk["link_len"]))
            s.fk_sphere_frac = _dptr(arr(fk["sphere_frac"]))
            s.fk_axes = arr(fk["axes"], np.int32).ctypes.data_as(C.POINTER(C.c_int32))
            s.fk_sphere_link = arr(fk["sphere_link"], np.int32).ctypes.data_as(C.POINTER(C.c_int32))
    if mu_init is not None:
        s.mu_init = _dptr(arr(np.asarray(mu_init).reshape(N, n)))
    s.segments = int(prob.get("segments", _tuned_segments(prob)))
    s.expect_group = int(prob.get("expect_group", 0))
    s.quadrature = {"tensor": _abi.QUAD_TENSOR, "sparse": _abi.QUAD_SPARSE}[prob.get("quadrature", "tensor")]
    s.update = {"prox": _abi.UPDATE_PROX, "ngd": _abi.UPDATE_NGD}[prob.get("update", "prox")]
    return s, keep


_TUNED = None


def _tuned_segments(prob):
    """Chain segments for a plan from the autotuner's table (tuned.json next
    to this file), keyed by the plan's own state dimension and length only;
    0 = library default."""
    global _TUNED
    if _TUNED is None:
        import json
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
        _TUNED = json.load(open(path)) if os.path.exists(path) else {}
    table = _TUNED.get("segments", {}).get(str(int(prob["n"])))
    if not table:
        return 0
    # entries [N, segments] sorted by N: take the nearest tuned length
    N = int(prob["N"])
    return min(table, key=lambda e: abs(e[0] - N))[1]


class Context:
    """A live engine: the C context handle plus the torch arena and stream."""

    def __init__(self, handle, n, cfg, arena, stream):
        self.handle = handle
        self.n = n
        self.cfg = cfg
        self._arena = arena
        self._stream = stream
        self.plan_N = {}

    def __del__(self):
        try:
            if self.handle:
                pgvimp_destroy(self)
        except Exception:
            pass


def pgvimp_arena_bytes(n, max_plans, max_states, heap_bytes, trial_width=0, trial_slots=0):
    cfg = _abi.EngineCfg()
    cfg.n, cfg.max_plans, cfg.max_states, cfg.heap_bytes = n, max_plans, max_states, heap_bytes
    cfg.trial_width = trial_width
    cfg.trial_slots = trial_slots
    return int(_abi.load().pgvimp_arena_bytes(C.byref(cfg)))


def _heap_need(probs):
    """Context heap bytes for the problems (the library's per-plan sizing)."""
    total = 0
    for p in probs:
        st, keep = problem_struct(p)
        b = int(_abi.load().pgvimp_plan_heap_bytes(C.byref(st)))
        _check(b if b < 0 else 0)
        total += b
    return total


def pgvimp_create(problems, n=None, precision=FP64, max_plans=None, max_states=None, heap_bytes=None,
                  device=0, use_torch=True, stream=None, segments=0, expect_group=0, use_graph=True, mu_init=None,
                  trial_width=0, trial_lookahead=0, trial_slots=0):
    """Create a context holding `problems` (list of dicts); see pgvimp_create
    in include/pgvimp.h.  With use_torch the device arena is a torch uint8
    tensor and the work runs on a torch stream."""
    lib = _abi.load()
    problems = list(problems)
    if n is None:
        n = int(problems[0]["n"])
    max_plans = max_plans or max(1, len(problems))
    max_states = max_states or max(1, sum(int(p["N"]) for p in problems))
    heap_bytes = heap_bytes if heap_bytes is not None else _heap_need(problems) + (1 << 20)
    cfg = _abi.EngineCfg()
    cfg.device, cfg.n, cfg.precision, cfg.max_plans = device, n, precision, max_plans
    cfg.max_states, cfg.heap_bytes = max_states, heap_bytes
    cfg.segments, cfg.expect_group = segments, expect_group
    cfg.use_graph = int(use_graph) if not isinstance(use_graph, bool) else (1 if use_graph else 0)
    cfg.trial_width = trial_width
    cfg.trial_lookahead = trial_lookahead
    cfg.trial_slots = trial_slots
    arena = None
    tstream = None
    if use_torch:
        import torch
        need = int(lib.pgvimp_arena_bytes(C.byref(cfg)))
        if need < 0:
            _check(need)
        arena = torch.empty(need + 256, dtype=torch.uint8, device=f"cuda:{device}")
        ptr = arena.data_ptr()
        aligned = (ptr + 255) // 256 * 256
        cfg.dev_arena = C.c_void_p(aligned)
        cfg.arena_bytes = need
        tstream = stream if stream is not None else torch.cuda.Stream(device=device)
        cfg.stream = C.c_void_p(tstream.cuda_stream)
    structs, keep = [], []
    for k, p in enumerate(problems):
        s, kp = problem_struct(p, None if mu_init is None else mu_init[k])
        structs.append(s)
        keep.append(kp)
    arr = (_abi.Problem * max(1, len(structs)))(*structs)
    h = C.c_void_p()
    rc = lib.pgvimp_create(arr, len(structs), C.byref(cfg), C.byref(h))
    _check(rc, None)
    ctx = Context(h, n, cfg, arena, tstream)
    for k, p in enumerate(problems):
        ctx.plan_N[k] = int(p["N"])
    return ctx


def pgvimp_destroy(ctx):
    if ctx.handle:
        _abi.load().pgvimp_destroy(ctx.handle)
        ctx.handle = None


def pgvimp_add_plan(ctx, prob, mu_init=None):
    s, keep = problem_struct(prob, mu_init)
    pid = C.c_int32()
    _check(_abi.load().pgvimp_add_plan(ctx.handle, C.byref(s), C.byref(pid)), ctx.handle)
    ctx.plan_N[pid.value] = int(prob["N"])
    return pid.value


def pgvimp_remove_plan(ctx, plan):
    _check(_abi.load().pgvimp_remove_plan(ctx.handle, plan), ctx.handle)
    ctx.plan_N.pop(plan, None)


def pgvimp_marginals(ctx, plan):
    N, n = ctx.plan_N[plan], ctx.n
    S = np.zeros((N, n, n))
    So = np.zeros((max(N - 1, 0), n, n))
    ld = C.c_double()
    _check(_abi.load().pgvimp_marginals(ctx.handle, plan, S.ctypes.data, So.ctypes.data if So.size else None,
                                        C.byref(ld)), ctx.handle)
    return S, So, ld.value


def pgvimp_expect_all(ctx, reps=1):
    """Collision expectations of every live plan at its current state, reps
    times, left on the device (see pgvimp_expect_all in include/pgvimp.h)."""
    _check(_abi.load().pgvimp_expect_all(ctx.handle, int(reps)), ctx.handle)


def pgvimp_factor_expectations(ctx, plan):
    N, n = ctx.plan_N[plan], ctx.n
    E = np.zeros(N)
    g = np.zeros((N, n))
    H = np.zeros((N, n, n))
    Ep = np.zeros(N + 1)
    _check(_abi.load().pgvimp_factor_expectations(ctx.handle, plan, E.ctypes.data, g.ctypes.data,
                                                  H.ctypes.data, Ep.ctypes.data), ctx.handle)
    return E, g, H, Ep


def pgvimp_factor_expectations_noalloc(ctx, plan):
    """As pgvimp_factor_expectations, through the library's allocation-free
    entry point (fixed per-device staging array)."""
    N, n = ctx.plan_N[plan], ctx.n
    E = np.zeros(N)
    g = np.zeros((N, n))
    H = np.zeros((N, n, n))
    Ep = np.zeros(N + 1)
    _check(_abi.load().pgvimp_factor_expectations_noalloc(ctx.handle, plan, E.ctypes.data, g.ctypes.data,
                                                          H.ctypes.data, Ep.ctypes.data), ctx.handle)
    return E, g, H, Ep


def pgvimp_prox_step(ctx, n_iters=1):
    """Run n_iters iterations on all live plans; returns {plan: stats dict}."""
    P = ctx.cfg.max_plans
    st = (_abi.Stats * P)()
    _check(_abi.load().pgvimp_prox_step(ctx.handle, n_iters, st), ctx.handle)
    return {k: st[k].as_dict() for k in ctx.plan_N}


def pgvimp_solve(ctx, n_iters):
    """Restart every live plan from its prior and run n_iters iterations."""
    P = ctx.cfg.max_plans
    st = (_abi.Stats * P)()
    _check(_abi.load().pgvimp_solve(ctx.handle, n_iters, st), ctx.handle)
    return {k: st[k].as_dict() for k in ctx.plan_N}


def pgvimp_slr_linearize(ctx, plan, gravity=9.81, gh_points=3, rebuild_prior=True):
    N, n = ctx.plan_N[plan], ctx.n
    A = np.zeros((N, n, n))
    a = np.zeros((N, n))
    prm = np.array([gravity], dtype=np.float64)
    _check(_abi.load().pgvimp_slr_linearize(ctx.handle, plan, _abi.MODEL_QUAD2D, _dptr(prm), gh_points,
                                            1 if rebuild_prior else 0, A.ctypes.data, a.ctypes.data), ctx.handle)
    return A, a


def pgvimp_slr_round(ctx, plan, gravity=9.81, gh_points=3, n_iters=0, nominal_mean=None, nominal_cov=None):
    """One round of Alg. 2 in the library (see pgvimp_slr_round in
    include/pgvimp.h); returns (A_t, a_t)."""
    N, n = ctx.plan_N[plan], ctx.n
    A = np.zeros((N, n, n))
    a = np.zeros((N, n))
    prm = np.array([gravity], dtype=np.float64)
    m = c = None
    if nominal_mean is not None:
        m = np.ascontiguousarray(nominal_mean, dtype=np.float64).reshape(N, n)
        c = np.ascontiguousarray(nominal_cov, dtype=np.float64).reshape(N, n, n)
    _check(_abi.load().pgvimp_slr_round(ctx.handle, plan, _abi.MODEL_QUAD2D, _dptr(prm), gh_points,
                                        None if m is None else m.ctypes.data, None if c is None else c.ctypes.data,
                                        int(n_iters), A.ctypes.data, a.ctypes.data), ctx.handle)
    return A, a


def pgvimp_slr_round_many(ctx, plans, gravity=9.81, gh_points=3, n_iters=0):
    """A later round of Alg. 2 for several plans at once (see
    pgvimp_slr_round_many in include/pgvimp.h); returns the per-plan status
    codes (OK or ENOTPD)."""
    pl = np.ascontiguousarray(plans, dtype=np.int32)
    st = np.zeros(pl.size, dtype=np.int32)
    prm = np.array([gravity], dtype=np.float64)
    _check(_abi.load().pgvimp_slr_round_many(ctx.handle, int(pl.size), pl.ctypes.data, _abi.MODEL_QUAD2D,
                                             _dptr(prm), gh_points, int(n_iters), st.ctypes.data), ctx.handle)
    return st


def ipgvimp_next_round_many(ctx, plans, prob):
    """Later rounds of Alg. 2 for several plans sharing prob's model."""
    return pgvimp_slr_round_many(ctx, plans, gravity=prob["quad"]["gravity"], gh_points=prob.get("slr_points", 3),
                                 n_iters=int(prob["n_iters"]))


def ipgvimp_begin(ctx, plan, prob):
    """First round of Alg. 2 for a nonlinear plan: pgvimp_slr_round about the
    nominal trajectory (prob['nominal_mean'], prob['nominal_cov'])."""
    return pgvimp_slr_round(ctx, plan, gravity=prob["quad"]["gravity"], gh_points=prob.get("slr_points", 3),
                            n_iters=int(prob["n_iters"]), nominal_mean=prob["nominal_mean"],
                            nominal_cov=prob["nominal_cov"])


def ipgvimp_next_round(ctx, plan, prob):
    """Later rounds of Alg. 2: pgvimp_slr_round about the plan's current
    marginals."""
    return pgvimp_slr_round(ctx, plan, gravity=prob["quad"]["gravity"], gh_points=prob.get("slr_points", 3),
                            n_iters=int(prob["n_iters"]))


def pgvimp_get_state(ctx, plan):
    N, n = ctx.plan_N[plan], ctx.n
    mu = np.zeros((N, n))
    D = np.zeros((N, n, n))
    U = np.zeros((max(N - 1, 0), n, n))
    _check(_abi.load().pgvimp_get_state(ctx.handle, plan, mu.ctypes.data, D.ctypes.data,
                                        U.ctypes.data if U.size else None), ctx.handle)
    return mu, D, U


def pgvimp_set_state(ctx, plan, mu=None, D=None, U=None):
    conv = [None if x is None else np.ascontiguousarray(x, dtype=np.float64) for x in (mu, D, U)]
    ptrs = [None if x is None or x.size == 0 else x.ctypes.data for x in conv]
    _check(_abi.load().pgvimp_set_state(ctx.handle, plan, *ptrs), ctx.handle)


def pgvimp_set_budget(ctx, plan, iters_left):
    _check(_abi.load().pgvimp_set_budget(ctx.handle, plan, iters_left), ctx.handle)


def pgvimp_set_temperature(ctx, plan, temperature):
    _check(_abi.load().pgvimp_set_temperature(ctx.handle, plan, float(temperature)), ctx.handle)


def pgvimp_profile(ctx, enable=True):
    _check(_abi.load().pgvimp_profile(ctx.handle, 1 if enable else 0), ctx.handle)


def pgvimp_kernel_times(ctx, reset=True):
    """{kind: (mean_ms, launches)} for kinds expect, prep, trial, select, restart."""
    k = len(_abi.KERNEL_KINDS)
    ms = (C.c_double * k)()
    cnt = (C.c_int64 * k)()
    _check(_abi.load().pgvimp_kernel_times(ctx.handle, 1 if reset else 0, ms, cnt), ctx.handle)
    return {name: (ms[i], cnt[i]) for i, name in enumerate(_abi.KERNEL_KINDS)}


def pgvimp_launch_shape(ctx, N):
    s, l = C.c_int32(), C.c_int32()
    _check(_abi.load().pgvimp_launch_shape(ctx.handle, N, C.byref(s), C.byref(l)), ctx.handle)
    return s.value, l.value


def nan_to_none(x):
    return None if (x is None or (isinstance(x, float) and math.isnan(x))) else x
