"""ctypes mirror of include/pgvimp.h and loader of the in-tree libpgvimp.so.

Loading fails loudly (RuntimeError) when the library has not been built:
there is no CPU fallback for any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpgvimp.so")

OK, EINVAL, ENOMEM, ENOTPD, ENOCONV, EDEVICE, EBUSY = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
COLL_NONE, COLL_POINT2D, COLL_POINT3D, COLL_ARM3D = 0, 1, 2, 3
QUAD_TENSOR, QUAD_SPARSE = 0, 1
UPDATE_PROX, UPDATE_NGD = 0, 1
MODEL_QUAD2D = 1
MAX_COLL_DIM, MAX_SPHERES, ARM_DOF = 8, 32, 7
KERNEL_KINDS = ("expect", "prep", "trial", "select", "restart")

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)


class Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("m", C.c_int32), ("N", C.c_int32),
        ("dt", C.c_double),
        ("ltv", C.c_int32),
        ("A", _dp), ("a", _dp), ("B", _dp), ("Qc", _dp),
        ("mu_start", _dp), ("Sig_start", _dp), ("mu_goal", _dp), ("Sig_goal", _dp),
        ("temperature", C.c_double), ("beta_max", C.c_double), ("kl_bound", C.c_double),
        ("max_bisect", C.c_int32), ("n_iters", C.c_int32),
        ("coll_kind", C.c_int32), ("coll_dim", C.c_int32),
        ("coll_index", C.c_int32 * MAX_COLL_DIM),
        ("gh_points", C.c_int32), ("coll_states", C.c_int32),
        ("sdf", _fp),
        ("gx", C.c_int32), ("gy", C.c_int32), ("gz", C.c_int32),
        ("origin", C.c_double * 3),
        ("cell", C.c_double), ("hinge_eps", C.c_double), ("obs_weight", C.c_double),
        ("n_spheres", C.c_int32),
        ("sphere_radius", _dp),
        ("fk_base", _dp), ("fk_link_len", _dp), ("fk_sphere_frac", _dp),
        ("fk_axes", _ip), ("fk_sphere_link", _ip),
        ("mu_init", _dp),
        ("segments", C.c_int32), ("expect_group", C.c_int32),
        ("quadrature", C.c_int32), ("update", C.c_int32),
    ]


class EngineCfg(C.Structure):
    _fields_ = [
        ("device", C.c_int32), ("n", C.c_int32), ("precision", C.c_int32), ("max_plans", C.c_int32),
        ("max_states", C.c_int64), ("heap_bytes", C.c_int64),
        ("stream", C.c_void_p), ("dev_arena", C.c_void_p), ("arena_bytes", C.c_uint64),
        ("io_on_device", C.c_int32), ("segments", C.c_int32), ("expect_group", C.c_int32),
        ("use_graph", C.c_int32), ("trial_width", C.c_int32), ("trial_lookahead", C.c_int32),
        ("trial_slots", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("beta", C.c_double), ("kl", C.c_double), ("E_coll", C.c_double), ("E_prior", C.c_double),
        ("logdet", C.c_double), ("entropy", C.c_double),
        ("temperature", C.c_double), ("entropy_cost", C.c_double), ("total_cost", C.c_double),
        ("status", C.c_int32), ("trials", C.c_int32), ("iters_done", C.c_int32), ("iters_left", C.c_int32),
        ("trials_total", C.c_int32), ("evals_total", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes)
SIGNATURES = [
    ("pgvimp_create", C.c_int, [C.POINTER(Problem), C.c_int32, C.POINTER(EngineCfg), C.POINTER(C.c_void_p)]),
    ("pgvimp_destroy", C.c_int, [C.c_void_p]),
    ("pgvimp_add_plan", C.c_int, [C.c_void_p, C.POINTER(Problem), C.POINTER(C.c_int32)]),
    ("pgvimp_remove_plan", C.c_int, [C.c_void_p, C.c_int32]),
    ("pgvimp_marginals", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, _dp]),
    ("pgvimp_factor_expectations", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pgvimp_factor_expectations_noalloc", C.c_int,
     [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pgvimp_expect_all", C.c_int, [C.c_void_p, C.c_int32]),
    ("pgvimp_prox_step", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Stats)]),
    ("pgvimp_solve", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Stats)]),
    ("pgvimp_slr_linearize", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _dp, C.c_int32, C.c_int32,
                                       C.c_void_p, C.c_void_p]),
    ("pgvimp_slr_round_many", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, _dp, C.c_int32, C.c_int32,
                                        C.c_void_p]),
    ("pgvimp_slr_round", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _dp, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_int32, C.c_void_p, C.c_void_p]),
    ("pgvimp_get_state", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pgvimp_set_state", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pgvimp_set_budget", C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    ("pgvimp_set_temperature", C.c_int, [C.c_void_p, C.c_int32, C.c_double]),
    ("pgvimp_set_stream", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pgvimp_sync", C.c_int, [C.c_void_p]),
    ("pgvimp_launch_shape", C.c_int, [C.c_void_p, C.c_int32, _ip, _ip]),
    ("pgvimp_profile", C.c_int, [C.c_void_p, C.c_int32]),
    ("pgvimp_kernel_times", C.c_int, [C.c_void_p, C.c_int32, _dp, C.POINTER(C.c_int64)]),
    ("pgvimp_device_bytes", C.c_int64, [C.c_void_p]),
    ("pgvimp_arena_bytes", C.c_int64, [C.POINTER(EngineCfg)]),
    ("pgvimp_plan_heap_bytes", C.c_int64, [C.POINTER(Problem)]),
    ("pgvimp_last_error", C.c_char_p, [C.c_void_p]),
]

_lib = None


def load():
    """Load libpgvimp.so; raise if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime under the same soname as the
        # system one; importing it first makes the library bind to the
        # runtime that owns torch's device memory and streams.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is not built; run paper_2411_03416_amd.build.build() "
                "(there is no CPU fallback)")
        lib = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
