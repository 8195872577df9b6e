"""ctypes declarations of libhjg.so (the C interface in include/hjg.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any part of the sweep in Python.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhjg.so")

# enum values of include/hjg.h
HJG_OK, HJG_ENOTCONVERGED = 0, 1
HJG_EINVAL, HJG_ENOMEM, HJG_EHIP, HJG_ENONFINITE, HJG_EUNSUPPORTED = -1, -2, -3, -4, -5
HAMILTONIANS = {"quadratic": 0, "dubins_pairs": 1, "zero": 2, "double_integrator": 3, "pursuit_evasion": 4,
                "rockets": 5, "murmuration": 6}
DATUMS = {"half_sqnorm": 0, "ball": 1, "min_pair_disks": 2, "knn_balls": 3, "linear": 4, "capture": 5,
          "disc_union": 6}
SAMPLE_MODES = {"fresh": 0, "crn_step": 1}


class Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("ham", C.c_int32),
        ("ham_p", C.c_double * 8),
        ("datum", C.c_int32),
        ("datum_p", C.c_double * 4),
        ("datum_aux", C.c_void_p),
        ("nu", C.c_double),
        ("eta", C.c_double),
        ("c_min", C.c_double),
        ("c_max", C.c_double),
        ("tilt", C.c_int32),
        ("sample_mode", C.c_int32),
        ("sample_bf16", C.c_int32),
        ("grad_cv", C.c_int32),
        ("seed", C.c_uint64),
        ("problem_id", C.c_uint32),
        ("tube", C.c_int32),
    ]


class TrainCfg(C.Structure):
    _fields_ = [
        ("epochs", C.c_int32),
        ("batch", C.c_int32),
        ("lr", C.c_double),
        ("lr_min", C.c_double),
        ("weight_decay", C.c_double),
        ("beta1", C.c_double),
        ("beta2", C.c_double),
        ("eps", C.c_double),
        ("grad_weight", C.c_double),
        ("seed", C.c_uint64),
    ]


class Budget(C.Structure):
    _fields_ = [
        ("C1", C.c_double),
        ("rho", C.c_double),
        ("K", C.c_int32),
        ("C2", C.c_double),
        ("N", C.c_int64),
        ("delta_p", C.c_double),
        ("eps_ql", C.c_double),
        ("C3", C.c_double),
        ("delta", C.c_double),
    ]


class HJGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hjg error {code}: {msg}")
        self.code = code


_lib = None

# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("hjg_ctx_create", C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    ("hjg_ctx_destroy", None, [C.c_void_p]),
    ("hjg_last_error", C.c_char_p, []),
    ("hjg_version", C.c_char_p, []),
    ("hjg_philox4x32_10", C.c_int, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64, C.c_void_p,
                                    C.c_void_p]),
    ("hjg_sample_table", C.c_int, [C.c_void_p, C.POINTER(Problem), C.c_int32, C.c_uint32, C.c_void_p,
                                   C.c_void_p]),
    ("hjg_value_grad", C.c_int, [C.c_void_p, C.POINTER(Problem), C.c_int64, C.c_void_p, C.c_double, C.c_int32,
                                 C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_int32, C.c_void_p]),
    ("hjg_value_grad_noalloc", C.c_int, [C.c_void_p, C.POINTER(Problem), C.c_int64, C.c_void_p, C.c_double,
                                         C.c_int32, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hjg_picard_sweep_batched", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Problem), C.POINTER(C.c_int64),
                                           C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                           C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                           C.POINTER(C.c_int32), C.c_void_p]),
    ("hjg_knn_grid", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float),
                               C.c_float, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hjg_autotune_sweep", C.c_int, [C.c_void_p, C.POINTER(Problem), C.c_int64, C.c_void_p, C.c_double,
                                     C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double), C.c_void_p]),
    ("hjg_autotune_batched", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Problem), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                       C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double), C.c_void_p]),
    ("hjg_tuning_save", C.c_int, [C.c_void_p, C.c_char_p]),
    ("hjg_tuning_load", C.c_int, [C.c_void_p, C.c_char_p]),
    ("hjg_probe_valu_rate", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.c_void_p]),
    ("hjg_surrogate_create", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                       C.POINTER(C.c_void_p)]),
    ("hjg_surrogate_destroy", None, [C.c_void_p]),
    ("hjg_surrogate_param_count", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("hjg_surrogate_set_params", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hjg_surrogate_get_params", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hjg_surrogate_predict", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p]),
    ("hjg_surrogate_loss_grad", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_double, C.POINTER(C.c_double), C.c_void_p, C.c_void_p]),
    ("hjg_surrogate_train", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(TrainCfg), C.c_void_p, C.c_void_p]),
    ("hjg_surrogate_sweep", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Problem), C.c_int64, C.c_void_p,
                                      C.c_double, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                      C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                                      C.c_void_p]),
    ("hjg_surrogate_tube_step", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Problem), C.c_int64, C.c_void_p,
                                          C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_double, C.c_uint32,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                          C.POINTER(C.c_int32), C.c_void_p]),
    ("hjg_error_budget", C.c_int, [C.POINTER(Budget), C.POINTER(C.c_double)]),
    ("hjg_mc_margin", C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double,
                                C.c_double, C.c_void_p, C.c_void_p]),
    ("hjg_certify", C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hjg_avoid_project", C.c_int, [C.POINTER(Problem), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    ("hjg_topology", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    ("hjg_topology_events", C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hjg_smooth_slices", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_double, C.c_void_p,
                                    C.c_void_p]),
    ("hjg_isocontour", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_float, C.c_void_p, C.c_void_p,
                                 C.c_int64, C.c_void_p, C.c_void_p]),
    ("hjg_surrogate_save", C.c_int, [C.c_void_p, C.c_char_p]),
    ("hjg_surrogate_load", C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_void_p)]),
    ("hjg_set_timing", C.c_int, [C.c_void_p, C.c_int32]),
    ("hjg_sweep_time", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    ("hjg_picard_sweep", C.c_int, [C.c_void_p, C.POINTER(Problem), C.c_int64, C.c_void_p, C.c_double, C.c_int32,
                                   C.c_int32, C.c_double, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                   C.POINTER(C.c_int32), C.c_void_p]),
]


def lib():
    """The loaded library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc, gfx950); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int, allow=(HJG_OK,)) -> int:
    if code not in allow:
        raise HJGError(code, lib().hjg_last_error().decode())
    return code
