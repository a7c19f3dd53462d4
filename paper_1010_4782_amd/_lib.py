"""ctypes mirror of include/stagcg.h and the loader of libstagcg.so.

Argument marshalling only: every step of the solver runs in the HIP library.
If the library has not been built, importing the high-level API still works,
but the first call raises (there is no fallback implementation).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstagcg.so")

STAG_OK = 0
STAG_ERR_ARG = 1
STAG_ERR_HIP = 2
STAG_ERR_NOMEM = 3
STAG_ERR_STATE = 4
STAG_ERR_NOT_CONVERGED = 5
STAG_ERR_NAN = 6
STATUS_NAMES = {0: "STAG_OK", 1: "STAG_ERR_ARG", 2: "STAG_ERR_HIP", 3: "STAG_ERR_NOMEM", 4: "STAG_ERR_STATE",
                5: "STAG_ERR_NOT_CONVERGED", 6: "STAG_ERR_NAN"}

PREC = {"f64": 0, "f32": 1, "f16": 2}
PRECOND = {"none": 0, "net": 1}


class StagParams(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("max_iter", C.c_int32),
        ("prec", C.c_int32),
        ("reliable_interval", C.c_int32),
        ("reliable_delta", C.c_double),
        ("check_interval", C.c_int32),
        ("max_restarts", C.c_int32),
        ("precond", C.c_int32),
        ("net", C.c_void_p),
        ("stall_window", C.c_int32),
        ("stall_ratio", C.c_double),
        ("profile", C.c_int32),
        ("history_len", C.c_int32),
        ("history", C.POINTER(C.c_double)),
        ("autotune", C.c_int32),
        ("reserved", C.c_int32 * 7),
    ]


class StagInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int32),
        ("restarts", C.c_int32),
        ("n_reliable", C.c_int32),
        ("fell_back", C.c_int32),
        ("converged", C.c_int32),
        ("status", C.c_int32),
        ("true_resid", C.c_double),
        ("ms", C.c_double),
        ("dslash_ms", C.c_double),
        ("dslash_calls", C.c_int32),
        ("dslash_prec", C.c_int32),
        ("dslash_sites", C.c_double),
        ("dslash_wg", C.c_int32),
        ("dslash_rhs", C.c_int32),
        ("dslash_lds", C.c_int32),
        ("dslash_order", C.c_int32),
        ("dslash_chunks", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class StagShape(C.Structure):
    _fields_ = [("wg", C.c_int32), ("rhs_per_lane", C.c_int32), ("lds_stage", C.c_int32), ("tile_order", C.c_int32),
                ("t_chunks", C.c_int32), ("us", C.c_double)]


class StagProblem(C.Structure):
    _fields_ = [
        ("lat", C.c_void_p),
        ("nrhs", C.c_int32),
        ("mass", C.POINTER(C.c_double)),
        ("b", C.c_void_p),
        ("x", C.c_void_p),
    ]


class StagTrainParams(C.Structure):
    _fields_ = [
        ("epochs", C.c_int32),
        ("batch", C.c_int32),
        ("lr", C.c_double),
        ("beta1", C.c_double),
        ("beta2", C.c_double),
        ("eps", C.c_double),
        ("seed", C.c_uint64),
        ("loss_kind", C.c_int32),
        ("reserved0", C.c_int32),
        ("mass", C.c_double),
        ("reserved", C.c_int32 * 6),
    ]


class StagTrainInfo(C.Structure):
    _fields_ = [
        ("loss_first", C.c_double),
        ("loss_last", C.c_double),
        ("epochs", C.c_int32),
        ("steps", C.c_int32),
        ("ms", C.c_double),
    ]


# name -> (restype, argtypes); every function of include/stagcg.h
SIGNATURES = {
    "stag_cg_params_default": (None, [C.POINTER(StagParams)]),
    "stag_last_error": (C.c_char_p, []),
    "stag_create_lattice": (C.c_int, [C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_void_p)]),
    "stag_destroy_lattice": (C.c_int, [C.c_void_p]),
    "stag_lattice_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "stag_load_links": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_uint32, C.c_void_p]),
    "stag_dslash": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "stag_apply_m": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "stag_fatten_links": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "stag_apply_m_noalloc": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_int32,
                                       C.c_void_p]),
    "stag_dslash_slab": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                   C.c_int32, C.c_void_p]),
    "stag_cg_solve": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_int32,
                                C.POINTER(StagParams), C.POINTER(StagInfo), C.c_void_p]),
    "stag_cg_solve_batch": (C.c_int, [C.c_int32, C.POINTER(StagProblem), C.POINTER(StagParams),
                                      C.POINTER(StagInfo), C.c_void_p]),
    "stag_tune_dslash": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(StagShape), C.POINTER(StagShape),
                                   C.c_int32, C.POINTER(C.c_int32), C.c_void_p]),
    "stag_set_dslash_shape": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(StagShape)]),
    "stag_slice_norm2": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                   C.c_void_p, C.c_void_p]),
    "stag_pion_correlator": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_void_p]),
    "stag_stream_read": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "stag_tune_cache_save": (C.c_int, [C.c_char_p]),
    "stag_tune_cache_load": (C.c_int, [C.c_char_p]),
    "stag_net_create": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_uint32, C.c_uint64,
                                  C.POINTER(C.c_void_p)]),
    "stag_net_destroy": (C.c_int, [C.c_void_p]),
    "stag_net_num_weights": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "stag_net_set_weights": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int64]),
    "stag_net_get_weights": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int64]),
    "stag_net_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "stag_net_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_double,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "stag_train_params_default": (None, [C.POINTER(StagTrainParams)]),
    "stag_net_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(StagTrainParams),
                                 C.POINTER(StagTrainInfo), C.c_void_p]),
}

_LIB = None


class StagError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


def lib():
    """The loaded library; raises if it was not built (no fallback exists)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1010_4782_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _LIB = h
    return _LIB


def check(status: int, where: str, allow=()):
    if status != STAG_OK and status not in allow:
        msg = lib().stag_last_error()
        raise StagError(status, where, msg.decode() if msg else "")
    return status


def default_params() -> StagParams:
    p = StagParams()
    lib().stag_cg_params_default(C.byref(p))
    return p
