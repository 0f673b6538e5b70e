"""ctypes binding of libconcpd.so (the C ABI declared in include/concpd.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libconcpd.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
OK, EINVAL, ENOTSUP, ENONFINITE, EHIP, ESTATE = 0, 1, 2, 3, 4, 5
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOTSUP", 3: "ENONFINITE", 4: "EHIP", 5: "ESTATE"}


MAX_ORDER = 6   # CONCPD_MAX_ORDER


class Config(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("num_blocks", ctypes.c_int32),
        ("rank", ctypes.c_int32),
        ("coupled", ctypes.c_int32 * MAX_ORDER),
        ("dims", ctypes.POINTER(ctypes.c_int64)),
        ("tensor_dtype", ctypes.c_int32),
        ("compute_dtype", ctypes.c_int32),
        ("update_core", ctypes.c_int32),
        ("restart", ctypes.c_int32),
        ("delta_w", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("max_it", ctypes.c_int32),
        ("tucker_ranks", ctypes.POINTER(ctypes.c_int32)),
        ("block_ranks", ctypes.POINTER(ctypes.c_int32)),
        ("coupled_blocks", ctypes.POINTER(ctypes.c_uint64)),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64),
        ("F", ctypes.c_double),
        ("relerr", ctypes.c_double),
        ("fit", ctypes.c_double),
        ("restarts", ctypes.c_int64),
        ("restarted_last", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("nonfinite", ctypes.c_int32),
        ("lra", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [
        ("k2_rows", ctypes.c_int32),
        ("graph_sweeps", ctypes.c_int32),
        ("us_per_sweep", ctypes.c_double),
        ("us_per_sweep_default", ctypes.c_double),
        ("candidates", ctypes.c_int32),
        ("p1_split", ctypes.c_int32),
        ("p1_dma", ctypes.c_int32),
        ("overlap", ctypes.c_int32),
        ("fuse", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


STATIC_WORKSPACE_BYTES = 32 << 20   # CONCPD_STATIC_WORKSPACE_BYTES of concpd.h

OPT_GRAPH_SWEEPS, OPT_OVERLAP, OPT_K2_ROWS, OPT_P1_SPLIT, OPT_P1_DMA, OPT_FUSE, OPT_FUSE_LRA = 1, 2, 3, 4, 5, 6, 7

_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_DPP = ctypes.POINTER(ctypes.POINTER(ctypes.c_double))
_DP = ctypes.POINTER(ctypes.c_double)
_I32P = ctypes.POINTER(ctypes.c_int32)

SIGNATURES = {
    "concpd_last_error": (ctypes.c_char_p, []),
    "concpd_query_workspace": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]),
    "concpd_init": (ctypes.c_int, [ctypes.POINTER(Config), _PP, _DPP, _DPP, ctypes.c_uint64, _P, ctypes.c_size_t, _P,
                                   ctypes.POINTER(_P)]),
    "concpd_init_static": (ctypes.c_int, [ctypes.POINTER(Config), _PP, _DPP, _DPP, ctypes.c_uint64, _P,
                                          ctypes.POINTER(_P)]),
    "concpd_step": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(Stats)]),
    "concpd_fit": (ctypes.c_int, [_P, ctypes.POINTER(Stats)]),
    "lra_compress": (ctypes.c_int, [_P, _I32P, ctypes.POINTER(Stats)]),
    "lra_step": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(Stats)]),
    "concpd_launch_floor": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _DP, _DP]),
    "concpd_get_state": (ctypes.c_int, [_P, _DPP, _DPP, _DPP, _DPP, _DP, _DP, _DP, _DP,
                                        ctypes.POINTER(ctypes.c_int64)]),
    "lra_compress_cp": (ctypes.c_int, [_P, _DPP, ctypes.c_uint64, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                       _I32P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(Stats)]),
    "lra_get_tucker": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _DP]),
    "concpd_set_option": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64]),
    "concpd_get_option": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "concpd_autotune": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(Tuning)]),
    "concpd_global_fit": (ctypes.c_int, [_P, _DP]),
    "concpd_get_factor": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _DP]),
    "concpd_get_lambda": (ctypes.c_int, [_P, ctypes.c_int32, _DP]),
    "concpd_get_lipschitz": (ctypes.c_int, [_P, _DP, _DP, _DP]),
    "concpd_set_state": (ctypes.c_int, [_P, _DPP, _DPP, _DPP, _DPP, _DP, _DP, _DP, ctypes.c_double, ctypes.c_int64]),
    "concpd_loss_grad": (ctypes.c_int, [_P, _PP, _PP, ctypes.c_int32, _DP, _PP, _PP]),
    "concpd_debug_mttkrp": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
    "concpd_debug_spectral_norm": (ctypes.c_int, [_DP, ctypes.c_int32, ctypes.c_int32, _DP]),
    "concpd_profile": (ctypes.c_int, [_P, ctypes.c_int32]),
    "concpd_profile_read": (ctypes.c_int, [_P, _DP, _DP, ctypes.POINTER(ctypes.c_int64)]),
    "concpd_destroy": (ctypes.c_int, [_P]),
}

_lib = None


class ConcpdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_05119_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != OK:
        msg = load().concpd_last_error()
        raise ConcpdError(status, msg.decode() if msg else "")
