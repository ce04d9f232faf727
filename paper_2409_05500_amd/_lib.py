"""ctypes view of libvarlingam.so (the gfx950 HIP library).  No fallback: if the shared
library is missing or fails to load, importing this module raises."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvarlingam.so")

VL_OK = 0
VL_ERR_INVALID_ARG = -1
VL_ERR_SHAPE = -2
VL_ERR_DEGENERATE = -3
VL_ERR_SINGULAR = -4
VL_ERR_NONFINITE = -5
VL_ERR_WORKSPACE = -6
VL_ERR_HIP = -7

PREC = {"fp32": 0, "mixed": 1, "bf16": 2, "fp32_refined": 3, "sliced": 4}
PAIRWISE_COMPENSATED = 16   # flag OR-ed into the precision of the pairwise calls

_p = C.c_void_p
_i64 = C.c_int64
_i32 = C.c_int
_sz = C.c_size_t
_f64 = C.c_double

# name -> (restype, argtypes); the names and argument order are those of include/varlingam.h
class VlInstance(C.Structure):
    """Mirror of vl_instance (include/varlingam.h): one problem of a batched fit."""
    _fields_ = [("X", C.c_void_p), ("n", _i64), ("m", _i64), ("ldx", _i64), ("p", _i32),
                ("reserved", _i32), ("M", C.c_void_p), ("intercept", C.c_void_p),
                ("E", C.c_void_p), ("lde", _i64), ("S", C.c_void_p), ("order", C.c_void_p),
                ("margin", C.c_void_p), ("B0", C.c_void_p), ("Blag", C.c_void_p)]


SIGNATURES = {
    "varlingam_status_string": (C.c_char_p, [_i32]),
    "varlingam_fit_var_workspace_bytes": (_sz, [_i64, _i64, _i32, _i32]),
    "varlingam_fit_var": (_i32, [_p, _i64, _i64, _i64, _i32, _i32, _p, _p, _p, _i64, _p, _sz,
                                 _p, _p]),
    "varlingam_select_lag_workspace_bytes": (_sz, [_i64, _i64, _i32]),
    "varlingam_select_lag": (_i32, [_p, _i64, _i64, _i64, _i32, _p, _p, _p, _p, _p, _sz, _p,
                                    _p]),
    "pairwise_stats_workspace_bytes": (_sz, [_i64, _i64, _i32]),
    "pairwise_stats": (_i32, [_p, _i64, _i64, _i64, _i32, _p, _p, _p, _p, _p, _sz, _p, _p]),
    "pairwise_stats_noalloc_max_bytes": (_sz, []),
    "pairwise_stats_noalloc": (_i32, [_p, _i64, _i64, _i64, _i32, _p, _p, _p, _p, _p, _p]),
    "pairwise_stats_backward_workspace_bytes": (_sz, [_i64, _i64, _i32]),
    "pairwise_stats_saved_doubles": (_sz, [_i64]),
    "pairwise_stats_save": (_i32, [_p, _i64, _i64, _i64, _i32, _p, _p, _p, _p, _p, _p, _sz, _p,
                                   _p]),
    "pairwise_stats_backward": (_i32, [_p, _i64, _i64, _i64, _i32, _p, _p, _p, _i64, _p, _sz,
                                       _p, _p]),
    "approx_order_certified_workspace_bytes": (_sz, [_i64, _i64]),
    "approx_order_certified": (_i32, [_p, _i64, _i64, _i64, _p, _f64, _p, _p, _p,
                                      C.POINTER(_i64), _p, _sz, _p, _p]),
    "approx_order_workspace_bytes": (_sz, [_i64]),
    "approx_order": (_i32, [_p, _i64, _p, _p, _p, _sz, _p, _p]),
    "varlingam_order_iterative_workspace_bytes": (_sz, [_i64, _i64, _i32]),
    "varlingam_order_iterative": (_i32, [_p, _i64, _i64, _i64, _i32, _p, _p, _p, _sz, _p, _p]),
    "varlingam_order_hybrid_workspace_bytes": (_sz, [_i64, _i64, _i32]),
    "varlingam_order_hybrid": (_i32, [_p, _i64, _i64, _i64, _i32, _i64, _p, _p, _p, _sz, _p,
                                      _p]),
    "estimate_B_workspace_bytes": (_sz, [_i64, _i32]),
    "estimate_B": (_i32, [_p, _p, _p, _i64, _i32, _p, _p, _p, _sz, _p, _p]),
    "varlingam_var_simulate_workspace_bytes": (_sz, [_i64, _i32]),
    "varlingam_var_simulate": (_i32, [_p, _p, _i64, _i32, _p, _i64, _p, _i64, _i64, _p, _i64,
                                      _i64, _p, _i64, _i64, _p, _sz, _p, _p]),
    "varlingam_edge_frequency_workspace_bytes": (_sz, [_i64, _i64]),
    "varlingam_edge_frequency": (_i32, [_p, _p, _p, _i64, _i64, _i32, _f64, _p, _p, _p, _p,
                                        _p, _p, _sz, _p, _p]),
    "varlingam_prune_workspace_bytes": (_sz, [_i64, _i64, _i32, _i64]),
    "varlingam_prune": (_i32, [_p, _i64, _i64, _i64, _i32, _p, _p, _p, _i64, _p, _p, _p, _p,
                               _sz, _p, _p]),
    "varlingam_batch_create": (_i32, [C.POINTER(VlInstance), _i32, _i32,
                                      C.POINTER(C.c_void_p)]),
    "varlingam_batch_workspace_bytes": (_sz, [_p]),
    "varlingam_batch_bind": (_i32, [_p, _p, _sz, _p]),
    "varlingam_fit_batched": (_i32, [_p, _p, _p, _p]),
    "varlingam_batch_autotune": (_i32, [_p, _p, _sz, _p, _p]),
    "varlingam_batch_chunk_len": (_i32, [_p]),
    "varlingam_batch_chunk_len_of": (_i32, [_p, _i32]),
    "varlingam_batch_destroy": (None, [_p]),
    "varlingam_probe_workspace_bytes": (_sz, []),
    "varlingam_probe_rates": (_i32, [C.POINTER(C.c_double), _p, _sz, _p]),
    "varlingam_profile_enable": (None, [C.c_char_p]),
    "varlingam_profile_read": (_i32, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(_i64)]),
}


class VarLiNGAMError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} ({code})")


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2409_05500_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def status_string(code: int) -> str:
    return lib.varlingam_status_string(int(code)).decode()


def profile_enable(stages: str | None) -> None:
    """Record HIP events around the named stages ("*" = all, None = off); clears totals."""
    lib.varlingam_profile_enable(stages.encode() if stages else None)


def profile_read(stage: str) -> tuple[float, int]:
    """(total milliseconds, launches) recorded for one stage; waits for its events."""
    ms = C.c_double()
    cnt = _i64()
    check(lib.varlingam_profile_read(stage.encode(), C.byref(ms), C.byref(cnt)), "profile_read")
    return ms.value, cnt.value


def check(code: int, where: str) -> None:
    if code != VL_OK:
        raise VarLiNGAMError(code, where)
