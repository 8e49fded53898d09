"""ctypes declarations of the C ABI in ``include/tvstencil.h``.

This module only loads ``libtvstencil.so`` and declares argument types; it
raises ``ImportError`` if the library has not been built.  There is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TVS_LIBRARY: a host-sanitized build of the same sources (build.py --sanitize)
LIB_PATH = os.environ.get("TVS_LIBRARY") or os.path.join(HERE, "libtvstencil.so")

TVS_OK = 0
ERRORS = {
    -1: "TVS_E_INVALID", -2: "TVS_E_SHAPE", -3: "TVS_E_ORDER", -4: "TVS_E_UNSUPPORTED",
    -5: "TVS_E_NOMEM", -6: "TVS_E_DEVICE", -7: "TVS_E_BUSY", -8: "TVS_E_NOTFOUND",
}

i64 = ctypes.c_int64
vp = ctypes.c_void_p
dp = ctypes.POINTER(ctypes.c_double)


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("dims", i64 * 3), ("dtype", ctypes.c_int),
        ("shape", ctypes.c_int), ("order", ctypes.c_int), ("dependence", ctypes.c_int),
        ("boundary", ctypes.c_int), ("radius", ctypes.c_int), ("method", ctypes.c_int),
        ("k", ctypes.c_int), ("s", ctypes.c_int), ("tile_w", ctypes.c_int),
        ("tile_h", ctypes.c_int), ("tile_l", ctypes.c_int), ("lane_c", ctypes.c_int),
        ("lanemap", ctypes.c_int), ("scratch_bytes", ctypes.c_size_t),
        ("pl", ctypes.c_int), ("kern", ctypes.c_int), ("tuning", ctypes.c_char * 160),
        ("rule", ctypes.c_int), ("varcoef_tuning", ctypes.c_char * 160),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("dims", i64 * 3), ("dtype", ctypes.c_int),
        ("shape", ctypes.c_int), ("order", ctypes.c_int), ("dependence", ctypes.c_int),
        ("boundary", ctypes.c_int), ("coeffs", dp), ("T", i64), ("host_in", vp),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
        ("chunks", ctypes.c_uint64), ("resident", ctypes.c_uint64),
        ("bytes_in_use", ctypes.c_size_t), ("busy_seconds", ctypes.c_double),
        ("updates", ctypes.c_double),
    ]


# (name, restype, argtypes) for every symbol the header declares
SIGNATURES = [
    ("stencil_plan", ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(i64),
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_char_p]),
    ("stencil_plan_life", ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(i64),
                                         ctypes.c_int, ctypes.c_char_p]),
    ("stencil_plan_info", ctypes.c_int, [vp, ctypes.POINTER(PlanInfo)]),
    ("stencil_plan_destroy", ctypes.c_int, [vp]),
    ("stencil_run", ctypes.c_int, [vp, vp, dp, i64, vp]),
    ("stencil_run_varcoef", ctypes.c_int, [vp, vp, vp, i64, vp]),
    ("stencil_plan_check", ctypes.c_int, [vp]),
    ("stencil_run_simple", ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(i64), ctypes.c_int,
                                          dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, i64, vp]),
    ("stencil_batch_run", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(dp), ctypes.POINTER(i64), vp]),
    ("stencil_tune", ctypes.c_int, [vp, vp, dp, i64, vp, ctypes.c_char_p, ctypes.c_size_t]),
    ("stencil_server_create", ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_size_t, ctypes.c_int,
                                             ctypes.c_int]),
    ("stencil_server_submit", ctypes.c_int, [vp, ctypes.POINTER(Request),
                                             ctypes.POINTER(ctypes.c_uint64)]),
    ("stencil_server_poll", ctypes.c_int, [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), vp,
                                           dp]),
    ("stencil_server_wait", ctypes.c_int, [vp, ctypes.c_uint64, vp, dp]),
    ("stencil_server_stats", ctypes.c_int, [vp, ctypes.POINTER(ServerStats)]),
    ("stencil_server_now", ctypes.c_double, [vp]),
    ("stencil_server_destroy", ctypes.c_int, [vp]),
    ("stencil_lcs_plan", ctypes.c_int, [ctypes.POINTER(vp), i64, i64, ctypes.c_char_p]),
    ("stencil_lcs_tile_width", ctypes.c_int, [vp]),
    ("stencil_lcs_tile_rows", ctypes.c_int, [vp]),
    ("stencil_lcs_run", ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
    ("stencil_lcs_run_noalloc", ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
    ("stencil_lcs_destroy", ctypes.c_int, [vp]),
    ("stencil_last_error", ctypes.c_char_p, []),
    ("stencil_version", ctypes.c_char_p, []),
]

_lib = None


def load():
    """Load the built library (raises ImportError if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2010_04868_amd/build.py "
                          "(or __graft_entry__.build())")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (same
    # SONAME as the system one).  Loading torch first makes this library bind
    # to that runtime, so the device pointers and stream handles torch hands
    # us belong to the runtime our kernels are launched on.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class StencilError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(rc: int) -> None:
    if rc != TVS_OK:
        raise StencilError(rc, (load().stencil_last_error() or b"").decode())
