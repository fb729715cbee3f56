"""ctypes binding of libfwht.so (the C ABI declared in include/fwht.h).

Argument marshalling only: every step of every transform runs in the HIP
kernels of the library.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfwht.so")

FWHT_OK, FWHT_E_INVAL, FWHT_E_RANGE, FWHT_E_CAPACITY, FWHT_E_NOMEM, FWHT_E_HIP, FWHT_E_UNSUPPORTED = range(7)
FWHT_I32, FWHT_I64, FWHT_F32 = 0, 1, 2
FWHT_PREC_FP32, FWHT_PREC_FP16_MFMA, FWHT_PREC_BF16_MFMA = 0, 1, 2
FWHT_NOALLOC_MAX_TRANSFORMS = 65536

STATUS_NAMES = {0: "FWHT_OK", 1: "FWHT_E_INVAL", 2: "FWHT_E_RANGE", 3: "FWHT_E_CAPACITY",
                4: "FWHT_E_NOMEM", 5: "FWHT_E_HIP", 6: "FWHT_E_UNSUPPORTED"}

# Every symbol include/fwht.h declares.
EXPORTS = ("fwht_int", "fwht_float", "fwht_float_out", "fwht_batched", "fwht_batched_noalloc", "fwht_threshold", "fwht_norms",
           "fwht_set_schedule", "fwht_get_schedule", "fwht_list_variants", "fwht_trace_enable", "fwht_trace_read",
           "fwht_copy", "fwht_fold", "fwht_fold_planted", "fwht_subspace_hits", "fwht_prime_omega", "fwht_last_error",
           "fwht_version", "fwht_set_batched_tiles", "fwht_get_batched_tiles", "fwht_set_batched_graphs",
           "fwht_get_batched_graphs")


class fwht_thresh_t(C.Structure):
    _fields_ = [("T", C.c_int64), ("Tf", C.c_double), ("idx", C.c_void_p), ("val", C.c_void_p),
                ("cap", C.c_uint64), ("count", C.c_void_p)]


class FWHTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> C.CDLL:
    """Load libfwht.so (built by __graft_entry__.build / paper_1607_01039_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes libfwht.so bind to that one, so both share one runtime
    # (one device context, torch's streams valid in the library).
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64 = C.c_void_p, C.c_int, C.c_int64, C.c_uint64
    L.fwht_int.argtypes = [vp, i32, i32, C.POINTER(fwht_thresh_t), vp]
    L.fwht_float.argtypes = [vp, i32, i64, i32, i32, vp]
    L.fwht_float_out.argtypes = [vp, vp, i32, i64, i32, i32, vp]
    L.fwht_batched.argtypes = [vp, vp, vp, C.c_int32, i32, i32, vp]
    L.fwht_batched_noalloc.argtypes = [vp, vp, vp, C.c_int32, i32, i32, vp]
    L.fwht_set_batched_tiles.argtypes = [i32, C.c_char_p]
    L.fwht_get_batched_tiles.argtypes = [i32, C.c_char_p, i32]
    L.fwht_set_batched_graphs.argtypes = [i32]
    L.fwht_get_batched_graphs.argtypes = []
    L.fwht_threshold.argtypes = [vp, i32, i32, C.POINTER(fwht_thresh_t), vp]
    L.fwht_norms.argtypes = [vp, vp, vp, vp, vp, C.c_int32, vp, vp]
    L.fwht_set_schedule.argtypes = [i32, i32, C.c_char_p]
    L.fwht_get_schedule.argtypes = [i32, i32, C.c_char_p, i32]
    L.fwht_list_variants.argtypes = [i32, C.c_char_p, i32]
    L.fwht_copy.argtypes = [vp, vp, u64, vp]
    L.fwht_trace_enable.argtypes = [i32]
    L.fwht_trace_read.argtypes = [vp, i32, C.POINTER(C.c_int), C.c_char_p, i32]
    L.fwht_fold.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
    L.fwht_fold_planted.argtypes = [i32, i32, i32, vp, u64, u64, u64, vp, vp, vp]
    L.fwht_subspace_hits.argtypes = [vp, u64, vp, i32, vp, vp]
    L.fwht_prime_omega.argtypes = [vp, i32, i32, vp]
    L.fwht_last_error.restype = C.c_char_p
    L.fwht_version.restype = C.c_char_p
    for name in ("fwht_int", "fwht_float", "fwht_float_out", "fwht_batched", "fwht_batched_noalloc", "fwht_threshold", "fwht_norms",
                 "fwht_set_schedule", "fwht_get_schedule", "fwht_list_variants", "fwht_copy",
                 "fwht_trace_enable", "fwht_trace_read", "fwht_fold", "fwht_fold_planted",
                 "fwht_subspace_hits", "fwht_prime_omega", "fwht_set_batched_tiles", "fwht_get_batched_tiles",
                 "fwht_set_batched_graphs", "fwht_get_batched_graphs"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != FWHT_OK:
        raise FWHTError(rc, lib().fwht_last_error().decode())
