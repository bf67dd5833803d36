"""ctypes binding of ``lib/libofmi.so`` with the C ABI's names.

This layer only marshals arguments: every step of the method runs in the HIP library.
PyTorch supplies device memory (workspaces, outputs) and streams.  If the library has not
been built, :func:`load` raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libofmi.so")

OF_OK, OF_EINVAL, OF_ENOMEM, OF_EHIP, OF_ESTATE = range(5)
OF_FLAG_FP16_STORAGE = 1 << 0
OF_FLAG_INPUT_F32 = 1 << 1
OF_FLAG_NO_GRAPH = 1 << 2
OF_FLAG_NORMALIZE = 1 << 3
OF_FLAG_GAUSSIAN_WINDOW = 1 << 4
OF_FLAG_GRAPH = 1 << 5
OF_STAGE_REDUCE = 0
OF_STAGE_ITERATE = 1
OF_KERNEL_ITERATE = 0
OF_KERNEL_REDUCE = 1
OF_TIMING_LAUNCH = 1
OF_TIMING_LEVEL = 2


def OF_KERNEL_LEVEL(level: int) -> int:
    return 16 + level
OF_TILE_NARROW = 0
OF_TILE_WIDE = 1
OF_TILE_WIDE_LEAN = 2
OF_TILE_WIDE32 = 3
OF_TILE_WIDE16 = 4
OF_TILE_WIDE32X2 = 5
OF_TILE_WIDE16X2 = 6
OF_TILE_LEAN32X2 = 7

# exported symbol -> (restype, argtypes)
_c_int, _c_uint, _c_size, _vp = ctypes.c_int, ctypes.c_uint, ctypes.c_size_t, ctypes.c_void_p
_VPP = ctypes.POINTER(ctypes.c_void_p)
_INTP = ctypes.POINTER(ctypes.c_int)
SIGNATURES = {
    "of_plan_workspace_bytes": (_c_size, [_c_int, _c_int, _c_int, _c_int, _c_int, _c_uint]),
    "of_plan_create": (_vp, [_c_int, _c_int, _c_int, _c_int, _c_int]),
    "of_plan_create_ex": (_vp, [_c_int, _c_int, _c_int, _c_int, _c_int, _c_uint, _vp, _c_size]),
    "of_compute": (_c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "of_plan_destroy": (None, [_vp]),
    "of_noalloc_scratch_bytes": (_c_size, []),
    "of_compute_noalloc": (_c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, _c_uint, _vp, _vp, _vp, _vp, _vp]),
    "of_plan_set_mask": (_c_int, [_vp, _vp, _vp]),
    "of_levels_for_displacement": (_c_int, [ctypes.c_float, _c_int, _c_int]),
    "of_last_error": (ctypes.c_char_p, []),
    "of_debug_stage": (_c_int, [_vp, _c_int, _c_int, _VPP, _VPP, _vp]),
    "of_batch_workspace_bytes": (_c_size, [_c_int, _INTP, _INTP, _c_int, _c_int, _c_int, _c_uint]),
    "of_batch_create": (_vp, [_c_int, _INTP, _INTP, _c_int, _c_int, _c_int, _c_uint, _vp, _c_size]),
    "of_batch_compute": (_c_int, [_vp, _VPP, _VPP, _VPP, _VPP, _vp]),
    "of_batch_get_config": (_c_int, [_vp, _INTP, _INTP, _INTP]),
    "of_batch_set_config": (_c_int, [_vp, _INTP, _INTP, _INTP]),
    "of_batch_autotune": (_c_int, [_vp, _VPP, _VPP, _VPP, _VPP, _vp, _c_int]),
    "of_batch_set_timing": (_c_int, [_vp, _c_int]),
    "of_batch_read_timing": (_c_int, [_vp, _c_int, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "of_batch_destroy": (None, [_vp]),
    "of_batch_set_masks": (_c_int, [_vp, _VPP, _vp]),
    "of_session_set_mask": (_c_int, [_vp, _vp, _vp]),
    "of_session_bytes": (_c_size, [_c_int, _c_int, _c_int, _c_int, _c_int, _c_uint]),
    "of_server_create": (_vp, [_c_int, _c_int, _c_int, _c_uint, _c_size]),
    "of_server_open": (_vp, [_vp, _c_int, _c_int]),
    "of_server_open_ex": (_vp, [_vp, _c_int, _c_int, _vp, _c_size]),
    "of_session_create": (_vp, [_c_int, _c_int, _c_int, _c_int, _c_int, _c_uint, _vp, _c_size]),
    "of_session_push_many": (_c_int, [_VPP, _c_int, _VPP, _VPP, _VPP, _INTP, _vp]),
    "of_session_destroy": (None, [_vp]),
    "of_server_push": (_c_int, [_vp, _VPP, _c_int, _VPP, _VPP, _VPP, _INTP, _vp]),
    "of_session_push": (_c_int, [_vp, _vp, _vp, _vp, _vp, _INTP]),
    "of_session_resident_bytes": (_c_size, [_vp]),
    "of_server_resident_bytes": (_c_size, [_vp]),
    "of_server_close": (_c_int, [_vp, _vp]),
    "of_server_destroy": (None, [_vp]),
    "of_normalize": (_c_int, [_vp, _vp, _c_int, _c_int, _c_int, ctypes.c_float, _c_uint, _vp]),
    "of_field_mean_update": (_c_int, [_vp, _vp, ctypes.c_longlong, _c_int, _vp]),
    "of_field_minmax": (_c_int, [_vp, ctypes.c_longlong, _vp, _vp, _vp]),
    "of_count_at_most": (_c_int, [_vp, ctypes.c_longlong, ctypes.c_float, _vp, _vp]),
    "of_plan_set_bubble": (_c_int, [_vp, _vp, _vp]),
    "of_bubble_step": (_c_int, [_vp, _vp, ctypes.c_longlong, _c_int, _vp, _vp, _vp, _vp, _vp]),
    "of_plan_get_config": (_c_int, [_vp, _INTP, _INTP]),
    "of_plan_set_config": (_c_int, [_vp, _INTP, _INTP]),
    "of_plan_autotune": (_c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _c_int]),
    "of_plan_set_timing": (_c_int, [_vp, _c_int]),
    "of_plan_read_timing": (_c_int, [_vp, _c_int, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


class OfError(RuntimeError):
    """A call into the HIP library failed; the message is the library's error text."""


def load(path: str = LIB_PATH):
    """Load the HIP library (once).  Raises if it is missing: build it with build()."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OfError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return (load().of_last_error() or b"").decode()


def check(status: int, what: str):
    if status != OF_OK:
        raise OfError(f"{what} failed (status {status}): {last_error()}")


def ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[int(p) for p in ptrs])
    return ctypes.cast(arr, _VPP), arr
