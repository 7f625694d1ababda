"""ctypes view of libtensornet.so (declarations mirror include/tensornet.h)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TN_LIBRARY names another build of the same library (the host-side AddressSanitizer build of
# the CPU tests); by default the one built next to this file
LIB_PATH = os.environ.get("TN_LIBRARY") or os.path.join(HERE, "libtensornet.so")

TN_OK = 0
TN_E_ARG, TN_E_BLOB, TN_E_HIP, TN_E_BOX, TN_E_WORKSPACE, TN_E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
TN_STATUS_OVERFLOW, TN_STATUS_BATCH, TN_STATUS_Z, TN_STATUS_NONFINITE = 1, 2, 4, 8
TN_FP32, TN_BF16, TN_FP64 = 0, 1, 2
TN_FUSED, TN_PLAIN, TN_MOLECULE = 0, 1, 2
TN_NBR_AUTO, TN_NBR_CELL, TN_NBR_BRUTE = 0, 1, 2
TN_STATIC_WS_BYTES = 128 << 20   # size of the library's static scratch (tn_energy_forces_static)

_c = ctypes
_vp, _i32, _i64, _sz, _dbl = _c.c_void_p, _c.c_int, _c.c_int64, _c.c_size_t, _c.c_double

# name -> (restype, argtypes)
PROTOTYPES = {
    "tn_status_string": (_c.c_char_p, [_i32]),
    "tn_model_create": (_i32, [_vp, _sz, _i32, _c.POINTER(_vp)]),
    "tn_model_destroy": (None, [_vp]),
    "tn_model_info": (_i32, [_vp, _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32),
                             _c.POINTER(_c.c_int32), _c.POINTER(_dbl), _c.POINTER(_dbl)]),
    "tn_neighbor_workspace_bytes": (_sz, [_i64, _i64, _vp, _dbl]),
    "tn_build_neighbors": (_i32, [_vp, _i64, _vp, _i32, _vp, _vp, _dbl, _i64, _vp, _vp, _vp, _vp, _sz]),
    "tn_build_neighbors_method": (_i32, [_vp, _i64, _vp, _i32, _vp, _vp, _dbl, _i64, _vp, _vp, _vp, _vp, _sz, _i32]),
    "tn_workspace_bytes": (_sz, [_vp, _i64, _i64, _i64, _vp, _i32, _i32, _i32]),
    "tn_energy": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _sz]),
    "tn_energy_forces": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp,
                                _vp, _sz]),
    "tn_energy_forces_static": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp,
                                       _vp, _vp]),
    "tn_md_capture": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _dbl, _i32, _i64, _i32, _i32, _vp,
                             _vp, _vp, _vp, _vp, _sz, _c.POINTER(_vp)]),
    "tn_graph_replay": (_i32, [_vp, _vp]),
    "tn_graph_destroy": (_i32, [_vp]),
    "tn_pair_variant_count": (_i32, [_i32]),
    "tn_model_set_pair_variant": (_i32, [_vp, _i32, _i32, _i32]),
    "tn_autotune": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _i32,
                           _vp]),
    "tn_param_count": (_i64, [_vp]),
    "tn_train_workspace_bytes": (_sz, [_vp, _i64, _i64, _i64, _vp, _i32]),
    "tn_train_grad": (_i32, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _i64, _i32, _vp, _vp, _dbl, _dbl, _vp, _vp,
                             _vp, _vp, _vp, _vp, _vp, _sz]),
    "tn_timing_enable": (_i32, [_i32]),
    "tn_timing_reset": (_i32, []),
    "tn_timing_read": (_i32, [_c.c_char_p, _c.POINTER(_dbl), _c.POINTER(_i64)]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """Load the HIP library once; raises LibraryMissing if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(code: int) -> str:
    return lib().tn_status_string(int(code)).decode()
