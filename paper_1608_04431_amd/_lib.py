"""ctypes loader for libd8flow.so (the C ABI in include/d8flow.h).

The library is built in-tree by ``paper_1608_04431_amd.build``.  There is no
fallback: if the shared library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libd8flow.so")

# every symbol declared in include/d8flow.h
EXPORTS = ("d8_directions", "d8_directions_rho8", "d8_workspace_bytes", "flow_accum", "flow_accum_adjoint",
           "d8_absorb_workspace_bytes", "flow_accum_absorb", "flow_accum_absorb_adjoint",
           "flow_accum_absorb_alpha_grad",
           "d8_stream_workspace_bytes", "flow_accum_streamed", "flow_accum_streamed_f32",
           "flow_accum_adjoint_streamed", "flow_accum_noalloc",
           "d8_batch_workspace_bytes", "flow_accum_batched", "d8_graph_create",
           "d8_graph_launch", "d8_graph_destroy",
           "d8_check_status", "d8_strerror", "d8_version", "d8_timing_enable",
           "d8_timing_report", "d8_last_error_message")

D8_OK, D8_EINVAL, D8_EWORKSPACE, D8_EHIP, D8_EDIRCODE, D8_ECYCLE = 0, -1, -2, -3, -4, -5
D8_ACC_U32, D8_ACC_F32 = 0, 1
D8_BATCH_FWD, D8_BATCH_ADJ = 1, 2


class BatchItem(ctypes.Structure):
    """d8_batch_item of include/d8flow.h (device pointers as integers)."""
    _fields_ = [("dirs", ctypes.c_void_p), ("weights", ctypes.c_void_p), ("acc", ctypes.c_void_p),
                ("grad_acc", ctypes.c_void_p), ("grad_weights", ctypes.c_void_p),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("tile_rows", ctypes.c_int), ("tile_cols", ctypes.c_int)]

D8_MAX_TILE_SIDE = 64

_lib = None


class D8Error(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        lib = load()
        msg = lib.d8_strerror(code).decode()
        if code == D8_EHIP:
            detail = lib.d8_last_error_message().decode()
            if detail:
                msg += f" [{detail}]"
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libd8flow.so is not built ({LIB_PATH}); run "
                           "`python -m paper_1608_04431_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    lib.d8_directions.argtypes = [vp, vp, i64, i64, ctypes.c_float, vp]
    lib.d8_directions.restype = i32
    lib.d8_directions_rho8.argtypes = [vp, vp, vp, i64, i64, ctypes.c_float, vp]
    lib.d8_directions_rho8.restype = i32
    lib.d8_workspace_bytes.argtypes = [i64, i64, i32, i32]
    lib.d8_workspace_bytes.restype = sz
    lib.flow_accum.argtypes = [vp, vp, vp, i32, i64, i64, i32, i32, vp, sz, vp]
    lib.flow_accum.restype = i32
    lib.flow_accum_noalloc.argtypes = [vp, vp, vp, i32, i64, i64, i32, i32, vp, vp]
    lib.flow_accum_noalloc.restype = i32
    lib.flow_accum_adjoint.argtypes = [vp, vp, vp, i64, i64, i32, i32, vp, sz, vp]
    lib.flow_accum_adjoint.restype = i32
    lib.d8_absorb_workspace_bytes.argtypes = [i64, i64, i32, i32]
    lib.d8_absorb_workspace_bytes.restype = sz
    lib.flow_accum_absorb.argtypes = [vp, vp, vp, vp, i64, i64, i32, i32, vp, sz, vp]
    lib.flow_accum_absorb.restype = i32
    lib.flow_accum_absorb_adjoint.argtypes = [vp, vp, vp, vp, i64, i64, i32, i32, vp, sz, vp]
    lib.flow_accum_absorb_adjoint.restype = i32
    lib.flow_accum_absorb_alpha_grad.argtypes = [vp, vp, vp, vp, i64, i64, vp]
    lib.flow_accum_absorb_alpha_grad.restype = i32
    lib.d8_stream_workspace_bytes.argtypes = [i64, i64, i32, i32, i64]
    lib.d8_stream_workspace_bytes.restype = sz
    lib.flow_accum_streamed.argtypes = [vp, vp, i64, i64, i32, i32, i64, vp, sz, vp]
    lib.flow_accum_streamed.restype = i32
    for name in ("flow_accum_streamed_f32", "flow_accum_adjoint_streamed"):
        getattr(lib, name).argtypes = [vp, vp, vp, i64, i64, i32, i32, i64, vp, sz, vp]
        getattr(lib, name).restype = i32
    items = ctypes.POINTER(BatchItem)
    lib.d8_batch_workspace_bytes.argtypes = [items, i32]
    lib.d8_batch_workspace_bytes.restype = sz
    lib.flow_accum_batched.argtypes = [items, i32, i32, vp, sz, vp]
    lib.flow_accum_batched.restype = i32
    lib.d8_graph_create.argtypes = [items, i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
    lib.d8_graph_create.restype = i32
    lib.d8_graph_launch.argtypes = [vp, vp]
    lib.d8_graph_launch.restype = i32
    lib.d8_graph_destroy.argtypes = [vp]
    lib.d8_graph_destroy.restype = i32
    lib.d8_check_status.argtypes = [vp, vp]
    lib.d8_check_status.restype = i32
    lib.d8_strerror.argtypes = [i32]
    lib.d8_strerror.restype = ctypes.c_char_p
    lib.d8_version.argtypes = []
    lib.d8_version.restype = i32
    lib.d8_last_error_message.argtypes = []
    lib.d8_last_error_message.restype = ctypes.c_char_p
    lib.d8_timing_enable.argtypes = [i32]
    lib.d8_timing_enable.restype = i32
    lib.d8_timing_report.argtypes = [ctypes.POINTER(ctypes.c_char_p),
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64), i32]
    lib.d8_timing_report.restype = i32
    _lib = lib
    return lib


def check(rc: int, what: str = ""):
    if rc != D8_OK:
        raise D8Error(rc, what)
