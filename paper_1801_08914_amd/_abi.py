"""ctypes declarations of include/hyb.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhyb.so")

HYB_OK = 0
HYB_E_ARG = -1
HYB_E_MESH = -2
HYB_E_JACOBIAN = -3
HYB_E_NOT_SPD = -4
HYB_E_STATE = -5
HYB_E_NOMEM = -6
HYB_E_NOCONV = -7
HYB_E_HIP = -8
HYB_E_INTERNAL = -9
HYB_E_REFINE = -10
HYB_FP64 = 0
HYB_MIXED = 1
HYB_HYBRID = 0
HYB_STATIC = 1

# Every extern "C" symbol declared in include/hyb.h.
EXPORTS = [
    "hyb_plan_create", "hyb_plan_topology", "hyb_last_detail", "hyb_bind", "hyb_setup", "hyb_rhs",
    "hyb_pcg", "hyb_pcg_noalloc", "hyb_solve", "hyb_get_csr", "hyb_fallback_count", "hyb_recover", "hyb_status", "hyb_strerror", "hyb_destroy",
    "hyb_timing_enable", "hyb_timing_read", "hyb_set_stream",
    "hyb_batch_create", "hyb_batch_set", "hyb_batch_setup", "hyb_batch_recover", "hyb_batch_set_tiles",
    "hyb_batch_get_tiles", "hyb_batch_graph", "hyb_batch_autotune", "hyb_batch_timing_enable",
    "hyb_batch_timing_read", "hyb_batch_destroy",
]


class HybBatchTiles(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("items_per_block", ctypes.c_int32)]


class HybError(RuntimeError):
    def __init__(self, code: int, msg: str, detail: int):
        super().__init__(f"hyb error {code} ({msg}), detail {detail}")
        self.code = code
        self.detail = detail


class HybMesh(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("ne", ctypes.c_int64), ("xyz", ctypes.c_void_p),
                ("e2v", ctypes.c_void_p), ("ess", ctypes.c_void_p)]


class HybOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("stream", ctypes.c_void_p), ("kernel_variant", ctypes.c_int),
                ("refine_sweeps", ctypes.c_int), ("pcg_reduce", ctypes.c_int), ("system", ctypes.c_int),
                ("weighted_c", ctypes.c_int), ("quad_q", ctypes.c_int)]


class HybSizes(ctypes.Structure):
    _fields_ = [("ne", ctypes.c_int64), ("k", ctypes.c_int32), ("n_local", ctypes.c_int32),
                ("n_interior", ctypes.c_int32), ("n_face_dofs", ctypes.c_int32),
                ("n_faces", ctypes.c_int64), ("n_boundary_faces", ctypes.c_int64), ("m", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("factor_len", ctypes.c_int64), ("bytes_maps", ctypes.c_int64),
                ("bytes_factor", ctypes.c_int64), ("bytes_y", ctypes.c_int64), ("bytes_work", ctypes.c_int64)]


BUFFER_FIELDS = ["maps", "factor", "y", "row_ptr", "col", "val", "r", "work", "status"]


class HybBuffers(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in BUFFER_FIELDS]


class HybSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("rel_res", ctypes.c_double)]


_LIB = None


def load_library():
    """Load libhyb.so from the package directory; raise if it was not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.hyb_plan_create.argtypes = [vp, ci, vp, vp, vp]
    lib.hyb_plan_topology.argtypes = [vp] * 7
    lib.hyb_last_detail.restype = i64
    lib.hyb_last_detail.argtypes = []
    lib.hyb_bind.argtypes = [vp, vp]
    lib.hyb_setup.argtypes = [vp, vp, vp, vp, vp]
    lib.hyb_rhs.argtypes = [vp, vp, vp]
    lib.hyb_pcg.argtypes = [vp, ctypes.c_double, ci, vp, vp]
    lib.hyb_pcg_noalloc.argtypes = [vp, ctypes.c_double, ci, vp, vp]
    lib.hyb_solve.argtypes = [vp, vp, vp, ctypes.c_double, ci, vp, vp, vp]
    lib.hyb_get_csr.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.hyb_fallback_count.argtypes = [vp, vp]
    lib.hyb_recover.argtypes = [vp, vp, vp]
    lib.hyb_status.argtypes = [vp, vp]
    lib.hyb_strerror.restype = ctypes.c_char_p
    lib.hyb_strerror.argtypes = [ci]
    lib.hyb_timing_enable.argtypes = [vp, ci]
    lib.hyb_timing_read.argtypes = [vp, vp, vp, vp, vp]
    lib.hyb_destroy.argtypes = [vp]
    lib.hyb_destroy.restype = None
    lib.hyb_set_stream.argtypes = [vp, vp]
    lib.hyb_batch_create.argtypes = [vp, ctypes.c_int32, vp]
    lib.hyb_batch_set.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp]
    lib.hyb_batch_setup.argtypes = [vp]
    lib.hyb_batch_recover.argtypes = [vp]
    lib.hyb_batch_set_tiles.argtypes = [vp, vp]
    lib.hyb_batch_get_tiles.argtypes = [vp, vp]
    lib.hyb_batch_graph.argtypes = [vp, ci]
    lib.hyb_batch_autotune.argtypes = [vp, ci, vp]
    lib.hyb_batch_timing_enable.argtypes = [vp, ci]
    lib.hyb_batch_timing_read.argtypes = [vp, vp, vp, vp, vp]
    lib.hyb_batch_destroy.argtypes = [vp]
    lib.hyb_batch_destroy.restype = None
    for name in EXPORTS:
        if name not in ("hyb_destroy", "hyb_last_detail", "hyb_strerror", "hyb_batch_destroy"):
            getattr(lib, name).restype = ci
    _LIB = lib
    return lib


def check(lib, rc: int):
    if rc != HYB_OK:
        raise HybError(rc, lib.hyb_strerror(rc).decode(), int(lib.hyb_last_detail()))
