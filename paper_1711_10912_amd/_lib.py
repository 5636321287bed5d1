"""ctypes loader for libtlib.so (the HIP kernels behind the C ABI in include/tlib.h).

Loading fails loudly when the library has not been built; there is no
fallback implementation of any operation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtlib.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
OK, EINVAL, ESHAPE, EMODE, EDTYPE, EALIAS, ESTRIDE, ENOMEM, EHIP = range(9)
MAX_ORDER = 16

EXPORTS = (
    "tlib_ttv", "tlib_ttm", "tlib_ttm2", "tlib_ttt", "tlib_ttt_noalloc", "tlib_inner", "tlib_norm", "tlib_normalize", "tlib_add", "tlib_scale",
    "tlib_transpose", "tlib_times_vectors", "tlib_batch_table_bytes", "tlib_batch_plan", "tlib_batch_run",
    "tlib_request_check", "tlib_request_groupable", "tlib_server_create", "tlib_server_submit", "tlib_server_drain", "tlib_server_stats",
    "tlib_server_result", "tlib_server_reset_stats", "tlib_server_destroy",
    "tlib_strides_from_layout", "tlib_last_error", "tlib_strerror", "tlib_set_plan_only",
    "tlib_last_plan", "tlib_set_autotune", "tlib_autotune_entries", "tlib_autotune_clear", "tlib_autotune_save",
    "tlib_autotune_load", "tlib_version", "tlib_plan_cache_stats", "tlib_plan_cache_clear", "tlib_workspace_reserve", "tlib_workspace_size", "tlib_workspace_release",
)


class TensorDesc(ctypes.Structure):
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("extents", ctypes.POINTER(ctypes.c_int64)),
        ("strides", ctypes.POINTER(ctypes.c_int64)),
        ("layout", ctypes.POINTER(ctypes.c_int32)),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("A", ctypes.POINTER(TensorDesc)),
        ("B", ctypes.POINTER(TensorDesc)),
        ("C", ctypes.POINTER(TensorDesc)),
        ("q", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("phi", ctypes.POINTER(ctypes.c_int32)),
        ("psi", ctypes.POINTER(ctypes.c_int32)),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("completed", ctypes.c_int64), ("grouped", ctypes.c_int64), ("errors", ctypes.c_int64),
        ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double),
        ("req_per_s", ctypes.c_double),
    ]


class TlibError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("tlib error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libtlib.so is not built (%s); run __graft_entry__.build() or "
                              "python -m paper_1711_10912_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(TensorDesc)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        vp = ctypes.c_void_p
        L.tlib_ttv.argtypes = [P, P, ctypes.c_int32, P, vp]
        L.tlib_ttm.argtypes = [P, P, ctypes.c_int32, P, vp]
        L.tlib_ttm2.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_int32, P, vp]
        L.tlib_ttt.argtypes = [P, P, ctypes.c_int32, i32p, i32p, P, vp]
        L.tlib_ttt_noalloc.argtypes = [P, P, ctypes.c_int32, i32p, i32p, P, vp]
        L.tlib_inner.argtypes = [P, P, vp, vp]
        L.tlib_norm.argtypes = [P, vp, vp]
        L.tlib_normalize.argtypes = [P, vp, P, vp]
        L.tlib_add.argtypes = [ctypes.c_double, P, ctypes.c_double, P, P, vp]
        L.tlib_scale.argtypes = [ctypes.c_double, P, P, vp]
        L.tlib_transpose.argtypes = [P, i32p, P, vp]
        L.tlib_times_vectors.argtypes = [P, ctypes.POINTER(P), ctypes.c_int32, P, vp]
        L.tlib_strides_from_layout.argtypes = [ctypes.c_int32, i64p, i32p, i64p]
        L.tlib_batch_table_bytes.argtypes = [ctypes.c_int32]
        L.tlib_batch_table_bytes.restype = ctypes.c_size_t
        L.tlib_batch_plan.argtypes = [ctypes.POINTER(Request), ctypes.c_int32, vp, ctypes.c_size_t, i64p, i32p]
        L.tlib_batch_plan.restype = ctypes.c_int
        L.tlib_batch_run.argtypes = [vp, ctypes.c_int32, vp]
        L.tlib_batch_run.restype = ctypes.c_int
        L.tlib_request_check.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, ctypes.c_int32, i32p, i32p, P]
        L.tlib_request_check.restype = ctypes.c_int
        L.tlib_request_groupable.argtypes = [ctypes.POINTER(Request)]
        L.tlib_request_groupable.restype = ctypes.c_int
        L.tlib_plan_cache_stats.argtypes = [i64p, i64p, i64p]
        L.tlib_plan_cache_stats.restype = None
        L.tlib_plan_cache_clear.argtypes = []
        L.tlib_plan_cache_clear.restype = None
        L.tlib_workspace_reserve.argtypes = [vp, ctypes.c_size_t]
        L.tlib_workspace_reserve.restype = ctypes.c_int
        L.tlib_workspace_size.argtypes = [vp]
        L.tlib_workspace_size.restype = ctypes.c_size_t
        L.tlib_workspace_release.argtypes = [vp]
        L.tlib_workspace_release.restype = ctypes.c_int
        L.tlib_server_create.argtypes = [ctypes.c_int32, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_int32]
        L.tlib_server_create.restype = vp
        L.tlib_server_submit.argtypes = [vp, ctypes.c_int32, P, P, ctypes.c_int32, ctypes.c_int32, i32p, i32p, P,
                                         i64p]
        L.tlib_server_submit.restype = ctypes.c_int
        L.tlib_server_drain.argtypes = [vp, ctypes.c_double]
        L.tlib_server_drain.restype = ctypes.c_int
        L.tlib_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.tlib_server_stats.restype = ctypes.c_int
        L.tlib_server_result.argtypes = [vp, ctypes.c_int64, P, i32p]
        L.tlib_server_result.restype = ctypes.c_int
        L.tlib_server_reset_stats.argtypes = [vp]
        L.tlib_server_reset_stats.restype = None
        L.tlib_server_destroy.argtypes = [vp]
        L.tlib_server_destroy.restype = None
        for f in ("tlib_ttv", "tlib_ttm", "tlib_ttm2", "tlib_ttt", "tlib_ttt_noalloc", "tlib_inner", "tlib_norm", "tlib_normalize", "tlib_add",
                  "tlib_scale", "tlib_transpose", "tlib_times_vectors", "tlib_strides_from_layout"):
            getattr(L, f).restype = ctypes.c_int
        L.tlib_last_error.restype = ctypes.c_char_p
        L.tlib_last_error.argtypes = []
        L.tlib_strerror.restype = ctypes.c_char_p
        L.tlib_strerror.argtypes = [ctypes.c_int]
        L.tlib_set_plan_only.argtypes = [ctypes.c_int]
        L.tlib_set_plan_only.restype = None
        L.tlib_last_plan.restype = ctypes.c_char_p
        L.tlib_last_plan.argtypes = []
        L.tlib_set_autotune.argtypes = [ctypes.c_int]
        L.tlib_set_autotune.restype = ctypes.c_int
        L.tlib_autotune_entries.argtypes = []
        L.tlib_autotune_entries.restype = ctypes.c_int64
        L.tlib_autotune_clear.argtypes = []
        L.tlib_autotune_clear.restype = None
        for f in ("tlib_autotune_save", "tlib_autotune_load"):
            getattr(L, f).argtypes = [ctypes.c_char_p]
            getattr(L, f).restype = ctypes.c_int
        L.tlib_version.restype = ctypes.c_char_p
        L.tlib_version.argtypes = []
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != OK:
        L = lib()
        msg = L.tlib_last_error().decode() or L.tlib_strerror(rc).decode()
        raise TlibError(rc, msg)


def desc(ptr: int, dtype: int, shape, strides=None, layout=None) -> TensorDesc:
    """Build a descriptor from plain values (the arrays stay referenced by the struct)."""
    p = len(shape)
    d = TensorDesc()
    d.data = ctypes.c_void_p(int(ptr))
    d.dtype = dtype
    d.order = p
    ext = (ctypes.c_int64 * max(1, p))(*[int(v) for v in shape])
    d.extents = ctypes.cast(ext, ctypes.POINTER(ctypes.c_int64))
    d._ext = ext
    if strides is not None:
        st = (ctypes.c_int64 * max(1, p))(*[int(v) for v in strides])
        d.strides = ctypes.cast(st, ctypes.POINTER(ctypes.c_int64))
        d._st = st
    if layout is not None:
        ly = (ctypes.c_int32 * max(1, p))(*[int(v) for v in layout])
        d.layout = ctypes.cast(ly, ctypes.POINTER(ctypes.c_int32))
        d._ly = ly
    return d


def i32_array(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int32 * max(1, len(vals)))(*vals)
