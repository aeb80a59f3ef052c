"""ctypes declarations for libxdrop.so (include/xdrop.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# XDROP_LIB=stamps selects the instrumented build of the same sources
# (per-wave busy intervals, paper_2001_10049_amd/imbalance.py)
_VARIANT = os.environ.get("XDROP_LIB", "")
LIB_PATH = os.path.join(HERE, "libxdrop%s.so" % ("_" + _VARIANT if _VARIANT else ""))

XD_OK, XD_EINVAL, XD_ENOMEM, XD_EDEVICE, XD_EAGAIN = 0, -1, -2, -3, -4
TASK_OK, TASK_BAD_READ, TASK_BAD_SEED, TASK_BAD_X, TASK_BAND_OVERFLOW = 0, 1, 2, 3, 4
TASK_NO_SEED = 5
TASK_OPS_OVERFLOW, TASK_TRACE_FAULT = 6, 7
OP_M, OP_I, OP_D = 0, 1, 2
X_MAX = 1 << 20
BAND_MAX = 48
SCORE_LIMIT = 1000
BANDED_SCORE_LIMIT = 127
READ_MAX = 1 << 22
OVERLAP_K_MAX = 31
OVERLAP_M_MAX = 64

# every symbol include/xdrop.h declares
EXPORTS = (
    "xd_pack_reads", "xd_store_create", "xd_store_create_from_codes", "xd_store_destroy",
    "xd_store_info", "xd_align_batch", "xd_align_batch_noalloc", "xd_batch_scratch_bytes",
    "xd_align_batch_persistent",
    "xd_align_pairs",
    "xd_banded_batch", "xd_banded_traceback", "xd_find_overlaps", "xd_find_overlaps_strands",
    "xd_plan_create",
    "xd_plan_launch", "xd_plan_destroy", "xd_profile_enable", "xd_profile_read",
    "xd_server_request_bytes", "xd_server_fixed_bytes", "xd_server_create", "xd_server_submit", "xd_server_poll",
    "xd_server_cancel", "xd_server_stats", "xd_server_destroy", "xd_last_error",
    "xd_release_memory",
)


class Tuning(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int32), ("group_steps", ctypes.c_int32),
                ("order", ctypes.c_int32), ("x_tier1", ctypes.c_int32),
                ("x_tier2", ctypes.c_int32), ("band_blocks", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("slots", ctypes.c_int32),
                ("max_batch_tasks", ctypes.c_int32), ("max_pending", ctypes.c_int32),
                ("k", ctypes.c_int32), ("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap", ctypes.c_int32), ("tuning", Tuning)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("batch", ctypes.c_uint64),
                ("batch_tasks", ctypes.c_uint64)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("tasks", ctypes.c_uint64), ("cells", ctypes.c_uint64),
                ("peak_inflight_bytes", ctypes.c_uint64), ("peak_busy_slots", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("busy_s", ctypes.c_double),
                ("pending", ctypes.c_uint64), ("inflight_bytes", ctypes.c_uint64)]


class OverlapCounts(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "kmers", "bloom_repeats", "table_keys", "table_slots", "non_singletons", "retained",
        "occurrences", "seeds", "pairs")]


class Profile(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("extensions", ctypes.c_uint64),
                ("to_tier2", ctypes.c_uint64), ("to_tier3", ctypes.c_uint64),
                ("to_tier4", ctypes.c_uint64), ("to_tier5", ctypes.c_uint64),
                ("to_band", ctypes.c_uint64),
                ("ms_tier1", ctypes.c_double), ("ms_wide", ctypes.c_double),
                ("ms_combine", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("resumed", ctypes.c_uint64)]


class XdropError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libxdrop error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("%s is not built (run __graft_entry__.build() or "
                          "python -m paper_2001_10049_amd.build)" % os.path.basename(LIB_PATH))
    try:
        # torch's HIP runtime is loaded first so that the library binds to the
        # same instance; a process whose first HIP runtime came in with the
        # library found no GPU through torch afterwards
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    lib.xd_pack_reads.argtypes = [vp, vp, vp, u32, vp, vp, ctypes.POINTER(u64)]
    lib.xd_pack_reads.restype = ctypes.c_int
    lib.xd_store_create.argtypes = [vp, u64, vp, vp, u32, ctypes.POINTER(vp)]
    lib.xd_store_create.restype = ctypes.c_int
    lib.xd_store_create_from_codes.argtypes = [vp, vp, vp, u32, ctypes.POINTER(vp)]
    lib.xd_store_create_from_codes.restype = ctypes.c_int
    lib.xd_store_destroy.argtypes = [vp]
    lib.xd_store_destroy.restype = None
    lib.xd_store_info.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u32),
                                  ctypes.POINTER(u32)]
    lib.xd_store_info.restype = ctypes.c_int
    lib.xd_align_batch.argtypes = [vp, vp, vp, vp, i32, u64, i32, i32, i32, i32, vp, vp, vp,
                                   vp, vp, vp]
    lib.xd_align_batch.restype = ctypes.c_int
    lib.xd_align_batch_noalloc.argtypes = lib.xd_align_batch.argtypes
    lib.xd_align_batch_noalloc.restype = ctypes.c_int
    batch = [vp, vp, vp, vp, i32, u64, i32, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.xd_align_batch_persistent.argtypes = batch + [ctypes.POINTER(Tuning), vp]
    lib.xd_align_batch_persistent.restype = ctypes.c_int
    lib.xd_align_pairs.argtypes = [vp, u64, vp, vp, vp, vp, u64, vp, i32, i32, i32, i32, i32,
                                   i32, i32, vp, vp, vp, vp, vp, vp, vp,
                                   ctypes.POINTER(Tuning), vp]
    lib.xd_align_pairs.restype = ctypes.c_int
    lib.xd_banded_batch.argtypes = [vp, vp, vp, vp, i32, u64, i32, i32, i32, i32, vp, vp, vp,
                                    vp, vp]
    lib.xd_banded_batch.restype = ctypes.c_int
    lib.xd_banded_traceback.argtypes = [vp, vp, vp, vp, i32, u64, i32, i32, i32, i32, u32, u64,
                                        vp, vp, vp, vp, vp, vp, vp, vp]
    lib.xd_banded_traceback.restype = ctypes.c_int
    lib.xd_find_overlaps.argtypes = [vp, i32, u32, u32, u64, u64, vp, vp, u64, vp,
                                     ctypes.POINTER(OverlapCounts), vp]
    lib.xd_find_overlaps.restype = ctypes.c_int
    lib.xd_find_overlaps_strands.argtypes = [vp, i32, u32, u32, u64, i32, u64, vp, vp, vp, u64,
                                             vp, ctypes.POINTER(OverlapCounts), vp]
    lib.xd_find_overlaps_strands.restype = ctypes.c_int
    lib.xd_plan_create.argtypes = batch + [ctypes.POINTER(Tuning), ctypes.POINTER(vp)]
    lib.xd_plan_create.restype = ctypes.c_int
    lib.xd_plan_launch.argtypes = [vp, vp]
    lib.xd_plan_launch.restype = ctypes.c_int
    lib.xd_plan_destroy.argtypes = [vp]
    lib.xd_plan_destroy.restype = None
    lib.xd_batch_scratch_bytes.argtypes = [vp, u64, ctypes.POINTER(Tuning)]
    lib.xd_batch_scratch_bytes.restype = u64
    lib.xd_server_request_bytes.argtypes = [u64]
    lib.xd_server_request_bytes.restype = u64
    lib.xd_server_fixed_bytes.argtypes = [vp, ctypes.POINTER(ServerConfig)]
    lib.xd_server_fixed_bytes.restype = u64
    lib.xd_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.xd_server_create.restype = ctypes.c_int
    lib.xd_server_submit.argtypes = [vp, vp, vp, vp, i32, u64, ctypes.POINTER(u64)]
    lib.xd_server_submit.restype = ctypes.c_int
    lib.xd_server_poll.argtypes = [vp, u64, i32, vp, vp, vp, vp, vp, ctypes.POINTER(RequestInfo)]
    lib.xd_server_poll.restype = ctypes.c_int
    lib.xd_server_cancel.argtypes = [vp, u64]
    lib.xd_server_cancel.restype = ctypes.c_int
    lib.xd_server_stats.argtypes = [vp, ctypes.POINTER(ServerCounters)]
    lib.xd_server_stats.restype = ctypes.c_int
    lib.xd_server_destroy.argtypes = [vp]
    lib.xd_server_destroy.restype = None
    lib.xd_profile_enable.argtypes = [ctypes.c_int]
    lib.xd_profile_enable.restype = ctypes.c_int
    lib.xd_profile_read.argtypes = [ctypes.POINTER(Profile), ctypes.c_int]
    lib.xd_profile_read.restype = ctypes.c_int
    lib.xd_release_memory.argtypes = []
    lib.xd_release_memory.restype = ctypes.c_int
    lib.xd_last_error.argtypes = []
    lib.xd_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(rc: int) -> int:
    if rc < 0:
        raise XdropError(rc, load().xd_last_error().decode(errors="replace"))
    return rc
