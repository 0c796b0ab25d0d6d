"""ctypes view of the C ABI in include/d2.h (structs, enums, prototypes).

Loads the in-tree ``libd2.so``.  There is no fallback of any kind: if the
library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libd2.so")

D2_OK, D2_EINVAL, D2_EWORKSPACE, D2_EUNSUPPORTED, D2_EHIP, D2_ENOMEM, D2_ESCRATCH = range(7)
D2_NOALLOC_SCRATCH_BYTES = 32 << 20
D2_F64, D2_F32 = 0, 1
D2_COST_F64_DIRECT, D2_COST_BF16_MFMA = 0, 1
D2_INIT_AUTO, D2_INIT_NWC, D2_INIT_VOGEL, D2_INIT_LCM = 0, 1, 2, 3
D2_SCHED_AUTO, D2_SCHED_PLAIN = 0, 1
D2_FLAG_EAGER = 1
(D2_PAIR_OK, D2_PAIR_BAD_WEIGHTS, D2_PAIR_TOO_LARGE, D2_PAIR_PIVOT_CAP, D2_PAIR_BAD_POINTS,
 D2_PAIR_UNLABELLED, D2_PAIR_INTERNAL) = range(7)
(WHICH_COST_TILES, WHICH_EMD_BATCH, WHICH_ASSIGN, WHICH_PAIRWISE, WHICH_UPDATE, WHICH_MULTI,
 WHICH_UPDATE_FREE, WHICH_MERGE) = range(8)

# Every function the header declares (checked against the header by the tests).
EXPORTS = ["d2_create", "d2_destroy", "d2_status_string", "d2_max_support", "d2_version",
           "d2_workspace_bytes", "d2_cost_tiles", "d2_emd_batch", "d2_assign", "d2_pairwise",
           "d2_tune_pairwise", "d2_centroid_update", "d2_emd_cost_batch",
           "d2_assign_multi", "d2_assign_segmented", "d2_assign_noalloc",
           "d2_centroid_update_free", "d2_merge_level", "d2_emd_batch_basis"]


class d2_set(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("offsets", ctypes.c_void_p), ("points", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("max_support", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class d2_opts(ctypes.Structure):
    _fields_ = [("cost_mode", ctypes.c_int32), ("init", ctypes.c_int32),
                ("max_pivots", ctypes.c_int32), ("want_sqrt", ctypes.c_int32),
                ("opt_tol", ctypes.c_double), ("schedule", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("bland_after", ctypes.c_int32)]


class LibraryMissing(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded libd2.so (raises LibraryMissing when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    P, S = ctypes.c_void_p, ctypes.POINTER(d2_set)
    O = ctypes.POINTER(d2_opts)
    I64, I32, SZ = ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    L.d2_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    L.d2_destroy.argtypes = [P]
    L.d2_status_string.argtypes = [ctypes.c_int]
    L.d2_status_string.restype = ctypes.c_char_p
    L.d2_max_support.argtypes = []
    L.d2_version.argtypes = []
    L.d2_version.restype = ctypes.c_char_p
    L.d2_workspace_bytes.argtypes = [P, ctypes.c_int, S, S, I64, O]
    L.d2_workspace_bytes.restype = SZ
    L.d2_cost_tiles.argtypes = [P, S, S, P, I64, I32, P, P, P, SZ, P]
    L.d2_emd_batch.argtypes = [P, S, S, P, I64, O, P, P, P, P, P, P, P, P, SZ, P]
    L.d2_assign.argtypes = [P, S, S, O, P, P, P, P, P, SZ, P]
    L.d2_assign_noalloc.argtypes = [P, S, S, O, P, P, P, P, P]
    L.d2_pairwise.argtypes = [P, S, O, P, P, P, SZ, P]
    L.d2_tune_pairwise.argtypes = [P, S, O, P, P, P, SZ, P, ctypes.POINTER(ctypes.c_double)]
    L.d2_centroid_update.argtypes = [P, S, S, P, P, O, P, P, P, P, P, P, SZ, P]
    L.d2_centroid_update_free.argtypes = [P, S, S, P, P, I32, O, P, P, P, P, P, P, P, P, P, I64, P, SZ, P]
    L.d2_emd_batch_basis.argtypes = [P, S, S, P, I64, O, P, P, P, P, P, P]
    L.d2_merge_level.argtypes = [P, S, I64, P, P, I64, P, P, P, P, P, P, P, SZ, P]
    L.d2_assign_segmented.argtypes = [P, S, S, P, I64, P, O, P, P, P, P]
    L.d2_assign_multi.argtypes = [P, I32, S, S, O, P, P, P, P, P, SZ, P]
    L.d2_emd_cost_batch.argtypes = [P, I64, P, P, P, P, P, P, I32, I32, O, P, P, P, P, P, SZ, P]
    for name in ("d2_create", "d2_destroy", "d2_cost_tiles", "d2_emd_batch", "d2_assign",
                 "d2_pairwise", "d2_max_support", "d2_tune_pairwise", "d2_centroid_update",
                 "d2_emd_cost_batch", "d2_assign_multi", "d2_assign_segmented",
                 "d2_assign_noalloc", "d2_centroid_update_free", "d2_merge_level",
                 "d2_emd_batch_basis"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class D2Error(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().d2_status_string(code).decode()
        super().__init__(f"{where}: {msg} (status {code})")


def check(code: int, where: str):
    if code != D2_OK:
        raise D2Error(code, where)
