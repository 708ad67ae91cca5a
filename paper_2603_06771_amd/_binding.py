"""ctypes binding of libsfcoct.so (the C ABI declared in include/sfcoct.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and the stream
(torch.cuda.current_stream()).  There is no CPU fallback: if the library is
missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfcoct.so")

SFC_OK, SFC_EINVAL, SFC_EWORKSPACE, SFC_ECAPACITY, SFC_EHIP, SFC_ENOTSUP = 0, -1, -2, -3, -4, -5
MORTON, HILBERT = 0, 1
SPHERE, CIRCLE, CUBE, SQUARE = 0, 1, 2, 3
REUSE_COUNTS, NO_PRUNE, QUERIES_ORDERED, RECORD_HITS = 1, 2, 4, 8
STAGE_64, STAGE_256 = 16, 32
STAGE_FLAGS = {64: STAGE_64, 128: 0, 256: STAGE_256}

# every exported symbol of include/sfcoct.h
EXPORTS = ("encode_sfc", "octree_bytes", "build_linear_octree", "radius_search", "knn_search",
           "octree_batch_layout", "build_linear_octree_batched", "radius_search_batched", "knn_search_batched",
           "radius_search_struct", "knn_locality", "gather_points", "radius_search_check",
           "radius_search_noalloc", "octree_batch_compact", "sfc_last_error", "sfc_version")

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
U32 = ctypes.c_uint32
U64 = ctypes.c_uint64
SZ = ctypes.c_size_t
F32 = ctypes.c_float


class SfcFrame(ctypes.Structure):
    _fields_ = [("lo", F32 * 3), ("scale", F32), ("bits", I32), ("curve", I32)]


class SfcTreeInfo(ctypes.Structure):
    _fields_ = [("n_points", I64), ("n_internal", I64), ("n_leaves", I64), ("n_nodes", I64),
                ("depth", I32), ("status", I32), ("level_nodes_off", I64 * 23)]


class SfcOctree(ctypes.Structure):
    _fields_ = [
        ("n", I64), ("max_nodes", I64), ("max_leaves", I64),
        ("bits", I32), ("curve", I32), ("leaf_size", U32), ("reserved", U32),
        ("frame", P), ("points", P), ("keys", P), ("perm", P), ("leaves", P), ("counts", P),
        ("nodes", P), ("child", P), ("node_key", P), ("node_level", P), ("info", P),
    ]


class SfcCloud(ctypes.Structure):
    _fields_ = [
        ("offset", I64), ("n", I64), ("curve", I32), ("bits", I32), ("leaf_size", U32), ("kernel", I32),
        ("r", F32), ("k", I32), ("q_offset", I64), ("nq", I64), ("stage", U32), ("record", U32),
        ("tree", SfcOctree),
    ]


class SfcError(RuntimeError):
    pass


class SfcCapacityError(SfcError):
    """The neighbour total exceeds the output capacity; nothing was written.
    `total` is the capacity a second call needs."""

    def __init__(self, msg: str, total: int):
        super().__init__(msg)
        self.total = int(total)


_lib = None


def load(path: str = LIB_PATH):
    """Load the library once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise SfcError(f"{path} not found: build it with `python -m paper_2603_06771_amd.build`")
    L = ctypes.CDLL(path)
    L.encode_sfc.argtypes = [P, I64, I32, I32, P, P, P, ctypes.POINTER(SZ), P]
    L.octree_bytes.argtypes = [I64, U32, I32, ctypes.POINTER(SZ)]
    L.build_linear_octree.argtypes = [P, I64, I32, I32, U32, P, SZ, ctypes.POINTER(SfcOctree), P,
                                      ctypes.POINTER(SZ), P]
    L.radius_search.argtypes = [ctypes.POINTER(SfcOctree), P, I64, I32, F32, P, P, P, U64, U32, P,
                                ctypes.POINTER(SZ), P]
    L.knn_search.argtypes = [ctypes.POINTER(SfcOctree), P, I64, I32, P, P, P, ctypes.POINTER(SZ), P]
    CL = ctypes.POINTER(SfcCloud)
    L.octree_batch_layout.argtypes = [I32, CL, P, ctypes.POINTER(SZ)]
    L.build_linear_octree_batched.argtypes = [P, I32, CL, P, ctypes.POINTER(SZ), P]
    L.radius_search_batched.argtypes = [I32, CL, P, I64, P, P, P, U64, U32, P, ctypes.POINTER(SZ), P]
    L.knn_search_batched.argtypes = [I32, CL, P, I64, I32, P, P, P, ctypes.POINTER(SZ), P]
    L.gather_points.argtypes = [P, I64, P, I64, P, P]
    L.radius_search_struct.argtypes = [ctypes.POINTER(SfcOctree), P, I64, I32, F32, P, P, P, U64, P, P, P, U64, U32,
                                       P, ctypes.POINTER(SZ), P]
    L.knn_locality.argtypes = [ctypes.POINTER(SfcOctree), P, I64, P, I32, I32, P, P, P, ctypes.POINTER(SZ), P]
    L.radius_search_check.argtypes = [P, I64, U64, ctypes.POINTER(U64), P]
    L.octree_batch_compact.argtypes = [I32, ctypes.POINTER(SfcCloud), P, ctypes.POINTER(SZ), ctypes.POINTER(SfcCloud),
                                       P]
    L.radius_search_noalloc.argtypes = [ctypes.POINTER(SfcOctree), P, I64, I32, F32, P, P, P, U64, U32, P]
    L.sfc_last_error.restype = ctypes.c_char_p
    L.sfc_version.restype = ctypes.c_char_p
    for name in EXPORTS[:-2]:
        getattr(L, name).restype = I32
    _lib = L
    return L


def check_capacity(offsets, nq: int, capacity: int, stream, what: str) -> int:
    """radius_search_check on a device offsets array: returns the neighbour
    total, raises SfcCapacityError when it exceeds `capacity`."""
    total = U64(0)
    rc = load().radius_search_check(ctypes.c_void_p(offsets.data_ptr()), int(nq), int(capacity), ctypes.byref(total),
                                    stream)
    if rc == SFC_ECAPACITY:
        raise SfcCapacityError(f"{what}: {load().sfc_last_error().decode(errors='replace')}", total.value)
    check(rc, what)
    return int(total.value)


def check(rc: int, what: str) -> None:
    if rc != SFC_OK:
        msg = load().sfc_last_error().decode(errors="replace")
        raise SfcError(f"{what} failed with status {rc}: {msg}")
