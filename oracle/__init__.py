"""Plain CPU reference (the oracle) for the SFC / linear-octree / search path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the GPU library
never does and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, fp32 expressions evaluated as
written with contraction off); this module marshals numpy arrays through
ctypes, and computes the kNN locality histogram (integer counting and fp64
moments) in numpy.  Each function names the part of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MORTON, HILBERT = 0, 1
SPHERE, CIRCLE, CUBE, SQUARE = 0, 1, 2, 3
KERNELS = {"sphere": SPHERE, "circle": CIRCLE, "cube": CUBE, "square": SQUARE}
CURVES = {"morton": MORTON, "hilbert": HILBERT}

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int
F32 = ctypes.c_float
F64 = ctypes.c_double
U32 = ctypes.c_uint32
U64 = ctypes.c_uint64


class _Tree(ctypes.Structure):
    _fields_ = [
        ("n_leaves", I64), ("n_internal", I64), ("n_nodes", I64),
        ("leaves", P), ("counts", P), ("node_start", P), ("node_level", P),
        ("node_begin", P), ("node_end", P), ("node_child", P), ("node_box", P),
    ]


def _declare(L):
    L.or_set_threads.argtypes = [I32]
    L.or_get_threads.restype = I32
    L.or_frame.argtypes = [P, I64, I32, P, P]
    L.or_cell.argtypes = [F32, F32, F32, I32]
    L.or_cell.restype = U32
    L.or_morton_encode.argtypes = [U32, U32, U32, I32]
    L.or_morton_encode.restype = U64
    L.or_morton_decode.argtypes = [U64, I32, P]
    L.or_hilbert_encode.argtypes = [U32, U32, U32, I32]
    L.or_hilbert_encode.restype = U64
    L.or_hilbert_decode.argtypes = [U64, I32, P]
    L.or_encode.argtypes = [P, I64, I32, I32, P, P, P]
    L.or_sort.argtypes = [P, I64, P, P]
    L.or_build_tree.argtypes = [P, P, P, I64, I32, U32]
    L.or_build_tree.restype = ctypes.POINTER(_Tree)
    L.or_tree_free.argtypes = [ctypes.POINTER(_Tree)]
    L.or_kernel_test.argtypes = [I32, P, P, F32]
    L.or_kernel_test.restype = I32
    L.or_dist2.argtypes = [P, P]
    L.or_dist2.restype = F32
    L.or_grid_build.argtypes = [P, I64, F64, I32]
    L.or_grid_build.restype = P
    L.or_grid_free.argtypes = [P]
    L.or_grid_radius_count.argtypes = [P, P, I64, I32, F32, P]
    L.or_grid_radius_fill.argtypes = [P, P, I64, I32, F32, P, P]
    L.or_grid_knn.argtypes = [P, P, I64, I32, P, P]


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _xyz(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("expected an (n, 3) float32 array")
    return a


def set_threads(t: int) -> None:
    lib().or_set_threads(int(t))


def get_threads() -> int:
    return int(lib().or_get_threads())


# --- Section 4: frame, discretisation, Morton (4.1) and Hilbert (4.2) codes ---

def frame(xyz, bits: int = 21):
    xyz = _xyz(xyz)
    lo = np.zeros(3, np.float32)
    s = np.zeros(1, np.float32)
    lib().or_frame(_p(xyz), xyz.shape[0], bits, _p(lo), _p(s))
    return lo, np.float32(s[0])


def cell(x: float, lo: float, s: float, bits: int) -> int:
    return int(lib().or_cell(float(np.float32(x)), float(np.float32(lo)), float(np.float32(s)), bits))


def morton_encode(x: int, y: int, z: int, bits: int) -> int:
    return int(lib().or_morton_encode(x, y, z, bits))


def morton_decode(key: int, bits: int):
    out = np.zeros(3, np.uint32)
    lib().or_morton_decode(key, bits, _p(out))
    return tuple(int(v) for v in out)


def hilbert_encode(x: int, y: int, z: int, bits: int) -> int:
    return int(lib().or_hilbert_encode(x, y, z, bits))


def hilbert_decode(key: int, bits: int):
    out = np.zeros(3, np.uint32)
    lib().or_hilbert_decode(key, bits, _p(out))
    return tuple(int(v) for v in out)


def encode(xyz, curve="morton", bits: int = 21):
    """Codes of every point (Section 4, reorder step 1). Returns (keys, lo, scale)."""
    xyz = _xyz(xyz)
    c = CURVES[curve] if isinstance(curve, str) else int(curve)
    keys = np.zeros(xyz.shape[0], np.uint64)
    lo = np.zeros(3, np.float32)
    s = np.zeros(1, np.float32)
    lib().or_encode(_p(xyz), xyz.shape[0], c, bits, _p(lo), _p(s), _p(keys))
    return keys, lo, np.float32(s[0])


def sort(keys):
    """Ascending codes, ties by original index (Section 4, reorder step 2)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    ks = np.zeros_like(keys)
    perm = np.zeros(keys.shape[0], np.uint32)
    lib().or_sort(_p(keys), keys.shape[0], _p(ks), _p(perm))
    return ks, perm


# --- Section 5.1: linear octree -----------------------------------------------

def build_tree(xyz, keys_sorted, perm, bits: int = 21, max_leaf: int = 32) -> dict:
    """leaves / counts by the iterative refinement, plus every node's
    (level, start code, point range, first child, tight box), nodes ordered by
    (level, start code)."""
    xyz = _xyz(xyz)
    ks = np.ascontiguousarray(keys_sorted, dtype=np.uint64)
    pm = np.ascontiguousarray(perm, dtype=np.uint32)
    tp = lib().or_build_tree(_p(xyz), _p(ks), _p(pm), xyz.shape[0], bits, max_leaf)
    t = tp.contents
    nl, nn = t.n_leaves, t.n_nodes

    def arr(ptr, ctype, count, dtype):
        if count == 0:
            return np.zeros(0, dtype)
        buf = ctypes.cast(ptr, ctypes.POINTER(ctype * count)).contents
        return np.frombuffer(buf, dtype=dtype).copy()

    out = {
        "n_leaves": int(nl), "n_internal": int(t.n_internal), "n_nodes": int(nn),
        "leaves": arr(t.leaves, ctypes.c_uint64, nl + 1, np.uint64),
        "counts": arr(t.counts, ctypes.c_uint32, nl, np.uint32),
        "node_start": arr(t.node_start, ctypes.c_uint64, nn, np.uint64),
        "node_level": arr(t.node_level, ctypes.c_int32, nn, np.int32),
        "node_begin": arr(t.node_begin, ctypes.c_int64, nn, np.int64),
        "node_end": arr(t.node_end, ctypes.c_int64, nn, np.int64),
        "node_child": arr(t.node_child, ctypes.c_int64, nn, np.int64),
        "node_box": arr(t.node_box, ctypes.c_float, 6 * nn, np.float32).reshape(nn, 6),
    }
    lib().or_tree_free(tp)
    return out


# --- Section 3.2 / 3.3: kernels, distance, grid searches ----------------------

def kernel_test(kernel, p, c, r) -> bool:
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    p = np.ascontiguousarray(p, np.float32)
    c = np.ascontiguousarray(c, np.float32)
    return bool(lib().or_kernel_test(k, _p(p), _p(c), float(np.float32(r))))


class Grid:
    """The oracle's uniform grid over a cloud (cell side h, 2 or 3 gridded axes)."""

    def __init__(self, xyz, h: float, dims: int = 3):
        self.xyz = _xyz(xyz)  # kept alive: the C side points into it
        self.h = float(h)
        self.dims = int(dims)
        self.ptr = lib().or_grid_build(_p(self.xyz), self.xyz.shape[0], self.h, self.dims)

    def __del__(self):
        try:
            if self.ptr:
                lib().or_grid_free(self.ptr)
                self.ptr = None
        except Exception:
            pass

    def radius_count(self, queries, kernel, r) -> np.ndarray:
        q = _xyz(queries)
        k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        counts = np.zeros(q.shape[0], np.uint32)
        lib().or_grid_radius_count(self.ptr, _p(q), q.shape[0], k, float(np.float32(r)), _p(counts))
        return counts

    def radius_search(self, queries, kernel, r):
        """CSR (counts, offsets[nq+1], indices) with each row ascending."""
        q = _xyz(queries)
        k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        counts = self.radius_count(q, k, r)
        offsets = np.zeros(q.shape[0] + 1, np.int64)
        np.cumsum(counts, out=offsets[1:])
        indices = np.zeros(int(offsets[-1]), np.uint32)
        lib().or_grid_radius_fill(self.ptr, _p(q), q.shape[0], k, float(np.float32(r)),
                                  _p(offsets), _p(indices))
        return counts, offsets, indices

    def knn(self, queries, k: int):
        q = _xyz(queries)
        idx = np.zeros((q.shape[0], k), np.uint32)
        d2 = np.zeros((q.shape[0], k), np.float32)
        lib().or_grid_knn(self.ptr, _p(q), q.shape[0], int(k), _p(idx), _p(d2))
        return idx, d2


def radius_search(xyz, queries, kernel, r):
    """Grid oracle for fixed-radius search; cell side r (xy cells for the 2D kernels)."""
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    dims = 2 if k in (CIRCLE, SQUARE) else 3
    h = float(r) if r > 0 else 1.0
    return Grid(xyz, h, dims).radius_search(queries, k, r)


def knn(xyz, queries, k: int, h: float | None = None):
    """Grid oracle for k nearest neighbours (ties by index, padded with
    (0xFFFFFFFF, +inf) when k exceeds the cloud)."""
    xyz = _xyz(xyz)
    if h is None:
        n = max(xyz.shape[0], 1)
        ext = float(np.max(xyz.max(0) - xyz.min(0))) if xyz.shape[0] else 1.0
        h = max(ext * (k / n) ** (1.0 / 3.0), ext / 1024.0, 1e-6)
    return Grid(xyz, h, 3).knn(queries, k)


def locality_histogram(perm, knn_idx, rows=None):
    """Section 5.2, the kNN locality histogram: H_k(d) counts the pairs (i, j)
    with j among the k nearest neighbours of the point stored at position i
    and |i - j| = d, positions in the stored (sorted) order.

    perm[i] is the original index of the point at position i; knn_idx[r] holds
    the original indices of the neighbours of the query at position rows[r]
    (rows = 0 .. len(knn_idx) - 1 when None); 0xFFFFFFFF entries (k beyond the
    cloud) are skipped.  Returns (H, stats): H int64 of length n; stats total,
    mean, std, g1 (Fisher-Pearson skewness E[((d - mean) / std)^3]), q1 / q2 /
    q3 (smallest d whose cumulative count reaches 1/4, 1/2, 3/4 of the total)
    and max, in fp64."""
    perm = np.asarray(perm).astype(np.int64)
    n = perm.size
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    idx = np.asarray(knn_idx).astype(np.int64)
    rows = np.arange(idx.shape[0], dtype=np.int64) if rows is None else np.asarray(rows).astype(np.int64)
    valid = idx != 0xFFFFFFFF
    d = np.abs(rows[:, None] - pos[np.where(valid, idx, 0)])[valid]
    H = np.bincount(d, minlength=n).astype(np.int64)
    total = int(H.sum())
    dv = np.arange(n, dtype=np.float64)
    stats = {"total": float(total), "mean": 0.0, "std": 0.0, "g1": 0.0, "q1": 0.0, "q2": 0.0, "q3": 0.0,
             "max": float(d.max()) if d.size else 0.0}
    if total:
        mean = float((H * dv).sum() / total)
        var = float((H * (dv - mean) ** 2).sum() / total)
        std = var ** 0.5
        stats["mean"], stats["std"] = mean, std
        stats["g1"] = float((H * ((dv - mean) / std) ** 3).sum() / total) if std > 0 else 0.0
        cum = np.cumsum(H)
        for name, q in (("q1", 1), ("q2", 2), ("q3", 3)):
            stats[name] = float(np.searchsorted(cum, (q * total + 3) // 4))
    return H, stats
