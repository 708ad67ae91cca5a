"""MI355X (gfx950) space-filling-curve reordering, linear octrees and
neighbourhood search for 3D point clouds (arXiv 2603.06771).

Thin PyTorch-facing wrappers over the C ABI of libsfcoct.so (include/sfcoct.h):
tensors provide device memory, torch's current stream provides ordering.  All
computation runs in the library's HIP kernels; nothing here falls back to the
CPU.  Importing the package does not load the library; the first call does.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _binding as B

__all__ = ["encode_sfc", "build_linear_octree", "radius_search", "radius_count", "radius_fill", "knn_search", "Octree",
           "Batch", "build_batch", "radius_search_batched", "knn_search_batched", "knn_locality", "choose_curve",
           "radius_search_struct", "SfcError", "SfcCapacityError",
           "CURVES", "KERNELS", "library_path"]

CURVES = {"morton": B.MORTON, "hilbert": B.HILBERT}
KERNELS = {"sphere": B.SPHERE, "circle": B.CIRCLE, "cube": B.CUBE, "square": B.SQUARE}
library_path = B.LIB_PATH
SfcError = B.SfcError
SfcCapacityError = B.SfcCapacityError


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise B.SfcError("no GPU visible: the sfcoct library runs on MI355X only")
    return torch


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _xyz(torch, xyz):
    if not (xyz.is_cuda and xyz.dtype == torch.float32 and xyz.dim() == 2 and xyz.shape[1] == 3):
        raise ValueError("expected a CUDA float32 tensor of shape (n, 3)")
    return xyz.contiguous()


def _ws(torch, nbytes: int):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


def _code(table, v):
    return table[v] if isinstance(v, str) else int(v)


def encode_sfc(xyz, curve="morton", bits: int = 21):
    """Section 4: frame and codes of every point.  Returns (keys int64 tensor
    holding the uint64 codes, frame as a host SfcFrame)."""
    torch = _torch()
    L = B.load()
    xyz = _xyz(torch, xyz)
    n = xyz.shape[0]
    keys = torch.empty(n, dtype=torch.int64, device="cuda")
    frame = torch.empty(ctypes.sizeof(B.SfcFrame), dtype=torch.uint8, device="cuda")
    need = ctypes.c_size_t(0)
    B.check(L.encode_sfc(_ptr(xyz), n, _code(CURVES, curve), bits, _ptr(frame), _ptr(keys), None,
                         ctypes.byref(need), None), "encode_sfc(size)")
    ws = _ws(torch, need.value)
    B.check(L.encode_sfc(_ptr(xyz), n, _code(CURVES, curve), bits, _ptr(frame), _ptr(keys), _ptr(ws),
                         ctypes.byref(need), _stream(torch)), "encode_sfc")
    return keys, frame


@dataclass
class Octree:
    """A built linear octree: `mem` owns the device memory, `view` is the C
    struct of device pointers into it."""
    mem: object
    view: B.SfcOctree
    curve: int
    bits: int
    leaf_size: int
    n: int

    def _slice(self, ptr, count, dtype, elem):
        off = ptr - self.mem.data_ptr()
        return self.mem[off:off + count * elem].view(dtype)

    def info(self) -> dict:
        torch = _torch()
        raw = self._slice(self.view.info, ctypes.sizeof(B.SfcTreeInfo), torch.uint8, 1).cpu().numpy()
        st = B.SfcTreeInfo.from_buffer_copy(raw.tobytes())
        return {"n_points": st.n_points, "n_internal": st.n_internal, "n_leaves": st.n_leaves,
                "n_nodes": st.n_nodes, "depth": st.depth, "status": st.status,
                "level_nodes_off": list(st.level_nodes_off)}

    def frame(self) -> B.SfcFrame:
        torch = _torch()
        raw = self._slice(self.view.frame, ctypes.sizeof(B.SfcFrame), torch.uint8, 1).cpu().numpy()
        return B.SfcFrame.from_buffer_copy(raw.tobytes())

    # views (tensors sharing the tree memory); counts from info()
    def points(self):
        torch = _torch()
        return self._slice(self.view.points, 4 * self.n, torch.float32, 4).view(self.n, 4)

    def keys(self):
        torch = _torch()
        return self._slice(self.view.keys, self.n, torch.int64, 8)

    def perm(self):
        torch = _torch()
        return self._slice(self.view.perm, self.n, torch.int32, 4)

    def arrays(self, info: dict | None = None) -> dict:
        """leaves / counts / nodes / child / node_key / node_level sized by info()."""
        torch = _torch()
        info = info or self.info()
        nl, nn = info["n_leaves"], info["n_nodes"]
        v = self.view
        return {
            "leaves": self._slice(v.leaves, nl + 1, torch.int64, 8),
            "counts": self._slice(v.counts, nl, torch.int32, 4),
            "nodes": self._slice(v.nodes, 8 * nn, torch.float32, 4).view(nn, 8),
            "child": self._slice(v.child, nn, torch.int32, 4),
            "node_key": self._slice(v.node_key, nn, torch.int64, 8),
            "node_level": self._slice(v.node_level, nn, torch.uint8, 1),
        }


def build_linear_octree(xyz, curve="morton", bits: int = 21, leaf_size: int = 32) -> Octree:
    """Sections 4 and 5.1: encode, sort, reorder and build the complete linear
    octree (split while a node holds more than leaf_size points)."""
    torch = _torch()
    L = B.load()
    xyz = _xyz(torch, xyz)
    n = xyz.shape[0]
    c = _code(CURVES, curve)
    tb = ctypes.c_size_t(0)
    B.check(L.octree_bytes(n, leaf_size, bits, ctypes.byref(tb)), "octree_bytes")
    mem = torch.empty(tb.value, dtype=torch.uint8, device="cuda")
    need = ctypes.c_size_t(0)
    view = B.SfcOctree()
    B.check(L.build_linear_octree(_ptr(xyz), n, c, bits, leaf_size, _ptr(mem), tb.value, ctypes.byref(view),
                                  None, ctypes.byref(need), None), "build_linear_octree(size)")
    ws = _ws(torch, need.value)
    B.check(L.build_linear_octree(_ptr(xyz), n, c, bits, leaf_size, _ptr(mem), tb.value, ctypes.byref(view),
                                  _ptr(ws), ctypes.byref(need), _stream(torch)), "build_linear_octree")
    return Octree(mem=mem, view=view, curve=c, bits=bits, leaf_size=leaf_size, n=n)


def _stage_flag(stage) -> int:
    try:
        return B.STAGE_FLAGS[int(stage)]
    except (KeyError, TypeError, ValueError):
        raise ValueError(f"stage must be 64, 128 or 256, not {stage!r}") from None


def radius_search(tree: Octree, queries=None, kernel="sphere", r: float = 1.0, capacity: int | None = None,
                  prune: bool = True, record: bool = False, check: bool = True, stage: int = 128):
    """Section 3.2 / 5.1: CSR (counts int32, offsets int64 [nq+1], indices
    int32 original point indices).  queries=None searches around every cloud
    point, rows in sorted (curve) order.  Without a capacity the count pass
    runs first and the host reads the total before the fill pass.  With a
    capacity both passes run in one call; then the host waits for the result
    and raises SfcCapacityError (its `total` is the capacity needed) if the
    indices did not fit, unless check=False (no host wait: the caller
    compares offsets[-1] with the capacity itself).  record: the fill writes
    rows from the hits the count pass recorded (same result, larger
    workspace).  stage: the staging tile (points per sweep round: 64, 128
    or 256; same result)."""
    torch = _torch()
    L = B.load()
    if queries is not None:
        queries = _xyz(torch, queries)
        nq = queries.shape[0]
    else:
        nq = tree.n
    k = _code(KERNELS, kernel)
    flags = (0 if prune else B.NO_PRUNE) | (B.RECORD_HITS if record else 0) | _stage_flag(stage)
    counts = torch.empty(nq, dtype=torch.int32, device="cuda")
    offsets = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    need = ctypes.c_size_t(0)
    args = (ctypes.byref(tree.view), _ptr(queries), nq, k, float(r), _ptr(counts), _ptr(offsets))
    B.check(L.radius_search(*args, None, 0, flags, None, ctypes.byref(need), None), "radius_search(size)")
    ws = _ws(torch, need.value)
    stream = _stream(torch)
    if capacity is None:
        B.check(L.radius_search(*args, None, 0, flags, _ptr(ws), ctypes.byref(need), stream), "radius_search(count)")
        total = int(offsets[nq].item())
        indices = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
        B.check(L.radius_search(*args, _ptr(indices), total, flags | B.REUSE_COUNTS, _ptr(ws), ctypes.byref(need),
                                stream), "radius_search(fill)")
        return counts, offsets, indices[:total]
    indices = torch.empty(max(int(capacity), 1), dtype=torch.int32, device="cuda")
    B.check(L.radius_search(*args, _ptr(indices), int(capacity), flags, _ptr(ws), ctypes.byref(need), stream),
            "radius_search")
    if check:
        B.check_capacity(offsets, nq, int(capacity), stream, "radius_search")
    return counts, offsets, indices


def _radius_args(torch, tree, queries, kernel, r, counts, offsets):
    if queries is not None:
        queries = _xyz(torch, queries)
        nq = queries.shape[0]
    else:
        nq = tree.n
    return queries, nq, (ctypes.byref(tree.view), _ptr(queries), nq, _code(KERNELS, kernel), float(r),
                         _ptr(counts), _ptr(offsets))


def _radius_ws(torch, L, args):
    need = ctypes.c_size_t(0)
    B.check(L.radius_search(*args, None, 0, 0, None, ctypes.byref(need), None), "radius_search(size)")
    return _ws(torch, need.value), need


def radius_count(tree: Octree, queries=None, kernel="sphere", r: float = 1.0, prune: bool = True):
    """Count pass only: (counts int32 [nq], offsets int64 [nq + 1]); the
    host does not synchronise."""
    torch = _torch()
    L = B.load()
    nq = tree.n if queries is None else queries.shape[0]
    counts = torch.empty(nq, dtype=torch.int32, device="cuda")
    offsets = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    queries, nq, args = _radius_args(torch, tree, queries, kernel, r, counts, offsets)
    ws, need = _radius_ws(torch, L, args)
    B.check(L.radius_search(*args, None, 0, 0 if prune else B.NO_PRUNE, _ptr(ws), ctypes.byref(need),
                            _stream(torch)), "radius_search(count)")
    return counts, offsets


def radius_fill(tree: Octree, counts, offsets, indices, queries=None, kernel="sphere", r: float = 1.0,
                prune: bool = True):
    """Fill pass only, into `indices` (int32, capacity = its length), using
    counts/offsets from radius_count with the same arguments."""
    torch = _torch()
    L = B.load()
    queries, nq, args = _radius_args(torch, tree, queries, kernel, r, counts, offsets)
    ws, need = _radius_ws(torch, L, args)
    flags = B.REUSE_COUNTS | (0 if prune else B.NO_PRUNE)
    B.check(L.radius_search(*args, _ptr(indices), indices.numel(), flags, _ptr(ws), ctypes.byref(need),
                            _stream(torch)), "radius_search(fill)")
    return indices


def knn_search(tree: Octree, queries=None, k: int = 8):
    """Section 3.3: (idx int32 [nq, k], d2 float32 [nq, k]), each row ascending
    by (d2, index); queries=None uses every cloud point in sorted order."""
    torch = _torch()
    L = B.load()
    if queries is not None:
        queries = _xyz(torch, queries)
        nq = queries.shape[0]
    else:
        nq = tree.n
    idx = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    d2 = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    need = ctypes.c_size_t(0)
    args = (ctypes.byref(tree.view), _ptr(queries), nq, int(k), _ptr(idx), _ptr(d2))
    B.check(L.knn_search(*args, None, ctypes.byref(need), None), "knn_search(size)")
    ws = _ws(torch, need.value)
    B.check(L.knn_search(*args, _ptr(ws), ctypes.byref(need), _stream(torch)), "knn_search")
    return idx, d2


# ---------------------------------------------------------------- batches
def _per_cloud(v, B_, name):
    if isinstance(v, (list, tuple)):
        if len(v) != B_:
            raise ValueError(f"{name}: expected {B_} values, got {len(v)}")
        return list(v)
    return [v] * B_


@dataclass
class Batch:
    """Trees of a batch of independent clouds built in one pass: `mem` owns
    the device memory, `clouds` is the C table (sfc_cloud[B]) with each
    cloud's tree view.  tree(c) gives an Octree view of cloud c that the
    single-cloud calls accept."""
    mem: object
    clouds: object
    sizes: list
    offsets: list

    @property
    def B(self) -> int:
        return len(self.sizes)

    def tree(self, c: int) -> Octree:
        t = self.clouds[c].tree
        return Octree(mem=self.mem, view=t, curve=t.curve, bits=t.bits, leaf_size=t.leaf_size, n=t.n)


def build_batch(xyz, sizes, curve="hilbert", bits=21, leaf_size=32) -> Batch:
    """Sections 4 and 5.1 for a batch: xyz (n_total, 3) holds the clouds one
    after the other (cloud c has sizes[c] points); curve, bits and leaf_size
    are one value or one per cloud.  One launch sequence builds every tree."""
    torch = _torch()
    L = B.load()
    xyz = _xyz(torch, xyz)
    sizes = [int(x) for x in sizes]
    nb = len(sizes)
    if nb < 1 or sum(sizes) != xyz.shape[0]:
        raise ValueError("sizes must be non-empty and sum to the number of points")
    curves = _per_cloud(curve, nb, "curve")
    bitss = _per_cloud(bits, nb, "bits")
    leafs = _per_cloud(leaf_size, nb, "leaf_size")
    clouds = (B.SfcCloud * nb)()
    off = 0
    offsets = []
    for c in range(nb):
        clouds[c].offset = off
        clouds[c].n = sizes[c]
        clouds[c].curve = _code(CURVES, curves[c])
        clouds[c].bits = int(bitss[c])
        clouds[c].leaf_size = int(leafs[c])
        offsets.append(off)
        off += sizes[c]
    tb = ctypes.c_size_t(0)
    B.check(L.octree_batch_layout(nb, clouds, None, ctypes.byref(tb)), "octree_batch_layout(size)")
    mem = torch.empty(tb.value, dtype=torch.uint8, device="cuda")
    B.check(L.octree_batch_layout(nb, clouds, _ptr(mem), ctypes.byref(tb)), "octree_batch_layout")
    need = ctypes.c_size_t(0)
    B.check(L.build_linear_octree_batched(_ptr(xyz), nb, clouds, None, ctypes.byref(need), None),
            "build_linear_octree_batched(size)")
    ws = _ws(torch, need.value)
    B.check(L.build_linear_octree_batched(_ptr(xyz), nb, clouds, _ptr(ws), ctypes.byref(need), _stream(torch)),
            "build_linear_octree_batched")
    return Batch(mem=mem, clouds=clouds, sizes=sizes, offsets=offsets)


def _query_rows(torch, batch, queries, q_sizes):
    """Sets q_offset / nq of every cloud; returns (queries, nq_total)."""
    if queries is None:
        for c in range(batch.B):
            batch.clouds[c].q_offset = batch.offsets[c]
            batch.clouds[c].nq = batch.sizes[c]
        return None, sum(batch.sizes)
    queries = _xyz(torch, queries)
    q_sizes = [int(x) for x in q_sizes]
    if len(q_sizes) != batch.B or sum(q_sizes) != queries.shape[0]:
        raise ValueError("q_sizes must give one query count per cloud, summing to the number of queries")
    off = 0
    for c in range(batch.B):
        batch.clouds[c].q_offset = off
        batch.clouds[c].nq = q_sizes[c]
        off += q_sizes[c]
    return queries, off


def radius_search_batched(batch: Batch, queries=None, q_sizes=None, kernel="sphere", r=1.0,
                          capacity: int | None = None, prune: bool = True, record=False,
                          check: bool = True, stage=128):
    """Radius search of every cloud of the batch (its own kernel and radius)
    in one launch per pass.  One CSR over all rows (cloud c's rows follow
    cloud c - 1's); indices are local to each cloud.  queries=None: every
    cloud's own points, rows in each cloud's sorted order.  capacity, check:
    as for radius_search; record and stage (the staging tile): one value or
    one per cloud."""
    torch = _torch()
    L = B.load()
    kernels = _per_cloud(kernel, batch.B, "kernel")
    radii = _per_cloud(r, batch.B, "r")
    records = _per_cloud(record, batch.B, "record")
    stages = _per_cloud(stage, batch.B, "stage")
    for c in range(batch.B):
        batch.clouds[c].kernel = _code(KERNELS, kernels[c])
        batch.clouds[c].r = float(radii[c])
        _stage_flag(stages[c])
        batch.clouds[c].stage = int(stages[c])
        batch.clouds[c].record = 1 if records[c] else 0
    queries, nq = _query_rows(torch, batch, queries, q_sizes)
    flags = 0 if prune else B.NO_PRUNE
    counts = torch.empty(nq, dtype=torch.int32, device="cuda")
    offsets = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    need = ctypes.c_size_t(0)
    head = (batch.B, batch.clouds, _ptr(queries), nq, _ptr(counts), _ptr(offsets))
    B.check(L.radius_search_batched(*head, None, 0, flags, None, ctypes.byref(need), None),
            "radius_search_batched(size)")
    ws = _ws(torch, need.value)
    stream = _stream(torch)
    if capacity is None:
        B.check(L.radius_search_batched(*head, None, 0, flags, _ptr(ws), ctypes.byref(need), stream),
                "radius_search_batched(count)")
        total = int(offsets[nq].item())
        indices = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
        B.check(L.radius_search_batched(*head, _ptr(indices), total, flags | B.REUSE_COUNTS, _ptr(ws),
                                        ctypes.byref(need), stream), "radius_search_batched(fill)")
        return counts, offsets, indices[:total]
    indices = torch.empty(max(int(capacity), 1), dtype=torch.int32, device="cuda")
    B.check(L.radius_search_batched(*head, _ptr(indices), int(capacity), flags, _ptr(ws), ctypes.byref(need),
                                    stream), "radius_search_batched")
    if check:
        B.check_capacity(offsets, nq, int(capacity), stream, "radius_search_batched")
    return counts, offsets, indices


def knn_search_batched(batch: Batch, queries=None, q_sizes=None, k=8, kstride: int | None = None):
    """k-NN of every cloud of the batch (its own k) in one launch: (idx int32
    [nq, kstride], d2 float32 [nq, kstride]); entries past a cloud's k are
    (-1, +inf)."""
    torch = _torch()
    L = B.load()
    ks = [int(x) for x in _per_cloud(k, batch.B, "k")]
    kstride = int(kstride or max(ks))
    for c in range(batch.B):
        batch.clouds[c].k = ks[c]
    queries, nq = _query_rows(torch, batch, queries, q_sizes)
    idx = torch.empty((nq, kstride), dtype=torch.int32, device="cuda")
    d2 = torch.empty((nq, kstride), dtype=torch.float32, device="cuda")
    need = ctypes.c_size_t(0)
    head = (batch.B, batch.clouds, _ptr(queries), nq, kstride, _ptr(idx), _ptr(d2))
    B.check(L.knn_search_batched(*head, None, ctypes.byref(need), None), "knn_search_batched(size)")
    ws = _ws(torch, need.value)
    B.check(L.knn_search_batched(*head, _ptr(ws), ctypes.byref(need), _stream(torch)), "knn_search_batched")
    return idx, d2


# ------------------------------------------------------ locality (Section 5.2)
LOCALITY_STATS = ("total", "mean", "std", "g1", "q1", "q2", "q3", "max")


def knn_locality(tree: Octree, k: int = 8, rows=None, sample: float | None = None, seed: int = 0):
    """Section 5.2: the kNN locality histogram of the tree's stored order.
    rows: stored positions of the query points (default all points); with
    `sample`, a seeded random fraction of the points (the subset estimate).
    Returns (hist int32 [n], stats dict: total, mean, std, g1, q1, q2, q3,
    max)."""
    import numpy as np
    torch = _torch()
    L = B.load()
    n = tree.n
    if sample is not None:
        m = max(1, min(n, int(round(float(sample) * n))))
        rows = np.sort(np.random.default_rng(seed).choice(n, m, replace=False))
    if rows is None:
        idx, _ = knn_search(tree, None, k)
        rows_t, nq = None, n
    else:
        rows_t = torch.as_tensor(np.asarray(rows, dtype=np.int64)).cuda()
        queries = tree.points()[rows_t, :3].contiguous()
        idx, _ = knn_search(tree, queries, k)
        rows_t = rows_t.to(torch.int32)
        nq = int(rows_t.numel())
    hist = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    stats = torch.empty(8, dtype=torch.float64, device="cuda")
    need = ctypes.c_size_t(0)
    args = (ctypes.byref(tree.view), _ptr(rows_t), nq, _ptr(idx), int(k), int(k), _ptr(hist), _ptr(stats))
    B.check(L.knn_locality(*args, None, ctypes.byref(need), None), "knn_locality(size)")
    ws = _ws(torch, need.value)
    B.check(L.knn_locality(*args, _ptr(ws), ctypes.byref(need), _stream(torch)), "knn_locality")
    return hist, dict(zip(LOCALITY_STATS, stats.cpu().tolist()))


def choose_curve(xyz, k: int = 8, sample: float = 0.01, seed: int = 0, bits: int = 21, leaf_size: int = 64):
    """Section 5.2's use of the histogram: build the cloud along both curves
    and keep the order whose locality histogram, estimated on a random subset
    of the points, is the more left-skewed (larger G1).  Returns (curve name,
    tree, {curve: stats})."""
    best, stats = None, {}
    trees = {}
    for curve in ("morton", "hilbert"):
        t = build_linear_octree(xyz, curve, bits, leaf_size)
        _, st = knn_locality(t, k, sample=sample, seed=seed)
        stats[curve] = st
        trees[curve] = t
        if best is None or st["g1"] > stats[best]["g1"]:
            best = curve
    return best, trees[best], stats


def radius_search_struct(tree: Octree, queries=None, kernel="sphere", r: float = 1.0, prune: bool = True):
    """Section 5.1, neighboursStruct: ((rcounts, roffsets, ranges int32 [R, 2]
    of sorted positions), (pcounts, poffsets, points int32 original indices)).
    The count pass runs first and the host reads both totals before the fill."""
    torch = _torch()
    L = B.load()
    if queries is not None:
        queries = _xyz(torch, queries)
        nq = queries.shape[0]
    else:
        nq = tree.n
    flags = 0 if prune else B.NO_PRUNE
    rc = torch.empty(nq, dtype=torch.int32, device="cuda")
    ro = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    pc = torch.empty(nq, dtype=torch.int32, device="cuda")
    po = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    head = (ctypes.byref(tree.view), _ptr(queries), nq, _code(KERNELS, kernel), float(r), _ptr(rc), _ptr(ro))
    need = ctypes.c_size_t(0)
    B.check(L.radius_search_struct(*head, None, 0, _ptr(pc), _ptr(po), None, 0, flags, None, ctypes.byref(need),
                                   None), "radius_search_struct(size)")
    ws = _ws(torch, need.value)
    stream = _stream(torch)
    B.check(L.radius_search_struct(*head, None, 0, _ptr(pc), _ptr(po), None, 0, flags, _ptr(ws), ctypes.byref(need),
                                   stream), "radius_search_struct(count)")
    nr, npt = int(ro[nq].item()), int(po[nq].item())
    ranges = torch.empty((max(nr, 1), 2), dtype=torch.int32, device="cuda")
    points = torch.empty(max(npt, 1), dtype=torch.int32, device="cuda")
    B.check(L.radius_search_struct(*head, _ptr(ranges), nr, _ptr(pc), _ptr(po), _ptr(points), npt,
                                   flags | B.REUSE_COUNTS, _ptr(ws), ctypes.byref(need), stream),
            "radius_search_struct(fill)")
    return (rc, ro, ranges[:nr]), (pc, po, points[:npt])
