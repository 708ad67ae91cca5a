"""Pre-allocated batched pipelines: build + radius search (or k-NN) of a batch
of clouds with every buffer sized once, so that one step issues only kernel
launches (no allocation, no host synchronisation) and can be captured in a
HIP graph and replayed.

A step is: build_linear_octree_batched, then for a radius plan the count
pass, the scan and the fill pass of radius_search_batched (the fill writes
only when the output capacity holds the total), for a k-NN plan
knn_search_batched.  All launches go to the stream current at call time.
"""
from __future__ import annotations

import ctypes

from . import _binding as B
from . import CURVES, KERNELS, _code, _per_cloud, _ptr, _torch, _xyz


class BatchPlan:
    """One batch of clouds (xyz holds them one after the other, cloud c has
    sizes[c] points) with per-cloud curve / leaf size and either per-cloud
    (kernel, r) for radius search or per-cloud k for k-NN; every cloud's own
    points are its queries."""

    def __init__(self, xyz, sizes, curve="hilbert", bits=21, leaf_size=32, kernel="sphere", r=1.0, k=None,
                 capacity: int | None = None, record=False, stage=128):
        torch = _torch()
        # record (one value or one per cloud): the count pass records the
        # cloud's hits and the fill writes its rows from them (larger
        # workspace); stage (one value or one per cloud): the staging tile
        self.flags = 0
        self.L = B.load()
        self.xyz = _xyz(torch, xyz)
        self.sizes = [int(x) for x in sizes]
        nb = len(self.sizes)
        if nb < 1 or sum(self.sizes) != self.xyz.shape[0]:
            raise ValueError("sizes must be non-empty and sum to the number of points")
        self.B = nb
        self.n = sum(self.sizes)
        self.knn = k is not None
        curves = _per_cloud(curve, nb, "curve")
        bitss = _per_cloud(bits, nb, "bits")
        leafs = _per_cloud(leaf_size, nb, "leaf_size")
        kernels = _per_cloud(kernel, nb, "kernel")
        radii = _per_cloud(r, nb, "r")
        ks = _per_cloud(k if k is not None else 1, nb, "k")
        records = _per_cloud(record, nb, "record")
        stages = _per_cloud(stage, nb, "stage")
        cl = (B.SfcCloud * nb)()
        off = 0
        for c in range(nb):
            cl[c].offset = off
            cl[c].n = self.sizes[c]
            cl[c].curve = _code(CURVES, curves[c])
            cl[c].bits = int(bitss[c])
            cl[c].leaf_size = int(leafs[c])
            cl[c].kernel = _code(KERNELS, kernels[c])
            cl[c].r = float(radii[c])
            cl[c].k = int(ks[c])
            cl[c].q_offset = off
            cl[c].nq = self.sizes[c]
            if int(stages[c]) not in (64, 128, 256):
                raise ValueError(f"stage must be 64, 128 or 256, not {stages[c]!r}")
            cl[c].stage = int(stages[c])
            cl[c].record = 1 if (records[c] and k is None) else 0
            off += self.sizes[c]
        self.clouds = cl
        tb = ctypes.c_size_t(0)
        B.check(self.L.octree_batch_layout(nb, cl, None, ctypes.byref(tb)), "octree_batch_layout(size)")
        self.tree_mem = torch.empty(max(tb.value, 256), dtype=torch.uint8, device="cuda")
        B.check(self.L.octree_batch_layout(nb, cl, _ptr(self.tree_mem), ctypes.byref(tb)), "octree_batch_layout")
        need = ctypes.c_size_t(0)
        B.check(self.L.build_linear_octree_batched(_ptr(self.xyz), nb, cl, None, ctypes.byref(need), None),
                "build_linear_octree_batched(size)")
        self.build_ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
        self.build_need = ctypes.c_size_t(need.value)
        if self.knn:
            self.kstride = max(int(x) for x in ks)
            self.idx = torch.empty((self.n, self.kstride), dtype=torch.int32, device="cuda")
            self.d2 = torch.empty((self.n, self.kstride), dtype=torch.float32, device="cuda")
            B.check(self.L.knn_search_batched(nb, cl, None, self.n, self.kstride, _ptr(self.idx), _ptr(self.d2),
                                              None, ctypes.byref(need), None), "knn_search_batched(size)")
        else:
            self.counts = torch.empty(self.n, dtype=torch.int32, device="cuda")
            self.offsets = torch.empty(self.n + 1, dtype=torch.int64, device="cuda")
            B.check(self.L.radius_search_batched(nb, cl, None, self.n, _ptr(self.counts), _ptr(self.offsets), None,
                                                 0, self.flags, None, ctypes.byref(need), None),
                    "radius_search_batched(size)")
        self.search_ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
        self.search_need = ctypes.c_size_t(need.value)
        self.indices = None
        self.capacity = 0
        if not self.knn:
            if capacity is None:
                # size the output from one counting step
                self.run()
                capacity = int(self.offsets[self.n].item())
            self.capacity = int(capacity)
            self.indices = torch.empty(max(self.capacity, 1), dtype=torch.int32, device="cuda")
        self.graph = None

    def _stream(self):
        torch = _torch()
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def build(self):
        s = self._stream()
        B.check(self.L.build_linear_octree_batched(_ptr(self.xyz), self.B, self.clouds, _ptr(self.build_ws),
                                                   ctypes.byref(self.build_need), s), "build_linear_octree_batched")

    def search(self, count: bool = True, fill: bool = True):
        s = self._stream()
        if self.knn:
            B.check(self.L.knn_search_batched(self.B, self.clouds, None, self.n, self.kstride, _ptr(self.idx),
                                              _ptr(self.d2), _ptr(self.search_ws), ctypes.byref(self.search_need),
                                              s), "knn_search_batched")
            return
        head = (self.B, self.clouds, None, self.n, _ptr(self.counts), _ptr(self.offsets))
        if count:
            B.check(self.L.radius_search_batched(*head, None, 0, self.flags, _ptr(self.search_ws),
                                                 ctypes.byref(self.search_need), s), "radius_search_batched(count)")
        if fill and self.indices is not None:
            B.check(self.L.radius_search_batched(*head, _ptr(self.indices), self.capacity,
                                                 B.REUSE_COUNTS | self.flags, _ptr(self.search_ws),
                                                 ctypes.byref(self.search_need), s), "radius_search_batched(fill)")

    def run(self):
        """One step: build every tree, then search (launches only)."""
        self.build()
        self.search()

    def capture(self):
        """Captures one step in a HIP graph (torch.cuda.CUDAGraph on ROCm);
        replay() then re-runs it with one launch from the host."""
        torch = _torch()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()  # warm the stream before capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            self.run()
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def total(self) -> int:
        return int(self.offsets[self.n].item())

    def rows(self, c: int):
        """(first row, rows) of cloud c in the outputs."""
        return int(self.clouds[c].q_offset), int(self.clouds[c].nq)

    def tree(self, c: int):
        from . import Octree
        t = self.clouds[c].tree
        return Octree(mem=self.tree_mem, view=t, curve=t.curve, bits=t.bits, leaf_size=t.leaf_size, n=t.n)
