"""Serving loop: octrees resident in HBM, continuous batching of radius and
k-NN requests, admission by memory, overlap on several streams.

* ``Resident`` keeps clouds and their linear octrees in device memory.  Clouds
  are admitted in groups (one batched build per group) while their bytes fit
  the budget; a group can be dropped to make room.
* ``Server.run`` replays a request stream in real time.  Each request names a
  resident cloud, a set of its points as queries, and a radius search (kernel,
  r) or a k-NN search (k).  Requests that have arrived wait in a FIFO queue;
  whenever one of the server's slots is free, the head of the queue is packed
  into a batch (up to a request count, a query count and an output-memory
  budget, so a batch never needs more memory than its slot holds) and the
  batch runs on the slot's stream: query ids are copied in, the query points
  gathered, one radius_search_batched (count, scan, fill) for the batch's
  radius requests and one knn_search_batched for its k-NN requests.  While a
  batch runs, newly arrived requests are packed into the next free slot, so
  the work of several batches overlaps on the GPU.
* Latency of a request = completion of its batch (a device event, placed on
  the host clock through a reference event) minus its arrival time.

With ``max_requests=1`` and one slot the same loop is the one-launch-per-
request FIFO server used as the baseline.

Results stay in device memory (views into the slot's buffers) until the slot
is reused; ``on_result`` receives them when the batch has completed.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field

import numpy as np

from . import _binding as B
from . import CURVES, KERNELS, _code, _ptr, _torch

KMAX = 32


class Resident:
    """Clouds and their octrees resident in device memory.  A group of clouds
    is built in memory sized by the node upper bound (so the build needs no
    host round trip) and, with compact=True, then copied into exactly the
    memory its actual trees need (octree_batch_compact); the budget is
    charged the exact bytes, and the upper bound only has to fit while the
    group is being built."""

    def __init__(self, budget_bytes: int, curve="hilbert", bits: int = 21, leaf_size: int = 64,
                 compact: bool = True):
        self.budget = int(budget_bytes)
        self.curve = curve
        self.bits = bits
        self.leaf = leaf_size
        self.compact = compact
        self.groups = []       # (xyz, tree_mem, clouds table, first cloud id)
        self.cloud = []        # cloud id -> (group, index in group)
        self.used = 0

    def bytes_for(self, sizes) -> int:
        """Device bytes a group of clouds needs while it is built (points +
        trees at the node upper bound)."""
        L = B.load()
        nb = len(sizes)
        cl = (B.SfcCloud * nb)()
        off = 0
        for c, n in enumerate(sizes):
            cl[c].offset, cl[c].n, cl[c].bits, cl[c].leaf_size = off, int(n), self.bits, self.leaf
            cl[c].curve = _code(CURVES, self.curve)
            off += int(n)
        tb = ctypes.c_size_t(0)
        B.check(L.octree_batch_layout(nb, cl, None, ctypes.byref(tb)), "octree_batch_layout(size)")
        return int(tb.value) + 12 * off

    def admit(self, clouds_xyz) -> list | None:
        """Builds the trees of a group of clouds (host or device float32
        (n, 3) arrays) if they fit the budget; returns their cloud ids, or
        None (nothing allocated) if they do not fit."""
        torch = _torch()
        L = B.load()
        sizes = [int(x.shape[0]) for x in clouds_xyz]
        need = self.bytes_for(sizes)
        if self.used + need > self.budget:
            return None
        parts = [x if hasattr(x, "is_cuda") else torch.from_numpy(np.ascontiguousarray(x, np.float32))
                 for x in clouds_xyz]
        xyz = torch.cat([p.cuda() for p in parts]).contiguous()
        nb = len(sizes)
        cl = (B.SfcCloud * nb)()
        off = 0
        for c, n in enumerate(sizes):
            cl[c].offset, cl[c].n, cl[c].bits, cl[c].leaf_size = off, n, self.bits, self.leaf
            cl[c].curve = _code(CURVES, self.curve)
            off += n
        tb = ctypes.c_size_t(0)
        B.check(L.octree_batch_layout(nb, cl, None, ctypes.byref(tb)), "octree_batch_layout(size)")
        mem = torch.empty(max(tb.value, 256), dtype=torch.uint8, device="cuda")
        B.check(L.octree_batch_layout(nb, cl, _ptr(mem), ctypes.byref(tb)), "octree_batch_layout")
        wsb = ctypes.c_size_t(0)
        B.check(L.build_linear_octree_batched(_ptr(xyz), nb, cl, None, ctypes.byref(wsb), None), "build(size)")
        ws = torch.empty(max(wsb.value, 256), dtype=torch.uint8, device="cuda")
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        B.check(L.build_linear_octree_batched(_ptr(xyz), nb, cl, _ptr(ws), ctypes.byref(wsb), stream), "build")
        torch.cuda.synchronize()
        del ws
        if self.compact:
            # the trees copied into exactly the memory their actual sizes need
            cb = ctypes.c_size_t(0)
            B.check(L.octree_batch_compact(nb, cl, None, ctypes.byref(cb), None, stream), "octree_batch_compact(size)")
            cmem = torch.empty(max(cb.value, 256), dtype=torch.uint8, device="cuda")
            out = (B.SfcCloud * nb)()
            B.check(L.octree_batch_compact(nb, cl, _ptr(cmem), ctypes.byref(cb), out, stream), "octree_batch_compact")
            torch.cuda.synchronize()
            del mem
            mem, cl = cmem, out
            need = int(cb.value) + 12 * off
        g = len(self.groups)
        first = len(self.cloud)
        self.groups.append({"xyz": xyz, "mem": mem, "clouds": cl, "first": first, "sizes": sizes,
                            "offsets": np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64), "bytes": need})
        for c in range(nb):
            self.cloud.append((g, c))
        self.used += need
        return list(range(first, first + nb))

    def drop(self, group: int) -> None:
        """Frees a group (its cloud ids stay allocated but become invalid)."""
        g = self.groups[group]
        if g is None:
            return
        self.used -= g["bytes"]
        self.groups[group] = None

    def tree(self, cid: int):
        g, c = self.cloud[cid]
        return self.groups[g]["clouds"][c].tree

    def size(self, cid: int) -> int:
        g, c = self.cloud[cid]
        return self.groups[g]["sizes"][c]

    def octree(self, cid: int):
        """Octree view of a resident cloud (accepted by the single-cloud calls)."""
        from . import Octree
        g, c = self.cloud[cid]
        t = self.groups[g]["clouds"][c].tree
        return Octree(mem=self.groups[g]["mem"], view=t, curve=t.curve, bits=t.bits, leaf_size=t.leaf_size, n=t.n)

    def xyz_rows(self, cid: int):
        """(group xyz tensor, first row of the cloud in it)."""
        g, c = self.cloud[cid]
        return self.groups[g]["xyz"], int(self.groups[g]["offsets"][c])


@dataclass
class Request:
    id: int
    arrival: float
    cloud: int
    rows: np.ndarray          # query point ids (rows of the cloud)
    op: str                   # "radius" or "knn"
    kernel: str = "sphere"
    radius: float = 1.0
    k: int = 8
    est_out: int = 0          # estimated output entries (admission)


def estimate_neighbours(kernel: str, r: float, density: float = 10.0) -> float:
    """Expected neighbours per query on a LiDAR tile of `density` ground points
    per square metre, with margin for vegetation (admission estimate only)."""
    area = np.pi * r * r if kernel in ("sphere", "circle") else 4.0 * r * r
    return 2.0 * density * area + 8.0


@dataclass
class _Slot:
    stream: object
    rows: object
    qr: object
    qk: object
    counts: object
    offsets: object
    indices: object
    kidx: object
    kd2: object
    ws: object
    ws_bytes: int
    table_r: object
    table_k: object
    total_host: object
    done: object
    batch: list = field(default_factory=list)
    nq_r: int = 0
    spans: dict = field(default_factory=dict)


class Server:
    """Continuous-batching server over a Resident set (see module docstring)."""

    def __init__(self, resident: Resident, slots: int = 3, max_requests: int = 64, max_queries: int = 4 << 20,
                 out_entries: int = 1 << 30):
        torch = _torch()
        self.L = B.load()
        self.res = resident
        self.max_requests = int(max_requests)
        self.table_size = int(max_requests)
        self.max_queries = int(max_queries)
        self.out_entries = int(out_entries)
        self.slots = []
        for _ in range(int(slots)):
            mq = self.max_queries
            need = ctypes.c_size_t(0)
            # workspace for the largest batch: table + scan of max_queries rows
            cl = (B.SfcCloud * self.max_requests)()
            for c in range(self.max_requests):
                cl[c].tree = resident.tree(0)
                cl[c].nq = mq if c == 0 else 0
                cl[c].q_offset = 0 if c == 0 else mq
                cl[c].k = 1
            B.check(self.L.radius_search_batched(self.max_requests, cl, ctypes.c_void_p(256), mq,
                                                 ctypes.c_void_p(256), ctypes.c_void_p(256), None, 0, 0, None,
                                                 ctypes.byref(need), None), "server ws size")
            wr = need.value
            B.check(self.L.knn_search_batched(self.max_requests, cl, ctypes.c_void_p(256), mq, KMAX,
                                              ctypes.c_void_p(256), ctypes.c_void_p(256), None, ctypes.byref(need),
                                              None), "server ws size")
            wsb = max(wr, need.value, 256)
            self.slots.append(_Slot(
                stream=torch.cuda.Stream(),
                rows=torch.empty(mq, dtype=torch.int32, device="cuda"),
                qr=torch.empty((mq, 3), dtype=torch.float32, device="cuda"),
                qk=torch.empty((mq, 3), dtype=torch.float32, device="cuda"),
                counts=torch.empty(mq, dtype=torch.int32, device="cuda"),
                offsets=torch.empty(mq + 1, dtype=torch.int64, device="cuda"),
                indices=torch.empty(self.out_entries, dtype=torch.int32, device="cuda"),
                kidx=torch.empty((mq, KMAX), dtype=torch.int32, device="cuda"),
                kd2=torch.empty((mq, KMAX), dtype=torch.float32, device="cuda"),
                ws=torch.empty(wsb, dtype=torch.uint8, device="cuda"), ws_bytes=wsb,
                table_r=(B.SfcCloud * self.max_requests)(), table_k=(B.SfcCloud * self.max_requests)(),
                total_host=torch.zeros(1, dtype=torch.int64, pin_memory=True),
                done=torch.cuda.Event(enable_timing=True)))

    # -------------------------------------------------------------- payload
    def stage(self, requests):
        """The requests' query ids, as a pinned host buffer of point ids in the
        cloud's group (the "network receive buffer"); one contiguous block per
        request."""
        torch = _torch()
        total = sum(len(r.rows) for r in requests)
        buf = torch.empty(max(total, 1), dtype=torch.int32, pin_memory=True)
        view = buf.numpy()
        self._span = {}
        at = 0
        for r in requests:
            _, first = self.res.xyz_rows(r.cloud)
            n = len(r.rows)
            view[at:at + n] = (np.asarray(r.rows, np.int64) + first).astype(np.int32)
            self._span[r.id] = (at, n)
            if r.op == "radius":
                r.est_out = int(n * estimate_neighbours(r.kernel, r.radius))
            at += n
        self._payload = buf

    # ------------------------------------------------------------ batching
    def _take(self, queue):
        """Pops the head of the queue into a batch within the slot limits."""
        batch, nq, out = [], 0, 0
        while queue and len(batch) < self.max_requests:
            r = queue[0]
            n = len(r.rows)
            if batch and (nq + n > self.max_queries or out + r.est_out > self.out_entries):
                break
            batch.append(queue.popleft())
            nq += n
            out += r.est_out
        return batch

    def _submit(self, s: _Slot, batch):
        torch = _torch()
        L = self.L
        s.batch = batch
        rad = [r for r in batch if r.op == "radius"]
        knn = [r for r in batch if r.op == "knn"]
        with torch.cuda.stream(s.stream):
            sp = ctypes.c_void_p(s.stream.cuda_stream)
            # query ids in, then the query points of each request
            at = 0
            spans = {}
            for group, dst in ((rad, s.qr), (knn, s.qk)):
                q0 = 0
                for r in group:
                    p0, n = self._span[r.id]
                    s.rows[at:at + n].copy_(self._payload[p0:p0 + n], non_blocking=True)
                    xyz, _ = self.res.xyz_rows(r.cloud)
                    B.check(L.gather_points(_ptr(xyz), xyz.shape[0], ctypes.c_void_p(s.rows.data_ptr() + 4 * at), n,
                                            ctypes.c_void_p(dst.data_ptr() + 12 * q0), sp), "gather_points")
                    spans[r.id] = (q0, n)
                    q0 += n
                    at += n
            need = ctypes.c_size_t(s.ws_bytes)
            nq_r = sum(len(r.rows) for r in rad)
            if rad:
                for i, r in enumerate(rad):
                    e = s.table_r[i]
                    e.tree = self.res.tree(r.cloud)
                    e.offset, e.n = 0, e.tree.n
                    e.kernel = _code(KERNELS, r.kernel)
                    e.r = float(r.radius)
                    e.q_offset, e.nq = spans[r.id]
                head = (len(rad), s.table_r, _ptr(s.qr), nq_r, _ptr(s.counts), _ptr(s.offsets))
                # count, scan and fill in one call (the fill writes only if the slot's buffer holds the total)
                B.check(L.radius_search_batched(*head, _ptr(s.indices), s.indices.numel(), 0, _ptr(s.ws),
                                                ctypes.byref(need), sp), "radius")
                s.total_host.copy_(s.offsets[nq_r:nq_r + 1], non_blocking=True)
            if knn:
                nq_k = 0
                for i, r in enumerate(knn):
                    e = s.table_k[i]
                    e.tree = self.res.tree(r.cloud)
                    e.offset, e.n = 0, e.tree.n
                    e.k = int(r.k)
                    e.q_offset, e.nq = spans[r.id]
                    nq_k += len(r.rows)
                B.check(L.knn_search_batched(len(knn), s.table_k, _ptr(s.qk), nq_k, KMAX, _ptr(s.kidx), _ptr(s.kd2),
                                             _ptr(s.ws), ctypes.byref(need), sp), "knn")
            s.done.record(s.stream)
        s.nq_r = nq_r
        s.spans = spans

    def _finish(self, s: _Slot, on_result):
        """Called once the slot's batch has completed: checks the output fit
        and hands out results."""
        torch = _torch()
        if any(r.op == "radius" for r in s.batch):
            total = int(s.total_host[0])
            if total > s.indices.numel():
                # the estimate was too small: fill again into a buffer of the right size
                L = self.L
                rad = [r for r in s.batch if r.op == "radius"]
                big = torch.empty(total, dtype=torch.int32, device="cuda")
                need = ctypes.c_size_t(s.ws_bytes)
                with torch.cuda.stream(s.stream):
                    head = (len(rad), s.table_r, _ptr(s.qr), s.nq_r, _ptr(s.counts), _ptr(s.offsets))
                    B.check(L.radius_search_batched(*head, _ptr(big), total, B.REUSE_COUNTS, _ptr(s.ws),
                                                    ctypes.byref(need), ctypes.c_void_p(s.stream.cuda_stream)),
                            "fill (regrown)")
                    s.done.record(s.stream)
                s.done.synchronize()
                self.regrown += 1
                s.big = big
            else:
                s.big = None
        if on_result is not None:
            for r in s.batch:
                q0, n = s.spans[r.id]
                if r.op == "radius":
                    ind = s.big if s.big is not None else s.indices
                    off = s.offsets[q0:q0 + n + 1]
                    a, b = int(off[0]), int(off[-1])
                    on_result(r, (s.counts[q0:q0 + n], off - a, ind[a:b]))
                else:
                    on_result(r, (s.kidx[q0:q0 + n, :r.k], s.kd2[q0:q0 + n, :r.k]))
        s.batch = []

    # ----------------------------------------------------------------- loop
    def run(self, requests, on_result=None, max_requests: int | None = None, n_slots: int | None = None,
            log=None, log_every: float = 5.0):
        """Replays `requests` (sorted by arrival, seconds from start) in real
        time.  Returns per-request latency (s) and the run's span."""
        torch = _torch()
        self.max_requests = min(int(max_requests), self.table_size) if max_requests else self.table_size
        slots = self.slots[:n_slots] if n_slots else self.slots
        self.stage(requests)
        self.regrown = 0
        reqs = list(requests)
        torch.cuda.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record()
        ref.synchronize()
        t0 = time.perf_counter()
        queue = collections.deque()
        free = list(slots)
        busy = []
        done_at = {}
        batches = 0
        i = 0
        next_log = log_every
        while i < len(reqs) or queue or busy:
            now = time.perf_counter() - t0
            if log is not None and now >= next_log:
                log(f"[serve] t={now:.1f} s: {i} arrived, {len(queue)} queued, {len(busy)} batches on the GPU, "
                    f"{len(done_at)} done, {batches} batches")
                next_log += log_every
            while i < len(reqs) and reqs[i].arrival <= now:
                queue.append(reqs[i])
                i += 1
            still = []
            for s in busy:
                if s.done.query():
                    self._finish(s, on_result)
                    t_done = ref.elapsed_time(s.done) / 1e3
                    for r_id in s.spans:
                        done_at[r_id] = t_done
                    free.append(s)
                else:
                    still.append(s)
            busy = still
            progressed = False
            while free and queue:
                s = free.pop(0)
                self._submit(s, self._take(queue))
                busy.append(s)
                batches += 1
                progressed = True
            if not progressed:
                if not queue and not busy and i < len(reqs):
                    wait = reqs[i].arrival - (time.perf_counter() - t0)
                    if wait > 2e-4:
                        time.sleep(wait - 1e-4)
                else:
                    time.sleep(2e-5)
        lat = np.array([done_at[r.id] - r.arrival for r in reqs])
        span = max(done_at.values()) - min(r.arrival for r in reqs) if reqs else 0.0
        return {"latency_s": lat, "span_s": span, "batches": batches, "regrown": self.regrown,
                "queries": int(sum(len(r.rows) for r in reqs))}
