"""Helpers shared by the GPU parity tests (comparison only; no method
arithmetic)."""
import sys

import numpy as np


def announce(msg: str) -> None:
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def sorted_csr(counts, offsets, indices):
    """Row-sorted copy of a CSR (order inside a GPU row is unspecified)."""
    counts = np.asarray(counts, np.int64)
    offsets = np.asarray(offsets, np.int64)
    indices = np.asarray(indices).astype(np.uint32)
    assert offsets[0] == 0 and np.array_equal(np.diff(offsets), counts)
    rows = np.repeat(np.arange(counts.size), counts)
    order = np.lexsort((indices, rows))
    return indices[order]


def assert_csr_equal(gpu, ref, what=""):
    gc, go, gi = gpu
    rc, ro, ri = ref
    gc = np.asarray(gc).astype(np.int64)
    rc = np.asarray(rc).astype(np.int64)
    if not np.array_equal(gc, rc):
        bad = np.nonzero(gc != rc)[0]
        raise AssertionError(f"{what}: {bad.size} rows differ in count, first row {bad[0]}: "
                             f"gpu {gc[bad[0]]} oracle {rc[bad[0]]}")
    assert np.array_equal(np.asarray(go, np.int64), np.asarray(ro, np.int64)), f"{what}: offsets differ"
    a = sorted_csr(gc, go, gi)
    b = np.asarray(ri).astype(np.uint32)
    if not np.array_equal(a, b):
        bad = np.nonzero(a != b)[0]
        raise AssertionError(f"{what}: {bad.size} neighbour entries differ, first at {bad[0]}")


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def check_tree(t, pts, curve, bits, leaf):
    """Every array of a built tree (an Octree view) against the oracle's
    encode, sort and build of the same cloud."""
    import oracle
    info = t.info()
    rk, lo, s = oracle.encode(pts, curve, bits)
    ks, perm = oracle.sort(rk)
    ref = oracle.build_tree(pts, ks, perm, bits, leaf)
    assert info["status"] == 0
    assert info["n_points"] == pts.shape[0]
    f = t.frame()
    assert list(f.lo) == [float(v) for v in lo] and f.scale == float(s)
    assert np.array_equal(_u64(t.keys()), ks)
    assert np.array_equal(t.perm().cpu().numpy().view(np.uint32), perm)
    p = t.points().cpu().numpy()
    assert np.array_equal(p[:, :3], pts[perm])
    assert np.array_equal(p[:, 3].view(np.uint32), perm)
    assert info["n_internal"] == ref["n_internal"] and info["n_leaves"] == ref["n_leaves"]
    assert info["n_nodes"] == ref["n_nodes"]
    arr = t.arrays(info)
    assert np.array_equal(_u64(arr["leaves"]), ref["leaves"])
    assert np.array_equal(arr["counts"].cpu().numpy().view(np.uint32), ref["counts"])
    assert np.array_equal(arr["node_level"].cpu().numpy().astype(np.int32), ref["node_level"])
    assert np.array_equal(_u64(arr["node_key"]), ref["node_start"])
    nodes = arr["nodes"].cpu().numpy()
    assert np.array_equal(nodes[:, 3].view(np.uint32).astype(np.int64), ref["node_begin"])
    assert np.array_equal(nodes[:, 7].view(np.uint32).astype(np.int64), ref["node_end"])
    assert np.array_equal(arr["child"].cpu().numpy().astype(np.int64), ref["node_child"])
    box = np.concatenate([nodes[:, 0:3], nodes[:, 4:7]], axis=1)
    assert np.array_equal(box, ref["node_box"])
