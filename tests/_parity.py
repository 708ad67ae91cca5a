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
