"""GPU parity of the range form of radius search (neighboursStruct, Section
5.1): per query, the ranges of contained nodes expanded through the
permutation, together with the listed points, are exactly the oracle's
neighbour set, with no point twice."""
import numpy as np
import pytest

import oracle
from paper_2603_06771_amd import datagen
from tests._parity import announce

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _expand(perm, rng_csr, pt_csr):
    """(row, original index) pairs of the range form, sorted by row then index."""
    rc, ro, ranges = (x.cpu().numpy() for x in rng_csr)
    pc, po, pts = (x.cpu().numpy() for x in pt_csr)
    nq = rc.size
    assert ro[0] == 0 and np.array_equal(np.diff(ro), rc) and np.array_equal(np.diff(po), pc)
    b = ranges[:, 0].astype(np.int64)
    e = ranges[:, 1].astype(np.int64)
    ln = e - b
    assert np.all(ln > 0)
    rrow = np.repeat(np.arange(nq), rc)
    start = np.repeat(b - np.concatenate([[0], np.cumsum(ln)[:-1]]), ln) + np.arange(int(ln.sum()))
    rows = np.concatenate([np.repeat(rrow, ln), np.repeat(np.arange(nq), pc)])
    idx = np.concatenate([perm[start].astype(np.int64), pts.astype(np.uint32).astype(np.int64)])
    order = np.lexsort((idx, rows))
    return rows[order], idx[order], int(ln.sum())


@pytest.mark.parametrize("curve", ["morton", "hilbert"])
@pytest.mark.parametrize("kernel", ["sphere", "circle", "cube", "square"])
def test_struct_matches_radius_set(curve, kernel):
    import torch
    import paper_2603_06771_amd as sfc
    pts = datagen.lidar_tile(60000, seed=41)
    t = sfc.build_linear_octree(_dev(pts), curve, 21, 16)
    perm = t.perm().cpu().numpy().view(np.uint32).astype(np.int64)
    for r in (0.5, 1.5, 3.0):
        announce(f"struct {curve} {kernel} r={r}")
        rng, pt = sfc.radius_search_struct(t, None, kernel, r)
        torch.cuda.synchronize()
        rows, idx, in_ranges = _expand(perm, rng, pt)
        rc, ro, ri = oracle.radius_search(pts, pts[perm], kernel, r)
        ref_rows = np.repeat(np.arange(rc.size), rc.astype(np.int64))
        assert rows.size == ri.size, (rows.size, ri.size)
        assert np.array_equal(rows, ref_rows) and np.array_equal(idx, np.asarray(ri).astype(np.int64))
        if r >= 1.5:
            assert in_ranges > 0  # some nodes are wholly inside a neighbourhood


def test_struct_external_and_no_prune():
    import torch
    import paper_2603_06771_amd as sfc
    rng_ = np.random.default_rng(42)
    pts = datagen.lidar_tile(40000, seed=43)
    lo, hi = pts.min(0), pts.max(0)
    q = (lo + (hi - lo) * rng_.uniform(-0.05, 1.05, (5000, 3))).astype(np.float32)
    t = sfc.build_linear_octree(_dev(pts), "hilbert", 21, 32)
    perm = t.perm().cpu().numpy().view(np.uint32).astype(np.int64)
    rc, ro, ri = oracle.radius_search(pts, q, "sphere", 2.5)
    ref_rows = np.repeat(np.arange(rc.size), rc.astype(np.int64))
    for prune in (True, False):
        announce(f"struct external prune={prune}")
        rng, pt = sfc.radius_search_struct(t, _dev(q), "sphere", 2.5, prune=prune)
        torch.cuda.synchronize()
        rows, idx, in_ranges = _expand(perm, rng, pt)
        assert np.array_equal(rows, ref_rows) and np.array_equal(idx, np.asarray(ri).astype(np.int64))
        if not prune:
            assert in_ranges == 0 and int(rng[1][-1]) == 0
