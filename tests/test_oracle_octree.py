"""Pins for the oracle's linear octree (paper Section 5.1): a depth-first
recursion written independently of the oracle's iterative refinement, and the
structural invariants of a complete octree."""
import bisect

import numpy as np
import pytest

import oracle
from paper_2603_06771_amd import datagen


def _dfs_leaves(keys, bits, max_leaf, start=0, level=0, out=None):
    # split a node while it holds more than max_leaf points and is above level L
    if out is None:
        out = []
    length = 1 << (3 * (bits - level))
    cnt = bisect.bisect_left(keys, start + length) - bisect.bisect_left(keys, start)
    if cnt > max_leaf and level < bits:
        part = length // 8
        for c in range(8):
            _dfs_leaves(keys, bits, max_leaf, start + c * part, level + 1, out)
    else:
        out.append((start, level, cnt))
    return out


def _tree_for(pts, curve, bits, max_leaf):
    keys, lo, s = oracle.encode(pts, curve, bits)
    ks, perm = oracle.sort(keys)
    return ks, perm, oracle.build_tree(pts, ks, perm, bits, max_leaf)


@pytest.mark.parametrize("curve", ["morton", "hilbert"])
@pytest.mark.parametrize("n,bits,max_leaf", [(0, 21, 8), (5, 21, 8), (300, 21, 4), (2000, 21, 16),
                                              (1500, 3, 4), (4000, 2, 32)])
def test_leaves_match_dfs_and_invariants(curve, n, bits, max_leaf):
    pts = datagen.uniform(n, seed=100 + n)
    if n:
        pts = datagen.with_duplicates(pts, n // 10, seed=n)
    ks, perm, t = _tree_for(pts, curve, bits, max_leaf)
    keys = [int(k) for k in ks]
    ref = _dfs_leaves(keys, bits, max_leaf)
    nl = t["n_leaves"]
    assert nl == len(ref)
    assert [int(v) for v in t["leaves"][:-1]] == [r[0] for r in ref]
    assert int(t["leaves"][-1]) == 1 << (3 * bits)
    assert [int(c) for c in t["counts"]] == [r[2] for r in ref]
    # complete octree: every split adds 7 leaves
    assert nl % 7 == 1 and t["n_internal"] == (nl - 1) // 7
    assert int(t["counts"].sum()) == len(keys)
    lv = t["leaves"].astype(object)
    for i in range(nl):
        ln = lv[i + 1] - lv[i]
        assert ln & (ln - 1) == 0 and (ln.bit_length() - 1) % 3 == 0  # 8^m long
        assert lv[i] % ln == 0                                          # 8^m aligned
        level = bits - (ln.bit_length() - 1) // 3
        assert t["counts"][i] <= max_leaf or level == bits


@pytest.mark.parametrize("curve", ["morton", "hilbert"])
def test_node_ranges_boxes_children(curve):
    pts = datagen.with_duplicates(datagen.lidar_tile(3000, seed=9), 200, seed=4)
    bits, max_leaf = 21, 8
    ks, perm, t = _tree_for(pts, curve, bits, max_leaf)
    nn = t["n_nodes"]
    assert nn == t["n_leaves"] + t["n_internal"]
    lvl, st = t["node_level"], t["node_start"]
    # ordered by (level, start)
    order = np.lexsort((st, lvl))
    assert np.array_equal(order, np.arange(nn))
    assert lvl[0] == 0 and st[0] == 0 and t["node_begin"][0] == 0 and t["node_end"][0] == len(ks)
    sorted_pts = pts[perm]
    for i in range(nn):
        b, e = int(t["node_begin"][i]), int(t["node_end"][i])
        length = 1 << (3 * (bits - int(lvl[i])))
        # internalRanges: the points whose codes fall in the node's code range
        assert np.all(ks[b:e] >= st[i]) and np.all(ks[b:e] < int(st[i]) + length)
        assert (b == 0 or ks[b - 1] < st[i]) and (e == len(ks) or ks[e] >= int(st[i]) + length)
        box = t["node_box"][i]
        if e > b:
            assert np.array_equal(box[:3], sorted_pts[b:e].min(0))
            assert np.array_equal(box[3:], sorted_pts[b:e].max(0))
        else:
            assert np.all(np.isinf(box[:3]) & (box[:3] > 0)) and np.all(np.isinf(box[3:]) & (box[3:] < 0))
        c = int(t["node_child"][i])
        if c >= 0:
            # internal: more points than the threshold; 8 consecutive children
            # that partition its range
            assert e - b > max_leaf and lvl[i] < bits
            assert np.all(lvl[c:c + 8] == lvl[i] + 1)
            assert [int(v) for v in st[c:c + 8]] == [int(st[i]) + j * (length // 8) for j in range(8)]
            assert t["node_begin"][c] == b and t["node_end"][c + 7] == e
            assert np.all(t["node_end"][c:c + 7] == t["node_begin"][c + 1:c + 8])
        else:
            assert e - b <= max_leaf or lvl[i] == bits


def test_single_leaf_and_level_cap():
    # n <= threshold: the root is the only leaf
    pts = datagen.uniform(7, seed=1)
    _, _, t = _tree_for(pts, "morton", 21, 8)
    assert t["n_leaves"] == 1 and t["n_internal"] == 0
    assert list(t["leaves"]) == [0, 1 << 63] and list(t["counts"]) == [7]
    # 40 copies of one point at L = 2: the level-2 leaf keeps all 40
    pts = np.repeat(np.array([[0.3, 0.3, 0.3]], np.float32), 40, axis=0)
    pts = np.concatenate([pts, np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]], np.float32)])
    _, _, t = _tree_for(pts, "morton", 2, 4)
    assert t["n_internal"] == 2 and t["n_leaves"] == 15
    assert max(t["counts"]) == 40
