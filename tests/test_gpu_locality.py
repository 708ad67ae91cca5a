"""GPU parity of the kNN locality histogram (Section 5.2) against the oracle:
the histogram bit-exact, the statistics within 1e-9 relative (fp64 sums in a
different order), for all points and for a random subset of query points."""
import numpy as np
import pytest

import oracle
from paper_2603_06771_amd import datagen
from tests._parity import announce

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _check(hist, st, H, ref):
    import numpy as np
    assert np.array_equal(hist.cpu().numpy().astype(np.int64), H)
    for key, v in ref.items():
        assert abs(st[key] - v) <= 1e-9 * max(1.0, abs(v)), (key, st[key], v)


@pytest.mark.parametrize("curve", ["morton", "hilbert"])
@pytest.mark.parametrize("kind,k", [("lidar", 8), ("lidar", 16), ("dup", 8)])
def test_locality_all_points(curve, kind, k):
    import torch
    import paper_2603_06771_amd as sfc
    if kind == "lidar":
        pts = datagen.lidar_tile(30000, seed=31)
    else:
        pts = datagen.with_duplicates(datagen.uniform(20000, seed=32), 2000, seed=33)
    announce(f"locality {curve} {kind} k={k}")
    t = sfc.build_linear_octree(_dev(pts), curve, 21, 32)
    hist, st = sfc.knn_locality(t, k)
    torch.cuda.synchronize()
    perm = t.perm().cpu().numpy().view(np.uint32).astype(np.int64)
    idx, _ = oracle.knn(pts, pts[perm], k)
    H, ref = oracle.locality_histogram(perm, idx)
    _check(hist, st, H, ref)
    assert st["total"] == k * pts.shape[0]
    if kind == "lidar":
        assert hist[0].item() == pts.shape[0]  # every centre finds itself (no duplicates)


def test_locality_subset_and_choice():
    import torch
    import paper_2603_06771_amd as sfc
    pts = datagen.lidar_tile(50000, seed=34)
    t = sfc.build_linear_octree(_dev(pts), "hilbert", 21, 64)
    announce("locality subset 5 %")
    hist, st = sfc.knn_locality(t, 8, sample=0.05, seed=7)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(7).choice(50000, 2500, replace=False))
    perm = t.perm().cpu().numpy().view(np.uint32).astype(np.int64)
    idx, _ = oracle.knn(pts, pts[perm][rows], 8)
    H, ref = oracle.locality_histogram(perm, idx, rows)
    _check(hist, st, H, ref)
    announce("curve choice")
    curve, tree, stats = sfc.choose_curve(_dev(pts), k=8, sample=0.02)
    assert curve in ("morton", "hilbert") and tree.curve == sfc.CURVES[curve]
    assert stats[curve]["g1"] >= max(s["g1"] for s in stats.values())
