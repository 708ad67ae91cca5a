"""GPU check of radius_search_noalloc, the entry point that takes no
workspace (its workspace is the library's fixed per-GPU array): its counts,
offsets and indices equal those of radius_search with a caller workspace,
on two calls in a row, the second with a smaller input (the array keeps the
first call's contents), for cloud queries, sorted external queries and the
recorded-hits fill; a call that needs more than the fixed array is refused."""
import ctypes

import numpy as np
import pytest

from paper_2603_06771_amd import _binding as B
from paper_2603_06771_amd import datagen
from tests._parity import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfc():
    import torch  # noqa: F401
    import paper_2603_06771_amd as sfc
    return sfc


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)).cuda()


def _noalloc(sfc, tree, queries, nq, kernel, r, capacity, flags=0):
    """counts, offsets, indices from radius_search_noalloc (count and fill in
    one call; capacity from the workspace form's total)."""
    import torch
    L = B.load()
    counts = torch.full((nq,), -7, dtype=torch.int32, device="cuda")
    offsets = torch.full((nq + 1,), -7, dtype=torch.int64, device="cuda")
    indices = torch.full((max(capacity, 1),), -7, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    q = None if queries is None else ctypes.c_void_p(queries.data_ptr())
    rc = L.radius_search_noalloc(ctypes.byref(tree.view), q, nq, sfc.KERNELS[kernel], float(r),
                                 ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                                 ctypes.c_void_p(indices.data_ptr()), int(capacity), flags, ctypes.c_void_p(stream))
    B.check(rc, "radius_search_noalloc")
    torch.cuda.synchronize()
    return counts, offsets, indices


def _compare(sfc, pts, curve, kernel, r, queries=None, record=False):
    import torch
    tree = sfc.build_linear_octree(_dev(pts), curve, 21, 32)
    q = None if queries is None else _dev(queries)
    nq = pts.shape[0] if queries is None else queries.shape[0]
    rc, ro, ri = sfc.radius_search(tree, q, kernel, r, record=record)
    torch.cuda.synchronize()
    total = int(ro[-1])
    flags = B.RECORD_HITS if record else 0
    nc, no, ni = _noalloc(sfc, tree, q, nq, kernel, r, total, flags)
    assert np.array_equal(rc.cpu().numpy(), nc.cpu().numpy()), "counts differ"
    assert np.array_equal(ro.cpu().numpy(), no.cpu().numpy()), "offsets differ"
    assert np.array_equal(ri.cpu().numpy()[:total], ni.cpu().numpy()[:total]), "indices differ"
    return total


@pytest.mark.parametrize("kernel", ["sphere", "cube", "circle", "square"])
def test_noalloc_cloud_queries_two_calls(sfc, kernel):
    big = datagen.lidar_tile(200_000, seed=71)
    small = datagen.lidar_tile(30_001, seed=72)
    announce(f"noalloc cloud queries {kernel} 200000 then 30001")
    t1 = _compare(sfc, big, "hilbert", kernel, 1.5)
    t2 = _compare(sfc, small, "morton", kernel, 1.0)
    assert t1 > t2 > 0


def test_noalloc_external_queries_two_calls(sfc):
    pts = datagen.lidar_tile(150_000, seed=73)
    rng = np.random.default_rng(74)
    q1 = pts[rng.choice(pts.shape[0], 40_000, replace=False)] + rng.normal(0, 0.2, (40_000, 3)).astype(np.float32)
    q2 = q1[:5_003][::-1].copy()
    announce("noalloc external queries 40000 then 5003")
    _compare(sfc, pts, "hilbert", "sphere", 2.0, queries=q1)
    _compare(sfc, pts, "hilbert", "sphere", 2.0, queries=q2)


def test_noalloc_recorded_hits_two_calls(sfc):
    pts = datagen.lidar_tile(60_000, seed=75)
    announce("noalloc recorded hits 60000 then 7000")
    _compare(sfc, pts, "hilbert", "sphere", 1.0, record=True)
    _compare(sfc, pts[:7000].copy(), "hilbert", "cube", 0.5, record=True)


def test_noalloc_refuses_beyond_the_array(sfc):
    import torch
    pts = datagen.lidar_tile(100_000, seed=76)
    tree = sfc.build_linear_octree(_dev(pts), "hilbert", 21, 32)
    L = B.load()
    # 100k queries with recorded hits need about 75 MB of workspace: refused, nothing written
    counts = torch.full((100_000,), -7, dtype=torch.int32, device="cuda")
    offsets = torch.full((100_001,), -7, dtype=torch.int64, device="cuda")
    rc = L.radius_search_noalloc(ctypes.byref(tree.view), None, 100_000, 0, 1.0, ctypes.c_void_p(counts.data_ptr()),
                                 ctypes.c_void_p(offsets.data_ptr()), None, 0, B.RECORD_HITS,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == B.SFC_EWORKSPACE
    torch.cuda.synchronize()
    assert int(counts.min()) == -7 and int(counts.max()) == -7 and int(offsets.max()) == -7
