"""Full-size GPU checks on the 10M-point LiDAR tile, in the launch
configuration the benchmark times (leaf size 64, every point a query, the
count pass recording the hits and the fill writing rows from the records,
through the C ABI as the benchmark calls it); the search fill is checked the
same way on one curve.

Radius search (Section 3.2 kernels, Section 5.1 pruning): the whole count
vector of every run is compared with the oracle's grid count over all 10M
points; at r = 0.5 m every index row is compared with the oracle's rows;
at r = 3 m (more than 2^31 neighbour indices in total, so 64-bit row
offsets) sampled rows are compared element by element and the rest is
checked through properties that hold at any size: every output slot is
written, every row holds its own centre, sampled neighbour pairs are
symmetric.

k-NN (Section 3.3) on the Hilbert tree with k = 8, 16, 32 over all 10M
points: sampled rows against the oracle (indices and squared-distance bits),
and on every row: ascending by (d2, index), no padding, d2 equal to the
fp32 expression recomputed from the coordinates, and the centre first among
the points at d2 = 0."""
import numpy as np
import pytest

import oracle
from paper_2603_06771_amd import datagen
from tests._parity import announce

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 10_000_000
LEAF = 64
SAMPLE = 1500


def _count_fill(tree, kernel, r, record):
    """Count call, then fill call into a buffer pre-set to -1, on one
    workspace and the current stream (the benchmark's two calls)."""
    import ctypes

    import torch

    import paper_2603_06771_amd as sfc
    from paper_2603_06771_amd import _binding as B
    L = B.load()
    counts = torch.empty(N, dtype=torch.int32, device="cuda")
    offsets = torch.empty(N + 1, dtype=torch.int64, device="cuda")
    base = (ctypes.byref(tree.view), None, N, sfc.KERNELS[kernel], float(r),
            ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(offsets.data_ptr()))
    flags = B.RECORD_HITS if record else 0
    need = ctypes.c_size_t(0)
    B.check(L.radius_search(*base, None, 0, flags, None, ctypes.byref(need), None), "size")
    ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    B.check(L.radius_search(*base, None, 0, flags, ctypes.c_void_p(ws.data_ptr()), ctypes.byref(need), stream),
            "count")
    total = int(offsets[-1].item())
    idx = torch.full((total,), -1, dtype=torch.int32, device="cuda")
    B.check(L.radius_search(*base, ctypes.c_void_p(idx.data_ptr()), total, B.REUSE_COUNTS | flags,
                            ctypes.c_void_p(ws.data_ptr()), ctypes.byref(need), stream), "fill")
    torch.cuda.synchronize()
    del ws
    return counts, offsets, idx, total


@pytest.fixture(scope="module")
def cloud():
    return datagen.lidar_tile(N, seed=datagen.SEED_LIDAR)


@pytest.fixture(scope="module")
def dev(cloud):
    import torch
    return torch.from_numpy(cloud).cuda()


@pytest.fixture(scope="module")
def ref():
    """Oracle results shared by the tests, computed once: counts of every
    point (original order) per (kernel, r), and the full rows at r = 0.5."""
    return {}


def _grid(ref, cloud, r):
    key = ("grid", r)
    if key not in ref:
        for k in [k for k in ref if k[0] == "grid"]:
            del ref[k]  # one grid at a time
        ref[key] = oracle.Grid(cloud, r, 3)  # sphere and cube share the 3D grid of side r
    return ref[key]


def _ref_counts(ref, cloud, kernel, r):
    key = ("counts", kernel, r)
    if key not in ref:
        ref[key] = _grid(ref, cloud, r).radius_count(cloud, kernel, r)
    return ref[key]


def _ref_rows(ref, cloud, kernel, r):
    key = ("rows", kernel, r)
    if key not in ref:
        _, ro, ri = _grid(ref, cloud, r).radius_search(cloud, kernel, r)
        ref[key] = (ro, ri)
    return ref[key]


def _rows_in_original_order(perm_dev, counts, idx):
    """The GPU's CSR (row i = the point at sorted position i) as one array of
    neighbour indices, rows in original point order and each row ascending:
    sorted by (original row, index) on the GPU."""
    import torch
    rows = torch.repeat_interleave(perm_dev.to(torch.int64), counts.to(torch.int64))
    key = (rows << 32) | (idx.to(torch.int64) & 0xFFFFFFFF)
    del rows
    key = torch.sort(key).values
    return (key & 0xFFFFFFFF).cpu().numpy().astype(np.uint32)


@pytest.mark.parametrize("curve,record", [("hilbert", True), ("morton", True), ("hilbert", False)])
def test_radius_fullsize(cloud, dev, ref, curve, record):
    import torch

    import paper_2603_06771_amd as sfc
    tree = sfc.build_linear_octree(dev, curve, 21, LEAF)
    perm = tree.perm().cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(17)
    rows = np.sort(rng.choice(N, SAMPLE, replace=False))
    for r in (0.5, 3.0):
        for kernel in ("sphere", "cube"):
            announce(f"fullsize {curve} {kernel} r={r} record={record}")
            counts, offsets, idx, total = _count_fill(tree, kernel, r, record)
            if r == 3.0:
                assert total > 2 ** 31  # 64-bit offsets in use
            # every slot written, every row holds its own centre
            assert not bool((idx == -1).any().item())
            cnt = counts.cpu().numpy()
            off = offsets.cpu().numpy()
            assert np.all(cnt >= 1) and off[0] == 0 and np.array_equal(np.diff(off), cnt.astype(np.int64))
            # the whole count vector against the oracle's (row i is point perm[i])
            rc = _ref_counts(ref, cloud, kernel, r)
            bad = np.nonzero(cnt.view(np.uint32) != rc[perm])[0]
            assert bad.size == 0, f"{bad.size} of {N} counts differ, first sorted row {bad[:1]}"
            if r == 0.5 and record:
                # every row, element by element
                ro, ri = _ref_rows(ref, cloud, kernel, r)
                assert int(ro[-1]) == total
                got = _rows_in_original_order(tree.perm(), counts, idx)
                diff = np.nonzero(got != ri)[0]
                assert diff.size == 0, f"{diff.size} neighbour entries differ, first at {diff[:1]}"
                del got
            else:
                # sampled rows against the oracle
                grid = _grid(ref, cloud, r)
                ref_c, ref_o, ref_i = grid.radius_search(cloud[perm[rows]], kernel, r)
                assert np.array_equal(cnt[rows].astype(np.int64), ref_c.astype(np.int64))
                for k, row in enumerate(rows):
                    got = np.sort(idx[int(off[row]):int(off[row + 1])].cpu().numpy().view(np.uint32))
                    assert np.array_equal(got, ref_i[ref_o[k]:ref_o[k + 1]]), f"row {row}"
                    assert perm[row] in set(got.tolist())
                # symmetry on sampled pairs: j in N(i) => i in N(j)
                inv = np.empty(N, np.int64)
                inv[perm] = np.arange(N)
                for k, row in enumerate(rows[:200]):
                    nb = ref_i[ref_o[k]:ref_o[k + 1]]
                    j = int(nb[rng.integers(0, nb.size)])
                    rj = int(inv[j])
                    back = idx[int(off[rj]):int(off[rj + 1])].cpu().numpy().view(np.uint32)
                    assert perm[row] in set(back.tolist())
            del idx, counts, offsets
            torch.cuda.empty_cache()
    del tree


@pytest.fixture(scope="module")
def htree(dev):
    import paper_2603_06771_amd as sfc
    return sfc.build_linear_octree(dev, "hilbert", 21, LEAF)


@pytest.mark.parametrize("k", [8, 16, 32])
def test_knn_fullsize(cloud, dev, ref, htree, k):
    import torch

    import paper_2603_06771_amd as sfc
    announce(f"fullsize knn hilbert k={k}")
    idx, d2 = sfc.knn_search(htree, None, k)
    torch.cuda.synchronize()
    perm_dev = htree.perm().to(torch.int64)
    # no padding (k < n), indices in range
    assert bool(((idx >= 0) & (idx < N)).all().item())
    # rows ascending by (d2, index)
    up = (d2[:, 1:] > d2[:, :-1]) | ((d2[:, 1:] == d2[:, :-1]) & (idx[:, 1:] > idx[:, :-1]))
    assert bool(up.all().item()), "a row is not ascending by (d2, index)"
    # d2 equals the fp32 expression ((dx*dx + dy*dy) + dz*dz) from the coordinates
    q = dev[perm_dev]
    for c0 in range(0, k, 8):
        p = dev[idx[:, c0:c0 + 8].to(torch.int64)]
        dd = p - q[:, None, :]
        sq = dd * dd
        e = (sq[..., 0] + sq[..., 1]) + sq[..., 2]
        assert torch.equal(e.view(torch.int32), d2[:, c0:c0 + 8].contiguous().view(torch.int32)), \
            f"d2 differs from the coordinates in columns {c0}..{c0 + 7}"
        del p, dd, sq, e
    # the centre is at d2 = 0; it comes first unless an identical point has a smaller index
    assert bool((d2[:, 0] == 0).all().item())
    alone = d2[:, 1] > 0
    assert bool((idx[:, 0].to(torch.int64)[alone] == perm_dev[alone]).all().item())
    assert bool((idx[:, 0].to(torch.int64) <= perm_dev).all().item())
    # sampled rows against the oracle, element by element
    rng = np.random.default_rng(19 + k)
    rows = np.sort(rng.choice(N, 2000, replace=False))
    perm = htree.perm().cpu().numpy().view(np.uint32)
    ridx, rd2 = oracle.knn(cloud, cloud[perm[rows]], k)
    gi = idx[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32)
    gd = d2[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert np.array_equal(gi, ridx)
    assert np.array_equal(gd.view(np.uint32), rd2.view(np.uint32))
    del idx, d2, q
    torch.cuda.empty_cache()
