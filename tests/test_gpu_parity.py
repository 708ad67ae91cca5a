"""GPU parity: every stage of the HIP path against the CPU oracle on the same
seeded inputs.  Bit-exact throughout: codes, permutation, octree arrays,
neighbour sets and k-NN lists (integer results and fp32 values computed by the
same fixed expressions on both sides)."""
import numpy as np
import pytest

import oracle
from paper_2603_06771_amd import datagen
from tests._parity import announce, assert_csr_equal, check_tree

pytestmark = pytest.mark.gpu

CURVES = ["morton", "hilbert"]
KERNELS = ["sphere", "circle", "cube", "square"]


@pytest.fixture(scope="module")
def sfc():
    import torch  # noqa: F401
    import paper_2603_06771_amd as sfc
    return sfc


def _cloud(kind, n, seed=3):
    if kind == "uniform":
        return datagen.uniform(n, seed=seed)
    if kind == "lidar":
        return datagen.lidar_tile(n, seed=seed)
    base = datagen.uniform(n - n // 8, seed=seed)
    return datagen.with_duplicates(base, n // 8, seed=seed)


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("curve", CURVES)
@pytest.mark.parametrize("kind,n", [("uniform", 1), ("uniform", 4097), ("lidar", 100003), ("dup", 30011)])
@pytest.mark.parametrize("bits", [21, 7])
def test_encode(sfc, curve, kind, n, bits):
    announce(f"encode {curve} {kind} n={n} bits={bits}")
    pts = _cloud(kind, n)
    keys, frame = sfc.encode_sfc(_dev(pts), curve, bits)
    import torch
    torch.cuda.synchronize()
    rk, lo, s = oracle.encode(pts, curve, bits)
    assert np.array_equal(_u64(keys), rk)
    f = np.frombuffer(frame.cpu().numpy().tobytes(), dtype=np.float32, count=4)
    assert np.array_equal(f[:3], lo) and f[3] == s


def test_encode_empty(sfc):
    import torch
    keys, frame = sfc.encode_sfc(torch.zeros((0, 3), dtype=torch.float32, device="cuda"), "hilbert", 21)
    torch.cuda.synchronize()
    f = np.frombuffer(frame.cpu().numpy().tobytes(), dtype=np.float32, count=4)
    assert keys.numel() == 0 and list(f) == [0, 0, 0, 2.0 ** 21]


def _check_tree(sfc, pts, curve, bits, leaf):
    import torch
    t = sfc.build_linear_octree(_dev(pts), curve, bits, leaf)
    torch.cuda.synchronize()
    check_tree(t, pts, curve, bits, leaf)
    return t


@pytest.mark.parametrize("curve", CURVES)
@pytest.mark.parametrize("kind,n,leaf", [("uniform", 100003, 32), ("lidar", 65537, 16), ("dup", 20000, 8),
                                         ("lidar", 9000, 128), ("uniform", 5, 8), ("uniform", 0, 8)])
def test_build(sfc, curve, kind, n, leaf):
    announce(f"build {curve} {kind} n={n} leaf={leaf}")
    pts = _cloud(kind, n) if n else np.zeros((0, 3), np.float32)
    _check_tree(sfc, pts, curve, 21, leaf)


def test_build_coarse_levels(sfc):
    # few levels: many level-L leaves above the threshold (duplicate cells)
    announce("build coarse bits=3")
    pts = _cloud("dup", 5000)
    _check_tree(sfc, pts, "hilbert", 3, 4)
    _check_tree(sfc, pts, "morton", 2, 16)


def _radius_case(sfc, pts, curve, leaf, kernel, r, queries=None, prune=True):
    import torch
    t = sfc.build_linear_octree(_dev(pts), curve, 21, leaf)
    q = None if queries is None else _dev(queries)
    c, o, i = sfc.radius_search(t, q, kernel, r, prune=prune)
    torch.cuda.synchronize()
    perm = t.perm().cpu().numpy().view(np.uint32)
    qpts = pts[perm] if queries is None else queries
    ref = oracle.radius_search(pts, qpts, kernel, r)
    assert_csr_equal((c.cpu().numpy(), o.cpu().numpy(), i.cpu().numpy()), ref, f"{kernel} r={r}")
    return c, o, i


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("curve", CURVES)
def test_radius_lidar(sfc, kernel, curve):
    pts = _cloud("lidar", 60001, seed=11)
    for r in (0.5, 1.0, 3.0):
        announce(f"radius lidar {kernel} {curve} r={r}")
        _radius_case(sfc, pts, curve, 32, kernel, r)


@pytest.mark.parametrize("kernel", KERNELS)
def test_radius_uniform_small_config(sfc, kernel):
    # the 100k uniform configuration: Morton, leaf 32, r = 0.01 (and a larger r)
    pts = _cloud("uniform", 100000, seed=datagen.SEED_UNIFORM)
    for r in (0.01, 0.0212):
        announce(f"radius uniform100k {kernel} r={r}")
        _radius_case(sfc, pts, "morton", 32, kernel, r)


@pytest.mark.parametrize("leaf", [1, 8, 64, 200])
def test_radius_leaf_sizes_and_duplicates(sfc, leaf):
    pts = _cloud("dup", 20000, seed=5)
    for kernel in ("sphere", "square"):
        announce(f"radius dup leaf={leaf} {kernel}")
        _radius_case(sfc, pts, "hilbert", leaf, kernel, 0.03)


def test_radius_nonpositive_and_tiny(sfc):
    pts = _cloud("uniform", 3000, seed=2)
    for r in (0.0, -1.0, 1e-30):
        announce(f"radius r={r}")
        c, o, i = _radius_case(sfc, pts, "morton", 8, "cube", r)
        if r <= 0:
            assert int(o[-1]) == 0


def test_radius_external_queries(sfc):
    rng = np.random.default_rng(4)
    pts = _cloud("lidar", 40000, seed=8)
    lo, hi = pts.min(0), pts.max(0)
    q = (lo + (hi - lo) * rng.uniform(-0.1, 1.1, (7001, 3))).astype(np.float32)
    for kernel in KERNELS:
        announce(f"radius external {kernel}")
        _radius_case(sfc, pts, "hilbert", 32, kernel, 2.0, queries=q)


@pytest.mark.parametrize("kernel", KERNELS)
def test_radius_sparse_queries(sfc, kernel):
    # queries far apart (a small random subset of the cloud, and points off
    # the cloud): waves take their queries one at a time
    rng = np.random.default_rng(21)
    pts = _cloud("lidar", 100000, seed=22)
    sub = pts[np.sort(rng.choice(pts.shape[0], 700, replace=False))]
    lo, hi = pts.min(0), pts.max(0)
    off = (lo + (hi - lo) * rng.uniform(-0.05, 1.05, (300, 3))).astype(np.float32)
    q = np.concatenate([sub, off]).astype(np.float32)
    for r in (0.3, 1.5, 3.0):
        announce(f"radius sparse queries {kernel} r={r}")
        _radius_case(sfc, pts, "hilbert", 16, kernel, r, queries=q)
        announce(f"radius sparse queries {kernel} r={r} no-prune")
        _radius_case(sfc, pts, "morton", 32, kernel, r, queries=q, prune=False)


@pytest.mark.parametrize("curve", CURVES)
def test_radius_georeferenced(sfc, curve):
    # a tile at map coordinates: fp32 spacing 0.03 m in x and 0.5 m in y, so
    # the arithmetic rounds coarsely and many points coincide (the walk's
    # start node and every exactness argument must still hold)
    pts = _cloud("lidar", 30000, seed=31)
    geo = (pts.astype(np.float64) + np.array([512345.5, 4312345.25, 120.0])).astype(np.float32)
    for kernel in KERNELS:
        for r in (0.5, 2.0):
            announce(f"radius georeferenced {curve} {kernel} r={r}")
            _radius_case(sfc, geo, curve, 32, kernel, r)
    announce(f"knn georeferenced {curve}")
    _knn_case(sfc, geo, curve, 32, 16)


def test_radius_degenerate_clouds(sfc):
    # every point the same (zero extent), points on a line (zero extent in y
    # and z), a single point: frames, cells, start nodes and ties
    rng = np.random.default_rng(33)
    same = np.tile(np.array([[3.25, -1.5, 7.0]], np.float32), (3000, 1))
    line = np.zeros((4000, 3), np.float32)
    line[:, 0] = np.sort(rng.uniform(0.0, 40.0, 4000)).astype(np.float32)
    one = np.array([[0.5, 0.5, 0.5]], np.float32)
    for name, pts in (("same", same), ("line", line), ("one", one)):
        for kernel in KERNELS:
            announce(f"radius degenerate {name} {kernel}")
            _radius_case(sfc, pts, "hilbert", 16, kernel, 0.3)
        announce(f"knn degenerate {name}")
        _knn_case(sfc, pts, "morton", 16, 8)


def test_radius_no_prune_flag(sfc):
    pts = _cloud("lidar", 30000, seed=9)
    announce("radius no-prune")
    _radius_case(sfc, pts, "morton", 16, "sphere", 2.5, prune=False)


def test_radius_capacity_protocol(sfc):
    import torch
    pts = _cloud("uniform", 20000, seed=6)
    t = sfc.build_linear_octree(_dev(pts), "morton", 21, 32)
    announce("radius capacity too small")
    c, o, i = sfc.radius_search(t, None, "sphere", 0.05, capacity=10, check=False)
    torch.cuda.synchronize()
    total = int(o[-1])
    assert total > 10
    # the checked form raises, with the capacity a second call needs
    with pytest.raises(sfc.SfcCapacityError) as e:
        sfc.radius_search(t, None, "sphere", 0.05, capacity=total - 1)
    assert e.value.total == total
    # nothing written: the buffer keeps whatever it held, the counts are valid
    c2, o2, i2 = sfc.radius_search(t, None, "sphere", 0.05, capacity=total)
    torch.cuda.synchronize()
    assert torch.equal(c, c2) and torch.equal(o, o2)
    perm = t.perm().cpu().numpy().view(np.uint32)
    ref = oracle.radius_search(pts, pts[perm], "sphere", 0.05)
    assert_csr_equal((c2.cpu().numpy(), o2.cpu().numpy(), i2.cpu().numpy()), ref, "capacity")


def test_radius_deterministic(sfc):
    import torch
    pts = _cloud("lidar", 50000, seed=10)
    t = sfc.build_linear_octree(_dev(pts), "hilbert", 21, 32)
    announce("radius determinism")
    a = sfc.radius_search(t, None, "sphere", 1.5)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = sfc.radius_search(t, None, "sphere", 1.5)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def _knn_case(sfc, pts, curve, leaf, k, queries=None):
    import torch
    t = sfc.build_linear_octree(_dev(pts), curve, 21, leaf)
    q = None if queries is None else _dev(queries)
    idx, d2 = sfc.knn_search(t, q, k)
    torch.cuda.synchronize()
    perm = t.perm().cpu().numpy().view(np.uint32)
    qpts = pts[perm] if queries is None else queries
    ridx, rd2 = oracle.knn(pts, qpts, k)
    gi = idx.cpu().numpy().view(np.uint32)
    gd = d2.cpu().numpy()
    bad = np.nonzero(np.any(gi != ridx, axis=1) | np.any(gd.view(np.uint32) != rd2.view(np.uint32), axis=1))[0]
    assert bad.size == 0, f"k={k}: {bad.size} rows differ, first {bad[0]}: gpu {gi[bad[0]]} {gd[bad[0]]} " \
                          f"oracle {ridx[bad[0]]} {rd2[bad[0]]}"


@pytest.mark.parametrize("k", [1, 5, 8, 16, 32, 33, 48, 64])
@pytest.mark.parametrize("curve", CURVES)
def test_knn_lidar(sfc, k, curve):
    pts = _cloud("lidar", 40001, seed=12)
    announce(f"knn lidar k={k} {curve}")
    _knn_case(sfc, pts, curve, 32, k)


@pytest.mark.parametrize("k", [1, 8, 32, 64])
def test_knn_sparse_queries(sfc, k):
    # queries far apart: waves take them one at a time
    rng = np.random.default_rng(23)
    pts = _cloud("lidar", 100000, seed=24)
    sub = pts[np.sort(rng.choice(pts.shape[0], 900, replace=False))]
    lo, hi = pts.min(0), pts.max(0)
    off = (lo + (hi - lo) * rng.uniform(-0.05, 1.05, (200, 3))).astype(np.float32)
    q = np.concatenate([sub, off]).astype(np.float32)
    announce(f"knn sparse queries k={k}")
    _knn_case(sfc, pts, "hilbert", 16, k, queries=q)
    announce(f"knn sparse queries k={k}, duplicates")
    dup = _cloud("dup", 30000, seed=25)
    _knn_case(sfc, dup, "morton", 8, k, queries=dup[np.sort(rng.choice(dup.shape[0], 500, replace=False))])


@pytest.mark.parametrize("k", [65, 100, 300, 512])
def test_knn_large_k(sfc, k):
    # k above the register lists: one query per wave, LDS candidate buffer
    pts = _cloud("lidar", 20000, seed=26)
    announce(f"knn large k={k}")
    _knn_case(sfc, pts, "hilbert", 64, k)
    rng = np.random.default_rng(27)
    lo, hi = pts.min(0), pts.max(0)
    q = (lo + (hi - lo) * rng.uniform(-0.05, 1.05, (700, 3))).astype(np.float32)
    announce(f"knn large k={k}, external queries")
    _knn_case(sfc, pts, "morton", 16, k, queries=q)


def test_knn_large_k_small_cloud_and_ties(sfc):
    announce("knn large k, k > n and duplicates")
    _knn_case(sfc, _cloud("uniform", 150, seed=28), "hilbert", 8, 200)
    _knn_case(sfc, _cloud("dup", 5000, seed=29), "morton", 8, 96)


def test_knn_duplicates_ties(sfc):
    pts = _cloud("dup", 20000, seed=13)
    for k in (4, 16, 32, 64):
        announce(f"knn dup k={k}")
        _knn_case(sfc, pts, "hilbert", 8, k)


def test_knn_external_and_padding(sfc):
    rng = np.random.default_rng(5)
    pts = _cloud("uniform", 30000, seed=14)
    q = rng.uniform(-0.2, 1.2, (5003, 3)).astype(np.float32)
    announce("knn external")
    _knn_case(sfc, pts, "morton", 32, 16, queries=q)
    announce("knn k > n")
    small = _cloud("uniform", 11, seed=3)
    _knn_case(sfc, small, "hilbert", 4, 32)


@pytest.mark.parametrize("stage", [64, 256])
@pytest.mark.parametrize("kernel", KERNELS)
def test_radius_staging_tiles(sfc, stage, kernel):
    """Every staging tile gives the oracle's sets, and the same rows in the
    same order as the default tile (count + search fill, and recorded hits),
    for cloud queries and for external queries the call sorts."""
    import torch
    pts = datagen.lidar_tile(50021, seed=31)
    t = sfc.build_linear_octree(_dev(pts), "hilbert", 21, 32)
    perm = t.perm().cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(32)
    ext = (pts[rng.choice(pts.shape[0], 7001, replace=False)] + rng.normal(0, 0.3, (7001, 3))).astype(np.float32)
    for queries, qpts in ((None, pts[perm]), (ext, ext)):
        for r in (0.5, 2.5):
            for record in (False, True):
                announce(f"staging tile {stage} {kernel} r={r} record={record} external={queries is not None}")
                q = None if queries is None else _dev(queries)
                ref = sfc.radius_search(t, q, kernel, r, record=record)
                got = sfc.radius_search(t, q, kernel, r, record=record, stage=stage)
                torch.cuda.synchronize()
                for x, y, name in zip(ref, got, ("counts", "offsets", "indices")):
                    assert np.array_equal(x.cpu().numpy(), y.cpu().numpy()), f"{name} differ from stage 128"
                if not record:
                    assert_csr_equal(tuple(x.cpu().numpy() for x in got), oracle.radius_search(pts, qpts, kernel, r),
                                     f"stage {stage} {kernel} r={r}")
