"""GPU parity of the batched path: many independent clouds built and searched
in one launch sequence, each cloud against the oracle run on that cloud
alone.  Bit-exact like the single-cloud tests; batches mix sizes (empty, one
point, fewer points than a leaf), curves, leaf sizes, kernels, radii and k."""
import numpy as np
import pytest

import oracle
from paper_2603_06771_amd import datagen
from tests._parity import announce, assert_csr_equal, check_tree

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfc():
    import torch  # noqa: F401
    import paper_2603_06771_amd as sfc
    return sfc


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)).cuda()


# (kind, n, curve, bits, leaf)
MIXED = [
    ("lidar", 20011, "hilbert", 21, 16),
    ("uniform", 0, "morton", 21, 8),
    ("uniform", 1, "hilbert", 21, 8),
    ("dup", 5003, "morton", 21, 8),
    ("uniform", 30011, "morton", 21, 32),
    ("lidar", 7, "hilbert", 21, 128),
    ("uniform", 4096, "hilbert", 7, 4),
    ("lidar", 9001, "morton", 21, 64),
]


def _cloud(kind, n, seed):
    if n == 0:
        return np.zeros((0, 3), np.float32)
    if kind == "uniform":
        return datagen.uniform(n, seed=seed)
    if kind == "lidar":
        return datagen.lidar_tile(n, seed=seed)
    base = datagen.uniform(n - n // 8, seed=seed)
    return datagen.with_duplicates(base, n // 8, seed=seed)


def _mixed_batch(sfc):
    import torch
    clouds = [_cloud(kind, n, 40 + i) for i, (kind, n, _, _, _) in enumerate(MIXED)]
    xyz = np.concatenate(clouds, axis=0)
    batch = sfc.build_batch(_dev(xyz), [c.shape[0] for c in clouds], curve=[m[2] for m in MIXED],
                            bits=[m[3] for m in MIXED], leaf_size=[m[4] for m in MIXED])
    torch.cuda.synchronize()
    return batch, clouds


def test_batch_build(sfc):
    announce("batch build mixed")
    batch, clouds = _mixed_batch(sfc)
    for c, (kind, n, curve, bits, leaf) in enumerate(MIXED):
        announce(f"  cloud {c}: {kind} n={n} {curve} bits={bits} leaf={leaf}")
        check_tree(batch.tree(c), clouds[c], curve, bits, leaf)


def test_batch_of_one_equals_single(sfc):
    import torch
    pts = _cloud("lidar", 30001, 3)
    announce("batch of one vs single build")
    b = sfc.build_batch(_dev(pts), [pts.shape[0]], "hilbert", 21, 16)
    t = sfc.build_linear_octree(_dev(pts), "hilbert", 21, 16)
    torch.cuda.synchronize()
    bt = b.tree(0)
    ia, ib = bt.info(), t.info()
    assert ia == ib
    for name, x in bt.arrays(ia).items():
        assert torch.equal(x, t.arrays(ib)[name]), name
    assert torch.equal(bt.points(), t.points()) and torch.equal(bt.keys(), t.keys())


def _rows(c, o, i, q0, nq):
    """CSR rows [q0, q0 + nq) of a global CSR, re-based to 0."""
    o = o.astype(np.int64)
    a, b = o[q0], o[q0 + nq]
    return c[q0:q0 + nq], o[q0:q0 + nq + 1] - a, i[a:b]


KERN = ["sphere", "square", "cube", "circle", "sphere", "cube", "square", "circle"]
RADII = [1.0, 0.5, 0.05, 0.0, 0.03, 5.0, 0.1, 2.5]


def test_batch_radius_cloud_queries(sfc):
    import torch
    batch, clouds = _mixed_batch(sfc)
    announce("batch radius, cloud queries, mixed kernels and radii")
    c, o, i = sfc.radius_search_batched(batch, None, None, KERN, RADII)
    torch.cuda.synchronize()
    c, o, i = c.cpu().numpy(), o.cpu().numpy(), i.cpu().numpy()
    q0 = 0
    for cl, pts in enumerate(clouds):
        n = pts.shape[0]
        perm = batch.tree(cl).perm().cpu().numpy().view(np.uint32)
        ref = oracle.radius_search(pts, pts[perm], KERN[cl], RADII[cl])
        assert_csr_equal(_rows(c, o, i, q0, n), ref, f"cloud {cl} {KERN[cl]} r={RADII[cl]}")
        q0 += n
    assert q0 == c.size


def test_batch_radius_per_cloud_tile_and_record(sfc):
    """Per-cloud staging tiles and per-cloud recorded fills in one launch
    give the rows of the default batch (same order inside every row), and
    each cloud matches the oracle."""
    import torch
    batch, clouds = _mixed_batch(sfc)
    stages = [64, 256, 128, 256, 64, 128, 256, 64]
    records = [True, False, True, True, False, True, False, True]
    announce("batch radius, per-cloud staging tiles and recorded fills")
    ref = sfc.radius_search_batched(batch, None, None, KERN, RADII)
    got = sfc.radius_search_batched(batch, None, None, KERN, RADII, record=records, stage=stages)
    total = int(ref[1][-1])
    cap = sfc.radius_search_batched(batch, None, None, KERN, RADII, capacity=total, record=records, stage=stages)
    torch.cuda.synchronize()
    for x, y, name in zip(ref, got, ("counts", "offsets", "indices")):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy()), f"{name} differ"
    for x, y, name in zip(ref[:2], cap[:2], ("counts", "offsets")):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy()), f"one call: {name} differ"
    assert np.array_equal(ref[2].cpu().numpy()[:total], cap[2].cpu().numpy()[:total]), "one call: indices differ"
    c, o, i = (x.cpu().numpy() for x in got)
    q0 = 0
    for cl, pts in enumerate(clouds):
        n = pts.shape[0]
        perm = batch.tree(cl).perm().cpu().numpy().view(np.uint32)
        ref_cl = oracle.radius_search(pts, pts[perm], KERN[cl], RADII[cl])
        assert_csr_equal(_rows(c, o, i, q0, n), ref_cl, f"cloud {cl} stage {stages[cl]} record {records[cl]}")
        q0 += n


def test_batch_radius_external_queries(sfc):
    import torch
    batch, clouds = _mixed_batch(sfc)
    rng = np.random.default_rng(7)
    qs = []
    for cl, pts in enumerate(clouds):
        nq = [513, 64, 0, 1000, 2049, 3, 777, 128][cl]
        if pts.shape[0]:
            lo, hi = pts.min(0), pts.max(0)
        else:
            lo, hi = np.zeros(3, np.float32), np.ones(3, np.float32)
        qs.append((lo + (hi - lo) * rng.uniform(-0.1, 1.1, (nq, 3))).astype(np.float32))
    q = np.concatenate(qs, axis=0)
    announce("batch radius, external queries")
    c, o, i = sfc.radius_search_batched(batch, _dev(q), [x.shape[0] for x in qs], KERN, RADII)
    torch.cuda.synchronize()
    c, o, i = c.cpu().numpy(), o.cpu().numpy(), i.cpu().numpy()
    q0 = 0
    for cl, pts in enumerate(clouds):
        ref = oracle.radius_search(pts, qs[cl], KERN[cl], RADII[cl])
        assert_csr_equal(_rows(c, o, i, q0, qs[cl].shape[0]), ref, f"cloud {cl}")
        q0 += qs[cl].shape[0]


def test_batch_radius_capacity(sfc):
    import torch
    batch, clouds = _mixed_batch(sfc)
    announce("batch radius, capacity too small then exact")
    c, o, _ = sfc.radius_search_batched(batch, None, None, "sphere", 0.5, capacity=5, check=False)
    torch.cuda.synchronize()
    total = int(o[-1])
    assert total > 5
    with pytest.raises(sfc.SfcCapacityError) as e:
        sfc.radius_search_batched(batch, None, None, "sphere", 0.5, capacity=total - 1)
    assert e.value.total == total
    c2, o2, i2 = sfc.radius_search_batched(batch, None, None, "sphere", 0.5, capacity=total)
    torch.cuda.synchronize()
    assert torch.equal(c, c2) and torch.equal(o, o2)
    c2, o2, i2 = c2.cpu().numpy(), o2.cpu().numpy(), i2.cpu().numpy()
    q0 = 0
    for cl, pts in enumerate(clouds):
        perm = batch.tree(cl).perm().cpu().numpy().view(np.uint32)
        ref = oracle.radius_search(pts, pts[perm], "sphere", 0.5)
        assert_csr_equal(_rows(c2, o2, i2, q0, pts.shape[0]), ref, f"cloud {cl}")
        q0 += pts.shape[0]


KS = [8, 3, 1, 32, 16, 4, 12, 24]
KS64 = [8, 3, 1, 48, 16, 64, 12, 40]  # largest k of the register kernel


@pytest.mark.parametrize("ks,kstride", [(KS, 32), (KS64, 64)])
@pytest.mark.parametrize("external", [False, True])
def test_batch_knn(sfc, external, ks, kstride):
    import torch
    batch, clouds = _mixed_batch(sfc)
    rng = np.random.default_rng(9)
    if external:
        qs = [rng.uniform(-0.1, 1.1, (m, 3)).astype(np.float32) * (p.max(0) - p.min(0) if p.shape[0] else 1)
              + (p.min(0) if p.shape[0] else 0)
              for p, m in zip(clouds, [300, 10, 5, 700, 64, 9, 1025, 0])]
        qs = [np.ascontiguousarray(x, dtype=np.float32) for x in qs]
        q = _dev(np.concatenate(qs, axis=0))
        q_sizes = [x.shape[0] for x in qs]
    else:
        qs, q, q_sizes = None, None, None
    announce(f"batch knn mixed k (max {max(ks)}), external={external}")
    idx, d2 = sfc.knn_search_batched(batch, q, q_sizes, ks, kstride=kstride)
    torch.cuda.synchronize()
    gi = idx.cpu().numpy().view(np.uint32)
    gd = d2.cpu().numpy()
    q0 = 0
    for cl, pts in enumerate(clouds):
        if external:
            qp = qs[cl]
        else:
            perm = batch.tree(cl).perm().cpu().numpy().view(np.uint32)
            qp = pts[perm]
        k = ks[cl]
        ridx, rd2 = oracle.knn(pts, qp, k)
        rows = slice(q0, q0 + qp.shape[0])
        assert np.array_equal(gi[rows, :k], ridx), f"cloud {cl} k={k}: indices differ"
        assert np.array_equal(gd[rows, :k].view(np.uint32), rd2.view(np.uint32)), f"cloud {cl}: d2 differ"
        assert np.all(gi[rows, k:] == 0xFFFFFFFF) and np.all(np.isinf(gd[rows, k:]))
        q0 += qp.shape[0]


def test_many_small_clouds(sfc):
    """More clouds than one sort digit covers (two cloud passes) and than one
    table upload carries."""
    import torch
    rng = np.random.default_rng(datagen.SEED_BATCH)
    B = 300
    sizes = np.exp(rng.uniform(np.log(10), np.log(3000), B)).astype(np.int64)
    sizes[17] = 0
    clouds = [datagen.uniform(int(n), seed=1000 + c) if n else np.zeros((0, 3), np.float32)
              for c, n in enumerate(sizes)]
    curves = ["hilbert" if c % 2 else "morton" for c in range(B)]
    leafs = [int(x) for x in rng.choice([4, 16, 32], B)]
    kern = [["sphere", "circle", "cube", "square"][c % 4] for c in range(B)]
    radii = [float(x) for x in rng.uniform(0.02, 0.15, B)]
    announce(f"batch of {B} small clouds: build")
    batch = sfc.build_batch(_dev(np.concatenate(clouds)), sizes.tolist(), curves, 21, leafs)
    torch.cuda.synchronize()
    for c in range(0, B, 7):
        check_tree(batch.tree(c), clouds[c], curves[c], 21, leafs[c])
    announce(f"batch of {B} small clouds: radius")
    cc, oo, ii = sfc.radius_search_batched(batch, None, None, kern, radii)
    ks = [int(x) for x in rng.choice([1, 8, 16, 32], B)]
    announce(f"batch of {B} small clouds: knn")
    idx, d2 = sfc.knn_search_batched(batch, None, None, ks, kstride=32)
    torch.cuda.synchronize()
    cc, oo, ii = cc.cpu().numpy(), oo.cpu().numpy(), ii.cpu().numpy()
    gi, gd = idx.cpu().numpy().view(np.uint32), d2.cpu().numpy()
    q0 = 0
    for c in range(B):
        pts = clouds[c]
        n = pts.shape[0]
        perm = batch.tree(c).perm().cpu().numpy().view(np.uint32)
        assert np.array_equal(np.sort(perm), np.arange(n, dtype=np.uint32))
        ref = oracle.radius_search(pts, pts[perm], kern[c], radii[c])
        assert_csr_equal(_rows(cc, oo, ii, q0, n), ref, f"cloud {c}")
        ridx, rd2 = oracle.knn(pts, pts[perm], ks[c])
        assert np.array_equal(gi[q0:q0 + n, :ks[c]], ridx), f"cloud {c}: knn indices"
        assert np.array_equal(gd[q0:q0 + n, :ks[c]].view(np.uint32), rd2.view(np.uint32)), f"cloud {c}: knn d2"
        q0 += n


@pytest.mark.slow
@pytest.mark.parametrize("record", [False, True])
def test_batch_mix_largest_clouds(sfc, record):
    """The four largest clouds of the 256-cloud batch mix (1.76M-1.86M points,
    uniform and LiDAR, cube and circle kernels, r = 1.4-2.3 m) and its four
    smallest, built and searched in one batch as the batched benchmark runs
    them (Hilbert, leaf 64 and 128): every row's count against the oracle's,
    sampled rows and k-NN rows element by element."""
    import torch
    specs = datagen.batch_mix_specs(256, seed=datagen.SEED_BATCH)
    order = sorted(range(len(specs)), key=lambda i: specs[i]["n"])
    pick = order[-4:] + order[:4]
    sp = [specs[i] for i in pick]
    clouds = [datagen.batch_cloud(s) for s in sp]
    sizes = [c.shape[0] for c in clouds]
    leafs = [64, 128, 64, 128, 64, 128, 64, 128]
    kern = [s["kernel"] for s in sp]
    radii = [s["radius"] for s in sp]
    announce(f"batch mix largest/smallest clouds {sizes} record={record}")
    batch = sfc.build_batch(_dev(np.concatenate(clouds)), sizes, "hilbert", 21, leafs)
    c, o, i = sfc.radius_search_batched(batch, None, None, kern, radii, record=record)
    torch.cuda.synchronize()
    c, o = c.cpu().numpy(), o.cpu().numpy()
    rng = np.random.default_rng(23)
    q0 = 0
    for cl, pts in enumerate(clouds):
        n = pts.shape[0]
        perm = batch.tree(cl).perm().cpu().numpy().view(np.uint32)
        dims = 2 if kern[cl] in ("circle", "square") else 3
        grid = oracle.Grid(pts, radii[cl], dims)
        rc = grid.radius_count(pts, kern[cl], radii[cl])
        got = c[q0:q0 + n].view(np.uint32)
        bad = np.nonzero(got != rc[perm])[0]
        assert bad.size == 0, f"cloud {cl}: {bad.size} counts differ"
        rows = np.sort(rng.choice(n, min(n, 300), replace=False))
        ref_c, ref_o, ref_i = grid.radius_search(pts[perm[rows]], kern[cl], radii[cl])
        for k, row in enumerate(rows):
            a, b = int(o[q0 + row]), int(o[q0 + row + 1])
            g = np.sort(i[a:b].cpu().numpy().view(np.uint32))
            assert np.array_equal(g, ref_i[ref_o[k]:ref_o[k + 1]]), f"cloud {cl} row {row}"
        del grid
        q0 += n
    del i
    torch.cuda.empty_cache()
    if record:
        return
    ks = [16, 32, 8, 16, 32, 8, 16, 32]
    announce("batch mix largest/smallest clouds: knn")
    idx, d2 = sfc.knn_search_batched(batch, None, None, ks, kstride=32)
    torch.cuda.synchronize()
    q0 = 0
    for cl, pts in enumerate(clouds):
        n = pts.shape[0]
        perm = batch.tree(cl).perm().cpu().numpy().view(np.uint32)
        rows = np.sort(rng.choice(n, min(n, 500), replace=False))
        ridx, rd2 = oracle.knn(pts, pts[perm[rows]], ks[cl])
        sel = torch.from_numpy(q0 + rows).cuda()
        gi = idx[sel].cpu().numpy().view(np.uint32)
        gd = d2[sel].cpu().numpy()
        assert np.array_equal(gi[:, :ks[cl]], ridx), f"cloud {cl}: knn indices"
        assert np.array_equal(gd[:, :ks[cl]].view(np.uint32), rd2.view(np.uint32)), f"cloud {cl}: knn d2"
        q0 += n
