"""The serving loop: every request's result is the same when it runs alone
(single-cloud call on the resident tree) and when it runs in a batch with
other requests, in the continuous-batching server and in the one-request
FIFO server; a sample is also checked against the oracle.  Also the memory
admission of clouds and the path that regrows an output buffer whose size
estimate was too small."""
import numpy as np
import pytest

import oracle
from paper_2603_06771_amd import datagen
from tests._parity import announce, assert_csr_equal

pytestmark = pytest.mark.gpu

SIZES = [60001, 150000, 9000, 200003]


@pytest.fixture(scope="module")
def world():
    import torch  # noqa: F401
    from paper_2603_06771_amd import serve
    clouds = [datagen.lidar_tile(n, seed=datagen.SEED_SERVED + 1 + i) for i, n in enumerate(SIZES)]
    res = serve.Resident(budget_bytes=1 << 32, curve="hilbert", leaf_size=32)
    ids = res.admit(clouds)
    assert ids == [0, 1, 2, 3]
    reqs = []
    for d in datagen.request_stream(48, len(SIZES), SIZES, rate_per_s=4000.0, q_min=10, q_max=6000):
        reqs.append(serve.Request(id=d["id"], arrival=d["arrival"], cloud=d["cloud"], rows=d["rows"], op=d["op"],
                                  kernel=d.get("kernel", "sphere"), radius=d.get("radius", 1.0), k=d.get("k", 8)))
    return serve, res, clouds, reqs


def _alone(sfc, res, clouds, r):
    import torch
    q = torch.from_numpy(np.ascontiguousarray(clouds[r.cloud][r.rows])).cuda()
    t = res.octree(r.cloud)
    if r.op == "radius":
        c, o, i = sfc.radius_search(t, q, r.kernel, r.radius)
        torch.cuda.synchronize()
        return c.cpu().numpy(), o.cpu().numpy(), i.cpu().numpy()
    idx, d2 = sfc.knn_search(t, q, r.k)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), d2.cpu().numpy()


def _collect(store):
    def on_result(r, res):
        store[r.id] = tuple(x.cpu().numpy() for x in res)
    return on_result


def _same(a, b, r):
    if r.op == "radius":
        assert_csr_equal(a, (b[0], b[1], _rowsorted(b)), f"request {r.id}")
    else:
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32)), \
            f"request {r.id}"


def _rowsorted(csr):
    from tests._parity import sorted_csr
    return sorted_csr(*csr)


@pytest.mark.parametrize("mode", ["continuous", "fifo", "regrow"])
def test_alone_equals_mix(world, mode):
    import paper_2603_06771_amd as sfc
    serve, res, clouds, reqs = world
    out = 1 << 22 if mode != "regrow" else 2000
    srv = serve.Server(res, slots=1 if mode == "fifo" else 2, max_requests=16, max_queries=1 << 16,
                       out_entries=out)
    got = {}
    announce(f"serve {mode}: run")
    stats = srv.run(reqs, on_result=_collect(got), max_requests=1 if mode == "fifo" else None)
    assert len(got) == len(reqs) and np.all(stats["latency_s"] > 0)
    if mode == "continuous":
        assert stats["batches"] < len(reqs)  # requests were batched
    if mode == "regrow":
        assert stats["regrown"] > 0
    announce(f"serve {mode}: alone")
    for r in reqs:
        alone = _alone(sfc, res, clouds, r)
        _same(got[r.id], alone, r)


def test_mix_matches_oracle_sample(world):
    serve, res, clouds, reqs = world
    srv = serve.Server(res, slots=2, max_requests=16, max_queries=1 << 16, out_entries=1 << 22)
    got = {}
    announce("serve: oracle sample")
    srv.run(reqs, on_result=_collect(got))
    for r in reqs[:12]:
        pts = clouds[r.cloud]
        q = pts[r.rows]
        if r.op == "radius":
            ref = oracle.radius_search(pts, q, r.kernel, r.radius)
            assert_csr_equal(got[r.id], ref, f"request {r.id}")
        else:
            ridx, rd2 = oracle.knn(pts, q, r.k)
            assert np.array_equal(got[r.id][0].view(np.uint32), ridx)
            assert np.array_equal(got[r.id][1].view(np.uint32), rd2.view(np.uint32))


def test_cloud_admission_by_memory():
    import torch  # noqa: F401
    from paper_2603_06771_amd import serve
    a = datagen.lidar_tile(50000, seed=1)
    b = datagen.lidar_tile(80000, seed=2)
    res = serve.Resident(budget_bytes=1 << 62, compact=False)
    need_a = res.bytes_for([a.shape[0]])
    need_b = res.bytes_for([b.shape[0]])
    res = serve.Resident(budget_bytes=need_a + need_b // 2, compact=False)
    announce("serve: admission")
    assert res.admit([a]) == [0]
    assert res.admit([b]) is None and res.used == need_a   # does not fit: nothing allocated
    res.drop(0)
    assert res.used == 0
    assert res.admit([b]) == [1]


def test_compacted_trees_admit_more_with_same_results():
    """Trees copied into exactly the memory their actual sizes need
    (octree_batch_compact): the same budget holds more clouds, and searches
    on the copies give the rows of the trees built in place."""
    import torch
    import paper_2603_06771_amd as sfc
    from paper_2603_06771_amd import serve
    clouds = [datagen.lidar_tile(60000, seed=90 + i) for i in range(6)]
    need = serve.Resident(budget_bytes=1 << 62).bytes_for([60000])
    budget = int(2.2 * need)
    announce("serve: admission with and without compaction")
    loose = serve.Resident(budget_bytes=budget, compact=False)
    tight = serve.Resident(budget_bytes=budget, compact=True)
    n_loose = sum(loose.admit([c]) is not None for c in clouds)
    n_tight = sum(tight.admit([c]) is not None for c in clouds)
    assert n_loose == 2 and n_tight > n_loose
    assert tight.used < 0.5 * n_tight * need
    for cid in range(n_loose):
        t0, t1 = loose.octree(cid), tight.octree(cid)
        for kernel, r in (("sphere", 1.5), ("square", 0.7)):
            a = sfc.radius_search(t0, None, kernel, r, record=True)
            b = sfc.radius_search(t1, None, kernel, r, record=True)
            torch.cuda.synchronize()
            for x, y in zip(a, b):
                assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
        i0, d0 = sfc.knn_search(t0, None, 16)
        i1, d1 = sfc.knn_search(t1, None, 16)
        torch.cuda.synchronize()
        assert np.array_equal(i0.cpu().numpy(), i1.cpu().numpy())
        assert np.array_equal(d0.cpu().numpy().view(np.uint32), d1.cpu().numpy().view(np.uint32))
    # an empty cloud and a one-point cloud compact too
    announce("serve: compaction of an empty and a one-point cloud")
    small = serve.Resident(budget_bytes=1 << 30, compact=True)
    assert small.admit([np.zeros((0, 3), np.float32), a_point()]) == [0, 1]
    c, o, i = sfc.radius_search(small.octree(1), None, "sphere", 1.0)
    torch.cuda.synchronize()
    assert int(o[-1]) == 1


def a_point():
    return np.array([[1.0, 2.0, 3.0]], np.float32)
