"""CPU checks of the host-side logic around the kernels: request batching of
the server, the admission estimate, and the seeded request / cloud
generators."""
import collections

import numpy as np

from paper_2603_06771_amd import datagen


def _server_stub(max_requests, max_queries, out_entries):
    from paper_2603_06771_amd import serve
    s = serve.Server.__new__(serve.Server)
    s.max_requests, s.max_queries, s.out_entries = max_requests, max_queries, out_entries
    return s


def _req(i, nq, est):
    from paper_2603_06771_amd import serve
    return serve.Request(id=i, arrival=0.0, cloud=0, rows=np.arange(nq), op="radius", est_out=est)


def test_batches_take_the_queue_head_within_limits():
    srv = _server_stub(max_requests=3, max_queries=100, out_entries=1000)
    q = collections.deque([_req(0, 40, 10), _req(1, 40, 10), _req(2, 40, 10), _req(3, 5, 10)])
    b = srv._take(q)
    assert [r.id for r in b] == [0, 1]          # a third would exceed 100 queries
    b = srv._take(q)
    assert [r.id for r in b] == [2, 3]
    assert not q
    # the request count limit
    q = collections.deque([_req(i, 1, 1) for i in range(7)])
    assert [r.id for r in srv._take(q)] == [0, 1, 2]
    # output budget
    srv = _server_stub(max_requests=8, max_queries=10**6, out_entries=25)
    q = collections.deque([_req(0, 1, 10), _req(1, 1, 10), _req(2, 1, 10)])
    assert [r.id for r in srv._take(q)] == [0, 1]
    # a request larger than every limit still runs (alone)
    srv = _server_stub(max_requests=4, max_queries=10, out_entries=5)
    q = collections.deque([_req(0, 50, 500), _req(1, 1, 1)])
    assert [r.id for r in srv._take(q)] == [0]
    assert [r.id for r in srv._take(q)] == [1]


def test_neighbour_estimate():
    from paper_2603_06771_amd.serve import estimate_neighbours
    for k in ("sphere", "circle", "cube", "square"):
        a = [estimate_neighbours(k, r) for r in (0.5, 1.0, 2.0, 3.0)]
        assert all(x < y for x, y in zip(a, a[1:]))
    assert estimate_neighbours("cube", 1.0) > estimate_neighbours("sphere", 1.0)


def test_request_stream():
    sizes = [5000, 20000, 300]
    a = datagen.request_stream(60, 3, sizes, rate_per_s=100.0, q_min=10, q_max=4000)
    b = datagen.request_stream(60, 3, sizes, rate_per_s=100.0, q_min=10, q_max=4000)
    c = datagen.request_stream(60, 3, sizes, rate_per_s=400.0, q_min=10, q_max=4000)
    t = [r["arrival"] for r in a]
    assert all(x < y for x, y in zip(t, t[1:]))
    for ra, rb, rc in zip(a, b, c):
        assert ra["cloud"] == rb["cloud"] == rc["cloud"] and np.array_equal(ra["rows"], rb["rows"])
        assert np.isclose(ra["arrival"], 4.0 * rc["arrival"])
        rows = ra["rows"]
        assert rows.size >= 1 and rows.size <= min(4000, sizes[ra["cloud"]])
        assert np.all(np.diff(rows) > 0) and rows[0] >= 0 and rows[-1] < sizes[ra["cloud"]]
        if ra["op"] == "radius":
            assert ra["kernel"] in ("sphere", "circle", "cube", "square") and 0.5 <= ra["radius"] <= 3.0
        else:
            assert ra["k"] in (8, 16, 32)
    ops = [r["op"] for r in a]
    assert 0 < ops.count("knn") < len(ops)


def test_sampling_without_replacement_covers_small_clouds():
    rng = np.random.default_rng(0)
    for n, k in ((10, 10), (100, 60), (10**6, 1000)):
        rows = datagen._sample_rows(rng, n, k)
        assert rows.size == k and np.unique(rows).size == k and rows.min() >= 0 and rows.max() < n


def test_served_and_batch_generators():
    s = datagen.served_sizes(8)
    assert len(s) == 8 and all(3.5e6 <= x <= 9e6 for x in s)
    assert s == datagen.served_sizes(8)
    m = datagen.batch_mix(4, n_min=1000, n_max=3000)
    for c in m:
        n = c["points"].shape[0]
        assert 1000 <= n <= 3000 and c["points"].dtype == np.float32
        assert c["kernel"] in ("sphere", "circle", "cube", "square") and 0.5 <= c["radius"] <= 3.0
        if c["kind"] == "uniform":
            side = n ** (1.0 / 3.0)
            assert c["points"].min() >= 0.0 and c["points"].max() <= side


def test_source_sha_ignores_comments_only(tmp_path):
    """The traffic record is tied to the kernel code: comment and whitespace
    edits keep its hash, a code change voids it."""
    from paper_2603_06771_amd.rocprof_summary import source_sha
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("// header\nint f(int x) {\n    return x + 1;  // one\n}\n/* block\n comment */\n")
    b.write_text("// another header\n\nint f(int x) {\n  return x + 1;\n}\n")
    c.write_text("// header\nint f(int x) {\n    return x + 2;  // one\n}\n")
    assert source_sha(str(a)) == source_sha(str(b))
    assert source_sha(str(a)) != source_sha(str(c))


def test_stage_record_sums_the_stage_kernels(tmp_path):
    """Stage traffic: counters of every dispatch of the named kernels (and no
    other), scaled by the calibration copy, divided by the stage count."""
    from paper_2603_06771_amd.rocprof_summary import COPY_BYTES, stage_record
    half_kib = COPY_BYTES // 2 / 1024
    head = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    rows_f = [(1, "__amd_rocclr_copyBuffer", half_kib / 2),  # counter reads half: scale 2
              (2, "sfc::k_radius_fill_rec(sfc::SearchArgs)", 100.0),
              (3, "sfc::k_radius_fill_rows(sfc::SearchArgs)", 300.0),
              (4, "sfc::k_radius_fill(sfc::SearchArgs)", 50.0),
              (5, "sfc::k_radius_count_rec(sfc::SearchArgs)", 1000.0)]
    rows_w = [(1, "__amd_rocclr_copyBuffer", half_kib), (2, "sfc::k_radius_fill_rec(sfc::SearchArgs)", 10.0),
              (3, "sfc::k_radius_fill_rows(sfc::SearchArgs)", 30.0),
              (4, "sfc::k_radius_fill(sfc::SearchArgs)", 0.0),
              (5, "sfc::k_radius_count_rec(sfc::SearchArgs)", 7.0)]
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    f.write_text(head + "".join(f"{d},\"{k}\",FETCH_SIZE,{v}\n" for d, k, v in rows_f))
    w.write_text(head + "".join(f"{d},\"{k}\",WRITE_SIZE,{v}\n" for d, k, v in rows_w))
    src = tmp_path / "s.hip"
    src.write_text("int x;\n")
    r = stage_record(str(f), str(w), ["k_radius_fill_rec", "k_radius_fill_rows", "k_radius_fill"], 2, str(src))
    assert r["fetch_bytes_per_launch"] == (100.0 + 300.0 + 50.0) * 1024 * 2 / 2
    assert r["write_bytes_per_launch"] == (10.0 + 30.0) * 1024 / 2
    assert r["bytes_per_launch"] == r["fetch_bytes_per_launch"] + r["write_bytes_per_launch"]
    assert r["fetch_bytes_by_kernel"]["k_radius_fill_rows"]["dispatches"] == 1
