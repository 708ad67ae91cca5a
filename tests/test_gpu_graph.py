"""Pre-allocated batched plans replayed from a HIP graph: every replay (with
eager work and synchronisations between replays) must reproduce the eager
result, which itself matches the oracle; and the autotuner of leaf size,
staging tile and fill."""
import numpy as np
import pytest

import oracle
from paper_2603_06771_amd import datagen
from tests._parity import announce, assert_csr_equal

pytestmark = pytest.mark.gpu

SIZES = [3001, 0, 17, 12007, 640, 5000]
KERN = ["sphere", "cube", "circle", "square", "cube", "sphere"]
RADII = [0.06, 0.1, 0.3, 0.05, 0.2, 0.08]
LEAF = [16, 8, 32, 64, 4, 128]


def _clouds():
    return [datagen.uniform(n, seed=70 + i) if n else np.zeros((0, 3), np.float32) for i, n in enumerate(SIZES)]


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)).cuda()


def _csr(plan):
    return plan.counts.cpu().numpy(), plan.offsets.cpu().numpy(), plan.indices.cpu().numpy()


@pytest.mark.parametrize("record", [False, True])
def test_radius_plan_graph_replays(tmp_path, record):
    import torch
    from paper_2603_06771_amd.plan import BatchPlan
    clouds = _clouds()
    xyz = _dev(np.concatenate(clouds))
    announce(f"radius plan: eager (record={record})")
    plan = BatchPlan(xyz, SIZES, "hilbert", 21, LEAF, KERN, RADII, record=record)
    plan.run()
    torch.cuda.synchronize()
    c, o, i = _csr(plan)
    q0 = 0
    for cl, pts in enumerate(clouds):
        perm = plan.tree(cl).perm().cpu().numpy().view(np.uint32)
        ref = oracle.radius_search(pts, pts[perm], KERN[cl], RADII[cl])
        a, b = o[q0], o[q0 + pts.shape[0]]
        assert_csr_equal((c[q0:q0 + pts.shape[0]], o[q0:q0 + pts.shape[0] + 1] - a, i[a:b]), ref, f"cloud {cl}")
        q0 += pts.shape[0]
    eager = (c.copy(), o.copy(), i[:o[-1]].copy())
    announce("radius plan: capture")
    plan.capture()
    other = BatchPlan(_dev(datagen.uniform(20000, seed=5)), [20000], "morton", 21, 32, "sphere", 0.05)
    for rep in range(3):
        # clobber the outputs, do unrelated eager work, then replay
        plan.counts.fill_(7)
        plan.indices.fill_(-1)
        other.run()
        torch.cuda.synchronize()
        announce(f"radius plan: replay {rep}")
        plan.replay()
        torch.cuda.synchronize()
        c, o, i = _csr(plan)
        assert np.array_equal(c, eager[0]) and np.array_equal(o, eager[1])
        assert np.array_equal(i[:o[-1]], eager[2]), f"replay {rep}: indices differ"


def test_knn_plan_graph_replays():
    import torch
    from paper_2603_06771_amd.plan import BatchPlan
    clouds = _clouds()
    ks = [8, 3, 1, 32, 16, 5]
    xyz = _dev(np.concatenate(clouds))
    announce("knn plan: eager")
    plan = BatchPlan(xyz, SIZES, "morton", 21, LEAF, k=ks)
    plan.run()
    torch.cuda.synchronize()
    gi, gd = plan.idx.cpu().numpy().view(np.uint32).copy(), plan.d2.cpu().numpy().copy()
    q0 = 0
    for cl, pts in enumerate(clouds):
        perm = plan.tree(cl).perm().cpu().numpy().view(np.uint32)
        ridx, rd2 = oracle.knn(pts, pts[perm], ks[cl])
        rows = slice(q0, q0 + pts.shape[0])
        assert np.array_equal(gi[rows, :ks[cl]], ridx)
        assert np.array_equal(gd[rows, :ks[cl]].view(np.uint32), rd2.view(np.uint32))
        q0 += pts.shape[0]
    plan.capture()
    for rep in range(3):
        plan.idx.fill_(0)
        plan.d2.fill_(0)
        torch.cuda.synchronize()
        announce(f"knn plan: replay {rep}")
        plan.replay()
        torch.cuda.synchronize()
        assert np.array_equal(plan.idx.cpu().numpy().view(np.uint32), gi)
        assert np.array_equal(plan.d2.cpu().numpy().view(np.uint32), gd.view(np.uint32))


def test_autotune_leaf_tile_fill(tmp_path):
    """The tuner picks (leaf, staging tile, fill) per group of clouds from the
    candidates, caches the choice, and a plan built with its per-cloud choices
    gives the same rows as the default plan."""
    import torch
    from paper_2603_06771_amd import autotune
    from paper_2603_06771_amd.plan import BatchPlan
    clouds = _clouds()
    xyz = _dev(np.concatenate(clouds))
    path = str(tmp_path / "tune.json")
    announce("autotune")
    kw = dict(candidates=(8, 32), stages=(64, 256), buckets=2, repeats=1, cache_path=path)
    t = autotune.tune(xyz, SIZES, KERN, RADII, "hilbert", **kw)
    assert not t["cached"] and len(t["leaf"]) == len(SIZES) == len(t["stage"]) == len(t["record"])
    assert set(t["leaf"]) <= {8, 32} and set(t["stage"]) <= {64, 128, 256}
    for g, ms in t["table"].items():
        assert sum(k.startswith("leaf=") and "/" not in k for k in ms) == 2
        # the default tile at the chosen leaf, then stage x fill (64 and 256, search and record)
        assert sum("/" in k for k in ms) == 5
    # groups that chose different fills: the whole batch was timed with them and with one fill for all
    groups = {}
    for b, rec in zip(t["bucket"], t["record"]):
        groups.setdefault(b, set()).add(rec)
    assert all(len(v) == 1 for v in groups.values())
    if t["whole"]:
        assert {"per_group", "search", "record"} <= set(t["whole"]) and all(v > 0 for v in t["whole"].values())
    t2 = autotune.tune(xyz, SIZES, KERN, RADII, "hilbert", **kw)
    assert t2["cached"] and (t2["leaf"], t2["stage"], t2["record"]) == (t["leaf"], t["stage"], t["record"])
    # a zero record budget keeps every group on the search fill
    t3 = autotune.tune(xyz, SIZES, KERN, RADII, "hilbert", record_budget=0, **kw)
    assert not any(t3["record"]) and all("fill=record" not in k for ms in t3["table"].values() for k in ms)
    # the tuned plan gives the rows of the default plan
    announce("autotune: tuned plan against the default plan")
    ref = BatchPlan(xyz, SIZES, "hilbert", 21, LEAF, KERN, RADII)
    ref.run()
    tuned = BatchPlan(xyz, SIZES, "hilbert", 21, t["leaf"], KERN, RADII, record=t["record"], stage=t["stage"])
    tuned.run()
    torch.cuda.synchronize()
    rc, ro, ri = _csr(ref)
    c, o, i = _csr(tuned)
    assert np.array_equal(c, rc) and np.array_equal(o, ro)
    # leaf sizes change the stored order (rows keep the query's position; the
    # order inside a row may differ): compare the row sets
    rows = np.repeat(np.arange(c.size), c)
    a = i[:o[-1]][np.lexsort((i[:o[-1]], rows))]
    b = ri[:ro[-1]][np.lexsort((ri[:ro[-1]], rows))]
    assert np.array_equal(a, b)
