#!/usr/bin/env python3
"""Benchmark: fixed-radius neighbourhood search on a 10M-point LiDAR tile.

One step is one pass of the whole hot path over the workload:
  for each curve in (Morton, Hilbert):
      encode -> radix sort -> reorder -> linear octree build
      for each kernel in (sphere, cube), r in (0.5, 1, 2, 3) m:
          radius_search over every cloud point (count pass recording each
          group's hits, scan, fill stage writing the rows from the records)
so a step answers 16 x 10M radius queries.  Inputs are resident in HBM before
the timed region; the output buffer is sized once (capacity protocol), so no
host synchronisation happens inside a step.  --no-record times the search
fill instead (the same result).

Prints ONE JSON line.  `roofline` is that of whole radius_search calls
(count pass + scan + fill stage, event-timed on the launch stream), with
algorithmic bytes per call
  (16 + 4 + 8) B x queries (point read, count and row offset written)
  + 4 B x neighbours (indices written) + 36 B x nodes (tree read once);
`fill_stage` keeps the fill stage alone (row offsets read, indices written).
After the timed steps (outside them): `knn` (k = 8, 16, 32 on the same tile,
16 + 8k B per query), `c1` (the 100k-point uniform configuration), the CPU
baseline (the oracle on a bounded sample, and on one thread for the 100k
configuration) and `served` (64 resident clouds, Poisson requests, p50/p99
latency at 95 % of the continuous-batching capacity).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the fill stage of a recorded-hits search: the two record-writing forms and
# the search fill for groups whose records did not fit
FILL_STAGE = "k_radius_fill_rec + k_radius_fill_rows + k_radius_fill"
# one radius_search call: count pass, scan of the counts, fill stage
SEARCH = "radius_search: k_radius_count_rec + k_scan_* + " + FILL_STAGE
SEARCH_NO_RECORD = "radius_search: k_radius_count + k_scan_* + k_radius_fill"
KNN_K = (8, 16, 32)
CURVES = ("morton", "hilbert")
KERNELS = ("sphere", "cube")
RADII = (0.5, 1.0, 2.0, 3.0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--points", type=int, default=10_000_000)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--cpu-sample", type=int, default=100_000, help="queries per (kernel, r) for the oracle")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-knn", action="store_true", help="radius: skip the k-NN leg")
    ap.add_argument("--no-served", action="store_true", help="radius: skip the served leg")
    ap.add_argument("--no-record", action="store_true",
                    help="radius: the fill searches again instead of writing rows from the hits the count "
                         "pass recorded (SFC_RECORD_HITS, the default)")
    ap.add_argument("--record-batched", action="store_true",
                    help="batched: fill every cloud from recorded hits instead of the autotuner's per-group choice")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a plain 256 MiB device copy and a 256 MiB elementwise kernel first (reference "
                         "dispatches for HBM counters)")
    ap.add_argument("--workload", default="radius", choices=["radius", "batched", "served", "subset"],
                    help="radius: 10M LiDAR radius sweep (default); batched: 256 clouds, build + radius search; "
                         "served: 64 resident clouds, Poisson radius / k-NN requests")
    ap.add_argument("--requests", type=int, default=1500, help="served: requests per run")
    ap.add_argument("--served-clouds", type=int, default=64, help="served: resident clouds")
    ap.add_argument("--clouds", type=int, default=256, help="batched: number of clouds")
    ap.add_argument("--tune-repeats", type=int, default=2, help="batched: timed steps per autotune candidate")
    return ap.parse_args()


def cpu_baseline(pts, sample: int):
    """The oracle (unchanged) on a bounded sample of the same workload."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(pts.shape[0], min(sample, pts.shape[0]), replace=False))
    q = np.ascontiguousarray(pts[rows])
    t_build = 0.0
    t_search = 0.0
    nq = 0
    for r in RADII:
        t0 = time.perf_counter()
        grid = oracle.Grid(pts, r, 3)  # sphere and cube share the 3D grid of side r
        t_build += time.perf_counter() - t0
        for kernel in KERNELS:
            t0 = time.perf_counter()
            grid.radius_search(q, kernel, r)
            t_search += time.perf_counter() - t0
            nq += q.shape[0]
        del grid
    # projected on the full workload (every point a query, for each kernel and r)
    frac = pts.shape[0] / q.shape[0]
    full_queries = len(RADII) * len(KERNELS) * pts.shape[0]
    full_time = t_build + t_search * frac
    return {"value": full_queries / full_time, "unit": "queries/s", "cores": oracle.get_threads(),
            "kind": "oracle",
            "sample": f"{q.shape[0]} random query points x {len(KERNELS)} kernels x {len(RADII)} radii "
                      f"(count + fill), plus the grid build per radius; time scaled to all "
                      f"{pts.shape[0]} queries: build {t_build:.2f} s, sample search {t_search:.2f} s"}


def _events(torch, n):
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]


def _count(items) -> dict:
    out = {}
    for x in items:
        out[x] = out.get(x, 0) + 1
    return out


def bench_batched(args):
    """256 independent clouds (log-uniform 1e4..2e6 points, uniform / LiDAR,
    per-cloud kernel and radius): build + radius search of every cloud.
    Batched (one launch per stage for all clouds), eager and replayed from a
    HIP graph, against one launch sequence per cloud (eager, and all of them
    captured in one graph)."""
    import numpy as np
    import torch

    from paper_2603_06771_amd import autotune, datagen
    from paper_2603_06771_amd.plan import BatchPlan

    t0 = time.perf_counter()
    clouds = datagen.batch_mix(args.clouds, seed=datagen.SEED_BATCH)
    sizes = [c["points"].shape[0] for c in clouds]
    kernels = [c["kernel"] for c in clouds]
    radii = [c["radius"] for c in clouds]
    xyz = torch.from_numpy(np.concatenate([c["points"] for c in clouds])).cuda()
    n = int(sum(sizes))
    del clouds
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    log(f"[bench] generated {len(sizes)} clouds, {n} points in {time.perf_counter() - t0:.1f} s")

    tune = autotune.tune(xyz, sizes, kernels, radii, "hilbert", repeats=args.tune_repeats,
                         cache_path=os.path.join(tempfile.gettempdir(), "sfcoct_bench_autotune.json"), log=log)
    leaves, stages = tune["leaf"], tune["stage"]
    record = [True] * len(sizes) if args.record_batched else tune["record"]
    plan = BatchPlan(xyz, sizes, "hilbert", 21, leaves, kernels, radii, record=record, stage=stages)
    total = plan.total()
    log(f"[bench] batched plan: {total} neighbours ({total * 4 / 1e9:.2f} GB)")

    def timed(fn, steps):
        ev = _events(torch, steps)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) * 1e3 / steps
        return wall, float(np.median([a.elapsed_time(b) for a, b in ev]))

    for _ in range(args.warmup):
        plan.run()
    eager_wall, eager_gpu = timed(plan.run, args.steps)
    plan.capture()
    for _ in range(args.warmup):
        plan.replay()
    graph_wall, graph_gpu = timed(plan.replay, args.steps)
    batched_counts = plan.counts.clone()
    log(f"[bench] batched eager {eager_wall:.2f} ms, graph {graph_wall:.2f} ms per step")

    # kernel times inside the batched step (build, count, fill)
    stage_ms = {}
    ev = _events(torch, 3)
    ev[0][0].record()
    plan.build()
    ev[0][1].record()
    ev[1][0].record()
    plan.search(count=True, fill=False)
    ev[1][1].record()
    ev[2][0].record()
    plan.search(count=False, fill=True)
    ev[2][1].record()
    torch.cuda.synchronize()
    for name, (a, b) in zip(("build", "count+scan", "fill"), ev):
        stage_ms[name] = round(a.elapsed_time(b), 3)
    del plan
    torch.cuda.empty_cache()

    # baseline: one launch sequence per cloud
    starts = np.concatenate([[0], np.cumsum(sizes)])
    singles = [BatchPlan(xyz[starts[c]:starts[c + 1]], [sizes[c]], "hilbert", 21, leaves[c], kernels[c], radii[c],
                         record=record[c], stage=stages[c]) for c in range(len(sizes))]

    def per_cloud():
        for p in singles:
            p.run()

    for _ in range(args.warmup):
        per_cloud()
    base_wall, base_gpu = timed(per_cloud, args.steps)
    same = all(torch.equal(p.counts, batched_counts[starts[c]:starts[c + 1]]) for c, p in enumerate(singles))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        per_cloud()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        g.replay()
    base_graph_wall, base_graph_gpu = timed(g.replay, args.steps)
    log(f"[bench] per-cloud eager {base_wall:.2f} ms, graph {base_graph_wall:.2f} ms per step; counts equal: {same}")

    # algorithmic bytes of the searches (every point a query): the point read
    # once, its count and row offset written, 4 B per neighbour (the tree's
    # node bytes, under 2 % at these leaf sizes, left out)
    search_bytes = (16 + 4 + 8) * n + 8 + 4 * total
    search_ms = stage_ms["count+scan"] + stage_ms["fill"]
    out = {
        "metric": "batched build + radius-search queries/s (256 clouds, one HIP graph)",
        "value": n / (graph_wall / 1e3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": graph_wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch256_mix_build_radius", "clouds": len(sizes), "points": n,
                   "neighbours": total, "curve": "hilbert",
                   "leaf_stage_fill": "autotuned per mu group" + (", every cloud recorded" if args.record_batched
                                                                  else "")},
        "batched": {"graph_ms": round(graph_wall, 3), "graph_gpu_ms": round(graph_gpu, 3),
                    "eager_ms": round(eager_wall, 3), "eager_gpu_ms": round(eager_gpu, 3), "stages_ms": stage_ms},
        "one_launch_sequence_per_cloud": {"eager_ms": round(base_wall, 3), "eager_gpu_ms": round(base_gpu, 3),
                                          "graph_ms": round(base_graph_wall, 3),
                                          "graph_gpu_ms": round(base_graph_gpu, 3), "counts_equal": same},
        "speedup_vs_per_cloud": {"eager": base_wall / eager_wall, "graph": base_graph_wall / graph_wall,
                                 "graph_vs_per_cloud_eager": base_wall / graph_wall},
        "roofline": {"bound": "hbm", "kernel": "radius_search_batched (count + scan + fill)",
                     "achieved": search_bytes / search_ms / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": search_bytes / search_ms / 1e6 / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_query": "16 + 4 + 8 + 4 mu"},
        "autotune": {"table_ms": tune["table"], "whole_batch_ms": tune.get("whole", {}), "mu_edges": tune["edges"],
                     "cached": tune["cached"],
                     "choice_histogram": {f"leaf={lf}/stage={st}/fill={'record' if rc else 'search'}": cnt
                                          for (lf, st, rc), cnt in
                                          sorted(_count(zip(leaves, stages, record)).items())}},
    }
    print(json.dumps(out), flush=True)


def _gen_served_cloud(args):
    from paper_2603_06771_amd import datagen
    n, seed = args
    return datagen.lidar_tile(n, seed=seed)


def served_measure(args, n_requests: int):
    """64 resident LiDAR clouds (3.5M..9M points each, Hilbert octrees in HBM);
    a Poisson stream of requests, each naming a cloud, 1e3..1e6 of its points
    as queries and a radius search (kernel, r ~ U(0.5, 3)) or a k-NN search
    (k in 8, 16, 32).  Capacity is measured with every request queued at t=0;
    then the stream is replayed at 50 / 80 / 95 % of the continuous-batching
    capacity, by the continuous-batching server and by the one-request FIFO
    server on the same GPU."""
    import multiprocessing as mp

    import numpy as np
    import torch

    from paper_2603_06771_amd import datagen, serve

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    sizes = datagen.served_sizes(args.served_clouds, seed=datagen.SEED_SERVED)
    res = serve.Resident(budget_bytes=160 << 30, curve="hilbert", leaf_size=64)
    t0 = time.perf_counter()
    build_s = 0.0
    group = 16
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        for g0 in range(0, len(sizes), group):
            part = [(sizes[c], datagen.SEED_SERVED + 1 + c) for c in range(g0, min(len(sizes), g0 + group))]
            clouds = pool.map(_gen_served_cloud, part)
            torch.cuda.synchronize()
            b0 = time.perf_counter()
            ids = res.admit(clouds)
            build_s += time.perf_counter() - b0
            if ids is None:
                raise SystemExit("served: clouds do not fit the memory budget")
            del clouds
    n_points = int(sum(sizes))
    log(f"[bench] {len(sizes)} resident clouds, {n_points} points, {res.used / 1e9:.1f} GB; generated + built in "
        f"{time.perf_counter() - t0:.1f} s (builds {build_s:.2f} s)")

    base = datagen.request_stream(n_requests, len(sizes), sizes, rate_per_s=1.0)
    log(f"[bench] {len(base)} requests, {sum(len(d['rows']) for d in base)} queries")

    def requests(rate):
        out = []
        for d in base:
            out.append(serve.Request(id=d["id"], arrival=0.0 if rate is None else d["arrival"] / rate,
                                     cloud=d["cloud"], rows=d["rows"], op=d["op"], kernel=d.get("kernel", "sphere"),
                                     radius=d.get("radius", 1.0), k=d.get("k", 8)))
        return out

    log("[bench] allocating server slots")
    srv = serve.Server(res, slots=3, max_requests=64, max_queries=4 << 20, out_entries=1 << 30)
    modes = {"continuous": dict(max_requests=64, n_slots=3), "fifo": dict(max_requests=1, n_slots=1)}

    def summary(st):
        lat = st["latency_s"] * 1e3
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "queries_per_s": st["queries"] / st["span_s"],
                "requests_per_s": len(lat) / st["span_s"], "batches": st["batches"], "regrown": st["regrown"]}

    log("[bench] server ready; warm-up")
    srv.run(requests(None)[:64], log=log, **modes["continuous"])  # warm-up
    cap = {}
    for m, kw in modes.items():
        log(f"[bench] capacity run, {m}")
        st = srv.run(requests(None), log=log, **kw)
        cap[m] = summary(st)
        log(f"[bench] capacity {m}: {cap[m]['requests_per_s']:.0f} req/s, {cap[m]['queries_per_s']:.3g} q/s")
    loads = {}
    for frac in (0.5, 0.8, 0.95):
        rate = frac * cap["continuous"]["requests_per_s"]
        loads[str(frac)] = {}
        for m, kw in modes.items():
            st = srv.run(requests(rate), log=log, **kw)
            loads[str(frac)][m] = summary(st)
            log(f"[bench] load {frac:.2f} ({rate:.0f} req/s) {m}: p50 {loads[str(frac)][m]['p50_ms']:.2f} ms, "
                f"p99 {loads[str(frac)][m]['p99_ms']:.2f} ms")
    out = {"clouds": len(sizes), "points": n_points, "requests": n_requests, "slots": 3,
           "max_batch_requests": 64, "capacity": cap, "loads": loads, "resident_gb": res.used / 1e9,
           "build_s": build_s}
    del srv, res
    torch.cuda.empty_cache()
    return out


def served_line(args, sv):
    """The JSON line of --workload served."""
    at95 = sv["loads"]["0.95"]["continuous"]
    return {
        "metric": "served p50/p99 latency at 95% of capacity (continuous batching), queries/s",
        "value": at95["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": sv["requests"],
        "warmup": 64,
        "ms_per_step": at95["mean_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "served64_lidar_poisson", "clouds": sv["clouds"], "points": sv["points"],
                   "requests": sv["requests"], "slots": sv["slots"], "max_batch_requests": sv["max_batch_requests"]},
        "p50_ms": at95["p50_ms"],
        "p99_ms": at95["p99_ms"],
        **{k: sv[k] for k in ("capacity", "loads", "resident_gb", "build_s")},
    }


def bench_subset(args):
    """The paper's random-subset workload: 5000 random points of the 10M tile
    as query centres, sphere and cube searches at r = 0.5, 1, 2, 3 m, on the
    Morton and the Hilbert order (count + fill per query set, median of
    `steps` repetitions)."""
    import numpy as np
    import torch

    import paper_2603_06771_amd as sfc
    from paper_2603_06771_amd import datagen

    pts = datagen.lidar_tile(args.points, seed=datagen.SEED_LIDAR)
    n = pts.shape[0]
    rows = np.sort(np.random.default_rng(datagen.SEED_LIDAR).choice(n, 5000, replace=False))
    xyz = torch.from_numpy(pts).cuda()
    q = torch.from_numpy(np.ascontiguousarray(pts[rows])).cuda()
    out = {}
    for curve in CURVES:
        t = sfc.build_linear_octree(xyz, curve, 21, args.leaf)
        for k in KERNELS:
            for r in RADII:
                c, o, _ = sfc.radius_search(t, q, k, r)
                cap = int(o[-1])
                ts = []
                for _ in range(args.warmup + args.steps):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    sfc.radius_search(t, q, k, r, capacity=cap, check=False)
                    b.record()
                    b.synchronize()
                    ts.append(a.elapsed_time(b))
                ms = float(np.median(ts[args.warmup:]))
                out[f"{curve}/{k}/r={r}"] = {"ms": round(ms, 4), "mu": cap / 5000.0}
                print(f"[bench] subset {curve} {k} r={r}: {ms:.3f} ms", file=sys.stderr, flush=True)
        del t
    total_ms = sum(v["ms"] for v in out.values())
    res = {"metric": "random-subset radius search (5000 centres) queries/s", "value": 5000 * len(out) / (total_ms / 1e3),
           "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": total_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "lidar_tile_10M_subset5000", "points": n, "leaf_size": args.leaf},
           "detail": out}
    print(json.dumps(res), flush=True)


def copy_bandwidth(torch, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Achievable HBM bandwidth beside the nominal peak: a plain device copy
    of nbytes (bytes read + bytes written over the event-timed copy), GB/s."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2.0 * nbytes / ms / 1e6


def knn_leg(torch, sfc, B, L, xyz, n: int, leaf: int, reps: int):
    """k-NN on the same 10M-point tile: Hilbert tree, every point a query,
    k = 8, 16, 32 (event-timed calls on the current stream, mean of `reps`
    after one warm-up).  Algorithmic bytes per query: 16 (the query point) +
    8k (index and squared distance of each neighbour)."""
    import ctypes

    import numpy as np
    tree = sfc.build_linear_octree(xyz, "hilbert", 21, leaf)
    stream = torch.cuda.current_stream()
    out = {}
    tot_b, tot_ms = 0.0, 0.0
    for k in KNN_K:
        idx = torch.empty((n, k), dtype=torch.int32, device="cuda")
        d2 = torch.empty((n, k), dtype=torch.float32, device="cuda")
        need = ctypes.c_size_t(0)
        args = (ctypes.byref(tree.view), None, n, k, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()))
        B.check(L.knn_search(*args, None, ctypes.byref(need), None), "knn_search(size)")
        ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
        call = (ctypes.c_void_p(ws.data_ptr()), ctypes.byref(need), ctypes.c_void_p(stream.cuda_stream))
        B.check(L.knn_search(*args, *call), "knn_search")
        ev = _events(torch, reps)
        for a, b in ev:
            a.record(stream)
            B.check(L.knn_search(*args, *call), "knn_search")
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        by = (16.0 + 8.0 * k) * n
        tot_b += by
        tot_ms += ms
        out[f"k={k}"] = {"ms": round(ms, 4), "queries_per_s": n / (ms / 1e3),
                         "frac": by / ms / 1e6 / HBM_PEAK_GBS}
        del idx, d2, ws
    del tree
    torch.cuda.empty_cache()
    return {"workload": "lidar_tile_10M_knn", "curve": "hilbert", "leaf_size": leaf,
            "queries_per_s": len(KNN_K) * n / (tot_ms / 1e3), "ms_total": round(tot_ms, 4),
            "roofline": {"bound": "hbm", "achieved": tot_b / tot_ms / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": tot_b / tot_ms / 1e6 / HBM_PEAK_GBS, "alg_bytes_per_query": "16 + 8k"},
            "detail": out}


def c1_leg(torch, sfc, reps: int = 20):
    """The 100k-point uniform configuration (Morton, leaf 32, every point a
    query, sphere r = 0.01): GPU latency of one radius_search (count + fill,
    median of `reps`), and the oracle on one host thread on the same input."""
    import numpy as np

    from paper_2603_06771_amd import datagen
    pts = datagen.uniform(100_000, seed=datagen.SEED_UNIFORM)
    xyz = torch.from_numpy(pts).cuda()
    tree = sfc.build_linear_octree(xyz, "morton", 21, 32)
    c, o, _ = sfc.radius_search(tree, None, "sphere", 0.01)
    cap = int(o[-1])
    ts = []
    for i in range(reps + 2):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sfc.radius_search(tree, None, "sphere", 0.01, capacity=cap, check=False)
        b.record()
        b.synchronize()
        if i >= 2:
            ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    return pts, {"workload": "uniform_100k_sphere_r0.01", "gpu_ms": round(ms, 4),
                 "queries_per_s": pts.shape[0] / (ms / 1e3), "mu": cap / pts.shape[0]}


def c1_single_thread(pts):
    """The oracle on one host thread over the whole 100k-point configuration
    (grid build + count + fill)."""
    import oracle
    t_prev = oracle.get_threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.radius_search(pts, pts, "sphere", 0.01)
        s = time.perf_counter() - t0
    finally:
        oracle.set_threads(t_prev)
    return {"value": pts.shape[0] / s, "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"all {pts.shape[0]} queries of the 100k uniform configuration (grid build + count + fill): "
                      f"{s:.3f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the search is built for one "
              f"GPU's share of the data; sharding across GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "served":
        print(json.dumps(served_line(args, served_measure(args, args.requests))), flush=True)
        return
    if args.workload == "subset":
        bench_subset(args)
        return
    import ctypes

    import numpy as np
    import torch

    import paper_2603_06771_amd as sfc
    from paper_2603_06771_amd import _binding as B
    from paper_2603_06771_amd import datagen

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    pts = datagen.lidar_tile(args.points, seed=datagen.SEED_LIDAR)
    log(f"[bench] generated {pts.shape[0]} points in {time.perf_counter() - t0:.1f} s")
    xyz = torch.from_numpy(pts).cuda()
    n = pts.shape[0]
    if args.copy_calib:
        # reference dispatches of known size for the HBM counters: the
        # runtime's device copy and an elementwise kernel (256 MiB read,
        # 256 MiB written each)
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.current_stream()
    L = B.load()

    # size the output once: the largest neighbour total over the workload
    trees = {c: sfc.build_linear_octree(xyz, c, 21, args.leaf) for c in CURVES}
    cap = 0
    totals = {}
    for c in CURVES:
        for k in KERNELS:
            for r in RADII:
                counts, offsets = sfc.radius_count(trees[c], None, k, r)
                totals[c, k, r] = int(offsets[-1].item())
                cap = max(cap, totals[c, k, r])
    infos = {c: trees[c].info() for c in CURVES}
    del trees
    torch.cuda.synchronize()
    log(f"[bench] output capacity {cap} indices ({cap * 4 / 1e9:.2f} GB)")

    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    indices = torch.empty(cap, dtype=torch.int32, device="cuda")
    need = ctypes.c_size_t(0)
    record = not args.no_record
    rf = B.RECORD_HITS if record else 0
    combos = [(c, k, r) for c in CURVES for k in KERNELS for r in RADII]

    def step(events=None, build_events=None):
        i = 0
        for ci, c in enumerate(CURVES):
            if build_events is not None:
                build_events[ci][0].record(stream)
            tree = sfc.build_linear_octree(xyz, c, 21, args.leaf)
            if build_events is not None:
                build_events[ci][1].record(stream)
            sp = stream.cuda_stream
            for k in KERNELS:
                for r in RADII:
                    base = (ctypes.byref(tree.view), None, n, sfc.KERNELS[k], float(r),
                            ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(offsets.data_ptr()))
                    if need.value == 0:
                        B.check(L.radius_search(*base, None, 0, rf, None, ctypes.byref(need), None), "size")
                        step.ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
                    ws = ctypes.c_void_p(step.ws.data_ptr())
                    if events is not None:
                        events[i][0].record(stream)
                    # count pass + scan
                    B.check(L.radius_search(*base, None, 0, rf, ws, ctypes.byref(need), ctypes.c_void_p(sp)),
                            "radius count")
                    if events is not None:
                        events[i][1].record(stream)
                    # fill pass only (counts/offsets from the call above)
                    B.check(L.radius_search(*base, ctypes.c_void_p(indices.data_ptr()), cap, B.REUSE_COUNTS | rf,
                                            ws, ctypes.byref(need), ctypes.c_void_p(sp)), "radius fill")
                    if events is not None:
                        events[i][2].record(stream)
                    i += 1
            del tree

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [[tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in combos] for _ in range(args.steps)]
    ev_build = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in CURVES]
                for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s], ev_build[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps

    count_ms = {cb: float(np.mean([ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(args.steps)]))
                for i, cb in enumerate(combos)}
    fill_ms = {cb: float(np.mean([ev[s][i][1].elapsed_time(ev[s][i][2]) for s in range(args.steps)]))
               for i, cb in enumerate(combos)}
    build_ms = {c: float(np.mean([ev_build[s][i][0].elapsed_time(ev_build[s][i][1]) for s in range(args.steps)]))
                for i, c in enumerate(CURVES)}

    # algorithmic bytes of one radius_search over every point: the query point
    # read once (16 B), its count (4 B) and row offset (8 B) written, the
    # indices (4 B per neighbour) and the tree read once (36 B per node: the
    # 32-B node record and the child link); the fill stage alone: the row
    # offsets read and the indices written
    def search_bytes(c, total):
        return (16 + 4 + 8) * n + 8 + 4 * total + 36 * infos[c]["n_nodes"]

    def fill_bytes(total):
        return 8 * (n + 1) + 4 * total

    s_bytes = s_ms = f_bytes = f_ms = 0.0
    detail = {}
    for cb in combos:
        c, k, r = cb
        sb, fb = search_bytes(c, totals[cb]), fill_bytes(totals[cb])
        ms = count_ms[cb] + fill_ms[cb]
        s_bytes += sb
        s_ms += ms
        f_bytes += fb
        f_ms += fill_ms[cb]
        detail[f"{c}/{k}/r={r}"] = {"mu": totals[cb] / n, "count_ms": round(count_ms[cb], 4),
                                    "fill_ms": round(fill_ms[cb], 4), "search_ms": round(ms, 4),
                                    "frac": sb / ms / 1e6 / HBM_PEAK_GBS}
    achieved = s_bytes / s_ms / 1e6  # GB/s over whole radius_search calls
    f_achieved = f_bytes / f_ms / 1e6

    def traffic_of(name):
        """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
        copy-calibrated), valid only while the kernel source is the one the
        counters were taken on."""
        try:
            from paper_2603_06771_amd import rocprof_summary
            rec = json.load(open(os.path.join(ROOT, "profiles", name)))
            src = os.path.join(ROOT, "paper_2603_06771_amd", "csrc", "search.hip")
            if rec.get("source_sha") == rocprof_summary.source_sha(src) and args.leaf == 64 and n == 10_000_000:
                return rec["bytes_per_launch"]
        except (OSError, ValueError, KeyError):
            pass
        return None

    queries_per_step = len(combos) * n
    value = queries_per_step / (ms_per_step / 1e3)
    log(f"[bench] {ms_per_step:.2f} ms per step; radius_search {s_ms / len(combos):.3f} ms per call on average")
    copy_gbs = copy_bandwidth(torch)

    out = {
        "metric": "radius-search queries/s at 10M pts (+% HBM roofline); served p50/p99 ms",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lidar_tile_10M_radius_sweep", "points": n, "curves": list(CURVES),
                   "kernels": list(KERNELS), "radii_m": list(RADII), "leaf_size": args.leaf,
                   "queries_per_step": queries_per_step, "builds_per_step": len(CURVES),
                   "record_hits": record},
        "roofline": {"bound": "hbm", "kernel": SEARCH if record else SEARCH_NO_RECORD, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_of("radius_search_record_lidar10M_traffic.json" if record
                                           else "radius_search_lidar10M_traffic.json"),
                     "alg_bytes_per_launch": s_bytes / len(combos), "ms_per_launch": s_ms / len(combos),
                     "alg_bytes_per_query": "16 + 4 + 8 + 4 mu + 36 nodes / n",
                     "stream_copy_GBps": copy_gbs},
        "fill_stage": {"kernel": FILL_STAGE if record else "k_radius_fill", "achieved": f_achieved,
                       "frac": f_achieved / HBM_PEAK_GBS, "alg_bytes_per_launch": f_bytes / len(combos),
                       "ms_per_launch": f_ms / len(combos),
                       "traffic": traffic_of("radius_fill_stage_record_lidar10M_traffic.json" if record
                                             else "k_radius_fill_lidar10M_traffic.json")},
        "build_ms": {c: round(v, 3) for c, v in build_ms.items()},
        # beside the end-to-end value: the searches alone (the step less its
        # event-timed builds) and the build throughput
        "search_only": {"queries_per_s": queries_per_step / ((ms_per_step - sum(build_ms.values())) / 1e3),
                        "ms_per_step": ms_per_step - sum(build_ms.values())},
        "build_points_per_s": {c: n / (v / 1e3) for c, v in build_ms.items()},
        "tree": {c: {"n_nodes": infos[c]["n_nodes"], "n_leaves": infos[c]["n_leaves"], "depth": infos[c]["depth"]}
                 for c in CURVES},
        "detail": detail,
    }
    del indices, counts, offsets
    step.ws = None
    torch.cuda.empty_cache()
    if not args.no_knn:
        log("[bench] k-NN leg")
        out["knn"] = knn_leg(torch, sfc, B, L, xyz, n, args.leaf, 3)
    c1_pts, out["c1"] = c1_leg(torch, sfc)
    del xyz
    torch.cuda.empty_cache()
    if not args.no_cpu:
        log("[bench] timing the oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(pts, args.cpu_sample)
        out["cpu_baseline"]["c1_single_thread"] = c1_single_thread(c1_pts)
    del pts
    if not args.no_served:
        log("[bench] served leg")
        sv = served_measure(args, args.requests)
        at95 = sv["loads"]["0.95"]["continuous"]
        out["served"] = {"p50_ms": at95["p50_ms"], "p99_ms": at95["p99_ms"],
                         "queries_per_s": at95["queries_per_s"], "requests_per_s": at95["requests_per_s"],
                         "offered_load": 0.95, **sv}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
