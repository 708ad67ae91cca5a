"""Sweep statistics of the radius count: point tests per neighbour found.

A group of 64 queries sweeps the union of its queries' reaches, so every
query is tested against points only its neighbours in the group can reach.
This measures how many (query, point) tests the count makes per neighbour it
finds, on the 10M-point LiDAR tile of the benchmark (leaf 64, every point a
query), for each curve, kernel and radius: tests / hits, tests per query and
staged points per group, for the recording count (the benchmark's) and the
plain count.

It needs libsfcoct_stats.so (built beside libsfcoct.so by build.py), the same
kernels with counters that sum, over every group, the staged points it swept
times its valid queries and the neighbours it counted, and the shader-clock
time of each phase of a group's work (segments, start node, walk,
classification, staging, tests, the rest), as shares of the total.

    python -m paper_2603_06771_amd.sweep_stats [--points N] [--leaf L]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os

from . import _binding as B
from .build import STATS_LIB


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--points", type=int, default=10_000_000)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--json", default=None, help="also write the table as JSON here")
    args = ap.parse_args()
    if not os.path.exists(STATS_LIB):
        raise SystemExit(f"{STATS_LIB} not found: build it with `python -m paper_2603_06771_amd.build`")
    import torch
    torch.zeros(1, device="cuda")  # the device is set up before the library's first call
    B._lib = None
    L = B.load(STATS_LIB)
    L.sfc_sweep_stats.argtypes = [ctypes.POINTER(ctypes.c_ulonglong), ctypes.c_int]

    import paper_2603_06771_amd as sfc
    from . import datagen
    pts = datagen.lidar_tile(args.points, seed=datagen.SEED_LIDAR)
    xyz = torch.from_numpy(pts).cuda()
    n = pts.shape[0]
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = (ctypes.c_ulonglong * 16)()
    B.check(L.sfc_sweep_stats(out, 1), "sfc_sweep_stats")
    rows = []
    phases = ("segments", "start", "walk", "classify", "staging", "tests", "rest")
    print(f"{'curve':8s} {'kernel':7s} {'r':>4s} {'count':6s} {'mu':>7s} {'tests/hit':>9s} {'tests/query':>11s} "
          f"{'staged/group':>12s}  phase shares (%): " + " ".join(f"{p:>8s}" for p in phases), flush=True)
    for curve in ("morton", "hilbert"):
        tree = sfc.build_linear_octree(xyz, curve, 21, args.leaf)
        for kernel in ("sphere", "cube"):
            for r in (0.5, 1.0, 2.0, 3.0):
                for record in (True, False):
                    flags = B.RECORD_HITS if record else 0
                    call = (ctypes.byref(tree.view), None, n, sfc.KERNELS[kernel], float(r),
                            ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), None, 0, flags)
                    need = ctypes.c_size_t(0)
                    B.check(L.radius_search(*call, None, ctypes.byref(need), None), "radius_search(size)")
                    ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
                    B.check(L.radius_search(*call, ctypes.c_void_p(ws.data_ptr()), ctypes.byref(need), stream),
                            "radius_search(count)")
                    B.check(L.sfc_sweep_stats(out, 1), "sfc_sweep_stats")
                    del ws
                    s = list(out)[4:8] if record else list(out)[:4]
                    tests, hits, groups, swept = s
                    clock = list(out)[8:15]
                    total = max(list(out)[15], 1)
                    row = {"curve": curve, "kernel": kernel, "r": r, "count": "record" if record else "plain",
                           "mu": hits / n, "tests_per_hit": tests / max(hits, 1), "tests_per_query": tests / n,
                           "staged_per_group": swept / max(groups, 1), "groups": groups,
                           "phase_share": {p: c / total for p, c in zip(phases, clock)}}
                    rows.append(row)
                    print(f"{curve:8s} {kernel:7s} {r:4.1f} {row['count']:6s} {row['mu']:7.1f} "
                          f"{row['tests_per_hit']:9.2f} {row['tests_per_query']:11.1f} "
                          f"{row['staged_per_group']:12.1f}                    " +
                          " ".join(f"{100 * row['phase_share'][p]:8.1f}" for p in phases), flush=True)
        del tree
    if args.json:
        with open(args.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
