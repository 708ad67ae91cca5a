"""Autotuner of leaf size, staging tile and fill for batches of clouds.

The best octree threshold N_max depends on how many neighbours a query has:
small leaves prune finely when neighbourhoods are small, large leaves cut
traversal work when they are large.  The search's staging tile (points
staged in LDS per sweep round: 64, 128 or 256) trades per-round work
against resident waves, and the fill either searches again or writes the
rows from the hits the count pass recorded (faster for long rows, but
48 KB of workspace per 64 queries).  The tuner measures instead of
guessing:

  1. one counting step of the whole batch (leaf 32) gives every cloud's mean
     neighbour count mu;
  2. clouds are split into `buckets` groups by mu (quantiles);
  3. each group is built and searched as its own batch with every candidate
     leaf size at the default tile (stage 128, search fill), then, at the
     fastest leaf, with every candidate (stage, fill) pair (median of
     `repeats` timed steps after a warm-up each); recorded fills are tried
     only while the group's records fit `record_budget` bytes;
  4. every cloud gets its group's fastest (leaf, stage, fill);
  5. when the groups' fills differ, the whole batch is timed with those
     fills, with every cloud on the search fill and (within the budget) with
     every cloud recorded, each at the chosen leaves and tiles, and the
     fastest is kept: in one batch the fills run one launch after another
     (recorded-row kernels, then the search fill), and the recording count
     costs every recorded cloud more than the plain count, so the groups'
     choices need not add up to the fastest batch.

Results are cached in a JSON file keyed by the batch description (sizes,
kernels, radii, curve, candidates, budget, device name), so a repeated
workload skips the measurement.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from .plan import BatchPlan

CANDIDATES = (16, 32, 64, 128)
STAGES = (64, 128, 256)
FILLS = ("search", "record")
RECORD_BYTES_PER_GROUP = 4096 * 12  # recorded hits: 4096 (index, mask) slots per 64 queries
DEFAULT_RECORD_BUDGET = 64 << 30


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "sfcoct", "autotune.json")


def _key(sizes, kernels, radii, curve, candidates, stages, fills, buckets, budget, device) -> str:
    h = hashlib.sha256()
    h.update(json.dumps(["whole-batch fill check", list(map(int, sizes)), list(map(str, kernels)),
                         [float(x) for x in radii], str(curve),
                         list(map(int, candidates)), list(map(int, stages)), list(map(str, fills)), int(buckets),
                         int(budget), str(device)]).encode())
    return h.hexdigest()[:32]


def _time_step(plan: BatchPlan, repeats: int) -> float:
    import torch
    plan.run()  # warm-up
    ts = []
    for _ in range(repeats):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plan.run()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def record_bytes(sizes) -> int:
    """Workspace the recorded fill needs for clouds of these sizes."""
    return sum((int(n) + 63) // 64 for n in sizes) * RECORD_BYTES_PER_GROUP


def tune(xyz, sizes, kernel, r, curve="hilbert", candidates=CANDIDATES, stages=STAGES, fills=FILLS,
         buckets: int = 4, repeats: int = 2, record_budget: int = DEFAULT_RECORD_BUDGET,
         cache_path: str | None = None, log=None) -> dict:
    """Returns {"leaf", "stage", "record": per-cloud choices, "bucket": per-cloud
    group, "mu": per-cloud mean neighbour count, "table": {group: {"leaf=L":
    ms, "leaf=L/stage=S/fill=F": ms}}, "whole": {"per_group" | "search" |
    "record": ms of the whole batch} (empty when the groups agree on the
    fill), "edges", "cached": bool}."""
    import torch
    sizes = [int(x) for x in sizes]
    nb = len(sizes)
    kernels = kernel if isinstance(kernel, (list, tuple)) else [kernel] * nb
    radii = r if isinstance(r, (list, tuple)) else [r] * nb
    device = torch.cuda.get_device_name(0)
    key = _key(sizes, kernels, radii, curve, candidates, stages, fills, buckets, record_budget, device)
    path = cache_path or default_cache_path()
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
    if key in cache:
        out = dict(cache[key])
        out["cached"] = True
        return out

    # 1. neighbour counts of every cloud
    probe = BatchPlan(xyz, sizes, curve, 21, 32, kernels, radii, capacity=0)
    probe.run()
    off = probe.offsets.cpu().numpy().astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    mu = np.array([(off[starts[c + 1]] - off[starts[c]]) / max(sizes[c], 1) for c in range(nb)])
    del probe
    # 2. groups by mu
    nbk = max(1, min(int(buckets), nb))
    edges = np.quantile(mu, np.linspace(0, 1, nbk + 1)[1:-1]) if nbk > 1 else np.array([])
    group = np.searchsorted(edges, mu, side="right") if nbk > 1 else np.zeros(nb, np.int64)
    # 3. per group: the leaf at the default tile, then the tile at that leaf
    table = {}
    best = {}
    for g in range(nbk):
        members = [c for c in range(nb) if group[c] == g and sizes[c] > 0]
        if not members:
            continue
        sub = torch.cat([xyz[starts[c]:starts[c + 1]] for c in members])
        msz = [sizes[c] for c in members]
        mk = [kernels[c] for c in members]
        mr = [radii[c] for c in members]

        def timed(leaf, stage, fill):
            plan = BatchPlan(sub, msz, curve, 21, int(leaf), mk, mr, record=(fill == "record"), stage=int(stage))
            ms = _time_step(plan, repeats)
            del plan
            torch.cuda.empty_cache()
            if log:
                log(f"[autotune] group {g} ({len(members)} clouds, mu {mu[members].min():.1f}-"
                    f"{mu[members].max():.1f}): leaf {leaf} stage {stage} {fill} fill {ms:.2f} ms")
            return ms

        ms = {}
        by_leaf = {}
        for leaf in candidates:
            by_leaf[int(leaf)] = ms[f"leaf={int(leaf)}"] = timed(leaf, 128, "search")
        leaf = min(by_leaf, key=by_leaf.get)
        tiles = {(128, "search"): by_leaf[leaf]}
        fits = record_bytes(msz) <= record_budget
        for stage in stages:
            for fill in fills:
                if (int(stage), fill) in tiles or (fill == "record" and not fits):
                    continue
                tiles[(int(stage), fill)] = timed(leaf, stage, fill)
        for (stage, fill), v in tiles.items():
            ms[f"leaf={leaf}/stage={stage}/fill={fill}"] = v
        stage, fill = min(tiles, key=tiles.get)
        table[g] = ms
        best[g] = (leaf, stage, fill)
    fallback = (min(candidates), 128, "search")
    choice = [best.get(int(group[c]), fallback) for c in range(nb)]
    leaves = [int(x[0]) for x in choice]
    stages_c = [int(x[1]) for x in choice]
    record = [x[2] == "record" for x in choice]
    # 5. the whole batch with the groups' fills against one fill for all
    whole = {}
    if len(set(record)) > 1:
        fills_whole = {"per_group": record, "search": [False] * nb}
        if record_bytes(sizes) <= record_budget:
            fills_whole["record"] = [True] * nb
        for name, rec in fills_whole.items():
            plan = BatchPlan(xyz, sizes, curve, 21, leaves, kernels, radii, record=rec, stage=stages_c)
            whole[name] = _time_step(plan, repeats)
            del plan
            torch.cuda.empty_cache()
            if log:
                log(f"[autotune] whole batch, {name} fills: {whole[name]:.2f} ms")
        record = fills_whole[min(whole, key=whole.get)]
    out = {"leaf": leaves, "stage": stages_c, "record": record, "bucket": [int(x) for x in group],
           "mu": [float(x) for x in mu], "table": {str(g): t for g, t in table.items()},
           "whole": whole, "edges": [float(x) for x in edges]}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cache[key] = out
        with open(path, "w") as f:
            json.dump(cache, f)
    except OSError:
        pass
    out = dict(out)
    out["cached"] = False
    return out
