"""Leaf-size autotuner for batches of clouds.

The best octree threshold N_max depends on how many neighbours a query has:
small leaves prune finely when neighbourhoods are small, large leaves cut
traversal work when they are large.  The tuner measures it instead of
guessing:

  1. one counting step of the whole batch (leaf 32) gives every cloud's mean
     neighbour count mu;
  2. clouds are split into `buckets` groups by mu (quantiles);
  3. each group is built and searched as its own batch with every candidate
     leaf size (median of `repeats` timed steps after a warm-up);
  4. every cloud gets the fastest leaf size of its group.

Results are cached in a JSON file keyed by the batch description (sizes,
kernels, radii, curve, candidates, device name), so a repeated workload skips
the measurement.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from .plan import BatchPlan

CANDIDATES = (16, 32, 64, 128)


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "sfcoct", "autotune.json")


def _key(sizes, kernels, radii, curve, candidates, buckets, device) -> str:
    h = hashlib.sha256()
    h.update(json.dumps([list(map(int, sizes)), list(map(str, kernels)), [float(x) for x in radii], str(curve),
                         list(map(int, candidates)), int(buckets), str(device)]).encode())
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


def tune_leaf(xyz, sizes, kernel, r, curve="hilbert", candidates=CANDIDATES, buckets: int = 4, repeats: int = 2,
              cache_path: str | None = None, log=None) -> dict:
    """Returns {"leaf": per-cloud leaf sizes, "bucket": per-cloud group,
    "mu": per-cloud mean neighbour count, "table": {group: {leaf: ms}},
    "cached": bool}."""
    import torch
    sizes = [int(x) for x in sizes]
    nb = len(sizes)
    kernels = kernel if isinstance(kernel, (list, tuple)) else [kernel] * nb
    radii = r if isinstance(r, (list, tuple)) else [r] * nb
    device = torch.cuda.get_device_name(0)
    key = _key(sizes, kernels, radii, curve, candidates, buckets, device)
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
    # 3. time every group with every candidate
    table = {}
    best = {}
    for g in range(nbk):
        members = [c for c in range(nb) if group[c] == g and sizes[c] > 0]
        if not members:
            continue
        sub = torch.cat([xyz[starts[c]:starts[c + 1]] for c in members])
        ms = {}
        for leaf in candidates:
            plan = BatchPlan(sub, [sizes[c] for c in members], curve, 21, int(leaf), [kernels[c] for c in members],
                             [radii[c] for c in members])
            ms[int(leaf)] = _time_step(plan, repeats)
            del plan
            if log:
                log(f"[autotune] group {g} ({len(members)} clouds, mu {mu[members].min():.1f}-"
                    f"{mu[members].max():.1f}): leaf {leaf} {ms[int(leaf)]:.2f} ms")
        table[g] = ms
        best[g] = min(ms, key=ms.get)
    fallback = min(candidates)
    leaf = [int(best.get(int(group[c]), fallback)) for c in range(nb)]
    out = {"leaf": leaf, "bucket": [int(x) for x in group], "mu": [float(x) for x in mu],
           "table": {str(g): {str(k): v for k, v in ms.items()} for g, ms in table.items()},
           "edges": [float(x) for x in edges]}
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
