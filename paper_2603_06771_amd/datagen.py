"""Seeded synthetic point clouds and request streams.

This module holds no arithmetic of the search method: it only draws inputs.
Both the GPU path and the CPU oracle receive the same arrays from it.  The
random source is numpy's PCG64 (O'Neill, "PCG: A family of simple fast
space-efficient statistically good algorithms for random number generation",
2014); values are drawn in float64 and stored as float32.

Workloads (stand-ins for the paper's LiDAR datasets, which are not shipped):

* ``uniform(n, seed)``: n points uniform in [0, 1)^3.
* ``lidar_tile(n, seed)``: an aerial-LiDAR-like tile.  90% of the points are
  ground, (x, y) uniform over a square of side 1000 m * sqrt(n / 1e7) and
  z = h(x, y) + N(0, 0.05^2), h a sum of 8 random-phase plane sines with
  amplitudes U(0, 2.5) m (|h| <= 20 m), wavelengths log-uniform in
  [20, 1000] m and uniform random directions.  10% are vegetation: clusters
  of 500 points ~ N(centre, sigma^2 I), sigma ~ U(1, 3) m, centre (x, y)
  uniform, centre z = h + U(2, 10) m.  At n = 1e7 this is 9 ground points per
  square metre and 2000 clusters.  Original order: ground, then clusters.
* ``batch_mix``: many clouds of log-uniform size, half uniform (1 point per
  cubic metre), half LiDAR tiles, each with its own radius and kernel.
* ``request_stream``: Poisson arrivals of radius / k-NN requests on resident
  clouds.
"""
from __future__ import annotations

import numpy as np

SEED_UNIFORM = 1
SEED_LIDAR = 2603
SEED_BATCH = 10000
SEED_SERVED = 20000
SEED_STREAM = 30000


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform(n: int, seed: int = SEED_UNIFORM, side: float = 1.0) -> np.ndarray:
    """n points uniform in [0, side)^3 as float32 (n, 3)."""
    rng = _rng(seed)
    pts = rng.random((int(n), 3), dtype=np.float32)
    if side != 1.0:
        pts = (pts.astype(np.float64) * side).astype(np.float32)
        np.minimum(pts, np.nextafter(np.float32(side), np.float32(0)), out=pts)
    return pts


def _heightfield(rng: np.random.Generator, nsines: int = 8):
    amp = rng.uniform(0.0, 2.5, nsines)
    lam = np.exp(rng.uniform(np.log(20.0), np.log(1000.0), nsines))
    ang = rng.uniform(0.0, 2.0 * np.pi, nsines)
    phase = rng.uniform(0.0, 2.0 * np.pi, nsines)
    ux, uy = np.cos(ang), np.sin(ang)

    def h(x: np.ndarray, y: np.ndarray) -> np.ndarray:
        z = np.zeros_like(x)
        for i in range(nsines):
            z += amp[i] * np.sin(2.0 * np.pi * (ux[i] * x + uy[i] * y) / lam[i] + phase[i])
        return z

    return h


def lidar_tile(n: int = 10_000_000, seed: int = SEED_LIDAR, cluster_points: int = 500,
               veg_fraction: float = 0.1) -> np.ndarray:
    """Synthetic LiDAR tile of n points (float32 (n, 3)), see module docstring."""
    n = int(n)
    rng = _rng(seed)
    side = 1000.0 * np.sqrt(n / 1e7)
    h = _heightfield(rng)
    n_clusters = int(round(n * veg_fraction / cluster_points))
    n_veg = n_clusters * cluster_points
    n_ground = n - n_veg
    out = np.empty((n, 3), np.float32)
    chunk = 1 << 22
    for s in range(0, n_ground, chunk):
        e = min(n_ground, s + chunk)
        x = rng.uniform(0.0, side, e - s)
        y = rng.uniform(0.0, side, e - s)
        z = h(x, y) + rng.normal(0.0, 0.05, e - s)
        out[s:e, 0] = x
        out[s:e, 1] = y
        out[s:e, 2] = z
    if n_clusters:
        cx = rng.uniform(0.0, side, n_clusters)
        cy = rng.uniform(0.0, side, n_clusters)
        cz = h(cx, cy) + rng.uniform(2.0, 10.0, n_clusters)
        sig = rng.uniform(1.0, 3.0, n_clusters)
        g = rng.normal(0.0, 1.0, (n_veg, 3))
        rep = np.repeat(np.arange(n_clusters), cluster_points)
        out[n_ground:, 0] = cx[rep] + sig[rep] * g[:, 0]
        out[n_ground:, 1] = cy[rep] + sig[rep] * g[:, 1]
        out[n_ground:, 2] = cz[rep] + sig[rep] * g[:, 2]
    return out


def with_duplicates(pts: np.ndarray, n_dup: int, seed: int = 7) -> np.ndarray:
    """Append n_dup exact copies of randomly chosen points (ties in every key)."""
    rng = _rng(seed)
    pick = rng.integers(0, pts.shape[0], int(n_dup))
    return np.concatenate([pts, pts[pick]], axis=0)


def batch_mix_specs(n_clouds: int = 256, seed: int = SEED_BATCH, n_min: float = 1e4, n_max: float = 2e6):
    """Descriptors {n, kind, kernel, radius, seed} of the clouds of batch_mix,
    without generating the points (so a test can pick some of them).

    Sizes are log-uniform in [n_min, n_max]; each cloud is uniform (one point
    per cubic metre) or a LiDAR tile with probability 1/2; the radius is
    U(0.5, 3) m and the kernel uniform over the four kernels."""
    rng = _rng(seed)
    kernels = ["sphere", "circle", "cube", "square"]
    out = []
    for i in range(int(n_clouds)):
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        kind = "uniform" if rng.random() < 0.5 else "lidar"
        out.append({"n": n, "kind": kind, "kernel": kernels[int(rng.integers(0, 4))],
                    "radius": float(np.float32(rng.uniform(0.5, 3.0))), "seed": seed + 1 + i})
    return out


def batch_cloud(spec) -> np.ndarray:
    """The points of one batch_mix_specs descriptor."""
    n = spec["n"]
    if spec["kind"] == "uniform":
        return uniform(n, seed=spec["seed"], side=float(n) ** (1.0 / 3.0))
    return lidar_tile(n, seed=spec["seed"])


def batch_mix(n_clouds: int = 256, seed: int = SEED_BATCH, n_min: float = 1e4, n_max: float = 2e6):
    """List of cloud descriptors {points, kind, kernel, radius} for the batched
    workload (see batch_mix_specs)."""
    out = []
    for spec in batch_mix_specs(n_clouds, seed, n_min, n_max):
        out.append({"points": batch_cloud(spec), "kind": spec["kind"], "kernel": spec["kernel"],
                    "radius": spec["radius"]})
    return out


def served_sizes(n_clouds: int = 64, seed: int = SEED_SERVED, n_min: float = 3.5e6, n_max: float = 9e6):
    """Point counts of the resident clouds of the served workload (uniform in
    [n_min, n_max]); cloud i is lidar_tile(sizes[i], seed + 1 + i)."""
    rng = _rng(seed)
    return [int(x) for x in np.round(rng.uniform(n_min, n_max, int(n_clouds)))]


def _sample_rows(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """k distinct row ids of [0, n), ascending (draws with replacement, keeps
    the distinct ones and tops up, then keeps a random subset of exactly k)."""
    if 2 * k >= n:
        return np.sort(rng.permutation(n)[:k]).astype(np.int64)
    got = np.unique(rng.integers(0, n, k + k // 2 + 16))
    while got.size < k:
        got = np.unique(np.concatenate([got, rng.integers(0, n, k - got.size + 16)]))
    return np.sort(rng.permutation(got)[:k]).astype(np.int64)


def request_stream(n_requests: int, n_clouds: int, cloud_sizes, rate_per_s: float,
                   seed: int = SEED_STREAM, q_min: float = 1e3, q_max: float = 1e6):
    """Poisson request stream: arrival time, cloud id, query rows (distinct
    points of that cloud), and either a radius search (r ~ U(0.5, 3), kernel
    uniform) or a k-NN search (k in {8, 16, 32}).  Arrival times scale as
    1 / rate_per_s; everything else does not depend on the rate."""
    rng = _rng(seed)
    kernels = ["sphere", "circle", "cube", "square"]
    t = 0.0
    out = []
    for i in range(int(n_requests)):
        t += rng.exponential(1.0)
        cid = int(rng.integers(0, n_clouds))
        n = int(cloud_sizes[cid])
        nq = int(round(np.exp(rng.uniform(np.log(q_min), np.log(q_max)))))
        nq = max(1, min(nq, n))
        rows = _sample_rows(rng, n, nq)
        if rng.random() < 0.5:
            req = {"op": "radius", "kernel": kernels[int(rng.integers(0, 4))],
                   "radius": float(np.float32(rng.uniform(0.5, 3.0)))}
        else:
            req = {"op": "knn", "k": int([8, 16, 32][int(rng.integers(0, 3))])}
        req.update({"id": i, "arrival": t / float(rate_per_s), "cloud": cid, "rows": rows})
        out.append(req)
    return out
