"""Pins of the oracle's kNN locality histogram (Section 5.2): a hand-worked
example, the two identities the paper states (H_k(0) = N, sum H_k = kN), and
the shape under a random permutation, where the distance between two random
positions follows the triangular law of |U1 - U2| whose skewness is
2*sqrt(2)/5."""
import os

import numpy as np

import oracle
from paper_2603_06771_amd import datagen

GOLD = os.path.join(os.path.dirname(__file__), "golden", "locality_line.txt")
GOLD_SKEWED = os.path.join(os.path.dirname(__file__), "golden", "locality_skewed.txt")


def _gold(path=GOLD):
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        out[key] = [float(v) for v in vals]
    return out


def test_hand_worked_line():
    g = _gold()
    x = np.array(g["points"], np.float32)
    pts = np.stack([x, np.zeros_like(x), np.zeros_like(x)], axis=1)
    k = int(g["k"][0])
    idx, _ = oracle.knn(pts, pts, k)
    H, st = oracle.locality_histogram(np.arange(5), idx)
    assert list(H) == [int(v) for v in g["hist"]]
    for key in ("total", "mean", "std", "g1", "q1", "q2", "q3", "max"):
        assert abs(st[key] - g[key][0]) < 1e-12, key
    # stored in reverse order: position i holds original point 4 - i
    rev = pts[::-1].copy()
    idx, _ = oracle.knn(rev, rev, k)
    H, _ = oracle.locality_histogram(np.arange(5)[::-1], np.arange(5)[::-1][idx])
    assert list(H) == [int(v) for v in g["reversed_hist"]]


def test_hand_worked_skewed():
    """An asymmetric example: one pair at distance 3 among pairs at distance
    1 gives G1 = 352/243 (worked by hand in the fixture)."""
    g = _gold(GOLD_SKEWED)
    x = np.array(g["points"], np.float32)
    pts = np.stack([x, np.zeros_like(x), np.zeros_like(x)], axis=1)
    k = int(g["k"][0])
    idx, _ = oracle.knn(pts, pts, k)
    H, st = oracle.locality_histogram(np.arange(5), idx)
    assert list(H) == [int(v) for v in g["hist"]]
    for key in ("total", "mean", "std", "g1", "q1", "q2", "q3", "max"):
        assert abs(st[key] - g[key][0]) < 1e-12, key
    assert abs(st["g1"] - 352.0 / 243.0) < 1e-12


def _random_order_g1(k: int) -> float:
    """Skewness of the full histogram under a random storage order: a point
    mass at 0 (the centre, weight 1/k) mixed with the triangular law of
    |U1 - U2| on [0, 1] (density 2(1 - t); raw moments 1/3, 1/6, 1/10)."""
    w = 1.0 - 1.0 / k
    m1, m2, m3 = w / 3.0, w / 6.0, w / 10.0
    var = m2 - m1 * m1
    mu3 = m3 - 3.0 * m1 * m2 + 2.0 * m1 ** 3
    return mu3 / var ** 1.5


def _sorted_cloud(n, curve, seed):
    pts = datagen.uniform(n, seed=seed)
    keys, _, _ = oracle.encode(pts, curve, 21)
    _, perm = oracle.sort(keys)
    return pts[perm], perm


def test_identities_in_curve_order():
    for curve in ("morton", "hilbert"):
        sp, perm = _sorted_cloud(3000, curve, 3)
        k = 8
        # queries are the stored points in order; neighbours as original indices
        idx, _ = oracle.knn(sp, sp, k)
        H, st = oracle.locality_histogram(perm, perm[idx])
        assert H[0] == 3000 and H.sum() == k * 3000 and st["total"] == k * 3000
        assert st["g1"] > 3.0  # strongly left-skewed: neighbours are stored close


def test_random_order_skewness():
    n, k = 20000, 8
    pts = datagen.uniform(n, seed=5)
    rng = np.random.default_rng(5)
    perm = rng.permutation(n)
    sp = pts[perm]
    idx, _ = oracle.knn(sp, sp, k)
    H, st = oracle.locality_histogram(perm, perm[idx])
    assert H[0] == n and H.sum() == k * n
    # without the centres the distances are those of random pairs of positions
    Hn = H.copy()
    Hn[0] = 0
    d = np.arange(n, dtype=np.float64)
    w = Hn / Hn.sum()
    m = (w * d).sum()
    s = np.sqrt((w * (d - m) ** 2).sum())
    g1 = (w * ((d - m) / s) ** 3).sum()
    assert abs(m / n - 1.0 / 3.0) < 0.01
    assert abs(g1 - 2.0 * np.sqrt(2.0) / 5.0) < 0.03
    # with the centres: the point mass at 0 mixed with the triangular law
    assert abs(st["g1"] - _random_order_g1(k)) < 0.03
    assert abs(st["mean"] / n - (1.0 - 1.0 / k) / 3.0) < 0.01


def test_subset_rows():
    sp, perm = _sorted_cloud(4000, "hilbert", 9)
    rows = np.sort(np.random.default_rng(2).choice(4000, 400, replace=False))
    idx, _ = oracle.knn(sp, sp[rows], 6)
    H, st = oracle.locality_histogram(perm, perm[idx], rows)
    assert H[0] == 400 and H.sum() == 6 * 400
    # the full histogram restricted to those rows
    idx_all, _ = oracle.knn(sp, sp, 6)
    Hf, _ = oracle.locality_histogram(perm, perm[idx_all[rows]], rows)
    assert np.array_equal(H, Hf)
