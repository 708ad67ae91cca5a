"""Pins for the oracle's fixed-radius (Section 3.2) and k-NN (Section 3.3)
searches: closed-form neighbourhoods on integer lattices, all-pairs brute
force on tiny clouds (a different algorithm from the oracle's grid), the real
(fp64) definition away from the boundary, and k-NN / radius consistency."""
import numpy as np
import pytest

import oracle
from paper_2603_06771_amd import datagen

KERNELS = ["sphere", "circle", "cube", "square"]


def _lattice(m=5):
    g = np.indices((m, m, m)).reshape(3, -1).T.astype(np.float32)
    return g


# closed-form neighbourhood sizes of the centre (2,2,2) of the 5^3 lattice
LATTICE_COUNTS = {
    # r = 1: strict inequalities exclude the unit-distance points
    (1.0, "sphere"): 1, (1.0, "cube"): 1, (1.0, "circle"): 5, (1.0, "square"): 5,
    # r = 1.5: d2 in {0,1,2}; cube 3x3x3; 2D kernels 3x3 columns of 5
    (1.5, "sphere"): 19, (1.5, "cube"): 27, (1.5, "circle"): 45, (1.5, "square"): 45,
    # r = 2: d2 = 3 corners in, d2 = 4 axis points out
    (2.0, "sphere"): 27, (2.0, "cube"): 27, (2.0, "circle"): 45, (2.0, "square"): 45,
    # r = 2.5: sphere d2 < 6.25 -> 1+6+12+8+6(d2=4)+24(d2=5)+24(d2=6) = 81; cube 5^3
    (2.5, "sphere"): 81, (2.5, "cube"): 125, (2.5, "circle"): 105, (2.5, "square"): 125,
}


@pytest.mark.parametrize("key", sorted(LATTICE_COUNTS))
def test_lattice_closed_form(key):
    r, kernel = key
    pts = _lattice()
    c = np.array([[2, 2, 2]], np.float32)
    counts, off, idx = oracle.radius_search(pts, c, kernel, r)
    assert int(counts[0]) == LATTICE_COUNTS[key]
    # non-positive radius: the empty set
    assert int(oracle.radius_search(pts, c, kernel, 0.0)[0][0]) == 0
    assert int(oracle.radius_search(pts, c, kernel, -1.0)[0][0]) == 0


def _brute(pts, q, kernel, r):
    r = np.float32(r)
    out = []
    for c in q:
        dx = pts[:, 0] - c[0]
        dy = pts[:, 1] - c[1]
        dz = pts[:, 2] - c[2]
        if not r > 0:
            m = np.zeros(len(pts), bool)
        elif kernel == "sphere":
            m = ((dx * dx + dy * dy) + dz * dz) < r * r
        elif kernel == "circle":
            m = (dx * dx + dy * dy) < r * r
        elif kernel == "cube":
            m = (np.abs(dx) < r) & (np.abs(dy) < r) & (np.abs(dz) < r)
        else:
            m = (np.abs(dx) < r) & (np.abs(dy) < r)
        out.append(np.nonzero(m)[0].astype(np.uint32))
    return out


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("gen", ["uniform", "lidar"])
def test_grid_matches_brute_force(kernel, gen):
    rng = np.random.default_rng(17)
    pts = datagen.uniform(1500, seed=4) if gen == "uniform" else datagen.lidar_tile(1500, seed=4)
    pts = datagen.with_duplicates(pts, 100, seed=2)
    ext = float(np.max(pts.max(0) - pts.min(0)))
    # queries: every cloud point plus outside / on-the-box-corner centres
    extra = np.array([pts.min(0), pts.max(0), pts.min(0) - 0.05 * ext, pts.max(0) + 0.01 * ext], np.float32)
    q = np.concatenate([pts, extra])
    for r in [0.0, ext * 0.004, ext * 0.03, ext * float(rng.uniform(0.05, 0.12))]:
        counts, off, idx = oracle.radius_search(pts, q, kernel, r)
        ref = _brute(pts, q, kernel, r)
        assert np.array_equal(counts, np.array([len(x) for x in ref], np.uint32))
        for i in range(len(q)):
            assert np.array_equal(idx[off[i]:off[i + 1]], ref[i])


def test_fp32_predicate_agrees_with_real_definition_off_boundary():
    pts = datagen.uniform(800, seed=8)
    q = pts[:200]
    r = 0.09
    counts, off, idx = oracle.radius_search(pts, q, "sphere", r)
    p64, q64 = pts.astype(np.float64), q.astype(np.float64)
    d = np.sqrt(((p64[None, :, :] - q64[:, None, :]) ** 2).sum(-1))
    for i in range(len(q)):
        got = set(idx[off[i]:off[i + 1]].tolist())
        inside = set(np.nonzero(d[i] < r * (1 - 1e-5))[0].tolist())
        outside = set(np.nonzero(d[i] > r * (1 + 1e-5))[0].tolist())
        assert inside <= got and not (got & outside)


def test_kernel_inclusions_and_monotonicity():
    pts = datagen.lidar_tile(3000, seed=12)
    q = pts[::7]
    sets = {}
    for kernel in KERNELS:
        for r in (1.0, 2.0):
            c, o, i = oracle.radius_search(pts, q, kernel, r)
            sets[kernel, r] = [set(i[o[j]:o[j + 1]].tolist()) for j in range(len(q))]
    for j in range(len(q)):
        for r in (1.0, 2.0):
            assert sets["sphere", r][j] <= sets["cube", r][j] <= sets["square", r][j]
            assert sets["sphere", r][j] <= sets["circle", r][j] <= sets["square", r][j]
        for kernel in KERNELS:
            assert sets[kernel, 1.0][j] <= sets[kernel, 2.0][j]


def _brute_knn(pts, q, k):
    idx = np.full((len(q), k), 0xFFFFFFFF, np.uint32)
    d2 = np.full((len(q), k), np.inf, np.float32)
    for i, c in enumerate(q):
        dx = pts[:, 0] - c[0]
        dy = pts[:, 1] - c[1]
        dz = pts[:, 2] - c[2]
        d = (dx * dx + dy * dy) + dz * dz
        order = np.lexsort((np.arange(len(pts)), d))[:k]
        idx[i, :len(order)] = order
        d2[i, :len(order)] = d[order]
    return idx, d2


def test_knn_lattice_closed_form():
    pts = _lattice()
    centre = 2 * 25 + 2 * 5 + 2
    idx, d2 = oracle.knn(pts, pts[[centre]], 19, h=1.0)
    # self, then the 6 face neighbours (d2 = 1) and 12 edge neighbours (d2 = 2),
    # ties in index order
    faces = sorted([centre + s for s in (-25, 25, -5, 5, -1, 1)])
    edges = sorted([centre + a + b for a in (-25, 25) for b in (-5, 5, -1, 1)] + [centre + a + b for a in (-5, 5) for b in (-1, 1)])
    assert idx[0].tolist() == [centre] + faces + edges
    assert d2[0].tolist() == [0.0] + [1.0] * 6 + [2.0] * 12


@pytest.mark.parametrize("k", [1, 8, 32])
@pytest.mark.parametrize("gen", ["uniform", "lidar"])
def test_knn_grid_matches_brute_force(k, gen):
    pts = datagen.uniform(1200, seed=21) if gen == "uniform" else datagen.lidar_tile(1200, seed=21)
    pts = datagen.with_duplicates(pts, 150, seed=5)
    q = np.concatenate([pts[::3], pts.min(0, keepdims=True) - 0.5])
    ext = float(np.max(pts.max(0) - pts.min(0)))
    for h in (ext / 40, ext / 7):
        idx, d2 = oracle.knn(pts, q, k, h=h)
        ridx, rd2 = _brute_knn(pts, q, k)
        assert np.array_equal(idx, ridx)
        assert np.array_equal(d2, rd2)


def test_knn_padding_when_k_exceeds_n():
    pts = datagen.uniform(5, seed=1)
    idx, d2 = oracle.knn(pts, pts, 8, h=0.5)
    assert np.all(idx[:, 5:] == 0xFFFFFFFF) and np.all(np.isinf(d2[:, 5:]))
    assert np.array_equal(idx[:, 0], np.arange(5))


def test_knn_radius_consistency():
    # the k-NN set of a centre is sandwiched between two sphere searches:
    # sphere(r_in) <= kNN <= sphere(r_out) with fl(r_in^2) <= d2_k < fl(r_out^2)
    pts = datagen.lidar_tile(4000, seed=31)
    q = pts[::11]
    k = 16
    idx, d2 = oracle.knn(pts, q, k, h=2.0)
    for i in range(len(q)):
        kth = np.float32(d2[i, -1])
        r_in = np.float32(np.sqrt(kth))
        while r_in * r_in > kth:
            r_in = np.nextafter(r_in, np.float32(0))
        r_out = np.float32(np.sqrt(kth))
        while not r_out * r_out > kth:
            r_out = np.nextafter(r_out, np.float32(np.inf))
        knn_set = set(idx[i].tolist())
        _, _, inner = oracle.radius_search(pts, q[i:i + 1], "sphere", float(r_in))
        _, _, outer = oracle.radius_search(pts, q[i:i + 1], "sphere", float(r_out))
        assert set(inner.tolist()) <= knn_set <= set(outer.tolist())
