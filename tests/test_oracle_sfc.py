"""Pins for the oracle's frame, discretisation, Morton and Hilbert codes and
sort (paper Section 4).  Each test ties the oracle to something other than
itself: the paper's worked example, the SFC definitions (bijectivity,
recursivity, continuity), closed forms and library sorts."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _all_cells(bits):
    n = 1 << bits
    g = np.indices((n, n, n)).reshape(3, -1).T
    return [tuple(int(v) for v in row) for row in g]


def test_morton_worked_example():
    # Section 4.1: (3, 7, 2) at L = 3 -> 190
    rows = [l.split() for l in open(os.path.join(GOLDEN, "morton_example.txt")) if l.strip() and not l.startswith("#")]
    for bits, x, y, z, key in rows:
        assert oracle.morton_encode(int(x), int(y), int(z), int(bits)) == int(key)
        assert oracle.morton_decode(int(key), int(bits)) == (int(x), int(y), int(z))


@pytest.mark.parametrize("curve", ["morton", "hilbert"])
@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_bijection_exhaustive(curve, bits):
    enc = oracle.morton_encode if curve == "morton" else oracle.hilbert_encode
    dec = oracle.morton_decode if curve == "morton" else oracle.hilbert_decode
    cells = _all_cells(bits)
    keys = [enc(x, y, z, bits) for (x, y, z) in cells]
    # a bijection of S_L onto [0, 2^{3L})
    assert sorted(keys) == list(range(1 << (3 * bits)))
    for c, k in zip(cells, keys):
        assert dec(k, bits) == c


@pytest.mark.parametrize("curve", ["morton", "hilbert"])
@pytest.mark.parametrize("bits", [2, 3, 4])
def test_recursive_prefix_is_aligned_cube(curve, bits):
    # Definition of a recursive SFC: the codes sharing a 3l-bit prefix fill one
    # aligned sub-cube of side 2^(L-l) (the 8 sub-curves own consecutive ranges).
    dec = oracle.morton_decode if curve == "morton" else oracle.hilbert_decode
    pts = np.array([dec(k, bits) for k in range(1 << (3 * bits))])
    for level in range(bits + 1):
        side = 1 << (bits - level)
        group = side ** 3
        for g0 in range(0, 1 << (3 * bits), group):
            blk = pts[g0:g0 + group]
            lo = blk.min(0)
            assert np.all(lo % side == 0)
            assert np.all(blk.max(0) - lo == side - 1)
            assert len({tuple(p) for p in blk}) == group


@pytest.mark.parametrize("bits", [1, 2, 3, 4, 5])
def test_hilbert_continuity_exhaustive(bits):
    # Continuity (Section 4, Definition): consecutive codes are neighbouring
    # cells.  Hilbert curves are face-continuous: L1 distance exactly 1, which
    # implies the paper's L-infinity distance 1.
    pts = np.array([oracle.hilbert_decode(k, bits) for k in range(1 << (3 * bits))], dtype=np.int64)
    step = np.abs(np.diff(pts, axis=0))
    assert np.all(step.sum(1) == 1)
    assert tuple(pts[0]) == (0, 0, 0)


def test_morton_is_not_continuous():
    # Section 4.2: Morton codes jump between sub-blocks (L-inf distance > 1 exists)
    bits = 3
    pts = np.array([oracle.morton_decode(k, bits) for k in range(1 << (3 * bits))], dtype=np.int64)
    step = np.abs(np.diff(pts, axis=0)).max(1)
    assert step.max() > 1


def test_codes_at_21_bits_random_roundtrip():
    rng = np.random.default_rng(5)
    for curve in ("morton", "hilbert"):
        enc = oracle.morton_encode if curve == "morton" else oracle.hilbert_encode
        dec = oracle.morton_decode if curve == "morton" else oracle.hilbert_decode
        cells = rng.integers(0, 1 << 21, (2000, 3))
        seen = set()
        for x, y, z in cells:
            k = enc(int(x), int(y), int(z), 21)
            assert k < (1 << 63)  # 63-bit code, top bit of the 64-bit word unused
            assert dec(k, 21) == (int(x), int(y), int(z))
            seen.add(k)
        assert len(seen) == len({tuple(c) for c in cells.tolist()})
        assert enc((1 << 21) - 1, (1 << 21) - 1, (1 << 21) - 1, 21) < (1 << 63)


def test_hilbert_continuity_at_21_bits_sampled():
    rng = np.random.default_rng(11)
    for k in rng.integers(1, (1 << 63) - 1, 3000, dtype=np.int64):
        a = np.array(oracle.hilbert_decode(int(k) - 1, 21), np.int64)
        b = np.array(oracle.hilbert_decode(int(k), 21), np.int64)
        assert np.abs(a - b).sum() == 1


def test_frame_and_cells_closed_form():
    # Section 4 steps 1-2: lower corner -> cell 0, upper corner clamped to the
    # last cell (B is half-open), isotropic scale 2^L / E.
    pts = np.array([[1.0, 2.0, 3.0], [5.0, 4.0, 3.5], [3.0, 3.0, 3.25]], np.float32)
    lo, s = oracle.frame(pts, 21)
    assert list(lo) == [1.0, 2.0, 3.0]
    assert s == np.float32(2.0 ** 21 / 4.0)  # E = 4 (x side)
    assert oracle.cell(1.0, 1.0, s, 21) == 0
    assert oracle.cell(5.0, 1.0, s, 21) == (1 << 21) - 1
    assert oracle.cell(3.0, 1.0, s, 21) == 1 << 20  # midpoint of the x side
    assert oracle.cell(0.0, 1.0, s, 21) == 0        # below the box: first cell
    # y spans only half of E: its last point sits in the middle of the grid
    assert oracle.cell(4.0, 2.0, s, 21) == 1 << 20
    # degenerate cloud: E = 1
    lo, s = oracle.frame(np.ones((4, 3), np.float32), 21)
    assert s == np.float32(2.0 ** 21)
    # empty cloud
    lo, s = oracle.frame(np.zeros((0, 3), np.float32), 21)
    assert list(lo) == [0, 0, 0] and s == np.float32(2.0 ** 21)


def test_encode_uses_frame_and_curve():
    pts = np.array([[0, 0, 0], [1, 1, 1], [0.5, 0.25, 0.75]], np.float32)
    for curve, enc in (("morton", oracle.morton_encode), ("hilbert", oracle.hilbert_encode)):
        keys, lo, s = oracle.encode(pts, curve, 4)
        assert s == np.float32(16.0)
        assert keys[0] == enc(0, 0, 0, 4)
        assert keys[1] == enc(15, 15, 15, 4)
        assert keys[2] == enc(8, 4, 12, 4)


def test_sort_matches_library_lexsort():
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 50, 5000).astype(np.uint64)  # many ties
    ks, perm = oracle.sort(keys)
    ref = np.lexsort((np.arange(keys.size), keys))
    assert np.array_equal(perm, ref.astype(np.uint32))
    assert np.array_equal(ks, keys[ref])
    ks0, perm0 = oracle.sort(np.zeros(0, np.uint64))
    assert ks0.size == 0 and perm0.size == 0
