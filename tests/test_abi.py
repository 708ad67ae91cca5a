"""CPU checks of the C ABI: the library loads, exports every function that
include/sfcoct.h declares, and its host-only paths (size queries, argument
validation) behave as documented.  No call here launches GPU work."""
import ctypes
import os
import re

import pytest

from paper_2603_06771_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfcoct.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2603_06771_amd import build
        build.build()
    return B.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_lists_the_entry_points():
    names = _declared()
    for n in ("encode_sfc", "octree_bytes", "build_linear_octree", "radius_search", "knn_search",
              "sfc_last_error", "sfc_version"):
        assert n in names
    assert set(names) == set(B.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.sfc_version()


def test_octree_bytes_bound(lib):
    b = ctypes.c_size_t(0)
    assert lib.octree_bytes(0, 8, 21, ctypes.byref(b)) == B.SFC_OK and b.value > 0
    assert lib.octree_bytes(10_000_000, 16, 21, ctypes.byref(b)) == B.SFC_OK
    small = b.value
    assert lib.octree_bytes(10_000_000, 128, 21, ctypes.byref(b)) == B.SFC_OK
    assert b.value < small
    # invalid arguments
    assert lib.octree_bytes(-1, 8, 21, ctypes.byref(b)) == B.SFC_EINVAL
    assert lib.octree_bytes(10, 0, 21, ctypes.byref(b)) == B.SFC_EINVAL
    assert lib.octree_bytes(10, 8, 22, ctypes.byref(b)) == B.SFC_EINVAL
    assert b"invalid" in lib.sfc_last_error()
    # node bound beyond int32 is refused, not overflowed
    assert lib.octree_bytes(0xFFFFFFFF, 1, 21, ctypes.byref(b)) == B.SFC_ENOTSUP


def test_workspace_size_queries_do_not_launch(lib):
    need = ctypes.c_size_t(0)
    # encode: ws == NULL only reports the size
    assert lib.encode_sfc(None, 0, 0, 21, None, None, None, ctypes.byref(need), None) == B.SFC_OK
    assert need.value >= 256
    # invalid curve / bits are rejected before anything is enqueued
    fake = ctypes.c_void_p(256)
    rc = lib.encode_sfc(fake, 10, 7, 21, fake, fake, fake, ctypes.byref(ctypes.c_size_t(1 << 20)), None)
    assert rc == B.SFC_EINVAL
    rc = lib.encode_sfc(fake, 10, 0, 0, fake, fake, fake, ctypes.byref(ctypes.c_size_t(1 << 20)), None)
    assert rc == B.SFC_EINVAL
    # too small a workspace is reported as such
    rc = lib.encode_sfc(fake, 10, 0, 21, fake, fake, fake, ctypes.byref(ctypes.c_size_t(16)), None)
    assert rc == B.SFC_EWORKSPACE
    # build: size query, then invalid leaf size
    assert lib.build_linear_octree(None, 1000, 1, 21, 16, None, 0, None, None, ctypes.byref(need), None) == B.SFC_OK
    assert need.value > 0
    assert lib.build_linear_octree(None, 1000, 1, 21, 0, None, 0, None, None, ctypes.byref(need), None) \
        == B.SFC_EINVAL


def test_search_argument_validation(lib):
    need = ctypes.c_size_t(0)
    view = B.SfcOctree()  # all-null view: rejected
    rc = lib.radius_search(ctypes.byref(view), None, 0, 0, 1.0, None, None, None, 0, 0, None, ctypes.byref(need),
                           None)
    assert rc == B.SFC_EINVAL
    rc = lib.knn_search(ctypes.byref(view), None, 0, 8, None, None, None, ctypes.byref(need), None)
    assert rc == B.SFC_EINVAL
    # a syntactically valid view with bad parameters
    view.nodes = view.child = view.points = view.keys = view.frame = 256
    view.n = 10
    fake = ctypes.c_void_p(256)
    assert lib.radius_search(ctypes.byref(view), None, 10, 9, 1.0, fake, fake, None, 0, 0, None,
                             ctypes.byref(need), None) == B.SFC_EINVAL  # kernel out of range
    assert lib.radius_search(ctypes.byref(view), None, 11, 0, 1.0, fake, fake, None, 0, 0, None,
                             ctypes.byref(need), None) == B.SFC_EINVAL  # nq != n for cloud queries
    assert lib.radius_search(ctypes.byref(view), None, 10, 0, float("nan"), fake, fake, None, 0, 0, None,
                             ctypes.byref(need), None) == B.SFC_EINVAL
    assert lib.radius_search(ctypes.byref(view), None, 10, 0, 1.0, fake, fake, None, 0, 0, None,
                             ctypes.byref(need), None) == B.SFC_OK and need.value > 0
    assert lib.knn_search(ctypes.byref(view), None, 10, 513, fake, fake, None, ctypes.byref(need), None) \
        == B.SFC_ENOTSUP
    assert lib.knn_search(ctypes.byref(view), None, 10, 0, fake, fake, None, ctypes.byref(need), None) \
        == B.SFC_EINVAL


def test_batched_host_validation(lib):
    nb = 3
    cl = (B.SfcCloud * nb)()
    off = 0
    for c, n in enumerate((1000, 0, 50)):
        cl[c].offset, cl[c].n, cl[c].curve, cl[c].bits, cl[c].leaf_size = off, n, 1, 21, 16
        off += n
    need = ctypes.c_size_t(0)
    assert lib.octree_batch_layout(nb, cl, None, ctypes.byref(need)) == B.SFC_OK and need.value > 0
    # the layout size of a batch of one equals octree_bytes
    one = (B.SfcCloud * 1)()
    one[0].n, one[0].curve, one[0].bits, one[0].leaf_size = 1000, 1, 21, 16
    b1, b2 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.octree_batch_layout(1, one, None, ctypes.byref(b1)) == B.SFC_OK
    assert lib.octree_bytes(1000, 16, 21, ctypes.byref(b2)) == B.SFC_OK and b1.value == b2.value
    # offsets must be the running sum of the sizes
    cl[2].offset = 999
    assert lib.octree_batch_layout(nb, cl, None, ctypes.byref(need)) == B.SFC_EINVAL
    cl[2].offset = 1000
    cl[1].leaf_size = 0
    assert lib.build_linear_octree_batched(None, nb, cl, None, ctypes.byref(need), None) == B.SFC_EINVAL
    cl[1].leaf_size = 16
    assert lib.build_linear_octree_batched(None, nb, cl, None, ctypes.byref(need), None) == B.SFC_OK
    assert need.value > 0
    # searches: trees not laid out -> rejected; kstride above 32 -> not supported
    fake = ctypes.c_void_p(256)
    assert lib.radius_search_batched(nb, cl, None, 1050, fake, fake, None, 0, 0, None, ctypes.byref(need),
                                     None) == B.SFC_EINVAL
    assert lib.knn_search_batched(nb, cl, None, 1050, 513, fake, fake, None, ctypes.byref(need), None) \
        == B.SFC_ENOTSUP


def test_gather_points_validation(lib):
    fake = ctypes.c_void_p(256)
    assert lib.gather_points(fake, 10, fake, 0, fake, None) == B.SFC_OK  # nothing to do, nothing launched
    assert lib.gather_points(fake, 10, None, 5, fake, None) == B.SFC_EINVAL
    assert lib.gather_points(fake, -1, fake, 5, fake, None) == B.SFC_EINVAL


def test_flag_constants_match_header():
    text = open(HEADER).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define SFC_([A-Z_]+) (\d+)u", text)}
    assert defs["REUSE_COUNTS"] == B.REUSE_COUNTS and defs["NO_PRUNE"] == B.NO_PRUNE
    assert defs["QUERIES_ORDERED"] == B.QUERIES_ORDERED and defs["RECORD_HITS"] == B.RECORD_HITS
    assert len({B.REUSE_COUNTS, B.NO_PRUNE, B.QUERIES_ORDERED, B.RECORD_HITS}) == 4


def test_record_hits_workspace_size(lib):
    # recording adds one region per group of 64 queries (4096 records of a
    # 4-byte index and an 8-byte mask, plus the group's record count)
    view = B.SfcOctree()
    view.nodes = view.child = view.points = view.keys = view.frame = 256
    fake = ctypes.c_void_p(256)
    for n in (10, 64, 65, 100_000):
        view.n = n
        plain, rec = ctypes.c_size_t(0), ctypes.c_size_t(0)
        assert lib.radius_search(ctypes.byref(view), None, n, 0, 1.0, fake, fake, None, 0, 0, None,
                                 ctypes.byref(plain), None) == B.SFC_OK
        assert lib.radius_search(ctypes.byref(view), None, n, 0, 1.0, fake, fake, None, 0, B.RECORD_HITS, None,
                                 ctypes.byref(rec), None) == B.SFC_OK
        groups = (n + 63) // 64
        assert rec.value - plain.value >= groups * 4096 * 12 + groups * 4
        assert rec.value - plain.value <= (n // 64 + 2) * (4096 * 12 + 4) + 4 * 256


def test_workspace_alignment_and_capacity_check_validation(lib):
    view = B.SfcOctree()
    view.nodes = view.child = view.points = view.keys = view.frame = 256
    view.n = 1000
    fake = ctypes.c_void_p(256)
    need = ctypes.c_size_t(0)
    assert lib.knn_search(ctypes.byref(view), None, 1000, 8, fake, fake, None, ctypes.byref(need), None) == B.SFC_OK
    big = ctypes.c_size_t(need.value + 4096)
    # a workspace that is not 256-byte aligned is refused before anything runs
    assert lib.knn_search(ctypes.byref(view), None, 1000, 8, fake, fake, ctypes.c_void_p(256 + 64),
                          ctypes.byref(big), None) == B.SFC_EWORKSPACE
    assert b"256-aligned" in lib.sfc_last_error()
    assert lib.radius_search(ctypes.byref(view), None, 1000, 0, 1.0, fake, fake, None, 0, 0,
                             ctypes.c_void_p(256 + 8), ctypes.byref(big), None) == B.SFC_EWORKSPACE
    # the capacity check validates its arguments on the host
    total = ctypes.c_uint64(0)
    assert lib.radius_search_check(None, 10, 0, ctypes.byref(total), None) == B.SFC_EINVAL
    assert lib.radius_search_check(fake, -1, 0, ctypes.byref(total), None) == B.SFC_EINVAL
    assert lib.radius_search_check(fake, 10, 0, None, None) == B.SFC_EINVAL


def test_noalloc_host_checks(lib):
    """radius_search_noalloc validates its arguments and refuses a call whose
    workspace exceeds the fixed array before any GPU work (or HIP call)."""
    text = open(HEADER).read()
    limit = int(re.search(r"#define SFC_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text).group(1)) << 20
    view = B.SfcOctree()
    fake = ctypes.c_void_p(256)
    # an all-null tree view is rejected
    assert lib.radius_search_noalloc(ctypes.byref(view), None, 0, 0, 1.0, fake, fake, None, 0, 0, None) \
        == B.SFC_EINVAL
    view.nodes = view.child = view.points = view.keys = view.frame = 256
    view.n = 100_000
    assert lib.radius_search_noalloc(ctypes.byref(view), None, 100_000, 9, 1.0, fake, fake, None, 0, 0, None) \
        == B.SFC_EINVAL  # kernel out of range
    # recorded hits for 100k queries need more than the fixed array: refused
    need = ctypes.c_size_t(0)
    assert lib.radius_search(ctypes.byref(view), None, 100_000, 0, 1.0, fake, fake, None, 0, B.RECORD_HITS, None,
                             ctypes.byref(need), None) == B.SFC_OK
    assert need.value > limit
    assert lib.radius_search_noalloc(ctypes.byref(view), None, 100_000, 0, 1.0, fake, fake, None, 0,
                                     B.RECORD_HITS, None) == B.SFC_EWORKSPACE
    assert b"beyond the fixed" in lib.sfc_last_error()
    # external queries that the call sorts: about 24 bytes each, so 3M of them are refused
    view.n = 1000
    assert lib.radius_search_noalloc(ctypes.byref(view), fake, 3_000_000, 0, 1.0, fake, fake, None, 0, 0, None) \
        == B.SFC_EWORKSPACE
