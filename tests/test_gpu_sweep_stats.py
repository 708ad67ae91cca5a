"""The statistics build (libsfcoct_stats.so, SFC_SWEEP_STATS) counts the
same neighbours as the search and at least one test per neighbour found."""
import ctypes

import numpy as np
import pytest

from paper_2603_06771_amd import datagen
from tests._parity import announce

pytestmark = pytest.mark.gpu


def test_sweep_stats_consistent():
    import torch

    import paper_2603_06771_amd as sfc
    from paper_2603_06771_amd import _binding as B
    from paper_2603_06771_amd.build import STATS_LIB
    S = ctypes.CDLL(STATS_LIB)
    S.radius_search.argtypes = B.load().radius_search.argtypes
    S.sfc_sweep_stats.argtypes = [ctypes.POINTER(ctypes.c_ulonglong), ctypes.c_int]
    pts = datagen.lidar_tile(50000, seed=41)
    t = sfc.build_linear_octree(torch.from_numpy(pts).cuda(), "hilbert", 21, 64)
    n = pts.shape[0]
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    out = (ctypes.c_ulonglong * 16)()
    assert S.sfc_sweep_stats(out, 1) == 0
    for kernel, r in (("sphere", 0.5), ("cube", 3.0)):
        for flags in (B.RECORD_HITS, 0):
            announce(f"sweep stats {kernel} r={r} flags={flags}")
            call = (ctypes.byref(t.view), None, n, sfc.KERNELS[kernel], r, ctypes.c_void_p(counts.data_ptr()),
                    ctypes.c_void_p(offsets.data_ptr()), None, 0, flags)
            need = ctypes.c_size_t(0)
            assert S.radius_search(*call, None, ctypes.byref(need), None) == 0
            ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
            assert S.radius_search(*call, ctypes.c_void_p(ws.data_ptr()), ctypes.byref(need),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
            assert S.sfc_sweep_stats(out, 1) == 0
            s = np.array(list(out), dtype=np.int64)
            tests, hits, groups, swept = s[4:8] if flags else s[:4]
            ref = sfc.radius_count(t, None, kernel, r)[1][-1].item()
            assert hits == ref and groups == (n + 63) // 64 and tests >= hits and swept > 0
            assert not (s[:4] if flags else s[4:8]).any()  # only one kind of count ran
            assert s[15] > 0 and s[8:15].sum() <= s[15]  # phase clocks within the whole
