"""Builds the gfx950 shared library libsfcoct.so from csrc/*.hip with hipcc.

Device flags: no fp contraction (every fp32 expression evaluated as written),
denormals kept, correctly rounded fp32 division, packed-fp32 instructions
disabled.  The library is built in-tree, next to this file.  Beside it,
libsfcoct_stats.so is the same library with the count kernels' sweep
statistics compiled in (SFC_SWEEP_STATS: tests and hits per search, read by
sweep_stats.py); the search results are the same.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsfcoct.so")
STATS_LIB = os.path.join(HERE, "libsfcoct_stats.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every .hip source and link libsfcoct.so and libsfcoct_stats.so
    (always rebuilds); returns the path of libsfcoct.so."""
    objdir = tempfile.mkdtemp(prefix="sfcoct_build_")
    # (source, extra flags, object); search.hip a second time for the statistics build
    jobs_list = [(src, [], os.path.join(objdir, os.path.basename(src) + ".o")) for src in sources()]
    search = [src for src in sources() if os.path.basename(src) == "search.hip"]
    stats_obj = os.path.join(objdir, "search_stats.hip.o")
    jobs_list += [(src, ["-DSFC_SWEEP_STATS"], stats_obj) for src in search]
    procs = []
    for src, extra, obj in jobs_list:
        cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if out and (verbose or p.returncode):
            sys.stdout.write(out.decode(errors="replace"))
        if p.returncode:
            failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    plain = [obj for _, extra, obj in jobs_list if not extra]
    stats = [obj for obj in plain if os.path.basename(obj) != "search.hip.o"] + [stats_obj]
    for lib, objs in ((LIB, plain), (STATS_LIB, stats)):
        tmp = lib + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, lib)
    for _, _, obj in jobs_list:
        os.remove(obj)
    os.rmdir(objdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
