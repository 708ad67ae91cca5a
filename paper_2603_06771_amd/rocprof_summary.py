"""Summaries of rocprofv3 CSV output (kernel statistics and HBM counters).

    python -m paper_2603_06771_amd.rocprof_summary stats <kernel_stats.csv>
    python -m paper_2603_06771_amd.rocprof_summary trace <kernel_trace.csv> <kernel-name> [min_us]
    python -m paper_2603_06771_amd.rocprof_summary sq <counter_collection.csv> <kernel-name>
    python -m paper_2603_06771_amd.rocprof_summary l2 <counter_collection.csv> <kernel-name>
    python -m paper_2603_06771_amd.rocprof_summary lds <counter_collection.csv> <kernel-name>
    python -m paper_2603_06771_amd.rocprof_summary traffic <fetch_counter_collection.csv>
        <write_counter_collection.csv> [kernel-substring]
    python -m paper_2603_06771_amd.rocprof_summary record <fetch.csv> <write.csv> <kernel> <source>
    python -m paper_2603_06771_amd.rocprof_summary stage <fetch.csv> <write.csv> <k1,k2,...> <stages> <source>
    python -m paper_2603_06771_amd.rocprof_summary call <fetch.csv> <write.csv> <k1[@grid],k2,...> <source>

`traffic` reports FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the matching
kernel, scaled by what the same counters read for a reference dispatch of
known size in the same run (256 MiB read, 256 MiB written): by default the
runtime's device copy (`copyBuffer`); a trailing argument `calib=<name>`
picks another reference, e.g. `calib=elementwise` for the elementwise kernel
that bench.py --copy-calib also runs.
"""
from __future__ import annotations

import csv
import statistics
import sys

COPY_BYTES = 2 * (64 << 20) * 4  # 256 MiB read + 256 MiB written by the calibration copy
CALIB = "copyBuffer"  # name (substring) of the reference dispatch


def _ref(rows, calib):
    """Counter value of the reference dispatch: the largest one whose kernel
    name contains `calib`."""
    vals = [v for _, k, v in rows if calib in k]
    return max(vals) if vals else None


def stats(path: str, top: int = 25) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows[:top]:
        out.append(f"{r['Name'][:70]:70s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")
    return "\n".join(out)


def trace(path: str, kernel: str, min_us: float = 100.0) -> str:
    """Per-dispatch durations of the kernels whose name starts with `kernel`
    (after any namespace), dispatches shorter than min_us left out (e.g.
    fills launched with a zero capacity, which return at once)."""
    durs, short = [], 0
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"].split("(")[0].split("::")[-1]
        if name != kernel:
            continue
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        if us < min_us:
            short += 1
        else:
            durs.append(us)
    if not durs:
        return f"{kernel}: no dispatch of at least {min_us} us ({short} shorter)"
    return (f"{kernel}: {len(durs)} dispatches >= {min_us:g} us (+{short} shorter, left out): "
            f"avg {statistics.mean(durs):.1f} us, median {statistics.median(durs):.1f} us, "
            f"min {min(durs):.1f} us, max {max(durs):.1f} us")


def sq(path: str, kernel: str) -> str:
    """Per-dispatch instruction mix of `kernel` from SQ counters: instructions,
    wait and wave cycles per wave."""
    per = {}
    for r in csv.DictReader(open(path)):
        if r["Kernel_Name"].split("(")[0].split("::")[-1] != kernel:
            continue
        d = per.setdefault(int(r["Dispatch_Id"]), {})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
        d["dur_us"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    out = [f"{'dispatch':>8s} {'dur_us':>9s} {'waves':>8s} {'VALU/w':>8s} {'SALU/w':>8s} {'LDS/w':>7s} "
           f"{'VMEM/w':>7s} {'wait/w':>8s} {'cycles/w':>9s}"]
    for dsp in sorted(per):
        d = per[dsp]
        w = max(d.get("SQ_WAVES_sum", d.get("SQ_WAVES", 1.0)), 1.0)

        def g(name):
            return d.get(name + "_sum", d.get(name, float("nan")))
        out.append(f"{dsp:8d} {d['dur_us']:9.0f} {w:8.0f} {g('SQ_INSTS_VALU') / w:8.0f} {g('SQ_INSTS_SALU') / w:8.0f} "
                   f"{g('SQ_INSTS_LDS') / w:7.0f} {g('SQ_INSTS_VMEM_RD') / w:7.0f} {g('SQ_WAIT_INST_ANY') / w:8.0f} "
                   f"{g('SQ_WAVE_CYCLES') / w:9.0f}")
    return "\n".join(out)


def l2(path: str, kernel: str) -> str:
    """Per-dispatch L2 hit rate of `kernel` from TCC_HIT / TCC_MISS."""
    per = {}
    for r in csv.DictReader(open(path)):
        if r["Kernel_Name"].split("(")[0].split("::")[-1] != kernel:
            continue
        d = per.setdefault(int(r["Dispatch_Id"]), {})
        d[r["Counter_Name"].replace("_sum", "")] = float(r["Counter_Value"])
        d["dur_us"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    out = [f"{'dispatch':>8s} {'dur_us':>9s} {'hits':>12s} {'misses':>12s} {'hit_rate':>9s}"]
    for dsp in sorted(per):
        d = per[dsp]
        h, m = d.get("TCC_HIT", 0.0), d.get("TCC_MISS", 0.0)
        out.append(f"{dsp:8d} {d['dur_us']:9.0f} {h:12.0f} {m:12.0f} {h / max(h + m, 1.0):9.3f}")
    return "\n".join(out)


def lds(path: str, kernel: str) -> str:
    """Per-dispatch LDS behaviour and occupancy of `kernel`: LDS instructions
    and address-conflict cycles per wave, bank conflicts per LDS access
    (derived counter LdsBankConflict) and the mean resident waves per CU
    (MeanOccupancyPerCU)."""
    per = {}
    for r in csv.DictReader(open(path)):
        if r["Kernel_Name"].split("(")[0].split("::")[-1] != kernel:
            continue
        d = per.setdefault(int(r["Dispatch_Id"]), {})
        d[r["Counter_Name"].replace("_sum", "")] = float(r["Counter_Value"])
        d["dur_us"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    out = [f"{'dispatch':>8s} {'dur_us':>9s} {'waves':>8s} {'LDS/w':>7s} {'addr/w':>8s} {'bank/access':>12s} "
           f"{'waves/CU':>9s}"]
    for dsp in sorted(per):
        d = per[dsp]
        w = max(d.get("SQ_WAVES", 1.0), 1.0)
        out.append(f"{dsp:8d} {d['dur_us']:9.0f} {w:8.0f} {d.get('SQ_INSTS_LDS', float('nan')) / w:7.0f} "
                   f"{d.get('SQ_LDS_ADDR_CONFLICT', float('nan')) / w:8.1f} {d.get('LdsBankConflict', float('nan')):12.4f} "
                   f"{d.get('MeanOccupancyPerCU', float('nan')):9.1f}")
    return "\n".join(out)


def _per_dispatch(path: str, counter: str):
    rows = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def traffic(fetch_path: str, write_path: str, kernel: str = "k_radius_fill", min_kib: float = 1024.0,
            calib: str = CALIB) -> str:
    """Per-dispatch FETCH_SIZE / WRITE_SIZE of `kernel` (dispatches reading or
    writing at least min_kib), scaled by the calibration copy's readings."""
    fetch = _per_dispatch(fetch_path, "FETCH_SIZE")
    write = _per_dispatch(write_path, "WRITE_SIZE")

    fc, wc = _ref(fetch, calib), _ref(write, calib)
    half = COPY_BYTES // 2
    ffac = half / (fc * 1024) if fc else 1.0
    wfac = half / (wc * 1024) if wc else 1.0
    lines = [f"calibration: reference dispatch '{calib}' reading and writing {half} B each",
             f"  FETCH_SIZE {fc} KiB -> scale {ffac:.4f};  WRITE_SIZE {wc} KiB -> scale {wfac:.4f}",
             f"{'dispatch':>8s} {'fetch_KiB':>12s} {'write_KiB':>12s} {'fetch_B_scaled':>15s} {'write_B_scaled':>15s}  kernel"]
    wmap = {d: v for d, k, v in write if kernel in k}
    for d, k, v in fetch:
        if kernel not in k:
            continue
        w = wmap.get(d, float("nan"))
        if max(v, w if w == w else 0.0) < min_kib:
            continue
        lines.append(f"{d:8d} {v:12.0f} {w:12.0f} {v * 1024 * ffac:15.4g} {w * 1024 * wfac:15.4g}  {k[:60]}")
    return "\n".join(lines)


def source_sha(path: str) -> str:
    """Hash of a source file's code: comments and whitespace left out, so a
    record stays valid across comment edits and is void once the code
    changes."""
    import hashlib
    import re
    text = open(path, encoding="utf-8").read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()[:16]


def traffic_record(fetch_path: str, write_path: str, kernel: str, source: str, min_kib: float = 1024.0,
                   calib: str = CALIB) -> dict:
    """Mean scaled HBM bytes per launch of `kernel`, tagged with the hash of
    the kernel's source file (a reader uses it only while the hash matches)."""
    fetch = _per_dispatch(fetch_path, "FETCH_SIZE")
    write = {d: v for d, k, v in _per_dispatch(write_path, "WRITE_SIZE") if kernel in k}
    fc = _ref(fetch, calib)
    wc = _ref(_per_dispatch(write_path, "WRITE_SIZE"), calib)
    half = COPY_BYTES // 2
    ffac, wfac = half / (fc * 1024), half / (wc * 1024)
    f_b, w_b = [], []
    for d, k, v in fetch:
        if kernel in k and d in write and max(v, write[d]) >= min_kib:
            f_b.append(v * 1024 * ffac)
            w_b.append(write[d] * 1024 * wfac)
    return {"kernel": kernel, "source_sha": source_sha(source), "launches": len(f_b),
            "fetch_bytes_per_launch": statistics.mean(f_b), "write_bytes_per_launch": statistics.mean(w_b),
            "bytes_per_launch": statistics.mean(f_b) + statistics.mean(w_b),
            "fetch_scale": ffac, "write_scale": wfac}


def _base(kernel_name: str) -> str:
    return kernel_name.split("(")[0].split("::")[-1]


def stage_record(fetch_path: str, write_path: str, kernels: list, stages: int, source: str,
                 calib: str = CALIB) -> dict:
    """Scaled HBM bytes of a stage made of several kernels (exact base names):
    the sum over every dispatch of those kernels in the run, divided by the
    number of stages the run executed; tagged like traffic_record."""
    fetch = _per_dispatch(fetch_path, "FETCH_SIZE")
    write = _per_dispatch(write_path, "WRITE_SIZE")
    fc, wc = _ref(fetch, calib), _ref(write, calib)
    half = COPY_BYTES // 2
    ffac, wfac = half / (fc * 1024), half / (wc * 1024)
    names = set(kernels)
    f_sum = sum(v for _, k, v in fetch if _base(k) in names) * 1024 * ffac
    w_sum = sum(v for _, k, v in write if _base(k) in names) * 1024 * wfac
    per = {}
    for _, k, v in fetch:
        if _base(k) in names:
            per.setdefault(_base(k), [0, 0.0])
            per[_base(k)][0] += 1
            per[_base(k)][1] += v * 1024 * ffac
    return {"kernels": sorted(names), "source_sha": source_sha(source), "stages": stages,
            "fetch_bytes_per_launch": f_sum / stages, "write_bytes_per_launch": w_sum / stages,
            "bytes_per_launch": (f_sum + w_sum) / stages, "fetch_scale": ffac, "write_scale": wfac, "calib": calib,
            "fetch_bytes_by_kernel": {k: {"dispatches": c, "bytes_per_stage": b / stages} for k, (c, b) in per.items()}}


def _rows_grid(path: str, counter: str):
    rows = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return rows


def call_record(fetch_path: str, write_path: str, kernels: list, source: str, calib: str = CALIB,
                wcalib: str | None = None) -> dict:
    """Scaled HBM bytes of one call made of several kernels, each launched
    once per call: the sum over `kernels` of the mean scaled bytes per
    dispatch of that kernel.  An entry is a base kernel name, optionally
    with `@<grid size>` to keep only the dispatches of that grid (kernels
    that other steps of the run also launch, at other sizes).  Tagged like
    traffic_record.  wcalib: the reference for WRITE_SIZE when it differs
    from the one for FETCH_SIZE ("raw": no scaling)."""
    fetch = _rows_grid(fetch_path, "FETCH_SIZE")
    write = _rows_grid(write_path, "WRITE_SIZE")
    wcalib = wcalib or calib
    fc = _ref([(d, k, v) for d, k, _, v in fetch], calib)
    half = COPY_BYTES // 2
    ffac = half / (fc * 1024)
    if wcalib == "raw":
        wfac = 1.0
    else:
        wfac = half / (_ref([(d, k, v) for d, k, _, v in write], wcalib) * 1024)
    per = {}
    f_sum = w_sum = 0.0
    for spec in kernels:
        name, _, grid = spec.partition("@")

        def sel(rows):
            return [v for _, k, g, v in rows if _base(k) == name and (not grid or g == int(grid))]
        fv, wv = sel(fetch), sel(write)
        if not fv or not wv:
            raise ValueError(f"no dispatch of {spec}")
        fb, wb = statistics.mean(fv) * 1024 * ffac, statistics.mean(wv) * 1024 * wfac
        per[spec] = {"dispatches": len(fv), "fetch_bytes": fb, "write_bytes": wb}
        f_sum += fb
        w_sum += wb
    return {"kernels": list(kernels), "source_sha": source_sha(source), "fetch_bytes_per_launch": f_sum,
            "write_bytes_per_launch": w_sum, "bytes_per_launch": f_sum + w_sum, "fetch_scale": ffac,
            "write_scale": wfac, "calib": calib, "wcalib": wcalib, "by_kernel": per}


if __name__ == "__main__":
    WCALIB = None
    while sys.argv[-1].startswith(("calib=", "wcalib=")):
        opt = sys.argv.pop()
        if opt.startswith("wcalib="):
            WCALIB = opt[len("wcalib="):]
        else:
            CALIB = opt[len("calib="):]
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    elif sys.argv[1] == "l2":
        print(l2(sys.argv[2], sys.argv[3]))
    elif sys.argv[1] == "lds":
        print(lds(sys.argv[2], sys.argv[3]))
    elif sys.argv[1] == "sq":
        print(sq(sys.argv[2], sys.argv[3]))
    elif sys.argv[1] == "trace":
        print(trace(sys.argv[2], sys.argv[3], float(sys.argv[4]) if len(sys.argv) > 4 else 100.0))
    elif sys.argv[1] == "stage":
        import json
        print(json.dumps(stage_record(sys.argv[2], sys.argv[3], sys.argv[4].split(","), int(sys.argv[5]),
                                      sys.argv[6], calib=CALIB), indent=1))
    elif sys.argv[1] == "call":
        import json
        print(json.dumps(call_record(sys.argv[2], sys.argv[3], sys.argv[4].split(","), sys.argv[5], calib=CALIB,
                                     wcalib=WCALIB), indent=1))
    elif sys.argv[1] == "record":
        import json
        print(json.dumps(traffic_record(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], calib=CALIB), indent=1))
    else:
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else "k_radius_fill", calib=CALIB))
