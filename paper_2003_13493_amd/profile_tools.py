"""Summaries of rocprofv3 CSV output for the committed profile records.

    python -m paper_2003_13493_amd.profile_tools trace    <kernel_stats.csv> [out.md "command"]
    python -m paper_2003_13493_amd.profile_tools traffic  <fetch_dir> <write_dir> <copy_bytes> [out.json "cmd" ...]
    python -m paper_2003_13493_amd.profile_tools counters <pmc_dir> [out.md "command" ...]

`traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch, two separate
--pmc runs) of the batched detect kernel into HBM bytes per launch.  Each
counter is scaled by the ratio between the bytes a plain device-to-device copy
of known size must move and what the same counter reads for that copy (the
largest copy dispatch of the run, which must be the copy of copy_bytes).
`counters` averages SQ_* counters per dispatch of the batched kernel.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import statistics
import sys


def _rows(path_or_dir: str):
    paths = [path_or_dir] if path_or_dir.endswith(".csv") else \
        glob.glob(os.path.join(path_or_dir, "**", "*counter_collection.csv"), recursive=True)
    rows = []
    for p in paths:
        with open(p) as f:
            rows += list(csv.DictReader(f))
    return rows


def per_dispatch(rows, counter: str, name_part: str) -> list[float]:
    acc: dict[str, float] = {}
    for r in rows:
        if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]:
            acc[r["Dispatch_Id"]] = acc.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return list(acc.values())


def traffic(fetch_dir: str, write_dir: str, copy_bytes: int) -> dict:
    fr, wr = _rows(fetch_dir), _rows(write_dir)
    det_f = per_dispatch(fr, "FETCH_SIZE", "detect_batch_kernel")
    det_w = per_dispatch(wr, "WRITE_SIZE", "detect_batch_kernel")
    # the calibration copy is the largest copy dispatch
    cp_f = max(per_dispatch(fr, "FETCH_SIZE", "copyBuffer") or [0.0])
    cp_w = max(per_dispatch(wr, "WRITE_SIZE", "copyBuffer") or [0.0])
    kf = copy_bytes / (cp_f * 1024.0) if cp_f else None
    kw = copy_bytes / (cp_w * 1024.0) if cp_w else None
    fetch = statistics.median(det_f) * 1024.0 * kf if det_f and kf else None
    write = statistics.median(det_w) * 1024.0 * kw if det_w and kw else None
    return {"fetch_kib_per_dispatch": statistics.median(det_f) if det_f else None,
            "write_kib_per_dispatch": statistics.median(det_w) if det_w else None,
            "copy_fetch_kib": cp_f, "copy_write_kib": cp_w, "copy_bytes": copy_bytes,
            "fetch_scale": kf, "write_scale": kw,
            "hbm_fetch_bytes": fetch, "hbm_write_bytes": write,
            "hbm_bytes_per_launch": (fetch + write) if fetch and write else None}


def trace(stats_csv: str) -> list[dict]:
    with open(stats_csv) as f:
        return [{"name": r["Name"], "calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                 "total_ns": int(float(r["TotalDurationNs"]))} for r in csv.DictReader(f)]


# What decides the detector's kernels and their launch: the kernels, the
# shared declarations (sub-tile and fused-level constants) and the runtime
# (launch defaults, region layout, work-item order).
DETECT_SOURCES = ("fastgrid_kernels.hip", "fg_internal.h", "fastgrid_runtime.hip")


def kernel_source_hash(names=DETECT_SOURCES) -> str:
    """sha256[:16] of kernel and runtime sources with comments and blank space
    removed, so that a record stays valid across comment-only edits, and of
    the hipcc flags the library is built with."""
    import hashlib
    import re
    if isinstance(names, str):
        names = (names,)
    parts = []
    for name in names:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", name)
        with open(path) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        parts.append("\n".join(line.strip() for line in text.splitlines() if line.strip()))
    from .build import HIPCC_FLAGS
    parts.append(" ".join(HIPCC_FLAGS))
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()[:16]


def short_name(name: str) -> str:
    for key in ("detect_batch_kernel", "detect_plain_kernel", "pyr_batch_kernel", "pyr_kernel"):
        if key + "(" in name:
            return key
    if "FillFunctor" in name:
        return "torch fill (harness)"
    return name[:60]


def trace_md(stats_csv: str, command: str) -> str:
    rows = trace(stats_csv)
    lines = ["| kernel | calls | average ns | total ns |", "|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {short_name(r['name'])} | {r['calls']} | {r['avg_ns']:.0f} | {r['total_ns']} |")
    return "\n".join([
        "# Kernel trace: batched detect kernel on the 64-frame batch (one MI355X)", "",
        "Command (repo root):", "", "    " + command, "",
        f"Summary: `python -m paper_2003_13493_amd.profile_tools trace {stats_csv}`.",
        "detect_batch_kernel is one persistent launch over the whole 64-frame batch (pyramid levels 1-2",
        "are built inside it); detect_plain_kernel is the plain path, one launch per frame.",
        f"Kernel source hash (sha256[:16] of the kernel and runtime sources without comments, and the hipcc flags) = {kernel_source_hash()}.", "", *lines, ""])


def counters(pmc_dir: str, name_part: str = "detect_batch_kernel") -> dict:
    rows = _rows(pmc_dir)
    names = sorted({r["Counter_Name"] for r in rows})
    return {n: statistics.median(per_dispatch(rows, n, name_part)) for n in names
            if per_dispatch(rows, n, name_part)}


TRACK_MODES = ("t", "t+offset", "t+gain", "t+gain+offset")
TRACK_SIZES = ((100, 200), (1000, 200), (10000, 40))   # (features, timed calls) as bench.py runs them
TRACK_WARMUP = 5


def track_md(trace_csv: str, command: str) -> str:
    """Per-(mode, feature count) averages of the tracking kernel from a kernel
    trace of ``bench.py --tracking-only``: its dispatches come in the bench's
    order (for each mode, for each count: warm-up calls, then timed calls)."""
    durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in _rows(trace_csv)
            if "track_kernel" in r["Kernel_Name"]]
    lines = ["# Kernel trace: Lucas-Kanade tracking kernel (one MI355X)", "", "Command (repo root):", "",
             "    " + command, "",
             f"Summary: `python -m paper_2003_13493_amd.profile_tools track {trace_csv}`.",
             "track_kernel is one launch per call, one wave64 per feature; the frames are two 752x480 crops of one",
             "synthetic scene moved by (3, -2), 3 levels, max 30 iterations per level, eps 0.01.",
             f"Kernel source hash (sha256[:16] of the kernel and runtime sources without comments, and the hipcc flags) = {track_source_hash()}.", "",
             "| parameters | features | calls | average ns | min ns | max ns |", "|---|---|---|---|---|---|"]
    i = 0
    for mode in TRACK_MODES:
        for n, reps in TRACK_SIZES:
            block = durs[i + TRACK_WARMUP:i + TRACK_WARMUP + reps]
            i += TRACK_WARMUP + reps
            if not block:
                continue
            lines.append(f"| {mode} | {n} | {len(block)} | {sum(block) // len(block)} | {min(block)} | "
                         f"{max(block)} |")
    lines.append("")
    return "\n".join(lines)


def track_counters_md(pmc_dir: str, command: str) -> str:
    """Per-(mode, feature count) medians of SQ counters of the tracking kernel,
    per wave, from a ``--pmc`` run of ``bench.py --tracking-only`` (dispatches
    in the bench's order, as for track_md)."""
    rows = [r for r in _rows(pmc_dir) if "track_kernel" in r["Kernel_Name"]]
    order, per = [], {}
    for r in rows:
        d = int(r["Dispatch_Id"])
        if d not in per:
            per[d] = {}
            order.append(d)
        per[d][r["Counter_Name"]] = per[d].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    order.sort()
    lines = ["# SQ counters: Lucas-Kanade tracking kernel (one MI355X)", "", "Command (repo root):", "",
             "    " + command, "",
             f"Summary: `python -m paper_2003_13493_amd.profile_tools track-counters {pmc_dir}`.",
             "Medians over each configuration's timed dispatches, per wave (one wave is one feature).",
             "wait = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES; VALU active = SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES.",
             f"Kernel source hash (sha256[:16] of the kernel and runtime sources without comments, and the hipcc flags) = {track_source_hash()}.", "",
             "| parameters | features | VALU instr / wave | SALU instr / wave | VMEM instr / wave | "
             "wave cycles / wave | wait | VALU active |", "|---|---|---|---|---|---|---|---|"]
    i = 0
    for mode in TRACK_MODES:
        for n, reps in TRACK_SIZES:
            block = [per[d] for d in order[i + TRACK_WARMUP:i + TRACK_WARMUP + reps]]
            i += TRACK_WARMUP + reps
            if not block:
                continue

            def med(key):
                vals = [b.get(key, 0.0) / max(b.get("SQ_WAVES", 1.0), 1.0) for b in block]
                return statistics.median(vals)

            cyc = med("SQ_WAVE_CYCLES")
            lines.append(f"| {mode} | {n} | {med('SQ_INSTS_VALU'):.0f} | {med('SQ_INSTS_SALU'):.0f} | "
                         f"{med('SQ_INSTS_VMEM'):.0f} | {cyc:.0f} | "
                         f"{med('SQ_WAIT_INST_ANY') / cyc if cyc else 0:.2f} | "
                         f"{med('SQ_ACTIVE_INST_VALU') / cyc if cyc else 0:.2f} |")
    lines.append("")
    return "\n".join(lines)


def track_source_hash() -> str:
    return kernel_source_hash("fasttrack_kernels.hip")


if __name__ == "__main__":
    if sys.argv[1] == "track-counters":
        md = track_counters_md(sys.argv[2], sys.argv[4] if len(sys.argv) > 4 else "")
        if len(sys.argv) > 3:
            with open(sys.argv[3], "w") as f:
                f.write(md)
        print(md)
    elif sys.argv[1] == "track":
        md = track_md(sys.argv[2], sys.argv[4] if len(sys.argv) > 4 else "")
        if len(sys.argv) > 3:
            with open(sys.argv[3], "w") as f:
                f.write(md)
        print(md)
    elif sys.argv[1] == "trace":
        if len(sys.argv) > 3:
            with open(sys.argv[3], "w") as f:
                f.write(trace_md(sys.argv[2], sys.argv[4]))
        for r in trace(sys.argv[2]):
            print(f"{r['calls']:6d} {r['avg_ns']:12.0f} ns  {r['name'][:110]}")
    elif sys.argv[1] == "traffic":
        rec = traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]))
        if len(sys.argv) > 5:
            rec["kernel_source_sha256_16"] = kernel_source_hash()
            rec["commands"] = sys.argv[6:]
            with open(sys.argv[5], "w") as f:
                json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))
    elif sys.argv[1] == "counters":
        rec = counters(sys.argv[2])
        if len(sys.argv) > 3:
            lines = ["| counter | per dispatch (median) |", "|---|---|"]
            lines += [f"| {k} | {v:.0f} |" for k, v in rec.items()]
            with open(sys.argv[3], "w") as f:
                f.write("\n".join(["# SQ counters: batched detect kernel on the 64-frame batch", "",
                                    "Commands (repo root), one run per counter set:", "",
                                    *["    " + c for c in sys.argv[4:]], "",
                                    f"Summary: `python -m paper_2003_13493_amd.profile_tools counters {sys.argv[2]}` "
                                    "(median over the runs' dispatches of the batched kernel; whole-device totals "
                                    "per dispatch).", "",
                                    f"Kernel source hash (sha256[:16] of the kernel and runtime sources without comments, and the hipcc flags) = {kernel_source_hash()}.", "",
                                    *lines, ""]))
        print(json.dumps(rec, indent=1))
