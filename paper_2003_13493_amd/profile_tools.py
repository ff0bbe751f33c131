"""Summaries of rocprofv3 CSV output for the committed profile records.

    python -m paper_2003_13493_amd.profile_tools trace  <kernel_stats.csv>
    python -m paper_2003_13493_amd.profile_tools traffic <fetch_dir> <write_dir> <copy_bytes>

`traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch, two separate
--pmc runs) of the batched detect kernel into HBM bytes per launch.  Each
counter is scaled by the ratio between the bytes a plain device-to-device copy
of known size must move and what the same counter reads for that copy.
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


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        for r in trace(sys.argv[2]):
            print(f"{r['calls']:6d} {r['avg_ns']:12.0f} ns  {r['name'][:110]}")
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], int(sys.argv[4])), indent=1))
