"""Host logic of the profile summaries: the traffic figure the bench line
reports comes from FETCH_SIZE / WRITE_SIZE rows scaled by what the same
counter reads for a device copy of known size."""
import csv
import os

import pytest

from paper_2003_13493_amd import profile_tools

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_rows(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_traffic_sums_per_dispatch_and_scales_by_the_copy(tmp_path):
    det = "(anonymous namespace)::detect_batch_kernel(fg_job const*, fg_item const*, int, unsigned int*)"
    cp = "__amd_rocclr_copyBuffer"
    copy_bytes = 1 << 20
    # FETCH_SIZE arrives as several rows per dispatch (one per counter
    # instance); the copy's fetch reads half of what it moves
    fetch = [(1, det, "FETCH_SIZE", 100.0), (1, det, "FETCH_SIZE", 20.0),
             (2, det, "FETCH_SIZE", 150.0), (2, det, "FETCH_SIZE", 10.0),
             (3, det, "FETCH_SIZE", 90.0),
             (4, cp, "FETCH_SIZE", 256.0), (4, cp, "FETCH_SIZE", 256.0),
             (5, cp, "FETCH_SIZE", 8.0)]
    write = [(1, det, "WRITE_SIZE", 30.0), (2, det, "WRITE_SIZE", 40.0), (3, det, "WRITE_SIZE", 50.0),
             (4, cp, "WRITE_SIZE", 1024.0)]
    write_rows(str(tmp_path / "f"), fetch)
    write_rows(str(tmp_path / "w"), write)
    rec = profile_tools.traffic(str(tmp_path / "f"), str(tmp_path / "w"), copy_bytes)
    # per dispatch: 120, 160, 90 KiB -> median 120; copy: 512 KiB for 1 MiB
    assert rec["fetch_kib_per_dispatch"] == 120.0
    assert rec["copy_fetch_kib"] == 512.0
    assert rec["fetch_scale"] == pytest.approx(2.0)
    assert rec["hbm_fetch_bytes"] == pytest.approx(120 * 1024 * 2.0)
    assert rec["write_kib_per_dispatch"] == 40.0
    assert rec["write_scale"] == pytest.approx(1.0)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(120 * 1024 * 2.0 + 40 * 1024)


def test_counters_take_the_median_per_dispatch(tmp_path):
    det = "detect_batch_kernel(x)"
    rows = [(1, det, "SQ_WAVES", 3072), (2, det, "SQ_WAVES", 3072), (3, det, "SQ_WAVES", 3072),
            (1, det, "SQ_INSTS_VALU", 10), (1, det, "SQ_INSTS_VALU", 5), (2, det, "SQ_INSTS_VALU", 30),
            (3, det, "SQ_INSTS_VALU", 20), (4, "other_kernel", "SQ_INSTS_VALU", 1e9)]
    write_rows(str(tmp_path / "s"), rows)
    rec = profile_tools.counters(str(tmp_path / "s"))
    assert rec == {"SQ_INSTS_VALU": 20.0, "SQ_WAVES": 3072.0}


def test_source_hash_covers_the_build_flags(monkeypatch):
    from paper_2003_13493_amd import build
    h = profile_tools.kernel_source_hash()
    monkeypatch.setattr(build, "HIPCC_FLAGS", build.HIPCC_FLAGS + ["-DX"])
    assert profile_tools.kernel_source_hash() != h
