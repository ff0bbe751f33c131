"""Host-side logic of the serving loop (no GPU): admission by HBM budget,
Poisson arrival schedules, latency percentiles, resident-byte accounting."""
import numpy as np

from paper_2003_13493_amd import serve, synth


def test_admission_respects_budget_in_order():
    admitted, rejected = serve.plan_admission([100, 200, 50, 400], budget=300)
    assert admitted == [0, 1] and rejected == [2, 3]
    admitted, rejected = serve.plan_admission([100, 200, 50], budget=10 ** 9)
    assert admitted == [0, 1, 2] and rejected == []
    admitted, rejected = serve.plan_admission([100], budget=99)
    assert admitted == [] and rejected == [0]


def test_waiting_streams_admitted_in_queue_order_as_they_fit():
    need = [100, 300, 50, 200]
    # room 260: 100 fits, 300 does not (keeps its place), 50 fits; 200 no longer fits
    assert serve.admit_waiting([0, 1, 2, 3], need, 260) == ([0, 2], [1, 3])
    assert serve.admit_waiting([1, 3], need, 500) == ([1, 3], [])
    assert serve.admit_waiting([1, 3], need, 199) == ([], [1, 3])
    assert serve.admit_waiting([], need, 10) == ([], [])


def test_poisson_schedule_rates_and_order():
    sched = serve.poisson_arrivals([100.0, 1000.0], duration_s=20.0, seed=1)
    times = [t for t, _, _ in sched]
    assert times == sorted(times) and all(0 <= t < 20.0 for t in times)
    n0 = sum(1 for _, s, _ in sched if s == 0)
    n1 = sum(1 for _, s, _ in sched if s == 1)
    assert abs(n0 - 2000) < 4 * np.sqrt(2000) and abs(n1 - 20000) < 4 * np.sqrt(20000)
    ks = [k for _, s, k in sched if s == 1]
    assert ks == list(range(len(ks)))          # frame indices count up per stream
    assert sched == serve.poisson_arrivals([100.0, 1000.0], 20.0, seed=1)


def test_percentiles():
    p = serve.percentiles(list(range(1, 101)))
    assert abs(p["p50"] - 50.5) < 1e-9 and abs(p["p99"] - 99.01) < 1e-9
    assert serve.percentiles([]) == {"p50": None, "p99": None}


def test_resident_bytes_counts_pool_slots_and_grid():
    s = synth.StreamSpec(0, 640, 480, 3, 10, 9, 32, 100.0, seed=1)
    b = serve.resident_bytes(s, pool_frames=2, slots=3)
    lvl0 = 480 * 640
    upper = 240 * 320 + 120 * 192
    cells = 20 * 15
    assert b == 2 * lvl0 + 3 * (upper + 8 * cells)
    # frames uploaded per request: a level-0 plane per slot instead of the pool
    assert serve.resident_bytes(s, 2, 3, upload=True) == 3 * (lvl0 + upper + 8 * cells)


def test_stream_workload_recipe():
    streams = synth.streams32()
    need = [serve.resident_bytes(s, 4, 4) for s in streams]
    assert sum(need) < 2 << 30                  # fits easily in 288 GB
    assert {(s.width, s.height) for s in streams} == set(synth.STREAM_SIZES)
