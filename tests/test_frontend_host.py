"""Host logic of the detect-and-track loop (CPU): which cell winners a
re-detection adds, and the cell of a level-0 position."""
import numpy as np

from paper_2003_13493_amd import fastgrid, frontend


def slots_of(entries, gw, gh):
    s = np.zeros(gw * gh, dtype=fastgrid.FEATURE_DTYPE)
    s["x"], s["y"], s["level"] = 0xFFFF, 0xFFFF, 0xFF
    for cell, (x, y, score, level) in entries.items():
        s[cell] = (x, y, score, level, 0)
    return s.reshape(gh, gw)


def test_pick_new_strongest_free_cells_first():
    gw, gh = 4, 3
    slots = slots_of({0: (5, 6, 40, 0), 1: (20, 3, 90, 1), 5: (9, 9, 90, 0), 7: (31, 2, 10, 2),
                      11: (3, 4, 70, 0)}, gw, gh)
    taken = np.zeros(gw * gh, dtype=bool)
    taken[11] = True
    got = frontend.pick_new(slots, taken, 3)
    # scores 90 (cells 1 and 5: the lower cell first), then 40; cell 11 is taken
    assert got.tolist() == [[40.0, 6.0], [9.0, 9.0], [5.0, 6.0]]
    assert len(frontend.pick_new(slots, taken, 10)) == 4          # only four free winners
    assert frontend.pick_new(slots, taken, 0).shape == (0, 2)
    got = frontend.pick_new(slots, np.zeros(gw * gh, dtype=bool), 10)
    assert [31.0 * 4, 2.0 * 4] in got.tolist()                   # level 2 scaled to level 0


def test_cell_of():
    xy = np.array([[0.0, 0.0], [31.9, 0.0], [32.0, 0.0], [0.0, 32.0], [100.5, 70.2]])
    assert frontend.cell_of(xy, 32, 5).tolist() == [0, 0, 1, 5, 13]


def test_redetect_threshold_matches_float_rule():
    for target in (1, 7, 60, 100, 150, 1024):
        for frac in (0.0, 0.1, 0.3, 0.5, 0.9, 0.95, 1.0):
            below = frontend.redetect_below(target, frac)
            for live in range(target + 1):
                assert (live < below) == (live < frac * target), (target, frac, live)
