"""Host logic of the autotuner (no GPU): a candidate whose output differs from
the expected answer is never timed or chosen; the fastest exact one wins;
refused shapes are recorded; a table tuned on another device kind is not
loaded."""
import json

import numpy as np

from paper_2003_13493_amd import fastgrid, tune


def test_gate_rejects_mismatches_and_picks_fastest_exact():
    want = [np.arange(6, dtype=np.uint16)]
    outputs = {(1,): [want[0].copy()], (2,): [want[0] + 1], (3,): [want[0].copy()], (4,): [want[0].copy()]}
    times = {(1,): 2.0, (2,): 0.1, (3,): 1.5, (4,): 3.0}
    timed = []

    def run(c):
        if c == (5,):
            raise fastgrid.FastError(-1, "set_launch", "region out of range")
        return outputs[c]

    def timer(c):
        timed.append(c)
        return times[c]

    rows, best = tune.choose([(1,), (2,), (3,), (4,), (5,)], run, timer, want)
    assert best["candidate"] == [3] and best["ms"] == 1.5
    assert (2,) not in timed                       # the fastest is wrong: never timed
    assert [r["exact"] for r in rows] == [True, False, True, True, False]
    assert "error" in rows[4]
    # nothing exact: no choice
    rows, best = tune.choose([(2,)], run, timer, want)
    assert best is None
    # a different number of outputs is a mismatch
    rows, best = tune.choose([(1,)], lambda c: [], timer, want)
    assert best is None


def test_load_checks_device_kind(tmp_path):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"device": "gfx950", "shapes": [], "batch": None}))
    assert tune.load(str(p), device="gfx950")["device"] == "gfx950"
    assert tune.load(str(p), device="gfx942") is None
    assert tune.load(str(tmp_path / "missing.json")) is None


def test_default_shapes_cover_the_workloads():
    keys = {(s.width, s.height, s.levels, s.cell) for s in tune.default_shapes()}
    assert (752, 480, 3, 32) in keys and (1920, 1080, 4, 64) in keys and (320, 240, 1, 32) in keys
    for w, h in ((752, 480), (1280, 720), (640, 480)):
        for c in (16, 32, 64):
            assert (w, h, 3, c) in keys
    assert any(k[:2] == (4096, 2160) for k in keys)
    assert len(keys) == len(tune.default_shapes())
