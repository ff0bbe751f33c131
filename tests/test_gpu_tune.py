"""The autotuner on the GPU: on a small workload every candidate it times is
bit-exact with the oracle, the chosen region side is the one the library then
applies to that frame shape, and detection with the chosen shapes (one-frame
and batched) is the oracle's answer.  The shipped table, when present, is
what a new context applies."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2003_13493_amd import fastgrid, synth, tune  # noqa: E402


@pytest.fixture()
def ctx():
    assert torch.cuda.is_available()
    c = fastgrid.Context(0, tuned=False)
    yield c
    torch.cuda.synchronize()
    c.close()


def slots(spec, img):
    return oracle.detect_grid(img, spec.width, spec.levels, spec.t, spec.n, spec.cell)[0]


def test_shape_table_rules(ctx):
    # default rule: a small 3-level frame uses 32-pixel regions, a large one 64
    assert ctx.shape_region(752, 480, 3, 32) == 32
    assert ctx.shape_region(1920, 1080, 4, 64) == 64
    ctx.set_shape_table([(752, 480, 3, 32, 64), (1920, 1080, 4, 64, 128)])
    assert ctx.shape_region(752, 480, 3, 32) == 64
    assert ctx.shape_region(1920, 1080, 4, 64) == 128
    assert ctx.shape_region(752, 480, 3, 16) == 32          # another cell: the default rule
    ctx.set_launch(32, 256, 3)                               # an explicit side overrides the table
    assert ctx.shape_region(752, 480, 3, 32) == 32
    ctx.reset_launch()
    assert ctx.shape_region(752, 480, 3, 32) == 64
    with pytest.raises(fastgrid.FastError):
        ctx.set_shape_table([(752, 480, 3, 32, 8)])         # region below 16
    with pytest.raises(fastgrid.FastError):
        ctx.set_shape_table([(752, 480, 3, 32, 64), (752, 480, 3, 32, 32)])   # listed twice
    with pytest.raises(fastgrid.FastError):
        ctx.set_shape_table([(752, 480, 3, 30, 64)])         # cell not a multiple of 2^(L-1)
    assert ctx.shape_region(752, 480, 3, 32) == 64          # a rejected table leaves the old one
    ctx.set_shape_table([])
    assert ctx.shape_region(752, 480, 3, 32) == 32


def test_tuner_gates_and_applies(ctx):
    specs = [synth.PLAIN_320, synth.PLAIN_752]
    cases = []
    for s in specs:
        img = s.make()
        cases.append((s, img, slots(s, img)))
    print("case tune shapes", flush=True)
    rows = tune.tune_shapes(ctx, cases, regions=(16, 32, 64), reps=10, warmup=2)
    for row, (s, img, want) in zip(rows, cases):
        assert row["region"] is not None and all(c["exact"] for c in row["candidates"])
        best = min(row["candidates"], key=lambda c: c["us"])
        assert row["region"] == best["region"]
        assert ctx.shape_region(s.width, s.height, s.levels, s.cell) == row["region"]
        pyr = fastgrid.Pyramid(s.width, s.height, s.levels)
        pyr.upload(img)
        g = fastgrid.Grid(s.width, s.height, s.cell)
        ctx.detect(pyr, s.t, s.n, s.cell, g)
        torch.cuda.synchronize()
        assert np.array_equal(g.fetch(), want)
    print("case tune batch", flush=True)
    bspecs = synth.batch64()[:6]
    frames = [s.make() for s in bspecs]
    want = [slots(s, f) for s, f in zip(bspecs, frames)]
    res = tune.tune_batch(ctx, bspecs, frames, want, candidates=[(256, 3), (256, 2), (512, 1)], reps=10,
                          warmup=2)
    assert all(c["exact"] for c in res["candidates"])
    assert [res["block"], res["blocks_per_cu"]] in [[c["block"], c["blocks_per_cu"]] for c in res["candidates"]]
    # the context runs at the chosen shape: a submission is still the oracle's answer
    pyrs = [fastgrid.Pyramid(s.width, s.height, s.levels) for s in bspecs]
    grids = [fastgrid.Grid(s.width, s.height, s.cell) for s in bspecs]
    for p, f in zip(pyrs, frames):
        p.upload(f)
    tk = ctx.submit(fastgrid.Context.make_jobs((p, s.t, s.n, s.cell, g) for p, s, g in zip(pyrs, bspecs, grids)))
    assert ctx.wait(tk, 60_000)
    for g, w in zip(grids, want):
        assert np.array_equal(g.fetch(), w)


def test_shipped_table_is_applied():
    table = tune.load()
    if table is None:
        pytest.skip("no tuned table shipped")
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    c = fastgrid.Context(0)
    try:
        if table["device"] != arch:
            assert c.tuned is None
            return
        assert c.tuned == tune.TABLE_PATH
        for e in table["shapes"]:
            if e["region"]:
                assert c.shape_region(e["width"], e["height"], e["levels"], e["cell"]) == e["region"]
        s = synth.PLAIN_752
        img = s.make()
        pyr = fastgrid.Pyramid(s.width, s.height, s.levels)
        pyr.upload(img)
        g = fastgrid.Grid(s.width, s.height, s.cell)
        c.detect(pyr, s.t, s.n, s.cell, g)
        torch.cuda.synchronize()
        assert np.array_equal(g.fetch(), slots(s, img))
    finally:
        c.close()
