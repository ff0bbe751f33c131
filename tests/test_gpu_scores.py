"""GPU parity for the corner score kinds (Section II-D): the arc sum (SAD-A) and
the maximum threshold (MT) through the plain and batched entry points, bit for
bit against the CPU oracle, plus their argument checks."""
import numpy as np
import pytest

import oracle
from conftest import as_tuples

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2003_13493_amd import fastgrid, synth  # noqa: E402

KINDS = [fastgrid.FAST_SCORE_SADA, fastgrid.FAST_SCORE_MT]
KIND_IDS = ["sada", "mt"]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fastgrid.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def compare(got, want, tag):
    if not np.array_equal(got, want):
        g, wt = as_tuples(got), as_tuples(want)
        bad = [i for i in range(len(g)) if g[i] != wt[i]]
        raise AssertionError(f"{tag}: {len(bad)} cells differ, first {bad[:5]}: "
                             f"got {[g[i] for i in bad[:3]]} want {[wt[i] for i in bad[:3]]}")


@pytest.mark.parametrize("kind", KINDS, ids=KIND_IDS)
@pytest.mark.parametrize("spec", [synth.PLAIN_320, synth.PLAIN_752, synth.PLAIN_1080],
                         ids=["320x240_L1", "752x480_L3", "1920x1080_L4"])
def test_plain_score_kinds_bit_exact(ctx, spec, kind):
    print(f"case {spec} kind {kind}", flush=True)
    img = spec.make()
    pyr = fastgrid.Pyramid(spec.width, spec.height, spec.levels)
    grid = fastgrid.Grid(spec.width, spec.height, spec.cell)
    pyr.upload(img)
    ctx.detect(pyr, spec.t, spec.n, spec.cell, grid, score=kind)
    torch.cuda.synchronize()
    want, planes = oracle.detect_grid(img, spec.width, spec.levels, spec.t, spec.n, spec.cell, kind)
    for k in range(1, spec.levels):
        p, w = planes[k]
        assert np.array_equal(pyr.level(k), p[:, :w])
    got = grid.fetch()
    compare(got, want, f"{spec.width}x{spec.height} kind {kind}")
    assert (got["score"] > 0).sum() > len(got) // 2
    if kind == fastgrid.FAST_SCORE_MT:
        s = got["score"][got["score"] > 0]
        assert s.min() > spec.t and s.max() <= 255


@pytest.mark.parametrize("kind", KINDS, ids=KIND_IDS)
@pytest.mark.parametrize("n", [1, 3, 5, 7, 9, 12, 16])
def test_score_kinds_every_arc_length(ctx, kind, n):
    """Every doubling/remainder path of the window minimum and the arc cover."""
    img = synth.frame(200, 150, seed=40 + n, nshapes=40, sigma=5)
    pyr = fastgrid.Pyramid(200, 150, 2)
    grid = fastgrid.Grid(200, 150, 16)
    pyr.upload(img)
    ctx.detect(pyr, 8, n, 16, grid, score=kind)
    torch.cuda.synchronize()
    want, _ = oracle.detect_grid(img, 200, 2, 8, n, 16, kind)
    compare(grid.fetch(), want, f"n={n} kind {kind}")


@pytest.mark.parametrize("shape", [(64, 256, 3), (128, 256, 3)], ids=["pipelined", "generic"])
def test_batch_mixed_score_kinds(ctx, shape):
    """One launch whose jobs use all three kinds, 1..5 levels (deep levels go
    through the upper-level kernels), with both persistent kernels."""
    rng = np.random.default_rng(5)
    specs, pyrs, grids, items, want = [], [], [], [], []
    for i in range(12):
        levels = 1 + i % 5
        kind = i % 3
        w = int(rng.integers(max(64, 7 << (levels - 1)), 600))
        h = int(rng.integers(max(48, 7 << (levels - 1)), 400))
        cell = int(rng.choice([16, 32, 64]))
        s = synth.FrameSpec(w, h, levels, synth.BATCH_T[i % 4], synth.BATCH_N[i % 3], cell,
                            seed=700 + i, nshapes=60, sigma=4.0)
        img = s.make()
        p = fastgrid.Pyramid(w, h, levels)
        p.upload(img)
        g = fastgrid.Grid(w, h, cell)
        specs.append(s)
        pyrs.append(p)
        grids.append(g)
        items.append((p, s.t, s.n, cell, g, kind))
        want.append(oracle.detect_grid(img, w, levels, s.t, s.n, cell, kind))
    print(f"case batch mixed kinds shape {shape}", flush=True)
    try:
        ctx.set_launch(*shape)
        jobs = fastgrid.Context.make_jobs(items)
        tk = ctx.submit(jobs)
        assert ctx.wait(tk, 60_000)
    finally:
        ctx.reset_launch()
    for i, (s, p, g) in enumerate(zip(specs, pyrs, grids)):
        slots, planes = want[i]
        for k in range(1, s.levels):
            pl, pw = planes[k]
            assert np.array_equal(p.level(k), pl[:, :pw]), f"job {i} level {k}"
        compare(g.fetch(), slots, f"job {i} kind {i % 3} levels {s.levels}")


def test_unknown_score_kind_rejected(ctx):
    pyr = fastgrid.Pyramid(64, 64, 1)
    grid = fastgrid.Grid(64, 64, 16)
    for bad in (-1, 3, 100):
        with pytest.raises(fastgrid.FastError) as ei:
            fastgrid.fast_detect_grid_score(ctx.handle, pyr.planes, 1, 10, 9, 16, bad, grid.ptr)
        assert ei.value.code == fastgrid.FAST_EINVAL
        jobs = fastgrid.Context.make_jobs([(pyr, 10, 9, 16, grid, bad)])
        with pytest.raises(fastgrid.FastError) as ei:
            ctx.submit(jobs)
        assert ei.value.code == fastgrid.FAST_EINVAL
