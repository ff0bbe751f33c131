"""GPU parity for the score-map entry point and the standalone NMS over wider
neighbourhoods (Section I-B, radius 1..4) with the cell arg-max, bit for bit
against the CPU oracle."""
import numpy as np
import pytest

import oracle
from conftest import as_tuples

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2003_13493_amd import fastgrid, synth  # noqa: E402

SPECS = [synth.PLAIN_320, synth.PLAIN_752, synth.PLAIN_1080]
SPEC_IDS = ["320x240_L1", "752x480_L3", "1920x1080_L4"]


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


def score_maps(ctx, spec, img, kind):
    pyr = fastgrid.Pyramid(spec.width, spec.height, spec.levels)
    pyr.upload(img)
    maps = fastgrid.ScoreMaps(spec.width, spec.height, spec.levels)
    for t in maps.tensors:
        t.fill_(0x5A5A)
    ctx.score_maps(pyr, spec.t, spec.n, maps, score=kind)
    torch.cuda.synchronize()
    return pyr, maps


@pytest.mark.parametrize("kind", [fastgrid.FAST_SCORE_SADB, fastgrid.FAST_SCORE_MT], ids=["sadb", "mt"])
@pytest.mark.parametrize("spec", SPECS, ids=SPEC_IDS)
def test_score_maps_every_level(ctx, spec, kind):
    print(f"case score maps {spec} kind {kind}", flush=True)
    img = spec.make()
    pyr, maps = score_maps(ctx, spec, img, kind)
    planes = oracle.pyr_build(img, spec.width, spec.levels)
    for k, (p, w) in enumerate(planes):
        if k:
            assert np.array_equal(pyr.level(k), p[:, :w]), f"level {k}"
        want = oracle.score_map(p, w, spec.t, spec.n, kind)
        assert np.array_equal(maps.level(k), want), f"score map of level {k}"


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("spec", SPECS, ids=SPEC_IDS)
def test_nms_grid_radius(ctx, spec, radius):
    print(f"case nms radius {radius} {spec}", flush=True)
    img = spec.make()
    _, maps = score_maps(ctx, spec, img, fastgrid.FAST_SCORE_SADB)
    grid = fastgrid.Grid(spec.width, spec.height, spec.cell)
    grid.tensor.fill_(0x77)
    ctx.nms_grid(maps, radius, spec.cell, grid)
    torch.cuda.synchronize()
    want, _ = oracle.detect_grid(img, spec.width, spec.levels, spec.t, spec.n, spec.cell,
                                 oracle.SCORE_SADB, radius)
    got = grid.fetch()
    compare(got, want, f"{spec.width}x{spec.height} radius {radius}")
    if radius == 1:
        g2 = fastgrid.Grid(spec.width, spec.height, spec.cell)
        pyr = fastgrid.Pyramid(spec.width, spec.height, spec.levels)
        pyr.upload(img)
        ctx.detect(pyr, spec.t, spec.n, spec.cell, g2)
        torch.cuda.synchronize()
        assert np.array_equal(g2.fetch(), got)


@pytest.mark.parametrize("radius", [2, 4])
def test_nms_grid_odd_sizes_and_cells(ctx, radius):
    """Frames whose sizes and cells do not divide evenly, several levels."""
    for i, (w, h, levels, cell) in enumerate([(333, 222, 3, 20), (97, 301, 2, 6), (640, 90, 4, 64)]):
        img = synth.frame(w, h, seed=500 + i, nshapes=40, sigma=5)
        spec = synth.FrameSpec(w, h, levels, 8, 9, cell, seed=0, nshapes=0, sigma=0)
        pyr = fastgrid.Pyramid(w, h, levels)
        pyr.upload(img)
        maps = fastgrid.ScoreMaps(w, h, levels)
        ctx.score_maps(pyr, spec.t, spec.n, maps)
        grid = fastgrid.Grid(w, h, cell)
        ctx.nms_grid(maps, radius, cell, grid)
        torch.cuda.synchronize()
        want, _ = oracle.detect_grid(img, w, levels, spec.t, spec.n, cell, oracle.SCORE_SADB, radius)
        compare(grid.fetch(), want, f"{w}x{h} L{levels} cell {cell} radius {radius}")


def test_nms_grid_rejects_bad_arguments(ctx):
    maps = fastgrid.ScoreMaps(64, 64, 2)
    grid = fastgrid.Grid(64, 64, 16)
    for kw in (dict(radius=0), dict(radius=5), dict(cell=3), dict(cell=512)):
        args = dict(radius=2, cell=16)
        args.update(kw)
        with pytest.raises(fastgrid.FastError) as ei:
            fastgrid.fast_nms_grid(ctx.handle, maps.ptrs, maps.pitches, 64, 64, 2, args["radius"],
                                   args["cell"], grid.ptr)
        assert ei.value.code == fastgrid.FAST_EINVAL
    short = (fastgrid.ctypes.c_int32 * 2)(63, 32)
    with pytest.raises(fastgrid.FastError) as ei:
        fastgrid.fast_nms_grid(ctx.handle, maps.ptrs, short, 64, 64, 2, 2, 16, grid.ptr)
    assert ei.value.code == fastgrid.FAST_EINVAL
    with pytest.raises(fastgrid.FastError) as ei:
        fastgrid.fast_nms_grid(ctx.handle, maps.ptrs, maps.pitches, 64, 64, 2, 2, 16, 0)
    assert ei.value.code == fastgrid.FAST_EINVAL
