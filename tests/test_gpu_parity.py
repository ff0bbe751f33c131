"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for
bit, on every slot and every pyramid level.  Integer work only, so the bar is
exact equality."""
import numpy as np
import pytest

import oracle
from conftest import as_tuples

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2003_13493_amd import fastgrid, synth  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fastgrid.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def run_plain(ctx, img, width, levels, t, n, cell):
    h = img.shape[0]
    pyr = fastgrid.Pyramid(width, h, levels)
    grid = fastgrid.Grid(width, h, cell)
    pyr.upload(img)
    ctx.detect(pyr, t, n, cell, grid)
    torch.cuda.synchronize()
    return grid.fetch(), [pyr.level(k) for k in range(levels)]


def check_against_oracle(got, levels_got, img, width, levels, t, n, cell, tag=""):
    want, planes = oracle.detect_grid(img, width, levels, t, n, cell)
    for k in range(1, levels):
        p, w = planes[k]
        assert np.array_equal(levels_got[k], p[:, :w]), f"{tag} level {k} differs"
    if not np.array_equal(got, want):
        g, wt = as_tuples(got), as_tuples(want)
        bad = [i for i in range(len(g)) if g[i] != wt[i]]
        raise AssertionError(f"{tag}: {len(bad)} cells differ, first {bad[:5]}: "
                             f"got {[g[i] for i in bad[:3]]} want {[wt[i] for i in bad[:3]]}")


@pytest.mark.parametrize("spec", [synth.PLAIN_320, synth.PLAIN_752, synth.PLAIN_1080],
                         ids=["320x240_L1", "752x480_L3", "1920x1080_L4"])
def test_plain_configs_bit_exact(ctx, spec):
    print(f"case {spec}", flush=True)
    img = spec.make()
    got, lv = run_plain(ctx, img, spec.width, spec.levels, spec.t, spec.n, spec.cell)
    check_against_oracle(got, lv, img, spec.width, spec.levels, spec.t, spec.n, spec.cell,
                         f"{spec.width}x{spec.height}")
    assert (got["score"] > 0).sum() > len(got) // 2


FUZZ = []
_rng = np.random.default_rng(2024)
for _i in range(40):
    _levels = int(_rng.integers(1, 6))
    _w = int(_rng.integers(7 << (_levels - 1), 420))
    _h = int(_rng.integers(7 << (_levels - 1), 300))
    _t = int(_rng.choice([0, 1, 10, 254, 255, int(_rng.integers(2, 60))]))
    _n = int(_rng.integers(1, 17))
    _cell = int(_rng.choice([16, 32, 64, 128])) if _levels <= 5 else 16
    if _cell % (1 << (_levels - 1)):
        _cell = 1 << (_levels - 1)
    FUZZ.append((_w, _h, _levels, _t, _n, _cell, 9000 + _i))


@pytest.mark.parametrize("w,h,levels,t,n,cell,seed", FUZZ)
def test_fuzz_sizes_params_and_padding(ctx, w, h, levels, t, n, cell, seed):
    print(f"case w={w} h={h} L={levels} t={t} n={n} cell={cell} seed={seed}", flush=True)
    pitch = (w + 63) // 64 * 64
    img = synth.frame(w, h, seed=seed, nshapes=40, sigma=4 + seed % 5, pitch=pitch,
                      pad_garbage=True)
    got, lv = run_plain(ctx, img, w, levels, t, n, cell)
    check_against_oracle(got, lv, img, w, levels, t, n, cell, f"fuzz{seed}")


@pytest.mark.parametrize("w,h,levels,cell", [
    (7, 7, 1, 1), (6, 9, 1, 4), (8, 8, 2, 2), (13, 7, 1, 256), (64, 8, 4, 8),
    (512, 512, 8, 128), (300, 200, 1, 3), (255, 129, 2, 6), (1000, 40, 3, 256),
])
def test_edge_shapes(ctx, w, h, levels, cell):
    print(f"case edge w={w} h={h} L={levels} cell={cell}", flush=True)
    img = synth.frame(w, h, seed=w * 31 + h, nshapes=10, sigma=8, pad_garbage=True)
    for t, n in ((0, 1), (10, 9), (20, 16)):
        got, lv = run_plain(ctx, img, w, levels, t, n, cell)
        check_against_oracle(got, lv, img, w, levels, t, n, cell, f"edge {w}x{h} t={t} n={n}")


def test_constant_and_extreme_images(ctx):
    for v in (0, 255):
        img = np.full((64, 64), v, np.uint8)
        got, _ = run_plain(ctx, img, 64, 2, 0, 1, 16)
        assert all(s == fastgrid.EMPTY for s in as_tuples(got))
    rng = np.random.default_rng(5)
    img = (rng.integers(0, 2, size=(96, 128)) * 255).astype(np.uint8)   # max contrast
    for t, n in ((0, 1), (0, 9), (254, 3)):
        got, lv = run_plain(ctx, img, 128, 3, t, n, 32)
        check_against_oracle(got, lv, img, 128, 3, t, n, 32, f"binary t={t} n={n}")


def test_launch_shapes_agree(ctx):
    spec = synth.PLAIN_752
    img = spec.make()
    want, _ = oracle.detect_grid(img, spec.width, spec.levels, spec.t, spec.n, spec.cell)
    try:
        for region, block in ((32, 64), (64, 256), (128, 512), (256, 128), (96, 128), (0, 256), (16, 256)):
            ctx.set_launch(region, block, 4)
            got, _ = run_plain(ctx, img, spec.width, spec.levels, spec.t, spec.n, spec.cell)
            assert np.array_equal(got, want), (region, block)
    finally:
        ctx.reset_launch()


def test_set_launch_rejects_bad_shapes(ctx):
    """Blocks must be multiples of 64 in 64..512, regions 16..256, 1..16
    workgroups per CU (region 0: the defaults); a rejected shape leaves the
    previous one in force."""
    try:
        for region, block, bpc in ((64, 100, 3), (64, 0, 3), (64, 576, 3), (8, 256, 3), (300, 256, 3), (-1, 256, 3),
                                   (64, 256, 0), (64, 256, 17)):
            with pytest.raises(fastgrid.FastError) as ei:
                ctx.set_launch(region, block, bpc)
            assert ei.value.code == fastgrid.FAST_EINVAL
        for block in (192, 320, 448):
            ctx.set_launch(64, block, 2)
    finally:
        ctx.reset_launch()
    spec = synth.PLAIN_320
    img = spec.make()
    want, _ = oracle.detect_grid(img, spec.width, spec.levels, spec.t, spec.n, spec.cell)
    got, _ = run_plain(ctx, img, spec.width, spec.levels, spec.t, spec.n, spec.cell)
    assert np.array_equal(got, want)


def test_pyr_build_entry_point(ctx):
    img = synth.frame(333, 222, seed=77, nshapes=20, sigma=5, pad_garbage=True)
    pyr = fastgrid.Pyramid(333, 222, 5)
    pyr.upload(img)
    ctx.pyr_build(pyr)
    torch.cuda.synchronize()
    planes = oracle.pyr_build(img, 333, 5)
    for k in range(1, 5):
        p, w = planes[k]
        assert np.array_equal(pyr.level(k), p[:, :w])


def test_invalid_arguments_enqueue_nothing(ctx):
    pyr = fastgrid.Pyramid(64, 64, 2)
    grid = fastgrid.Grid(64, 64, 16)
    bad = [dict(t=-1), dict(t=256), dict(n=0), dict(n=17), dict(cell=3), dict(cell=512),
           dict(cell=0)]
    for b in bad:
        args = dict(t=10, n=9, cell=16)
        args.update(b)
        with pytest.raises(fastgrid.FastError) as ei:
            ctx.detect(pyr, args["t"], args["n"], args["cell"], grid)
        assert ei.value.code == fastgrid.FAST_EINVAL
    # misaligned pitch and wrong level size
    planes = (fastgrid.fast_plane * 2)(*pyr.planes)
    planes[0].pitch = 72
    with pytest.raises(fastgrid.FastError):
        fastgrid.fast_detect_grid(ctx.handle, planes, 2, 10, 9, 16, grid.ptr)
    planes = (fastgrid.fast_plane * 2)(*pyr.planes)
    planes[1].width = 33
    with pytest.raises(fastgrid.FastError):
        fastgrid.fast_detect_grid(ctx.handle, planes, 2, 10, 9, 16, grid.ptr)
    planes = (fastgrid.fast_plane * 2)(*pyr.planes)
    planes[0].data = planes[0].data + 8
    with pytest.raises(fastgrid.FastError):
        fastgrid.fast_detect_grid(ctx.handle, planes, 2, 10, 9, 16, grid.ptr)
    with pytest.raises(fastgrid.FastError):
        fastgrid.fast_detect_grid(ctx.handle, pyr.planes, 2, 10, 9, 16, 0)


def test_largest_stream_frame_4096x2160_five_levels(ctx):
    """The largest frame of the camera-stream workload (4096x2160, 5 levels)
    through the plain path and through a one-job batch, every slot and level
    against the oracle."""
    spec = synth.streams32()[3]
    assert (spec.width, spec.height) == (4096, 2160)
    img = spec.frame(0)
    print("case 4096x2160 L=5", flush=True)
    got, lv = run_plain(ctx, img, spec.width, 5, spec.t, spec.n, spec.cell)
    check_against_oracle(got, lv, img, spec.width, 5, spec.t, spec.n, spec.cell, "4k plain")
    pyr = fastgrid.Pyramid(spec.width, spec.height, 5)
    pyr.upload(img)
    grid = fastgrid.Grid(spec.width, spec.height, spec.cell)
    jobs = fastgrid.Context.make_jobs([(pyr, spec.t, spec.n, spec.cell, grid)])
    assert ctx.wait(ctx.submit(jobs), 60_000)
    assert np.array_equal(grid.fetch(), got)


@pytest.mark.parametrize("w,h,levels,cell", [(8192, 16, 1, 16), (16, 4096, 2, 16), (6000, 40, 3, 32)])
def test_extreme_aspect_ratios(ctx, w, h, levels, cell):
    print(f"case aspect {w}x{h} L={levels}", flush=True)
    img = synth.frame(w, h, seed=w + h, nshapes=30, sigma=5, pad_garbage=True)
    got, lv = run_plain(ctx, img, w, levels, 10, 9, cell)
    check_against_oracle(got, lv, img, w, levels, 10, 9, cell, f"aspect {w}x{h}")
