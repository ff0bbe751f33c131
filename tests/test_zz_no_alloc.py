"""GPU check of fast_submit_static, the batched entry point that allocates
nothing: through the C ABI, its slots and pyramid levels must equal
fast_submit's bit for bit (and the oracle's), on two calls in a row, the
second with a smaller batch, and it must reject batches beyond its scratch
limits without enqueuing anything."""
import ctypes

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2003_13493_amd import fastgrid, synth  # noqa: E402

LIB_HDR_MAX_JOBS = 256
LIB_HDR_MAX_ITEMS = 32768


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = fastgrid.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def resident(specs, frames):
    pyrs, grids = [], []
    for s, img in zip(specs, frames):
        p = fastgrid.Pyramid(s.width, s.height, s.levels)
        p.upload(img)
        pyrs.append(p)
        grids.append(fastgrid.Grid(s.width, s.height, s.cell))
    jobs = fastgrid.Context.make_jobs((p, s.t, s.n, s.cell, g) for p, s, g in zip(pyrs, specs, grids))
    return pyrs, grids, jobs


def run_both(ctx, specs, frames):
    """The same frames through fast_submit and fast_submit_static (separate
    pyramids and grids); returns both sets of slots and levels."""
    outs = []
    for static in (False, True):
        pyrs, grids, jobs = resident(specs, frames)
        # poison the outputs so stale values cannot pass
        for g in grids:
            g.tensor.fill_(0xA5)
        for p in pyrs:
            for t in p.tensors[1:]:
                t.fill_(0x5A)
        if static:
            tk = ctx.submit_static(jobs)
        else:
            tk = ctx.submit(jobs)
        assert ctx.wait(tk, 60_000)
        outs.append([(g.fetch().copy(), [p.level(k).copy() for k in range(1, s.levels)])
                     for s, p, g in zip(specs, pyrs, grids)])
    return outs


def check_equal(specs, frames, a, b, tag, with_oracle=True):
    for i, s in enumerate(specs):
        sa, la = a[i]
        sb, lb = b[i]
        assert np.array_equal(sa, sb), f"{tag}: frame {i} slots differ from fast_submit"
        for k in range(1, s.levels):
            assert np.array_equal(la[k - 1], lb[k - 1]), f"{tag}: frame {i} level {k} differs"
        if with_oracle:
            want, planes = oracle.detect_grid(frames[i], s.width, s.levels, s.t, s.n, s.cell)
            assert np.array_equal(sb, want), f"{tag}: frame {i} slots differ from the oracle"


def test_static_matches_submit_twice_second_smaller(ctx):
    # first call: 20 frames of the batch workload plus one 4-level 1920x1080
    # frame (its deeper level takes the second pass and its own work items)
    specs = synth.batch64()[:20] + [synth.PLAIN_1080]
    frames = [s.make() for s in specs]
    print(f"case static call 1: {len(specs)} jobs", flush=True)
    a, b = run_both(ctx, specs, frames)
    check_equal(specs, frames, a, b, "call 1")
    # second call, smaller: 5 other frames with other parameters
    specs2 = synth.batch64(instance=1)[40:45]
    frames2 = [s.make() for s in specs2]
    print(f"case static call 2: {len(specs2)} jobs", flush=True)
    a2, b2 = run_both(ctx, specs2, frames2)
    check_equal(specs2, frames2, a2, b2, "call 2")


def test_static_back_to_back_on_one_stream(ctx):
    """Three calls enqueued before any wait: the staging buffer and the scratch
    are reused in stream order, and every call's outputs are right."""
    specs = synth.batch64(instance=2)[:6]
    frames = [s.make() for s in specs]
    want = [oracle.detect_grid(img, s.width, s.levels, s.t, s.n, s.cell)[0] for s, img in zip(specs, frames)]
    sets = [resident(specs, frames) for _ in range(3)]
    print("case static back-to-back x3", flush=True)
    for _, grids, jobs in sets:
        for g in grids:
            g.tensor.fill_(0xA5)
        ctx.submit_static(jobs, ticket=False)
    torch.cuda.synchronize()
    for r, (_, grids, _) in enumerate(sets):
        for i, g in enumerate(grids):
            assert np.array_equal(g.fetch(), want[i]), f"call {r} frame {i}"


def test_static_rejects_beyond_limits(ctx):
    lib = fastgrid.load()
    s = synth.PLAIN_320
    pyr = fastgrid.Pyramid(s.width, s.height, s.levels)
    grid = fastgrid.Grid(s.width, s.height, s.cell)
    one = fastgrid.Context.make_jobs([(pyr, s.t, s.n, s.cell, grid)])
    tk = ctypes.c_uint64(0)
    # too many jobs
    many = (fastgrid.fast_job * (LIB_HDR_MAX_JOBS + 1))(*([one[0]] * (LIB_HDR_MAX_JOBS + 1)))
    rc = lib.fast_submit_static(ctx.handle, many, len(many), None, ctypes.byref(tk))
    assert rc == fastgrid.FAST_EINVAL and tk.value == 0
    assert b"static scratch" in lib.fast_last_error(ctx.handle)
    # too many work items: 16-pixel cells of a 4096x2160 frame give 16-pixel
    # regions, 256 x 135 = 34560 of them
    big = fastgrid.Pyramid(4096, 2160, 1)
    bgrid = fastgrid.Grid(4096, 2160, 16)
    ctx.set_launch(16, 256, 3)
    try:
        jb = fastgrid.Context.make_jobs([(big, 10, 9, 16, bgrid)])
        rc = lib.fast_submit_static(ctx.handle, jb, 1, None, ctypes.byref(tk))
        assert rc == fastgrid.FAST_EINVAL and tk.value == 0
        assert b"work items" in lib.fast_last_error(ctx.handle)
    finally:
        ctx.reset_launch()
    # zero jobs and a NULL job array
    assert lib.fast_submit_static(ctx.handle, one, 0, None, None) == fastgrid.FAST_EINVAL
    assert lib.fast_submit_static(ctx.handle, None, 1, None, None) == fastgrid.FAST_EINVAL
    # a bad job still rejects the whole call
    bad = fastgrid.Context.make_jobs([(pyr, 300, s.n, s.cell, grid)])
    assert lib.fast_submit_static(ctx.handle, bad, 1, None, None) == fastgrid.FAST_EINVAL
    # and after the rejections a normal call still works
    pyr.upload(s.make())
    t = ctx.submit_static(one)
    assert ctx.wait(t, 60_000)
    want, _ = oracle.detect_grid(s.make(), s.width, s.levels, s.t, s.n, s.cell)
    assert np.array_equal(grid.fetch(), want)
