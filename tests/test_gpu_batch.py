"""GPU parity of the batched entry points (persistent launch over a device work
queue, and graph-captured resident batches) against the oracle and against
the plain one-frame path."""
import numpy as np
import pytest

import oracle
from conftest import as_tuples

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2003_13493_amd import fastgrid, synth  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = fastgrid.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def batch():
    """The uneven 64-frame batch with its oracle answers."""
    specs = synth.batch64()
    frames = [s.make() for s in specs]
    want = []
    for s, img in zip(specs, frames):
        slots, planes = oracle.detect_grid(img, s.width, s.levels, s.t, s.n, s.cell)
        want.append((slots, [p[:, :w].copy() for p, w in planes]))
    return specs, frames, want


def make_resident(specs, frames):
    pyrs, grids = [], []
    for s, img in zip(specs, frames):
        p = fastgrid.Pyramid(s.width, s.height, s.levels)
        p.upload(img)
        pyrs.append(p)
        grids.append(fastgrid.Grid(s.width, s.height, s.cell))
    jobs = fastgrid.Context.make_jobs((p, s.t, s.n, s.cell, g) for p, s, g in zip(pyrs, specs, grids))
    return pyrs, grids, jobs


def check_all(specs, pyrs, grids, want, tag):
    for i, (s, p, g) in enumerate(zip(specs, pyrs, grids)):
        slots, planes = want[i]
        for k in range(1, s.levels):
            assert np.array_equal(p.level(k), planes[k]), f"{tag} frame {i} level {k}"
        got = g.fetch()
        if not np.array_equal(got, slots):
            gt, wt = as_tuples(got), as_tuples(slots)
            bad = [c for c in range(len(gt)) if gt[c] != wt[c]]
            raise AssertionError(f"{tag} frame {i} ({s.width}x{s.height} t={s.t} n={s.n} "
                                 f"cell={s.cell}): {len(bad)} cells differ, e.g. {bad[:3]}")


def test_submit_batch64_bit_exact(ctx, batch):
    specs, frames, want = batch
    print("case submit batch64", flush=True)
    pyrs, grids, jobs = make_resident(specs, frames)
    tk = ctx.submit(jobs)
    assert ctx.wait(tk, 60_000)
    assert ctx.poll(tk)
    check_all(specs, pyrs, grids, want, "submit")


def test_submit_back_to_back_reuses_queue(ctx, batch):
    """Several submissions in a row: the self-resetting queue counter must be
    re-armed by each launch."""
    specs, frames, want = batch
    sel = list(range(0, 64, 5))
    sp = [specs[i] for i in sel]
    pyrs, grids, jobs = make_resident(sp, [frames[i] for i in sel])
    tickets = []
    for r in range(6):
        for g in grids:
            g.tensor.fill_(0xAB)
        tickets.append(ctx.submit(jobs))
        assert ctx.wait(tickets[-1], 60_000)
        check_all(sp, pyrs, grids, [want[i] for i in sel], f"round {r}")
    assert all(ctx.poll(t) for t in tickets)


@pytest.mark.parametrize("graph", [False, True], ids=["direct", "graph"])
def test_plan_replays(ctx, batch, graph):
    specs, frames, want = batch
    print(f"case plan replays graph={graph}", flush=True)
    pyrs, grids, jobs = make_resident(specs, frames)
    pid = ctx.plan_create(jobs, graph=graph)
    try:
        for r in range(4):
            for g in grids:
                g.tensor.fill_(0x5A)
            for p in pyrs:
                for t in p.tensors[1:]:
                    t.fill_(0)
            torch.cuda.synchronize()
            if r % 2:
                assert ctx.plan_launch(pid, ticket=False) == 0
                torch.cuda.synchronize()
            else:
                tk = ctx.plan_launch(pid)
                assert ctx.wait(tk, 60_000)
            check_all(specs, pyrs, grids, want, f"replay {r}")
    finally:
        ctx.plan_destroy(pid)


@pytest.mark.parametrize("graph", [False, True], ids=["direct", "graph"])
def test_plan_mixed_levels(ctx, graph):
    """Frames with 1..5 levels in one plan: levels 4.. need the separate pyramid
    kernels before the persistent launch."""
    rng = np.random.default_rng(31)
    specs, frames, want = [], [], []
    for i in range(10):
        levels = 1 + i % 5
        w = int(rng.integers(7 << (levels - 1), 500))
        h = int(rng.integers(7 << (levels - 1), 400))
        cell = max(16, 1 << (levels - 1))
        s = synth.FrameSpec(w, h, levels, synth.BATCH_T[i % 4], synth.BATCH_N[i % 3], cell,
                            seed=600 + i, nshapes=60, sigma=4.0)
        img = s.make()
        specs.append(s)
        frames.append(img)
        slots, planes = oracle.detect_grid(img, w, levels, s.t, s.n, cell)
        want.append((slots, [p[:, :pw].copy() for p, pw in planes]))
    print(f"case plan mixed levels graph={graph}", flush=True)
    pyrs, grids, jobs = make_resident(specs, frames)
    pid = ctx.plan_create(jobs, graph=graph)
    try:
        for r in range(2):
            for g in grids:
                g.tensor.fill_(0x77)
            torch.cuda.synchronize()
            ctx.plan_launch(pid, ticket=False)
            torch.cuda.synchronize()
            check_all(specs, pyrs, grids, want, f"mixed replay {r}")
    finally:
        ctx.plan_destroy(pid)


def test_batch_single_subtile_regions_of_mixed_sides(ctx):
    """Cells of 16, 24, 32, 48 and 64 pixels give single-sub-tile regions 48 or
    64 pixels wide (plus clipped ones at frame edges) with 1..3 levels in one
    launch, so the pipelined kernel changes staged geometry from region to
    region and must not reuse compass group entries across geometries.
    (Regions always start on the 16-pixel grid: cells whose region would not,
    such as 20 or 40, get 80-pixel regions and the generic kernel.)"""
    rng = np.random.default_rng(123)
    specs, frames, want = [], [], []
    for i in range(15):
        levels = 1 + i % 3
        cell = (16, 24, 32, 48, 64)[i % 5]
        w = int(rng.integers(40, 420))
        h = int(rng.integers(30, 300))
        s = synth.FrameSpec(w, h, levels, synth.BATCH_T[i % 4], synth.BATCH_N[i % 3], cell,
                            seed=1300 + i, nshapes=50, sigma=4.0)
        img = s.make()
        specs.append(s)
        frames.append(img)
        slots, planes = oracle.detect_grid(img, w, levels, s.t, s.n, cell)
        want.append((slots, [p[:, :pw].copy() for p, pw in planes]))
    print("case batch mixed region sides", flush=True)
    pyrs, grids, jobs = make_resident(specs, frames)
    for r in range(2):
        for g in grids:
            g.tensor.fill_(0x77)
        torch.cuda.synchronize()
        tk = ctx.submit(jobs)
        assert ctx.wait(tk, 60_000)
        check_all(specs, pyrs, grids, want, f"mixed sides round {r}")


@pytest.mark.parametrize("nframes", [1, 9, 127, 128, 129, 255, 300])
def test_batch_region_counts_around_queue_runs(ctx, nframes):
    """The work queues hand out runs of 16 consecutive regions round-robin
    over 8 queues, then deal the remainder past the last full round of 128
    item by item.  Batches of 64x64 frames (one region each) with region
    counts below, at and around multiples of 128 must still have every region
    processed exactly once: every frame matches the oracle."""
    specs, frames, want = [], [], []
    for i in range(nframes):
        levels = 1 + i % 3
        s = synth.FrameSpec(64, 64, levels, synth.BATCH_T[i % 4], synth.BATCH_N[i % 3], (16, 32, 64)[i % 3],
                            seed=5000 + i, nshapes=12, sigma=4.0)
        img = s.make()
        specs.append(s)
        frames.append(img)
        slots, planes = oracle.detect_grid(img, 64, levels, s.t, s.n, s.cell)
        want.append((slots, [p[:, :pw].copy() for p, pw in planes]))
    print(f"case batch of {nframes} one-region frames", flush=True)
    pyrs, grids, jobs = make_resident(specs, frames)
    for r in range(2):
        for g in grids:
            g.tensor.fill_(0x5A)
        torch.cuda.synchronize()
        tk = ctx.submit(jobs)
        assert ctx.wait(tk, 60_000)
        check_all(specs, pyrs, grids, want, f"{nframes} frames round {r}")


def test_submit_grows_its_staging_buffer(ctx):
    """Two 4096x2160 frames with 16-pixel regions are about 69,000 work items,
    more than a submission slot first holds: the job table and items move to
    larger pinned and device buffers, and the result stays exact.  A small
    submission afterwards reuses the grown slot."""
    specs = [synth.FrameSpec(4096, 2160, 3, 12, 9, 16, seed=1500 + i, nshapes=150, sigma=4.0)
             for i in range(2)]
    frames = [s.make() for s in specs]
    want = []
    for s, img in zip(specs, frames):
        slots, planes = oracle.detect_grid(img, s.width, s.levels, s.t, s.n, s.cell)
        want.append((slots, [p[:, :pw].copy() for p, pw in planes]))
    print("case large submission", flush=True)
    try:
        ctx.set_launch(16, 256, 3)
        for rnd in range(2):
            sp, fr, wt = (specs, frames, want) if rnd == 0 else (specs[:1], frames[:1], want[:1])
            pyrs, grids, jobs = make_resident(sp, fr)
            tk = ctx.submit(jobs)
            assert ctx.wait(tk, 60_000)
            check_all(sp, pyrs, grids, wt, f"large submission round {rnd}")
    finally:
        ctx.reset_launch()


def test_plan_rejects_unknown_flags(ctx, batch):
    specs, frames, _ = batch
    pyrs, grids, jobs = make_resident(specs[:2], frames[:2])
    with pytest.raises(fastgrid.FastError) as ei:
        fastgrid.fast_plan_create(ctx.handle, jobs, 2, 6)
    assert ei.value.code == fastgrid.FAST_EINVAL


def test_batch_equals_plain_per_frame(ctx, batch):
    specs, frames, _ = batch
    sel = [0, 7, 13, 40, 63]
    sp = [specs[i] for i in sel]
    pyrs, grids, jobs = make_resident(sp, [frames[i] for i in sel])
    tk = ctx.submit(jobs)
    assert ctx.wait(tk, 60_000)
    for s, i, g in zip(sp, sel, grids):
        p = fastgrid.Pyramid(s.width, s.height, s.levels)
        p.upload(frames[i])
        g2 = fastgrid.Grid(s.width, s.height, s.cell)
        ctx.detect(p, s.t, s.n, s.cell, g2)
        torch.cuda.synchronize()
        assert np.array_equal(g.fetch(), g2.fetch())


def test_submit_rejects_bad_job_and_enqueues_nothing(ctx, batch):
    specs, frames, _ = batch
    sp = specs[:3]
    pyrs, grids, jobs = make_resident(sp, frames[:3])
    jobs[1].n = 0
    with pytest.raises(fastgrid.FastError) as ei:
        ctx.submit(jobs)
    assert ei.value.code == fastgrid.FAST_EINVAL


def test_poll_unknown_ticket(ctx):
    with pytest.raises(fastgrid.FastError):
        ctx.poll(10 ** 12)


@pytest.mark.parametrize("shape", [(64, 256, 3), (128, 256, 3), (256, 512, 2), (32, 128, 4),
                                   (64, 320, 3), (64, 448, 2), (128, 192, 4)],
                         ids=["r64", "r128", "r256", "r32_b128", "r64_b320", "r64_b448", "r128_b192"])
def test_batch_launch_shapes_with_deep_levels(ctx, shape):
    """The persistent kernel with regions of several sub-tiles (no register
    prefetch), small workgroups, and jobs of 1..5 levels, so the fused pass
    and the deep-level pass both run inside one submission."""
    rng = np.random.default_rng(77)
    specs, frames, want = [], [], []
    for i in range(12):
        levels = 1 + i % 5
        w = int(rng.integers(max(64, 7 << (levels - 1)), 700))
        h = int(rng.integers(max(48, 7 << (levels - 1)), 500))
        cell = int(rng.choice([16, 32, 64]))
        s = synth.FrameSpec(w, h, levels, synth.BATCH_T[i % 4], synth.BATCH_N[i % 3], cell,
                            seed=900 + i, nshapes=80, sigma=4.0)
        img = s.make()
        specs.append(s)
        frames.append(img)
        slots, planes = oracle.detect_grid(img, w, levels, s.t, s.n, cell)
        want.append((slots, [p[:, :pw].copy() for p, pw in planes]))
    print(f"case batch shape {shape}", flush=True)
    try:
        ctx.set_launch(*shape)
        pyrs, grids, jobs = make_resident(specs, frames)
        tk = ctx.submit(jobs)
        assert ctx.wait(tk, 60_000)
        check_all(specs, pyrs, grids, want, f"shape {shape}")
    finally:
        ctx.reset_launch()


def _hold_stream(stream, ms: float) -> None:
    """Enqueue a bounded spin of about `ms` on `stream` (torch's sleep kernel,
    which exits on its own), so that work enqueued behind it stays pending
    for that long without any kernel of this library waiting on anything."""
    probe = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(probe):
        e0.record()
        torch.cuda._sleep(1_000_000)
        e1.record()
    e1.synchronize()
    per_ms = 1_000_000 / max(e0.elapsed_time(e1), 1e-3)
    with torch.cuda.stream(stream):
        torch.cuda._sleep(int(per_ms * ms))


def test_ninth_outstanding_submission_is_busy_and_wait_times_out(ctx, batch):
    """Host-forced failure paths: with the stream held by a bounded spin, eight
    submissions take every in-flight job table, so the ninth returns
    FAST_EBUSY and enqueues nothing; fast_wait with a zero timeout returns
    FAST_ETIMEDOUT; after the spin ends every submission completes, bit-exact,
    and a new submission is accepted again."""
    specs, frames, want = batch
    stream = torch.cuda.Stream()
    sets = [make_resident(specs[i:i + 1], frames[i:i + 1]) for i in range(9)]
    torch.cuda.synchronize()
    _hold_stream(stream, 400.0)
    tickets = [ctx.submit(jobs, stream) for _, _, jobs in sets[:8]]
    with pytest.raises(fastgrid.FastError) as ei:
        ctx.submit(sets[8][2], stream)
    assert ei.value.code == fastgrid.FAST_EBUSY
    assert not ctx.poll(tickets[0])
    rc = fastgrid.load().fast_wait(ctx.handle, tickets[0], 0)
    assert rc == fastgrid.FAST_ETIMEDOUT
    assert ctx.wait(tickets[0], 0) is False
    assert ctx.wait(tickets[7], 30000)
    assert all(ctx.poll(t) for t in tickets)
    for i, (pyrs, grids, _) in enumerate(sets[:8]):
        check_all(specs[i:i + 1], pyrs, grids, want[i:i + 1], f"held submission {i}")
    # the rejected ninth enqueued nothing: its outputs are still zero
    assert not sets[8][1][0].tensor.any()
    tk = ctx.submit(sets[8][2], stream)
    assert ctx.wait(tk, 30000)
    check_all(specs[8:9], sets[8][0], sets[8][1], want[8:9], "ninth after the others")
