"""The detect-and-track loop of many camera streams with device-resident
feature lists (fast_frontend_step through frontend.MultiFrontend), each
stream against the same loop restated here on the CPU oracles.

Streams differ in size, levels, threshold, arc length, cell, target and
re-detection fraction, and not every stream takes part in every step, so a
batch mixes streams at different frames.

Every step is checked against the oracle step applied to the same input: the
feature list the device held before the step.  The tracking statuses, the
tracked count, the re-detection decision and the live count must be
identical; kept positions agree within the tracker tolerance; and the added
features must be exactly the oracle's choice given the cells the device's
kept features occupy.  (A kept feature can sit within a rounding error of a
cell border, since frames move by whole pixels and new features start at
whole pixels; which cell it takes there is decided by the last bit of its
fp32 track, so the choice is checked against the device's positions.)"""
import numpy as np
import pytest

import oracle
from oracle import lk
from lkdata import wave_frame

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2003_13493_amd import fastgrid, frontend, synth  # noqa: E402

# (width, height, levels, t, n, cell, target, redetect fraction)
STREAMS = [
    (752, 480, 3, 10, 9, 32, 100, 0.3),
    (640, 480, 3, 8, 10, 16, 150, 0.95),
    (376, 240, 2, 10, 9, 16, 60, 0.5),
    (1280, 720, 4, 15, 12, 64, 80, 0.9),
]


def sequence(w, h, nframes: int, seed: int):
    """Crops of a (w+64) x (h+64) scene (shapes plus plane waves) along a
    seeded random walk of up to 3 pixels per frame."""
    rng = np.random.default_rng(seed)
    shapes = synth.frame(w + 64, h + 64, seed=seed, nshapes=150, sigma=0.0)[:, :w + 64].astype(np.float64)
    waves = wave_frame(w + 64, h + 64, seed=seed).astype(np.float64)
    scene = np.clip(0.6 * shapes + 0.6 * (waves - 128) + 20, 0, 255).astype(np.uint8)
    o = np.array([32, 32])
    frames = []
    for f in range(nframes):
        if f:
            o = np.clip(o + rng.integers(-3, 4, size=2), 0, 64)
        frames.append(np.ascontiguousarray(scene[o[1]:o[1] + h, o[0]:o[0] + w]))
    return frames


def oracle_step(prev_planes, img, feats_in, w, levels, t, n, cell, target, frac, mode, eps, kept_device=None):
    """One step of the loop on the oracles, from the input features feats_in
    (level-0 positions): track them into img, keep the tracked ones, and below
    frac * target live detect (SAD-A) and add the strongest winners of cells
    holding no kept feature (the device's kept positions when given), equal
    scores by cell index.  Returns ((tracked, re-detected, live), kept
    positions, added positions, tracking statuses, img's pyramid)."""
    planes = oracle.pyr_build(img, w, levels)
    kept = np.zeros((0, 2))
    st = np.zeros(0, dtype=np.int32)
    if prev_planes is not None and len(feats_in):
        q, st, _ = lk.track(prev_planes, planes, feats_in.astype(np.float32).astype(np.float64), mode=mode,
                            eps=eps)
        q = q.astype(np.float32).astype(np.float64)
        keep = st == lk.TRACKED
        kept = feats_in[keep].astype(np.float64) + q[keep, :2]
    tracked = len(kept)
    redetect = tracked < frac * target
    new = np.zeros((0, 2))
    if redetect:
        gw = (w + cell - 1) // cell
        slots, _ = oracle.detect_grid(img, w, levels, t, n, cell, kind=oracle.SCORE_SADA)
        flat = slots.reshape(-1)
        base = kept if kept_device is None else kept_device
        busy = {int(np.floor(y / cell)) * gw + int(np.floor(x / cell)) for x, y in base}
        cands = sorted((-int(flat["score"][i]), i) for i in range(len(flat))
                       if flat["score"][i] > 0 and i not in busy)
        new = np.array([(float(int(flat["x"][i]) << int(flat["level"][i])),
                         float(int(flat["y"][i]) << int(flat["level"][i])))
                        for _, i in cands[:target - tracked]]).reshape(-1, 2)
    return (tracked, bool(redetect), tracked + len(new)), kept, new, st, planes


def check_step(tag, got_info, got_feats, want, tol=0.01):
    info, kept, new, _, _ = want
    assert got_info == info, f"{tag}: {got_info} vs {info}"
    tracked = info[0]
    d = np.abs(got_feats[:tracked] - kept).max(initial=0)
    assert d <= tol, f"{tag}: kept positions differ by {d}"
    assert np.array_equal(got_feats[tracked:], new), f"{tag}: added features differ"


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fastgrid.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("mode", [0, 3], ids=["t", "t+gain+offset"])
def test_multi_stream_loop_matches_oracle(ctx, mode):
    nframes, eps = 10, 1e-3
    seqs = [sequence(w, h, nframes, seed=70 + i) for i, (w, h, *_) in enumerate(STREAMS)]
    mf = frontend.MultiFrontend(ctx, [(w, h, L, t, n, c) for (w, h, L, t, n, c, _, _) in STREAMS],
                                targets=[s[6] for s in STREAMS], redetect_fracs=[s[7] for s in STREAMS],
                                mode=mode, eps=eps)
    prev = [None] * len(STREAMS)
    # stream 2 sits out steps 3 and 4, stream 3 joins at step 2: batches mix
    # streams at different frames
    step_frames = [0] * len(STREAMS)
    totals = np.zeros(3, dtype=np.int64)
    for step in range(nframes + 2):
        batch = [i for i in range(len(STREAMS))
                 if step_frames[i] < nframes and not (i == 2 and step in (3, 4)) and not (i == 3 and step < 2)]
        if not batch:
            continue
        print(f"case frontend multi mode {mode} step {step} streams {batch}", flush=True)
        inputs = {i: mf.features(i) if step_frames[i] else np.zeros((0, 2)) for i in batch}
        mf.step({i: seqs[i][step_frames[i]] for i in batch})
        torch.cuda.synchronize()
        for i in batch:
            f = step_frames[i]
            w, h, L, t, n, c, tg, fr = STREAMS[i]
            info = mf.info(i)
            got = mf.features(i)
            want = oracle_step(prev[i], seqs[i][f], inputs[i], w, L, t, n, c, tg, fr, mode, eps,
                               kept_device=got[:info[0]])
            # the tracker's statuses on the same inputs are identical
            st = mf.streams[i].status[:len(inputs[i])].cpu().numpy() if len(inputs[i]) else np.zeros(0)
            if prev[i] is not None:
                assert np.array_equal(st, want[3]), f"stream {i} frame {f}: statuses differ"
            check_step(f"stream {i} frame {f}", info, got, want)
            totals += (info[0], int(info[1]) * (f > 0), info[2])
            prev[i] = want[4]
            step_frames[i] += 1
    assert step_frames == [nframes] * len(STREAMS)
    # the loop did both things it is for: it tracked, and re-detected after the first frames
    assert totals[0] > 400 and totals[1] >= 3


def test_rejects_bad_jobs(ctx):
    mf = frontend.MultiFrontend(ctx, [(320, 240, 2, 10, 9, 16)], targets=[50], redetect_fracs=[0.3])
    st = mf.streams[0]
    jobs = (fastgrid.fast_frontend_job * 1)()
    jobs[0] = mf._job(0, prev=None)
    lib = fastgrid.load()
    assert lib.fast_frontend_step(ctx.handle, jobs, 1, 0, 30, 0.01, None, None) == 0
    torch.cuda.synchronize()
    for field, value in (("capacity", 0), ("capacity", fastgrid.FAST_MAX_TRACKS + 1), ("redetect_below", 51),
                         ("cell", 25), ("levels", 9)):
        bad = (fastgrid.fast_frontend_job * 1)()
        bad[0] = mf._job(0, prev=None)
        setattr(bad[0], field, value)
        assert lib.fast_frontend_step(ctx.handle, bad, 1, 0, 30, 0.01, None, None) == fastgrid.FAST_EINVAL, field
    bad = (fastgrid.fast_frontend_job * 1)()
    bad[0] = mf._job(0, prev=None)
    bad[0].feats = st.feats.data_ptr() + 2
    assert lib.fast_frontend_step(ctx.handle, bad, 1, 0, 30, 0.01, None, None) == fastgrid.FAST_EINVAL
    assert lib.fast_frontend_step(ctx.handle, jobs, 1, 4, 30, 0.01, None, None) == fastgrid.FAST_EINVAL
    assert lib.fast_frontend_step(ctx.handle, jobs, 0, 0, 30, 0.01, None, None) == fastgrid.FAST_EINVAL
