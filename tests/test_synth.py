"""The seeded input generator: determinism and the recipe's basic statistics."""
import numpy as np

from paper_2003_13493_amd import synth


def test_frame_is_deterministic_and_seeded():
    a = synth.frame(320, 240, seed=1, nshapes=60, sigma=4)
    b = synth.frame(320, 240, seed=1, nshapes=60, sigma=4)
    c = synth.frame(320, 240, seed=2, nshapes=60, sigma=4)
    assert a.shape == (240, 320) and np.array_equal(a, b) and not np.array_equal(a, c)


def test_noise_and_background_statistics():
    # no shapes: background in [40,200] plus N(0, sigma^2) noise
    img = synth.frame(512, 512, seed=9, nshapes=0, sigma=4)[:, :512].astype(float)
    assert 40 - 1 <= np.median(img) <= 200 + 1
    assert abs(img.std() - 4.0) < 0.1
    flat = synth.frame(64, 64, seed=9, nshapes=0, sigma=0)
    assert (flat == flat[0, 0]).all()


def test_gradient_spans_plus_minus_40():
    img = synth.frame(301, 201, seed=3, nshapes=0, sigma=0, gradient=True)[:, :301].astype(int)
    corners = [img[0, 0], img[0, -1], img[-1, 0], img[-1, -1]]
    assert max(corners) - min(corners) in (79, 80, 81)


def test_padding_garbage_only_touches_padding():
    a = synth.frame(100, 50, seed=4, nshapes=10, sigma=4, pitch=128)
    b = synth.frame(100, 50, seed=4, nshapes=10, sigma=4, pitch=128, pad_garbage=True)
    assert np.array_equal(a[:, :100], b[:, :100]) and b[:, 100:].any()


def test_workload_recipes():
    batch = synth.batch64()
    assert len(batch) == 64
    sizes = sorted((s.width, s.height) for s in batch)
    assert sizes.count((752, 480)) == 24 and sizes.count((1280, 720)) == 24
    assert sizes.count((640, 480)) == 16
    assert all(s.levels == 3 and s.t in synth.BATCH_T and s.n in synth.BATCH_N and
               s.cell in synth.BATCH_CELL for s in batch)
    assert sum(s.pixels for s in batch) == 35_696_640
    streams = synth.streams32()
    assert len(streams) == 32 and all(100 <= s.rate_fps <= 1000 for s in streams)
    assert all(3 <= s.levels <= 5 and s.cell % (1 << (s.levels - 1)) == 0 for s in streams)
    f0, f1 = streams[0].frame(0), streams[0].frame(1)
    assert f0.shape == f1.shape and not np.array_equal(f0, f1)
