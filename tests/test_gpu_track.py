"""GPU parity of the Lucas-Kanade tracker (Section II-E) through the C ABI
against the fp64 CPU oracle.  The kernel computes in fp32, so parameters agree
within a tolerance and statuses exactly.  A level stops once its step is under
eps, so the two sides may stop one iteration apart, and the last step moves t
by less than eps.  The translation tolerance is therefore 2 eps plus fp32
rounding; gain and offset get the matching bounds.  Parameters are compared on
every tracked feature, except on the noisy detected-corner frames, where the
compared tracks are chosen from the template alone (tests/wellposed.py)."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import lk
from lkdata import feature_grid, wave_frame
from wellposed import min_eig_per_level

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2003_13493_amd import fastgrid, synth  # noqa: E402

W, H = 320, 240
MODES = [0, fastgrid.FAST_TRACK_GAIN, fastgrid.FAST_TRACK_OFFSET,
         fastgrid.FAST_TRACK_GAIN | fastgrid.FAST_TRACK_OFFSET]
MODE_IDS = ["t", "t+gain", "t+offset", "t+gain+offset"]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fastgrid.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def device_pyramid(ctx, img, levels):
    p = fastgrid.Pyramid(img.shape[1], img.shape[0], levels)
    p.upload(img)
    ctx.pyr_build(p)
    return p


def gpu_track(ctx, tpl, img, levels, feats, q0=None, mode=3, max_iter=30, eps=0.01):
    tp, ip = device_pyramid(ctx, tpl, levels), device_pyramid(ctx, img, levels)
    n = len(feats)
    f = torch.tensor(np.asarray(feats, np.float32).reshape(n, 2), device="cuda")
    q = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    if q0 is not None:
        q.copy_(torch.tensor(np.asarray(q0, np.float32).reshape(n, 4)))
    st = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    it = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    ctx.track(tp, ip, f, q, st, it, mode=mode, max_iter=max_iter, eps=eps)
    torch.cuda.synchronize()
    return q.cpu().numpy().astype(np.float64), st.cpu().numpy(), it.cpu().numpy()


def cpu_track(tpl, img, levels, feats, q0=None, mode=3, max_iter=30, eps=0.01):
    f32 = np.asarray(feats, np.float32).astype(np.float64)   # the kernel sees float32 positions
    q0 = None if q0 is None else np.asarray(q0, np.float32).astype(np.float64)
    return lk.track(oracle.pyr_build(tpl, tpl.shape[1], levels), oracle.pyr_build(img, img.shape[1], levels),
                    f32, q0=q0, mode=mode, max_iter=max_iter, eps=eps)


def compare(got, want, eps, tag, t_tol=None, where=None):
    """Statuses must agree everywhere; parameters where the track is tracked
    and, if `where` is given, only there (see the tests that pass it)."""
    (qg, sg, ig), (qw, sw, iw) = got, want
    assert (sg == sw).all(), f"{tag}: status differs at {np.nonzero(sg != sw)[0][:8]}: {sg[sg != sw][:8]} vs {sw[sg != sw][:8]}"
    ok = sw == lk.TRACKED
    if where is not None:
        ok = ok & where
    t_tol = 2 * eps + 2e-3 if t_tol is None else t_tol
    dt = np.abs(qg[ok, :2] - qw[ok, :2]).max(initial=0)
    da = np.abs(qg[ok, 2] - qw[ok, 2]).max(initial=0)
    db = np.abs(qg[ok, 3] - qw[ok, 3]).max(initial=0)
    print(f"{tag}: {int(ok.sum())} compared, max |dt| {dt:.2e}, |dalpha| {da:.2e}, |dbeta| {db:.2e}", flush=True)
    assert dt <= t_tol, f"{tag}: translation differs by {dt}"
    assert da <= 2e-3 + 4 * eps * 0.05, f"{tag}: gain differs by {da}"
    assert db <= 0.25 + 4 * eps * 8, f"{tag}: offset differs by {db}"
    return ok


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("case", ["identical", "integer", "subpixel", "illumination"])
def test_track_matches_oracle_on_wave_frames(ctx, case, mode):
    print(f"case track {case} mode {mode}", flush=True)
    d, gain, off = {"identical": ((0, 0), 1, 0), "integer": ((5, -3), 1, 0), "subpixel": ((2.3, -1.6), 1, 0),
                    "illumination": ((1.5, 2.25), 1.15, -12.0)}[case]
    tpl = wave_frame(W, H, seed=20)
    img = wave_frame(W, H, seed=20, d=d, gain=gain, offset=off)
    feats = feature_grid(W, H, 30, 19) + np.array([0.25, 0.5])
    for eps in (0.01, 1e-3):
        got = gpu_track(ctx, tpl, img, 3, feats, mode=mode, eps=eps)
        want = cpu_track(tpl, img, 3, feats, mode=mode, eps=eps)
        ok = compare(got, want, eps, f"{case} mode {mode} eps {eps}")
        assert ok.sum() > len(feats) // 2
        assert np.abs(got[2] - want[2]).max() <= 3
    if case == "identical":
        assert (got[0] == 0).all() and (got[2] == 3).all()


@pytest.mark.parametrize("mode", [0, 3], ids=["t", "t+gain+offset"])
def test_track_detected_features_on_moving_frames(ctx, mode):
    """The tracker's own workload: FAST features detected on a synthetic
    752x480 frame, tracked into the next frame, a crop of the same scene moved
    by a few pixels with fresh noise.  Some corners of this scene sit on long
    straight edges, where the alignment is ill-posed along the edge: such a
    track can slide, and fp32 and fp64 rounding may send it to different
    places.  The tracks compared are chosen from the template alone: every
    level's patch has a translational Hessian block whose smaller eigenvalue
    is at least 16 (intensity^2 per pixel^2, patch mean), eight times the
    gradient variance of the sigma = 2 noise.  On those, parameters must agree
    within the tracker tolerance; statuses must agree everywhere, and the sets
    of tracks that recover the true motion may differ in a few ill-posed ones."""
    print(f"case track detected mode {mode}", flush=True)
    scene = synth.frame(752 + 16, 480 + 16, seed=31, nshapes=120, sigma=0.0)
    rng = np.random.default_rng(31)
    tpl = np.ascontiguousarray(scene[8:8 + 480, 8:8 + 752])
    dx, dy = 3, -2
    img = np.ascontiguousarray(scene[8 - dy:8 - dy + 480, 8 - dx:8 - dx + 752])
    noise = lambda a: np.clip(a + rng.normal(0, 2.0, a.shape).round(), 0, 255).astype(np.uint8)  # noqa: E731
    tpl, img = noise(tpl), noise(img)
    slots, _ = oracle.detect_grid(tpl, 752, 3, 10, 9, 32)
    sel = slots["score"] > 0
    feats = np.stack([slots["x"][sel].astype(np.float64) * (1 << slots["level"][sel]),
                      slots["y"][sel].astype(np.float64) * (1 << slots["level"][sel])], axis=1)
    assert len(feats) > 150
    lam = min_eig_per_level(oracle.pyr_build(tpl, 752, 3), feats)
    posed = np.nan_to_num(lam, nan=-1.0).min(axis=1) >= 16.0
    got = gpu_track(ctx, tpl, img, 3, feats, mode=mode, eps=1e-3)
    want = cpu_track(tpl, img, 3, feats, mode=mode, eps=1e-3)
    ok = compare(got, want, 1e-3, f"detected mode {mode}", where=posed)
    assert ok.sum() > 0.7 * (want[1] == lk.TRACKED).sum()
    truth = lambda q: np.hypot(q[:, 0] - dx, q[:, 1] - dy) < 0.25  # noqa: E731
    good_cpu = (want[1] == lk.TRACKED) & truth(want[0])
    good_gpu = (got[1] == lk.TRACKED) & truth(got[0])
    assert good_cpu.sum() > 0.6 * len(feats)
    assert (good_cpu != good_gpu).sum() <= max(2, len(feats) // 50)


def test_track_many_features_sampled(ctx):
    """10,000 features on a 1920x1080, 4-level pair; every 37th is checked
    against the oracle, and all of them for finite output and a valid status."""
    print("case track many", flush=True)
    tpl = wave_frame(1920, 1080, seed=40)
    img = wave_frame(1920, 1080, seed=40, d=(-4.5, 6.25), gain=0.9, offset=10.0)
    rng = np.random.default_rng(40)
    feats = np.stack([rng.uniform(0, 1920, 10000), rng.uniform(0, 1080, 10000)], axis=1)
    qg, sg, ig = gpu_track(ctx, tpl, img, 4, feats, mode=3, eps=1e-3)
    assert np.isin(sg, [0, 1, 2, 3]).all() and np.isfinite(qg).all()
    idx = np.arange(0, 10000, 37)
    want = cpu_track(tpl, img, 4, feats[idx], mode=3, eps=1e-3)
    ok = compare((qg[idx], sg[idx], ig[idx]), want, 1e-3, "many features")
    assert ok.sum() > 0.8 * len(idx)
    assert (sg == 0).sum() > 8000


def test_track_degenerate_inputs(ctx):
    tpl = wave_frame(W, H, seed=50)
    img = wave_frame(W, H, seed=50, d=(6, 0))
    flat = np.full((H, W), 90, np.uint8)
    feats = np.array([[16.0, 120.0], [20.0, 120.0], [160.0, 221.0], [160.0, 219.0], [np.nan, 10.0],
                      [-3.0, 50.0], [1e9, 5.0], [W - 12.0, 120.0], [160.0, 120.0]])
    got = gpu_track(ctx, tpl, img, 3, feats, mode=0)
    want = cpu_track(tpl, img, 3, feats, mode=0)
    assert list(got[1]) == list(want[1])
    assert got[1][0] == lk.TEMPLATE_OUTSIDE and got[1][4] == lk.TEMPLATE_OUTSIDE
    # single level: the feature near the right edge is carried out of the frame
    got = gpu_track(ctx, tpl, img, 1, feats[7:8], mode=0)
    assert got[1][0] == lk.LOST_OUTSIDE
    got = gpu_track(ctx, flat, flat, 2, feats[8:9], mode=0)
    assert got[1][0] == lk.SINGULAR
    # an initial estimate far outside is lost at once; none at all keeps q
    q0 = np.array([[5000.0, 0.0, 0.0, 0.0]])
    got = gpu_track(ctx, tpl, img, 1, feats[8:9], q0=q0, mode=0)
    assert got[1][0] == lk.LOST_OUTSIDE and got[2][0] == 0
    q0 = np.array([[0.5, -0.25, 0.3, 7.0]])
    got = gpu_track(ctx, tpl, img, 2, feats[8:9], q0=q0, mode=0, max_iter=0)
    assert got[1][0] == lk.TRACKED and (got[0] == q0.astype(np.float32)).all() and got[2][0] == 0


def test_track_rejects_bad_arguments(ctx):
    tp = device_pyramid(ctx, wave_frame(64, 64, seed=1), 2)
    ip = device_pyramid(ctx, wave_frame(64, 64, seed=2), 2)
    other = device_pyramid(ctx, wave_frame(96, 64, seed=3), 2)
    f = torch.zeros((4, 2), dtype=torch.float32, device="cuda")
    q = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    base = dict(mode=3, max_iter=10, eps=0.01, nfeat=4)
    for bad in (dict(mode=4), dict(max_iter=-1), dict(max_iter=1001), dict(eps=-1.0), dict(eps=float("nan")),
                dict(nfeat=-1)):
        a = dict(base)
        a.update(bad)
        with pytest.raises(fastgrid.FastError) as ei:
            fastgrid.fast_track(ctx.handle, tp.planes, ip.planes, 2, f.data_ptr(), q.data_ptr(), st.data_ptr(), 0,
                                a["nfeat"], a["mode"], a["max_iter"], a["eps"])
        assert ei.value.code == fastgrid.FAST_EINVAL
    with pytest.raises(fastgrid.FastError) as ei:
        fastgrid.fast_track(ctx.handle, tp.planes, other.planes, 2, f.data_ptr(), q.data_ptr(), st.data_ptr(), 0,
                            4, 3, 10, 0.01)
    assert ei.value.code == fastgrid.FAST_EINVAL
    with pytest.raises(fastgrid.FastError) as ei:
        fastgrid.fast_track(ctx.handle, tp.planes, ip.planes, 2, f.data_ptr(), 0, st.data_ptr(), 0, 4, 3, 10, 0.01)
    assert ei.value.code == fastgrid.FAST_EINVAL
    with pytest.raises(fastgrid.FastError) as ei:   # misaligned estimates
        fastgrid.fast_track(ctx.handle, tp.planes, ip.planes, 2, f.data_ptr(), q.data_ptr() + 2, st.data_ptr(), 0,
                            4, 3, 10, 0.01)
    assert ei.value.code == fastgrid.FAST_EINVAL
    # nothing to track is not an error
    fastgrid.fast_track(ctx.handle, tp.planes, ip.planes, 2, 0, 0, 0, 0, 0, 3, 10, 0.01)
    assert ctypes.sizeof(fastgrid.fast_plane) == 24


@pytest.mark.parametrize("levels", [1, 2, 5])
def test_track_pyramid_depths(ctx, levels):
    """One level (16x16 patches only), two, and five (three 8x8 levels) on a
    1280x720 pair, with a motion each depth can reach."""
    print(f"case track depth {levels}", flush=True)
    d = {1: (1.25, -0.75), 2: (3.5, 2.25), 5: (-9.0, 7.5)}[levels]
    wl = (14.0, 40.0) if levels < 5 else (40.0, 90.0)
    tpl = wave_frame(1280, 720, seed=70 + levels, wavelengths=wl)
    margin = 12 << (levels - 1) if levels > 1 else 12
    feats = feature_grid(1280, 720, min(margin, 200), 53) + np.array([0.5, 0.25])
    for mode in (0, 3):
        # the full model also sees an illumination change
        gain, off = (1.05, -3.0) if mode else (1.0, 0.0)
        img = wave_frame(1280, 720, seed=70 + levels, d=d, gain=gain, offset=off, wavelengths=wl)
        got = gpu_track(ctx, tpl, img, levels, feats, mode=mode, eps=1e-3)
        want = cpu_track(tpl, img, levels, feats, mode=mode, eps=1e-3)
        ok = compare(got, want, 1e-3, f"depth {levels} mode {mode}")
        assert ok.sum() > len(feats) // 2


def test_track_4k_frame(ctx):
    """Features across a 4096x2160, 5-level pair (the largest stream frame)."""
    print("case track 4k", flush=True)
    tpl = wave_frame(4096, 2160, seed=80, wavelengths=(30.0, 80.0))
    img = wave_frame(4096, 2160, seed=80, d=(6.5, -4.25), wavelengths=(30.0, 80.0))
    rng = np.random.default_rng(80)
    feats = np.stack([rng.uniform(0, 4096, 400), rng.uniform(0, 2160, 400)], axis=1)
    got = gpu_track(ctx, tpl, img, 5, feats, mode=3, eps=1e-3)
    want = cpu_track(tpl, img, 5, feats, mode=3, eps=1e-3)
    ok = compare(got, want, 1e-3, "4k")
    assert ok.sum() > 250


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_track_fixed_step_count_matches_tightly(ctx, mode):
    """With eps = 0 no level stops early: both sides take exactly max_iter
    Gauss-Newton steps per level, so iteration counts agree exactly and the
    estimates differ only by fp32 rounding."""
    print(f"case track fixed steps mode {mode}", flush=True)
    tpl = wave_frame(W, H, seed=90)
    img = wave_frame(W, H, seed=90, d=(1.75, -2.5), gain=1.1 if mode else 1.0, offset=-6.0 if mode else 0.0)
    feats = feature_grid(W, H, 30, 23) + np.array([0.375, 0.625])
    got = gpu_track(ctx, tpl, img, 3, feats, mode=mode, max_iter=6, eps=0.0)
    want = cpu_track(tpl, img, 3, feats, mode=mode, max_iter=6, eps=0.0)
    assert (got[1] == want[1]).all()
    ok = want[1] == lk.TRACKED
    assert ok.sum() > len(feats) // 2
    assert (got[2][ok] == 18).all() and (want[2][ok] == 18).all()
    # every tracked feature: only fp32 rounding separates the two sides
    assert np.abs(got[0][ok, :2] - want[0][ok, :2]).max() < 2e-3
    assert np.abs(got[0][ok, 2] - want[0][ok, 2]).max() < 1e-3
    assert np.abs(got[0][ok, 3] - want[0][ok, 3]).max() < 0.1
