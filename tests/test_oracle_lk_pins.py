"""Pins of the Lucas-Kanade tracker oracle (Section II-E) against facts that do
not come from the oracle itself: frames with an exactly known motion and
illumination change, one Gauss-Newton step rebuilt from a library bilinear
interpolator and a library least-squares solve, the forward/backward symmetry
of tracking, and the degenerate cases (flat patches, borders, zero
iterations)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle import lk
from lkdata import feature_grid, wave_frame

W, H = 320, 240
MODES = [0, lk.GAIN, lk.OFFSET, lk.GAIN | lk.OFFSET]
MODE_IDS = ["t", "t+gain", "t+offset", "t+gain+offset"]


def pyr(img, levels):
    return oracle.pyr_build(img, img.shape[1], levels)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_identical_frames_stay_put(mode):
    """Template and image equal: every residual is exactly zero, so one
    iteration per level returns the zero parameters exactly."""
    img = wave_frame(W, H, seed=1)
    feats = feature_grid(W, H, 40, 37)
    q, st, it = lk.track(pyr(img, 3), pyr(img, 3), feats, mode=mode)
    assert (st == lk.TRACKED).all()
    assert (q == 0).all()
    assert (it == 3).all()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("d", [(3, -2), (-5, 4), (7, 6)])
def test_integer_shift_is_recovered(d, mode):
    """I(x) = T(x - d) exactly (an integer shift of the sampled field): the
    track converges to t = d, with no illumination change."""
    tpl = wave_frame(W, H, seed=2)
    img = wave_frame(W, H, seed=2, d=d)
    feats = feature_grid(W, H, 48, 41)
    q, st, _ = lk.track(pyr(tpl, 3), pyr(img, 3), feats, mode=mode, eps=1e-4)
    assert (st == lk.TRACKED).all()
    assert np.abs(q[:, 0] - d[0]).max() < 0.01
    assert np.abs(q[:, 1] - d[1]).max() < 0.01
    assert np.abs(q[:, 2]).max() < 2e-3 and np.abs(q[:, 3]).max() < 0.3


@pytest.mark.parametrize("d", [(2.3, -1.6), (-0.45, 0.8), (4.75, 3.1)])
def test_subpixel_shift_is_recovered(d):
    """The field shifted by a fractional d before sampling: the only error
    left is the uint8 rounding of both frames."""
    tpl = wave_frame(W, H, seed=3)
    img = wave_frame(W, H, seed=3, d=d)
    feats = feature_grid(W, H, 48, 41)
    q, st, _ = lk.track(pyr(tpl, 3), pyr(img, 3), feats, mode=0, eps=1e-4)
    assert (st == lk.TRACKED).all()
    err = np.hypot(q[:, 0] - d[0], q[:, 1] - d[1])
    assert err.max() < 0.05 and err.mean() < 0.02


def test_gain_and_offset_are_recovered():
    """I = 1.15 T(x - d) - 12 before rounding: the full model recovers alpha =
    0.15, beta = -12 and d."""
    d = (1.5, 2.25)
    tpl = wave_frame(W, H, seed=4)
    img = wave_frame(W, H, seed=4, d=d, gain=1.15, offset=-12.0)
    feats = feature_grid(W, H, 48, 41)
    q, st, _ = lk.track(pyr(tpl, 3), pyr(img, 3), feats, mode=lk.GAIN | lk.OFFSET, eps=1e-4)
    assert (st == lk.TRACKED).all()
    # at a half-pixel shift bilinear interpolation of the 14-40 px waves is
    # biased by up to ~0.1 px on low-contrast patches
    err = np.hypot(q[:, 0] - d[0], q[:, 1] - d[1])
    assert err.max() < 0.15 and err.mean() < 0.05
    assert np.abs(q[:, 2] - 0.15).max() < 0.02
    # alpha and beta trade off through the patch mean; the pair must predict I
    assert np.abs(q[:, 3] + 12.0).max() < 3.0
    assert np.abs(q[:, 2] * 128 + q[:, 3] - (0.15 * 128 - 12.0)).max() < 0.5


def test_offset_alone_and_gain_alone():
    d = (-1.25, 0.5)
    tpl = wave_frame(W, H, seed=5)
    feats = feature_grid(W, H, 48, 41)
    img = wave_frame(W, H, seed=5, d=d, offset=20.0)
    q, st, _ = lk.track(pyr(tpl, 3), pyr(img, 3), feats, mode=lk.OFFSET, eps=1e-4)
    assert (st == lk.TRACKED).all()
    assert np.abs(q[:, 3] - 20.0).max() < 0.6 and (q[:, 2] == 0).all()
    assert np.abs(q[:, 0] - d[0]).max() < 0.15
    img = wave_frame(W, H, seed=5, d=d, gain=0.8)
    q, st, _ = lk.track(pyr(tpl, 3), pyr(img, 3), feats, mode=lk.GAIN, eps=1e-4)
    assert (st == lk.TRACKED).all()
    assert np.abs(q[:, 2] + 0.2).max() < 0.01 and (q[:, 3] == 0).all()
    assert np.abs(q[:, 1] - d[1]).max() < 0.15


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_one_step_is_the_linear_least_squares_solution(mode):
    """One iteration on one level equals the least-squares solution of the
    linearised problem of Section II-E, rebuilt here from scipy's bilinear
    interpolator and numpy's lstsq: rows U(x) = [(1+a) Tx, (1+a) Ty, T, 1] over
    the 16x16 patch at p + (i - 8, j - 8), right-hand side I(x + t) - (1+a) T - b;
    then t <- t - dt, a <- a + da, b <- b + db."""
    tpl = wave_frame(W, H, seed=6)
    img = wave_frame(W, H, seed=6, d=(1.3, -0.7), gain=1.1, offset=4.0)
    q0 = np.array([0.4, -0.3, 0.1, 3.0])
    for p in [(40.25, 37.5), (161.0, 120.75), (250.6, 190.1)]:
        q, st, it = lk.track([tpl], [img], [p], q0=q0[None], mode=mode, patch=[16], max_iter=1, eps=0.0)
        assert st[0] == lk.TRACKED and it[0] == 1
        jj, ii = np.mgrid[0:16, 0:16].astype(np.float64)
        xs, ys = p[0] + ii - 8, p[1] + jj - 8

        def interp(a, x, y):
            return ndimage.map_coordinates(a.astype(np.float64), [y.ravel(), x.ravel()], order=1)

        t = interp(tpl, xs, ys)
        tx = (interp(tpl, xs + 1, ys) - interp(tpl, xs - 1, ys)) / 2
        ty = (interp(tpl, xs, ys + 1) - interp(tpl, xs, ys - 1)) / 2
        g = 1 + q0[2]
        cols = [g * tx, g * ty]
        if mode & lk.GAIN:
            cols.append(t)
        if mode & lk.OFFSET:
            cols.append(np.ones_like(t))
        A = np.stack(cols, axis=1)
        r = interp(img, xs + q0[0], ys + q0[1]) - g * t - q0[3]
        dq, *_ = np.linalg.lstsq(A, r, rcond=None)
        want = q0.copy()
        want[0] -= dq[0]
        want[1] -= dq[1]
        k = 2
        if mode & lk.GAIN:
            want[2] += dq[k]
            k += 1
        if mode & lk.OFFSET:
            want[3] += dq[k]
        np.testing.assert_allclose(q[0], want, rtol=0, atol=1e-9)


def test_tracking_back_returns_the_opposite_motion():
    """Tracking T -> I from p and then I -> T from p + t lands on -t."""
    d = (2.6, -3.4)
    tpl = wave_frame(W, H, seed=7)
    img = wave_frame(W, H, seed=7, d=d)
    feats = feature_grid(W, H, 56, 43)
    q, st, _ = lk.track(pyr(tpl, 3), pyr(img, 3), feats, mode=0, eps=1e-5)
    assert (st == lk.TRACKED).all()
    back, st2, _ = lk.track(pyr(img, 3), pyr(tpl, 3), feats + q[:, :2], mode=0, eps=1e-5)
    assert (st2 == lk.TRACKED).all()
    assert np.abs(back[:, :2] + q[:, :2]).max() < 0.03


def test_coarse_to_fine_reaches_a_large_shift():
    """A 13 x -11 pixel motion of a long-wavelength field: four levels carry the
    estimate down (doubling it per level) to the exact shift."""
    d = (13, -11)
    tpl = wave_frame(W, H, seed=8, wavelengths=(40.0, 90.0))
    img = wave_frame(W, H, seed=8, d=d, wavelengths=(40.0, 90.0))
    feats = feature_grid(W, H, 100, 40)
    q, st, _ = lk.track(pyr(tpl, 4), pyr(img, 4), feats, mode=0, eps=1e-4, max_iter=50)
    assert (st == lk.TRACKED).all()
    assert np.abs(q[:, 0] - d[0]).max() < 0.01 and np.abs(q[:, 1] - d[1]).max() < 0.01
    # two iterations per level suffice only when each level starts from the
    # doubled estimate of the level above
    q, st, it = lk.track(pyr(tpl, 4), pyr(img, 4), feats, mode=0, eps=1e-4, max_iter=2)
    assert (st == lk.TRACKED).all() and it.max() <= 8
    assert np.abs(q[:, 0] - d[0]).max() < 0.01 and np.abs(q[:, 1] - d[1]).max() < 0.01


def test_degenerate_cases():
    tpl = wave_frame(W, H, seed=9)
    # a template patch that does not fit at the coarsest level
    q, st, it = lk.track(pyr(tpl, 3), pyr(tpl, 3), [(16.0, 120.0)])
    assert st[0] == lk.TEMPLATE_OUTSIDE and it[0] == 0
    q, st, it = lk.track(pyr(tpl, 3), pyr(tpl, 3), [(20.0, 120.0)])   # just fits (level 2: x = 5)
    assert st[0] == lk.TRACKED
    q, st, it = lk.track(pyr(tpl, 3), pyr(tpl, 3), [(160.0, 221.0)])   # level 2: y + 4 = 59.25 >= 59
    assert st[0] == lk.TEMPLATE_OUTSIDE and it[0] == 0
    q, st, it = lk.track(pyr(tpl, 3), pyr(tpl, 3), [(160.0, 219.0)])   # level 2: y + 4 = 58.75
    assert st[0] == lk.TRACKED
    # a flat patch has no gradient: singular translation block
    flat = np.full((H, W), 90, np.uint8)
    q, st, _ = lk.track(pyr(flat, 2), pyr(flat, 2), [(160.0, 120.0)], mode=0)
    assert st[0] == lk.SINGULAR
    # gain and offset on a flat patch: the T and 1 columns are parallel
    ramp = np.tile(np.arange(W, dtype=np.uint8) // 2, (H, 1))
    q, st, _ = lk.track([ramp], [ramp], [(100.0, 100.0)], mode=lk.GAIN | lk.OFFSET, patch=[16])
    assert st[0] == lk.SINGULAR      # a pure x ramp: Ty = 0
    # motion that carries the patch out of the frame
    img = wave_frame(W, H, seed=9, d=(6, 0))
    q, st, _ = lk.track([tpl], [img], [(W - 12.0, 120.0)], mode=0, patch=[16])
    assert st[0] == lk.LOST_OUTSIDE


def test_iteration_cap_and_untouched_parameters():
    tpl = wave_frame(W, H, seed=10)
    img = wave_frame(W, H, seed=10, d=(1.7, 0.9))
    q0 = np.array([[0.0, 0.0, 0.3, 7.0]])
    q, st, it = lk.track([tpl], [img], [(150.0, 110.0)], q0=q0, mode=0, patch=[16], max_iter=0)
    assert st[0] == lk.TRACKED and it[0] == 0 and (q == q0).all()
    q, st, it = lk.track([tpl], [img], [(150.0, 110.0)], q0=q0, mode=0, patch=[16], max_iter=1)
    assert it[0] == 1 and q[0, 2] == 0.3 and q[0, 3] == 7.0
    q, st, it = lk.track([tpl], [img], [(150.0, 110.0)], mode=0, patch=[16], max_iter=100, eps=1e-6)
    assert 1 < it[0] < 100
