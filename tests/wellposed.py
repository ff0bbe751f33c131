"""Which tracks have a unique answer, judged from the template alone.

The translation part of a Lucas-Kanade alignment (Section II-E) is well posed
where the template patch has texture in two directions: the 2x2 translational
block of the Hessian, sum over the patch of [Tx^2, Tx Ty; Tx Ty, Ty^2], has a
large smaller eigenvalue.  On a straight edge that eigenvalue is near zero,
the alignment may slide along the edge, and fp32 and fp64 rounding can then
send a track to different places.  The tracker tests compare parameters on the
tracks this module selects, without looking at where any tracker ended up.

The patch follows the tracker's reading of the section: side 16 on levels 0-1
and 8 above, at p + (i - S/2, j - S/2) around the level position p = f / 2^k,
bilinear samples, central-difference gradients.  This is a test-side
restatement for selection only; no expected value comes from it."""
from __future__ import annotations

import numpy as np
from scipy.ndimage import map_coordinates


def _side(k: int) -> int:
    return 16 if k < 2 else 8


def min_eig_per_level(tpl_levels, feats) -> np.ndarray:
    """N x L array: the smaller eigenvalue of the mean translational Hessian
    block of each feature's template patch on each level (NaN where the patch
    with its 1-pixel gradient margin does not fit the level)."""
    feats = np.asarray(feats, dtype=np.float64).reshape(-1, 2)
    out = np.full((len(feats), len(tpl_levels)), np.nan)
    for k, lv in enumerate(tpl_levels):
        arr, w = lv if isinstance(lv, tuple) else (lv, lv.shape[1])
        img = np.asarray(arr[:, :w], dtype=np.float64)
        h = img.shape[0]
        s = _side(k)
        off = np.arange(s, dtype=np.float64) - s // 2
        for i, f in enumerate(feats):
            if not np.all(np.isfinite(f)):
                continue
            p = f / (1 << k)
            xs = p[0] + off
            ys = p[1] + off
            if xs[0] - 1 < 0 or ys[0] - 1 < 0 or xs[-1] + 1 >= w - 1 or ys[-1] + 1 >= h - 1:
                continue
            yy, xx = np.meshgrid(ys, xs, indexing="ij")
            samp = lambda dx, dy: map_coordinates(img, [yy + dy, xx + dx], order=1)  # noqa: E731
            gx = (samp(1, 0) - samp(-1, 0)) / 2
            gy = (samp(0, 1) - samp(0, -1)) / 2
            a, b, c = (gx * gx).mean(), (gx * gy).mean(), (gy * gy).mean()
            out[i, k] = (a + c) / 2 - np.sqrt(((a - c) / 2) ** 2 + b * b)
    return out


def well_posed(tpl_levels, feats, threshold: float) -> np.ndarray:
    """True where every level's patch fits and its smaller eigenvalue is at
    least `threshold` (intensity^2 per pixel^2, averaged over the patch)."""
    lam = min_eig_per_level(tpl_levels, feats)
    return np.all(np.isfinite(lam), axis=1) & (np.nan_to_num(lam, nan=-1.0).min(axis=1) >= threshold)
