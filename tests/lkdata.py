"""Seeded synthetic frames for the Lucas-Kanade tracker tests: a smooth
intensity field made of a few plane waves, sampled on the pixel grid and
rounded to uint8.  Shifting the field by d before sampling gives a frame whose
true motion is exactly d, and a gain/offset applied before the rounding gives
a known illumination change.  No tracker arithmetic lives here."""
from __future__ import annotations

import numpy as np


def wave_frame(w: int, h: int, seed: int, d=(0.0, 0.0), gain: float = 1.0, offset: float = 0.0,
               wavelengths=(14.0, 40.0), waves: int = 6) -> np.ndarray:
    """I(x, y) = round(gain * f(x - dx, y - dy) + offset), f = 128 + a sum of
    `waves` plane waves with seeded directions, phases and wavelengths."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    x -= d[0]
    y -= d[1]
    f = np.full_like(x, 128.0)
    for _ in range(waves):
        wl = rng.uniform(*wavelengths)
        th = rng.uniform(0.0, np.pi)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        amp = rng.uniform(8.0, 13.0)
        f += amp * np.sin(2.0 * np.pi / wl * (np.cos(th) * x + np.sin(th) * y) + ph)
    return np.clip(np.floor(gain * f + offset + 0.5), 0, 255).astype(np.uint8)


def feature_grid(w: int, h: int, margin: int, step: int) -> np.ndarray:
    """Level-0 feature positions on a regular grid inside a margin."""
    ys, xs = np.mgrid[margin:h - margin:step, margin:w - margin:step]
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.float64)
