"""An independent, vectorised NumPy restatement of the detector, for pinning the
C oracle by brute force on tiny images.

It is deliberately built differently from the oracle so that one mistake is
unlikely to appear in both:

* the circle is derived, not tabulated: the 16 offsets are the integer points
  whose Euclidean distance rounds to 3 (the radius-3 Bresenham circle of
  Section II-D), ordered by angle;
* the arc decision is the longest circular run of a boolean sequence;
* NMS compares each pixel with its 8 shifted neighbours through one integer
  rank that folds the row-major tie-break into the score;
* cell selection sorts every survivor of every level by
  (cell, -score, level, index) and keeps the first per cell;
* the arc score (SAD-A) marks a circle point as on an arc when the maximal
  circular run through it is at least n long (runs measured forwards and
  backwards from the point), and the maximum-threshold score (MT) searches the
  thresholds t' = t..255 with the plain segment test.
"""
from __future__ import annotations

import math

import numpy as np


def circle_offsets() -> list[tuple[int, int]]:
    pts = [(dx, dy) for dy in range(-3, 4) for dx in range(-3, 4)
           if round(math.hypot(dx, dy)) == 3]
    pts.sort(key=lambda p: math.atan2(p[1], p[0]))
    assert len(pts) == 16
    return pts


def longest_circular_run(bits: np.ndarray) -> np.ndarray:
    """bits: (..., 16) bool.  Returns the longest run of True, wrapping around."""
    b = np.concatenate([bits, bits], axis=-1).astype(np.int32)
    run = np.zeros(b.shape[:-1], np.int32)
    best = np.zeros(b.shape[:-1], np.int32)
    for i in range(b.shape[-1]):
        run = (run + 1) * b[..., i]
        best = np.maximum(best, run)
    return np.minimum(best, 16)


def run_through(bits: np.ndarray) -> np.ndarray:
    """bits: (..., 16) bool.  Length of the maximal circular run of True through
    each position (0 where False, 16 when all are True)."""
    b = bits.astype(np.int32)
    fwd = np.zeros_like(b)
    bwd = np.zeros_like(b)
    for i in range(16):
        # run length starting at i going forwards, and ending at i going backwards
        f = np.zeros(b.shape[:-1], np.int32)
        alive = np.ones(b.shape[:-1], bool)
        for j in range(16):
            alive &= b[..., (i + j) % 16] == 1
            f += alive
        fwd[..., i] = f
        g = np.zeros(b.shape[:-1], np.int32)
        alive = np.ones(b.shape[:-1], bool)
        for j in range(16):
            alive &= b[..., (i - j) % 16] == 1
            g += alive
        bwd[..., i] = g
    return np.where(b == 1, np.minimum(fwd + bwd - 1, 16), 0)


def pyramid(img: np.ndarray, levels: int) -> list[np.ndarray]:
    out = [img.astype(np.int64)]
    for _ in range(1, levels):
        prev = out[-1]
        h, w = prev.shape[0] // 2, prev.shape[1] // 2
        blk = prev[:2 * h, :2 * w].reshape(h, 2, w, 2).sum(axis=(1, 3))
        out.append((blk + 2) // 4)
    return [p.astype(np.uint8) for p in out]


def score_map(img: np.ndarray, t: int, n: int, kind: int = 0) -> np.ndarray:
    """kind 0: whole-circle sums; 1: sums over the points on an arc of >= n;
    2: 1 + the largest threshold t' >= t at which the segment test passes."""
    I = img.astype(np.int64)
    h, w = I.shape
    out = np.zeros((h, w), np.int64)
    if h < 7 or w < 7:
        return out
    c = I[3:h - 3, 3:w - 3]
    ring = np.stack([I[3 + dy:h - 3 + dy, 3 + dx:w - 3 + dx] for dx, dy in circle_offsets()],
                    axis=-1)
    diff = ring - c[..., None]

    def passes(tt):
        return (longest_circular_run(diff > tt) >= n) | (longest_circular_run(diff < -tt) >= n)

    corner = passes(t)
    bright = diff > t
    dark = diff < -t
    if kind == 2:
        best = np.full(c.shape, -1, np.int64)
        for tt in range(t, 256):
            best = np.where(passes(tt), tt, best)
        out[3:h - 3, 3:w - 3] = np.where(corner, best + 1, 0)
        return out
    if kind == 1:
        bright = bright & (run_through(bright) >= n)
        dark = dark & (run_through(dark) >= n)
    sb = np.where(bright, diff - t, 0).sum(-1)
    sd = np.where(dark, -diff - t, 0).sum(-1)
    out[3:h - 3, 3:w - 3] = np.where(corner, np.maximum(sb, sd), 0)
    return out


def nms(score: np.ndarray, r: int = 1) -> np.ndarray:
    h, w = score.shape
    idx = np.arange(h * w, dtype=np.int64).reshape(h, w)
    rank = score.astype(np.int64) * (h * w) + (h * w - 1 - idx)
    pad = np.full((h + 2 * r, w + 2 * r), -1, np.int64)
    pad[r:r + h, r:r + w] = rank
    keep = score > 0
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dx or dy:
                keep &= rank > pad[r + dy:r + dy + h, r + dx:r + dx + w]
    return keep


def detect_grid(img: np.ndarray, levels: int, t: int, n: int, cell: int, kind: int = 0,
                radius: int = 1):
    """img: (H, W) uint8 without padding.  Returns (slots list of tuples, planes)."""
    planes = pyramid(img, levels)
    H, W = img.shape
    gw, gh = -(-W // cell), -(-H // cell)
    cands = []
    for k, P in enumerate(planes):
        s = score_map(P, t, n, kind)
        keep = nms(s, radius)
        ys, xs = np.nonzero(keep)
        for y, x in zip(ys.tolist(), xs.tolist()):
            cid = ((y << k) // cell) * gw + ((x << k) // cell)
            cands.append((cid, -int(s[y, x]), k, y * P.shape[1] + x, x, y))
    cands.sort()
    slots = [(0xFFFF, 0xFFFF, 0, 0xFF)] * (gw * gh)
    seen = set()
    for cid, ns, k, _, x, y in cands:
        if cid not in seen:
            seen.add(cid)
            slots[cid] = (x, y, -ns, k)
    return slots, planes
