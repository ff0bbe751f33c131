"""Detect-and-track front end of one camera: the paper's tracking workload
(Section III-D, the feature tracker evaluation).  FAST features (one per grid
cell) are tracked frame to frame by the Lucas-Kanade tracker, and detection
runs again whenever the number of live tracks falls below a fraction (30%) of
the target count.  Detection uses the second of the three corner scores that
Section II-D lists, the arc sum SAD-A, as the evaluation does.

Every frame: upload into one of two device pyramids, build its levels,
track the live features from the previous frame's pyramid, drop the lost
ones, and if fewer than ``redetect_frac * target`` remain, detect on the new
frame and add the strongest cell winners whose cells hold no live track
(strongest first; equal scores by cell index) up to the target.  All image
work runs in the HIP library.  `Frontend` keeps one camera's short feature
list on the host; `MultiFrontend` runs the same loop for many cameras with
every feature list in device memory (fast_frontend_step), so a step needs no
host round trip.
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np

from . import fastgrid


def cell_of(xy: np.ndarray, cell: int, gw: int) -> np.ndarray:
    """Row-major grid cell index of level-0 positions."""
    cx = np.floor(xy[:, 0] / cell).astype(np.int64)
    cy = np.floor(xy[:, 1] / cell).astype(np.int64)
    return cy * gw + cx


def pick_new(slots: np.ndarray, taken: np.ndarray, count: int) -> np.ndarray:
    """The `count` strongest cell winners outside the `taken` cells, as level-0
    (x, y); equal scores keep the lower cell index first."""
    flat = slots.reshape(-1)
    free = (flat["score"] > 0) & ~taken
    idx = np.nonzero(free)[0]
    order = np.lexsort((idx, -flat["score"][idx].astype(np.int64)))
    idx = idx[order][:max(count, 0)]
    lv = flat["level"][idx].astype(np.int64)
    return np.stack([(flat["x"][idx].astype(np.int64) << lv).astype(np.float64),
                     (flat["y"][idx].astype(np.int64) << lv).astype(np.float64)], axis=1)


class Frontend:
    def __init__(self, ctx: fastgrid.Context, width: int, height: int, levels: int = 3, t: int = 10,
                 n: int = 9, cell: int = 32, target: int = 100, redetect_frac: float = 0.3,
                 mode: int = fastgrid.FAST_TRACK_GAIN | fastgrid.FAST_TRACK_OFFSET, max_iter: int = 30,
                 eps: float = 0.01, score: int = fastgrid.FAST_SCORE_SADA):
        import torch
        self.ctx, self.w, self.h, self.levels = ctx, width, height, levels
        self.t, self.n, self.cell = t, n, cell
        self.target, self.redetect_frac = target, redetect_frac
        self.mode, self.max_iter, self.eps = mode, max_iter, eps
        self.score = score
        self.pyr = [fastgrid.Pyramid(width, height, levels) for _ in range(2)]
        self.grid = fastgrid.Grid(width, height, cell)
        self.gw = (width + cell - 1) // cell
        self.gh = (height + cell - 1) // cell
        self.cur = 0
        self.frames = 0
        self.feats = np.zeros((0, 2))     # live features, level-0 positions in the current frame
        self.last_q = np.zeros((0, 4))    # the last tracking call's estimates and statuses
        self.last_status = np.zeros(0, dtype=np.int32)
        self.f_dev = torch.zeros((target, 2), dtype=torch.float32, device="cuda")
        self.q_dev = torch.zeros((target, 4), dtype=torch.float32, device="cuda")
        self.s_dev = torch.zeros(target, dtype=torch.int32, device="cuda")

    def step(self, frame: np.ndarray) -> dict:
        """Process one frame (host uint8, height x >= width); returns what
        happened: live tracks before and after, whether detection ran."""
        import torch
        t0 = time.perf_counter()
        prev, cur = self.pyr[self.cur], self.pyr[1 - self.cur]
        cur.upload(frame)
        self.ctx.pyr_build(cur)
        tracked = 0
        if self.frames > 0 and len(self.feats):
            k = len(self.feats)
            self.f_dev[:k].copy_(torch.from_numpy(self.feats.astype(np.float32)))
            self.q_dev[:k].zero_()
            self.ctx.track(prev, cur, self.f_dev[:k], self.q_dev[:k], self.s_dev[:k], mode=self.mode,
                           max_iter=self.max_iter, eps=self.eps)
            q = self.q_dev[:k].cpu().numpy().astype(np.float64)
            st = self.s_dev[:k].cpu().numpy()
            keep = st == fastgrid.FAST_TRACK_OK
            self.last_q, self.last_status = q, st
            self.feats = self.feats[keep] + q[keep, :2]
            tracked = int(keep.sum())
        redetect = len(self.feats) < self.redetect_frac * self.target
        if redetect:
            self.ctx.detect(cur, self.t, self.n, self.cell, self.grid, score=self.score)
            slots = self.grid.fetch()
            taken = np.zeros(self.gw * self.gh, dtype=bool)
            if len(self.feats):
                c = cell_of(self.feats, self.cell, self.gw)
                taken[c[(c >= 0) & (c < len(taken))]] = True
            new = pick_new(slots, taken, self.target - len(self.feats))
            self.feats = np.concatenate([self.feats, new]) if len(self.feats) else new
        self.cur = 1 - self.cur
        self.frames += 1
        return {"tracked": tracked, "redetect": bool(redetect), "live": len(self.feats),
                "ms": (time.perf_counter() - t0) * 1e3}


def redetect_below(target: int, frac: float) -> int:
    """The live count below which the loop re-detects: live < frac * target
    exactly when live < this (for integer live)."""
    return max(0, min(target, math.ceil(frac * target)))


class _StreamState:
    """Device state of one stream: two pyramids (previous and current), this
    frame's cell winners, and the feature list with its scratch."""

    def __init__(self, width, height, levels, t, n, cell, target, below, device="cuda"):
        import torch
        self.w, self.h, self.levels, self.t, self.n, self.cell = width, height, levels, t, n, cell
        self.target, self.below = target, below
        self.pyr = [fastgrid.Pyramid(width, height, levels, device) for _ in range(2)]
        self.grid = fastgrid.Grid(width, height, cell, device)
        self.feats = torch.zeros((target, 2), dtype=torch.float32, device=device)
        self.q = torch.zeros((target, 4), dtype=torch.float32, device=device)
        self.status = torch.zeros(target, dtype=torch.int32, device=device)
        self.count = torch.zeros(1, dtype=torch.int32, device=device)
        self.info = torch.zeros(4, dtype=torch.int32, device=device)
        self.cur = 0            # index of the pyramid the next frame goes into
        self.frames = 0


class MultiFrontend:
    """The detect-and-track loop of many camera streams, with every feature
    list resident in device memory.  A step takes one frame from each of any
    subset of the streams: one batched detection (SAD-A, fast_submit) on the
    new frames, then one fast_frontend_step that tracks every stream's live
    features from its previous frame and re-detects where too few remain.
    The host moves no feature data; info() and features() read a stream's
    results when asked."""

    def __init__(self, ctx: fastgrid.Context, shapes, targets, redetect_fracs,
                 mode: int = fastgrid.FAST_TRACK_GAIN | fastgrid.FAST_TRACK_OFFSET, max_iter: int = 30,
                 eps: float = 0.01, score: int = fastgrid.FAST_SCORE_SADA):
        self.ctx, self.mode, self.max_iter, self.eps, self.score = ctx, mode, max_iter, eps, score
        self.streams = [_StreamState(w, h, L, t, n, c, tg, redetect_below(tg, fr))
                        for (w, h, L, t, n, c), tg, fr in zip(shapes, targets, redetect_fracs)]

    def _job(self, i: int, prev) -> fastgrid.fast_frontend_job:
        st = self.streams[i]
        cur = st.pyr[st.cur]
        P = ctypes.POINTER(fastgrid.fast_plane)
        return fastgrid.fast_frontend_job(
            ctypes.cast(prev.planes, P) if prev is not None else None, ctypes.cast(cur.planes, P),
            st.levels, st.grid.ptr, st.cell, st.target, st.below, st.feats.data_ptr(), st.count.data_ptr(),
            st.q.data_ptr(), st.status.data_ptr(), st.info.data_ptr())

    def step(self, frames: dict, stream=None) -> int:
        """frames: {stream index: host uint8 frame (height x >= width)}.
        Enqueues the step; returns the front-end ticket."""
        idx = sorted(frames)
        for i in idx:
            st = self.streams[i]
            st.pyr[st.cur].upload(frames[i])
        det = fastgrid.Context.make_jobs(
            (self.streams[i].pyr[self.streams[i].cur], self.streams[i].t, self.streams[i].n,
             self.streams[i].cell, self.streams[i].grid, self.score) for i in idx)
        self.ctx.submit(det, stream)
        jobs = (fastgrid.fast_frontend_job * len(idx))()
        for k, i in enumerate(idx):
            st = self.streams[i]
            jobs[k] = self._job(i, st.pyr[1 - st.cur] if st.frames > 0 else None)
        tk = fastgrid.fast_frontend_step(self.ctx.handle, jobs, len(idx), self.mode, self.max_iter, self.eps,
                                         stream)
        for i in idx:
            st = self.streams[i]
            st.cur = 1 - st.cur
            st.frames += 1
        return tk

    def info(self, i: int) -> tuple:
        """(tracked, re-detected, live) of stream i's last step."""
        v = self.streams[i].info.cpu().numpy()
        return int(v[0]), bool(v[1]), int(v[2])

    def features(self, i: int) -> np.ndarray:
        """Stream i's live features (level-0 positions in its last frame)."""
        st = self.streams[i]
        n = int(st.count.cpu().numpy()[0])
        return st.feats[:n].cpu().numpy().astype(np.float64)
