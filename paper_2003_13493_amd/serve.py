"""Continuous-batching server for simulated camera streams.

Each resident camera stream keeps, in HBM:
  * a pool of its frames (level 0 planes), so arrivals need no PCIe upload;
  * a ring of request slots: pyramid levels 1.. and an output grid per slot;
  * pinned host buffers that receive each slot's cell results.

With upload=True the frames stay in pinned host memory instead and every
request first copies its frame into the slot's own level-0 plane (host to
device, on the request's stream): the PCIe-inclusive variant.

Admission by free HBM: a stream becomes resident only while its resident
bytes fit in the budget (free memory at start-up minus a reserve, or an
explicit budget) next to the streams already resident, and, for a budget taken
from free memory, in what the device still has free.  Streams that do not fit
wait in a queue.  A stream may leave during a run: it stops sending frames,
and once its last request has completed its device buffers are released and
waiting streams are admitted, in queue order, as they fit.  Frames that a
waiting stream sends are refused (counted, not served).

With frontend=FrontendParams(...) every stream runs the detect-and-track loop
of the paper's tracker evaluation instead of detection alone: its frames are
served strictly in order (one in flight per stream), each batch is one
detection submission (SAD-A) followed by one fast_frontend_step that tracks
every stream's features from its previous frame and re-detects where too few
remain, with the feature lists resident in device memory; only the 16-byte
step summary (tracked, re-detected, live) is copied to the host.

Frames arrive by per-stream Poisson processes.  The loop keeps up to K batches
in flight on K HIP streams; whenever a launch slot is free, every frame that
has arrived and holds a request slot joins the next batch (up to a batch
limit), so frames that arrive while others run are admitted as slots free up
and their work overlaps on the device.  A batch is one `fast_submit`
(persistent launch over a device work queue) followed by the copy of its
results to the host; its ticket is polled, and the frame latency is the
poll-observed completion time minus the arrival time.  Python's garbage
collector is paused while the loop runs, and the loop allocates nothing per
batch (job arrays and completion events are made once per launch lane).
"""
from __future__ import annotations

import collections
import ctypes
import gc
import heapq
import time
from dataclasses import dataclass, field

import numpy as np

from . import fastgrid


# ---------------------------------------------------------------- host logic

def plan_admission(stream_bytes: list[int], budget: int) -> tuple[list[int], list[int]]:
    """Admit streams in order while their resident bytes fit in the budget."""
    admitted, rejected, used = [], [], 0
    for i, b in enumerate(stream_bytes):
        if used + b <= budget:
            admitted.append(i)
            used += b
        else:
            rejected.append(i)
    return admitted, rejected


def admit_waiting(waiting: list[int], need: list[int], room: int) -> tuple[list[int], list[int]]:
    """Admit waiting streams in queue order while each one fits in the room
    left (a stream too big for the room keeps its place; smaller ones behind it
    may pass).  Returns (admitted, still waiting)."""
    admitted, left = [], []
    for i in waiting:
        if need[i] <= room:
            admitted.append(i)
            room -= need[i]
        else:
            left.append(i)
    return admitted, left


def poisson_arrivals(rates: list[float], duration_s: float, seed: int) -> list[tuple[float, int, int]]:
    """Sorted (time, stream, frame index) of independent Poisson streams."""
    rng = np.random.default_rng(seed)
    out = []
    for s, lam in enumerate(rates):
        t, k = 0.0, 0
        while True:
            t += rng.exponential(1.0 / lam)
            if t >= duration_s:
                break
            out.append((t, s, k))
            k += 1
    out.sort()
    return out


def percentiles(values, qs=(50, 99)) -> dict:
    if len(values) == 0:
        return {f"p{q}": None for q in qs}
    a = np.asarray(values)
    return {f"p{q}": float(np.percentile(a, q)) for q in qs}


@dataclass
class FrontendParams:
    """The detect-and-track loop's parameters for frontend serving."""
    target: int = 100
    redetect_frac: float = 0.3
    mode: int = fastgrid.FAST_TRACK_GAIN | fastgrid.FAST_TRACK_OFFSET
    max_iter: int = 30
    eps: float = 0.01


def resident_bytes(spec, pool_frames: int, slots: int, upload: bool = False, frontend_target: int = 0) -> int:
    """HBM a stream holds while admitted: its frame pool (or, when frames are
    uploaded per request, a level-0 plane per slot), the levels 1.. and output
    grid of every slot; for the detect-and-track loop (frontend_target > 0),
    the pool, two sets of levels 1.., the grid and the feature list."""
    dims = fastgrid.fast_pyr_dims(spec.width, spec.height, spec.levels)
    gw, gh = fastgrid.fast_grid_dims(spec.width, spec.height, spec.cell)
    lvl0 = dims[0][1] * dims[0][2]
    upper = sum(h * p for (_, h, p) in dims[1:])
    if frontend_target:
        return pool_frames * lvl0 + 2 * upper + 8 * gw * gh + frontend_target * (8 + 16 + 4) + 4 + 16
    if upload:
        return slots * (lvl0 + upper + 8 * gw * gh)
    return pool_frames * lvl0 + slots * (upper + 8 * gw * gh)


# ---------------------------------------------------------------- device state

@dataclass
class _Slot:
    planes: ctypes.Array            # fast_plane[levels]; [0] set per request
    upper: list                     # torch tensors of levels 1..
    grid: object                    # torch uint8 tensor, 8 B per cell
    host: object                    # pinned torch uint8 tensor
    job: fastgrid.fast_job = None
    lvl0: object = None             # own level-0 plane (upload mode)


class _FrontendState:
    """One stream's detect-and-track state: two sets of levels 1.. (the
    previous and the current frame; level 0 is the pool frame), this frame's
    cell winners and the device feature list."""

    def __init__(self, torch, spec, fe: FrontendParams):
        from .frontend import redetect_below
        dims = fastgrid.fast_pyr_dims(spec.width, spec.height, spec.levels)
        gw, gh = fastgrid.fast_grid_dims(spec.width, spec.height, spec.cell)
        self.upper = [[torch.empty((h, p), dtype=torch.uint8, device="cuda") for (_, h, p) in dims[1:]]
                      for _ in range(2)]
        self.planes = []
        for b in range(2):
            planes = (fastgrid.fast_plane * spec.levels)()
            for k, (t, (w, h, p)) in enumerate(zip(self.upper[b], dims[1:]), start=1):
                planes[k] = fastgrid.fast_plane(t.data_ptr(), w, h, p)
            self.planes.append(planes)
        self.grid = torch.empty(gw * gh * 8, dtype=torch.uint8, device="cuda")
        self.feats = torch.zeros((fe.target, 2), dtype=torch.float32, device="cuda")
        self.q = torch.zeros((fe.target, 4), dtype=torch.float32, device="cuda")
        self.status = torch.zeros(fe.target, dtype=torch.int32, device="cuda")
        self.count = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.info = torch.zeros(4, dtype=torch.int32, device="cuda")
        self.info_host = torch.zeros(4, dtype=torch.int32, pin_memory=True)
        self.below = redetect_below(fe.target, fe.redetect_frac)
        self.cur = 0
        self.frames = 0


@dataclass
class _Stream:
    spec: object
    pool: list                      # torch tensors (level 0 planes; pinned host in upload mode)
    pool_planes: list               # fast_plane for each pool frame (device mode)
    slots: list
    free: collections.deque = field(default_factory=collections.deque)
    pixels: int = 0
    host_pool: list = field(default_factory=list)   # the pool frames as host arrays
    fe: object = None               # _FrontendState in frontend serving


@dataclass
class Request:
    rid: int
    stream: int                     # index into the server's specs
    frame: int
    arrival: float
    slot: int = -1
    done: float = 0.0


class _Lane:
    """One launch lane: a HIP stream, its reusable completion and timing
    events, and its job array (at most one batch in flight per lane)."""

    def __init__(self, torch, max_batch: int):
        self.stream = torch.cuda.Stream()
        self.done_ev = torch.cuda.Event()
        self.t0 = torch.cuda.Event(enable_timing=True)
        self.t1 = torch.cuda.Event(enable_timing=True)
        self.jobs = (fastgrid.fast_job * max_batch)()
        self.fejobs = (fastgrid.fast_frontend_job * max_batch)()


class Server:
    """Continuous batching over camera streams on one GPU, with admission by
    free HBM as streams join and leave."""

    def __init__(self, ctx: fastgrid.Context, specs, pool_frames: int = 4, slots_per_stream: int = 4,
                 hbm_budget: int | None = None, reserve: int = 2 << 30, max_batch: int = 64,
                 inflight: int = 4, download: bool = True, keep_results: bool = False, log=None,
                 upload: bool = False, frontend: FrontendParams | None = None):
        import torch
        self.ctx, self.torch = ctx, torch
        self.upload = upload
        self.frontend = frontend
        if frontend is not None:
            # frames of a stream are served in order, one at a time; a batch
            # takes two submission slots of the context (detection, front end)
            if upload:
                raise ValueError("frontend serving reads frames from the device pool")
            slots_per_stream = 1
            inflight = min(inflight, 4)
        self.max_batch, self.inflight, self.download = max_batch, inflight, download
        self.keep_results = keep_results
        self.log = log or (lambda m: None)
        self.pool_frames, self.slots_per_stream, self.reserve = pool_frames, slots_per_stream, reserve
        # a budget taken from free memory is also checked against what the
        # device has free at each admission
        self.live_check = hbm_budget is None
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = max(0, free - reserve)
        self.hbm_budget = hbm_budget
        self.specs = list(specs)
        self.need = [resident_bytes(s, pool_frames, slots_per_stream, upload,
                                    frontend.target if frontend else 0) for s in self.specs]
        self.streams: list[_Stream | None] = [None] * len(self.specs)
        self.used = 0
        self.waiting: list[int] = list(range(len(self.specs)))
        self.gone: set[int] = set()
        self.admission_log: list[tuple[float, int, str]] = []
        self._admit(-1.0)
        self.admitted = [self.specs[i] for i in range(len(self.specs)) if self.streams[i] is not None]
        self.rejected = [self.specs[i] for i in self.waiting]
        self.lanes = [_Lane(torch, max_batch) for _ in range(inflight)]
        self.results: dict[int, np.ndarray] = {}

    @property
    def resident(self) -> int:
        return self.used

    def hbm_room(self) -> int:
        """Bytes a new stream may take: the budget left, and for a budget taken
        from free memory also what the device has free (torch's cached blocks
        count as free) minus the reserve."""
        room = self.hbm_budget - self.used
        if self.live_check:
            torch = self.torch
            free, _ = torch.cuda.mem_get_info()
            cached = torch.cuda.memory_reserved() - torch.cuda.memory_allocated()
            room = min(room, free + cached - self.reserve)
        return room

    def _admit(self, now: float) -> list[int]:
        """Make waiting streams resident, in queue order, while they fit."""
        if not self.waiting:
            return []
        admitted, self.waiting = admit_waiting(self.waiting, self.need, self.hbm_room())
        for i in admitted:
            self.streams[i] = self._make_stream(self.specs[i])
            self.used += self.need[i]
            self.admission_log.append((now, i, "admitted"))
        return admitted

    def _release(self, i: int, now: float) -> None:
        """Free a departed stream's device buffers and give its bytes back."""
        st = self.streams[i]
        self.streams[i] = None
        self.used -= self.need[i]
        self.gone.add(i)
        del st
        self.admission_log.append((now, i, "released"))

    def _make_stream(self, spec) -> _Stream:
        torch = self.torch
        dims = fastgrid.fast_pyr_dims(spec.width, spec.height, spec.levels)
        w0, h0, p0 = dims[0]
        pool, pool_planes, host_pool = [], [], []
        for k in range(self.pool_frames):
            img = spec.frame(k)
            host_pool.append(img)
            src = np.zeros((h0, p0), np.uint8)
            src[:, :img.shape[1]] = img[:, :p0]
            if self.upload:
                t = torch.empty((h0, p0), dtype=torch.uint8, pin_memory=True)
                t.copy_(torch.from_numpy(src))
                pool.append(t)
            else:
                t = torch.zeros((h0, p0), dtype=torch.uint8, device="cuda")
                t.copy_(torch.from_numpy(src))
                pool.append(t)
                pool_planes.append(fastgrid.fast_plane(t.data_ptr(), w0, h0, p0))
        gw, gh = fastgrid.fast_grid_dims(spec.width, spec.height, spec.cell)
        slots = []
        for _ in range(self.slots_per_stream):
            if self.frontend is not None:   # the front-end state holds the buffers
                slots.append(_Slot(None, [], None, None))
                continue
            upper = [torch.zeros((h, p), dtype=torch.uint8, device="cuda") for (_, h, p) in dims[1:]]
            planes = (fastgrid.fast_plane * spec.levels)()
            lvl0 = None
            if self.upload:
                lvl0 = torch.zeros((h0, p0), dtype=torch.uint8, device="cuda")
                planes[0] = fastgrid.fast_plane(lvl0.data_ptr(), w0, h0, p0)
            else:
                planes[0] = pool_planes[0]
            for k, (t, (w, h, p)) in enumerate(zip(upper, dims[1:]), start=1):
                planes[k] = fastgrid.fast_plane(t.data_ptr(), w, h, p)
            grid = torch.zeros(gw * gh * 8, dtype=torch.uint8, device="cuda")
            host = torch.empty(gw * gh * 8, dtype=torch.uint8, pin_memory=True)
            sl = _Slot(planes, upper, grid, host, lvl0=lvl0)
            sl.job = fastgrid.fast_job(ctypes.cast(planes, ctypes.POINTER(fastgrid.fast_plane)),
                                       spec.levels, spec.t, spec.n, spec.cell, grid.data_ptr())
            slots.append(sl)
        # the pool copies and fills are done before any request reads them (the
        # launch lanes are other streams; no wait on their work)
        torch.cuda.current_stream().synchronize()
        st = _Stream(spec, pool, pool_planes, slots, host_pool=host_pool)
        if self.frontend is not None:
            st.fe = _FrontendState(torch, spec, self.frontend)
            torch.cuda.current_stream().synchronize()
        st.free.extend(range(self.slots_per_stream))
        st.pixels = spec.width * spec.height
        return st

    # -------------------------------------------------------------- loop

    def run(self, duration_s: float, seed: int = 5, batched: bool = True,
            rate_scale: float = 1.0, leave: dict | None = None, trace: list | None = None) -> dict:
        """Serve Poisson arrivals for duration_s of wall time; return stats.

        Every stream that has not left sends frames at its rate times
        rate_scale; frames of a stream that is not resident are refused.
        leave: {stream index: seconds} -- the stream stops sending at that time
        and is released once its requests have completed, which lets waiting
        streams in.  trace: a list that receives one record per batch (host
        times in ms from the start of the run, and the batch's device time
        between events around its launch and result copy)."""
        torch = self.torch
        leave = dict(leave or {})
        rates = [s.rate_fps * rate_scale for s in self.specs]
        schedule = poisson_arrivals(rates, duration_s, seed)
        schedule = [a for a in schedule
                    if a[1] not in self.gone and (a[1] not in leave or a[0] < leave[a[1]])]
        reqs = [Request(i, s, k, t) for i, (t, s, k) in enumerate(schedule)]
        refused = collections.Counter()
        # arrived requests, per stream in arrival order
        pending = [collections.deque() for _ in self.specs]
        outstanding = collections.Counter()   # per stream: pending + in flight
        leaving = sorted((t, i) for i, t in leave.items() if i not in self.gone)
        npending = 0
        inflight: list = []          # (lane index, [requests], t_submit_ms)
        free_lanes = collections.deque(range(self.inflight))
        nxt, done = 0, []
        batches, batch_sizes = 0, []
        self._admit(0.0)
        torch.cuda.synchronize()
        gc.collect()
        gc_was = gc.isenabled()
        gc.disable()
        t0 = time.perf_counter()
        try:
            while nxt < len(reqs) or npending or inflight or leaving:
                now = time.perf_counter() - t0
                while nxt < len(reqs) and reqs[nxt].arrival <= now:
                    r = reqs[nxt]
                    nxt += 1
                    if self.streams[r.stream] is None:
                        refused[r.stream] += 1
                        continue
                    pending[r.stream].append(r)
                    outstanding[r.stream] += 1
                    npending += 1
                # completions
                still = []
                for lane_i, group, t_sub in inflight:
                    lane = self.lanes[lane_i]
                    if lane.done_ev.query() and (not batched or self.ctx.poll(lane.ticket)):
                        tnow = time.perf_counter() - t0
                        for r in group:
                            r.done = tnow
                            st = self.streams[r.stream]
                            if self.keep_results:
                                if st.fe is not None:
                                    info = st.fe.info_host.numpy().copy()
                                    n = int(info[2])
                                    self.results[r.rid] = (info, st.fe.feats[:n].cpu().numpy().copy())
                                else:
                                    self.results[r.rid] = st.slots[r.slot].host.numpy().copy()
                            st.free.append(r.slot)
                            outstanding[r.stream] -= 1
                        done.extend(group)
                        free_lanes.append(lane_i)
                        if trace is not None:
                            trace.append({"n": len(group),
                                          "oldest_arrival_ms": min(r.arrival for r in group) * 1e3,
                                          "submit_ms": t_sub, "seen_done_ms": tnow * 1e3,
                                          "device_ms": lane.t0.elapsed_time(lane.t1)})
                    else:
                        still.append((lane_i, group, t_sub))
                inflight = still
                # departures: a stream past its leave time with nothing
                # outstanding is released, and waiting streams may come in
                while leaving and leaving[0][0] <= now and outstanding[leaving[0][1]] == 0:
                    _, i = leaving.pop(0)
                    if self.streams[i] is not None:
                        self._release(i, now)
                        self._admit(now)
                # launch: the oldest arrived frames whose stream has a free slot
                # form the next batch
                while free_lanes and npending:
                    limit = self.max_batch if batched else 1
                    heads = [(q[0].arrival, s) for s, q in enumerate(pending) if q and self.streams[s].free]
                    heapq.heapify(heads)
                    group = []
                    while heads and len(group) < limit:
                        _, s_ = heapq.heappop(heads)
                        r = pending[s_].popleft()
                        r.slot = self.streams[s_].free.popleft()
                        group.append(r)
                        if pending[s_] and self.streams[s_].free:
                            heapq.heappush(heads, (pending[s_][0].arrival, s_))
                    npending -= len(group)
                    if not group:
                        break
                    lane_i = free_lanes.popleft()
                    lane = self.lanes[lane_i]
                    hs = lane.stream
                    t_sub = (time.perf_counter() - t0) * 1e3
                    with torch.cuda.stream(hs):
                        if trace is not None:
                            lane.t0.record(hs)
                        if self.frontend is not None:
                            lane.ticket = self._frontend_batch(group, lane, hs)
                        elif batched:
                            for i, r in enumerate(group):
                                lane.jobs[i] = self._prepare(r, hs).job
                            lane.ticket = fastgrid.fast_submit(self.ctx.handle, lane.jobs, len(group), hs)
                        else:
                            r = group[0]
                            spec = self.specs[r.stream]
                            sl = self._prepare(r, hs)
                            fastgrid.fast_detect_grid(self.ctx.handle, sl.planes, spec.levels, spec.t,
                                                      spec.n, spec.cell, sl.grid.data_ptr(), hs)
                        if self.download and self.frontend is None:
                            for r in group:
                                sl = self.streams[r.stream].slots[r.slot]
                                sl.host.copy_(sl.grid, non_blocking=True)
                        if trace is not None:
                            lane.t1.record(hs)
                        lane.done_ev.record(hs)
                    inflight.append((lane_i, group, t_sub))
                    batches += 1
                    batch_sizes.append(len(group))
                if not (nxt < len(reqs) and reqs[nxt].arrival <= time.perf_counter() - t0):
                    time.sleep(0)
            wall = time.perf_counter() - t0
        finally:
            if gc_was:
                gc.enable()
        torch.cuda.synchronize()
        lat_ms = [(r.done - r.arrival) * 1e3 for r in done]
        per_res = collections.defaultdict(list)
        for r, l in zip(done, lat_ms):
            s = self.specs[r.stream]
            per_res[f"{s.width}x{s.height}"].append(l)
        px = sum(self.specs[r.stream].width * self.specs[r.stream].height for r in done)
        return {
            "mode": ("frontend" if self.frontend is not None else ("batched" if batched else "plain")) +
                    ("+upload" if self.upload else ""),
            "rate_scale": rate_scale,
            "frames": len(done), "offered_frames": len(reqs), "refused_frames": sum(refused.values()),
            "refused_by_stream": dict(refused), "duration_s": duration_s,
            "wall_s": wall, "mpixel_s": px / wall / 1e6,
            "latency_ms": percentiles(lat_ms),
            "latency_ms_by_resolution": {k: percentiles(v) for k, v in sorted(per_res.items())},
            "batches": batches, "mean_batch": float(np.mean(batch_sizes)) if batch_sizes else 0.0,
            "streams_admitted": sum(1 for st in self.streams if st is not None),
            "streams_waiting": len(self.waiting), "streams_rejected": len(self.waiting),
            "resident_bytes": self.used, "hbm_budget": self.hbm_budget,
            "requests": done,
        }

    def run_native(self, duration_s: float, seed: int = 5, batched: bool = True, rate_scale: float = 1.0,
                   max_seconds: float | None = None) -> dict:
        """The same arrivals and batching rule as run(), with the loop itself
        in the library (fast_pump_run): it replays the arrival schedule by the
        host clock, launches, copies results and polls completions without
        returning to Python.  Serves the streams resident now (no joins or
        leaves, no uploads); frames of other streams are
        refused.  With a front end (fast_pump_run_frontend) every stream
        starts afresh: its first frame in the run has no previous frame.
        Returns the same statistics as run(), plus "slot_of" (the result slot
        each request used), "served" (time, stream, frame of each request)
        and "done_s" (when its completion was seen), in request order."""
        if self.upload:
            raise ValueError("the native loop serves resident frames")
        torch = self.torch
        live = [i for i, st in enumerate(self.streams) if st is not None]
        index = {i: j for j, i in enumerate(live)}
        arr = (fastgrid.fast_pump_stream * len(live))()
        fes = (fastgrid.fast_pump_frontend * len(live))()
        keep = []   # ctypes arrays the descriptors point into
        for j, i in enumerate(live):
            st, spec = self.streams[i], self.specs[i]
            nup = spec.levels - 1
            pool = (fastgrid.fast_plane * len(st.pool_planes))(*st.pool_planes)
            keep.append(pool)
            if self.frontend is not None:
                fe = st.fe
                upper = (fastgrid.fast_plane * max(1, 2 * nup))()
                for b in range(2):
                    for lv in range(nup):
                        upper[b * nup + lv] = fe.planes[b][lv + 1]
                keep.append(upper)
                fes[j] = fastgrid.fast_pump_frontend(
                    upper, fe.grid.data_ptr(), fe.feats.data_ptr(), fe.count.data_ptr(), fe.q.data_ptr(),
                    fe.status.data_ptr(), fe.info.data_ptr(), fe.info_host.data_ptr(), self.frontend.target,
                    fe.below)
                arr[j] = fastgrid.fast_pump_stream(spec.levels, spec.t, spec.n, spec.cell, 0, len(pool), pool, 1,
                                                   None, None, None)
                continue
            upper = (fastgrid.fast_plane * max(1, len(st.slots) * nup))()
            for k, sl in enumerate(st.slots):
                for lv in range(nup):
                    upper[k * nup + lv] = sl.planes[lv + 1]
            out = (ctypes.c_void_p * len(st.slots))(*[sl.grid.data_ptr() for sl in st.slots])
            host = (ctypes.c_void_p * len(st.slots))(*[sl.host.data_ptr() for sl in st.slots])
            keep += [upper, out, host]
            arr[j] = fastgrid.fast_pump_stream(
                spec.levels, spec.t, spec.n, spec.cell, 0, len(pool), pool, len(st.slots), upper, out,
                host if self.download else None)
        rates = [s.rate_fps * rate_scale for s in self.specs]
        schedule = poisson_arrivals(rates, duration_s, seed)
        served = [(t, s, k) for t, s, k in schedule if s in index]
        refused = collections.Counter(s for _, s, _ in schedule if s not in index)
        reqs = (fastgrid.fast_pump_request * len(served))(
            *[fastgrid.fast_pump_request(index[s], k, t) for t, s, k in served])
        torch.cuda.synchronize()
        gc_was = gc.isenabled()
        gc.disable()
        limit = max_seconds if max_seconds is not None else 3.0 * duration_s + 10.0
        try:
            if self.frontend is not None:
                fp = self.frontend
                done, nb = fastgrid.fast_pump_run_frontend(
                    self.ctx.handle, arr, fes, len(live), reqs, len(served), self.inflight, self.max_batch,
                    fp.mode, fp.max_iter, fp.eps, limit)
                slot_of = np.zeros(len(served), dtype=np.int32)
            else:
                done, slot_of, nb = fastgrid.fast_pump_run(
                    self.ctx.handle, arr, len(live), reqs, len(served), self.inflight, self.max_batch, batched,
                    limit)
        finally:
            if gc_was:
                gc.enable()
        if self.frontend is not None:
            # the native loop starts every stream afresh (its first frame has
            # no previous one) with pyramid 0 current; carry its end state over
            # so that a later run() continues each stream's sequence
            last = {}
            counts = collections.Counter()
            for _, s_, k in served:
                last[s_] = k
                counts[s_] += 1
            for s_, n_ in counts.items():
                fe, st = self.streams[s_].fe, self.streams[s_]
                fe.planes[(n_ - 1) % 2][0] = st.pool_planes[last[s_] % len(st.pool)]
                fe.cur = n_ % 2
                fe.frames = n_
        lat_ms = [(d - t) * 1e3 for d, (t, _, _) in zip(done, served)]
        per_res = collections.defaultdict(list)
        for (t, s, _), l in zip(served, lat_ms):
            per_res[f"{self.specs[s].width}x{self.specs[s].height}"].append(l)
        wall = float(done.max()) if len(done) else 0.0
        px = sum(self.specs[s].width * self.specs[s].height for _, s, _ in served)
        return {
            "mode": ("frontend" if self.frontend is not None else ("batched" if batched else "plain")) + "-native",
            "rate_scale": rate_scale,
            "frames": len(served), "offered_frames": len(schedule), "refused_frames": sum(refused.values()),
            "refused_by_stream": dict(refused), "duration_s": duration_s,
            "wall_s": wall, "mpixel_s": px / wall / 1e6 if wall > 0 else 0.0,
            "latency_ms": percentiles(lat_ms),
            "latency_ms_by_resolution": {k: percentiles(v) for k, v in sorted(per_res.items())},
            "batches": nb, "mean_batch": len(served) / nb if nb else 0.0,
            "streams_admitted": len(live), "streams_waiting": len(self.waiting),
            "streams_rejected": len(self.waiting), "resident_bytes": self.used, "hbm_budget": self.hbm_budget,
            "requests": [], "slot_of": slot_of, "served": served, "done_s": done,
        }

    def _frontend_batch(self, group, lane, hs) -> int:
        """One batch of the detect-and-track loop: detection (SAD-A) of every
        request's frame into its stream's current pyramid, then the front-end
        step of every stream from its previous frame; the step summaries go
        to pinned host memory.  Returns the last ticket."""
        P = ctypes.POINTER(fastgrid.fast_plane)
        fp = self.frontend
        for i, r in enumerate(group):
            st = self.streams[r.stream]
            fe, spec = st.fe, st.spec
            cur = fe.planes[fe.cur]
            cur[0] = st.pool_planes[r.frame % len(st.pool)]
            lane.jobs[i] = fastgrid.fast_job(ctypes.cast(cur, P), spec.levels, spec.t, spec.n, spec.cell,
                                             fe.grid.data_ptr(), fastgrid.FAST_SCORE_SADA)
        fastgrid.fast_submit(self.ctx.handle, lane.jobs, len(group), hs)
        for i, r in enumerate(group):
            st = self.streams[r.stream]
            fe, spec = st.fe, st.spec
            prev = ctypes.cast(fe.planes[1 - fe.cur], P) if fe.frames > 0 else None
            lane.fejobs[i] = fastgrid.fast_frontend_job(
                prev, ctypes.cast(fe.planes[fe.cur], P), spec.levels, fe.grid.data_ptr(), spec.cell, fp.target,
                fe.below, fe.feats.data_ptr(), fe.count.data_ptr(), fe.q.data_ptr(), fe.status.data_ptr(),
                fe.info.data_ptr())
        tk = fastgrid.fast_frontend_step(self.ctx.handle, lane.fejobs, len(group), fp.mode, fp.max_iter, fp.eps,
                                         hs)
        for r in group:
            fe = self.streams[r.stream].fe
            fe.info_host.copy_(fe.info, non_blocking=True)
            fe.cur = 1 - fe.cur
            fe.frames += 1
        return tk

    def _prepare(self, r: Request, hs) -> _Slot:
        """Point the request's slot at its frame: the resident pool frame, or
        (upload mode) a host-to-device copy into the slot's level-0 plane on
        the request's stream."""
        st = self.streams[r.stream]
        sl = st.slots[r.slot]
        k = r.frame % len(st.pool)
        if self.upload:
            with self.torch.cuda.stream(hs):
                sl.lvl0.copy_(st.pool[k], non_blocking=True)
        else:
            sl.planes[0] = st.pool_planes[k]
        return sl

    def close(self):
        self.torch.cuda.synchronize()
        self.streams = [None] * len(self.specs)
