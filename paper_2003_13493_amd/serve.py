"""Continuous-batching server for simulated camera streams.

Each admitted camera stream keeps, resident in HBM:
  * a pool of its frames (level 0 planes), so arrivals need no PCIe upload;
  * a ring of request slots: pyramid levels 1.. and an output grid per slot;
  * pinned host buffers that receive each slot's cell results.

With upload=True the frames stay in pinned host memory instead and every
request first copies its frame into the slot's own level-0 plane (host to
device, on the request's stream): the PCIe-inclusive variant.

A stream is admitted only if its resident bytes fit in the HBM budget (free
memory at start-up minus a reserve, or an explicit budget).  Frames arrive by
per-stream Poisson processes.  The loop keeps up to K batches in flight on K
HIP streams; whenever a launch slot is free, every frame that has arrived and
holds a request slot joins the next batch (up to a batch limit), so frames that
arrive while others run are admitted as slots free up and their work overlaps
on the device.  A batch is one `fast_submit` (persistent launch over a device
work queue) followed by the copy of its results to the host; its ticket is
polled, and the frame latency is the poll-observed completion time minus the
arrival time.
"""
from __future__ import annotations

import collections
import ctypes
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


def resident_bytes(spec, pool_frames: int, slots: int, upload: bool = False) -> int:
    """HBM a stream holds while admitted: its frame pool (or, when frames are
    uploaded per request, a level-0 plane per slot), the levels 1.. and output
    grid of every slot."""
    dims = fastgrid.fast_pyr_dims(spec.width, spec.height, spec.levels)
    gw, gh = fastgrid.fast_grid_dims(spec.width, spec.height, spec.cell)
    lvl0 = dims[0][1] * dims[0][2]
    upper = sum(h * p for (_, h, p) in dims[1:])
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


@dataclass
class _Stream:
    spec: object
    pool: list                      # torch tensors (level 0 planes; pinned host in upload mode)
    pool_planes: list               # fast_plane for each pool frame (device mode)
    slots: list
    free: collections.deque = field(default_factory=collections.deque)
    pixels: int = 0


@dataclass
class Request:
    rid: int
    stream: int
    frame: int
    arrival: float
    slot: int = -1
    done: float = 0.0


class Server:
    """Continuous batching over camera streams on one GPU."""

    def __init__(self, ctx: fastgrid.Context, specs, pool_frames: int = 4, slots_per_stream: int = 4,
                 hbm_budget: int | None = None, reserve: int = 2 << 30, max_batch: int = 64,
                 inflight: int = 4, download: bool = True, keep_results: bool = False, log=None,
                 upload: bool = False):
        import torch
        self.ctx, self.torch = ctx, torch
        self.upload = upload
        self.max_batch, self.inflight, self.download = max_batch, inflight, download
        self.keep_results = keep_results
        self.log = log or (lambda m: None)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = max(0, free - reserve)
        self.hbm_budget = hbm_budget
        need = [resident_bytes(s, pool_frames, slots_per_stream, upload) for s in specs]
        admitted, rejected = plan_admission(need, hbm_budget)
        self.admitted = [specs[i] for i in admitted]
        self.rejected = [specs[i] for i in rejected]
        self.resident = sum(need[i] for i in admitted)
        self.streams: list[_Stream] = []
        for spec in self.admitted:
            self.streams.append(self._make_stream(spec, pool_frames, slots_per_stream))
        self.hip_streams = [torch.cuda.Stream() for _ in range(inflight)]
        self.results: dict[int, np.ndarray] = {}

    def _make_stream(self, spec, pool_frames, nslots) -> _Stream:
        torch = self.torch
        dims = fastgrid.fast_pyr_dims(spec.width, spec.height, spec.levels)
        w0, h0, p0 = dims[0]
        pool, pool_planes = [], []
        for k in range(pool_frames):
            img = spec.frame(k)
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
        for _ in range(nslots):
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
        st = _Stream(spec, pool, pool_planes, slots)
        st.free.extend(range(nslots))
        st.pixels = spec.width * spec.height
        return st

    # -------------------------------------------------------------- loop

    def run(self, duration_s: float, seed: int = 5, batched: bool = True,
            rate_scale: float = 1.0) -> dict:
        """Serve Poisson arrivals for duration_s of wall time (each stream's rate
        multiplied by rate_scale); return stats."""
        torch = self.torch
        rates = [st.spec.rate_fps * rate_scale for st in self.streams]
        schedule = poisson_arrivals(rates, duration_s, seed)
        reqs = [Request(i, s, k, t) for i, (t, s, k) in enumerate(schedule)]
        # arrived requests, per stream in arrival order
        pending = [collections.deque() for _ in self.streams]
        npending = 0
        inflight: list = []          # (ticket or event, [requests], hip stream index)
        free_lanes = collections.deque(range(self.inflight))
        nxt, done = 0, []
        batches, batch_sizes = 0, []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while nxt < len(reqs) or npending or inflight:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                pending[reqs[nxt].stream].append(reqs[nxt])
                npending += 1
                nxt += 1
            # completions
            still = []
            for tk, group, lane in inflight:
                fin = tk.done() if batched else tk.query()
                if fin:
                    tnow = time.perf_counter() - t0
                    for r in group:
                        r.done = tnow
                        st = self.streams[r.stream]
                        if self.keep_results:
                            self.results[r.rid] = st.slots[r.slot].host.numpy().copy()
                        st.free.append(r.slot)
                    done.extend(group)
                    free_lanes.append(lane)
                else:
                    still.append((tk, group, lane))
            inflight = still
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
                lane = free_lanes.popleft()
                hs = self.hip_streams[lane]
                if batched:
                    jobs = (fastgrid.fast_job * len(group))()
                    for i, r in enumerate(group):
                        jobs[i] = self._prepare(r, hs).job
                    with torch.cuda.stream(hs):
                        tk = self.ctx.submit(jobs, hs)
                        if self.download:
                            for r in group:
                                sl = self.streams[r.stream].slots[r.slot]
                                sl.host.copy_(sl.grid, non_blocking=True)
                        ev = torch.cuda.Event()
                        ev.record(hs)
                    inflight.append((_Ticket(self.ctx, tk, ev), group, lane))
                else:
                    r = group[0]
                    st = self.streams[r.stream]
                    sl = self._prepare(r, hs)
                    with torch.cuda.stream(hs):
                        fastgrid.fast_detect_grid(self.ctx.handle, sl.planes, st.spec.levels,
                                                  st.spec.t, st.spec.n, st.spec.cell,
                                                  sl.grid.data_ptr(), hs)
                        if self.download:
                            sl.host.copy_(sl.grid, non_blocking=True)
                        ev = torch.cuda.Event()
                        ev.record(hs)
                    inflight.append((ev, group, lane))
                batches += 1
                batch_sizes.append(len(group))
            if not (nxt < len(reqs) and reqs[nxt].arrival <= time.perf_counter() - t0):
                time.sleep(0)
        wall = time.perf_counter() - t0
        torch.cuda.synchronize()
        lat_ms = [(r.done - r.arrival) * 1e3 for r in done]
        per_res = collections.defaultdict(list)
        for r, l in zip(done, lat_ms):
            s = self.streams[r.stream].spec
            per_res[f"{s.width}x{s.height}"].append(l)
        px = sum(self.streams[r.stream].pixels for r in done)
        return {
            "mode": ("batched" if batched else "plain") + ("+upload" if self.upload else ""),
            "rate_scale": rate_scale,
            "frames": len(done), "offered_frames": len(reqs), "duration_s": duration_s,
            "wall_s": wall, "mpixel_s": px / wall / 1e6,
            "latency_ms": percentiles(lat_ms),
            "latency_ms_by_resolution": {k: percentiles(v) for k, v in sorted(per_res.items())},
            "batches": batches, "mean_batch": float(np.mean(batch_sizes)) if batch_sizes else 0.0,
            "streams_admitted": len(self.streams), "streams_rejected": len(self.rejected),
            "resident_bytes": self.resident, "hbm_budget": self.hbm_budget,
            "requests": done,
        }

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
        self.streams.clear()


class _Ticket:
    """Completion of a batch: the submission's ticket and its result copies."""

    def __init__(self, ctx, ticket, event):
        self.ctx, self.ticket, self.event = ctx, ticket, event

    def done(self) -> bool:
        return self.ctx.poll(self.ticket) and self.event.query()

