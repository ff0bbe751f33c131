"""ctypes binding of ``libfastgrid.so`` (see include/fastgrid.h).

Argument marshalling only: every step of the detector runs in the library's
HIP kernels.  The functions keep the C names; device memory and streams come
from PyTorch (``uint8`` CUDA tensors of shape (height, pitch) for planes, and
``torch.cuda.Stream`` / the current stream for ordering).

There is no fallback: if the library is missing or no GPU is present, the
calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastgrid.so")

FAST_OK, FAST_EINVAL, FAST_ENOMEM, FAST_EHIP, FAST_EBUSY, FAST_ETIMEDOUT = 0, -1, -2, -3, -4, -5
FAST_MAX_LEVELS = 8
FAST_PLAN_GRAPH = 1

FEATURE_DTYPE = np.dtype([("x", "<u2"), ("y", "<u2"), ("score", "<u2"),
                          ("level", "u1"), ("reserved", "u1")])
EMPTY = (0xFFFF, 0xFFFF, 0, 0xFF)

# Corner score kinds (fast_job.score, fast_detect_grid_score).
FAST_SCORE_SADB, FAST_SCORE_SADA, FAST_SCORE_MT = 0, 1, 2

EXPORTS = ("fast_ctx_create", "fast_ctx_destroy", "fast_strerror", "fast_last_error",
           "fast_pyr_dims", "fast_grid_dims", "fast_pyr_build", "fast_detect_grid",
           "fast_detect_grid_score", "fast_score_maps", "fast_nms_grid",
           "fast_submit", "fast_submit_static", "fast_poll", "fast_wait", "fast_plan_create", "fast_plan_launch",
           "fast_plan_destroy", "fast_set_launch", "fast_track", "fast_set_shape_table",
           "fast_shape_region_of", "fast_frontend_step", "fast_pump_run", "fast_pump_run_frontend")


class fast_plane(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("pitch", ctypes.c_int32)]


class fast_job(ctypes.Structure):
    _fields_ = [("pyr", ctypes.POINTER(fast_plane)), ("levels", ctypes.c_int32),
                ("t", ctypes.c_int32), ("n", ctypes.c_int32), ("cell", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("score", ctypes.c_int32)]


class fast_shape_region(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("cell", ctypes.c_int32), ("region", ctypes.c_int32)]


FAST_MAX_SHAPES = 1024
FAST_MAX_TRACKS = 1024
FAST_MAX_GRID_CELLS = 65536


class fast_frontend_job(ctypes.Structure):
    _fields_ = [("prev", ctypes.POINTER(fast_plane)), ("cur", ctypes.POINTER(fast_plane)),
                ("levels", ctypes.c_int32), ("slots", ctypes.c_void_p), ("cell", ctypes.c_int32),
                ("capacity", ctypes.c_int32), ("redetect_below", ctypes.c_int32),
                ("feats", ctypes.c_void_p), ("count", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("info", ctypes.c_void_p)]


class fast_pump_stream(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("t", ctypes.c_int32), ("n", ctypes.c_int32),
                ("cell", ctypes.c_int32), ("score", ctypes.c_int32), ("pool_frames", ctypes.c_int32),
                ("pool", ctypes.POINTER(fast_plane)), ("slots", ctypes.c_int32),
                ("upper", ctypes.POINTER(fast_plane)), ("out", ctypes.POINTER(ctypes.c_void_p)),
                ("host_out", ctypes.POINTER(ctypes.c_void_p))]


class fast_pump_request(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_int32), ("frame", ctypes.c_int32), ("arrival_s", ctypes.c_double)]


class fast_pump_frontend(ctypes.Structure):
    _fields_ = [("upper", ctypes.POINTER(fast_plane)), ("grid", ctypes.c_void_p), ("feats", ctypes.c_void_p),
                ("count", ctypes.c_void_p), ("q", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("info", ctypes.c_void_p), ("info_host", ctypes.c_void_p), ("capacity", ctypes.c_int32),
                ("redetect_below", ctypes.c_int32)]


FAST_PUMP_MAX_LANES = 8


class FastError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        super().__init__(f"{what}: {code} ({detail})" if detail else f"{what}: {code}")


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: build it with __graft_entry__.build()")
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes the library bind to that one, so the process holds a
        # single HIP runtime and torch's streams and memory are valid here.
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, u64p = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)
        P = ctypes.POINTER(fast_plane)
        sig = {
            "fast_ctx_create": ([i32, ctypes.POINTER(vp)], i32),
            "fast_ctx_destroy": ([vp], None),
            "fast_strerror": ([i32], ctypes.c_char_p),
            "fast_last_error": ([vp], ctypes.c_char_p),
            "fast_pyr_dims": ([i32, i32, i32, P], i32),
            "fast_grid_dims": ([i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
            "fast_pyr_build": ([vp, P, i32, vp], i32),
            "fast_detect_grid": ([vp, P, i32, i32, i32, i32, vp, vp], i32),
            "fast_detect_grid_score": ([vp, P, i32, i32, i32, i32, i32, vp, vp], i32),
            "fast_submit": ([vp, ctypes.POINTER(fast_job), i32, vp, u64p], i32),
            "fast_submit_static": ([vp, ctypes.POINTER(fast_job), i32, vp, u64p], i32),
            "fast_poll": ([vp, ctypes.c_uint64], i32),
            "fast_wait": ([vp, ctypes.c_uint64, i32], i32),
            "fast_plan_create": ([vp, ctypes.POINTER(fast_job), i32, i32, ctypes.POINTER(i32)], i32),
            "fast_plan_launch": ([vp, i32, vp, u64p], i32),
            "fast_plan_destroy": ([vp, i32], i32),
            "fast_set_launch": ([vp, i32, i32, i32], i32),
            "fast_score_maps": ([vp, P, i32, i32, i32, i32, ctypes.POINTER(vp), ctypes.POINTER(i32), vp], i32),
            "fast_nms_grid": ([vp, ctypes.POINTER(vp), ctypes.POINTER(i32), i32, i32, i32, i32, i32, vp, vp],
                              i32),
            "fast_track": ([vp, P, P, i32, vp, vp, vp, vp, i32, i32, i32, ctypes.c_float, vp], i32),
            "fast_set_shape_table": ([vp, ctypes.POINTER(fast_shape_region), i32], i32),
            "fast_shape_region_of": ([vp, i32, i32, i32, i32, ctypes.POINTER(i32)], i32),
            "fast_frontend_step": ([vp, ctypes.POINTER(fast_frontend_job), i32, i32, i32, ctypes.c_float, vp,
                                    u64p], i32),
            "fast_pump_run": ([vp, ctypes.POINTER(fast_pump_stream), i32, ctypes.POINTER(fast_pump_request), i32,
                               i32, i32, i32, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], i32),
            "fast_pump_run_frontend": ([vp, ctypes.POINTER(fast_pump_stream), ctypes.POINTER(fast_pump_frontend),
                                        i32, ctypes.POINTER(fast_pump_request), i32, i32, i32, i32, i32,
                                        ctypes.c_float, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int32)], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def _check(ctx, rc: int, what: str) -> int:
    if rc < 0:
        detail = load().fast_last_error(ctx).decode() if ctx else load().fast_strerror(rc).decode()
        raise FastError(rc, what, detail)
    return rc


# ------------------------------------------------------------- C entry points

def fast_ctx_create(device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    rc = load().fast_ctx_create(device, ctypes.byref(h))
    if rc < 0:
        raise FastError(rc, "fast_ctx_create", load().fast_strerror(rc).decode())
    return h


def fast_ctx_destroy(ctx) -> None:
    load().fast_ctx_destroy(ctx)


def fast_pyr_dims(width: int, height: int, levels: int) -> list[tuple[int, int, int]]:
    arr = (fast_plane * levels)()
    rc = load().fast_pyr_dims(width, height, levels, arr)
    if rc < 0:
        raise FastError(rc, "fast_pyr_dims")
    return [(p.width, p.height, p.pitch) for p in arr]


def fast_grid_dims(width: int, height: int, cell: int) -> tuple[int, int]:
    gw, gh = ctypes.c_int(), ctypes.c_int()
    rc = load().fast_grid_dims(width, height, cell, ctypes.byref(gw), ctypes.byref(gh))
    if rc < 0:
        raise FastError(rc, "fast_grid_dims")
    return gw.value, gh.value


def fast_pyr_build(ctx, planes, levels: int, stream=None) -> None:
    _check(ctx, load().fast_pyr_build(ctx, planes, levels, _stream(stream)), "fast_pyr_build")


def fast_detect_grid(ctx, planes, levels: int, t: int, n: int, cell: int, out_ptr: int,
                     stream=None) -> None:
    _check(ctx, load().fast_detect_grid(ctx, planes, levels, t, n, cell, out_ptr,
                                        _stream(stream)), "fast_detect_grid")


def fast_detect_grid_score(ctx, planes, levels: int, t: int, n: int, cell: int, score: int,
                           out_ptr: int, stream=None) -> None:
    _check(ctx, load().fast_detect_grid_score(ctx, planes, levels, t, n, cell, score, out_ptr,
                                              _stream(stream)), "fast_detect_grid_score")


def fast_submit(ctx, jobs, njobs: int, stream=None) -> int:
    tk = ctypes.c_uint64()
    _check(ctx, load().fast_submit(ctx, jobs, njobs, _stream(stream), ctypes.byref(tk)),
           "fast_submit")
    return tk.value


def fast_submit_static(ctx, jobs, njobs: int, stream=None, ticket: bool = True) -> int:
    """Returns the ticket, or 0 when ticket=False (no completion event recorded)."""
    if not ticket:
        _check(ctx, load().fast_submit_static(ctx, jobs, njobs, _stream(stream), None), "fast_submit_static")
        return 0
    tk = ctypes.c_uint64()
    _check(ctx, load().fast_submit_static(ctx, jobs, njobs, _stream(stream), ctypes.byref(tk)),
           "fast_submit_static")
    return tk.value


def fast_poll(ctx, ticket: int) -> bool:
    return _check(ctx, load().fast_poll(ctx, ticket), "fast_poll") == 1


def fast_wait(ctx, ticket: int, timeout_ms: int = -1) -> bool:
    """True when finished, False on time-out."""
    rc = load().fast_wait(ctx, ticket, timeout_ms)
    if rc == FAST_ETIMEDOUT:
        return False
    _check(ctx, rc, "fast_wait")
    return True


def fast_plan_create(ctx, jobs, njobs: int, flags: int = 0) -> int:
    pid = ctypes.c_int()
    _check(ctx, load().fast_plan_create(ctx, jobs, njobs, flags, ctypes.byref(pid)),
           "fast_plan_create")
    return pid.value


def fast_plan_launch(ctx, plan_id: int, stream=None, ticket: bool = True) -> int:
    """Returns the ticket, or 0 when ticket=False (no completion event recorded)."""
    if not ticket:
        _check(ctx, load().fast_plan_launch(ctx, plan_id, _stream(stream), None),
               "fast_plan_launch")
        return 0
    tk = ctypes.c_uint64()
    _check(ctx, load().fast_plan_launch(ctx, plan_id, _stream(stream), ctypes.byref(tk)),
           "fast_plan_launch")
    return tk.value


def fast_plan_destroy(ctx, plan_id: int) -> None:
    _check(ctx, load().fast_plan_destroy(ctx, plan_id), "fast_plan_destroy")


def fast_set_launch(ctx, region: int, block: int, blocks_per_cu: int) -> None:
    _check(ctx, load().fast_set_launch(ctx, region, block, blocks_per_cu), "fast_set_launch")


def fast_set_shape_table(ctx, entries) -> None:
    """entries: iterable of (width, height, levels, cell, region)."""
    entries = list(entries)
    arr = (fast_shape_region * max(1, len(entries)))(*[fast_shape_region(*e) for e in entries])
    _check(ctx, load().fast_set_shape_table(ctx, arr, len(entries)), "fast_set_shape_table")


def fast_shape_region_of(ctx, width: int, height: int, levels: int, cell: int) -> int:
    r = ctypes.c_int()
    _check(ctx, load().fast_shape_region_of(ctx, width, height, levels, cell, ctypes.byref(r)),
           "fast_shape_region_of")
    return r.value


def fast_frontend_step(ctx, jobs, njobs: int, mode: int, max_iter: int, eps: float, stream=None) -> int:
    tk = ctypes.c_uint64()
    _check(ctx, load().fast_frontend_step(ctx, jobs, njobs, mode, max_iter, eps, _stream(stream),
                                          ctypes.byref(tk)), "fast_frontend_step")
    return tk.value


def fast_pump_run(ctx, streams, nstreams: int, reqs, nreq: int, lanes: int, max_batch: int, batched: bool,
                  max_seconds: float):
    """Serve nreq requests natively; returns (done_s, slot_of, nbatches) with
    the per-request arrays as numpy."""
    done = np.zeros(nreq, dtype=np.float64)
    slot = np.zeros(nreq, dtype=np.int32)
    nb = ctypes.c_int32()
    _check(ctx, load().fast_pump_run(ctx, streams, nstreams, reqs, nreq, lanes, max_batch, int(bool(batched)),
                                     max_seconds, done.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     slot.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(nb)),
           "fast_pump_run")
    return done, slot, nb.value


def fast_pump_run_frontend(ctx, streams, fe, nstreams: int, reqs, nreq: int, lanes: int, max_batch: int,
                           mode: int, max_iter: int, eps: float, max_seconds: float):
    """Serve nreq front-end requests natively; returns (done_s, nbatches)."""
    done = np.zeros(nreq, dtype=np.float64)
    nb = ctypes.c_int32()
    _check(ctx, load().fast_pump_run_frontend(ctx, streams, fe, nstreams, reqs, nreq, lanes, max_batch, mode,
                                              max_iter, eps, max_seconds,
                                              done.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              ctypes.byref(nb)), "fast_pump_run_frontend")
    return done, nb.value


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------- torch helpers

class Pyramid:
    """Device planes of one frame's pyramid, owned by torch tensors."""

    def __init__(self, width: int, height: int, levels: int, device="cuda"):
        import torch
        self.width, self.height, self.levels = width, height, levels
        self.dims = fast_pyr_dims(width, height, levels)
        self.tensors = [torch.zeros((h, p), dtype=torch.uint8, device=device)
                        for (w, h, p) in self.dims]
        self.planes = (fast_plane * levels)(*[
            fast_plane(t.data_ptr(), w, h, p) for t, (w, h, p) in zip(self.tensors, self.dims)])

    def upload(self, img: np.ndarray, non_blocking: bool = False) -> None:
        """Copy a (height, >=width) uint8 host image into level 0."""
        import torch
        p = self.dims[0][2]
        src = np.zeros((self.height, p), np.uint8)
        cols = min(p, img.shape[1])
        src[:, :cols] = img[:, :cols]
        self.tensors[0].copy_(torch.from_numpy(src), non_blocking=non_blocking)

    def level(self, k: int) -> np.ndarray:
        w, h, _ = self.dims[k]
        return self.tensors[k][:, :w].cpu().numpy()


def fast_score_maps(ctx, planes, levels: int, t: int, n: int, score: int, maps, pitches,
                    stream=None) -> None:
    _check(ctx, load().fast_score_maps(ctx, planes, levels, t, n, score, maps, pitches, _stream(stream)),
           "fast_score_maps")


def fast_nms_grid(ctx, maps, pitches, width: int, height: int, levels: int, radius: int, cell: int,
                  out_ptr: int, stream=None) -> None:
    _check(ctx, load().fast_nms_grid(ctx, maps, pitches, width, height, levels, radius, cell, out_ptr,
                                     _stream(stream)), "fast_nms_grid")


FAST_TRACK_GAIN = 1
FAST_TRACK_OFFSET = 2
FAST_TRACK_OK, FAST_TRACK_TEMPLATE_OUTSIDE, FAST_TRACK_LOST_OUTSIDE, FAST_TRACK_SINGULAR = 0, 1, 2, 3


def fast_track(ctx, tpl_planes, img_planes, levels: int, feats_ptr: int, q_ptr: int, status_ptr: int,
               iters_ptr: int, nfeat: int, mode: int, max_iter: int, eps: float, stream=None) -> None:
    _check(ctx, load().fast_track(ctx, tpl_planes, img_planes, levels, feats_ptr, q_ptr, status_ptr,
                                  iters_ptr or None, nfeat, mode, max_iter, eps, _stream(stream)),
           "fast_track")


class ScoreMaps:
    """Device score maps of a pyramid: one (H_k, W_k) tensor of uint16 scores per
    level (held as int16), for fast_score_maps / fast_nms_grid."""

    def __init__(self, width: int, height: int, levels: int, device="cuda"):
        import torch
        self.width, self.height, self.levels = width, height, levels
        self.tensors = []
        w, h = width, height
        for _ in range(levels):
            self.tensors.append(torch.zeros((h, w), dtype=torch.int16, device=device))
            w, h = w // 2, h // 2
        self.ptrs = (ctypes.c_void_p * levels)(*[t.data_ptr() for t in self.tensors])
        self.pitches = (ctypes.c_int32 * levels)(*[t.shape[1] for t in self.tensors])

    def level(self, k: int) -> np.ndarray:
        return self.tensors[k].cpu().numpy().view(np.uint16)


class Grid:
    """Device array of cell slots for one frame."""

    def __init__(self, width: int, height: int, cell: int, device="cuda"):
        import torch
        self.gw, self.gh = fast_grid_dims(width, height, cell)
        self.tensor = torch.zeros(self.gw * self.gh * 8, dtype=torch.uint8, device=device)

    @property
    def ptr(self) -> int:
        return self.tensor.data_ptr()

    def fetch(self) -> np.ndarray:
        return self.tensor.cpu().numpy().view(FEATURE_DTYPE)


class Context:
    """Owns a fast_ctx; detect() is the plain path, submit()/plan_*() the batched one."""

    def __init__(self, device: int = 0, tuned: bool = True):
        """tuned: load the launch-shape table shipped next to the library
        (tune.TABLE_PATH) when it was tuned on this device kind."""
        self.handle = fast_ctx_create(device)
        self.tuned = None
        if tuned:
            import torch
            from . import tune
            arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
            table = tune.load(device=arch)
            if table is not None:
                tune.apply(self, table)
                self.tuned = tune.TABLE_PATH

    def close(self):
        if self.handle:
            fast_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, region: int, block: int, blocks_per_cu: int) -> None:
        """region 0 selects the default: 64, or 32 for one small frame."""
        fast_set_launch(self.handle, region, block, blocks_per_cu)

    def set_shape_table(self, entries) -> None:
        """Tuned region sides of one-frame calls: (width, height, levels, cell, region) rows."""
        fast_set_shape_table(self.handle, entries)

    def shape_region(self, width: int, height: int, levels: int, cell: int) -> int:
        """The region side a one-frame call on this frame shape uses now."""
        return fast_shape_region_of(self.handle, width, height, levels, cell)

    def reset_launch(self) -> None:
        """The launch shape of a new context."""
        fast_set_launch(self.handle, 0, 256, 3)

    def pyr_build(self, pyr: Pyramid, stream=None) -> None:
        fast_pyr_build(self.handle, pyr.planes, pyr.levels, stream)

    def detect(self, pyr: Pyramid, t: int, n: int, cell: int, grid: Grid, stream=None,
               score: int = FAST_SCORE_SADB) -> None:
        if score == FAST_SCORE_SADB:
            fast_detect_grid(self.handle, pyr.planes, pyr.levels, t, n, cell, grid.ptr, stream)
        else:
            fast_detect_grid_score(self.handle, pyr.planes, pyr.levels, t, n, cell, score, grid.ptr,
                                   stream)

    def score_maps(self, pyr: Pyramid, t: int, n: int, maps: ScoreMaps, score: int = FAST_SCORE_SADB,
                   stream=None) -> None:
        fast_score_maps(self.handle, pyr.planes, pyr.levels, t, n, score, maps.ptrs, maps.pitches, stream)

    def track(self, tpl: Pyramid, img: Pyramid, feats, q, status, iters=None,
              mode: int = FAST_TRACK_GAIN | FAST_TRACK_OFFSET, max_iter: int = 30, eps: float = 0.01,
              stream=None) -> None:
        """Lucas-Kanade tracking of feats (device float32, N x 2) from tpl to img;
        q (device float32, N x 4) holds the initial (tx, ty, alpha, beta) and
        receives the estimate; status and iters are device int32 of length N."""
        import torch
        n = int(feats.shape[0])
        assert feats.dtype == torch.float32 and feats.is_contiguous() and tuple(feats.shape) == (n, 2)
        assert q.dtype == torch.float32 and q.is_contiguous() and tuple(q.shape) == (n, 4)
        assert status.dtype == torch.int32 and status.numel() == n
        assert iters is None or (iters.dtype == torch.int32 and iters.numel() == n)
        assert tpl.levels == img.levels
        fast_track(self.handle, tpl.planes, img.planes, tpl.levels, feats.data_ptr(), q.data_ptr(),
                   status.data_ptr(), iters.data_ptr() if iters is not None else 0, n, mode, max_iter, eps,
                   stream)

    def nms_grid(self, maps: ScoreMaps, radius: int, cell: int, grid: Grid, stream=None) -> None:
        fast_nms_grid(self.handle, maps.ptrs, maps.pitches, maps.width, maps.height, maps.levels, radius,
                      cell, grid.ptr, stream)

    @staticmethod
    def make_jobs(items) -> ctypes.Array:
        """items: iterable of (Pyramid, t, n, cell, Grid) or (Pyramid, t, n, cell, Grid, score)."""
        items = list(items)
        arr = (fast_job * len(items))()
        for i, it in enumerate(items):
            pyr, t, n, cell, grid = it[:5]
            score = it[5] if len(it) > 5 else FAST_SCORE_SADB
            arr[i] = fast_job(ctypes.cast(pyr.planes, ctypes.POINTER(fast_plane)), pyr.levels,
                              t, n, cell, grid.ptr, score)
        return arr

    def submit(self, jobs: ctypes.Array, stream=None) -> int:
        return fast_submit(self.handle, jobs, len(jobs), stream)

    def submit_static(self, jobs: ctypes.Array, stream=None, ticket: bool = True) -> int:
        """fast_submit through the library's fixed device scratch (no allocation)."""
        return fast_submit_static(self.handle, jobs, len(jobs), stream, ticket)

    def poll(self, ticket: int) -> bool:
        return fast_poll(self.handle, ticket)

    def wait(self, ticket: int, timeout_ms: int = -1) -> bool:
        return fast_wait(self.handle, ticket, timeout_ms)

    def plan_create(self, jobs: ctypes.Array, graph: bool = False) -> int:
        return fast_plan_create(self.handle, jobs, len(jobs), FAST_PLAN_GRAPH if graph else 0)

    def plan_launch(self, plan_id: int, stream=None, ticket: bool = True) -> int:
        return fast_plan_launch(self.handle, plan_id, stream, ticket)

    def plan_destroy(self, plan_id: int) -> None:
        fast_plan_destroy(self.handle, plan_id)
