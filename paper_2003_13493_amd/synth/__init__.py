"""Seeded synthetic frames and workload recipes (input synthesis only).

The paper evaluates on the EuRoC Machine Hall sequences (Section III); those
images are not available, so every frame here comes from a seeded generator
of rectangles, triangles, an optional brightness ramp and Gaussian noise.  The
same bytes feed the CPU oracle and the GPU path.  Nothing in this module
computes any part of the detector.

The C source (``frames.c``) is compiled into ``libsynth.so`` next to this file
by the package build step.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        lib.synth_scene.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_uint64, ctypes.c_int]
        lib.synth_frame.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        lib.synth_crop_noise.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, u8p, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_double]
        lib.synth_pad_garbage.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_uint64]
        lib.synth_ints.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int32)]
        lib.synth_units.argtypes = [ctypes.c_uint64, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double)]
        lib.synth_raw.argtypes = [ctypes.c_uint64, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_uint64)]
        for f in (lib.synth_scene, lib.synth_frame, lib.synth_crop_noise,
                  lib.synth_pad_garbage, lib.synth_ints, lib.synth_units, lib.synth_raw):
            f.restype = None
        _lib = lib
    return _lib


def _u8p(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def pitch_for(width: int, align: int = 64) -> int:
    """Row pitch used for every plane built here: width rounded up to ``align``."""
    return max(align, (width + align - 1) // align * align)


def frame(width: int, height: int, seed: int, nshapes: int, sigma: float,
          gradient: bool = False, pitch: int | None = None,
          pad_garbage: bool = False) -> np.ndarray:
    """One seeded frame as a (height, pitch) uint8 array; columns >= width are padding."""
    pitch = pitch_for(width) if pitch is None else pitch
    out = np.zeros((height, pitch), dtype=np.uint8)
    _load().synth_frame(_u8p(out), width, height, pitch, seed, nshapes, float(sigma),
                        1 if gradient else 0)
    if pad_garbage and pitch > width:
        _load().synth_pad_garbage(_u8p(out), width, height, pitch, seed * 7919 + 1)
    return out


def scene(width: int, height: int, seed: int, nshapes: int) -> np.ndarray:
    """Noise-free scene (background and shapes), (height, width) uint8."""
    out = np.zeros((height, width), dtype=np.uint8)
    _load().synth_scene(_u8p(out), width, height, width, seed, nshapes)
    return out


def crop_noise(scene_img: np.ndarray, ox: int, oy: int, width: int, height: int,
               seed: int, sigma: float, pitch: int | None = None) -> np.ndarray:
    """A camera frame cropped from a resident scene at (ox, oy) with fresh noise."""
    pitch = pitch_for(width) if pitch is None else pitch
    sh, sw = scene_img.shape
    src = np.ascontiguousarray(scene_img)
    out = np.zeros((height, pitch), dtype=np.uint8)
    _load().synth_crop_noise(_u8p(src), sw, sh, sw, ox, oy, _u8p(out), width, height, pitch,
                             seed, float(sigma))
    return out


def ints(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int32)
    _load().synth_ints(seed, n, lo, hi, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return out


def units(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    _load().synth_units(seed, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def raw(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    _load().synth_raw(seed, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

@dataclass
class FrameSpec:
    """One detection request: frame recipe plus detector parameters."""
    width: int
    height: int
    levels: int
    t: int
    n: int
    cell: int
    seed: int
    nshapes: int
    sigma: float
    gradient: bool = False

    def make(self, pad_garbage: bool = False) -> np.ndarray:
        return frame(self.width, self.height, self.seed, self.nshapes, self.sigma,
                     self.gradient, pad_garbage=pad_garbage)

    @property
    def pixels(self) -> int:
        return self.width * self.height


PLAIN_320 = FrameSpec(320, 240, 1, 10, 9, 32, seed=1, nshapes=60, sigma=4.0)
PLAIN_752 = FrameSpec(752, 480, 3, 10, 10, 32, seed=2, nshapes=120, sigma=4.0)
PLAIN_1080 = FrameSpec(1920, 1080, 4, 15, 9, 64, seed=3, nshapes=400, sigma=6.0, gradient=True)

BATCH_T = (8, 10, 15, 20)
BATCH_N = (9, 10, 12)
BATCH_CELL = (16, 32, 64)


def batch64(instance: int = 0) -> list[FrameSpec]:
    """The uneven 64-frame batch: 24 x 752x480, 24 x 1280x720, 16 x 640x480, all
    with 3 pyramid levels; per-frame t, N, cell drawn from small sets; frame order
    shuffled by a master seed.  ``instance`` selects a distinct resident copy
    (different frame seeds, same shapes and parameters)."""
    sizes = [(752, 480)] * 24 + [(1280, 720)] * 24 + [(640, 480)] * 16
    u = units(4, 64 * 4)
    order = np.argsort(u[0::4], kind="stable")
    specs = []
    for j, src in enumerate(order):
        w, h = sizes[src]
        t = BATCH_T[int(u[4 * j + 1] * len(BATCH_T))]
        n = BATCH_N[int(u[4 * j + 2] * len(BATCH_N))]
        cell = BATCH_CELL[int(u[4 * j + 3] * len(BATCH_CELL))]
        specs.append(FrameSpec(w, h, 3, t, n, cell, seed=4000 + j + 100000 * instance,
                               nshapes=120, sigma=4.0))
    return specs


STREAM_SIZES = ((640, 480), (752, 480), (1920, 1080), (4096, 2160))


@dataclass
class StreamSpec:
    """One simulated camera: a resident scene, detector parameters and a rate."""
    index: int
    width: int
    height: int
    levels: int
    t: int
    n: int
    cell: int
    rate_fps: float
    seed: int
    nshapes: int = 200
    sigma: float = 4.0
    scene_img: np.ndarray | None = field(default=None, repr=False)

    def make_scene(self) -> np.ndarray:
        if self.scene_img is None:
            self.scene_img = scene(self.width + 16, self.height + 16, self.seed, self.nshapes)
        return self.scene_img

    def frame(self, k: int) -> np.ndarray:
        """Frame k: crop at (8+dx, 8+dy) with dx, dy uniform in [-8, 8], fresh noise."""
        sc = self.make_scene()
        d = ints(self.seed * 1_000_003 + k, 2, -8, 8)
        return crop_noise(sc, 8 + int(d[0]), 8 + int(d[1]), self.width, self.height,
                          seed=self.seed * 7_368_787 + k, sigma=self.sigma)


def streams32() -> list[StreamSpec]:
    """32 simulated cameras with mixed resolutions, 3-5 levels, per-stream t/N/cell
    and Poisson rates of 100-1000 frames per second."""
    u = units(5, 32 * 5)
    out = []
    for s in range(32):
        w, h = STREAM_SIZES[s % 4]
        levels = 3 + int(u[5 * s] * 3)
        t = BATCH_T[int(u[5 * s + 1] * len(BATCH_T))]
        n = BATCH_N[int(u[5 * s + 2] * len(BATCH_N))]
        cell = BATCH_CELL[int(u[5 * s + 3] * len(BATCH_CELL))]
        rate = 100.0 + 900.0 * u[5 * s + 4]
        out.append(StreamSpec(s, w, h, levels, t, n, cell, rate, seed=5000 + s))
    return out
