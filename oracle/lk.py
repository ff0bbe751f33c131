"""Python access to the Lucas-Kanade tracker oracle ``liblkref.so`` (TEST
INFRASTRUCTURE ONLY; Section II-E).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  Host numpy arrays in and out.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LKREF_LIB lets the mutation test load a deliberately broken copy.
LIB_PATH = os.environ.get("LKREF_LIB") or os.path.join(_HERE, "liblkref.so")

GAIN = 1
OFFSET = 2
TRACKED, TEMPLATE_OUTSIDE, LOST_OUTSIDE, SINGULAR = 0, 1, 2, 3


class _Plane(ctypes.Structure):
    _fields_ = [("data", ctypes.POINTER(ctypes.c_uint8)), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("pitch", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        pp = ctypes.POINTER(_Plane)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.lkref_track.argtypes = [pp, pp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_double,
                                    ctypes.c_double, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                    ctypes.POINTER(ctypes.c_int)]
        lib.lkref_track.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_patch(levels: int) -> list[int]:
    """16x16 patches on levels 0 and 1, 8x8 above (Section II-E: larger patches
    on the finer levels)."""
    return [16 if k < 2 else 8 for k in range(levels)]


def _planes(levels):
    """levels: a list of 2-D uint8 arrays (one per pyramid level) or of
    (array, width) pairs as returned by ``oracle.pyr_build``."""
    keep, out = [], (_Plane * len(levels))()
    for k, lv in enumerate(levels):
        arr, w = (lv if isinstance(lv, tuple) else (lv, lv.shape[1]))
        arr = np.ascontiguousarray(arr, dtype=np.uint8)
        keep.append(arr)
        out[k] = _Plane(arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), w, arr.shape[0], arr.shape[1])
    return out, keep


def track(tpl_levels, img_levels, feats, q0=None, mode: int = GAIN | OFFSET, patch=None,
          max_iter: int = 30, eps: float = 0.01):
    """Track every feature (N x 2 level-0 template positions) from the template
    pyramid into the current one.  Returns (q, status, iters): q is N x 4
    (tx, ty, alpha, beta) with the translation in level-0 pixels."""
    lib = _load()
    levels = len(tpl_levels)
    assert len(img_levels) == levels
    tp, keep_t = _planes(tpl_levels)
    ip, keep_i = _planes(img_levels)
    feats = np.asarray(feats, dtype=np.float64).reshape(-1, 2)
    n = len(feats)
    q0 = np.zeros((n, 4)) if q0 is None else np.asarray(q0, dtype=np.float64).reshape(n, 4)
    patch = default_patch(levels) if patch is None else list(patch)
    pa = (ctypes.c_int * levels)(*patch)
    q = np.zeros((n, 4))
    status = np.zeros(n, dtype=np.int32)
    iters = np.zeros(n, dtype=np.int32)
    qin = (ctypes.c_double * 4)()
    qout = (ctypes.c_double * 4)()
    it = ctypes.c_int()
    for i in range(n):
        for j in range(4):
            qin[j] = q0[i, j]
        st = lib.lkref_track(tp, ip, levels, pa, float(feats[i, 0]), float(feats[i, 1]), qin, mode,
                             max_iter, eps, qout, ctypes.byref(it))
        if st < 0:
            raise ValueError("lkref_track rejected its arguments")
        status[i] = st
        iters[i] = it.value
        q[i] = list(qout)
    del keep_t, keep_i
    return q, status, iters
