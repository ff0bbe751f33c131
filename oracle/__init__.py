"""Python access to the CPU oracle ``libfastref.so`` (TEST INFRASTRUCTURE ONLY).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and shares
no code with it.  Every function takes and returns host numpy arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FASTREF_LIB lets the mutation test load a deliberately broken copy.
LIB_PATH = os.environ.get("FASTREF_LIB") or os.path.join(_HERE, "libfastref.so")

FEATURE_DTYPE = np.dtype([("x", "<u2"), ("y", "<u2"), ("score", "<u2"),
                          ("level", "u1"), ("reserved", "u1")])


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
        lib.fastref_pyr_build.argtypes = [pp, ctypes.c_int]
        lib.fastref_arc.argtypes = [ctypes.c_uint32, ctypes.c_int]
        lib.fastref_score_at.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int]
        lib.fastref_score_map.argtypes = [pp, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_uint16)]
        lib.fastref_nms_mask.argtypes = [ctypes.POINTER(ctypes.c_uint16), ctypes.c_int,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_uint8)]
        lib.fastref_detect_grid.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_void_p]
        lib.fastref_score_kind_at.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int]
        lib.fastref_score_map_kind.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_uint16)]
        lib.fastref_detect_grid_kind.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.fastref_nms_mask_radius.argtypes = [ctypes.POINTER(ctypes.c_uint16), ctypes.c_int,
                                                ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8)]
        lib.fastref_detect_grid_nms.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        for f in (lib.fastref_pyr_build, lib.fastref_arc, lib.fastref_score_at,
                  lib.fastref_score_map, lib.fastref_nms_mask, lib.fastref_detect_grid,
                  lib.fastref_score_kind_at, lib.fastref_score_map_kind, lib.fastref_detect_grid_kind,
                  lib.fastref_nms_mask_radius, lib.fastref_detect_grid_nms):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _plane(arr: np.ndarray, width: int | None = None) -> _Plane:
    assert arr.dtype == np.uint8 and arr.ndim == 2 and arr.flags["C_CONTIGUOUS"]
    h, pitch = arr.shape
    w = pitch if width is None else width
    return _Plane(arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), w, h, pitch)


def level_dims(width: int, height: int, levels: int) -> list[tuple[int, int]]:
    dims = [(width, height)]
    for _ in range(1, levels):
        w, h = dims[-1]
        dims.append((w // 2, h // 2))
    return dims


def pyr_build(img: np.ndarray, width: int, levels: int) -> list[tuple[np.ndarray, int]]:
    """Return [(plane, width)] for levels 0..levels-1; plane k is (h_k, w_k) uint8
    (level 0 is the input array itself, with its pitch)."""
    h = img.shape[0]
    dims = level_dims(width, h, levels)
    planes = [(np.ascontiguousarray(img), width)]
    for k in range(1, levels):
        w, hh = dims[k]
        planes.append((np.zeros((max(hh, 1), max(w, 1)), np.uint8), w))
    arr = (_Plane * levels)(*[_plane(p, w) for p, w in planes])
    for k in range(1, levels):
        arr[k].height = dims[k][1]
    rc = _load().fastref_pyr_build(arr, levels)
    if rc != 0:
        raise ValueError(f"fastref_pyr_build failed ({rc})")
    return planes


def arc(mask16: int, n: int) -> bool:
    return bool(_load().fastref_arc(mask16, n))


# Score kinds (Section II-D): whole-circle sum, arc sum, maximum threshold.
SCORE_SADB, SCORE_SADA, SCORE_MT = 0, 1, 2


def score_at(img: np.ndarray, width: int, x: int, y: int, t: int, n: int,
             kind: int = SCORE_SADB) -> int:
    p = _plane(img, width)
    if kind == SCORE_SADB:
        return int(_load().fastref_score_at(ctypes.byref(p), x, y, t, n))
    return int(_load().fastref_score_kind_at(ctypes.byref(p), x, y, t, n, kind))


def score_map(img: np.ndarray, width: int, t: int, n: int, kind: int = SCORE_SADB) -> np.ndarray:
    p = _plane(img, width)
    out = np.zeros((img.shape[0], width), np.uint16)
    rc = _load().fastref_score_map_kind(ctypes.byref(p), t, n, kind,
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)))
    if rc != 0:
        raise ValueError(f"fastref_score_map failed ({rc})")
    return out


def nms_mask(score: np.ndarray, radius: int = 1) -> np.ndarray:
    s = np.ascontiguousarray(score, dtype=np.uint16)
    h, w = s.shape
    out = np.zeros((h, w), np.uint8)
    rc = _load().fastref_nms_mask_radius(s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)), w, h,
                                         radius, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != 0:
        raise ValueError(f"fastref_nms_mask failed ({rc})")
    return out


def grid_dims(width: int, height: int, cell: int) -> tuple[int, int]:
    return (width + cell - 1) // cell, (height + cell - 1) // cell


def detect_grid_levels(planes: list[tuple[np.ndarray, int]], t: int, n: int,
                       cell: int, kind: int = SCORE_SADB, radius: int = 1) -> np.ndarray:
    """Cell slots for an already-built pyramid [(plane, width)]."""
    levels = len(planes)
    arr = (_Plane * levels)(*[_plane(p, w) for p, w in planes])
    gw, gh = grid_dims(planes[0][1], planes[0][0].shape[0], cell)
    out = np.zeros(gw * gh, FEATURE_DTYPE)
    rc = _load().fastref_detect_grid_nms(arr, levels, t, n, cell, kind, radius, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"fastref_detect_grid failed ({rc})")
    return out


def detect_grid(img: np.ndarray, width: int, levels: int, t: int, n: int,
                cell: int, kind: int = SCORE_SADB,
                radius: int = 1) -> tuple[np.ndarray, list[tuple[np.ndarray, int]]]:
    """Build the pyramid, then select one feature per cell.  Returns (slots, planes)."""
    planes = pyr_build(img, width, levels)
    return detect_grid_levels(planes, t, n, cell, kind, radius), planes
