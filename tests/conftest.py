import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


def as_tuples(slots: np.ndarray) -> list[tuple[int, int, int, int]]:
    return [(int(s["x"]), int(s["y"]), int(s["score"]), int(s["level"])) for s in slots]


def padded(img: np.ndarray, pitch: int | None = None) -> np.ndarray:
    """Copy an (H, W) image into an (H, pitch) array (pitch defaults to W)."""
    h, w = img.shape
    pitch = w if pitch is None else pitch
    out = np.zeros((h, pitch), np.uint8)
    out[:, :w] = img
    return out
