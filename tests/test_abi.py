"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, and the pure host helpers behave (no GPU compute here)."""
import ctypes
import os
import re

import pytest

from paper_2003_13493_amd import fastgrid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fastgrid.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fast_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(fastgrid.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = fastgrid.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_library_exports_nothing_else():
    """Only the fast_* ABI is visible from the shared object."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", fastgrid.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert {s for s in syms if s.startswith("fast_")} == set(declared_functions())


def test_struct_layouts():
    assert ctypes.sizeof(fastgrid.fast_plane) == 24
    assert fastgrid.FEATURE_DTYPE.itemsize == 8
    assert ctypes.sizeof(fastgrid.fast_job) == 40
    assert ctypes.sizeof(fastgrid.fast_shape_region) == 20
    assert ctypes.sizeof(fastgrid.fast_pump_stream) == 64
    assert ctypes.sizeof(fastgrid.fast_pump_request) == 16
    assert ctypes.sizeof(fastgrid.fast_pump_frontend) == 72


def test_pyr_and_grid_dims():
    assert fastgrid.fast_pyr_dims(1920, 1080, 4) == [(1920, 1080, 1920), (960, 540, 960),
                                                     (480, 270, 512), (240, 135, 256)]
    assert fastgrid.fast_pyr_dims(752, 480, 3) == [(752, 480, 768), (376, 240, 384),
                                                   (188, 120, 192)]
    assert fastgrid.fast_grid_dims(752, 480, 32) == (24, 15)
    assert fastgrid.fast_grid_dims(1920, 1080, 64) == (30, 17)
    with pytest.raises(fastgrid.FastError):
        fastgrid.fast_pyr_dims(5, 5, 4)          # level 3 would be 0x0
    with pytest.raises(fastgrid.FastError):
        fastgrid.fast_pyr_dims(100, 100, 9)


def test_strerror_and_null_context():
    lib = fastgrid.load()
    assert lib.fast_strerror(0) == b"success"
    assert lib.fast_strerror(-5) == b"timed out"
    assert lib.fast_detect_grid(None, None, 1, 10, 9, 32, None, None) == fastgrid.FAST_EINVAL
    assert lib.fast_poll(None, 1) == fastgrid.FAST_EINVAL
    out = ctypes.c_void_p()
    assert lib.fast_ctx_create(0, None) == fastgrid.FAST_EINVAL
