"""The library's device code contains no packed FP32 additions, multiplies or
FMAs: each HIP source is compiled for gfx950 with the library's own flags to
AMD assembly (device pass only) and searched.  Without the flag that disables
them, hipcc -O3 turns plain float2 arithmetic into such instructions."""
import os
import re
import subprocess

import pytest

from paper_2003_13493_amd import build

PACKED_FP32 = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")


def device_asm(src: str, flags: list[str]) -> str:
    keep = [f for f in flags if f not in ("-shared", "-fPIC")]
    cmd = [build._hipcc(), *keep, "--cuda-device-only", "-S", "-o", "-", "-I", build.INCLUDE,
           "-I", build.CSRC, src]
    return subprocess.run(cmd, check=True, capture_output=True, text=True).stdout


@pytest.mark.slow
@pytest.mark.parametrize("name", build.HIP_SOURCES)
def test_no_packed_fp32_in_device_code(name):
    asm = device_asm(os.path.join(build.CSRC, name), build.HIPCC_FLAGS)
    assert "amdgcn" in asm                     # a device pass ran (the runtime has no kernels)
    assert not PACKED_FP32.search(asm), PACKED_FP32.search(asm).group(0)


@pytest.mark.slow
def test_the_flag_is_what_removes_them(tmp_path):
    """The check above can fail: the same float2 FMA compiles to v_pk_fma_f32
    without the flag and to scalar FMAs with it."""
    src = tmp_path / "probe.hip"
    src.write_text("#include <hip/hip_runtime.h>\n"
                   "__global__ void k(float2 *a, const float2 *b, float s) {\n"
                   "  int i = threadIdx.x; float2 x = a[i], y = b[i];\n"
                   "  x.x = x.x * s + y.x; x.y = x.y * s + y.y; a[i] = x; }\n")
    without = [f for f in build.HIPCC_FLAGS if f not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
    assert PACKED_FP32.search(device_asm(str(src), without))
    assert not PACKED_FP32.search(device_asm(str(src), build.HIPCC_FLAGS))
