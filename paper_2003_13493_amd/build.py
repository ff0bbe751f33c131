"""In-tree build of the native parts of the package.

* ``csrc/*.hip``   -> ``libfastgrid.so``  (hipcc, gfx950 only)
* ``synth/frames.c`` -> ``synth/libsynth.so`` (gcc; input synthesis only)

Every call recompiles.  The libraries land next to their sources so they travel
with the source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")

HIP_SOURCES = ["fastgrid_kernels.hip", "fasttrack_kernels.hip", "fastgrid_runtime.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # no packed-FP32 instructions (v_pk_add/mul/fma_f32) in the device code.
    # The device pass honours this feature (tests/test_build_flags.py shows a
    # float2 FMA becoming v_pk_fma_f32 without it and two FMAs with it); the
    # host pass does not know it and warns that it ignores it
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no atomic optimiser: its wave-level rewrite of a one-lane atomic reads
    # the result right after issuing it, which would put the work queue's
    # ticket latency on the persistent kernel's critical path
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-fvisibility=hidden",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build_synth(verbose: bool = False) -> str:
    src = os.path.join(HERE, "synth", "frames.c")
    out = os.path.join(HERE, "synth", "libsynth.so")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build_fastgrid(verbose: bool = False, extra: list[str] | None = None) -> str:
    out = os.path.join(HERE, "libfastgrid.so")
    srcs = [os.path.join(CSRC, s) for s in HIP_SOURCES]
    cmd = [_hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, *(extra or []),
           "-o", out + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build_all(verbose: bool = False) -> None:
    build_synth(verbose)
    build_fastgrid(verbose)


if __name__ == "__main__":
    build_all(verbose=True)
