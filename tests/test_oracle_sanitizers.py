"""Both CPU oracles built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and run through their full pin suites: an out-of-bounds
read, a signed overflow or a misaligned access anywhere on the paths the pins
exercise fails the run, on top of the pins' own checks."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def _runtime(name: str) -> str:
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else ""


@pytest.mark.slow
def test_oracle_pins_clean_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if not asan:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    flags = ["-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    libs = {}
    for src, env_name in (("fastref.c", "FASTREF_LIB"), ("lkref.c", "LKREF_LIB")):
        out = tmp_path / ("san_" + src.replace(".c", ".so"))
        subprocess.run(["gcc", *flags, "-o", str(out), os.path.join(ORACLE, src), "-lm"], check=True)
        libs[env_name] = str(out)
    env = dict(os.environ, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", **libs)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_lk_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    log = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, log
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, log
    assert " passed" in r.stdout
