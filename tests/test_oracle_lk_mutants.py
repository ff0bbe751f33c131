"""Mutation check of the Lucas-Kanade oracle's pins: plant one plausible
mistake at a time in a private copy of ``oracle/lkref.c`` (on the CPU),
rebuild it, and require the LK pin suite to fail against it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lkref.c")

MUTANTS = {
    "translation_update_sign": ("tkx -= dq[0];", "tkx += dq[0];"),
    "offset_update_sign": ("beta += dq[3];", "beta -= dq[3];"),
    "gain_update_sign": ("alpha += dq[2];", "alpha -= dq[2];"),
    "u_drops_gain_factor": ("u[0] = g * gx;", "u[0] = gx;"),
    "gradient_not_halved": ("const double gx = 0.5 * (", "const double gx = ("),
    "gradient_axes_swapped": ("const double gy = 0.5 * (bilinear(Tk, x, y + 1) - bilinear(Tk, x, y - 1));",
                              "const double gy = 0.5 * (bilinear(Tk, x + 1, y) - bilinear(Tk, x - 1, y));"),
    "residual_sign": ("const double r = bilinear(Ik, x + tkx, y + tky) - (1.0 + alpha) * T[j * S + i] - beta;",
                      "const double r = (1.0 + alpha) * T[j * S + i] + beta - bilinear(Ik, x + tkx, y + tky);"),
    "residual_drops_gain": ("- (1.0 + alpha) * T[j * S + i] - beta;", "- T[j * S + i] - beta;"),
    "residual_patch_shifted": ("const double x = px + (i - half), y = py + (j - half);\n                    const double r",
                               "const double x = px + (i - half + 1), y = py + (j - half);\n                    const double r"),
    "no_doubling_between_levels": ("tx = tkx * scale;\n        ty = tky * scale;", "tx = tkx;\n        ty = tky;"),
    "feature_not_scaled": ("const double px = fx / scale, py = fy / scale;", "const double px = fx, py = fy;"),
    "never_stops_early": ("if (dq[0] * dq[0] + dq[1] * dq[1] < eps * eps) break;", ""),
    "bilinear_weights_swapped": ("const double top = (1.0 - ax) * r0[0] + ax * r0[1];",
                                 "const double top = ax * r0[0] + (1.0 - ax) * r0[1];"),
    "image_far_corner_unchecked": ("if (!usable(Ik, px - half + tkx, py - half + tky) ||\n"
                                   "                !usable(Ik, px + half - 1 + tkx, py + half - 1 + tky)) {",
                                   "if (!usable(Ik, px - half + tkx, py - half + tky)) {"),
    "singular_check_dropped": ("if (!(s > 1e-6 * H[i][i])) return 1;", ""),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_lk_pins_kill_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "lkref.c"
    mut.write_text(src.replace(old, new))
    (tmp_path / "lkref.h").write_text(open(os.path.join(ROOT, "oracle", "lkref.h")).read())
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, LKREF_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_lk_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
