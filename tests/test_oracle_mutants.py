"""Mutation check of the oracle's pins: plant one plausible mistake at a time in
a private copy of the oracle source (on the CPU), rebuild it, and require the
pin suite to fail against it.  A mutant that survives would mean the pins
cannot tell that mistake from the definition."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fastref.c")

MUTANTS = {
    "bright_non_strict": ("if (p > c + t) {", "if (p >= c + t) {"),
    "dark_non_strict": ("} else if (p < c - t) {", "} else if (p <= c - t) {"),
    "bright_sum_drops_t": ("sum_bright += p - c - t;", "sum_bright += p - c;"),
    "score_sum_not_max": ("return sum_bright > sum_dark ? sum_bright : sum_dark;",
                          "return sum_bright + sum_dark;"),
    "circle_order_swapped": ("CIRCLE_DX[16] = {0, 1, 2, 3,", "CIRCLE_DX[16] = {1, 0, 2, 3,"),
    "arc_not_circular": ("((s + j) % 16)", "((s + j) < 16 ? (s + j) : 15)"),
    "pyramid_no_rounding": ("(uint8_t)((a + b + c + d + 2) >> 2)", "(uint8_t)((a + b + c + d) >> 2)"),
    "nms_tie_reversed": ("return ia < ib;", "return ia > ib;"),
    "level_tie_reversed": ("else if (k != f->level) better = k < f->level;",
                           "else if (k != f->level) better = k > f->level;"),
    "border_off_by_one": ("x > img->width - 4", "x > img->width - 3"),
    "no_level_scale_up": ("long cx = ((long)x << k) / cell", "long cx = (long)x / cell"),
    "nms_skips_diagonals": ("if (dx == 0 && dy == 0) continue;",
                            "if (dx == 0 || dy == 0) { if (dx == 0 && dy == 0) continue; } else continue;"),
    "arc_sum_counts_off_arc": ("if (on_arc(bright, n, i)) arc_bright", "if ((bright >> i) & 1u) arc_bright"),
    "arc_sum_drops_dark": ("return arc_bright > arc_dark ? arc_bright : arc_dark;", "return arc_bright;"),
    "max_threshold_off_by_one": ("return d > t ? d : 0;", "return d > t ? d - 1 : 0;"),
    "nms_radius_ignored": ("for (int dx = -r; dx <= r && keep; ++dx) {", "for (int dx = -1; dx <= 1 && keep; ++dx) {"),
    "max_threshold_short_window": ("            int q = v[(s + j) % 16];", "            if (j == n - 1) break;\n            int q = v[(s + j) % 16];"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_kill_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "fastref.c"
    mut.write_text(src.replace(old, new))
    (tmp_path / "fastref.h").write_text(open(os.path.join(ROOT, "oracle", "fastref.h")).read())
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-o", str(lib), str(mut)], check=True)
    env = dict(os.environ, FASTREF_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
