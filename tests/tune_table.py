"""Tuning driver: runs the launch-shape autotuner of the package on this
device, gating every candidate against the CPU oracle's answers, and writes
the table that `Context` loads at creation (package file tuned_<arch>.json).

    python tests/tune_table.py [--reps N] [--out PATH]

It lives with the tests because the gate uses the oracle, which only test
code may call.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2003_13493_amd import fastgrid, synth, tune  # noqa: E402


def oracle_slots(spec, img):
    return oracle.detect_grid(img, spec.width, spec.levels, spec.t, spec.n, spec.cell)[0]


def main(argv=None) -> int:
    import torch
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--reps", type=int, default=100)
    ap.add_argument("--out", default=tune.TABLE_PATH)
    args = ap.parse_args(argv)
    ctx = fastgrid.Context(0, tuned=False)
    log = lambda m: print(m, flush=True)   # noqa: E731
    cases = []
    for spec in tune.default_shapes():
        img = spec.make()
        cases.append((spec, img, oracle_slots(spec, img)))
    shapes = tune.tune_shapes(ctx, cases, reps=args.reps, log=log)
    specs = synth.batch64()
    frames = [s.make() for s in specs]
    batch = tune.tune_batch(ctx, specs, frames, [oracle_slots(s, f) for s, f in zip(specs, frames)],
                            reps=max(20, args.reps // 2), log=log)
    result = {"device": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
              "time": time.strftime("%Y-%m-%d %H:%M:%S"),
              "gate": "every candidate bit-exact with the CPU oracle before it is timed",
              "shapes": shapes, "batch": batch}
    with open(args.out, "w") as f:
        json.dump(result, f, indent=1)
    print(json.dumps({"shapes": [(e["width"], e["height"], e["levels"], e["cell"], e["region"], e["us"])
                                 for e in shapes],
                      "batch": [batch["block"], batch["blocks_per_cu"], batch["ms"]]}))
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
