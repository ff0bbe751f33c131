"""Launch-shape autotuner.

Two tables come out of a tuning run on the device:

* one-frame calls (fast_detect_grid*, fast_score_maps, fast_nms_grid): per
  frame shape (width, height, levels, cell), the side of the square region a
  workgroup owns.  A small frame wants small regions (more workgroups than the
  chip has compute units), a large one wants large regions (less halo).  The
  table is handed to the library with fast_set_shape_table; shapes without an
  entry keep the library's default rule;
* batched submissions and resident plans: the workgroup size and the number of
  persistent workgroups per compute unit, tuned on the batch workload.

Every candidate is first run once and its output compared bit for bit with
the expected answer for the same frames, which the caller supplies (the
tuning driver, tests/tune_table.py, takes it from the CPU oracle); only
candidates that match are timed, so a shape that would change a result can
never be chosen.  Timing is the mean of back-to-back launches, measured with
device events.

The result is JSON; `apply` loads it into a context, and `Context` in the
binding does so at creation when a table tuned on the same device kind is
shipped next to the library (`TABLE_PATH`).
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import fastgrid

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")

PLAIN_REGIONS = (16, 32, 64, 128, 256)
BATCH_CANDIDATES = [(256, 2), (256, 3), (256, 4), (320, 3), (384, 2), (448, 2), (512, 1), (512, 2),
                    (128, 4), (128, 6)]
DEFAULT_BATCH = (256, 3)


def signature(specs) -> str:
    """A stable key for a workload: the set of (W, H, levels, cell)."""
    keys = sorted({(s.width, s.height, s.levels, s.cell) for s in specs})
    return ";".join(f"{w}x{h}L{l}c{c}" for w, h, l, c in keys)


def choose(candidates, run, timer, want, log=None):
    """Gate, then time.  run(c) -> outputs of candidate c (or raises
    fastgrid.FastError for a shape the library refuses); want: the expected
    outputs; timer(c) -> ms.  A candidate is timed only if every output equals
    the expected one.  Returns (rows, best row or None)."""
    rows = []
    for c in candidates:
        try:
            got = run(c)
        except fastgrid.FastError as e:
            rows.append({"candidate": list(c), "exact": False, "error": str(e)})
            continue
        exact = len(got) == len(want) and all(np.array_equal(a, b) for a, b in zip(got, want))
        row = {"candidate": list(c), "exact": exact}
        if exact:
            row["ms"] = float(timer(c))
        rows.append(row)
        if log:
            log(f"tune {c}: exact={exact} ms={row.get('ms')}")
    timed = [r for r in rows if r["exact"] and "ms" in r]
    return rows, (min(timed, key=lambda r: r["ms"]) if timed else None)


def _events_ms(fn, reps: int, warmup: int) -> float:
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_shapes(ctx: fastgrid.Context, cases, regions=PLAIN_REGIONS, reps: int = 100, warmup: int = 10,
                log=None) -> list[dict]:
    """Per frame shape, the fastest exact region side of one-frame calls.
    cases: (spec, img, want) with spec a FrameSpec-like object (width, height,
    levels, t, n, cell), img its frame and want the expected slots.
    The context's table is left holding every tuned shape."""
    import torch
    out = []
    tuned = []
    for spec, img, want in cases:
        pyr = fastgrid.Pyramid(spec.width, spec.height, spec.levels)
        pyr.upload(img)
        grid = fastgrid.Grid(spec.width, spec.height, spec.cell)
        key = (spec.width, spec.height, spec.levels, spec.cell)
        # candidates that round to the same side are the same candidate
        sides = []
        for r in regions:
            ctx.set_shape_table(tuned + [key + (r,)])
            side = ctx.shape_region(*key)
            if side not in sides:
                sides.append(side)

        def run(c):
            ctx.set_shape_table(tuned + [key + (c[0],)])
            grid.tensor.fill_(0xA5)
            ctx.detect(pyr, spec.t, spec.n, spec.cell, grid)
            torch.cuda.synchronize()
            return [grid.fetch()]

        def timer(c):
            ctx.set_shape_table(tuned + [key + (c[0],)])
            return _events_ms(lambda s: ctx.detect(pyr, spec.t, spec.n, spec.cell, grid, s), reps, warmup)

        rows, best = choose([(s,) for s in sides], run, timer, [want], log)
        region = best["candidate"][0] if best else None
        if region is not None:
            tuned.append(key + (region,))
        out.append({"width": spec.width, "height": spec.height, "levels": spec.levels, "cell": spec.cell,
                    "region": region, "us": round(best["ms"] * 1e3, 2) if best else None,
                    "candidates": [{"region": r["candidate"][0], "exact": r["exact"],
                                    "us": round(r["ms"] * 1e3, 2) if "ms" in r else None} for r in rows]})
    ctx.set_shape_table(tuned)
    return out


def tune_batch(ctx: fastgrid.Context, specs, frames, want, candidates=None, reps: int = 50, warmup: int = 5,
               log=None) -> dict:
    """The fastest exact (block, workgroups per CU) of the batched kernel on a
    workload (want: the expected slots of every frame); the context is left
    at it."""
    import torch
    candidates = list(candidates or BATCH_CANDIDATES)
    pyrs, grids = [], []
    for s, img in zip(specs, frames):
        p = fastgrid.Pyramid(s.width, s.height, s.levels)
        p.upload(img)
        pyrs.append(p)
        grids.append(fastgrid.Grid(s.width, s.height, s.cell))
    jobs = fastgrid.Context.make_jobs((p, s.t, s.n, s.cell, g) for p, s, g in zip(pyrs, specs, grids))

    def run(c):
        ctx.set_launch(0, *c)
        for g in grids:
            g.tensor.fill_(0xA5)
        torch.cuda.synchronize()
        tk = ctx.submit(jobs)
        ctx.wait(tk)
        return [g.fetch() for g in grids]

    def timer(c):
        ctx.set_launch(0, *c)
        pid = ctx.plan_create(jobs)
        try:
            return _events_ms(lambda s: ctx.plan_launch(pid, s, ticket=False), reps, warmup)
        finally:
            ctx.plan_destroy(pid)

    rows, best = choose(candidates, run, timer, want, log)
    shape = best["candidate"] if best else list(DEFAULT_BATCH)
    ctx.set_launch(0, *shape)
    return {"signature": signature(specs), "block": shape[0], "blocks_per_cu": shape[1],
            "ms": best["ms"] if best else None,
            "candidates": [{"block": r["candidate"][0], "blocks_per_cu": r["candidate"][1], "exact": r["exact"],
                            "ms": r.get("ms")} for r in rows]}


def apply(ctx: fastgrid.Context, table: dict) -> None:
    """Load a tuning result into a context: the shape table of one-frame calls
    and the batched kernel's workgroup size and occupancy."""
    ctx.set_shape_table([(e["width"], e["height"], e["levels"], e["cell"], e["region"])
                         for e in table.get("shapes", []) if e.get("region")])
    b = table.get("batch")
    if b:
        ctx.set_launch(0, b["block"], b["blocks_per_cu"])


def load(path: str = TABLE_PATH, device: str | None = None) -> dict | None:
    """The table at path, or None if it is missing or was tuned on another
    device kind than `device` (a gfx name; None accepts any)."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    if device is not None and table.get("device") != device:
        return None
    return table


def default_shapes():
    """The frame shapes the shipped table covers: the one-frame workloads, the
    batch frames at every batch cell size, and the serving streams' shapes."""
    from . import synth
    out, seen = [], set()

    def add(spec):
        key = (spec.width, spec.height, spec.levels, spec.cell)
        if key not in seen:
            seen.add(key)
            out.append(spec)

    for s in (synth.PLAIN_320, synth.PLAIN_752, synth.PLAIN_1080):
        add(s)
    for s in synth.batch64():
        for cell in synth.BATCH_CELL:
            add(synth.FrameSpec(s.width, s.height, s.levels, s.t, s.n, cell, seed=s.seed, nshapes=s.nshapes,
                                sigma=s.sigma))
    for st in synth.streams32():
        add(synth.FrameSpec(st.width, st.height, st.levels, st.t, st.n, st.cell, seed=st.seed,
                            nshapes=st.nshapes, sigma=st.sigma))
    return out
