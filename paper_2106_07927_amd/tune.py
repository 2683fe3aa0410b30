"""Autotuner for the batched form, in two stages, both written into the JSON
table that sgm_batch_plan_create takes:

* per frame shape (W, H, D): the path-kernel lane-layout variant that runs
  fastest, each candidate timed as a one-frame batch plan;
* per batch: "chains", the number of streams inside the graph over which
  the frames of 100k pixels and more are spread (frames on different streams
  overlap, which fills the compute units that one frame's path pass leaves
  idle in its tail), each candidate timed as the whole batch plan.

Every choice computes identical results (the batch tests check that), so
tuning only changes speed.  Timing uses HIP events on the current stream.

    python -m paper_2106_07927_amd.tune 1242x375x128 1920x1080x256 ...
"""
from __future__ import annotations

import json
import sys

import numpy as np
import torch

from . import datagen, sgm


def variants(ndisp: int) -> int:
    return int(sgm.load_library().sgm_aggregate_variants(ndisp))


def time_variant(left, right, ndisp, params, variant, reps=5) -> float:
    """Milliseconds per run of a one-frame plan forced to `variant`."""
    key = f"{left.shape[1]}x{left.shape[0]}x{ndisp}"
    plan = sgm.BatchPlan([left], [right], [ndisp], params, tune_table=json.dumps({key: variant}))
    try:
        plan.run()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            plan.run()
        end.record()
        torch.cuda.synchronize()
        return start.elapsed_time(end) / reps
    finally:
        plan.close()


def tune(shapes, params: sgm.Params, device="cuda", reps=5, seed=7):
    """shapes: iterable of (W, H, D).  Returns (table dict, timings dict)."""
    table, timings = {}, {}
    for (w, h, nd) in sorted(set(shapes)):
        a, b = datagen.random_images(w, h, seed)
        left = torch.from_numpy(a).to(device)
        right = torch.from_numpy(b).to(device)
        ms = [time_variant(left, right, nd, params, v, reps) for v in range(variants(nd))]
        key = f"{w}x{h}x{nd}"
        table[key] = int(np.argmin(ms))
        timings[key] = [round(t, 4) for t in ms]
    return table, timings


def time_plan(lefts, rights, ndisps, params, table: dict, reps=3) -> float:
    """Milliseconds per run of the whole batch under `table`."""
    plan = sgm.BatchPlan(lefts, rights, ndisps, params, tune_table=json.dumps(table))
    try:
        plan.run()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            plan.run()
        end.record()
        torch.cuda.synchronize()
        return start.elapsed_time(end) / reps
    finally:
        plan.close()


def tune_chains(lefts, rights, ndisps, params: sgm.Params, table: dict, choices=(1, 2, 3, 4),
                reps=3):
    """Adds the fastest "chains" for this batch to a copy of `table`; returns
    (table, {chains: ms})."""
    ms = {c: round(time_plan(lefts, rights, ndisps, params, {**table, "chains": c}, reps), 4)
          for c in choices}
    best = min(ms, key=ms.get)
    return {**table, "chains": int(best)}, ms


def main(argv):
    shapes = [tuple(int(v) for v in a.split("x")) for a in argv] or [(1242, 375, 128)]
    table, timings = tune(shapes, sgm.Params(ndisp=0))
    print(json.dumps({"table": table, "ms": timings}))


if __name__ == "__main__":
    main(sys.argv[1:])
