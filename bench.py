#!/usr/bin/env python3
"""Benchmark of the SGM stereo hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

One step = one pass of the whole path over one synthetic stereo pair whose
images are already resident in HBM: census (left and right), Hamming cost,
8-path aggregation, WTA + approximate D^R + LR check + 3x3 median.  The
headline workload is a 1242x375 pair, D = 128, census 9x7, P1 = 10,
P2 = 120.  The timed path is the streamlined one (aggregation fused with the
selection, sgm_aggregate_select).

Launch mode: eager launches on one stream, a hipGraph replay, and frames in
flight (consecutive steps round-robin over 2 or 4 engines with their own
buffers and streams) are each timed over a long untimed sample; the fastest
is then timed over exactly K steps for the headline, and the eager
single-stream figure is reported beside it.

Prints ONE JSON line: throughput in MDE/s (W * H * D / step time, the
paper's Eq. mdes) and FPS; the roofline of the dominant unit
(sgm_aggregate_select, timed with HIP events on its launch stream) on the
aggregation's algorithmic bytes (R + 2) N D; the 320x240 and 1920x1080
workloads; the four-call form and the other forms; the batched form (64
mixed pairs, one hipGraph) against plain per-frame launches; the served form
(16 Poisson camera streams, continuous batching against plain FIFO); and the
CPU oracle timed on the host cores (one thread and all of them).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MDE/s and FPS at 1242x375 D=128 8-path; batched vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0
HEADLINE = "c2_1242x375_d128_r8"


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--select-steps", type=int, default=200,
                    help="untimed steps per launch mode when choosing the headline's mode")
    ap.add_argument("--cpu-frames", type=int, default=3,
                    help="frames of the single-threaded CPU-oracle sample (0 skips the CPU legs)")
    ap.add_argument("--batch-reps", type=int, default=5,
                    help="timed replays of the 64-pair batch (0 skips the batched form)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served trace (0 skips the served form)")
    ap.add_argument("--serve-short-seconds", type=float, default=10.0,
                    help="length of the tight-budget and overload traces")
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    ap.add_argument("--max-streams", type=int, default=4,
                    help="largest frames-in-flight count timed (1: single-stream modes only, "
                         "so that a kernel trace sees no overlapping frames)")
    ap.add_argument("--other-configs", type=int, default=1,
                    help="time the 320x240 and 1920x1080 workloads too (0 skips them)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the path, run a plain device copy of this many MiB five "
                         "times (the known-size kernel that scales HBM counter readings)")
    return ap.parse_args()


# Counter readings for the dominant unit at the 1242x375 / D=128 / 8-path
# frame (profiles/), per call: HBM bytes (MB) from FETCH_SIZE and WRITE_SIZE,
# each scaled by its reading for a plain copy of known size, and the VALU-busy
# share of the call's kernels (SQ_INSTS_VALU x 4 cycles over 1024 SIMDs at
# 2.4 GHz and the kernels' durations).  An entry holds only for the kernel
# sources whose digest it names; otherwise the figures are null.
COUNTERS = {
    "sgm_aggregate_select": {"sources": "627a9e995945069a", "traffic": 1474.9, "valu_busy": 0.605},
}

KERNEL_SOURCES = ("census.hip", "cost.hip", "aggregate.hip", "paths.hip", "wta_lrc.hip",
                  "sgm_internal.h")


def sources_digest():
    import hashlib
    hsh = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2106_07927_amd", "csrc", name), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()[:16]


def counters(unit, digest):
    entry = COUNTERS.get(unit)
    if entry is None or entry["sources"] != digest:
        return None, None
    return entry["traffic"], entry["valu_busy"]


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def percentile(sorted_vals, q):
    return sorted_vals[min(len(sorted_vals) - 1, int(q * len(sorted_vals)))]


def copy_probe(torch, dev, mib):
    """A plain elementwise copy of known size: reads and writes `mib` MiB per
    launch.  Its FETCH_SIZE / WRITE_SIZE readings calibrate the counters."""
    n = mib * 2 ** 20 // 4
    src = torch.arange(n, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def params_of(sgm, cfg):
    return sgm.Params(win_w=cfg["win_w"], win_h=cfg["win_h"], ndisp=cfg["ndisp"],
                      npaths=cfg["npaths"], p1=cfg["p1"], p2=cfg["p2"],
                      lr_tolerance=cfg["lr_tolerance"], median3x3=cfg["median3x3"])


def workload_desc(name, cfg):
    return (f"{name}: {cfg['width']}x{cfg['height']} uint8 pair, D={cfg['ndisp']}, census "
            f"{cfg['win_w']}x{cfg['win_h']}, {cfg['npaths']} paths, P1={cfg['p1']}, P2={cfg['p2']}, "
            f"LR tol {cfg['lr_tolerance']}, median {int(cfg['median3x3'])}")


class Frame:
    """One workload's pair on the device and the calls of one step."""

    def __init__(self, torch, sgm, datagen, name, dev):
        self.torch, self.sgm = torch, sgm
        self.name = name
        self.cfg = cfg = datagen.CONFIGS[name]
        self.w, self.h, self.nd, self.npaths = cfg["width"], cfg["height"], cfg["ndisp"], cfg["npaths"]
        self.prm = params_of(sgm, cfg)
        self.pair = datagen.config_pair(name)
        self.left = torch.from_numpy(self.pair["left"]).to(dev)
        self.right = torch.from_numpy(self.pair["right"]).to(dev)
        self.dev = dev
        self.des = self.w * self.h * self.nd

    def engine(self, fused=True):
        return self.sgm.StereoSGM(self.w, self.h, self.prm, device=self.dev, fused=fused)

    def step(self, eng, stream, ev=None, fused=True):
        """The whole path once; with `ev`, events at the stage boundaries."""
        sgm, prm = self.sgm, self.prm

        def mark(i):
            if ev is not None:
                ev[i].record(stream)
        mark(0)
        if fused:
            sgm.sgm_census_pair(self.left, self.right, prm.win_w, prm.win_h, out_left=eng.census_left,
                                out_right=eng.census_right, stream=stream)
        else:
            sgm.sgm_census(self.left, prm.win_w, prm.win_h, out=eng.census_left, stream=stream)
            sgm.sgm_census(self.right, prm.win_w, prm.win_h, out=eng.census_right, stream=stream)
        mark(1)
        sgm.sgm_cost(eng.census_left, eng.census_right, self.nd, out=eng.cost, stream=stream)
        mark(2)
        if fused:
            sgm.sgm_aggregate_select(eng.cost, self.npaths, prm.p1, prm.p2, prm.lr_tolerance,
                                     prm.median3x3, out=eng.disp, out_right=eng.disp_right,
                                     work=eng.select_work, stream=stream)
            mark(3)
        else:
            sgm.sgm_aggregate(eng.cost, self.npaths, prm.p1, prm.p2, out=eng.agg, work=eng.agg_work,
                              stream=stream)
            mark(3)
            sgm.sgm_wta_lrc(eng.agg, prm.lr_tolerance, prm.median3x3, out=eng.disp,
                            out_right=eng.disp_right, work=eng.work, stream=stream)
            mark(4)

    def stage_times(self, eng, stream, steps, fused=True):
        """Per-stage average ms and sorted per-step ms over `steps` eager steps,
        from events on the launch stream."""
        torch = self.torch
        names = ("census", "cost", "aggregate_select") if fused else \
            ("census", "cost", "aggregate", "wta_lrc")
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
               for _ in range(steps)]
        torch.cuda.synchronize()
        for i in range(steps):
            self.step(eng, stream, evs[i], fused)
        torch.cuda.synchronize()
        per_step = sorted(e[0].elapsed_time(e[-1]) for e in evs)
        stages = {nm: sum(e[a].elapsed_time(e[a + 1]) for e in evs) / steps
                  for a, nm in enumerate(names)}
        return stages, per_step

    def roofline(self, agg_ms, digest=None):
        """The aggregation's algorithmic bytes (R + 2) N D -- R reads of the
        uint8 cost volume and one uint16 write of S_bar -- over the duration of
        the sgm_aggregate_select call (paths, fused selection, check/median)."""
        b = (self.npaths + 2) * self.des
        achieved = b / (agg_ms * 1e-3) / 1e9
        traffic, valu = counters("sgm_aggregate_select", digest) if digest else (None, None)
        second = self.npaths * self.des + 4 * self.w * self.h
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "sgm_aggregate_select (paths_kernel + select_fused_kernel + "
                          "check_median_kernel)",
                "algorithmic_bytes": b, "t_agg_us": round(agg_ms * 1e3, 2),
                "basis": "(R+2)*N*D: the cost volume streamed once per path plus S_bar written "
                         "once, over the whole aggregate_select call",
                "valu_busy": valu,
                "frac_on_read_bytes": round(second / (agg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def headline(args, torch, sgm, datagen, dev):
    fr = Frame(torch, sgm, datagen, args.workload, dev)
    stream = torch.cuda.current_stream()
    eng = fr.engine()
    for _ in range(args.warmup):
        fr.step(eng, stream)
    torch.cuda.synchronize()

    def run_eager(n):
        for _ in range(n):
            fr.step(eng, stream)

    graph = eng.capture(fr.left, fr.right)

    def run_graph(n):
        for _ in range(n):
            graph.replay()

    def make_streams(k):
        engs = [fr.engine() for _ in range(k)]
        side = [torch.cuda.Stream(device=dev) for _ in range(k)]

        def run(n):
            for i in range(n):
                engs[i % k].run(fr.left, fr.right, stream=side[i % k])
        return run, engs

    modes = {"eager": run_eager, "hipgraph": run_graph}
    stream_engines = []
    for k in (2, 4):
        if k <= args.max_streams:
            run, engs = make_streams(k)
            modes[f"streams{k}"] = run
            stream_engines += engs

    def wall_ms(run, n):
        run(max(2, args.warmup // 2))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(n)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    # choose the launch mode on long untimed samples
    mode_ms = {m: wall_ms(run, args.select_steps) for m, run in modes.items()}
    mode = min(mode_ms, key=mode_ms.get)
    # the headline: exactly K steps in that mode, synchronised on both sides
    run = modes[mode]
    run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    for e in stream_engines:
        if not (torch.equal(e.disp, eng.disp) and torch.equal(e.disp_right, eng.disp_right)):
            raise RuntimeError("a frames-in-flight result differs from the single-stream one")
    # eager single stream with stage events: the dominant unit's duration
    stages, per_step = fr.stage_times(eng, stream, max(args.steps, 20))
    return fr, eng, {"mode": mode, "ms": ms, "mode_ms": mode_ms, "stages": stages,
                     "per_step": per_step}


def other_config(args, torch, sgm, datagen, dev, name, digest):
    fr = Frame(torch, sgm, datagen, name, dev)
    stream = torch.cuda.current_stream()
    eng = fr.engine()
    steps = max(20, min(args.steps, 200 if fr.des < 10 ** 8 else 30))
    for _ in range(3):
        fr.step(eng, stream)
    stages, per_step = fr.stage_times(eng, stream, steps)
    ms = sum(stages.values())
    out = {"workload": workload_desc(name, fr.cfg), "steps": steps, "ms_per_step": round(ms, 5),
           "value": round(fr.des / (ms * 1e-3) / 1e6, 1), "unit": "MDE/s",
           "fps": round(1000.0 / ms, 1), "launch": "eager",
           "stages_ms": {k: round(v, 5) for k, v in stages.items()},
           "step_ms_p50": round(percentile(per_step, 0.5), 5),
           "step_ms_p99": round(percentile(per_step, 0.99), 5),
           "roofline": fr.roofline(stages["aggregate_select"])}
    # the same frame with 4 frames in flight (engines and streams in turn)
    engs = [eng] + [fr.engine() for _ in range(3)]
    side = [torch.cuda.Stream(device=dev) for _ in range(4)]
    for i in range(8):
        engs[i % 4].run(fr.left, fr.right, stream=side[i % 4])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        engs[i % 4].run(fr.left, fr.right, stream=side[i % 4])
    torch.cuda.synchronize()
    ms4 = (time.perf_counter() - t0) * 1e3 / steps
    out["in_flight_4"] = {"ms_per_frame": round(ms4, 5), "value": round(fr.des / (ms4 * 1e-3) / 1e6, 1),
                          "fps": round(1000.0 / ms4, 1)}
    del eng, engs
    torch.cuda.empty_cache()
    return out


def four_call(args, torch, fr):
    stream = torch.cuda.current_stream()
    eng = fr.engine(fused=False)
    for _ in range(args.warmup):
        fr.step(eng, stream, fused=False)
    stages, per_step = fr.stage_times(eng, stream, max(args.steps, 20), fused=False)
    ms = sum(stages.values())
    agg_bytes = (fr.npaths + 2) * fr.des
    ach = agg_bytes / (stages["aggregate"] * 1e-3) / 1e9
    del eng
    return {"ms_per_step": round(ms, 5), "value": round(fr.des / (ms * 1e-3) / 1e6, 1),
            "stages_ms": {k: round(v, 5) for k, v in stages.items()},
            "step_ms_p50": round(percentile(per_step, 0.5), 5),
            "step_ms_p99": round(percentile(per_step, 0.99), 5),
            "roofline_sgm_aggregate": {
                "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "sgm_aggregate (paths_kernel + merge_kernel)",
                "algorithmic_bytes": agg_bytes}}


def other_forms(args, torch, sgm, fr, eng):
    """The same frame through the subpixel form (the paper's "fine"), the
    exact consistency check ("exact-cc") and the NCC cost, timed like the
    main path."""
    left, right, prm, stream, des = fr.left, fr.right, fr.prm, torch.cuda.current_stream(), fr.des
    reps = max(1, min(50, args.steps))
    fine_work = sgm._aligned_bytes(sgm.aggregate_select_subpixel_work_bytes(
        fr.w, fr.h, prm.ndisp, prm.npaths, prm.p2), left.device)
    fine_out = torch.empty((fr.h, fr.w), dtype=torch.float32, device=left.device)
    exact_work = sgm._aligned_bytes(sgm.disparity_exact_lr_work_bytes(fr.w, fr.h, prm), left.device)

    def fine():
        sgm.sgm_census_pair(left, right, prm.win_w, prm.win_h, out_left=eng.census_left,
                            out_right=eng.census_right)
        sgm.sgm_cost(eng.census_left, eng.census_right, prm.ndisp, out=eng.cost)
        sgm.sgm_aggregate_select_subpixel(eng.cost, prm.npaths, prm.p1, prm.p2, prm.lr_tolerance,
                                          prm.median3x3, out=fine_out, work=fine_work)

    def exact():
        sgm.sgm_disparity_exact_lr(left, right, prm, out=eng.disp, work=exact_work)

    # NCC cost with the paper's KITTI penalties for it (P1 = 90, P2 = 880:
    # uint16 pair slices, still the fused selection)
    ncc_work = sgm._aligned_bytes(sgm.aggregate_select_work_bytes(
        fr.w, fr.h, prm.ndisp, prm.npaths, 880), left.device)

    def ncc(win):
        def run():
            sgm.sgm_cost_ncc(left, right, win, prm.ndisp, out=eng.cost)
            sgm.sgm_aggregate_select(eng.cost, prm.npaths, 90, 880, prm.lr_tolerance,
                                     prm.median3x3, out=eng.disp, work=ncc_work)
        return run

    out = {}
    for name, fn in (("subpixel", fine), ("exact_lr_check", exact), ("ncc5x5", ncc(5)),
                     ("ncc9x9", ncc(9))):
        for _ in range(3):
            fn()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        for _ in range(reps):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        out[name] = {"ms_per_step": round(ms, 5), "value": round(des / (ms * 1e-3) / 1e6, 1),
                     "unit": "MDE/s"}
    out["paper_context"] = {"subpixel": 633.1, "exact_lr_check": 361.8, "ncc5x5": 442.4,
                            "ncc9x9": 344.1, "unit": "MDE/s", "hardware": "Jetson AGX Xavier",
                            "config": "8-path SGM, LR check + median (CT9x7 for subpixel "
                                      "and exact_lr_check)"}
    return out


def pcie_frame(args, torch, fr, eng):
    """PCIe-inclusive frame (context only): pinned H2D of the pair, the path,
    D2H of D."""
    stream = torch.cuda.current_stream()
    hl = torch.from_numpy(fr.pair["left"]).pin_memory()
    hr = torch.from_numpy(fr.pair["right"]).pin_memory()
    hd = torch.empty((fr.h, fr.w), dtype=torch.uint16).pin_memory()
    n = max(1, min(50, args.steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        fr.left.copy_(hl, non_blocking=True)
        fr.right.copy_(hr, non_blocking=True)
        fr.step(eng, stream)
        hd.copy_(eng.disp, non_blocking=True)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / n


def batched_form(args, torch, dev, sgm, datagen):
    """64 mixed pairs: one hipGraph replay per batch vs 64 plain per-frame
    pipelines on one stream."""
    from paper_2106_07927_amd import tune
    specs = datagen.batch_specs()
    base = datagen.CONFIGS[HEADLINE]
    params = params_of(sgm, {**base, "ndisp": 0})
    lefts, rights = [], []
    for (w, h, nd, seed) in specs:
        pair = datagen.make_pair(w, h, nd, seed, base["planes"], base["occlusion"])
        lefts.append(torch.from_numpy(pair["left"]).to(dev))
        rights.append(torch.from_numpy(pair["right"]).to(dev))
    table, tune_ms = tune.tune([(w, h, nd) for (w, h, nd, _) in specs], params, device=dev)
    ndisps = [s[2] for s in specs]
    table, chains_ms = tune.tune_chains(lefts, rights, ndisps, params, table)
    plan = sgm.BatchPlan(lefts, rights, ndisps, params, tune_table=json.dumps(table))
    plan.run()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.batch_reps):
        plan.run()
    t1.record()
    torch.cuda.synchronize()
    batch_ms = t0.elapsed_time(t1) / args.batch_reps
    plan.close()
    del plan
    engines = {}
    for (w, h, nd, _) in specs:
        if (w, h, nd) not in engines:
            engines[(w, h, nd)] = sgm.StereoSGM(w, h, sgm.Params(**{**params.__dict__, "ndisp": nd}),
                                                device=dev)

    def plain():
        for i, (w, h, nd, _) in enumerate(specs):
            engines[(w, h, nd)].run(lefts[i], rights[i])

    plain()
    torch.cuda.synchronize()
    t0.record()
    reps = max(1, args.batch_reps // 2)
    for _ in range(reps):
        plain()
    t1.record()
    torch.cuda.synchronize()
    plain_ms = t0.elapsed_time(t1) / reps
    des = sum(w * h * nd for (w, h, nd, _) in specs)
    del engines
    torch.cuda.empty_cache()
    return {"pairs": len(specs), "des_per_batch": des,
            "ms_per_batch": round(batch_ms, 3), "mdes": round(des / batch_ms / 1e3, 1),
            "fps": round(len(specs) / batch_ms * 1e3, 1),
            "plain_ms_per_batch": round(plain_ms, 3), "plain_mdes": round(des / plain_ms / 1e3, 1),
            "speedup": round(plain_ms / batch_ms, 3), "tune_table": table, "tune_ms": tune_ms,
            "chains_ms": chains_ms,
            "launch": "one hipGraph replay (work-list kernels for the small frames, the "
                      "single-frame kernels for the others, spread over the tuned number of "
                      "streams inside the graph)"}


def served_form(args, torch, sgm, datagen):
    """16 Poisson camera streams at 30 Hz: continuous batching vs plain FIFO
    on the same trace; a budget below the streams' slots; twice the rate."""
    from paper_2106_07927_amd import serve
    params = params_of(sgm, {**datagen.CONFIGS[HEADLINE], "ndisp": 0})
    specs = [serve.StreamSpec(*s) for s in datagen.stream_specs()]
    budget = int(args.serve_budget_gib * 2 ** 30)
    backend = serve.GpuBackend(specs, params, frames_per_stream=2, arena_bytes=budget)
    # standalone device time of one frame per stream shape: the GPU-busy estimate
    frame_ms = {}
    stream = torch.cuda.current_stream()
    for s, sp in enumerate(specs):
        key = (sp.width, sp.height, sp.ndisp)
        if key in frame_ms:
            continue
        prm = sgm.Params(**{**params.__dict__, "ndisp": sp.ndisp})
        eng = sgm.StereoSGM(sp.width, sp.height, prm)
        hl, hr = backend.pool[s][0]
        l, r = hl.cuda(), hr.cuda()
        for _ in range(3):
            eng.run(l, r)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(10):
            eng.run(l, r)
        b.record(stream)
        torch.cuda.synchronize()
        frame_ms[key] = a.elapsed_time(b) / 10
        del eng
    torch.cuda.empty_cache()

    def busy(stats):
        span = max((r.done for r in stats.results), default=0.0)
        dev_s = sum(frame_ms[(specs[r.request.stream].width, specs[r.request.stream].height,
                              specs[r.request.stream].ndisp)] for r in stats.results) * 1e-3
        return round(dev_s / span, 3) if span > 0 else None

    def run(trace, hip_streams=4):
        torch.cuda.synchronize()
        st = serve.Server(specs, backend, budget_bytes=backend.arena.capacity,
                          hip_streams=hip_streams).run(trace)
        torch.cuda.synchronize()
        return {**st.summary(specs), "gpu_busy": busy(st)}

    def fifo(trace):
        st = serve.serve_plain(trace, specs, backend)
        torch.cuda.synchronize()
        return {**st.summary(specs), "gpu_busy": busy(st)}

    trace = serve.make_trace(specs, 30.0, args.serve_seconds, 2, seed=2110)
    short = [r for r in trace if r.arrival < args.serve_short_seconds]
    # warm-up (not reported): the first launches of every shape
    run([r for r in trace if r.arrival < 1.0])
    before = torch.cuda.memory_allocated()
    mix = run(trace)
    grown = torch.cuda.memory_allocated() - before
    # the plain FIFO reference and continuous batching on the same prefix
    prefix = [r for r in trace if r.arrival < args.serve_short_seconds]
    prefix_mix = run(prefix)
    plain = fifo(prefix)
    # a budget below the streams' slots: waits and evictions inside the arena
    tight_gib = 8.0
    tight_backend = serve.GpuBackend(specs, params, frames_per_stream=2,
                                     arena_bytes=int(tight_gib * 2 ** 30))
    tb = serve.Server(specs, tight_backend, budget_bytes=tight_backend.arena.capacity,
                      hip_streams=4).run(short)
    torch.cuda.synchronize()
    tight = {**tb.summary(specs), "gpu_busy": busy(tb)}
    del tight_backend
    torch.cuda.empty_cache()
    # over-load: twice the rate
    # above the load: 2x and 3x the rate, each trace served both ways
    overload = {}
    for mult in (2, 3):
        fast = serve.make_trace(specs, 30.0 * mult, args.serve_short_seconds, 2, seed=2110 + mult)
        overload[f"{30 * mult}hz_{args.serve_short_seconds:g}s"] = {"continuous": run(fast),
                                                                     "plain_fifo": fifo(fast)}
    offered = sum(s.width * s.height * s.ndisp for s in specs) * 30.0 / 1e6
    return {"streams": len(specs), "rate_hz": 30.0, "seconds": args.serve_seconds,
            "offered_mdes": round(offered, 1), "arena_gib": round(backend.arena.capacity / 2 ** 30, 2),
            "slot_gib_all_streams": round(sum(serve.slot_bytes(s, params.npaths, params.p2)
                                              for s in specs) / 2 ** 30, 2),
            "device_bytes_allocated_while_serving": grown,
            "continuous": mix,
            f"first_{args.serve_short_seconds:g}s": {"continuous": prefix_mix, "plain_fifo": plain},
            f"tight_arena_{int(tight_gib)}gib_{args.serve_short_seconds:g}s": tight,
            "overload": overload,
            "frame_ms_by_shape": {f"{w}x{h}x{d}": round(v, 4) for (w, h, d), v in frame_ms.items()}}


def cpu_baseline(fr, frames):
    """The oracle on the host: single-threaded (the oracle as it stands) on
    `frames` frames, then its threaded driver on every core the process may
    use, checked bit for bit against the single-threaded maps."""
    import numpy as np
    import oracle
    cfg = fr.cfg
    prm = oracle.Params(win_w=cfg["win_w"], win_h=cfg["win_h"], ndisp=cfg["ndisp"],
                        npaths=cfg["npaths"], p1=cfg["p1"], p2=cfg["p2"],
                        lr_tolerance=cfg["lr_tolerance"], median3x3=cfg["median3x3"])
    t0 = time.perf_counter()
    for _ in range(frames):
        ref = oracle.run(fr.pair["left"], fr.pair["right"], prm)
    dt = time.perf_counter() - t0
    des = fr.des * frames
    cores = len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mt_frames = 3 * frames
    t1 = time.perf_counter()
    for _ in range(mt_frames):
        mt = oracle.run_threaded(fr.pair["left"], fr.pair["right"], prm, cores)
    dt_mt = time.perf_counter() - t1
    same = all(np.array_equal(mt[k], ref[k]) for k in ("disp_left", "disp_right", "disp"))
    if not same:
        raise RuntimeError("the threaded oracle differs from the single-threaded one")
    return {"value": round(des / dt / 1e6, 3), "unit": "MDE/s", "cores": 1, "kind": "oracle",
            "sample": f"{frames} full frames of the {fr.w}x{fr.h} D={fr.nd} {fr.npaths}-path "
                      f"workload, single-threaded C oracle, {dt:.1f} s",
            "cpu_model": model,
            "all_cores": {"value": round(fr.des * mt_frames / dt_mt / 1e6, 3), "unit": "MDE/s",
                          "cores": cores, "kind": "oracle (threaded driver, same functions)",
                          "sample": f"{mt_frames} frames, {dt_mt:.1f} s; maps bit-identical to "
                                    f"the single-threaded run"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards "
              f"by frame and needs no collective, see the design notes.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2106_07927_amd import datagen, sgm

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe_mib > 0:
        copy_probe(torch, dev, args.copy_probe_mib)
    digest = sources_digest()

    log(f"headline {args.workload}: launch modes over {args.select_steps} steps each, then {args.steps} timed")
    fr, eng, main_t = headline(args, torch, sgm, datagen, dev)
    log(f"headline done: {main_t['ms']:.4f} ms/step ({main_t['mode']})")
    ms_step = main_t["ms"]
    stages = main_t["stages"]
    per_step = main_t["per_step"]
    eager_ms = sum(stages.values())
    out = {
        "metric": METRIC,
        "value": round(fr.des / (ms_step * 1e-3) / 1e6, 1),
        "unit": "MDE/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": workload_desc(args.workload, fr.cfg), "width": fr.w, "height": fr.h,
                   "ndisp": fr.nd, "npaths": fr.npaths, "frames_per_step": 1,
                   "launch": main_t["mode"]},
        "fps": round(1000.0 / ms_step, 1),
        "launch_modes_ms": {k: round(v, 5) for k, v in main_t["mode_ms"].items()},
        "mode_select_steps": args.select_steps,
        "eager_single_stream": {"ms_per_step": round(eager_ms, 5),
                                "value": round(fr.des / (eager_ms * 1e-3) / 1e6, 1),
                                "fps": round(1000.0 / eager_ms, 1)},
        "stages_ms": {k: round(v, 5) for k, v in stages.items()},
        "step_ms_p50": round(percentile(per_step, 0.5), 5),
        "step_ms_p99": round(percentile(per_step, 0.99), 5),
        "roofline": fr.roofline(stages["aggregate_select"], digest),
    }
    log("four-call form")
    out["four_call"] = four_call(args, torch, fr)
    log("PCIe-inclusive frame and the other forms")
    out["e2e_pcie_ms_per_frame"] = round(pcie_frame(args, torch, fr, eng), 4)
    out["other_forms"] = other_forms(args, torch, sgm, fr, eng)
    out["paper_context"] = {"value": 644.9, "unit": "MDE/s",
                            "hardware": "Jetson AGX Xavier, 512-core Volta GPU",
                            "config": "CT9x7, 8-path SGM, LR check + median, incl. transfers"}
    del eng
    torch.cuda.empty_cache()
    if args.other_configs:
        out["other_configs"] = {}
        for n in ("c1_320x240_d64_r4", "c3_1920x1080_d256_r8"):
            log(f"workload {n}")
            out["other_configs"][n] = other_config(args, torch, sgm, datagen, dev, n, digest)
    if args.batch_reps > 0:
        log("batched form: tuning, plan, replays, plain launches")
        out["batched"] = batched_form(args, torch, dev, sgm, datagen)
    if args.serve_seconds > 0:
        log(f"served form: {args.serve_seconds:g} s trace, then the tight-budget and overload traces")
        out["served"] = served_form(args, torch, sgm, datagen)
    if args.cpu_frames > 0:
        log(f"CPU oracle: {args.cpu_frames} frame(s) single-threaded, then all cores")
        out["cpu_baseline"] = cpu_baseline(fr, args.cpu_frames)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
