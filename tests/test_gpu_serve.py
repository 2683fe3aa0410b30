"""GPU: served form.  Frames from several Poisson camera streams run
concurrently on a pool of HIP streams, with their buffers carved from one
device arena of the HBM budget's size.

The streams have the four distinct shapes of the 16-stream camera workload
(640x512 at D 128 / 256, 1242x375 and 1920x1080 at D 128).  Every served
disparity map is compared with the oracle (stored digests of the oracle's
maps for those frames, tests/golden/oracle_digests.json).  The tests assert
that frames were in flight together, that a budget below the sum of the
streams' slots makes the server defer and evict on the GPU with the same
bits, and that serving allocates no device memory beyond the arena.
"""
import os
import sys

import numpy as np
import pytest

from paper_2106_07927_amd import datagen, serve

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import oracle_digests as od  # noqa: E402

pytestmark = pytest.mark.gpu
PARAMS = dict(win_w=9, win_h=7, npaths=8, p1=10, p2=120, lr_tolerance=1, median3x3=True)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2106_07927_amd import sgm
    sgm.load_library()
    specs, seen = [], set()
    for (w, h, nd, seed) in datagen.stream_specs():
        if (w, h, nd) not in seen:
            seen.add((w, h, nd))
            specs.append(serve.StreamSpec(w, h, nd, seed))
    table = od.load()["cases"]
    want = {}
    for s, sp in enumerate(specs):
        for k in range(od.SERVE_FRAMES):
            case = table[od.stream_frame_case(sp.width, sp.height, sp.ndisp, sp.seed, k)]
            want[(s, k)] = case
    return specs, sgm.Params(ndisp=0, **PARAMS), want


def _check_results(stats, backend, want):
    assert len(backend.result_of) == stats.served
    for r in stats.results:
        got = backend.result_of[(r.request.stream, r.request.seq)]
        case = want[(r.request.stream, r.request.frame)]
        assert od.digest(got) == case["outputs"]["disp"], \
            f"stream {r.request.stream} seq {r.request.seq} frame {r.request.frame} differs from the oracle"


def _overlapping_pairs(stats):
    spans = sorted((r.start, r.done) for r in stats.results)
    n = 0
    for i, (a0, a1) in enumerate(spans):
        for (b0, b1) in spans[i + 1:]:
            if b0 >= a1:
                break
            n += 1
    return n


def test_served_frames_equal_oracle_and_overlap(setup):
    import torch
    specs, params, want = setup
    say("serve: 4 stream shapes of the camera workload, 0.4 s at 150 Hz, roomy arena")
    backend = serve.GpuBackend(specs, params, frames_per_stream=od.SERVE_FRAMES,
                               arena_bytes=16 << 30)
    # the pool's images are the stored cases' inputs
    for s, sp in enumerate(specs):
        for k in range(od.SERVE_FRAMES):
            hl, hr = backend.pool[s][k]
            assert od.digest(hl.numpy()) == want[(s, k)]["inputs"]["left"]
            assert od.digest(hr.numpy()) == want[(s, k)]["inputs"]["right"]
    trace = serve.make_trace(specs, 150.0, 0.4, od.SERVE_FRAMES, seed=3)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    srv = serve.Server(specs, backend, budget_bytes=backend.arena.capacity, hip_streams=4)
    stats = srv.run(trace, keep=lambda r: True)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before, "serving allocated device memory"
    assert stats.served == len(trace) and stats.rejected == 0
    assert stats.peak_bytes <= backend.arena.capacity
    assert backend.arena.used == 0, "the run did not hand its slots back"
    overlap = _overlapping_pairs(stats)
    say(f"served {stats.served}, overlapping pairs {overlap}, deferred {stats.deferred}")
    assert overlap > 0, "no two frames were in flight together"
    _check_results(stats, backend, want)


def test_tight_budget_defers_and_evicts_with_same_bits(setup):
    import torch
    specs, params, want = setup
    sizes = [serve.slot_bytes(sp, PARAMS["npaths"], PARAMS["p2"]) for sp in specs]
    budget = serve.Arena.round(max(sizes) + sorted(sizes)[-2])
    assert budget < sum(sizes)
    say(f"serve: tight arena of {budget / 2 ** 30:.2f} GiB (slots total {sum(sizes) / 2 ** 30:.2f} GiB)")
    backend = serve.GpuBackend(specs, params, frames_per_stream=od.SERVE_FRAMES,
                               arena_bytes=budget)
    trace = serve.make_trace(specs, 60.0, 0.6, od.SERVE_FRAMES, seed=4)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    srv = serve.Server(specs, backend, budget_bytes=budget, hip_streams=4)
    stats = srv.run(trace, keep=lambda r: True)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before, "serving allocated device memory"
    say(f"served {stats.served}, deferred {stats.deferred}, evictions {stats.evictions}")
    assert stats.served == len(trace) and stats.rejected == 0
    assert stats.deferred > 0 and stats.evictions > 0
    assert stats.peak_bytes <= budget and backend.arena.used <= backend.arena.capacity
    _check_results(stats, backend, want)
