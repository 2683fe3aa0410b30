"""GPU: served form.  Frames from several Poisson camera streams run
concurrently on a pool of HIP streams with resident per-stream buffers; each
served disparity map is bit-identical to the same frame computed alone."""
import sys

import numpy as np
import pytest

from paper_2106_07927_amd import serve

pytestmark = pytest.mark.gpu


def test_served_frames_equal_frames_alone():
    import torch
    from paper_2106_07927_amd import sgm
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    print("serve: 4 streams, 1.5 s", flush=True)
    sys.stdout.flush()
    specs = [serve.StreamSpec(320, 240, 64, 1), serve.StreamSpec(640, 512, 128, 2),
             serve.StreamSpec(1242, 375, 128, 3), serve.StreamSpec(640, 512, 256, 4)]
    params = sgm.Params(ndisp=0, win_w=9, win_h=7, npaths=8, p1=10, p2=120, lr_tolerance=1,
                        median3x3=True)
    backend = serve.GpuBackend(specs, params, frames_per_stream=3)
    trace = serve.make_trace(specs, 30.0, 1.5, 3, seed=3)
    budget = sum(serve.slot_bytes(s, 8, 120) for s in specs) + (64 << 20)
    srv = serve.Server(specs, backend, budget_bytes=budget, hip_streams=4)
    stats = srv.run(trace, keep=lambda r: True)
    torch.cuda.synchronize()
    assert stats.served == len(trace) and stats.rejected == 0
    assert stats.peak_bytes <= budget
    overlap = sum(1 for a in stats.results for b in stats.results
                  if a is not b and a.start < b.done and b.start < a.done)
    print(f"served {stats.served}, overlapping pairs {overlap}", flush=True)
    # the same frames alone, one at a time on the default stream
    alone = {}
    for s, sp in enumerate(specs):
        eng = sgm.StereoSGM(sp.width, sp.height, sgm.Params(**{**params.__dict__, "ndisp": sp.ndisp}))
        for k, (hl, hr) in enumerate(backend.pool[s]):
            eng.run(hl.cuda(), hr.cuda())
            torch.cuda.synchronize()
            alone[(s, k)] = eng.disp.cpu().numpy()
    for r in stats.results:
        got = backend.result_of[(r.request.stream, r.request.seq)]
        np.testing.assert_array_equal(got, alone[(r.request.stream, r.request.frame)],
                                      err_msg=f"stream {r.request.stream} seq {r.request.seq}")
