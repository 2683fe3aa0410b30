"""GPU parity of the streamlined call sgm_aggregate_select (aggregation fused
with WTA, approximate D^R, LR check and median; S_bar never leaves the chip)
against the CPU oracle on the same inputs.  Integer throughout, so every
comparison is exact.  (The 1920x1080 / D=256 frame is compared with the
oracle in full by test_gpu_large.py.)

Shapes cover: widths below, at and above the 64-pixel tile of the fused
pass and ragged last tiles; disparity ranges from 16 to 256 (D % 16 == 0)
and the unfused fallbacks (D % 16 != 0, P2 > 255); P2 = 127 / 128 on either
side of the bytewise pair-sum limit; 4 and 8 paths; graph replays.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2106_07927_amd import datagen

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2106_07927_amd import sgm
    sgm.load_library()
    return torch.device("cuda:0")


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def oracle_select(c, npaths, p1, p2, t, med):
    agg = oracle.aggregate(c, npaths, p1, p2)
    dl = oracle.wta(agg)
    dr = oracle.right_disparity(agg)
    d = oracle.lr_check(dl, dr, t) if t >= 0 else dl
    if med:
        d = oracle.median3x3(d)
    return d, dr


CASES = [
    # w, h, D, npaths, p1, p2, t, median
    (1, 1, 16, 8, 10, 120, 1, 1), (3, 5, 16, 4, 7, 86, -1, 0), (17, 9, 32, 8, 10, 120, 1, 1),
    (127, 6, 64, 8, 10, 120, 1, 1), (128, 7, 64, 4, 7, 86, 0, 0), (129, 5, 48, 8, 10, 127, 1, 1),
    (300, 9, 128, 8, 10, 120, 1, 1), (257, 4, 96, 8, 10, 128, 3, 1), (513, 3, 112, 4, 20, 255, 1, 0),
    (70, 11, 144, 8, 10, 120, 1, 1), (130, 6, 256, 8, 10, 120, 1, 1), (41, 13, 192, 4, 0, 0, -1, 1),
    (200, 8, 80, 8, 10, 120, 2, 1),
    # unfused fallbacks: D % 16 != 0, P2 > 255
    (99, 7, 100, 8, 10, 120, 1, 1), (65, 9, 7, 8, 10, 120, 1, 1), (90, 5, 64, 8, 10, 300, 1, 1),
]


@pytest.mark.parametrize("w,h,nd,npaths,p1,p2,t,med", CASES)
def test_aggregate_select_parity(dev, w, h, nd, npaths, p1, p2, t, med):
    from paper_2106_07927_amd import sgm
    say(f"aggregate_select {w}x{h} D{nd} R{npaths} P1={p1} P2={p2} t={t} median={med}")
    c = datagen.random_cost(w, h, nd, seed=w * 131 + h * 17 + nd, high=256)
    c[:, :, : nd // 3] = np.minimum(c[:, :, : nd // 3], 40)       # a low-cost band
    d, dr = sgm.sgm_aggregate_select(to_dev(c, dev), npaths, p1, p2, t, med, want_right=True)
    d_ref, dr_ref = oracle_select(c, npaths, p1, p2, t, med)
    np.testing.assert_array_equal(host(dr), dr_ref)
    np.testing.assert_array_equal(host(d), d_ref)


def test_aggregate_select_ties(dev):
    """Flat costs: every S_bar vector is constant, so every minimum is a tie."""
    from paper_2106_07927_amd import sgm
    say("aggregate_select ties")
    w, h, nd = 260, 6, 128
    c = np.full((h, w, nd), 5, np.uint8)
    c[2, 100:140, 60:64] = 0
    d, dr = sgm.sgm_aggregate_select(to_dev(c, dev), 8, 10, 120, 1, 1, want_right=True)
    d_ref, dr_ref = oracle_select(c, 8, 10, 120, 1, 1)
    np.testing.assert_array_equal(host(dr), dr_ref)
    np.testing.assert_array_equal(host(d), d_ref)


def test_aggregate_select_reuses_workspace(dev):
    """Two calls of different shapes on one workspace sized for the larger:
    nothing from the first call leaks into the second."""
    from paper_2106_07927_amd import sgm
    say("aggregate_select workspace reuse")
    big = datagen.random_cost(300, 20, 128, seed=1, high=256)
    small = datagen.random_cost(140, 9, 64, seed=2, high=256)
    work = sgm._aligned_bytes(sgm.aggregate_select_work_bytes(300, 20, 128, 8, 120), dev)
    for c in (big, small):
        d, dr = sgm.sgm_aggregate_select(to_dev(c, dev), 8, 10, 120, 1, 1, work=work, want_right=True)
        d_ref, dr_ref = oracle_select(c, 8, 10, 120, 1, 1)
        np.testing.assert_array_equal(host(dr), dr_ref)
        np.testing.assert_array_equal(host(d), d_ref)


@pytest.mark.parametrize("name", ["c1_320x240_d64_r4", "c2_1242x375_d128_r8"])
def test_fused_pipeline_full_frame(dev, name):
    from paper_2106_07927_amd import sgm
    say(f"fused pipeline {name}")
    cfg = datagen.CONFIGS[name]
    pair = datagen.config_pair(name)
    prm = sgm.Params(win_w=cfg["win_w"], win_h=cfg["win_h"], ndisp=cfg["ndisp"],
                     npaths=cfg["npaths"], p1=cfg["p1"], p2=cfg["p2"],
                     lr_tolerance=cfg["lr_tolerance"], median3x3=cfg["median3x3"])
    eng = sgm.StereoSGM(cfg["width"], cfg["height"], prm, device=dev)
    eng.run(to_dev(pair["left"], dev), to_dev(pair["right"], dev))
    ref = oracle.run(pair["left"], pair["right"],
                     oracle.Params(win_w=prm.win_w, win_h=prm.win_h, ndisp=prm.ndisp,
                                   npaths=prm.npaths, p1=prm.p1, p2=prm.p2,
                                   lr_tolerance=prm.lr_tolerance, median3x3=prm.median3x3))
    np.testing.assert_array_equal(host(eng.disp_right), ref["disp_right"])
    np.testing.assert_array_equal(host(eng.disp), ref["disp"])


def test_graph_replays_match_eager(dev):
    """The path captured into a HIP graph: every replay, with eager work and
    new inputs between replays, equals the eager result for those inputs."""
    import torch
    from paper_2106_07927_amd import sgm
    say("graph replays")
    w, h, nd = 300, 64, 128
    prm = sgm.Params(win_w=9, win_h=7, ndisp=nd, npaths=8, p1=10, p2=120, lr_tolerance=1,
                     median3x3=True)
    eng = sgm.StereoSGM(w, h, prm, device=dev)
    ref_eng = sgm.StereoSGM(w, h, prm, device=dev)
    l = torch.empty((h, w), dtype=torch.uint8, device=dev)
    r = torch.empty((h, w), dtype=torch.uint8, device=dev)
    pairs = [datagen.make_pair(w, h, nd, seed=900 + i, planes=(3, 5)) for i in range(4)]
    l.copy_(torch.from_numpy(pairs[0]["left"]))
    r.copy_(torch.from_numpy(pairs[0]["right"]))
    graph = eng.capture(l, r)
    for i, p in enumerate(pairs + pairs[:1]):
        l.copy_(torch.from_numpy(p["left"]))
        r.copy_(torch.from_numpy(p["right"]))
        graph.replay()
        torch.cuda.synchronize()
        got_d, got_r = eng.disp.clone(), eng.disp_right.clone()
        ref_eng.run(l, r)                          # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(got_d, ref_eng.disp), i
        assert torch.equal(got_r, ref_eng.disp_right), i
    ref = oracle.run(pairs[0]["left"], pairs[0]["right"],
                     oracle.Params(win_w=9, win_h=7, ndisp=nd, npaths=8, p1=10, p2=120,
                                   lr_tolerance=1, median3x3=True))
    np.testing.assert_array_equal(eng.disp.cpu().numpy(), ref["disp"])


def test_frames_in_flight_on_streams(dev):
    """Consecutive frames round-robin over engines on their own streams (the
    bench's frames-in-flight mode): every frame equals its oracle result."""
    import torch
    from paper_2106_07927_amd import sgm
    say("frames in flight, 3 streams")
    w, h, nd = 320, 96, 64
    prm = sgm.Params(win_w=9, win_h=7, ndisp=nd, npaths=8, p1=10, p2=120, lr_tolerance=1,
                     median3x3=True)
    pairs = [datagen.make_pair(w, h, nd, seed=700 + i, planes=(3, 5)) for i in range(6)]
    ins = [(to_dev(p["left"], dev), to_dev(p["right"], dev)) for p in pairs]
    engs = [sgm.StereoSGM(w, h, prm, device=dev) for _ in range(3)]
    streams = [torch.cuda.Stream(device=dev) for _ in range(3)]
    torch.cuda.synchronize()                   # inputs were copied on the default stream
    outs = [None] * len(pairs)
    for rnd in range(2):
        for i in range(rnd * 3, rnd * 3 + 3):
            k = i % 3
            engs[k].run(*ins[i], stream=streams[k])
        torch.cuda.synchronize()
        for i in range(rnd * 3, rnd * 3 + 3):
            outs[i] = engs[i % 3].disp.cpu().numpy()
    for i, p in enumerate(pairs):
        ref = oracle.run(p["left"], p["right"],
                         oracle.Params(win_w=9, win_h=7, ndisp=nd, npaths=8, p1=10, p2=120,
                                       lr_tolerance=1, median3x3=True))
        np.testing.assert_array_equal(outs[i], ref["disp"])
