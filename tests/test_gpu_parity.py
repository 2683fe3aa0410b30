"""GPU parity: every stage of the HIP path, called through the C ABI, against
the CPU oracle on the same seeded inputs.  Everything is integer, so every
comparison is exact (tolerance 0).

Sizes: small cases span several tiles and ragged tails and cover the edge
cases (1-pixel images, D = 1, odd D, D = 256, zero and maximal penalties);
the 1242x375 / D=128 / 8-path frame is compared in full.  The 1920x1080 /
D=256 frame is compared in full by test_gpu_large.py.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2106_07927_amd import datagen

pytestmark = pytest.mark.gpu
INV = 0xFFFF


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


def gpu_pipeline(left, right, prm, dev):
    from paper_2106_07927_amd import sgm
    l, r = to_dev(left, dev), to_dev(right, dev)
    cl = sgm.sgm_census(l, prm.win_w, prm.win_h)
    cr = sgm.sgm_census(r, prm.win_w, prm.win_h)
    c = sgm.sgm_cost(cl, cr, prm.ndisp)
    a = sgm.sgm_aggregate(c, prm.npaths, prm.p1, prm.p2)
    d, dr = sgm.sgm_wta_lrc(a, prm.lr_tolerance, prm.median3x3, want_right=True)
    return {"census_left": host(cl), "census_right": host(cr), "cost": host(c), "agg": host(a),
            "disp": host(d), "disp_right": host(dr)}


# ---------------------------------------------------------------- census ---
@pytest.mark.parametrize("win", [(5, 5), (9, 7)])
@pytest.mark.parametrize("w,h", [(1, 1), (2, 7), (7, 2), (63, 17), (64, 16), (65, 33), (321, 40)])
def test_census_parity(dev, win, w, h):
    from paper_2106_07927_amd import sgm
    say(f"census {w}x{h} win{win}")
    img, _ = datagen.random_images(w, h, seed=w * 1000 + h)
    out = host(sgm.sgm_census(to_dev(img, dev), *win))
    np.testing.assert_array_equal(out.view(np.uint64), oracle.census(img, *win))


def test_census_pitch(dev):
    from paper_2106_07927_amd import sgm
    say("census pitched")
    img, _ = datagen.random_images(80, 20, seed=9)
    out = host(sgm.sgm_census(to_dev(img, dev), 9, 7, width=67))
    np.testing.assert_array_equal(out, oracle.census(np.ascontiguousarray(img[:, :67]), 9, 7))


@pytest.mark.parametrize("win", [(5, 5), (9, 7)])
@pytest.mark.parametrize("w,h,width", [(1, 1, None), (7, 2, None), (65, 33, None), (80, 20, 67),
                                       (1242, 375, None)])
def test_census_pair_parity(dev, win, w, h, width):
    """One launch for both images: each output equals the oracle's census of
    its own image (pitched inputs included)."""
    from paper_2106_07927_amd import sgm
    say(f"census pair {w}x{h} width={width} win{win}")
    left, right = datagen.random_images(w, h, seed=w * 7 + h)
    cl, cr = sgm.sgm_census_pair(to_dev(left, dev), to_dev(right, dev), *win, width=width)
    ww = w if width is None else width
    np.testing.assert_array_equal(host(cl), oracle.census(np.ascontiguousarray(left[:, :ww]), *win))
    np.testing.assert_array_equal(host(cr), oracle.census(np.ascontiguousarray(right[:, :ww]), *win))


# ------------------------------------------------------------------ cost ---
@pytest.mark.parametrize("nd", [1, 3, 4, 16, 64, 96, 128, 256])
@pytest.mark.parametrize("w", [1, 7, 65, 321])
def test_cost_parity(dev, nd, w):
    from paper_2106_07927_amd import sgm
    say(f"cost w{w} D{nd}")
    rng = np.random.default_rng(nd * 7 + w)
    h = 5
    cl = rng.integers(0, 1 << 62, (h, w), dtype=np.uint64)
    cr = rng.integers(0, 1 << 62, (h, w), dtype=np.uint64)
    out = host(sgm.sgm_cost(to_dev(cl, dev), to_dev(cr, dev), nd))
    np.testing.assert_array_equal(out, oracle.cost(cl, cr, nd))


# ------------------------------------------------------------- aggregate ---
AGG_CASES = [
    # w, h, D, npaths, p1, p2
    (1, 1, 1, 4, 10, 120), (1, 9, 3, 8, 10, 120), (9, 1, 16, 8, 10, 120),
    (7, 5, 2, 8, 3, 3), (13, 11, 5, 4, 7, 86), (33, 20, 16, 8, 10, 120),
    (65, 17, 32, 8, 0, 0), (70, 31, 64, 4, 7, 86), (40, 70, 96, 8, 10, 120),
    (130, 9, 128, 8, 10, 120), (129, 66, 128, 8, 1, 7936), (50, 23, 256, 8, 10, 120),
    (37, 41, 256, 4, 200, 16128), (90, 14, 100, 8, 20, 20), (66, 5, 13, 8, 10, 120),
]


@pytest.mark.parametrize("w,h,nd,npaths,p1,p2", AGG_CASES)
def test_aggregate_parity(dev, w, h, nd, npaths, p1, p2):
    from paper_2106_07927_amd import sgm
    say(f"aggregate {w}x{h} D{nd} R{npaths} P1={p1} P2={p2}")
    c = datagen.random_cost(w, h, nd, seed=w * 31 + h * 7 + nd, high=256)
    c[:, :, : nd // 3] = np.minimum(c[:, :, : nd // 3], 40)   # a low-cost band
    out = host(sgm.sgm_aggregate(to_dev(c, dev), npaths, p1, p2))
    np.testing.assert_array_equal(out, oracle.aggregate(c, npaths, p1, p2))


def test_aggregate_deterministic(dev):
    from paper_2106_07927_amd import sgm
    say("aggregate repeat")
    c = datagen.random_cost(300, 97, 128, seed=3, high=64)
    tc = to_dev(c, dev)
    first = host(sgm.sgm_aggregate(tc, 8, 10, 120))
    for _ in range(3):
        np.testing.assert_array_equal(host(sgm.sgm_aggregate(tc, 8, 10, 120)), first)


# -------------------------------------------------------------- wta_lrc ---
@pytest.mark.parametrize("w,h,nd", [(1, 1, 1), (5, 3, 7), (130, 9, 64), (300, 7, 128),
                                    (257, 5, 256), (64, 64, 200), (129, 4, 3)])
@pytest.mark.parametrize("t,med", [(-1, 0), (1, 1), (0, 0), (3, 1)])
def test_wta_lrc_parity(dev, w, h, nd, t, med):
    from paper_2106_07927_amd import sgm
    say(f"wta_lrc {w}x{h} D{nd} t={t} median={med}")
    rng = np.random.default_rng(w + h + nd)
    agg = rng.integers(0, 12, (h, w, nd)).astype(np.uint16)   # many ties
    agg[rng.random((h, w, nd)) < 0.01] = 3000
    d, dr = sgm.sgm_wta_lrc(to_dev(agg, dev), t, med, want_right=True)
    dl_ref = oracle.wta(agg)
    dr_ref = oracle.right_disparity(agg)
    ref = oracle.lr_check(dl_ref, dr_ref, t) if t >= 0 else dl_ref
    if med:
        ref = oracle.median3x3(ref)
    np.testing.assert_array_equal(host(dr), dr_ref)
    np.testing.assert_array_equal(host(d), ref)


@pytest.mark.parametrize("w,h,nd", [(96, 3, 32), (70, 4, 48), (33, 2, 30)])
def test_wta_lrc_values_near_uint16_max(dev, w, h, nd):
    """S_bar values at the top of the uint16 range (the tile pass for
    D % 16 == 0 and the row-segment pass otherwise), with ties."""
    from paper_2106_07927_amd import sgm
    say(f"wta_lrc near 65535, {w}x{h} D{nd}")
    rng = np.random.default_rng(7 * w + nd)
    agg = (65535 - rng.integers(0, 6, (h, w, nd))).astype(np.uint16)
    d, dr = sgm.sgm_wta_lrc(to_dev(agg, dev), 1, True, want_right=True)
    dl_ref = oracle.wta(agg)
    dr_ref = oracle.right_disparity(agg)
    ref = oracle.median3x3(oracle.lr_check(dl_ref, dr_ref, 1))
    np.testing.assert_array_equal(host(dr), dr_ref)
    np.testing.assert_array_equal(host(d), ref)


# ------------------------------------------------------------ pipelines ---
def _params(cfg):
    return oracle.Params(win_w=cfg["win_w"], win_h=cfg["win_h"], ndisp=cfg["ndisp"],
                         npaths=cfg["npaths"], p1=cfg["p1"], p2=cfg["p2"],
                         lr_tolerance=cfg["lr_tolerance"], median3x3=cfg["median3x3"])


def _compare_all(got, ref):
    np.testing.assert_array_equal(got["census_left"], ref["census_left"])
    np.testing.assert_array_equal(got["census_right"], ref["census_right"])
    np.testing.assert_array_equal(got["cost"], ref["cost"])
    np.testing.assert_array_equal(got["agg"], ref["agg"])
    np.testing.assert_array_equal(got["disp_right"], ref["disp_right"])
    np.testing.assert_array_equal(got["disp"], ref["disp"])


@pytest.mark.parametrize("name", ["c1_320x240_d64_r4", "c2_1242x375_d128_r8"])
def test_pipeline_full_frame(dev, name):
    say(f"pipeline {name}")
    cfg = datagen.CONFIGS[name]
    pair = datagen.config_pair(name)
    prm = _params(cfg)
    got = gpu_pipeline(pair["left"], pair["right"], prm, dev)
    ref = oracle.run(pair["left"], pair["right"], prm)
    _compare_all(got, ref)


@pytest.mark.parametrize("d0", [0, 1, 17, 63])
def test_pipeline_pure_shift(dev, d0):
    say(f"pipeline pure shift d0={d0}")
    pair = datagen.pure_shift_pair(200, 48, d0, seed=77 + d0)
    prm = oracle.Params(win_w=9, win_h=7, ndisp=64, npaths=8, p1=10, p2=120,
                        lr_tolerance=1, median3x3=True)
    got = gpu_pipeline(pair["left"], pair["right"], prm, dev)
    ref = oracle.run(pair["left"], pair["right"], prm)
    _compare_all(got, ref)
