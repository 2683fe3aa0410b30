"""GPU parity of the exact consistency check (sgm_disparity_exact_lr: D^R
matched from scratch on the swapped, flipped pair) against the oracle's
swap-and-flip route, which the CPU suite pins to the right-reference
definition.  Integer throughout: exact comparison."""
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


def run_gpu(dev, left, right, prm):
    import torch
    from paper_2106_07927_amd import sgm
    l = torch.from_numpy(np.ascontiguousarray(left)).to(dev)
    r = torch.from_numpy(np.ascontiguousarray(right)).to(dev)
    p = sgm.Params(win_w=prm.win_w, win_h=prm.win_h, ndisp=prm.ndisp, npaths=prm.npaths,
                   p1=prm.p1, p2=prm.p2, lr_tolerance=prm.lr_tolerance, median3x3=prm.median3x3)
    d, dr = sgm.sgm_disparity_exact_lr(l, r, p, want_right=True)
    torch.cuda.synchronize()
    return d.cpu().numpy(), dr.cpu().numpy()


CASES = [
    # w, h, D, window, npaths, p1, p2, t, median
    (64, 20, 16, (5, 5), 4, 7, 86, 1, 1), (131, 17, 32, (9, 7), 8, 10, 120, 1, 1),
    (200, 24, 64, (9, 7), 8, 10, 120, 0, 0), (77, 9, 100, (9, 7), 8, 10, 120, 2, 1),
    (90, 11, 48, (5, 5), 8, 10, 300, 1, 1), (5, 3, 16, (9, 7), 8, 10, 120, 1, 1),
    (150, 12, 128, (9, 7), 8, 10, 120, -1, 1),
]


@pytest.mark.parametrize("w,h,nd,win,npaths,p1,p2,t,med", CASES)
def test_exact_lr_parity(dev, w, h, nd, win, npaths, p1, p2, t, med):
    say(f"exact lr {w}x{h} D{nd} {win} R{npaths} P2={p2} t={t} median={med}")
    pair = datagen.make_pair(w, h, nd, seed=w + 7 * h + nd, planes=(3, 5), occlusion=0.05)
    prm = oracle.Params(win_w=win[0], win_h=win[1], ndisp=nd, npaths=npaths, p1=p1, p2=p2,
                        lr_tolerance=t, median3x3=bool(med))
    d, dr = run_gpu(dev, pair["left"], pair["right"], prm)
    ref = oracle.run_exact_lr(pair["left"], pair["right"], prm)
    np.testing.assert_array_equal(dr, ref["disp_right"])
    np.testing.assert_array_equal(d, ref["disp"])


@pytest.mark.parametrize("name", ["c1_320x240_d64_r4", "c2_1242x375_d128_r8"])
def test_exact_lr_full_frame(dev, name):
    say(f"exact lr {name}")
    cfg = datagen.CONFIGS[name]
    pair = datagen.config_pair(name)
    prm = oracle.Params(win_w=cfg["win_w"], win_h=cfg["win_h"], ndisp=cfg["ndisp"],
                        npaths=cfg["npaths"], p1=cfg["p1"], p2=cfg["p2"], lr_tolerance=1,
                        median3x3=True)
    d, dr = run_gpu(dev, pair["left"], pair["right"], prm)
    ref = oracle.run_exact_lr(pair["left"], pair["right"], prm)
    np.testing.assert_array_equal(dr, ref["disp_right"])
    np.testing.assert_array_equal(d, ref["disp"])
