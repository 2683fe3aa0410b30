"""GPU parity of the NCC cost (sgm_cost_ncc) against the oracle: bit-exact,
since both sides form the same exact integer window sums and evaluate the
float part in float32 with IEEE operations in the same order; and the whole
path on an NCC cost volume."""
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


@pytest.mark.parametrize("win", [5, 9])
@pytest.mark.parametrize("w,h,nd", [(1, 1, 1), (7, 3, 5), (64, 9, 16), (65, 12, 64), (130, 6, 128),
                                    (100, 5, 256), (257, 4, 33)])
def test_ncc_cost_parity(dev, win, w, h, nd):
    import torch
    from paper_2106_07927_amd import sgm
    say(f"ncc {win}x{win} {w}x{h} D{nd}")
    pair = datagen.make_pair(w, h, max(nd, 2), seed=w * 3 + h + nd, planes=(2, 4))
    l = torch.from_numpy(pair["left"]).to(dev)
    r = torch.from_numpy(pair["right"]).to(dev)
    got = sgm.sgm_cost_ncc(l, r, win, nd)
    torch.cuda.synchronize()
    ref = oracle.ncc_cost(pair["left"], pair["right"], win, nd)
    np.testing.assert_array_equal(got.cpu().numpy(), ref)


def test_ncc_flat_and_shifted_inputs(dev):
    """Flat patches (no variance) and exact matches (cost 0) on the GPU."""
    import torch
    from paper_2106_07927_amd import sgm
    say("ncc flat and shifted")
    pair = datagen.pure_shift_pair(150, 20, 7, seed=3)
    left = pair["left"].copy()
    left[5:12, 30:60] = 90                                     # a flat block
    l = torch.from_numpy(left).to(dev)
    r = torch.from_numpy(pair["right"]).to(dev)
    got = sgm.sgm_cost_ncc(l, r, 5, 16)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.ncc_cost(left, pair["right"], 5, 16))


def test_ncc_full_path_frame(dev):
    """320x240, NCC 5x5, D = 64, 8 paths with the paper's NCC penalties
    (P1 = 90, P2 = 880: uint16 path slices): NCC cost, aggregation and
    selection against the oracle."""
    import torch
    from paper_2106_07927_amd import sgm
    say("ncc path 320x240")
    w, h, nd = 320, 240, 64
    pair = datagen.make_pair(w, h, nd, seed=2111, planes=(8, 12), occlusion=0.05)
    l = torch.from_numpy(pair["left"]).to(dev)
    r = torch.from_numpy(pair["right"]).to(dev)
    cost = sgm.sgm_cost_ncc(l, r, 5, nd)
    d, dr = sgm.sgm_aggregate_select(cost, 8, 90, 880, 1, True, want_right=True)
    torch.cuda.synchronize()
    c = oracle.ncc_cost(pair["left"], pair["right"], 5, nd)
    np.testing.assert_array_equal(cost.cpu().numpy(), c)
    agg = oracle.aggregate(c, 8, 90, 880)
    dl_ref = oracle.wta(agg)
    dr_ref = oracle.right_disparity(agg)
    ref = oracle.median3x3(oracle.lr_check(dl_ref, dr_ref, 1))
    np.testing.assert_array_equal(dr.cpu().numpy(), dr_ref)
    np.testing.assert_array_equal(d.cpu().numpy(), ref)
    gt = pair["disp_gt"].astype(np.int64)
    dd = d.cpu().numpy().astype(np.int64)
    good = (dd != oracle.INVALID) & ~pair["occluded"]
    assert np.mean(np.abs(dd - gt)[good] >= 3) < 0.05
