"""GPU parity at the size limits of the ABI, against the CPU oracle.

* The longest lines: 32768 x 2 and 2 x 32768 frames (SGM_MAX_SIDE), where a
  horizontal (or vertical) line is 32768 steps long and diagonal lines wrap
  at the border every second row -- in full, four-call and streamlined.
* The largest volume: 16383 x 1024 x 128 = 2,147,352,576 elements, just
  under SGM_MAX_VOLUME = 2^31 - 1, so the element offsets the path pass
  carries reach bit 30, next to the no-write bit it ORs into offsets.  The
  oracle computes S_bar there at sampled pixels (its per-pixel line
  recursions), D^L = its argmin, and D^R at two pixels from S_bar at the
  (up to D) pixels each depends on.

Inputs are seeded random cost volumes from datagen (the same bytes go to
both sides); tolerance 0 (integer results).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2106_07927_amd import datagen

pytestmark = pytest.mark.gpu

P1, P2 = 10, 120


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2106_07927_amd import sgm
    sgm.load_library()
    return torch, torch.device("cuda:0")


@pytest.mark.parametrize("w,h,nd", [(32768, 2, 16), (2, 32768, 16), (32768, 1, 32)])
def test_longest_lines_full(torch_dev, w, h, nd):
    torch, dev = torch_dev
    from paper_2106_07927_amd import sgm
    say(f"extreme lines {w}x{h} D={nd}")
    cost = datagen.random_cost(w, h, nd, seed=5000 + w + h)
    agg_ref = oracle.aggregate(cost, 8, P1, P2)
    dl_ref = oracle.wta(agg_ref)
    dr_ref = oracle.right_disparity(agg_ref)
    c = torch.from_numpy(cost).to(dev)
    agg = sgm.sgm_aggregate(c, 8, P1, P2)
    d4, dr4 = sgm.sgm_wta_lrc(agg, -1, False, want_right=True)
    ds, drs = sgm.sgm_aggregate_select(c, 8, P1, P2, -1, False, want_right=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(agg.cpu().numpy(), agg_ref)
    for got, want, name in ((d4, dl_ref, "D four-call"), (dr4, dr_ref, "D^R four-call"),
                            (ds, dl_ref, "D streamlined"), (drs, dr_ref, "D^R streamlined")):
        np.testing.assert_array_equal(got.cpu().numpy(), want, err_msg=name)


def test_largest_volume_sampled(torch_dev):
    torch, dev = torch_dev
    from paper_2106_07927_amd import sgm
    w, h, nd = 16383, 1024, 128
    assert w * h * nd <= 2 ** 31 - 1 and w * h * nd > 2 ** 31 - 2 ** 18
    say(f"largest volume {w}x{h}x{nd}: generating the cost volume")
    cost = datagen.random_cost(w, h, nd, seed=5100)
    rng = np.random.default_rng(5101)
    samples = [(0, 0), (w - 1, h - 1), (w - 1, 0), (0, h - 1), (w // 2, h // 2), (w - 2, h - 1)]
    samples += [(int(rng.integers(0, w)), int(rng.integers(0, h))) for _ in range(6)]
    c = torch.from_numpy(cost).to(dev)

    say("largest volume: four-call S_bar at sampled pixels")
    agg = sgm.sgm_aggregate(c, 8, P1, P2)
    torch.cuda.synchronize()
    ref = {}
    for (x, y) in samples:
        ref[(x, y)] = oracle.aggregate_at(cost, 8, P1, P2, x, y)
        np.testing.assert_array_equal(agg[y, x].cpu().numpy(), ref[(x, y)],
                                      err_msg=f"S_bar at ({x}, {y})")
    del agg
    torch.cuda.empty_cache()

    say("largest volume: streamlined D^L and D^R")
    d, dr = sgm.sgm_aggregate_select(c, 8, P1, P2, -1, False, want_right=True)
    torch.cuda.synchronize()
    d_h = d.cpu().numpy()
    dr_h = dr.cpu().numpy()
    for (x, y), s in ref.items():
        assert d_h[y, x] == int(np.argmin(s)), f"D^L at ({x}, {y})"      # argmin: smallest d
    # D^R(q) = smallest d minimising S_bar(q + d, d) over q + d < W
    for (q, y) in ((w // 3, h - 1), (w - 70, 7)):
        best, arg = None, None
        for dd in range(nd):
            if q + dd >= w:
                break
            v = int(oracle.aggregate_at(cost, 8, P1, P2, q + dd, y)[dd])
            if best is None or v < best:
                best, arg = v, dd
        assert dr_h[y, q] == arg, f"D^R at ({q}, {y})"
    del c, d, dr
    torch.cuda.empty_cache()
