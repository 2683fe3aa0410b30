"""sgm_aggregate_select_noalloc (the library's fixed per-GPU scratch as the
workspace) against sgm_aggregate_select with a caller workspace, through the
C ABI: bit-identical D and D^R on consecutive calls, the second on a smaller
frame (the scratch keeps the first call's bytes, which must not leak into
the second), with uint16 pair slices (P2 > 127) and the unfused fallback
(D % 16 != 0) too; a frame larger than the scratch is refused before any
launch and the next call still works."""
import sys

import numpy as np
import pytest

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


def cost_volume(w, h, nd, seed, dev):
    """The frame's census cost volume, from the library's own census and cost."""
    import torch
    from paper_2106_07927_amd import sgm
    pair = datagen.make_pair(w, h, nd, seed, (4, 10), 0.05)
    left = torch.from_numpy(pair["left"]).to(dev)
    right = torch.from_numpy(pair["right"]).to(dev)
    cl, cr = sgm.sgm_census_pair(left, right, 9, 7)
    return sgm.sgm_cost(cl, cr, nd)


def both(cost, npaths, p1, p2, t, med):
    import torch
    from paper_2106_07927_amd import sgm
    d_ref, dr_ref = sgm.sgm_aggregate_select(cost, npaths, p1, p2, t, med, want_right=True)
    d, dr = sgm.sgm_aggregate_select_noalloc(cost, npaths, p1, p2, t, med, want_right=True)
    torch.cuda.synchronize()
    return d_ref.cpu().numpy(), dr_ref.cpu().numpy(), d.cpu().numpy(), dr.cpu().numpy()


# consecutive calls, each smaller than the one before
SEQUENCE = [
    # w, h, D, npaths, p1, p2, t, median
    (1242, 375, 128, 8, 10, 120, 1, 1),     # the 1242x375 benchmark frame
    (321, 97, 64, 8, 10, 120, 1, 1),        # smaller, ragged tiles
    (200, 61, 48, 4, 7, 300, 0, 0),         # uint16 pair slices (P2 > 127)
    (65, 33, 37, 8, 10, 120, -1, 1),        # unfused fallback: S_bar in the scratch
]


def test_noalloc_equals_workspace_call_on_shrinking_frames(dev):
    for i, (w, h, nd, npaths, p1, p2, t, med) in enumerate(SEQUENCE):
        say(f"noalloc call {i}: {w}x{h} D={nd} paths={npaths} P1={p1} P2={p2} t={t} median={med}")
        cost = cost_volume(w, h, nd, 9300 + i, dev)
        d_ref, dr_ref, d, dr = both(cost, npaths, p1, p2, t, med)
        assert np.array_equal(d, d_ref), f"D differs on call {i}"
        assert np.array_equal(dr, dr_ref), f"D^R differs on call {i}"


def test_noalloc_repeat_after_larger_frame(dev):
    """The same small frame before and after a large one: identical bits."""
    small = cost_volume(97, 45, 32, 9400, dev)
    big = cost_volume(1242, 375, 128, 9401, dev)
    say("noalloc: small, large, small again")
    first = both(small, 8, 10, 120, 1, 1)
    both(big, 8, 10, 120, 1, 1)
    again = both(small, 8, 10, 120, 1, 1)
    for a, b in zip(first, again):
        assert np.array_equal(a, b)
    assert np.array_equal(first[0], first[2]) and np.array_equal(first[1], first[3])


def test_noalloc_rejects_frame_above_scratch(dev):
    import torch
    from paper_2106_07927_amd import sgm
    w, h, nd = 1920, 1080, 256
    assert sgm.aggregate_select_work_bytes(w, h, nd, 8, 120) > sgm.NOALLOC_SCRATCH_BYTES
    say("noalloc: 1920x1080 D=256 must be refused")
    cost = torch.zeros((h, w, nd), dtype=torch.uint8, device=dev)
    with pytest.raises(sgm.SGMError) as err:
        sgm.sgm_aggregate_select_noalloc(cost, 8, 10, 120, 1, True)
    assert err.value.status == sgm.SGM_ERR_TOO_LARGE
    del cost
    small = cost_volume(64, 16, 16, 9500, dev)
    d_ref, dr_ref, d, dr = both(small, 8, 10, 120, 1, 1)
    assert np.array_equal(d, d_ref) and np.array_equal(dr, dr_ref)
