"""GPU parity at the 1920x1080 / D=256 / 8-path frame, in full.

The oracle needs about 35 s of single-threaded CPU time for this frame, so
its outputs are stored as SHA-256 digests (tests/golden/oracle_digests.json,
written from the oracle alone by tests/golden/oracle_digests.py).  Both forms
of the path -- the four ABI calls and the streamlined sgm_aggregate_select --
are compared with them: census of both images, cost and S_bar (four-call
form), D^R and the final map (both forms), and D^L (both forms, as the final
map of a run with the LR check and the median switched off, which by
definition is D^L).  Tolerance 0: every result is integer.
"""
import os
import sys

import numpy as np
import pytest

from paper_2106_07927_amd import datagen

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import oracle_digests as od  # noqa: E402

pytestmark = pytest.mark.gpu
NAME = "c3_1920x1080_d256_r8"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def frame():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2106_07927_amd import sgm
    sgm.load_library()
    table = od.load()["cases"][NAME]
    pair = datagen.config_pair(NAME)
    assert od.digest(pair["left"]) == table["inputs"]["left"], \
        "the generator's left image changed: rerun tests/golden/oracle_digests.py"
    assert od.digest(pair["right"]) == table["inputs"]["right"], \
        "the generator's right image changed: rerun tests/golden/oracle_digests.py"
    dev = torch.device("cuda:0")
    return (torch.from_numpy(pair["left"]).to(dev), torch.from_numpy(pair["right"]).to(dev),
            table["outputs"])


def _params(lr, median):
    from paper_2106_07927_amd import sgm
    c = datagen.CONFIGS[NAME]
    return sgm.Params(win_w=c["win_w"], win_h=c["win_h"], ndisp=c["ndisp"], npaths=c["npaths"],
                      p1=c["p1"], p2=c["p2"], lr_tolerance=lr, median3x3=median)


def _check(name, t, want):
    import torch
    torch.cuda.synchronize()
    got = od.digest(t.cpu().numpy())
    assert got == want, f"{NAME}: {name} differs from the oracle"


@pytest.mark.parametrize("fused", [False, True], ids=["four_call", "streamlined"])
def test_c3_frame_full(frame, fused):
    from paper_2106_07927_amd import sgm
    left, right, want = frame
    c = datagen.CONFIGS[NAME]
    say(f"c3 full frame, {'streamlined' if fused else 'four-call'} form")
    eng = sgm.StereoSGM(c["width"], c["height"], _params(c["lr_tolerance"], c["median3x3"]),
                        device=left.device, fused=fused)
    eng.run(left, right)
    if not fused:
        _check("census_left", eng.census_left, want["census_left"])
        _check("census_right", eng.census_right, want["census_right"])
        _check("cost", eng.cost, want["cost"])
        _check("S_bar", eng.agg, want["agg"])
    _check("D^R", eng.disp_right, want["disp_right"])
    _check("D (LR check + median)", eng.disp, want["disp"])
    del eng
    # LR check and median off: the final map is D^L itself
    eng = sgm.StereoSGM(c["width"], c["height"], _params(-1, False), device=left.device,
                        fused=fused)
    eng.run(left, right)
    _check("D^L", eng.disp, want["disp_left"])
    _check("D^R (no LR check)", eng.disp_right, want["disp_right"])


def test_c3_frame_ground_truth(frame):
    """A property that holds at any size, beside the exact comparison: on
    the synthetic ground truth of the pair, the LR-checked, median-filtered
    map keeps most pixels and few of the kept non-occluded ones are off by
    3 px or more."""
    from paper_2106_07927_amd import sgm
    left, right, _ = frame
    c = datagen.CONFIGS[NAME]
    pair = datagen.config_pair(NAME)
    eng = sgm.StereoSGM(c["width"], c["height"], _params(c["lr_tolerance"], c["median3x3"]),
                        device=left.device)
    eng.run(left, right)
    import torch
    torch.cuda.synchronize()
    disp = eng.disp.cpu().numpy().astype(np.int64)
    valid = disp != 0xFFFF
    assert valid.mean() > 0.5
    good = valid & ~pair["occluded"]
    assert np.mean(np.abs(disp - pair["disp_gt"].astype(np.int64))[good] >= 3) < 0.05
