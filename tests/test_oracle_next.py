"""Pins of the oracle's exact consistency check and subpixel refinement
(Sec. 2.1.3, Sec. 3.1.2, Sec. 3.1.3) against definitions written another way,
closed forms and invariants."""
import numpy as np
import pytest

import oracle
from paper_2106_07927_amd import datagen

INV = oracle.INVALID


def _params(win=(9, 7), nd=32, npaths=8, p1=10, p2=120, t=1, med=True):
    return oracle.Params(win_w=win[0], win_h=win[1], ndisp=nd, npaths=npaths, p1=p1, p2=p2,
                         lr_tolerance=t, median3x3=med)


# ------------------------------------------------------ exact right map ---
@pytest.mark.parametrize("win,npaths", [((5, 5), 4), ((9, 7), 8)])
def test_exact_right_disparity_equals_right_reference_definition(oracle_lib, win, npaths):
    """The swap-and-flip route equals matching with the right image as the
    reference directly: C^R(x, y, d) = Hamming(CR(x, y), CL(x + d, y)) where
    x + d < W, else 255, aggregated over the same (mirror-closed) path set."""
    w, h, nd = 45, 13, 16
    left, right = datagen.random_images(w, h, seed=81)
    prm = _params(win, nd, npaths)
    cl = oracle.census(left, *win)
    cr = oracle.census(right, *win)
    c_r = np.full((h, w, nd), 255, np.uint8)
    for d in range(nd):
        if d < w:
            c_r[:, : w - d, d] = np.bitwise_count(cr[:, : w - d] ^ cl[:, d:]).astype(np.uint8)
    direct = oracle.wta(oracle.aggregate(c_r, npaths, prm.p1, prm.p2))
    np.testing.assert_array_equal(oracle.exact_right_disparity(left, right, prm), direct)
    # the whole exact-check path carries that map, not the approximation of
    # Eq. (right_disparity), which differs on these images
    out = oracle.run_exact_lr(left, right, prm)
    np.testing.assert_array_equal(out["disp_right"], direct)
    approx = oracle.run(left, right, prm)["disp_right"]
    assert np.any(approx != direct)


@pytest.mark.parametrize("d0", [0, 3, 11])
def test_exact_right_disparity_pure_shift(oracle_lib, d0):
    """R(x) = L(x + d0): the right view's disparity is d0 wherever the match
    x + d0 lies inside the image, away from the census borders."""
    w, h, nd = 96, 30, 16
    pair = datagen.pure_shift_pair(w, h, d0, seed=5 + d0)
    prm = _params((9, 7), nd, 8)
    dr = oracle.exact_right_disparity(pair["left"], pair["right"], prm)
    m = 8
    assert np.all(dr[m:-m, m: w - d0 - m] == d0)
    out = oracle.run_exact_lr(pair["left"], pair["right"], prm)
    assert np.all(out["disp_left"][m:-m, d0 + m: w - m] == d0)
    assert np.all(out["disp"][m + 1:-m - 1, d0 + m + 1: w - m - 1] == d0)


def test_exact_check_filters_occlusions(oracle_lib):
    w, h, nd = 400, 160, 64
    pair = datagen.make_pair(w, h, nd, seed=31, planes=(6, 10), occlusion=0.05)
    out = oracle.run_exact_lr(pair["left"], pair["right"], _params((9, 7), nd, 8))
    gt = pair["disp_gt"].astype(np.int64)
    d = out["disp"].astype(np.int64)
    valid = d != INV
    good = ~pair["occluded"] & valid
    assert np.mean(np.abs(d - gt)[good] >= 3) < 0.02
    wrong = pair["occluded"] & (np.abs(out["disp_left"].astype(np.int64) - gt) >= 3)
    assert np.mean(~valid[wrong]) > 0.6
    assert valid.mean() > 0.5


def test_exact_and_approximate_checks_share_d_left(oracle_lib):
    pair = datagen.make_pair(120, 40, 32, seed=9, planes=(4, 6), occlusion=0.05)
    prm = _params((5, 5), 32, 4, 7, 86)
    a = oracle.run(pair["left"], pair["right"], prm)
    e = oracle.run_exact_lr(pair["left"], pair["right"], prm)
    np.testing.assert_array_equal(a["disp_left"], e["disp_left"])
    # where the exact check keeps a pixel the approximate map may differ, but
    # both outputs are D^L or invalid before the median
    prm0 = _params((5, 5), 32, 4, 7, 86, med=False)
    e0 = oracle.run_exact_lr(pair["left"], pair["right"], prm0)["disp"]
    keep = e0 != INV
    np.testing.assert_array_equal(e0[keep], e["disp_left"][keep])


# --------------------------------------------------------------- subpixel ---
@pytest.mark.parametrize("k,vertex", [(16, 0.25), (4, -0.5), (64, 0.125), (2, 0.0), (36, -1 / 3)])
def test_subpixel_offset_recovers_sampled_parabola(k, vertex):
    """Samples of S(d) = k (d - v)^2 + c at d = -1, 0, 1 give back v exactly."""
    c = 7.0
    s = [k * (dd - vertex) ** 2 + c for dd in (-1, 0, 1)]
    assert oracle.subpixel_offset(*s) == pytest.approx(vertex, abs=1e-12)


def test_subpixel_offset_special_cases():
    assert oracle.subpixel_offset(5, 5, 5) == 0.0          # flat: no parabola
    assert oracle.subpixel_offset(9, 1, 9) == 0.0          # symmetric
    assert oracle.subpixel_offset(4, 4, 10) == -0.5        # tie with the left neighbour
    assert oracle.subpixel_offset(10, 4, 4) == 0.5
    rng = np.random.default_rng(3)
    for _ in range(2000):
        b = int(rng.integers(0, 1000))
        a, c = b + int(rng.integers(0, 500)), b + int(rng.integers(0, 500))
        off = oracle.subpixel_offset(a, b, c)
        assert -0.5 <= off <= 0.5                           # the minimum's own cell


def test_refine_subpixel_volume_and_borders():
    h, w, nd = 3, 4, 8
    agg = np.full((h, w, nd), 1000, np.uint16)
    dl = np.zeros((h, w), np.uint16)
    # pixel (0, 0): parabola 16 (d - 3.25)^2 sampled at 2, 3, 4 -> 3.25
    agg[0, 0, 2:5] = [25, 1, 9]
    dl[0, 0] = 3
    # pixel (1, 1): winner at d = 0 and (2, 3) at d = D - 1: no offset
    agg[1, 1, 0:2] = [0, 3]
    dl[1, 1] = 0
    agg[2, 3, nd - 2:] = [3, 0]
    dl[2, 3] = nd - 1
    fine = oracle.refine_subpixel(agg, dl)
    assert fine[0, 0] == pytest.approx(3.25, abs=1e-12)
    assert fine[1, 1] == 0.0 and fine[2, 3] == nd - 1
    # every other pixel: flat 1000s -> no offset
    assert fine[0, 1] == 0.0


def test_float_median_reduces_to_integer_median(oracle_lib):
    """On integral values the float median equals the integer 3x3 median of
    App. F (invalid = -1.0 there, 0xFFFF here)."""
    rng = np.random.default_rng(11)
    d = rng.integers(0, 40, (17, 23)).astype(np.uint16)
    d[rng.random(d.shape) < 0.2] = INV
    ref = oracle.median3x3(d).astype(np.float64)
    ref[ref == INV] = oracle.INVALID_F
    got = oracle.median3x3_float(d.astype(np.float64), d != INV)
    np.testing.assert_array_equal(got, ref)


def test_run_subpixel_stays_within_half_a_disparity(oracle_lib):
    pair = datagen.make_pair(120, 40, 32, seed=19, planes=(4, 6), occlusion=0.0)
    prm = _params((9, 7), 32, 8, med=False)
    out = oracle.run_subpixel(pair["left"], pair["right"], prm)
    valid = out["disp"] != INV
    np.testing.assert_array_equal(out["disp_fine"] == oracle.INVALID_F, ~valid)
    diff = out["disp_fine"][valid] - out["disp"][valid]
    assert np.all(np.abs(diff) <= 0.5)
    assert np.any(diff != 0)
