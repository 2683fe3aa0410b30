"""Oracle pins for WTA, the approximate right disparity, the LR check, the
median, and the whole path on pure-shift and synthetically warped pairs."""
import numpy as np
import pytest

import oracle as oracle_mod
from paper_2106_07927_amd import datagen

INV = 0xFFFF


def test_wta_ties_take_smallest_d(oracle_lib):
    agg = np.array([[[5, 3, 3, 7], [9, 9, 9, 9], [1, 0, 0, 0]]], np.uint16)
    np.testing.assert_array_equal(oracle_lib.wta(agg), [[1, 0, 1]])


def test_right_disparity_hand_example(oracle_lib):
    # S_bar(x, d):  x0: [5, 9]  x1: [4, 2]  x2: [7, 1]
    agg = np.array([[[5, 9], [4, 2], [7, 1]]], np.uint16)
    # D^R(0) = argmin(S(0,0)=5, S(1,1)=2) = 1
    # D^R(1) = argmin(S(1,0)=4, S(2,1)=1) = 1
    # D^R(2) = only d=0 keeps x + d inside the image -> 0
    np.testing.assert_array_equal(oracle_lib.right_disparity(agg), [[1, 1, 0]])
    np.testing.assert_array_equal(oracle_lib.wta(agg), [[0, 1, 1]])
    tie = np.full((1, 4, 3), 6, np.uint16)
    np.testing.assert_array_equal(oracle_lib.right_disparity(tie), [[0, 0, 0, 0]])


def test_lr_check_hand_examples(oracle_lib):
    dl = np.array([[0, 1, 1]], np.uint16)
    dr = np.array([[1, 1, 0]], np.uint16)
    # t=1: x0 |0 - D^R(0)=1| = 1 keep; x1 |1 - D^R(0)| = 0 keep; x2 |1 - D^R(1)| = 0 keep
    np.testing.assert_array_equal(oracle_lib.lr_check(dl, dr, 1), [[0, 1, 1]])
    np.testing.assert_array_equal(oracle_lib.lr_check(dl, dr, 0), [[INV, 1, 1]])
    dl = np.array([[1, 0, 2]], np.uint16)
    dr = np.array([[0, 0, 0]], np.uint16)
    # x0: 0 - 1 < 0 -> invalid; x1 keeps 0; x2: |2 - D^R(0)| = 2 > 1 -> invalid
    np.testing.assert_array_equal(oracle_lib.lr_check(dl, dr, 1), [[INV, 0, INV]])
    np.testing.assert_array_equal(oracle_lib.lr_check(dl, dr, 2), [[INV, 0, 2]])


def test_median3x3_definition(oracle_lib):
    rng = np.random.default_rng(2)
    for trial in range(20):
        h, w = rng.integers(1, 9, 2)
        d = rng.integers(0, 6, (h, w)).astype(np.uint16)
        d[rng.random((h, w)) < 0.2] = INV
        out = oracle_lib.median3x3(d)
        pad = np.full((h + 2, w + 2), INV, np.int64)
        pad[1:-1, 1:-1] = d
        for y in range(h):
            for x in range(w):
                if d[y, x] == INV:
                    assert out[y, x] == INV
                else:
                    assert out[y, x] == np.sort(pad[y:y + 3, x:x + 3].ravel())[4]


def test_median_corners_become_invalid(oracle_lib):
    d = np.full((5, 5), 3, np.uint16)
    out = oracle_lib.median3x3(d)
    # a corner sees 5 padding values of 0xFFFF and 4 valid ones
    assert out[0, 0] == INV and out[4, 4] == INV
    assert out[0, 2] == 3 and out[2, 2] == 3


def _params(win, nd, npaths, p1=10, p2=120, t=1, med=True):
    return oracle_mod.Params(win_w=win[0], win_h=win[1], ndisp=nd, npaths=npaths,
                             p1=p1, p2=p2, lr_tolerance=t, median3x3=med)


@pytest.mark.parametrize("win,npaths,d0", [((5, 5), 4, 0), ((5, 5), 4, 5),
                                           ((9, 7), 8, 12), ((9, 7), 8, 23)])
def test_pure_shift_recovers_constant_disparity(oracle_lib, win, npaths, d0):
    w, h, nd = 96, 40, 32
    pair = datagen.pure_shift_pair(w, h, d0, seed=500 + d0)
    out = oracle_lib.run(pair["left"], pair["right"], _params(win, nd, npaths))
    rx = (win[0] - 1) // 2
    x0, x1 = d0 + rx + 2, w - rx - 2
    assert np.all(out["disp_left"][:, x0:x1] == d0)
    # D^R(x) compares the left pixels x .. x + D - 1; near the left border
    # those include pixels whose true match lies outside the right image, so
    # the check starts where every candidate is an interior pixel
    assert np.all(out["disp_right"][:, x0: x1 - d0] == d0)
    assert np.all(out["disp"][1:-1, x0 + 1: x1 - 1] == d0)


def test_synthetic_ground_truth_small(oracle_lib):
    cfg = datagen.CONFIGS["c1_320x240_d64_r4"]
    pair = datagen.config_pair("c1_320x240_d64_r4")
    prm = _params((cfg["win_w"], cfg["win_h"]), cfg["ndisp"], cfg["npaths"], cfg["p1"],
                  cfg["p2"], cfg["lr_tolerance"], cfg["median3x3"])
    out = oracle_lib.run(pair["left"], pair["right"], prm)
    gt = pair["disp_gt"].astype(np.int64)
    d = out["disp"].astype(np.int64)
    good = ~pair["occluded"]
    d1 = np.mean(np.abs(d - gt)[good] >= 3)          # Eq. (accuracyKitti)
    assert d1 < 0.03, d1


@pytest.mark.slow
def test_synthetic_ground_truth_lr_check(oracle_lib):
    """With the LR check on: low D1 on valid non-occluded pixels, and most
    pixels the generator occluded are invalidated."""
    w, h, nd = 400, 160, 64
    pair = datagen.make_pair(w, h, nd, seed=31, planes=(6, 10), occlusion=0.05)
    out = oracle_lib.run(pair["left"], pair["right"], _params((9, 7), nd, 8))
    gt = pair["disp_gt"].astype(np.int64)
    d = out["disp"].astype(np.int64)
    valid = d != INV
    good = ~pair["occluded"] & valid
    d1 = np.mean(np.abs(d - gt)[good] >= 3)
    assert d1 < 0.02, d1
    # occluded pixels with a wrong WTA answer are mostly caught by the check
    wrong = pair["occluded"] & (np.abs(out["disp_left"].astype(np.int64) - gt) >= 3)
    caught = np.mean(~valid[wrong])
    assert caught > 0.6, caught
    assert valid.mean() > 0.5
