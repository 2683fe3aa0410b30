"""Oracle pins for the census transform and the Hamming cost.

Census: hand-derived descriptors (bit direction, raster order, zero margin,
window orientation), invariance under strictly increasing grey maps that fix
0, and shift equivariance.  The paper prints no census example, so the bit
layout itself rests on the readings listed with the design notes.
Cost: hand-built XOR/popcount, the 0xFF rule for x - d < 0, zero cost at
the true shift of a pure-shift pair, and census + cost together against a
count of disagreeing window comparisons taken straight from the images (no
descriptor formed), which holds for any bit layout of the descriptors.
"""
import numpy as np
import pytest

from paper_2106_07927_amd import datagen


def test_census_5x5_hand_examples(oracle_lib):
    img = np.arange(25, dtype=np.uint8).reshape(5, 5)
    cen = oracle_lib.census(img, 5, 5)
    # centre 12: raster neighbours 0..11 are smaller (1), 13..24 larger (0)
    assert int(cen[2, 2]) == int("1" * 12 + "0" * 12, 2)
    # value 0: nothing is smaller, the zero margin is not smaller either
    assert int(cen[0, 0]) == 0
    # value 24: every in-image neighbour and every margin zero is smaller
    assert int(cen[4, 4]) == (1 << 24) - 1
    # pixel (x=1, y=1), value 6, worked row by row (dy = -2 .. 2):
    #   margin row              -> 11111
    #   x=-1 margin, 0,1,2,3     -> 11111
    #   margin, 5, [centre], 7, 8 -> 1100
    #   margin, 10..13           -> 10000
    #   margin, 15..18           -> 10000
    assert int(cen[1, 1]) == int("11111" "11111" "1100" "10000" "10000", 2)


def test_census_9x7_is_nine_wide_seven_tall(oracle_lib):
    img = np.full((7, 9), 50, np.uint8)
    img[3, 4] = 100          # centre
    img[3, 8] = 200          # dx = +4, dy = 0: inside a 9-wide window only
    cen = int(oracle_lib.census(img, 9, 7)[3, 4])
    # raster index of (dy=0, dx=4): 3 full rows of 9, then 4 left of centre,
    # then dx = 1, 2, 3 -> 27 + 4 + 3 = 34 of 62; first bit ends highest
    expect = ((1 << 62) - 1) ^ (1 << (61 - 34))
    assert cen == expect
    img[3, 8] = 50
    img[0, 4] = 200          # dy = -3: inside a 7-tall window (first row)
    cen = int(oracle_lib.census(img, 9, 7)[3, 4])
    assert cen == ((1 << 62) - 1) ^ (1 << (61 - 4))


def test_census_ties_are_zero_and_margin_reads_zero(oracle_lib):
    img = np.full((1, 1), 7, np.uint8)
    assert int(oracle_lib.census(img, 9, 7)[0, 0]) == (1 << 62) - 1
    img = np.zeros((1, 1), np.uint8)
    assert int(oracle_lib.census(img, 9, 7)[0, 0]) == 0
    img = np.full((6, 6), 9, np.uint8)   # equal neighbours give 0, margin gives 1
    cen = oracle_lib.census(img, 5, 5)
    assert int(cen[3, 3]) == 0           # window fully inside
    assert bin(int(cen[0, 0])).count("1") == 24 - 8   # 8 in-image neighbours


@pytest.mark.parametrize("win", [(5, 5), (9, 7)])
def test_census_monotone_invariance(oracle_lib, win):
    rng = np.random.default_rng(3)
    img = rng.integers(0, 100, (23, 37), dtype=np.uint8)
    # strictly increasing map on 0..99 with g(0) = 0, so the zero margin maps
    # to itself and every comparison keeps its outcome
    g = np.zeros(100, np.int64)
    g[1:] = np.sort(rng.choice(np.arange(1, 256), 99, replace=False))
    mapped = g[img].astype(np.uint8)
    np.testing.assert_array_equal(oracle_lib.census(img, *win), oracle_lib.census(mapped, *win))
    # a map that does not fix 0 changes the border descriptors only
    shifted = (img.astype(np.int64) + 1).astype(np.uint8)
    a, b = oracle_lib.census(img, *win), oracle_lib.census(shifted, *win)
    rx, ry = (win[0] - 1) // 2, (win[1] - 1) // 2
    np.testing.assert_array_equal(a[ry:-ry, rx:-rx], b[ry:-ry, rx:-rx])
    assert np.any(a != b)


@pytest.mark.parametrize("win", [(5, 5), (9, 7)])
def test_census_shift_equivariance(oracle_lib, win):
    rng = np.random.default_rng(4)
    img = rng.integers(0, 256, (30, 40), dtype=np.uint8)
    sx, sy = 3, 2
    shifted = np.zeros_like(img)
    shifted[sy:, sx:] = img[:-sy, :-sx]
    a = oracle_lib.census(img, *win)
    b = oracle_lib.census(shifted, *win)
    rx, ry = (win[0] - 1) // 2, (win[1] - 1) // 2
    # away from every border both windows see the same pixels
    inner_a = a[ry: 30 - sy - ry, rx: 40 - sx - rx]
    inner_b = b[sy + ry: 30 - ry, sx + rx: 40 - rx]
    np.testing.assert_array_equal(inner_a, inner_b)


def test_cost_hand_example(oracle_lib):
    cl = np.array([[0b1011, 0b1111]], np.uint64)
    cr = np.array([[0b0110, 0b0000]], np.uint64)
    c = oracle_lib.cost(cl, cr, 3)
    # x=0: d=0 -> 1011^0110 = 1101 -> 3; d>=1 leaves the image -> 255
    # x=1: d=0 -> 1111^0000 -> 4; d=1 -> 1111^0110 = 1001 -> 2; d=2 -> 255
    np.testing.assert_array_equal(c[0], [[3, 255, 255], [4, 2, 255]])


def test_cost_full_width_descriptor(oracle_lib):
    cl = np.array([[(1 << 62) - 1, 0]], np.uint64)
    cr = np.array([[0, 0]], np.uint64)
    c = oracle_lib.cost(cl, cr, 2)
    assert c[0, 0, 0] == 62 and c[0, 1, 1] == 0 and c[0, 1, 0] == 0


@pytest.mark.parametrize("win,d0", [((5, 5), 0), ((5, 5), 7), ((9, 7), 13), ((9, 7), 31)])
def test_cost_zero_at_true_shift(oracle_lib, win, d0):
    w, h, nd = 80, 24, 32
    pair = datagen.pure_shift_pair(w, h, d0, seed=100 + d0)
    cl = oracle_lib.census(pair["left"], *win)
    cr = oracle_lib.census(pair["right"], *win)
    c = oracle_lib.cost(cl, cr, nd)
    rx = (win[0] - 1) // 2
    xs = np.arange(w)
    interior = (xs - d0 - rx >= 0) & (xs + rx <= w - 1)
    assert np.all(c[:, interior, d0] == 0)
    # the 0xFF rule and the descriptor-length bound
    bits = win[0] * win[1] - 1
    for d in range(nd):
        assert np.all(c[:, :d, d] == 255)
        assert np.all(c[:, d:, d] <= bits)


def _cost_from_images(left, right, win, nd):
    """Hamming cost written straight from the images: for every window offset,
    whether the neighbour is darker than the centre in the left image and in
    the right image at x - d, counted where the two disagree; a zero margin
    outside the image; 255 where x - d < 0.  No descriptor is formed, so the
    count does not depend on how the bits of a descriptor are laid out."""
    h, w = left.shape
    rx, ry = (win[0] - 1) // 2, (win[1] - 1) // 2
    pl = np.zeros((h + 2 * ry, w + 2 * rx), np.int64)
    pr = np.zeros_like(pl)
    pl[ry:ry + h, rx:rx + w] = left
    pr[ry:ry + h, rx:rx + w] = right
    bits_l, bits_r = [], []
    for dy in range(-ry, ry + 1):
        for dx in range(-rx, rx + 1):
            if dx == 0 and dy == 0:
                continue
            bits_l.append(pl[ry + dy:ry + dy + h, rx + dx:rx + dx + w] < left)
            bits_r.append(pr[ry + dy:ry + dy + h, rx + dx:rx + dx + w] < right)
    bl, br = np.stack(bits_l), np.stack(bits_r)          # [offsets][H][W]
    out = np.full((h, w, nd), 255, np.int64)
    for d in range(min(nd, w)):
        out[:, d:, d] = np.sum(bl[:, :, d:] != br[:, :, :w - d], axis=0)
    return out


@pytest.mark.parametrize("win,shape,nd,levels", [((5, 5), (17, 23), 12, 256), ((9, 7), (19, 31), 20, 256),
                                                 ((9, 7), (21, 26), 16, 4), ((5, 5), (13, 15), 8, 3),
                                                 ((9, 7), (5, 6), 9, 256), ((5, 5), (1, 9), 4, 2)])
def test_cost_equals_window_comparison_count(oracle_lib, win, shape, nd, levels):
    """The census + Hamming cost of the oracle equals the count above; few
    grey levels put many ties (and zeros against the margin) in every window."""
    rng = np.random.default_rng(7 + nd)
    h, w = shape
    left = rng.integers(0, levels, (h, w), dtype=np.uint8)
    right = rng.integers(0, levels, (h, w), dtype=np.uint8)
    right[:, ::3] = left[:, ::3]
    cost = oracle_lib.cost(oracle_lib.census(left, *win), oracle_lib.census(right, *win), nd)
    np.testing.assert_array_equal(cost.astype(np.int64), _cost_from_images(left, right, win, nd))
