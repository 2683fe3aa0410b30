"""Pins of the oracle's inverted, truncated NCC cost (Sec. 2.1.1, Sec. 2.2.1)
against the textbook zero-mean normalised cross-correlation, closed-form
invariances and special cases."""
import numpy as np
import pytest

import oracle
from paper_2106_07927_amd import datagen


def textbook_cost(left, right, win, ndisp):
    """float64 ZNCC from patch means and deviations, zero margin, then
    round(255 (1 - max(0, Phi))); returns (cost, 255 s before rounding)."""
    r = (win - 1) // 2
    h, w = left.shape
    pl = np.zeros((h + 2 * r, w + 2 * r))
    pr = np.zeros((h + 2 * r, w + 2 * r))
    pl[r:r + h, r:r + w] = left
    pr[r:r + h, r:r + w] = right
    cost = np.full((h, w, ndisp), 255, np.int64)
    raw = np.full((h, w, ndisp), np.nan)
    for y in range(h):
        for x in range(w):
            a = pl[y: y + win, x: x + win].ravel()
            a0 = a - a.mean()
            for d in range(min(ndisp, x + 1)):
                b = pr[y: y + win, x - d: x - d + win].ravel()
                b0 = b - b.mean()
                den = np.sqrt((a0 * a0).sum() * (b0 * b0).sum())
                phi = (a0 * b0).sum() / den if den > 0 else 0.0
                v = 255.0 * (1.0 - max(0.0, phi))
                raw[y, x, d] = v
                cost[y, x, d] = min(255, max(0, int(np.rint(v))))
    return cost, raw


@pytest.mark.parametrize("win", [5, 9])
def test_ncc_matches_textbook_definition(oracle_lib, win):
    left, right = datagen.random_images(23, 11, seed=40 + win)
    right = (right // 2 + left // 2).astype(np.uint8)          # correlated pair
    got = oracle.ncc_cost(left, right, win, 8).astype(np.int64)
    ref, raw = textbook_cost(left, right, win, 8)
    # float32 vs float64 may round differently only next to a .5 boundary
    near_tie = np.abs(raw - np.floor(raw) - 0.5) < 1e-3
    diff = got != ref
    assert not np.any(diff & ~near_tie), np.argwhere(diff & ~near_tie)[:5]
    assert np.all(np.abs(got - ref) <= 1)
    assert len(np.unique(got)) > 20


def test_ncc_pure_shift_is_zero_at_the_true_disparity(oracle_lib):
    d0, w, h = 5, 80, 24
    pair = datagen.pure_shift_pair(w, h, d0, seed=8)
    c = oracle.ncc_cost(pair["left"], pair["right"], 9, 12)
    m = 4
    assert np.all(c[m:-m, d0 + m: w - d0 - m, d0] == 0)


def _interior(c, win):
    """Elements whose two patches lie inside the image (the zero margin does
    not follow an intensity map)."""
    r = (win - 1) // 2
    h, w, nd = c.shape
    keep = np.zeros(c.shape, bool)
    for d in range(nd):
        keep[r: h - r, d + r: w - r, d] = True
    return keep


def test_ncc_invariant_to_positive_affine_intensity_maps(oracle_lib):
    """Phi is unchanged by I -> a I + b with a a power of two: the integer
    sums scale exactly, and so do the float32 square roots and quotient."""
    left, right = datagen.random_images(40, 14, seed=3)
    left, right = left // 3, right // 3                          # <= 85: no clipping
    for win in (5, 9):
        base = oracle.ncc_cost(left, right, win, 10)
        keep = _interior(base, win)
        for a, b in (((2 * left + 7), right), (left, (2 * right + 40)), (left + 100, right + 3)):
            got = oracle.ncc_cost(a.astype(np.uint8), b.astype(np.uint8), win, 10)
            np.testing.assert_array_equal(got[keep], base[keep])


def test_ncc_negated_image_flips_the_correlation(oracle_lib):
    """I_R -> 255 - I_R negates Phi exactly (num changes sign, the variances
    stay), so perfectly correlated patches become perfectly anti-correlated:
    cost 0 turns into 255 and the truncation makes every positive Phi 255."""
    d0, w, h = 4, 60, 20
    pair = datagen.pure_shift_pair(w, h, d0, seed=12)
    inv = (255 - pair["right"]).astype(np.uint8)
    c = oracle.ncc_cost(pair["left"], pair["right"], 5, 8)
    ci = oracle.ncc_cost(pair["left"], inv, 5, 8)
    m = 2
    assert np.all(ci[m:-m, d0 + m: w - d0 - m, d0] == 255)
    # with zero margin the border windows differ (255 - 0 != 0); inside they
    # pair up: cost < 255 on one side means Phi > 0, i.e. 255 on the other
    inner = (slice(m, -m), slice(8 + m, w - m))
    assert np.all((c[inner] == 255) | (ci[inner] == 255))


def test_ncc_special_cases(oracle_lib):
    flat = np.full((10, 20), 77, np.uint8)
    tex, _ = datagen.random_images(20, 10, seed=1)
    c = oracle.ncc_cost(tex, flat, 5, 6)
    # a zero-variance right patch has no correlation: cost 255 (the zero
    # margin gives border patches variance, so look inside)
    assert np.all(c[2:-2, 7:-2, :] == 255)
    c2 = oracle.ncc_cost(tex, tex, 5, 6)
    for d in range(6):
        assert np.all(c2[:, :d, d] == 255)                      # x - d < 0
    assert np.all(c2[:, :, 0] == 0)                              # identical patches
