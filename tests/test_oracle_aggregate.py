"""Oracle pins for the SGM path recursion and the path sum.

* Brute force: along every line of every direction, on tiny volumes, the exact
  minimum of the 1-D energy  sum_i C(p_i, d_i) + sum_i V(d_i, d_{i-1})  over all
  label sequences that end in d equals the oracle's L_r(p_k, d) plus the sum of
  the predecessor minima it subtracted (Eq. sgm_path, with V as printed).
* Closed forms: P1 = P2 = 0 and D = 1 both give S_bar = R * C.
* Bounds: C <= L_r <= C + P2 (the normalised form of L_r <= C + P2 + min L').
* Symmetry: mirroring x or y, or transposing, maps each path to its mirrored
  path; the 4- and 8-path sets are closed under these maps.
* The path sets: 4 = two horizontal + two vertical (Sec. 3.1.4), 8 adds the
  diagonals; aggregate_at agrees with the full volume everywhere.
"""
import itertools

import numpy as np
import pytest

import oracle as oracle_mod

DIRS = oracle_mod.DIRECTIONS


def _V(d, e, p1, p2):
    if d == e:
        return 0
    return p1 if abs(d - e) == 1 else p2


def _line_through(w, h, dx, dy, x, y):
    """Pixels of the path line that ends at (x, y), first pixel first."""
    pts = [(x, y)]
    while 0 <= pts[0][0] - dx < w and 0 <= pts[0][1] - dy < h:
        pts.insert(0, (pts[0][0] - dx, pts[0][1] - dy))
    return pts


def _brute_min_energy(costs, p1, p2):
    """costs: list of D-vectors along a line.  Returns, for the last pixel,
    min over all label sequences ending in d of the 1-D SGM energy."""
    n, nd = len(costs), len(costs[0])
    best = [None] * nd
    for seq in itertools.product(range(nd), repeat=n):
        e = sum(int(costs[i][seq[i]]) for i in range(n))
        e += sum(_V(seq[i], seq[i - 1], p1, p2) for i in range(1, n))
        d = seq[-1]
        if best[d] is None or e < best[d]:
            best[d] = e
    return best


@pytest.mark.parametrize("p1,p2", [(0, 0), (1, 5), (3, 3), (5, 40), (0, 7), (2, 9)])
def test_path_equals_brute_force_line_minimum(oracle_lib, p1, p2):
    rng = np.random.default_rng(p1 * 100 + p2)
    w, h, nd = 5, 4, 3
    c = rng.integers(0, 25, (h, w, nd), dtype=np.uint8)
    for (dx, dy) in DIRS:
        L = oracle_lib.path(c, (dx, dy), p1, p2).astype(np.int64)
        for y in range(h):
            for x in range(w):
                line = _line_through(w, h, dx, dy, x, y)
                if len(line) > 5:
                    continue
                costs = [c[py, px] for (px, py) in line]
                brute = _brute_min_energy(costs, p1, p2)
                offset = sum(int(L[py, px].min()) for (px, py) in line[:-1])
                assert list(L[y, x] + offset) == brute, ((dx, dy), (x, y))


def test_path_brute_force_wider_disparity_range(oracle_lib):
    rng = np.random.default_rng(77)
    c = rng.integers(0, 40, (1, 5, 5), dtype=np.uint8)
    for p1, p2 in [(4, 11), (1, 30)]:
        for (dx, dy) in ((1, 0), (-1, 0)):
            L = oracle_lib.path(c, (dx, dy), p1, p2).astype(np.int64)
            for x in range(5):
                line = _line_through(5, 1, dx, dy, x, 0)
                brute = _brute_min_energy([c[0, px] for (px, _) in line], p1, p2)
                offset = sum(int(L[0, px].min()) for (px, _) in line[:-1])
                assert list(L[0, x] + offset) == brute


def test_path_matches_literal_min_over_all_d_prime(oracle_lib):
    """The oracle's four-term form equals the printed min over every d' with the
    three-case V, minus the predecessor minimum, for P1 <= P2."""
    rng = np.random.default_rng(8)
    nd = 9
    c = rng.integers(0, 63, (1, 12, nd), dtype=np.uint8)
    for p1, p2 in [(0, 0), (3, 3), (7, 86), (10, 120)]:
        L = oracle_lib.path(c, (1, 0), p1, p2).astype(np.int64)
        prev = c[0, 0].astype(np.int64)
        assert np.array_equal(L[0, 0], prev)
        for x in range(1, 12):
            m = prev.min()
            cur = np.array([int(c[0, x, d]) + min(prev[e] + _V(d, e, p1, p2) for e in range(nd)) - m
                            for d in range(nd)])
            assert np.array_equal(L[0, x], cur)
            prev = cur


@pytest.mark.parametrize("npaths", [4, 8])
def test_zero_penalties_and_single_disparity_give_r_times_cost(oracle_lib, npaths):
    rng = np.random.default_rng(npaths)
    c = rng.integers(0, 256, (9, 13, 6), dtype=np.uint8)
    np.testing.assert_array_equal(oracle_lib.aggregate(c, npaths, 0, 0),
                                  npaths * c.astype(np.uint16))
    c1 = c[:, :, :1].copy()
    np.testing.assert_array_equal(oracle_lib.aggregate(c1, npaths, 10, 120),
                                  npaths * c1.astype(np.uint16))


@pytest.mark.parametrize("p1,p2", [(7, 86), (10, 120), (0, 255), (20, 20)])
def test_path_bounds(oracle_lib, p1, p2):
    rng = np.random.default_rng(p2)
    c = rng.integers(0, 256, (11, 14, 16), dtype=np.uint8)
    for r in DIRS:
        L = oracle_lib.path(c, r, p1, p2).astype(np.int64)
        assert np.all(L >= c) and np.all(L <= c.astype(np.int64) + p2)
        # at least one disparity keeps its full predecessor term: min_d (L - C) <= P2
        assert np.all((L - c).min(axis=2) <= p2)


def test_path_symmetries(oracle_lib):
    rng = np.random.default_rng(21)
    c = rng.integers(0, 256, (7, 10, 5), dtype=np.uint8)
    p1, p2 = 9, 70
    for (dx, dy) in DIRS:
        base = oracle_lib.path(c, (dx, dy), p1, p2)
        mx = oracle_lib.path(c[:, ::-1], (-dx, dy), p1, p2)
        np.testing.assert_array_equal(mx[:, ::-1], base)
        my = oracle_lib.path(c[::-1], (dx, -dy), p1, p2)
        np.testing.assert_array_equal(my[::-1], base)
        t = oracle_lib.path(c.transpose(1, 0, 2), (dy, dx), p1, p2)
        np.testing.assert_array_equal(t.transpose(1, 0, 2), base)


@pytest.mark.parametrize("npaths", [4, 8])
def test_path_sets_and_sum(oracle_lib, npaths):
    rng = np.random.default_rng(30 + npaths)
    c = rng.integers(0, 256, (8, 11, 7), dtype=np.uint8)
    p1, p2 = 10, 120
    expect = np.zeros(c.shape, np.int64)
    for r in DIRS[:npaths]:
        expect += oracle_lib.path(c, r, p1, p2)
    agg = oracle_lib.aggregate(c, npaths, p1, p2)
    np.testing.assert_array_equal(agg, expect)
    # the 4-path set is exactly the horizontal and vertical steps
    assert set(DIRS[:4]) == {(1, 0), (-1, 0), (0, 1), (0, -1)}
    assert set(DIRS) - set(DIRS[:4]) == {(1, 1), (-1, 1), (1, -1), (-1, -1)}
    # the sets are closed under mirroring and transposition
    for s in (DIRS[:npaths],):
        assert {(-a, b) for a, b in s} == set(s) and {(b, a) for a, b in s} == set(s)
    np.testing.assert_array_equal(oracle_lib.aggregate(c[:, ::-1].copy(), npaths, p1, p2)[:, ::-1], agg)
    np.testing.assert_array_equal(
        oracle_lib.aggregate(c.transpose(1, 0, 2).copy(), npaths, p1, p2).transpose(1, 0, 2), agg)
    for y in range(c.shape[0]):
        for x in range(c.shape[1]):
            np.testing.assert_array_equal(oracle_lib.aggregate_at(c, npaths, p1, p2, x, y), agg[y, x])


def test_aggregate_overflow_bound_is_enforced(oracle_lib):
    c = np.zeros((2, 2, 2), np.uint8)
    with pytest.raises(AssertionError):
        oracle_lib.aggregate(c, 8, 10, 8000)
    with pytest.raises(AssertionError):
        oracle_lib.aggregate(c, 8, 20, 10)
    oracle_lib.aggregate(c, 8, 10, 65535 // 8 - 255)
