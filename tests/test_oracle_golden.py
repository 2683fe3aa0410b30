"""Oracle pins from the worked examples the paper prints (tests/golden/)."""
import itertools

import numpy as np
from conftest import read_golden


def _halving_rounds(values):
    """Replay of the pairing the figure draws: element i meets element i + n/2."""
    vals = list(values)
    labels = list(range(1, len(vals) + 1))
    rounds = []
    while len(vals) > 1:
        half = len(vals) // 2
        nv, nl = [], []
        for i in range(half):
            a, b = (vals[i], labels[i]), (vals[i + half], labels[i + half])
            keep = a if a <= b else b
            nv.append(keep[0])
            nl.append(keep[1])
        vals, labels = nv, nl
        rounds.append((vals, labels))
    return rounds


def test_map_reduce_pairing_matches_figure():
    g = read_golden("map_reduce_min.txt")
    rounds = _halving_rounds(g["values"])
    assert rounds[0] == (g["round1_values"], g["round1_labels"])
    assert rounds[1] == (g["round2_values"], g["round2_labels"])
    assert rounds[2] == ([g["result_value"][0]], [g["result_label"][0]])


def test_map_reduce_argmin_worked_example(oracle_lib):
    g = read_golden("map_reduce_min.txt")
    idx = oracle_lib.map_reduce_argmin(g["values"])
    assert idx + 1 == g["result_label"][0]          # labels are 1-based in the figure
    assert g["values"][idx] == g["result_value"][0]


def test_wta_worked_example(oracle_lib):
    g = read_golden("map_reduce_min.txt")
    agg = np.array(g["values"], np.uint16).reshape(1, 1, 8)
    assert oracle_lib.wta(agg)[0, 0] == g["result_label"][0] - 1


def test_map_reduce_ties_keep_lowest_index(oracle_lib):
    rng = np.random.default_rng(5)
    for _ in range(200):
        v = rng.integers(0, 4, 16)
        assert oracle_lib.map_reduce_argmin(v) == int(np.argmin(v))


def test_median_network_worked_example(oracle_lib):
    g = read_golden("sorting_network_median.txt")
    assert sorted(g["inputs"]) == g["outputs"]
    assert oracle_lib.median9(g["inputs"]) == g["median"][0]
    img = np.array(g["inputs"], np.uint16).reshape(3, 3)
    assert oracle_lib.median3x3(img)[1, 1] == g["median"][0]


def test_bubble_first_pass_matches_figure():
    """The first pass the figure draws: comparators top to bottom, smaller up."""
    g = read_golden("sorting_network_median.txt")
    v = list(g["inputs"])
    for i in range(8):
        if v[i] > v[i + 1]:
            v[i], v[i + 1] = v[i + 1], v[i]
    assert v == g["after_pass1"]


def test_median9_equals_sorted_middle(oracle_lib):
    """Five passes suffice: the network's wire E equals the library sort's
    middle element on random and on heavily tied inputs."""
    rng = np.random.default_rng(11)
    for high in (3, 10, 0x10000):
        for _ in range(300):
            v = rng.integers(0, high, 9)
            assert oracle_lib.median9(v) == int(np.sort(v)[4])
    for v in itertools.product((0, 0xFFFF), repeat=9):
        assert oracle_lib.median9(v) == sorted(v)[4]
