"""The oracle's threaded driver (used only to time the oracle on every host
core) must give run()'s maps bit for bit: it splits the same functions over
independent images, rows and path lines and adds no arithmetic of its own."""
import numpy as np
import pytest

import oracle
from paper_2106_07927_amd import datagen


@pytest.mark.parametrize("w,h,nd,npaths,t,med,threads", [
    (97, 33, 32, 8, 1, True, 4),     # ragged sizes, more lines than threads
    (40, 70, 16, 4, 0, False, 3),    # tall frame, 4 paths, check without median
    (64, 48, 64, 8, -1, True, 8),    # no LR check
    (5, 3, 8, 8, 2, True, 16),       # more threads than rows or lines
    (1, 1, 4, 4, 1, True, 2),
])
def test_threaded_oracle_equals_run(oracle_lib, w, h, nd, npaths, t, med, threads):
    pair = datagen.make_pair(w, h, nd, 7100 + w + h, (2, 6), 0.05)
    prm = oracle.Params(win_w=9, win_h=7, ndisp=nd, npaths=npaths, p1=10, p2=120,
                        lr_tolerance=t, median3x3=med)
    ref = oracle.run(pair["left"], pair["right"], prm)
    got = oracle.run_threaded(pair["left"], pair["right"], prm, threads)
    for key in ("disp_left", "disp_right", "disp"):
        assert np.array_equal(got[key], ref[key]), key


def test_threaded_oracle_large_penalty(oracle_lib):
    """P2 above 255 (the NCC setting) through the threaded driver."""
    pair = datagen.make_pair(80, 30, 32, 7200, (2, 6), 0.0)
    prm = oracle.Params(win_w=5, win_h=5, ndisp=32, npaths=8, p1=90, p2=880,
                        lr_tolerance=1, median3x3=True)
    ref = oracle.run(pair["left"], pair["right"], prm)
    got = oracle.run_threaded(pair["left"], pair["right"], prm, 5)
    for key in ("disp_left", "disp_right", "disp"):
        assert np.array_equal(got[key], ref[key]), key
