"""CPU oracle for the SGM stereo hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``libsgm_oracle.so`` (plain
scalar C, built from ``sgm_oracle.c`` by :func:`build`) with NumPy arrays and
shares no code with the HIP product path.

Each wrapper names the passage of the paper (Ruf et al., 2021, "ReS2tAC") that
its C function follows.  Parity of every function is pinned by the CPU tests
(``tests/test_oracle_*.py``) against worked examples printed in the paper,
brute force on tiny inputs, closed forms and invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgm_oracle.so")
SRC_PATH = os.path.join(HERE, "sgm_oracle.c")
MT_SRC_PATH = os.path.join(HERE, "sgm_oracle_mt.c")
INVALID = 0xFFFF

# Step r of each path; the predecessor of p is p - r.  First four: the
# horizontal and vertical paths; the eight-path set adds the diagonals.
DIRECTIONS = ((1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, 1), (1, -1), (-1, -1))


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, -O2, no vector intrinsics; the
    threaded driver with POSIX threads)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu99", "-Wall", "-Wextra", "-ffp-contract=off", "-shared",
             "-fPIC", "-pthread", SRC_PATH, MT_SRC_PATH, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        lib.sgm_oracle_census.argtypes = [P, I, I, I, I, P]
        lib.sgm_oracle_cost.argtypes = [P, P, I, I, I, P]
        lib.sgm_oracle_path.argtypes = [P, I, I, I, I, I, I, I, P]
        lib.sgm_oracle_aggregate.argtypes = [P, I, I, I, I, I, I, P]
        lib.sgm_oracle_aggregate_at.argtypes = [P, I, I, I, I, I, I, I, I, P]
        lib.sgm_oracle_wta.argtypes = [P, I, I, I, P]
        lib.sgm_oracle_right_disparity.argtypes = [P, I, I, I, P]
        lib.sgm_oracle_lr_check.argtypes = [P, P, I, I, I, P]
        lib.sgm_oracle_median3x3.argtypes = [P, I, I, P]
        lib.sgm_oracle_median9.argtypes = [P]
        lib.sgm_oracle_median9.restype = ctypes.c_uint16
        lib.sgm_oracle_map_reduce_argmin.argtypes = [P, I]
        lib.sgm_oracle_map_reduce_argmin.restype = I
        lib.sgm_oracle_ncc_cost.argtypes = [P, P, I, I, I, I, P]
        lib.sgm_oracle_ncc_cost.restype = None
        lib.sgm_oracle_run_threaded.argtypes = [P, P, I, I, I, I, I, I, I, I, I, I, I, P, P, P]
        lib.sgm_oracle_run_threaded.restype = I
        for name in ("sgm_oracle_census", "sgm_oracle_cost", "sgm_oracle_path",
                     "sgm_oracle_aggregate", "sgm_oracle_aggregate_at",
                     "sgm_oracle_wta", "sgm_oracle_right_disparity",
                     "sgm_oracle_lr_check", "sgm_oracle_median3x3"):
            getattr(lib, name).restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def census(img: np.ndarray, win_w: int, win_h: int) -> np.ndarray:
    """Census transform (Sec. 2.2.1 / 2.3.1): uint8 [H][W] -> uint64 [H][W]."""
    img = _c(img, np.uint8)
    h, w = img.shape
    assert win_w % 2 == 1 and win_h % 2 == 1 and win_w * win_h - 1 <= 64
    out = np.empty((h, w), np.uint64)
    _load().sgm_oracle_census(_ptr(img), w, h, win_w, win_h, _ptr(out))
    return out


def cost(census_left: np.ndarray, census_right: np.ndarray, ndisp: int) -> np.ndarray:
    """Hamming cost volume, Eq. (image_matching): -> uint8 [H][W][D]."""
    cl = _c(census_left, np.uint64)
    cr = _c(census_right, np.uint64)
    h, w = cl.shape
    assert cr.shape == cl.shape and 1 <= ndisp <= 256
    out = np.empty((h, w, ndisp), np.uint8)
    _load().sgm_oracle_cost(_ptr(cl), _ptr(cr), w, h, ndisp, _ptr(out))
    return out


def ncc_cost(left: np.ndarray, right: np.ndarray, win: int, ndisp: int) -> np.ndarray:
    """Inverted, truncated NCC cost (Sec. 2.1.1, Sec. 2.2.1), round(255 s) as
    uint8 [H][W][D]; float32 evaluation of the exact integer window sums."""
    a = _c(left, np.uint8)
    b = _c(right, np.uint8)
    h, w = a.shape
    out = np.empty((h, w, ndisp), np.uint8)
    _load().sgm_oracle_ncc_cost(_ptr(a), _ptr(b), w, h, win, ndisp, _ptr(out))
    return out


def _check_penalties(npaths: int, p1: int, p2: int):
    assert npaths in (4, 8)
    assert 0 <= p1 <= p2, "the reduced form of Eq. (sgm_path) needs P1 <= P2"
    assert npaths * (255 + p2) <= 0xFFFF, "aggregated costs must fit uint16"


def path(cost_vol: np.ndarray, direction, p1: int, p2: int) -> np.ndarray:
    """One path L_r of Eq. (sgm_path) for the step r = (dx, dy)."""
    c = _c(cost_vol, np.uint8)
    h, w, nd = c.shape
    dx, dy = direction
    assert 0 <= p1 <= p2 and 255 + p2 <= 0xFFFF
    out = np.empty((h, w, nd), np.uint16)
    _load().sgm_oracle_path(_ptr(c), w, h, nd, dx, dy, p1, p2, _ptr(out))
    return out


def aggregate(cost_vol: np.ndarray, npaths: int, p1: int, p2: int) -> np.ndarray:
    """Aggregated volume S_bar, Eq. (sgm_path_aggr): -> uint16 [H][W][D]."""
    _check_penalties(npaths, p1, p2)
    c = _c(cost_vol, np.uint8)
    h, w, nd = c.shape
    out = np.empty((h, w, nd), np.uint16)
    _load().sgm_oracle_aggregate(_ptr(c), w, h, nd, npaths, p1, p2, _ptr(out))
    return out


def aggregate_at(cost_vol: np.ndarray, npaths: int, p1: int, p2: int,
                 x: int, y: int) -> np.ndarray:
    """S_bar(x, y, :) alone, from the line recursions that end at (x, y)."""
    _check_penalties(npaths, p1, p2)
    c = _c(cost_vol, np.uint8)
    h, w, nd = c.shape
    assert 0 <= x < w and 0 <= y < h
    out = np.empty((nd,), np.uint16)
    _load().sgm_oracle_aggregate_at(_ptr(c), w, h, nd, npaths, p1, p2, x, y, _ptr(out))
    return out


def wta(agg: np.ndarray) -> np.ndarray:
    """Eq. (wta), smallest d on ties: uint16 [H][W][D] -> uint16 [H][W]."""
    a = _c(agg, np.uint16)
    h, w, nd = a.shape
    out = np.empty((h, w), np.uint16)
    _load().sgm_oracle_wta(_ptr(a), w, h, nd, _ptr(out))
    return out


def right_disparity(agg: np.ndarray) -> np.ndarray:
    """Eq. (right_disparity), d restricted to px + d < W, smallest d on ties."""
    a = _c(agg, np.uint16)
    h, w, nd = a.shape
    out = np.empty((h, w), np.uint16)
    _load().sgm_oracle_right_disparity(_ptr(a), w, h, nd, _ptr(out))
    return out


def lr_check(disp_left: np.ndarray, disp_right: np.ndarray, tolerance: int) -> np.ndarray:
    """Eq. (LR_check) with tolerance t (inclusive)."""
    dl = _c(disp_left, np.uint16)
    dr = _c(disp_right, np.uint16)
    h, w = dl.shape
    out = np.empty((h, w), np.uint16)
    _load().sgm_oracle_lr_check(_ptr(dl), _ptr(dr), w, h, tolerance, _ptr(out))
    return out


def median3x3(disp: np.ndarray) -> np.ndarray:
    """3x3 median of valid pixels, 0xFFFF padding (Sec. 2.2.4, App. F)."""
    d = _c(disp, np.uint16)
    h, w = d.shape
    out = np.empty((h, w), np.uint16)
    _load().sgm_oracle_median3x3(_ptr(d), w, h, _ptr(out))
    return out


def median9(values) -> int:
    """Median of nine values by five bubble-sort passes (App. F)."""
    v = _c(values, np.uint16)
    assert v.shape == (9,)
    return int(_load().sgm_oracle_median9(_ptr(v)))


def map_reduce_argmin(values) -> int:
    """Index of the minimum by pairwise halving (App. D); n a power of two."""
    v = _c(values, np.uint16)
    n = v.shape[0]
    assert n >= 1 and n & (n - 1) == 0
    return int(_load().sgm_oracle_map_reduce_argmin(_ptr(v), n))


@dataclass(frozen=True)
class Params:
    """Pipeline parameters.  lr_tolerance < 0 disables the LR check."""
    win_w: int = 9
    win_h: int = 7
    ndisp: int = 128
    npaths: int = 8
    p1: int = 10
    p2: int = 120
    lr_tolerance: int = 1
    median3x3: bool = True


def run(left: np.ndarray, right: np.ndarray, params: Params) -> dict:
    """The whole path, every intermediate kept: census -> cost -> S_bar ->
    D^L, D^R -> LR check -> median."""
    cl = census(left, params.win_w, params.win_h)
    cr = census(right, params.win_w, params.win_h)
    c = cost(cl, cr, params.ndisp)
    agg = aggregate(c, params.npaths, params.p1, params.p2)
    dl = wta(agg)
    dr = right_disparity(agg)
    d = lr_check(dl, dr, params.lr_tolerance) if params.lr_tolerance >= 0 else dl.copy()
    if params.median3x3:
        d = median3x3(d)
    return {"census_left": cl, "census_right": cr, "cost": c, "agg": agg,
            "disp_left": dl, "disp_right": dr, "disp": d}


def run_threaded(left: np.ndarray, right: np.ndarray, params: Params, nthreads: int) -> dict:
    """run() with its independent work spread over nthreads threads (the
    oracle's own functions on independent rows, images and path lines); for
    timing on all host cores.  D^L, D^R and D equal run()'s bit for bit."""
    _check_penalties(params.npaths, params.p1, params.p2)
    a = _c(left, np.uint8)
    b = _c(right, np.uint8)
    h, w = a.shape
    dl = np.empty((h, w), np.uint16)
    dr = np.empty((h, w), np.uint16)
    d = np.empty((h, w), np.uint16)
    rc = _load().sgm_oracle_run_threaded(_ptr(a), _ptr(b), w, h, params.win_w, params.win_h,
                                         params.ndisp, params.npaths, params.p1, params.p2,
                                         params.lr_tolerance, int(bool(params.median3x3)),
                                         int(nthreads), _ptr(dl), _ptr(dr), _ptr(d))
    if rc != 0:
        raise MemoryError("oracle: out of memory")
    return {"disp_left": dl, "disp_right": dr, "disp": d}


# ---------------------------------------------------------------------------
# Exact right disparity map (Sec. 2.1.3, occlusion detection; Sec. 3.1.3):
# instead of Eq. (right_disparity), the pair is swapped and flipped
# horizontally and matched again by the same census, cost, aggregation and
# WTA; the resulting map, flipped back, is D^R.
# ---------------------------------------------------------------------------
def exact_right_disparity(left: np.ndarray, right: np.ndarray, params: Params) -> np.ndarray:
    """D^R from scratch: WTA of the swapped, horizontally flipped pair."""
    ref = np.ascontiguousarray(right[:, ::-1])      # the right image becomes the reference
    mat = np.ascontiguousarray(left[:, ::-1])
    c = cost(census(ref, params.win_w, params.win_h), census(mat, params.win_w, params.win_h),
             params.ndisp)
    flipped = wta(aggregate(c, params.npaths, params.p1, params.p2))
    return np.ascontiguousarray(flipped[:, ::-1])


def run_exact_lr(left: np.ndarray, right: np.ndarray, params: Params) -> dict:
    """The path with the exact consistency check: D^L of the pair, D^R of the
    swapped and flipped pair, Eq. (LR_check), median."""
    cl = census(left, params.win_w, params.win_h)
    cr = census(right, params.win_w, params.win_h)
    dl = wta(aggregate(cost(cl, cr, params.ndisp), params.npaths, params.p1, params.p2))
    dr = exact_right_disparity(left, right, params)
    d = lr_check(dl, dr, params.lr_tolerance) if params.lr_tolerance >= 0 else dl.copy()
    if params.median3x3:
        d = median3x3(d)
    return {"disp_left": dl, "disp_right": dr, "disp": d}


# ---------------------------------------------------------------------------
# Subpixel refinement (Sec. 2.1.3): a parabola through the aggregated costs at
# the WTA disparity d and at d - 1, d + 1; its vertex offset is added to d.
# Floating point, here in float64.  Invalid pixels are -1.0.
# ---------------------------------------------------------------------------
INVALID_F = -1.0


def subpixel_offset(s_prev: float, s_min: float, s_next: float) -> float:
    """Vertex of the parabola through (-1, s_prev), (0, s_min), (1, s_next)."""
    den = s_prev - 2.0 * s_min + s_next
    if den <= 0.0:
        return 0.0
    return (s_prev - s_next) / (2.0 * den)


def refine_subpixel(agg: np.ndarray, disp_left: np.ndarray) -> np.ndarray:
    """d + offset for every pixel, from S_bar at d - 1, d, d + 1; no offset at
    d = 0 or d = D - 1 (one neighbour is missing)."""
    a = np.asarray(agg, np.float64)
    h, w, nd = a.shape
    d = np.asarray(disp_left, np.int64)
    out = d.astype(np.float64)
    inner = (d > 0) & (d < nd - 1)
    ys, xs = np.nonzero(inner)
    dd = d[ys, xs]
    sp, s0, sn = a[ys, xs, dd - 1], a[ys, xs, dd], a[ys, xs, dd + 1]
    den = sp - 2.0 * s0 + sn
    off = np.where(den > 0, (sp - sn) / (2.0 * np.where(den > 0, den, 1.0)), 0.0)
    out[ys, xs] += off
    return out


def median3x3_float(values: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """3x3 median of a float map (Sec. 2.1.3): invalid pixels stay invalid;
    in the window, pixels outside the image and invalid pixels count as +inf;
    a median of +inf is invalid."""
    h, w = values.shape
    v = np.where(valid, values, np.inf)
    pad = np.full((h + 2, w + 2), np.inf)
    pad[1:-1, 1:-1] = v
    win = np.stack([pad[1 + dy: 1 + dy + h, 1 + dx: 1 + dx + w]
                    for dy in (-1, 0, 1) for dx in (-1, 0, 1)], axis=-1)
    med = np.sort(win, axis=-1)[..., 4]
    out = np.where(valid & np.isfinite(med), med, INVALID_F)
    return out


def run_subpixel(left: np.ndarray, right: np.ndarray, params: Params) -> dict:
    """The path with subpixel refinement: integer D^L, D^R and LR check as in
    run(); surviving pixels take d + offset; then the float median."""
    r = run(left, right, Params(**{**params.__dict__, "median3x3": False}))
    fine = refine_subpixel(r["agg"], r["disp_left"])
    valid = r["disp"] != INVALID
    if params.median3x3:
        d = median3x3_float(fine, valid)
    else:
        d = np.where(valid, fine, INVALID_F)
    return {**r, "disp_fine": d}
