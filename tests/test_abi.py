"""C ABI checks that need no GPU: libsgm.so loads, exports every function
declared in include/sgm.h, and rejects bad arguments before any launch
(every call below fails validation, so no kernel is ever enqueued)."""
import ctypes
import os
import re

import pytest

from paper_2106_07927_amd import sgm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgm.h")

OK, ARG, UNSUP, ALIGN, HIP, WS = 0, -1, -2, -3, -4, -5


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sgm.LIB_PATH):
        pytest.skip("libsgm.so not built (run python -m paper_2106_07927_amd.build)")
    return sgm.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"sgm_census", "sgm_cost", "sgm_aggregate", "sgm_wta_lrc"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    assert set(sgm.EXPORTS) == set(names)


def test_status_strings_and_version(lib):
    assert lib.sgm_abi_version() == 4
    for code in (OK, ARG, UNSUP, ALIGN, HIP, WS, sgm.SGM_ERR_TOO_LARGE):
        assert lib.sgm_status_string(code).decode().startswith("SGM_")
    assert lib.sgm_status_string(99) == b"unknown sgm status"


FAKE = 0x10000        # aligned, never dereferenced: validation fails first
NULL = 0


def P(v):
    return ctypes.c_void_p(v)


def test_census_validation(lib):
    f = lib.sgm_census
    assert f(P(NULL), 64, 64, 64, 9, 7, P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), 64, 64, 64, 9, 7, P(NULL), P(NULL)) == ARG
    assert f(P(FAKE), 0, 64, 64, 9, 7, P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), 64, -1, 64, 9, 7, P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), 64, 64, 63, 9, 7, P(FAKE), P(NULL)) == ARG      # pitch < width
    assert f(P(FAKE), 40000, 8, 40000, 9, 7, P(FAKE), P(NULL)) == ARG  # beyond the size limit
    assert f(P(FAKE), 64, 64, 64, 7, 9, P(FAKE), P(NULL)) == UNSUP
    assert f(P(FAKE), 64, 64, 64, 3, 3, P(FAKE), P(NULL)) == UNSUP
    assert f(P(FAKE), 64, 64, 64, 5, 5, P(FAKE + 4), P(NULL)) == ALIGN


def test_census_pair_validation(lib):
    f = lib.sgm_census_pair
    A, B = FAKE, FAKE + 0x1000
    assert f(P(NULL), P(FAKE), 64, 64, 64, 9, 7, P(A), P(B), P(NULL)) == ARG
    assert f(P(FAKE), P(NULL), 64, 64, 64, 9, 7, P(A), P(B), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 64, 64, 64, 9, 7, P(NULL), P(B), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 64, 64, 64, 9, 7, P(A), P(A), P(NULL)) == ARG    # one buffer twice
    assert f(P(FAKE), P(FAKE), 64, 64, 63, 9, 7, P(A), P(B), P(NULL)) == ARG    # pitch < width
    assert f(P(FAKE), P(FAKE), 0, 64, 64, 9, 7, P(A), P(B), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 64, 64, 64, 7, 9, P(A), P(B), P(NULL)) == UNSUP
    assert f(P(FAKE), P(FAKE), 64, 64, 64, 5, 5, P(A), P(B + 4), P(NULL)) == ALIGN


def test_cost_validation(lib):
    f = lib.sgm_cost
    assert f(P(NULL), P(FAKE), 8, 8, 16, P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 8, 8, 0, P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 8, 8, 257, P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 8, 8, 16, P(FAKE + 8), P(NULL)) == ALIGN
    assert f(P(FAKE + 4), P(FAKE), 8, 8, 16, P(FAKE), P(NULL)) == ALIGN


def test_cost_ncc_validation(lib):
    f = lib.sgm_cost_ncc
    assert f(P(NULL), P(FAKE), 8, 8, 8, 5, 16, P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 8, 8, 7, 5, 16, P(FAKE), P(NULL)) == ARG      # pitch < width
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 5, 0, P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 7, 16, P(FAKE), P(NULL)) == UNSUP
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 9, 16, P(FAKE + 8), P(NULL)) == ALIGN


def test_aggregate_validation(lib):
    f = lib.sgm_aggregate
    big = 1 << 40
    W = lambda v: ctypes.c_size_t(v)
    assert f(P(NULL), 8, 8, 16, 8, 10, 120, P(FAKE), P(FAKE), W(big), P(NULL)) == ARG
    assert f(P(FAKE), 8, 8, 16, 6, 10, 120, P(FAKE), P(FAKE), W(big), P(NULL)) == ARG   # npaths
    assert f(P(FAKE), 8, 8, 16, 8, 121, 120, P(FAKE), P(FAKE), W(big), P(NULL)) == ARG  # p1 > p2
    assert f(P(FAKE), 8, 8, 16, 8, -1, 120, P(FAKE), P(FAKE), W(big), P(NULL)) == ARG
    assert f(P(FAKE), 8, 8, 16, 8, 10, 7937, P(FAKE), P(FAKE), W(big), P(NULL)) == ARG  # 8 * (255 + p2) > 65535
    assert f(P(FAKE), 8, 8, 16, 4, 10, 16129, P(FAKE), P(FAKE), W(big), P(NULL)) == ARG
    assert f(P(FAKE), 8, 8, 300, 8, 10, 120, P(FAKE), P(FAKE), W(big), P(NULL)) == ARG
    assert f(P(FAKE), 32768, 32768, 4, 8, 10, 120, P(FAKE), P(FAKE), W(big), P(NULL)) == ARG  # volume
    assert f(P(FAKE), 8, 8, 16, 8, 10, 120, P(FAKE), P(NULL), W(big), P(NULL)) == WS
    need = lib.sgm_aggregate_work_bytes(8, 8, 16, 8, 120)
    assert need == 4 * 1024                      # 4 pair slices of 1024 uint8 (P2 <= 127)
    assert lib.sgm_aggregate_work_bytes(8, 8, 16, 8, 127) == 4 * 1024
    assert lib.sgm_aggregate_work_bytes(8, 8, 16, 8, 128) == 4 * 1024 * 2   # uint16 beyond
    assert lib.sgm_aggregate_work_bytes(8, 8, 16, 4, 256) == 2 * 1024 * 2
    assert lib.sgm_aggregate_work_bytes(8, 8, 16, 8, 7937) == 0
    assert f(P(FAKE), 8, 8, 16, 8, 10, 120, P(FAKE), P(FAKE), W(need - 1), P(NULL)) == WS
    assert f(P(FAKE + 8), 8, 8, 16, 8, 10, 120, P(FAKE), P(FAKE), W(need), P(NULL)) == ALIGN
    assert f(P(FAKE), 8, 8, 16, 8, 10, 120, P(FAKE + 2), P(FAKE), W(need), P(NULL)) == ALIGN
    assert f(P(FAKE), 8, 8, 16, 8, 10, 120, P(FAKE), P(FAKE + 4), W(need), P(NULL)) == ALIGN


def test_wta_lrc_validation(lib):
    f = lib.sgm_wta_lrc
    assert f(P(NULL), 8, 8, 16, 1, 1, P(FAKE), P(NULL), P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), 8, 8, 16, 1, 1, P(NULL), P(NULL), P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), 8, 8, 16, 1, 2, P(FAKE), P(NULL), P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), 8, 8, 0, 1, 1, P(FAKE), P(NULL), P(FAKE), P(NULL)) == ARG
    assert f(P(FAKE), 8, 8, 16, 1, 1, P(FAKE), P(NULL), P(NULL), P(NULL)) == WS
    assert f(P(FAKE + 8), 8, 8, 16, 1, 1, P(FAKE), P(NULL), P(FAKE), P(NULL)) == ALIGN
    assert f(P(FAKE), 8, 8, 16, 1, 1, P(FAKE + 2), P(NULL), P(FAKE), P(NULL)) == ALIGN
    assert f(P(FAKE), 8, 8, 16, 1, 1, P(FAKE), P(FAKE + 2), P(FAKE), P(NULL)) == ALIGN
    assert lib.sgm_wta_lrc_work_elems(10, 20) == 3 * 200
    assert lib.sgm_wta_lrc_work_elems(0, 20) == 0


def test_aggregate_select_noalloc_validation(lib):
    """Every rejection happens before the first HIP call (none here needs a
    GPU); a frame whose workspace exceeds the fixed scratch is refused."""
    f = lib.sgm_aggregate_select_noalloc
    args = lambda **k: [P(k.get("cost", FAKE)), k.get("w", 8), k.get("h", 8), k.get("nd", 16),
                        k.get("npaths", 8), k.get("p1", 10), k.get("p2", 120), k.get("t", 1),
                        k.get("med", 1), P(k.get("out", FAKE)), P(k.get("outr", NULL)), P(NULL)]
    TOO_LARGE = sgm.SGM_ERR_TOO_LARGE
    assert f(*args(cost=NULL)) == ARG
    assert f(*args(out=NULL)) == ARG
    assert f(*args(npaths=6)) == ARG
    assert f(*args(p1=121)) == ARG
    assert f(*args(nd=0)) == ARG
    assert f(*args(med=2)) == ARG
    assert f(*args(cost=FAKE + 8)) == ALIGN
    assert f(*args(out=FAKE + 2)) == ALIGN
    assert f(*args(outr=FAKE + 2)) == ALIGN
    cap = sgm.NOALLOC_SCRATCH_BYTES
    # 1242x375, D=128, 8 paths fits; 1920x1080, D=256 does not
    assert lib.sgm_aggregate_select_work_bytes(1242, 375, 128, 8, 120) <= cap
    assert lib.sgm_aggregate_select_work_bytes(1920, 1080, 256, 8, 120) > cap
    assert f(*args(w=1920, h=1080, nd=256)) == TOO_LARGE
    assert f(*args(w=1920, h=1080, nd=256, cost=FAKE + 8)) == TOO_LARGE   # size first
    assert lib.sgm_status_string(TOO_LARGE).decode().startswith("SGM_ERR_TOO_LARGE")


def test_aggregate_select_validation(lib):
    f = lib.sgm_aggregate_select
    W = lambda v: ctypes.c_size_t(v)
    big = 1 << 40
    args = lambda **k: [P(k.get("cost", FAKE)), k.get("w", 8), k.get("h", 8), k.get("nd", 16),
                        k.get("npaths", 8), k.get("p1", 10), k.get("p2", 120), k.get("t", 1),
                        k.get("med", 1), P(k.get("out", FAKE)), P(k.get("outr", NULL)),
                        P(k.get("work", FAKE)), W(k.get("wb", big)), P(NULL)]
    assert f(*args(cost=NULL)) == ARG
    assert f(*args(out=NULL)) == ARG
    assert f(*args(npaths=6)) == ARG
    assert f(*args(p1=121)) == ARG
    assert f(*args(p2=7937)) == ARG
    assert f(*args(nd=0)) == ARG
    assert f(*args(med=2)) == ARG
    assert f(*args(work=NULL)) == WS
    # fused form (D % 16 == 0): pair slices, D^R keys, D^L; no S_bar
    n = 8 * 8
    need = lib.sgm_aggregate_select_work_bytes(8, 8, 16, 8, 120)
    assert need == 4 * 1024 + 256 + 256
    assert f(*args(wb=need - 1)) == WS
    assert f(*args(work=FAKE + 16, wb=need)) == ALIGN           # 256-byte alignment
    assert f(*args(cost=FAKE + 8, wb=need)) == ALIGN
    assert f(*args(out=FAKE + 2, wb=need)) == ALIGN
    assert f(*args(outr=FAKE + 2, wb=need)) == ALIGN
    # the unfused fallback (D % 16 != 0) also holds S_bar in the workspace
    assert lib.sgm_aggregate_select_work_bytes(8, 8, 15, 8, 120) == \
        4 * 1024 + (2 * n * 15 + 255) // 256 * 256 + 256 + 256
    # P2 > 127: uint16 pair slices, still fused
    assert lib.sgm_aggregate_select_work_bytes(8, 8, 16, 8, 256) == 4 * 2048 + 256 + 256
    assert lib.sgm_aggregate_select_work_bytes(8, 8, 16, 8, 7937) == 0


def test_exact_lr_validation(lib):
    f = lib.sgm_disparity_exact_lr
    W = lambda v: ctypes.c_size_t(v)
    prm = sgm.SgmParams(9, 7, 8, 10, 120, 1, 1)
    R = ctypes.byref
    big = 1 << 40
    assert f(P(NULL), P(FAKE), 8, 8, 8, 16, R(prm), P(FAKE), P(NULL), P(FAKE), W(big), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 8, 8, 7, 16, R(prm), P(FAKE), P(NULL), P(FAKE), W(big), P(NULL)) == ARG
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 16, None, P(FAKE), P(NULL), P(FAKE), W(big), P(NULL)) == ARG
    bad = sgm.SgmParams(3, 3, 8, 10, 120, 1, 1)
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 16, R(bad), P(FAKE), P(NULL), P(FAKE), W(big), P(NULL)) == UNSUP
    bad = sgm.SgmParams(9, 7, 8, 121, 120, 1, 1)
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 16, R(bad), P(FAKE), P(NULL), P(FAKE), W(big), P(NULL)) == ARG
    assert lib.sgm_disparity_exact_lr_work_bytes(8, 8, 16, R(bad)) == 0
    need = lib.sgm_disparity_exact_lr_work_bytes(8, 8, 16, R(prm))
    n = 64
    # flipped pair, census x2, cost, the aggregation workspace, D^L and the flipped map
    assert need == 2 * 256 + 2 * 512 + 1024 + lib.sgm_aggregate_select_work_bytes(8, 8, 16, 8, 120) \
        + 2 * 256
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 16, R(prm), P(FAKE), P(NULL), P(NULL), W(need), P(NULL)) == WS
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 16, R(prm), P(FAKE), P(NULL), P(FAKE), W(need - 1), P(NULL)) == WS
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 16, R(prm), P(FAKE), P(NULL), P(FAKE + 64), W(need), P(NULL)) == ALIGN
    assert f(P(FAKE), P(FAKE), 8, 8, 8, 16, R(prm), P(FAKE + 2), P(NULL), P(FAKE), W(need), P(NULL)) == ALIGN
    assert n == 64


def test_python_binding_rejects_host_tensors(lib):
    import torch
    img = torch.zeros(4, 4, dtype=torch.uint8)
    with pytest.raises(ValueError):
        sgm.sgm_census(img, 5, 5, out=torch.zeros(4, 4, dtype=torch.uint64))


def test_batch_validation(lib):
    prm = sgm.SgmParams(9, 7, 8, 10, 120, 1, 1)
    pairs = (sgm.SgmPair * 2)()
    pairs[0] = sgm.SgmPair(FAKE, FAKE, 64, 48, 64, 64, FAKE, None)
    pairs[1] = sgm.SgmPair(FAKE, FAKE, 32, 16, 40, 16, FAKE, FAKE)
    need = lib.sgm_batch_workspace_bytes(pairs, 2, ctypes.byref(prm), None)
    # two frames of intermediates (census x2, cost, one uint8 slice per pair
    # of paths, keys, D^L; S_bar only for frames that cannot take the fused
    # selection) plus tables
    n0, n1 = 64 * 48, 32 * 16
    lower = sum(8 * 2 * n + n * nd + 4 * n * nd + 4 * n + 2 * n
                for n, nd in ((n0, 64), (n1, 16)))
    assert need >= lower
    # a tuning table that splits the path launches needs more table space
    split = lib.sgm_batch_workspace_bytes(pairs, 2, ctypes.byref(prm), b'{"64x48x64": 1}')
    assert split >= need
    assert lib.sgm_batch_workspace_bytes(pairs, 0, ctypes.byref(prm), None) == 0
    bad = sgm.SgmParams(7, 9, 8, 10, 120, 1, 1)                      # window
    assert lib.sgm_batch_workspace_bytes(pairs, 2, ctypes.byref(bad), None) == 0
    bad = sgm.SgmParams(9, 7, 8, 121, 120, 1, 1)                     # p1 > p2
    assert lib.sgm_batch_workspace_bytes(pairs, 2, ctypes.byref(bad), None) == 0
    handle = ctypes.c_void_p()
    pairs[1].pitch_bytes = 31                                        # pitch < width
    assert lib.sgm_batch_plan_create(pairs, 2, ctypes.byref(prm), P(FAKE), need, None,
                                     ctypes.byref(handle)) == ARG
    pairs[1].pitch_bytes = 40
    pairs[0].ndisp = 0
    assert lib.sgm_batch_plan_create(pairs, 2, ctypes.byref(prm), P(FAKE), need, None,
                                     ctypes.byref(handle)) == ARG
    pairs[0].ndisp = 64
    pairs[0].disp_out = FAKE + 2                                     # misaligned output
    assert lib.sgm_batch_plan_create(pairs, 2, ctypes.byref(prm), P(FAKE), need, None,
                                     ctypes.byref(handle)) == ARG
    pairs[0].disp_out = FAKE
    assert lib.sgm_batch_plan_create(pairs, 2, ctypes.byref(prm), P(NULL), need, None,
                                     ctypes.byref(handle)) == WS
    assert lib.sgm_batch_plan_create(pairs, 2, ctypes.byref(prm), P(FAKE), need - 1, None,
                                     ctypes.byref(handle)) == WS
    assert lib.sgm_batch_plan_create(pairs, 2, ctypes.byref(prm), P(FAKE + 16), need, None,
                                     ctypes.byref(handle)) == ALIGN
    assert not handle.value
    assert lib.sgm_batch_run(None, None) == ARG
    assert lib.sgm_batch_frames(None) == 0
    lib.sgm_batch_plan_destroy(None)
