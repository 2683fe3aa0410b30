"""Python binding of libsgm.so (include/sgm.h): argument marshalling only.

Every function takes and returns torch CUDA tensors (device memory on the
current ROCm device) and enqueues on the current torch stream unless a stream
is given.  All computation happens in the HIP kernels of libsgm.so; there is
no fallback: if the library is not built, or a tensor is not on the GPU, the
call raises.

Names follow the C ABI: sgm_census, sgm_cost, sgm_aggregate, sgm_wta_lrc, and
the streamlined sgm_aggregate_select (aggregation fused with the selection).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsgm.so")
INVALID = 0xFFFF

SGM_OK = 0
SGM_ERR_ARG = -1
SGM_ERR_UNSUPPORTED = -2
SGM_ERR_ALIGN = -3
SGM_ERR_HIP = -4
SGM_ERR_WORKSPACE = -5
SGM_ERR_TOO_LARGE = -6
NOALLOC_SCRATCH_BYTES = 256 << 20      # SGM_NOALLOC_SCRATCH_BYTES

EXPORTS = ("sgm_census", "sgm_census_pair", "sgm_cost", "sgm_cost_ncc", "sgm_aggregate",
           "sgm_aggregate_work_bytes", "sgm_wta_lrc", "sgm_wta_lrc_work_elems", "sgm_aggregate_select", "sgm_aggregate_select_work_bytes",
           "sgm_aggregate_select_noalloc",
           "sgm_aggregate_select_subpixel", "sgm_aggregate_select_subpixel_work_bytes",
           "sgm_disparity_exact_lr", "sgm_disparity_exact_lr_work_bytes",
           "sgm_batch_workspace_bytes", "sgm_batch_plan_create",
           "sgm_batch_run", "sgm_batch_frames", "sgm_batch_plan_destroy", "sgm_aggregate_variants",
           "sgm_status_string",
           "sgm_last_hip_error", "sgm_abi_version")


class SgmParams(ctypes.Structure):
    """sgm_params of include/sgm.h."""
    _fields_ = [("win_w", ctypes.c_int32), ("win_h", ctypes.c_int32), ("npaths", ctypes.c_int32),
                ("p1", ctypes.c_int32), ("p2", ctypes.c_int32), ("lr_tolerance", ctypes.c_int32),
                ("median3x3", ctypes.c_int32)]


class SgmPair(ctypes.Structure):
    """sgm_pair of include/sgm.h."""
    _fields_ = [("left", ctypes.c_void_p), ("right", ctypes.c_void_p), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("pitch_bytes", ctypes.c_int32), ("ndisp", ctypes.c_int32),
                ("disp_out", ctypes.c_void_p), ("disp_right_out", ctypes.c_void_p)]


class SGMError(RuntimeError):
    """A libsgm call returned a non-zero status."""

    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


_lib = None


def load_library(path: Optional[str] = None):
    """Load libsgm.so (or the library at `path`, kept for later calls) and
    declare its signatures (no GPU call is made).  The default is LIB_PATH
    as it stands at the first call."""
    global _lib
    if _lib is not None and (path is None or path == _lib._name):
        return _lib
    if path is None:
        path = LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2106_07927_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32 = ctypes.c_void_p, ctypes.c_int32
    lib.sgm_census.argtypes = [P, I32, I32, I32, I32, I32, P, P]
    lib.sgm_census_pair.argtypes = [P, P, I32, I32, I32, I32, I32, P, P, P]
    lib.sgm_cost.argtypes = [P, P, I32, I32, I32, P, P]
    lib.sgm_cost_ncc.argtypes = [P, P, I32, I32, I32, I32, I32, P, P]
    lib.sgm_cost_ncc.restype = I32
    lib.sgm_aggregate.argtypes = [P, I32, I32, I32, I32, I32, I32, P, P, ctypes.c_size_t, P]
    lib.sgm_aggregate_work_bytes.argtypes = [I32, I32, I32, I32, I32]
    lib.sgm_aggregate_work_bytes.restype = ctypes.c_size_t
    lib.sgm_wta_lrc.argtypes = [P, I32, I32, I32, I32, I32, P, P, P, P]
    lib.sgm_wta_lrc_work_elems.argtypes = [I32, I32]
    lib.sgm_wta_lrc_work_elems.restype = ctypes.c_size_t
    lib.sgm_aggregate_select.argtypes = [P, I32, I32, I32, I32, I32, I32, I32, I32, P, P, P,
                                         ctypes.c_size_t, P]
    lib.sgm_aggregate_select_work_bytes.argtypes = [I32, I32, I32, I32, I32]
    lib.sgm_aggregate_select_work_bytes.restype = ctypes.c_size_t
    lib.sgm_aggregate_select_noalloc.argtypes = [P, I32, I32, I32, I32, I32, I32, I32, I32, P, P, P]
    lib.sgm_aggregate_select_noalloc.restype = I32
    lib.sgm_aggregate_select_subpixel.argtypes = lib.sgm_aggregate_select.argtypes
    lib.sgm_aggregate_select_subpixel.restype = I32
    lib.sgm_aggregate_select_subpixel_work_bytes.argtypes = [I32, I32, I32, I32, I32]
    lib.sgm_aggregate_select_subpixel_work_bytes.restype = ctypes.c_size_t
    lib.sgm_disparity_exact_lr.argtypes = [P, P, I32, I32, I32, I32, ctypes.POINTER(SgmParams), P, P,
                                           P, ctypes.c_size_t, P]
    lib.sgm_disparity_exact_lr.restype = I32
    lib.sgm_disparity_exact_lr_work_bytes.argtypes = [I32, I32, I32, ctypes.POINTER(SgmParams)]
    lib.sgm_disparity_exact_lr_work_bytes.restype = ctypes.c_size_t
    PP = ctypes.POINTER(SgmPair)
    lib.sgm_batch_workspace_bytes.argtypes = [PP, I32, ctypes.POINTER(SgmParams), ctypes.c_char_p]
    lib.sgm_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.sgm_batch_plan_create.argtypes = [PP, I32, ctypes.POINTER(SgmParams), P, ctypes.c_size_t,
                                          ctypes.c_char_p, ctypes.POINTER(P)]
    lib.sgm_batch_plan_create.restype = I32
    lib.sgm_batch_run.argtypes = [P, P]
    lib.sgm_batch_run.restype = I32
    lib.sgm_batch_frames.argtypes = [P]
    lib.sgm_batch_frames.restype = I32
    lib.sgm_batch_plan_destroy.argtypes = [P]
    lib.sgm_batch_plan_destroy.restype = None
    lib.sgm_aggregate_variants.argtypes = [I32]
    lib.sgm_aggregate_variants.restype = I32
    lib.sgm_status_string.argtypes = [I32]
    lib.sgm_status_string.restype = ctypes.c_char_p
    lib.sgm_last_hip_error.argtypes = []
    lib.sgm_abi_version.argtypes = []
    for name in ("sgm_census", "sgm_census_pair", "sgm_cost", "sgm_aggregate", "sgm_wta_lrc",
                 "sgm_aggregate_select", "sgm_last_hip_error", "sgm_abi_version"):
        getattr(lib, name).restype = I32
    _lib = lib
    return lib


def _check(status: int):
    if status != SGM_OK:
        lib = load_library()
        msg = lib.sgm_status_string(status).decode()
        if status == SGM_ERR_HIP:
            msg += f" (hipError {lib.sgm_last_hip_error()})"
        raise SGMError(status, msg)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda:
        raise ValueError("libsgm takes device tensors only")
    if not t.is_contiguous():
        raise ValueError("libsgm takes contiguous tensors only")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _expect(t: torch.Tensor, dtype, shape, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected {dtype} {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


def _empty(shape, dtype, device, pad_bytes=16):
    """Contiguous device tensor whose allocation extends to a 16-byte multiple."""
    n = 1
    for s in shape:
        n *= s
    item = torch.empty((), dtype=dtype).element_size()
    total = (n * item + pad_bytes - 1) // pad_bytes * pad_bytes // item
    return torch.empty(max(total, 1), dtype=dtype, device=device)[:n].view(shape)


def sgm_census(img: torch.Tensor, win_w: int, win_h: int, out: Optional[torch.Tensor] = None,
               width: Optional[int] = None, stream=None) -> torch.Tensor:
    """Census transform.  img: uint8 [H][pitch] (width <= pitch, default all
    columns); returns uint64 [H][W] descriptors."""
    if img.dtype != torch.uint8 or img.dim() != 2:
        raise ValueError("img must be a 2-D uint8 tensor")
    h, pitch = img.shape
    w = pitch if width is None else width
    if out is None:
        out = _empty((h, w), torch.uint64, img.device)
    _expect(out, torch.uint64, (h, w), "out")
    _check(load_library().sgm_census(_ptr(img), w, h, pitch, win_w, win_h, _ptr(out), _stream(stream)))
    return out


def sgm_census_pair(left: torch.Tensor, right: torch.Tensor, win_w: int, win_h: int,
                    out_left: Optional[torch.Tensor] = None,
                    out_right: Optional[torch.Tensor] = None, width: Optional[int] = None,
                    stream=None):
    """Census of both images in one launch.  left, right: uint8 [H][pitch] of
    one shape; returns (census_left, census_right), uint64 [H][W] each."""
    for name, img in (("left", left), ("right", right)):
        if img.dtype != torch.uint8 or img.dim() != 2:
            raise ValueError(f"{name} must be a 2-D uint8 tensor")
    if left.shape != right.shape or left.stride() != right.stride():
        raise ValueError("left and right must have one shape and pitch")
    h, pitch = left.shape
    w = pitch if width is None else width
    if out_left is None:
        out_left = _empty((h, w), torch.uint64, left.device)
    if out_right is None:
        out_right = _empty((h, w), torch.uint64, left.device)
    _expect(out_left, torch.uint64, (h, w), "out_left")
    _expect(out_right, torch.uint64, (h, w), "out_right")
    _check(load_library().sgm_census_pair(_ptr(left), _ptr(right), w, h, pitch, win_w, win_h,
                                          _ptr(out_left), _ptr(out_right), _stream(stream)))
    return out_left, out_right


def sgm_cost(census_left: torch.Tensor, census_right: torch.Tensor, ndisp: int,
             out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Hamming cost volume; returns uint8 [H][W][ndisp]."""
    h, w = census_left.shape
    _expect(census_left, torch.uint64, (h, w), "census_left")
    _expect(census_right, torch.uint64, (h, w), "census_right")
    if out is None:
        out = _empty((h, w, ndisp), torch.uint8, census_left.device)
    _expect(out, torch.uint8, (h, w, ndisp), "out")
    _check(load_library().sgm_cost(_ptr(census_left), _ptr(census_right), w, h, ndisp,
                                   _ptr(out), _stream(stream)))
    return out


def sgm_cost_ncc(left: torch.Tensor, right: torch.Tensor, win: int, ndisp: int,
                 out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Inverted, truncated NCC cost volume (win 5 or 9); uint8 [H][W][ndisp]."""
    if left.dtype != torch.uint8 or left.dim() != 2 or right.shape != left.shape or \
            right.dtype != torch.uint8:
        raise ValueError("left and right must be uint8 [H][W] tensors of one shape")
    h, w = left.shape
    if out is None:
        out = _empty((h, w, ndisp), torch.uint8, left.device)
    _expect(out, torch.uint8, (h, w, ndisp), "out")
    _check(load_library().sgm_cost_ncc(_ptr(left), _ptr(right), w, h, w, win, ndisp, _ptr(out),
                                       _stream(stream)))
    return out


def aggregate_work_bytes(width: int, height: int, ndisp: int, npaths: int, p2: int) -> int:
    return int(load_library().sgm_aggregate_work_bytes(width, height, ndisp, npaths, p2))


def sgm_aggregate(cost: torch.Tensor, npaths: int, p1: int, p2: int,
                  out: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """SGM path aggregation; returns uint16 [H][W][D].  `work` is a uint8
    device scratch tensor of at least aggregate_work_bytes(...) bytes."""
    if cost.dtype != torch.uint8 or cost.dim() != 3:
        raise ValueError("cost must be a 3-D uint8 tensor")
    h, w, nd = cost.shape
    if out is None:
        out = _empty((h, w, nd), torch.uint16, cost.device)
    _expect(out, torch.uint16, (h, w, nd), "out")
    if work is None:
        work = _empty((max(1, aggregate_work_bytes(w, h, nd, npaths, p2)),), torch.uint8, cost.device)
    if work.dtype != torch.uint8:
        raise ValueError("work must be a uint8 tensor")
    _check(load_library().sgm_aggregate(_ptr(cost), w, h, nd, npaths, p1, p2, _ptr(out),
                                        _ptr(work), work.numel(), _stream(stream)))
    return out


def wta_lrc_work_elems(width: int, height: int) -> int:
    return int(load_library().sgm_wta_lrc_work_elems(width, height))


def sgm_wta_lrc(agg: torch.Tensor, lr_tolerance: int, median3x3: bool,
                out: Optional[torch.Tensor] = None, out_right: Optional[torch.Tensor] = None,
                work: Optional[torch.Tensor] = None, want_right: bool = False, stream=None):
    """WTA, approximate D^R, LR check, 3x3 median.  Returns (disp, disp_right
    or None), both uint16 [H][W], 0xFFFF = invalid."""
    if agg.dtype != torch.uint16 or agg.dim() != 3:
        raise ValueError("agg must be a 3-D uint16 tensor")
    h, w, nd = agg.shape
    dev = agg.device
    if out is None:
        out = _empty((h, w), torch.uint16, dev)
    _expect(out, torch.uint16, (h, w), "out")
    if want_right and out_right is None:
        out_right = _empty((h, w), torch.uint16, dev)
    if out_right is not None:
        _expect(out_right, torch.uint16, (h, w), "out_right")
    if work is None:
        work = _empty((wta_lrc_work_elems(w, h),), torch.uint16, dev)
    _check(load_library().sgm_wta_lrc(_ptr(agg), w, h, nd, lr_tolerance, int(bool(median3x3)),
                                      _ptr(out), _ptr(out_right), _ptr(work), _stream(stream)))
    return out, out_right


def aggregate_select_work_bytes(width: int, height: int, ndisp: int, npaths: int, p2: int) -> int:
    return int(load_library().sgm_aggregate_select_work_bytes(width, height, ndisp, npaths, p2))


def _aligned_bytes(nbytes: int, device, align: int = 256) -> torch.Tensor:
    """uint8 device tensor of nbytes whose data pointer is align-byte aligned."""
    raw = torch.empty(nbytes + align, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % align
    return raw[off: off + nbytes]


def sgm_aggregate_select(cost: torch.Tensor, npaths: int, p1: int, p2: int, lr_tolerance: int,
                         median3x3: bool, out: Optional[torch.Tensor] = None,
                         out_right: Optional[torch.Tensor] = None,
                         work: Optional[torch.Tensor] = None, want_right: bool = False,
                         stream=None):
    """Aggregation fused with WTA, approximate D^R, LR check and median; the
    path sum never reaches device memory.  Returns (disp, disp_right or None),
    bit-identical to sgm_aggregate followed by sgm_wta_lrc.  `work`: uint8,
    256-byte aligned, at least aggregate_select_work_bytes(...) bytes."""
    if cost.dtype != torch.uint8 or cost.dim() != 3:
        raise ValueError("cost must be a 3-D uint8 tensor")
    h, w, nd = cost.shape
    dev = cost.device
    if out is None:
        out = _empty((h, w), torch.uint16, dev)
    _expect(out, torch.uint16, (h, w), "out")
    if want_right and out_right is None:
        out_right = _empty((h, w), torch.uint16, dev)
    if out_right is not None:
        _expect(out_right, torch.uint16, (h, w), "out_right")
    if work is None:
        work = _aligned_bytes(max(1, aggregate_select_work_bytes(w, h, nd, npaths, p2)), dev)
    if work.dtype != torch.uint8:
        raise ValueError("work must be a uint8 tensor")
    _check(load_library().sgm_aggregate_select(_ptr(cost), w, h, nd, npaths, p1, p2, lr_tolerance,
                                               int(bool(median3x3)), _ptr(out), _ptr(out_right),
                                               _ptr(work), work.numel(), _stream(stream)))
    return out, out_right


def sgm_aggregate_select_noalloc(cost: torch.Tensor, npaths: int, p1: int, p2: int,
                                 lr_tolerance: int, median3x3: bool,
                                 out: Optional[torch.Tensor] = None,
                                 out_right: Optional[torch.Tensor] = None,
                                 want_right: bool = False, stream=None):
    """sgm_aggregate_select with the library's fixed per-GPU scratch as its
    workspace (no allocation in the call; frames needing more than
    NOALLOC_SCRATCH_BYTES are rejected).  Calls that overlap on one GPU
    race on that scratch.  Returns (disp, disp_right or None)."""
    if cost.dtype != torch.uint8 or cost.dim() != 3:
        raise ValueError("cost must be a 3-D uint8 tensor")
    h, w, nd = cost.shape
    if out is None:
        out = _empty((h, w), torch.uint16, cost.device)
    _expect(out, torch.uint16, (h, w), "out")
    if want_right and out_right is None:
        out_right = _empty((h, w), torch.uint16, cost.device)
    if out_right is not None:
        _expect(out_right, torch.uint16, (h, w), "out_right")
    _check(load_library().sgm_aggregate_select_noalloc(_ptr(cost), w, h, nd, npaths, p1, p2,
                                                       lr_tolerance, int(bool(median3x3)),
                                                       _ptr(out), _ptr(out_right),
                                                       _stream(stream)))
    return out, out_right


def aggregate_select_subpixel_work_bytes(width: int, height: int, ndisp: int, npaths: int,
                                         p2: int) -> int:
    return int(load_library().sgm_aggregate_select_subpixel_work_bytes(width, height, ndisp,
                                                                       npaths, p2))


def sgm_aggregate_select_subpixel(cost: torch.Tensor, npaths: int, p1: int, p2: int,
                                  lr_tolerance: int, median3x3: bool,
                                  out: Optional[torch.Tensor] = None,
                                  out_right: Optional[torch.Tensor] = None,
                                  work: Optional[torch.Tensor] = None, want_right: bool = False,
                                  stream=None):
    """sgm_aggregate_select with subpixel refinement.  Returns (disp float32
    [H][W] with -1.0 for invalid pixels, D^R uint16 or None)."""
    if cost.dtype != torch.uint8 or cost.dim() != 3:
        raise ValueError("cost must be a 3-D uint8 tensor")
    h, w, nd = cost.shape
    dev = cost.device
    if out is None:
        out = _empty((h, w), torch.float32, dev)
    _expect(out, torch.float32, (h, w), "out")
    if want_right and out_right is None:
        out_right = _empty((h, w), torch.uint16, dev)
    if out_right is not None:
        _expect(out_right, torch.uint16, (h, w), "out_right")
    if work is None:
        work = _aligned_bytes(max(1, aggregate_select_subpixel_work_bytes(w, h, nd, npaths, p2)), dev)
    _check(load_library().sgm_aggregate_select_subpixel(
        _ptr(cost), w, h, nd, npaths, p1, p2, lr_tolerance, int(bool(median3x3)), _ptr(out),
        _ptr(out_right), _ptr(work), work.numel(), _stream(stream)))
    return out, out_right


@dataclass(frozen=True)
class Params:
    """Pipeline parameters (lr_tolerance < 0 skips the LR check)."""
    win_w: int = 9
    win_h: int = 7
    ndisp: int = 128
    npaths: int = 8
    p1: int = 10
    p2: int = 120
    lr_tolerance: int = 1
    median3x3: bool = True


class StereoSGM:
    """Device buffers for one frame shape, reused across frames.  run()
    enqueues sgm_census_pair, sgm_cost and the streamlined sgm_aggregate_select
    on one stream; with fused=False it enqueues the four calls sgm_census (x2),
    sgm_cost, sgm_aggregate, sgm_wta_lrc instead (same bits, S_bar kept in
    self.agg)."""

    def __init__(self, width: int, height: int, params: Params, device="cuda", fused: bool = True,
                 alloc=None):
        """alloc(nbytes) -> uint8 device tensor of nbytes, 256-byte aligned:
        where every buffer comes from (default: a fresh allocation each)."""
        self.width, self.height, self.params, self.fused = width, height, params, fused
        dev = torch.device(device)
        nd = params.ndisp
        if alloc is None:
            def alloc(nbytes):
                return _aligned_bytes(nbytes, dev)

        def buf(shape, dtype):
            n = 1
            for s in shape:
                n *= s
            item = torch.empty((), dtype=dtype).element_size()
            return alloc(max(1, n) * item)[: n * item].view(dtype).view(shape)

        self.census_left = buf((height, width), torch.uint64)
        self.census_right = buf((height, width), torch.uint64)
        self.cost = buf((height, width, nd), torch.uint8)
        self.disp = buf((height, width), torch.uint16)
        self.disp_right = buf((height, width), torch.uint16)
        if fused:
            self.select_work = alloc(max(1, aggregate_select_work_bytes(width, height, nd,
                                                                        params.npaths, params.p2)))
        else:
            self.agg = buf((height, width, nd), torch.uint16)
            self.agg_work = alloc(max(1, aggregate_work_bytes(width, height, nd, params.npaths,
                                                              params.p2)))
            self.work = buf((wta_lrc_work_elems(width, height),), torch.uint16)

    @staticmethod
    def buffer_bytes(width: int, height: int, params: Params, fused: bool = True) -> list:
        """Sizes of the device buffers __init__ asks `alloc` for, in order."""
        n, nd = width * height, params.ndisp
        sizes = [8 * n, 8 * n, n * nd, 2 * n, 2 * n]
        if fused:
            sizes.append(aggregate_select_work_bytes(width, height, nd, params.npaths, params.p2))
        else:
            sizes += [2 * n * nd, aggregate_work_bytes(width, height, nd, params.npaths, params.p2),
                      2 * wta_lrc_work_elems(width, height)]
        return [max(1, b) for b in sizes]

    def run(self, left: torch.Tensor, right: torch.Tensor, stream=None) -> torch.Tensor:
        p = self.params
        if self.fused and left.shape == right.shape and left.stride() == right.stride():
            sgm_census_pair(left, right, p.win_w, p.win_h, out_left=self.census_left,
                            out_right=self.census_right, width=self.width, stream=stream)
        else:
            sgm_census(left, p.win_w, p.win_h, out=self.census_left, width=self.width,
                       stream=stream)
            sgm_census(right, p.win_w, p.win_h, out=self.census_right, width=self.width,
                       stream=stream)
        sgm_cost(self.census_left, self.census_right, p.ndisp, out=self.cost, stream=stream)
        if self.fused:
            sgm_aggregate_select(self.cost, p.npaths, p.p1, p.p2, p.lr_tolerance, p.median3x3,
                                 out=self.disp, out_right=self.disp_right, work=self.select_work,
                                 stream=stream)
        else:
            sgm_aggregate(self.cost, p.npaths, p.p1, p.p2, out=self.agg, work=self.agg_work,
                          stream=stream)
            sgm_wta_lrc(self.agg, p.lr_tolerance, p.median3x3, out=self.disp,
                        out_right=self.disp_right, work=self.work, stream=stream)
        return self.disp

    def capture(self, left: torch.Tensor, right: torch.Tensor):
        """Captures run(left, right) into a HIP graph (torch.cuda.CUDAGraph)
        and returns it: graph.replay() re-runs the path on whatever the two
        input tensors hold, into this object's buffers.  The library's calls
        allocate nothing and never synchronise, so they capture as they
        are."""
        side = torch.cuda.Stream(device=left.device)
        side.wait_stream(torch.cuda.current_stream(left.device))
        with torch.cuda.stream(side):
            self.run(left, right)                  # warm-up outside the graph
        torch.cuda.current_stream(left.device).wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.run(left, right)
        return graph


def _params_struct(p: Params) -> SgmParams:
    return SgmParams(p.win_w, p.win_h, p.npaths, p.p1, p.p2, p.lr_tolerance, int(bool(p.median3x3)))


def disparity_exact_lr_work_bytes(width: int, height: int, params: Params) -> int:
    prm = _params_struct(params)
    return int(load_library().sgm_disparity_exact_lr_work_bytes(width, height, params.ndisp,
                                                                ctypes.byref(prm)))


def sgm_disparity_exact_lr(left: torch.Tensor, right: torch.Tensor, params: Params,
                           out: Optional[torch.Tensor] = None,
                           out_right: Optional[torch.Tensor] = None,
                           work: Optional[torch.Tensor] = None, want_right: bool = False,
                           stream=None):
    """The whole path with the exact consistency check (D^R matched from
    scratch on the swapped, flipped pair).  left, right: uint8 [H][W] device
    images.  Returns (disp, exact D^R or None), uint16 [H][W]."""
    if left.dtype != torch.uint8 or left.dim() != 2 or right.shape != left.shape or \
            right.dtype != torch.uint8:
        raise ValueError("left and right must be uint8 [H][W] tensors of one shape")
    h, w = left.shape
    dev = left.device
    if out is None:
        out = _empty((h, w), torch.uint16, dev)
    _expect(out, torch.uint16, (h, w), "out")
    if want_right and out_right is None:
        out_right = _empty((h, w), torch.uint16, dev)
    if out_right is not None:
        _expect(out_right, torch.uint16, (h, w), "out_right")
    if work is None:
        work = _aligned_bytes(max(1, disparity_exact_lr_work_bytes(w, h, params)), dev)
    prm = _params_struct(params)
    _check(load_library().sgm_disparity_exact_lr(_ptr(left), _ptr(right), w, h, w, params.ndisp,
                                                 ctypes.byref(prm), _ptr(out), _ptr(out_right),
                                                 _ptr(work), work.numel(), _stream(stream)))
    return out, out_right


class BatchPlan:
    """Many pairs of uneven size and disparity range as one captured hipGraph.

    lefts / rights: uint8 [H][W] device tensors (kept alive by the plan);
    ndisps: disparity range per pair.  Outputs: self.disp[i] (and
    self.disp_right[i] if want_right), uint16 [H][W].  run() enqueues one
    graph launch; the inputs may be overwritten in place between runs.
    """

    def __init__(self, lefts, rights, ndisps, params: Params, tune_table: Optional[str] = None,
                 want_right: bool = False):
        lib = load_library()
        n = len(lefts)
        if not (n == len(rights) == len(ndisps)) or n < 1:
            raise ValueError("lefts, rights and ndisps must have the same, non-zero length")
        self.lefts, self.rights, self.params = list(lefts), list(rights), params
        dev = self.lefts[0].device
        self.disp, self.disp_right = [], []
        pairs = (SgmPair * n)()
        for i, (l, r, nd) in enumerate(zip(self.lefts, self.rights, ndisps)):
            if l.dtype != torch.uint8 or l.dim() != 2 or l.shape != r.shape or r.dtype != torch.uint8:
                raise ValueError(f"pair {i}: expected two uint8 [H][W] tensors of one shape")
            h, w = l.shape
            d = _empty((h, w), torch.uint16, dev)
            dr = _empty((h, w), torch.uint16, dev) if want_right else None
            self.disp.append(d)
            self.disp_right.append(dr)
            pairs[i] = SgmPair(_ptr(l).value, _ptr(r).value, w, h, w, int(nd), _ptr(d).value,
                               _ptr(dr).value if dr is not None else None)
        self._pairs = pairs
        prm = _params_struct(params)
        table = tune_table.encode() if tune_table else None
        need = int(lib.sgm_batch_workspace_bytes(pairs, n, ctypes.byref(prm), table))
        if need == 0:
            raise ValueError("invalid batch (sizes, disparity ranges or parameters)")
        self.workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        offset = (-base) % 256
        handle = ctypes.c_void_p()
        _check(lib.sgm_batch_plan_create(pairs, n, ctypes.byref(prm),
                                         ctypes.c_void_p(base + offset), need, table,
                                         ctypes.byref(handle)))
        self._handle = handle
        self.n = n

    def run(self, stream=None):
        if not self._handle:
            raise RuntimeError("plan destroyed")
        _check(load_library().sgm_batch_run(self._handle, _stream(stream)))

    def close(self):
        if self._handle:
            load_library().sgm_batch_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
