"""Python binding of libocsr (the gfx950 HIP library), through its C ABI.

Argument marshalling only: every step of the method runs in the library's
kernels. PyTorch supplies device memory (tensors) and streams; the library is
called on torch's current stream of the tensors' device. There is no fallback:
if the built library is missing, load() raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libocsr.so")

OK = 0
E_INVALID, E_WORKSPACE, E_CAPACITY, E_HIP, E_UNSUPPORTED = -1, -2, -3, -4, -5
REASONS = ["OK", "NOT_RANGED", "CLIPPED_EMPTY", "NO_ELIGIBLE_BLOCKS", "NO_VALID_BLOCKS",
           "TOO_FEW_CONSISTENT", "NONPOSITIVE_DISPARITY", "CAPACITY_OVERFLOW", "INTERNAL_TIMEOUT"]
MODE_TILED, MODE_GRID = 0, 1
AGG_SEGMENT_MEDIAN, AGG_TRIMMED_MEDIAN = 0, 1
BOX_RANGE = 1
MAX_BATCH_FRAMES = 16
MAX_CANDIDATES = 256
MAX_DY = 32
MAX_SELECT_BOXES = 16384
MAX_RECT_OFFSETS = 64
MAX_DY_CANDIDATES = 2048
MAX_CENSUS_JOBS = 64
DEFAULT_CAP_BLOCKS = 1 << 20

OPTION_FUSED, OPTION_WAVES_PER_CU, OPTION_GRAPH, OPTION_MATCH_WGS_PER_CU, OPTION_BLOCKS_PER_WAVE = 1, 2, 3, 4, 5
OPTION_FULL_CENSUS, OPTION_CENSUS_TILE_LIST, OPTION_LEVEL_LAUNCHES = 6, 7, 8

EXPORTS = ["ocsr_abi_version", "ocsr_last_error", "ocsr_ctx_create", "ocsr_ctx_destroy",
           "ocsr_census", "ocsr_census_many", "ocsr_match_workspace_bytes", "ocsr_match_boxes",
           "ocsr_frame_workspace_bytes", "ocsr_range_frame", "ocsr_batch_workspace_bytes",
           "ocsr_range_batch", "ocsr_ctx_set_option", "ocsr_ctx_set_timing",
           "ocsr_ctx_kernel_time", "ocsr_ctx_reset_timing", "ocsr_ctx_graph_stats",
           "ocsr_variant_candidates", "ocsr_ctx_set_variant", "ocsr_dense_workspace_bytes",
           "ocsr_dense_match", "ocsr_box_points", "ocsr_select_boxes",
           "ocsr_rect_workspace_bytes", "ocsr_rect_offset_counts", "ocsr_rect_filter_create",
           "ocsr_rect_filter_destroy", "ocsr_rect_filter_update", "ocsr_measure_int_rate",
           "ocsr_match_boxes_noalloc"]


class OcsrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ocsr status {code}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------------
# ABI structures (include/ocsr.h)
# ---------------------------------------------------------------------------------
class CensusParams(C.Structure):
    _fields_ = [("sx", C.c_int32), ("sy", C.c_int32), ("scale", C.c_int32), ("sentinel", C.c_int32)]


class CensusJob(C.Structure):
    _fields_ = [("img", C.c_void_p), ("out", C.c_void_p), ("width", C.c_int32),
                ("height", C.c_int32), ("pitch_bytes", C.c_int32), ("out_pitch_elems", C.c_int32),
                ("scale", C.c_int32), ("reserved", C.c_int32)]


class Level(C.Structure):
    _fields_ = [("L", C.c_void_p), ("R", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("pitch_elems", C.c_int32), ("scale", C.c_int32), ("sx", C.c_int32), ("sy", C.c_int32)]


class Path(C.Structure):
    _fields_ = [("mode", C.c_int32), ("bw", C.c_int32), ("bh", C.c_int32), ("n_side", C.c_int32),
                ("dmin", C.c_int32), ("dmax", C.c_int32)]


class MatchParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("tau_s", C.c_int32), ("far_path", Path),
                ("close_path", Path), ("lr_tol", C.c_int32), ("min_point_pct", C.c_int32),
                ("agg_mode", C.c_int32), ("tau_d", C.c_float), ("n_min", C.c_int32),
                ("trim_pct", C.c_int32), ("focal_px", C.c_float), ("baseline_m", C.c_float),
                ("d_eps", C.c_float), ("dy_min", C.c_int32), ("dy_max", C.c_int32)]


class FrameParams(C.Structure):
    _fields_ = [("sx", C.c_int32), ("sy", C.c_int32), ("sentinel", C.c_int32),
                ("close_scale", C.c_int32)]


class RectParams(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("roi_x0", "roi_y0", "roi_w", "roi_h", "delta_min",
                                         "delta_max", "dmin", "dmax", "radius", "lr_tol", "d_min")]


class SelectParams(C.Structure):
    _fields_ = [("max_objects", C.c_int32), ("crop_permille", C.c_int32 * 4)]


class Frame(C.Structure):
    _fields_ = [("imgL", C.c_void_p), ("imgR", C.c_void_p), ("width", C.c_int32),
                ("height", C.c_int32), ("pitch_bytes", C.c_int32), ("box_offset", C.c_int32),
                ("n_boxes", C.c_int32), ("reserved", C.c_int32)]


class Debug(C.Structure):
    _fields_ = [("cap_blocks", C.c_int32), ("cap_nd", C.c_int32), ("n_blocks", C.c_void_p),
                ("blocks", C.c_void_p), ("cost_fwd", C.c_void_p), ("cost_bwd", C.c_void_p)]


class PointParams(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("Q", C.c_double * 16),
                ("R", C.c_double * 9), ("t", C.c_double * 3), ("focal_px", C.c_double),
                ("baseline_m", C.c_double), ("var_d", C.c_double), ("var_x", C.c_double),
                ("var_y", C.c_double)]


BOX_POINT_DTYPE = np.dtype([("p_cam", "<f4", (3,)), ("p_imu", "<f4", (3,)), ("cov_imu", "<f4", (6,)),
                            ("var_z", "<f4"), ("valid", "<i4"), ("reserved", "<i4", (2,))])
assert BOX_POINT_DTYPE.itemsize == 64

BOX_RESULT_DTYPE = np.dtype([("disparity", "<f4"), ("depth", "<f4"), ("valid", "<i4"),
                             ("reason", "<i4"), ("n_blocks", "<i4"), ("n_eligible", "<i4"),
                             ("n_valid", "<i4"), ("n_used", "<i4")])
BLOCK_RECORD_DTYPE = np.dtype([("box", "<i4"), ("level_scale", "<i4"), ("u", "<i4"), ("v", "<i4"),
                               ("px0", "<i4"), ("py0", "<i4"), ("nx", "<i4"), ("ny", "<i4"),
                               ("mask", "<u8"), ("eligible", "<i4"), ("d_f", "<i4"),
                               ("d_b", "<i4"), ("lr_ok", "<i4"), ("d_sub", "<f4"),
                               ("valid", "<i4"), ("dlo", "<i4"), ("nd", "<i4"),
                               ("dy_f", "<i4"), ("dy_b", "<i4")])
assert BOX_RESULT_DTYPE.itemsize == 32 and BLOCK_RECORD_DTYPE.itemsize == 80

_lib = None
_lock = threading.Lock()
_ctx: dict[int, C.c_void_p] = {}


def load(path: str = LIB_PATH):
    """Loads the built library (raises if it is not built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"libocsr is not built: {path} missing "
                               "(run python -m paper_2604_07980_amd.build)")
        L = C.CDLL(path)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.ocsr_abi_version.restype = i32
        L.ocsr_last_error.restype = C.c_char_p
        L.ocsr_ctx_create.argtypes = [i32, C.POINTER(vp)]
        L.ocsr_ctx_create.restype = i32
        L.ocsr_ctx_destroy.argtypes = [vp]
        L.ocsr_ctx_destroy.restype = None
        L.ocsr_census.argtypes = [vp, vp, i32, i32, i32, C.POINTER(CensusParams), vp, i32, vp]
        L.ocsr_census.restype = i32
        L.ocsr_census_many.argtypes = [vp, C.POINTER(CensusJob), i32, i32, i32, i32, vp]
        L.ocsr_census_many.restype = i32
        L.ocsr_match_workspace_bytes.argtypes = [i32, i32]
        L.ocsr_match_workspace_bytes.restype = C.c_size_t
        L.ocsr_match_boxes.argtypes = [vp, C.POINTER(Level), C.POINTER(Level), vp, i32,
                                       C.POINTER(MatchParams), i32, vp, C.c_size_t, vp,
                                       C.POINTER(Debug), vp]
        L.ocsr_match_boxes.restype = i32
        L.ocsr_frame_workspace_bytes.argtypes = [i32, i32, C.POINTER(FrameParams), i32, i32]
        L.ocsr_frame_workspace_bytes.restype = C.c_size_t
        L.ocsr_range_frame.argtypes = [vp, vp, vp, i32, i32, i32, C.POINTER(FrameParams), vp, i32,
                                       C.POINTER(MatchParams), i32, vp, C.c_size_t, vp, vp]
        L.ocsr_range_frame.restype = i32
        L.ocsr_batch_workspace_bytes.argtypes = [C.POINTER(Frame), i32, C.POINTER(FrameParams), i32]
        L.ocsr_batch_workspace_bytes.restype = C.c_size_t
        L.ocsr_range_batch.argtypes = [vp, C.POINTER(Frame), i32, C.POINTER(FrameParams), vp,
                                       C.POINTER(MatchParams), i32, vp, C.c_size_t, vp, vp]
        L.ocsr_range_batch.restype = i32
        L.ocsr_ctx_set_option.argtypes = [vp, i32, i32]
        L.ocsr_ctx_set_option.restype = i32
        L.ocsr_ctx_set_timing.argtypes = [vp, i32]
        L.ocsr_ctx_set_timing.restype = i32
        L.ocsr_ctx_kernel_time.argtypes = [vp, C.c_char_p, C.POINTER(i64), C.POINTER(C.c_double)]
        L.ocsr_ctx_kernel_time.restype = i32
        L.ocsr_ctx_reset_timing.argtypes = [vp]
        L.ocsr_ctx_reset_timing.restype = i32
        L.ocsr_ctx_graph_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
        L.ocsr_ctx_graph_stats.restype = i32
        L.ocsr_variant_candidates.argtypes = [i32, i32, i32, C.POINTER(i32), C.POINTER(i32),
                                              C.POINTER(i32), i32]
        L.ocsr_variant_candidates.restype = i32
        L.ocsr_ctx_set_variant.argtypes = [vp, i32, i32, i32, i32, i32, i32]
        L.ocsr_ctx_set_variant.restype = i32
        L.ocsr_dense_workspace_bytes.argtypes = [i32, i32]
        L.ocsr_dense_workspace_bytes.restype = C.c_size_t
        L.ocsr_dense_match.argtypes = [vp, C.POINTER(Level), i32, i32, i32, i32, vp, vp, vp,
                                       C.c_size_t, vp]
        L.ocsr_dense_match.restype = i32
        L.ocsr_box_points.argtypes = [vp, vp, vp, i32, C.POINTER(PointParams), vp, vp]
        L.ocsr_box_points.restype = i32
        L.ocsr_select_boxes.argtypes = [vp, vp, i32, vp, C.POINTER(SelectParams), vp, vp, vp]
        L.ocsr_select_boxes.restype = i32
        L.ocsr_rect_workspace_bytes.argtypes = [C.POINTER(RectParams)]
        L.ocsr_rect_workspace_bytes.restype = C.c_size_t
        L.ocsr_rect_offset_counts.argtypes = [vp, C.POINTER(Level), C.POINTER(RectParams), vp, vp, vp,
                                              C.c_size_t, vp]
        L.ocsr_rect_offset_counts.restype = i32
        L.ocsr_rect_filter_create.argtypes = [i32, i32, i32, C.POINTER(vp)]
        L.ocsr_rect_filter_create.restype = i32
        L.ocsr_rect_filter_destroy.argtypes = [vp]
        L.ocsr_rect_filter_destroy.restype = None
        L.ocsr_rect_filter_update.argtypes = [vp, vp, i32, i32, C.POINTER(i32), C.POINTER(i32)]
        L.ocsr_rect_filter_update.restype = i32
        L.ocsr_match_boxes_noalloc.argtypes = [vp, C.POINTER(Level), C.POINTER(Level), vp, i32,
                                               C.POINTER(MatchParams), i32, vp, C.POINTER(Debug), vp]
        L.ocsr_match_boxes_noalloc.restype = i32
        L.ocsr_measure_int_rate.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ocsr_measure_int_rate.restype = i32
        _lib = L
        return L


def _check(rc: int):
    if rc != OK:
        raise OcsrError(rc, load().ocsr_last_error().decode())


def context(device: int | None = None) -> C.c_void_p:
    """The library context of a CUDA device (created once per device)."""
    L = load()
    if device is None:
        device = torch.cuda.current_device()
    with _lock:
        if device not in _ctx:
            h = C.c_void_p()
            _check(L.ocsr_ctx_create(device, C.byref(h)))
            _ctx[device] = h
        return _ctx[device]


def _stream(dev: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _dptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _need_cuda(*ts):
    for t in ts:
        if not (isinstance(t, torch.Tensor) and t.is_cuda):
            raise ValueError("expected CUDA tensors")


# ---------------------------------------------------------------------------------
# census
# ---------------------------------------------------------------------------------
def census(img: torch.Tensor, sx: int = 3, sy: int = 4, scale: int = 1, sentinel: int = 1,
           out: torch.Tensor | None = None) -> torch.Tensor:
    """Census descriptors of one uint8 image [H, W] (cuda) at level `scale`:
    int64 [H // scale, W // scale] holding the uint64 codes' bits."""
    _need_cuda(img)
    if img.dtype != torch.uint8 or img.dim() != 2 or img.stride(1) != 1:
        raise ValueError("img must be a row-contiguous uint8 [H, W] tensor")
    H, W = img.shape
    if out is None:
        out = torch.empty((H // scale, W // scale), dtype=torch.int64, device=img.device)
    p = CensusParams(sx, sy, scale, sentinel)
    L = load()
    _check(L.ocsr_census(context(img.device.index), _dptr(img), W, H, img.stride(0), C.byref(p),
                         _dptr(out), out.stride(0), _stream(img.device)))
    return out


def census_many(imgs, scales, sx: int = 3, sy: int = 4, sentinel: int = 1, outs=None):
    """Census of several images/levels in one launch; returns the list of outputs."""
    if len(imgs) != len(scales) or len(imgs) > MAX_CENSUS_JOBS:
        raise ValueError("bad job list")
    _need_cuda(*imgs)
    jobs = (CensusJob * max(1, len(imgs)))()
    res = []
    for k, (img, s) in enumerate(zip(imgs, scales)):
        H, W = img.shape
        o = outs[k] if outs is not None else torch.empty((H // s, W // s), dtype=torch.int64,
                                                         device=img.device)
        res.append(o)
        jobs[k] = CensusJob(img.data_ptr(), o.data_ptr(), W, H, img.stride(0), o.stride(0), s, 0)
    L = load()
    _check(L.ocsr_census_many(context(imgs[0].device.index), jobs, len(imgs), sx, sy, sentinel,
                              _stream(imgs[0].device)))
    return res


# ---------------------------------------------------------------------------------
# matching
# ---------------------------------------------------------------------------------
def make_params(p: dict) -> MatchParams:
    q = MatchParams()
    q.struct_size = C.sizeof(MatchParams)
    q.tau_s = int(min(p["tau_s"], 2**31 - 1))
    for name, dst in (("far", q.far_path), ("close", q.close_path)):
        src = p[name]
        for f in ("mode", "bw", "bh", "n_side", "dmin", "dmax"):
            setattr(dst, f, int(src[f]))
    q.lr_tol, q.min_point_pct, q.agg_mode = p["lr_tol"], p["min_point_pct"], p["agg_mode"]
    q.tau_d, q.n_min, q.trim_pct = p["tau_d"], p["n_min"], p["trim_pct"]
    q.focal_px, q.baseline_m, q.d_eps = p["focal_px"], p["baseline_m"], p["d_eps"]
    q.dy_min, q.dy_max = int(p.get("dy_min", 0)), int(p.get("dy_max", 0))
    return q


def results_to_numpy(res: torch.Tensor) -> np.ndarray:
    """Device result tensor (int32 [N, 8]) -> numpy structured array."""
    return res.cpu().numpy().view(BOX_RESULT_DTYPE).reshape(-1)


def _level(L: torch.Tensor, R: torch.Tensor, scale: int, sx: int, sy: int) -> Level:
    _need_cuda(L, R)
    if L.shape != R.shape or L.dtype != torch.int64 or R.dtype != torch.int64:
        raise ValueError("descriptor tensors must be int64 of equal shape")
    if L.stride(0) != R.stride(0) or L.stride(1) != 1 or R.stride(1) != 1:
        raise ValueError("descriptor tensors must share a row pitch and be row-contiguous")
    H, W = L.shape
    return Level(L.data_ptr(), R.data_ptr(), W, H, L.stride(0), scale, sx, sy)


def _workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + int(nbytes)]


class Workspace:
    """A reusable device workspace: grows on demand, or (with `region`) a fixed
    256-byte-aligned uint8 region of a caller's buffer that never grows."""

    def __init__(self, region: torch.Tensor | None = None):
        if region is not None and (region.dtype != torch.uint8 or region.dim() != 1 or
                                   region.data_ptr() % 256):
            raise ValueError("a workspace region is a 256-byte-aligned 1-D uint8 tensor")
        self.buf = region
        self.fixed = region is not None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.fixed:
            if self.buf.numel() < nbytes or self.buf.device != torch.device(device):
                raise ValueError(f"workspace region of {self.buf.numel()} bytes < {nbytes} needed")
            return self.buf
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != torch.device(device):
            self.buf = _workspace(nbytes, device)
        return self.buf


def match_boxes(L0, R0, L1, R1, boxes: torch.Tensor, params: dict, close_scale: int | None = None,
                cap_blocks: int = DEFAULT_CAP_BLOCKS, debug: bool = False, cap_nd: int = 256,
                workspace: Workspace | None = None, out: torch.Tensor | None = None):
    """Per-box disparity and depth from descriptors (int64 cuda tensors).

    boxes: int32 [N, 5] cuda (x0, y0, x1, y1, flags). Returns the int32 [N, 8] result
    tensor (see BOX_RESULT_DTYPE), plus (n_blocks, records, cost_fwd, cost_bwd)
    device tensors when debug is set.
    """
    _need_cuda(boxes)
    if boxes.dtype != torch.int32 or boxes.dim() != 2 or boxes.shape[1] != 5 or not boxes.is_contiguous():
        raise ValueError("boxes must be a contiguous int32 [N, 5] tensor")
    dev = boxes.device
    sx, sy = params["sx"], params["sy"]
    s = close_scale if close_scale is not None else params["close_scale"]
    lv0 = _level(L0, R0, 1, sx, sy)
    lv1 = _level(L1, R1, s, sx, sy) if L1 is not None else _level(L0, R0, 1, sx, sy)
    n = boxes.shape[0]
    L = load()
    nbytes = L.ocsr_match_workspace_bytes(n, cap_blocks)
    ws = (workspace or Workspace()).get(nbytes, dev)
    if out is None:
        out = torch.empty((n, 8), dtype=torch.int32, device=dev)
    dbg = None
    extra = None
    if debug:
        nb = torch.zeros(1, dtype=torch.int32, device=dev)
        cap_dbg = cap_blocks
        rec = torch.zeros((cap_dbg, BLOCK_RECORD_DTYPE.itemsize), dtype=torch.uint8, device=dev)
        cf = torch.zeros((cap_dbg, cap_nd), dtype=torch.int16, device=dev)
        cb = torch.zeros((cap_dbg, cap_nd), dtype=torch.int16, device=dev)
        dbg = Debug(cap_dbg, cap_nd, nb.data_ptr(), rec.data_ptr(), cf.data_ptr(), cb.data_ptr())
        extra = (nb, rec, cf, cb)
    q = make_params(params)
    _check(L.ocsr_match_boxes(context(dev.index), C.byref(lv0), C.byref(lv1), _dptr(boxes), n,
                              C.byref(q), cap_blocks, _dptr(ws), ws.numel(), _dptr(out),
                              C.byref(dbg) if dbg is not None else None, _stream(dev)))
    if debug:
        return out, extra
    return out


def match_boxes_noalloc(L0, R0, L1, R1, boxes: torch.Tensor, params: dict,
                        close_scale: int | None = None, cap_blocks: int = 1 << 16,
                        out: torch.Tensor | None = None) -> torch.Tensor:
    """match_boxes with the library's own device scratch (no workspace, nothing allocated
    by the library). Returns the int32 [N, 8] result tensor."""
    _need_cuda(boxes)
    if boxes.dtype != torch.int32 or boxes.dim() != 2 or boxes.shape[1] != 5 or not boxes.is_contiguous():
        raise ValueError("boxes must be a contiguous int32 [N, 5] tensor")
    dev = boxes.device
    sx, sy = params["sx"], params["sy"]
    s = close_scale if close_scale is not None else params["close_scale"]
    lv0 = _level(L0, R0, 1, sx, sy)
    lv1 = _level(L1, R1, s, sx, sy) if L1 is not None else _level(L0, R0, 1, sx, sy)
    n = boxes.shape[0]
    if out is None:
        out = torch.empty((n, 8), dtype=torch.int32, device=dev)
    q = make_params(params)
    _check(load().ocsr_match_boxes_noalloc(context(dev.index), C.byref(lv0), C.byref(lv1),
                                           _dptr(boxes), n, C.byref(q), cap_blocks, _dptr(out),
                                           None, _stream(dev)))
    return out


def debug_to_numpy(extra):
    nb, rec, cf, cb = extra
    n = int(nb.item())
    n_rec = min(n, rec.shape[0])
    recs = rec[:n_rec].cpu().numpy().view(BLOCK_RECORD_DTYPE).reshape(-1)
    cfn = cf[:n_rec].cpu().numpy().view(np.uint16)
    cbn = cb[:n_rec].cpu().numpy().view(np.uint16)
    return n, recs, cfn, cbn


def frame_workspace_bytes(W: int, H: int, params: dict, n_boxes: int,
                          cap_blocks: int = DEFAULT_CAP_BLOCKS) -> int:
    fp = FrameParams(params["sx"], params["sy"], params["sentinel"], params["close_scale"])
    return int(load().ocsr_frame_workspace_bytes(W, H, C.byref(fp), n_boxes, cap_blocks))


def range_frame(imgL: torch.Tensor, imgR: torch.Tensor, boxes: torch.Tensor, params: dict,
                cap_blocks: int = DEFAULT_CAP_BLOCKS, workspace: Workspace | None = None,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """Whole frame (census of both views at both levels, then matching)."""
    _need_cuda(imgL, imgR, boxes)
    if imgL.shape != imgR.shape or imgL.dtype != torch.uint8 or imgL.stride() != imgR.stride():
        raise ValueError("images must be uint8 tensors of equal shape and pitch")
    if boxes.dtype != torch.int32 or boxes.dim() != 2 or boxes.shape[1] != 5 or not boxes.is_contiguous():
        raise ValueError("boxes must be a contiguous int32 [N, 5] tensor")
    H, W = imgL.shape
    dev = imgL.device
    n = boxes.shape[0]
    fp = FrameParams(params["sx"], params["sy"], params["sentinel"], params["close_scale"])
    L = load()
    nbytes = L.ocsr_frame_workspace_bytes(W, H, C.byref(fp), n, cap_blocks)
    ws = (workspace or Workspace()).get(nbytes, dev)
    if out is None:
        out = torch.empty((n, 8), dtype=torch.int32, device=dev)
    q = make_params(params)
    _check(L.ocsr_range_frame(context(dev.index), _dptr(imgL), _dptr(imgR), W, H, imgL.stride(0),
                              C.byref(fp), _dptr(boxes), n, C.byref(q), cap_blocks, _dptr(ws),
                              ws.numel(), _dptr(out), _stream(dev)))
    return out


def _frame_params(params: dict) -> FrameParams:
    return FrameParams(params["sx"], params["sy"], params["sentinel"], params["close_scale"])


def batch_workspace_bytes(shapes, params: dict, cap_blocks: int = 1 << 16) -> int:
    """Workspace bytes of a range_batch call; shapes: list of (H, W, n_boxes)."""
    arr = (Frame * len(shapes))()
    off = 0
    for k, (H, W, nb) in enumerate(shapes):
        arr[k] = Frame(0, 0, W, H, W, off, int(nb), 0)
        off += int(nb)
    n = load().ocsr_batch_workspace_bytes(arr, len(shapes), C.byref(_frame_params(params)), cap_blocks)
    if n == 0:
        raise ValueError("invalid batch description")
    return n


def range_batch(frames, boxes: torch.Tensor, params: dict, cap_blocks: int = 1 << 16,
                workspace: Workspace | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Many frames in one launch sequence.

    frames: list of (imgL, imgR, n_boxes) with uint8 [H, W] cuda images; boxes: int32
    [sum n_boxes, 5] cuda, frame by frame. Returns int32 [sum n_boxes, 8] results.
    """
    if not frames or len(frames) > MAX_BATCH_FRAMES:
        raise ValueError(f"1..{MAX_BATCH_FRAMES} frames per batch")
    _need_cuda(boxes)
    if boxes.dtype != torch.int32 or boxes.dim() != 2 or boxes.shape[1] != 5 or not boxes.is_contiguous():
        raise ValueError("boxes must be a contiguous int32 [N, 5] tensor")
    arr = (Frame * len(frames))()
    off = 0
    for k, (L, R, nb) in enumerate(frames):
        _need_cuda(L, R)
        if L.shape != R.shape or L.dtype != torch.uint8 or L.stride() != R.stride() or L.stride(1) != 1:
            raise ValueError("frame images must be row-contiguous uint8 tensors of equal shape")
        H, W = L.shape
        arr[k] = Frame(L.data_ptr(), R.data_ptr(), W, H, L.stride(0), off, int(nb), 0)
        off += int(nb)
    if off != boxes.shape[0]:
        raise ValueError("box counts of the frames do not add up to the box array")
    dev = boxes.device
    fp = _frame_params(params)
    Lb = load()
    nbytes = Lb.ocsr_batch_workspace_bytes(arr, len(frames), C.byref(fp), cap_blocks)
    if nbytes == 0:
        raise ValueError("invalid batch description")
    ws = (workspace or Workspace()).get(nbytes, dev)
    if out is None:
        out = torch.empty((off, 8), dtype=torch.int32, device=dev)
    q = make_params(params)
    _check(Lb.ocsr_range_batch(context(dev.index), arr, len(frames), C.byref(fp), _dptr(boxes),
                               C.byref(q), cap_blocks, _dptr(ws), ws.numel(), _dptr(out),
                               _stream(dev)))
    return out


def dense(L: torch.Tensor, R: torch.Tensor, dmin: int = 0, dmax: int = 191, radius: int = 2,
          lr_tol: int = 1, right: bool = False, workspace: Workspace | None = None):
    """Dense counterpart on one level's descriptors (int64 [H, W] cuda): int16 [H, W]
    left-view disparity after the left/right check (-1 invalid), and with right=True
    also the right-view winner-take-all map."""
    lv = _level(L, R, 1, 0, 0)
    H, W = L.shape
    dev = L.device
    Lb = load()
    ws = (workspace or Workspace()).get(Lb.ocsr_dense_workspace_bytes(W, H), dev)
    disp = torch.empty((H, W), dtype=torch.int16, device=dev)
    disp_r = torch.empty((H, W), dtype=torch.int16, device=dev) if right else None
    _check(Lb.ocsr_dense_match(context(dev.index), C.byref(lv), dmin, dmax, radius, lr_tol,
                               _dptr(disp), _dptr(disp_r) if right else None, _dptr(ws),
                               ws.numel(), _stream(dev)))
    return (disp, disp_r) if right else disp


def point_params(geom: dict) -> PointParams:
    """ocsr_point_params from a dict: width, height, Q (4x4), R (3x3), t (3), focal_px,
    baseline_m, var_d, var_x, var_y."""
    pp = PointParams()
    pp.width, pp.height = int(geom["width"]), int(geom["height"])
    for name, n in (("Q", 16), ("R", 9), ("t", 3)):
        vals = np.asarray(geom[name], dtype=np.float64).reshape(-1)
        if vals.size != n:
            raise ValueError(f"{name} must have {n} entries")
        getattr(pp, name)[:] = vals.tolist()
    for name in ("focal_px", "baseline_m", "var_d", "var_x", "var_y"):
        setattr(pp, name, float(geom[name]))
    return pp


def box_points(boxes: torch.Tensor, results: torch.Tensor, geom: dict,
               out: torch.Tensor | None = None) -> torch.Tensor:
    """Per-box 3D point and covariance from ranging results (int32 [N, 8] cuda, as
    returned by range_frame / range_batch / match_boxes) and their boxes (int32 [N, 5]).
    Returns an int32 [N, 16] cuda tensor; points_to_numpy views it as BOX_POINT_DTYPE."""
    _need_cuda(boxes, results)
    n = boxes.shape[0]
    if boxes.dtype != torch.int32 or boxes.dim() != 2 or boxes.shape[1] != 5 or not boxes.is_contiguous():
        raise ValueError("boxes must be a contiguous int32 [N, 5] tensor")
    if results.dtype != torch.int32 or tuple(results.shape) != (n, 8) or not results.is_contiguous():
        raise ValueError("results must be a contiguous int32 [N, 8] tensor")
    if out is None:
        out = torch.empty((n, 16), dtype=torch.int32, device=boxes.device)
    pp = point_params(geom)
    _check(load().ocsr_box_points(context(boxes.device.index), _dptr(boxes), _dptr(results), n,
                                  C.byref(pp), _dptr(out), _stream(boxes.device)))
    return out


# ---------------------------------------------------------------------------------
# auto-rectification offset
# ---------------------------------------------------------------------------------
def rect_params(p: dict) -> RectParams:
    return RectParams(*[int(p[k]) for k in ("roi_x0", "roi_y0", "roi_w", "roi_h", "delta_min",
                                            "delta_max", "dmin", "dmax", "radius", "lr_tol",
                                            "d_min")])


def rect_offset_counts(L: torch.Tensor, R: torch.Tensor, p: dict, sx: int = 3, sy: int = 4,
                       with_maps: bool = False, workspace: Workspace | None = None,
                       counts: torch.Tensor | None = None):
    """Counts of ROI pixels with disparity > d_min for every vertical offset of the left
    descriptors (L, R: one level's uint64-as-int64 [H, W] cuda descriptors). Returns the
    int32 [n_offsets] counts, and with with_maps the int16 [n_offsets, roi_h, roi_w] maps."""
    _need_cuda(L, R)
    if L.shape != R.shape or L.dtype != torch.int64 or L.stride() != R.stride() or L.stride(1) != 1:
        raise ValueError("descriptors must be row-contiguous int64 tensors of equal shape")
    rp = rect_params(p)
    Lb = load()
    nbytes = Lb.ocsr_rect_workspace_bytes(C.byref(rp))
    if nbytes == 0:
        raise ValueError("invalid rectification parameters")
    dev = L.device
    ws = (workspace or Workspace()).get(nbytes, dev)
    nz = rp.delta_max - rp.delta_min + 1
    if counts is None:
        counts = torch.empty(nz, dtype=torch.int32, device=dev)
    maps = torch.empty((nz, rp.roi_h, rp.roi_w), dtype=torch.int16, device=dev) if with_maps else None
    lv = _level(L, R, 1, sx, sy)
    _check(Lb.ocsr_rect_offset_counts(context(dev.index), C.byref(lv), C.byref(rp), _dptr(counts),
                                      _dptr(maps) if with_maps else None, _dptr(ws), ws.numel(),
                                      _stream(dev)))
    return (counts, maps) if with_maps else counts


class RectFilter:
    """The library's temporal filter of the per-frame offset estimate (host only)."""

    def __init__(self, window: int, max_step: int, initial: int = 0):
        self._h = C.c_void_p()
        _check(load().ocsr_rect_filter_create(window, max_step, initial, C.byref(self._h)))

    def update(self, counts, delta_min: int) -> tuple[int, int]:
        c = np.ascontiguousarray(np.asarray(counts, dtype=np.int32))
        raw, filt = C.c_int32(), C.c_int32()
        _check(load().ocsr_rect_filter_update(self._h, c.ctypes.data_as(C.c_void_p), len(c),
                                              int(delta_min), C.byref(raw), C.byref(filt)))
        return raw.value, filt.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ocsr_rect_filter_destroy(self._h)
            self._h = None


# Central crop of the selection when none is given: the middle third of the width over
# the full height (the paper leaves the crop's size open).
DEFAULT_CROP_PERMILLE = (333, 0, 667, 1000)


def select_boxes(frames, boxes: torch.Tensor, max_objects: int,
                 crop_permille=DEFAULT_CROP_PERMILLE, out: torch.Tensor | None = None,
                 rank: torch.Tensor | None = None):
    """Priority selection under a per-frame budget. frames: list of (width, height,
    n_boxes), boxes int32 [sum n_boxes, 5] cuda, frame by frame. Returns (boxes with the
    range flag cleared on the candidates past the budget, int32 [N] rank per box, -1 for
    non-candidates)."""
    if not frames or len(frames) > MAX_BATCH_FRAMES:
        raise ValueError(f"1..{MAX_BATCH_FRAMES} frames per call")
    _need_cuda(boxes)
    if boxes.dtype != torch.int32 or boxes.dim() != 2 or boxes.shape[1] != 5 or not boxes.is_contiguous():
        raise ValueError("boxes must be a contiguous int32 [N, 5] tensor")
    arr = (Frame * len(frames))()
    off = 0
    for k, (W, H, nb) in enumerate(frames):
        arr[k] = Frame(None, None, int(W), int(H), int(W), off, int(nb), 0)
        off += int(nb)
    if off != boxes.shape[0]:
        raise ValueError("box counts of the frames do not add up to the box array")
    if out is None:
        out = torch.empty_like(boxes)
    if rank is None:
        rank = torch.empty(boxes.shape[0], dtype=torch.int32, device=boxes.device)
    sp = SelectParams(int(max_objects), (C.c_int32 * 4)(*[int(v) for v in crop_permille]))
    _check(load().ocsr_select_boxes(context(boxes.device.index), arr, len(frames), _dptr(boxes),
                                    C.byref(sp), _dptr(out), _dptr(rank), _stream(boxes.device)))
    return out, rank


def points_to_numpy(pts: torch.Tensor) -> np.ndarray:
    return pts.cpu().numpy().view(BOX_POINT_DTYPE).reshape(-1)


def set_option(option: int, value: int, device: int | None = None):
    _check(load().ocsr_ctx_set_option(context(device), option, value))


def set_fused(enable: bool, device: int | None = None):
    """Whole frames and batches as one persistent launch (True) or the multi-launch path."""
    set_option(OPTION_FUSED, 1 if enable else 0, device)


def set_graph(enable: bool, device: int | None = None):
    """Submit whole-frame and batch calls as cached HIP graphs (True) or launch by launch."""
    set_option(OPTION_GRAPH, 1 if enable else 0, device)


def variant_candidates(bw: int, bh: int, n_candidates: int) -> list[tuple[int, int, int]]:
    """Every (rows, cpl, passes) matching kernel that covers bw x bh blocks and
    n_candidates level candidates (host query, no device needed)."""
    L = load()
    rows, cpl, passes = (C.c_int32 * 64)(), (C.c_int32 * 64)(), (C.c_int32 * 64)()
    n = L.ocsr_variant_candidates(bw, bh, n_candidates, rows, cpl, passes, 64)
    if n < 0:
        raise OcsrError(n, L.ocsr_last_error().decode())
    return [(rows[i], cpl[i], passes[i]) for i in range(min(n, 64))]


def set_variant(bw: int, bh: int, n_candidates: int, rows: int, cpl: int, passes: int = 1,
                device: int | None = None):
    """Use the (rows, cpl, passes) kernel for paths of bw x bh blocks and n_candidates
    level candidates ((0, 0, 0) restores the default; (0, 4, 1) is the generic kernel)."""
    _check(load().ocsr_ctx_set_variant(context(device), bw, bh, n_candidates, rows, cpl, passes))


def level_candidates(path: dict, scale: int) -> int:
    """Level candidates of a path searched at level scale `scale`."""
    return -(-(path["dmax"] - path["dmin"] + 1) // scale)


def graph_stats(device: int | None = None) -> tuple[int, int]:
    """(replays of cached graphs, graph captures) of the device's context so far."""
    hits, builds = C.c_int64(0), C.c_int64(0)
    _check(load().ocsr_ctx_graph_stats(context(device), C.byref(hits), C.byref(builds)))
    return hits.value, builds.value


# ---------------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------------
def set_timing(enable: bool, device: int | None = None):
    _check(load().ocsr_ctx_set_timing(context(device), 1 if enable else 0))


def kernel_time(name: str, device: int | None = None) -> tuple[int, float]:
    n = C.c_int64()
    ms = C.c_double()
    _check(load().ocsr_ctx_kernel_time(context(device), name.encode(), C.byref(n), C.byref(ms)))
    return int(n.value), float(ms.value)


def reset_timing(device: int | None = None):
    _check(load().ocsr_ctx_reset_timing(context(device)))


def measure_int_rate(iters: int = 4096, device: int | None = None) -> tuple[float, float]:
    """The device's int32 vector-ALU rate (lane operations per second) and the timed
    launch's duration in ms, from the library's chain kernel."""
    ops, ms = C.c_double(0.0), C.c_double(0.0)
    _check(load().ocsr_measure_int_rate(context(device), iters, C.byref(ops), C.byref(ms)))
    return ops.value, ms.value
