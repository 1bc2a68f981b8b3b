"""ctypes front end of the C oracle (test infrastructure only).

The C source (ocsr_oracle.c) follows the paper step by step; this file only
marshals numpy arrays and the plain parameter dictionaries into the oracle's
own structures. It shares nothing with the HIP library's binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ocsr_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

REASONS = ["OK", "NOT_RANGED", "CLIPPED_EMPTY", "NO_ELIGIBLE_BLOCKS", "NO_VALID_BLOCKS",
           "TOO_FEW_CONSISTENT", "NONPOSITIVE_DISPARITY", "CAPACITY_OVERFLOW"]


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-ffp-contract=off",
           "-mpopcnt", "-shared", "-fPIC", SRC, "-o", LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Path(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("mode", "bw", "bh", "n_side", "dmin", "dmax")]


class _Params(C.Structure):
    _fields_ = [("sx", C.c_int32), ("sy", C.c_int32), ("close_scale", C.c_int32),
                ("tau_s", C.c_int32), ("far_path", _Path), ("close_path", _Path),
                ("lr_tol", C.c_int32), ("min_point_pct", C.c_int32), ("agg_mode", C.c_int32),
                ("tau_d", C.c_float), ("n_min", C.c_int32), ("trim_pct", C.c_int32),
                ("focal_px", C.c_float), ("baseline_m", C.c_float), ("d_eps", C.c_float),
                ("max_blocks_per_box", C.c_int32), ("cap_blocks", C.c_int32),
                ("dy_min", C.c_int32), ("dy_max", C.c_int32)]


BOX_RESULT_DT = np.dtype([("disparity", "<f4"), ("depth", "<f4"), ("valid", "<i4"),
                          ("reason", "<i4"), ("n_blocks", "<i4"), ("n_eligible", "<i4"),
                          ("n_valid", "<i4"), ("n_used", "<i4")])
BLOCK_DT = np.dtype([("box", "<i4"), ("level_scale", "<i4"), ("u", "<i4"), ("v", "<i4"),
                     ("px0", "<i4"), ("py0", "<i4"), ("nx", "<i4"), ("ny", "<i4"),
                     ("mask", "<u8"), ("eligible", "<i4"), ("d_f", "<i4"), ("d_b", "<i4"),
                     ("lr_ok", "<i4"), ("d_sub", "<f4"), ("valid", "<i4"),
                     ("dlo", "<i4"), ("nd", "<i4"), ("dy_f", "<i4"), ("dy_b", "<i4")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"oracle library missing: {LIB} (run oracle.oracle.build())")
        L = C.CDLL(LIB)
        vp = C.c_void_p
        i32 = C.c_int32
        L.orc_census.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, vp]
        L.orc_census.restype = i32
        L.orc_match_boxes.argtypes = [vp, vp, vp, vp, i32, i32, vp, i32, C.POINTER(_Params), vp,
                                      vp, vp, vp, i32, i32, i32]
        L.orc_match_boxes.restype = i32
        L.orc_aggregate.argtypes = [vp, i32, i32, i32, C.POINTER(_Params), vp]
        L.orc_aggregate.restype = None
        L.orc_dense.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, vp, vp, i32]
        L.orc_dense.restype = i32
        L.orc_dense_at.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, vp, i32, vp, i32]
        L.orc_dense_at.restype = i32
        d = C.c_double
        L.orc_box_points.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, d, d, d, d, d, vp]
        L.orc_box_points.restype = None
        L.orc_select_boxes.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp]
        L.orc_select_boxes.restype = None
        L.orc_rect_counts.argtypes = [vp, vp, i32, i32] + [i32] * 11 + [vp, vp, i32]
        L.orc_rect_counts.restype = i32
        L.orc_rect_filter.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp]
        L.orc_rect_filter.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def census(img: np.ndarray, sx: int = 3, sy: int = 4, s: int = 1, sentinel: int = 1) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    out = np.zeros((H // s, W // s), dtype=np.uint64)
    rc = lib().orc_census(_ptr(img), W, H, W, sx, sy, s, sentinel, _ptr(out))
    if rc != 0:
        raise ValueError("orc_census rejected its arguments")
    return out


def make_params(p: dict, cap_blocks: int = 0) -> _Params:
    q = _Params()
    q.sx, q.sy, q.close_scale, q.tau_s = p["sx"], p["sy"], p["close_scale"], p["tau_s"]
    for name, dst in (("far", q.far_path), ("close", q.close_path)):
        src = p[name]
        for f in ("mode", "bw", "bh", "n_side", "dmin", "dmax"):
            setattr(dst, f, int(src[f]))
    q.lr_tol, q.min_point_pct, q.agg_mode = p["lr_tol"], p["min_point_pct"], p["agg_mode"]
    q.tau_d, q.n_min, q.trim_pct = p["tau_d"], p["n_min"], p["trim_pct"]
    q.focal_px, q.baseline_m, q.d_eps = p["focal_px"], p["baseline_m"], p["d_eps"]
    # the method sets no per-box limit: 0 (the default) means none
    q.max_blocks_per_box = p.get("max_blocks_per_box", 0)
    q.cap_blocks = cap_blocks
    q.dy_min, q.dy_max = p.get("dy_min", 0), p.get("dy_max", 0)
    return q


def match_boxes(L0, R0, L1, R1, W: int, H: int, boxes: np.ndarray, params: dict,
                debug: bool = False, threads: int = 0, cap_blocks: int = 0,
                cap_dbg: int = 0):
    """Returns (box results [n] structured, blocks or None, cost_f, cost_b, n_total)."""
    boxes = np.ascontiguousarray(boxes, dtype=np.int32).reshape(-1, 5)
    n = boxes.shape[0]
    out = np.zeros(n, dtype=BOX_RESULT_DT)
    q = make_params(params, cap_blocks)
    L0 = np.ascontiguousarray(L0, dtype=np.uint64)
    R0 = np.ascontiguousarray(R0, dtype=np.uint64)
    L1 = None if L1 is None else np.ascontiguousarray(L1, dtype=np.uint64)
    R1 = None if R1 is None else np.ascontiguousarray(R1, dtype=np.uint64)
    blocks = cf = cb = None
    cap_nd = 0
    if debug:
        # a first pass to learn the block count
        total = lib().orc_match_boxes(_ptr(L0), _ptr(R0), _ptr(L1), _ptr(R1), W, H, _ptr(boxes),
                                      n, C.byref(q), _ptr(out), None, None, None, 0, 0, threads)
        if total < 0:
            raise ValueError("orc_match_boxes rejected its arguments")
        cap_dbg = max(cap_dbg, total, 1)
        cap_nd = 256
        blocks = np.zeros(cap_dbg, dtype=BLOCK_DT)
        cf = np.zeros((cap_dbg, cap_nd), dtype=np.uint16)
        cb = np.zeros((cap_dbg, cap_nd), dtype=np.uint16)
    total = lib().orc_match_boxes(_ptr(L0), _ptr(R0), _ptr(L1), _ptr(R1), W, H, _ptr(boxes), n,
                                  C.byref(q), _ptr(out), _ptr(blocks), _ptr(cf), _ptr(cb),
                                  cap_dbg, cap_nd, threads)
    if total < 0:
        raise ValueError("orc_match_boxes rejected its arguments")
    if debug:
        blocks, cf, cb = blocks[:total], cf[:total], cb[:total]
    return out, blocks, cf, cb, total


def aggregate(vals, n_blocks: int, params: dict, n_eligible: int | None = None,
              far: bool = True):
    """Aggregation + depth of one box from the full-res disparities of its valid blocks.
    far: the box is of type FAR (a FAR box of a single block takes its block result)."""
    v = np.ascontiguousarray(np.asarray(vals, dtype=np.float32).copy())
    out = np.zeros(1, dtype=BOX_RESULT_DT)
    out["n_eligible"] = len(v) if n_eligible is None else n_eligible
    q = make_params(params)
    lib().orc_aggregate(_ptr(v) if len(v) else None, len(v), n_blocks, int(bool(far)), C.byref(q),
                        _ptr(out))
    return out[0]


def run_scene(left, right, params: dict, boxes, debug=False, threads=0, cap_blocks=0):
    """Census of both views at both levels, then matching: the whole path on the CPU."""
    H, W = left.shape
    s = params["close_scale"]
    L0 = census(left, params["sx"], params["sy"], 1, params["sentinel"])
    R0 = census(right, params["sx"], params["sy"], 1, params["sentinel"])
    L1 = census(left, params["sx"], params["sy"], s, params["sentinel"])
    R1 = census(right, params["sx"], params["sy"], s, params["sentinel"])
    res = match_boxes(L0, R0, L1, R1, W, H, boxes, params, debug=debug, threads=threads,
                      cap_blocks=cap_blocks)
    return (L0, R0, L1, R1), res


class _Point(C.Structure):
    _fields_ = [("p_cam", C.c_double * 3), ("p_imu", C.c_double * 3), ("cov_imu", C.c_double * 6),
                ("var_z", C.c_double), ("valid", C.c_int32)]


POINT_DT = np.dtype({"names": ["p_cam", "p_imu", "cov_imu", "var_z", "valid"],
                     "formats": [("<f8", (3,)), ("<f8", (3,)), ("<f8", (6,)), "<f8", "<i4"],
                     "offsets": [0, 24, 48, 96, 104], "itemsize": C.sizeof(_Point)})


def box_points(boxes, results, geom: dict) -> np.ndarray:
    """Per-box 3D point and covariance (Sec. 4.3.6, 4.3.7), fp64: one POINT_DT record per
    box. results: BOX_RESULT_DT records (the disparity and validity of each box)."""
    L = lib()
    b = np.ascontiguousarray(boxes, dtype=np.int32).reshape(-1, 5)
    r = np.ascontiguousarray(results).view(BOX_RESULT_DT)
    n = b.shape[0]
    out = np.zeros(n, dtype=POINT_DT)
    dbl = lambda a, k: np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(k))
    Q, R, t = dbl(geom["Q"], 16), dbl(geom["R"], 9), dbl(geom["t"], 3)
    L.orc_box_points(_ptr(b), _ptr(r), n, int(geom["width"]), int(geom["height"]), _ptr(Q),
                     _ptr(R), _ptr(t), float(geom["focal_px"]), float(geom["baseline_m"]),
                     float(geom["var_d"]), float(geom["var_x"]), float(geom["var_y"]), _ptr(out))
    return out


def dense(CL, CR, dmin=0, dmax=191, radius=2, lr_tol=1, threads=0):
    CL = np.ascontiguousarray(CL, dtype=np.uint64)
    CR = np.ascontiguousarray(CR, dtype=np.uint64)
    H, W = CL.shape
    disp = np.zeros((H, W), dtype=np.int16)
    disp_r = np.zeros((H, W), dtype=np.int16)
    rc = lib().orc_dense(_ptr(CL), _ptr(CR), W, H, dmin, dmax, radius, lr_tol, _ptr(disp),
                         _ptr(disp_r), threads)
    if rc != 0:
        raise ValueError("orc_dense rejected its arguments")
    return disp, disp_r


def dense_at(CL, CR, xy, dmin=0, dmax=191, radius=2, lr_tol=1, threads=0):
    CL = np.ascontiguousarray(CL, dtype=np.uint64)
    CR = np.ascontiguousarray(CR, dtype=np.uint64)
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    H, W = CL.shape
    out = np.zeros(xy.shape[0], dtype=np.int16)
    rc = lib().orc_dense_at(_ptr(CL), _ptr(CR), W, H, dmin, dmax, radius, lr_tol, _ptr(xy),
                            xy.shape[0], _ptr(out), threads)
    if rc != 0:
        raise ValueError("orc_dense_at rejected its arguments")
    return out


def select_boxes(boxes, W: int, H: int, max_objects: int, crop_permille=(333, 0, 667, 1000)):
    """Priority selection of one frame's boxes (Sec. 4.3.5, last sentence). Returns (boxes
    with the new flags, rank per box, -1 for non-candidates)."""
    boxes = np.ascontiguousarray(boxes, dtype=np.int32).reshape(-1, 5)
    n = boxes.shape[0]
    flags = np.zeros(n, np.int32)
    rank = np.zeros(n, np.int32)
    crop = np.ascontiguousarray(crop_permille, dtype=np.int32)
    lib().orc_select_boxes(_ptr(boxes), n, W, H, max_objects, _ptr(crop), _ptr(flags), _ptr(rank))
    out = boxes.copy()
    out[:, 4] = flags
    return out, rank


def rect_counts(CL, CR, p: dict, maps: bool = False, threads: int = 0):
    """Per vertical offset, the ROI pixels with dense disparity > d_min (Sec. 5.1)."""
    CL = np.ascontiguousarray(CL, dtype=np.uint64)
    CR = np.ascontiguousarray(CR, dtype=np.uint64)
    H, W = CL.shape
    nz = p["delta_max"] - p["delta_min"] + 1
    counts = np.zeros(nz, np.int32)
    m = np.zeros((nz, p["roi_h"], p["roi_w"]), np.int16) if maps else None
    rc = lib().orc_rect_counts(_ptr(CL), _ptr(CR), W, H, p["roi_x0"], p["roi_y0"], p["roi_w"],
                               p["roi_h"], p["delta_min"], p["delta_max"], p["dmin"], p["dmax"],
                               p["radius"], p["lr_tol"], p["d_min"], _ptr(counts), _ptr(m), threads)
    if rc != 0:
        raise ValueError("orc_rect_counts rejected its arguments")
    return (counts, m) if maps else counts


def rect_filter(counts_seq, delta_min: int, window: int, max_step: int, initial: int = 0):
    """Offset estimates and filtered offsets of a sequence of frames' counts."""
    c = np.ascontiguousarray(np.asarray(counts_seq, dtype=np.int32))
    T, n = c.shape
    raw = np.zeros(T, np.int32)
    filt = np.zeros(T, np.int32)
    lib().orc_rect_filter(_ptr(c), T, n, delta_min, window, max_step, initial, _ptr(raw), _ptr(filt))
    return raw, filt
