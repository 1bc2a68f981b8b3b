"""Seeded synthetic stereo scenes and the matching presets of the five workloads.

This module is the only input source shared by the CPU oracle and the HIP
path. It renders rectified uint8 stereo pairs of textured fronto-parallel
planes and returns the detection boxes that cover them; it holds none of the
census / matching / aggregation arithmetic.

Scene recipe (one image pair):
  1. texture: U[0,1) noise, separable Gaussian blur (sigma 1.5, radius 5,
     symmetric padding), affine rescale to [0, 255], rint -> left image;
  2. planes: axis-aligned rectangles in left coordinates, each with a constant
     (fractional) disparity; the background has disparity 0.5; the visible
     surface at a left pixel is the covering plane of largest disparity;
  3. right pixel (x, y): among the surfaces whose left rectangle contains
     (x + d_k, y), plus the background, take the largest d_k; if the left
     surface visible at floor(x + d_k) and floor(x + d_k) + 1 is that same
     surface (both inside the image) the right value is the linear
     interpolation of the left image there, otherwise the pixel is occluded
     and takes a value from an independent blurred-noise field;
  4. radiometric change: R = g*R + o + N(0, 2^2), g ~ U[0.8, 1.2],
     o ~ U[-20, 20] per frame, rint, clip to [0, 255].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BOX_RANGE = 1  # box flag: produce a range for this box (others only occlude)

MODE_TILED = 0
MODE_GRID = 1
AGG_SEGMENT_MEDIAN = 0
AGG_TRIMMED_MEDIAN = 1


@dataclasses.dataclass
class Scene:
    left: np.ndarray      # uint8 [H, W]
    right: np.ndarray     # uint8 [H, W]
    boxes: np.ndarray     # int32 [N, 5]: x0, y0, x1, y1 (half-open, px), flags
    truth: np.ndarray     # float32 [N]: plane disparity of each box (px)
    seed: int


def _blur_kernel(sigma: float = 1.5, radius: int = 5) -> np.ndarray:
    i = np.arange(-radius, radius + 1, dtype=np.float64)
    k = np.exp(-(i * i) / (2.0 * sigma * sigma))
    return k / k.sum()


def blurred_noise(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    """Float field in [0, 255]: uniform noise, separable Gaussian blur, rescale."""
    k = _blur_kernel()
    r = (len(k) - 1) // 2
    t = rng.random((H, W))
    p = np.pad(t, ((0, 0), (r, r)), mode="symmetric")
    t = sum(k[i] * p[:, i:i + W] for i in range(len(k)))
    p = np.pad(t, ((r, r), (0, 0)), mode="symmetric")
    t = sum(k[i] * p[i:i + H, :] for i in range(len(k)))
    lo, hi = float(t.min()), float(t.max())
    return (t - lo) * (255.0 / max(hi - lo, 1e-12))


def render_pair(rng: np.random.Generator, H: int, W: int, planes) -> tuple[np.ndarray, np.ndarray]:
    """planes: list of (x0, y0, x1, y1, d) rectangles in left coordinates."""
    tex = blurred_noise(rng, H, W)
    left_f = np.rint(tex)
    left = left_f.astype(np.uint8)
    occl = blurred_noise(np.random.default_rng(rng.integers(1 << 62)), H, W)

    # visible surface in the left image
    vis_d = np.full((H, W), 0.5, dtype=np.float64)
    vis_id = np.full((H, W), -1, dtype=np.int32)
    for k, (x0, y0, x1, y1, d) in enumerate(planes):
        x0c, x1c, y0c, y1c = max(x0, 0), min(x1, W), max(y0, 0), min(y1, H)
        if x0c >= x1c or y0c >= y1c:
            continue
        sub = vis_d[y0c:y1c, x0c:x1c]
        upd = d > sub
        sub[upd] = d
        vis_id[y0c:y1c, x0c:x1c][upd] = k

    # best surface for each right pixel
    best_d = np.full((H, W), 0.5, dtype=np.float64)
    best_id = np.full((H, W), -1, dtype=np.int32)
    for k, (x0, y0, x1, y1, d) in enumerate(planes):
        # right x such that x0 <= x + d < x1
        rx0 = max(int(math.ceil(x0 - d)), 0)
        rx1 = min(int(math.ceil(x1 - d)), W)
        y0c, y1c = max(y0, 0), min(y1, H)
        if rx0 >= rx1 or y0c >= y1c:
            continue
        sub = best_d[y0c:y1c, rx0:rx1]
        upd = d > sub
        sub[upd] = d
        best_id[y0c:y1c, rx0:rx1][upd] = k

    xs = np.arange(W, dtype=np.float64)[None, :] + best_d
    xf = np.floor(xs).astype(np.int64)
    frac = xs - xf
    inside = (xf >= 0) & (xf + 1 < W)
    xa = np.clip(xf, 0, W - 1)
    xb = np.clip(xf + 1, 0, W - 1)
    rows = np.arange(H)[:, None]
    same = inside & (vis_id[rows, xa] == best_id) & (vis_id[rows, xb] == best_id)
    warped = (1.0 - frac) * left_f[rows, xa] + frac * left_f[rows, xb]
    right_f = np.where(same, warped, occl)
    g = rng.uniform(0.8, 1.2)
    o = rng.uniform(-20.0, 20.0)
    right_f = g * right_f + o + rng.normal(0.0, 2.0, size=(H, W))
    right = np.clip(np.rint(right_f), 0, 255).astype(np.uint8)
    return left, right


def drift_rows(img: np.ndarray, dy: int) -> np.ndarray:
    """The image moved down by dy rows (up for dy < 0), the vacated rows repeating the
    nearest edge row: out[y] = img[clamp(y - dy)]. Applied to the right view it stands
    for a residual vertical misalignment of the rectified pair, so that the match of
    left row y sits on right row y + dy."""
    H = img.shape[0]
    rows = np.clip(np.arange(H) - int(dy), 0, H - 1)
    return np.ascontiguousarray(img[rows])


def shifted_texture(seed: int, H: int, W: int, dx: int, dy: int,
                    mode: str = "2d") -> tuple[np.ndarray, np.ndarray]:
    """Left texture and a right view that is the same texture moved by (-dx, +dy), cut
    from one larger field: right(x - dx, y + dy) = left(x, y) wherever both exist.
    mode "2d": blurred noise; "cols": every row the same (varies along x only);
    "rows": every column the same (varies along y only)."""
    rng = np.random.default_rng(seed)
    pad = 8 + abs(dx) + abs(dy)
    if mode == "2d":
        big = blurred_noise(rng, H + 2 * pad, W + 2 * pad)
    elif mode == "cols":
        big = np.repeat(rng.integers(0, 256, (1, W + 2 * pad)).astype(np.float64), H + 2 * pad, 0)
    else:
        big = np.repeat(rng.integers(0, 256, (H + 2 * pad, 1)).astype(np.float64), W + 2 * pad, 1)
    big = np.rint(big).astype(np.uint8)
    left = big[pad:pad + H, pad:pad + W]
    right = big[pad - dy:pad - dy + H, pad + dx:pad + dx + W]
    return np.ascontiguousarray(left), np.ascontiguousarray(right)


def road_pair(seed: int = 4000, H: int = 1080, W: int = 1920, drift: int = 0):
    """A ground-like pair for the rectification-offset search: below the horizon
    (H / 2) 12 horizontal bands, each a fronto-parallel plane whose disparity grows
    toward the bottom (4, 12, ..., 92 px at 1080 rows), over a far background; the right
    view then moved down by `drift` rows (drift_rows)."""
    rng = np.random.default_rng(seed)
    h0 = H // 2
    band = max(1, (H - h0) // 12)
    planes = [(-100, h0 + k * band, W + 100, h0 + (k + 1) * band if k < 11 else H,
               (4.0 + 8.0 * k) * H / 1080.0) for k in range(12)]
    left, right = render_pair(rng, H, W, planes)
    return left, drift_rows(right, drift)


def _overlap(a, b) -> bool:
    return a[0] < b[2] and b[0] < a[2] and a[1] < b[3] and b[1] < a[3]


def _recip_uniform(rng, lo, hi):
    """Disparity whose reciprocal (depth) is uniform on [1/hi, 1/lo]."""
    return 1.0 / rng.uniform(1.0 / hi, 1.0 / lo)


# --------------------------------------------------------------------------------------
# matching presets (plain parameter dictionaries, consumed by both sides)
# --------------------------------------------------------------------------------------

def base_params() -> dict:
    return dict(
        sx=3, sy=4, sentinel=1, close_scale=2,
        tau_s=64,
        far=dict(mode=MODE_TILED, bw=4, bh=4, n_side=8, dmin=0, dmax=31),
        close=dict(mode=MODE_TILED, bw=8, bh=8, n_side=8, dmin=0, dmax=191),
        lr_tol=1, min_point_pct=50,
        agg_mode=AGG_TRIMMED_MEDIAN, tau_d=1.0, n_min=3, trim_pct=20,
        focal_px=2000.0, baseline_m=0.30, d_eps=0.0,
    )


def point_geometry(width: int, height: int, params: dict) -> dict:
    """Camera geometry of the point step for a rectified pair with the preset's f and b:
    principal point at the image centre, camera x/y/z mapped to vehicle z-up axes
    (x forward = camera z, y left = -camera x, z up = -camera y), camera 1.5 m above
    and 1.2 m ahead of the vehicle origin."""
    f, b = float(params["focal_px"]), float(params["baseline_m"])
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    Q = [[1, 0, 0, -cx], [0, 1, 0, -cy], [0, 0, 0, f], [0, 0, 1 / b, 0]]
    R = [[0, 0, 1], [-1, 0, 0], [0, -1, 0]]
    return dict(width=width, height=height, Q=Q, R=R, t=[1.2, 0.0, 1.5], focal_px=f,
                baseline_m=b, var_d=0.25, var_x=0.01, var_y=0.01)


def params_for(config: int, width: int = 1920) -> dict:
    p = base_params()
    if config == 1:
        p.update(tau_s=1 << 30, agg_mode=AGG_SEGMENT_MEDIAN)
        p["far"] = dict(mode=MODE_TILED, bw=8, bh=8, n_side=8, dmin=0, dmax=63)
    elif config in (2, 3, 4):
        pass
    elif config == 5:
        p["tau_s"] = int(round(64 * width / 1920))
    else:
        raise ValueError(config)
    return p


# --------------------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------------------

def scene_tiny(seed: int = 1000) -> Scene:
    """640x480, 4 planes 40x30..160x120 px at disparity U[2, 60], all boxes ranged."""
    rng = np.random.default_rng(seed)
    H, W = 480, 640
    while True:
        planes = []
        for _ in range(4):
            w = int(rng.integers(40, 161))
            h = int(round(0.75 * w))
            x0 = int(rng.integers(8, W - 8 - w + 1))
            y0 = int(rng.integers(8, H - 8 - h + 1))
            planes.append((x0, y0, x0 + w, y0 + h, float(rng.uniform(2.0, 60.0))))
        ok = True
        for a in planes:
            for b in planes:
                if a is not b and _overlap(a, b) and a[4] > b[4] and not (a[3] > b[3]):
                    ok = False  # a nearer plane must also have the larger bottom y
        if ok:
            break
    left, right = render_pair(rng, H, W, planes)
    boxes = np.array([[p[0], p[1], p[2], p[3], BOX_RANGE] for p in planes], dtype=np.int32)
    truth = np.array([p[4] for p in planes], dtype=np.float32)
    return Scene(left, right, boxes, truth, seed)


def scene_realistic(seed: int = 2000, H: int = 1080, W: int = 1920) -> Scene:
    """32 non-overlapping targets (19 far, 13 close), each with one nearer corner occluder."""
    rng = np.random.default_rng(seed)
    targets = []
    kinds = [0] * 19 + [1] * 13
    rng.shuffle(kinds)
    for kind in kinds:
        for _attempt in range(10000):
            if kind == 0:
                w = int(rng.integers(16, 64))
                d = _recip_uniform(rng, 2.0, 15.0)
            else:
                w = int(rng.integers(64, 401))
                d = _recip_uniform(rng, 16.0, 180.0)
            h = int(np.clip(round(w * rng.uniform(0.6, 1.0)), 16, 300))
            x0 = int(rng.integers(12, W - 12 - w + 1))
            y0 = int(rng.integers(12, H - 12 - h + 1))
            t = (x0, y0, x0 + w, y0 + h, d)
            # keep a margin so that each occluder can stay clear of other targets
            grown = (x0 - 10, y0 - 10, x0 + w + 10, y0 + h + 10)
            if all(not _overlap(grown, o) for o in targets):
                targets.append(t)
                break
        else:
            raise RuntimeError("placement failed")
    occluders = []
    for t in targets:
        x0, y0, x1, y1, d = t
        w, h = x1 - x0, y1 - y0
        ow, oh = max(1, int(round(0.5 * w))), max(1, int(round(0.3 * h)))
        for _attempt in range(1000):
            left_side = bool(rng.integers(0, 2))
            if left_side:
                ox0, ox1 = x0 - 8, x0 + ow
            else:
                ox0, ox1 = x1 - ow, x1 + 8
            oy0, oy1 = y1 - oh, y1 + 8
            o = (max(ox0, 0), oy0, min(ox1, W), min(oy1, H), d + float(rng.uniform(2.0, 8.0)))
            if all(not _overlap(o, u) for u in targets if u is not t) and \
               all(not _overlap(o, u) for u in occluders):
                occluders.append(o)
                break
        else:
            raise RuntimeError("occluder placement failed")
    planes = targets + occluders
    left, right = render_pair(rng, H, W, planes)
    boxes = np.array([[p[0], p[1], p[2], p[3], BOX_RANGE] for p in targets] +
                     [[p[0], p[1], p[2], p[3], 0] for p in occluders], dtype=np.int32)
    truth = np.array([p[4] for p in planes], dtype=np.float32)
    return Scene(left, right, boxes, truth, seed)


def random_boxes(rng, H, W, n, scale=1.0, far_band=(2.0, 15.0), close_band=(16.0, 180.0),
                 tau_s=64):
    """Box sizes log-uniform 12..512 px (times scale), class by max side vs tau_s."""
    planes = []
    for _ in range(n):
        w = int(round(math.exp(rng.uniform(math.log(12), math.log(512))) * scale))
        h = int(np.clip(round(w * rng.uniform(0.6, 1.0)), round(12 * scale), round(512 * scale)))
        w, h = min(w, W - 1), min(h, H - 1)
        far = max(w, h) < tau_s
        d = _recip_uniform(rng, *(far_band if far else close_band))
        x0 = int(rng.integers(0, W - w + 1))
        y0 = int(rng.integers(0, H - h + 1))
        planes.append((x0, y0, x0 + w, y0 + h, d))
    return planes


def scene_batch_frame(frame: int, H: int = 1200, W: int = 1920) -> Scene:
    """One frame of the 16-frame batch: min(128, Poisson(40)) boxes, overlaps allowed."""
    seed = 3000 + frame
    rng = np.random.default_rng(seed)
    n = min(128, int(rng.poisson(40)))
    planes = random_boxes(rng, H, W, n)
    left, right = render_pair(rng, H, W, planes)
    boxes = np.array([[p[0], p[1], p[2], p[3], BOX_RANGE] for p in planes],
                     dtype=np.int32).reshape(-1, 5)
    truth = np.array([p[4] for p in planes], dtype=np.float32)
    return Scene(left, right, boxes, truth, seed)


def scene_small(seed: int, H: int = 96, W: int = 128, n_planes: int = 3) -> Scene:
    """Small random scene for brute-force and parity sweeps (boxes may overlap)."""
    rng = np.random.default_rng(seed)
    planes = []
    for _ in range(n_planes):
        w = int(rng.integers(8, max(9, W // 2)))
        h = int(rng.integers(8, max(9, H // 2)))
        x0 = int(rng.integers(-4, W - w + 4))
        y0 = int(rng.integers(-4, H - h + 4))
        planes.append((x0, y0, x0 + w, y0 + h, float(rng.uniform(1.0, 12.0))))
    left, right = render_pair(rng, H, W, planes)
    flags = rng.integers(0, 4, size=n_planes)  # about one box in four only occludes
    boxes = np.array([[p[0], p[1], p[2], p[3], int(f != 0)] for p, f in zip(planes, flags)],
                     dtype=np.int32).reshape(-1, 5)
    truth = np.array([p[4] for p in planes], dtype=np.float32)
    return Scene(left, right, boxes, truth, seed)


def serving_pool_pair(res: tuple[int, int], i: int, seed: int = 5000) -> tuple[np.ndarray, np.ndarray]:
    """Pair i of the pre-rendered pool of one resolution."""
    H, W = res
    rng = np.random.default_rng(seed * 1000 + H * 7 + i)
    planes = random_boxes(rng, H, W, 24, scale=W / 1920, tau_s=64 * W / 1920)
    return render_pair(rng, H, W, planes)


def serving_pool(res: tuple[int, int], n: int, seed: int = 5000) -> list[tuple[np.ndarray, np.ndarray]]:
    """Pre-rendered image pairs of one resolution for the request stream."""
    return [serving_pool_pair(res, i, seed) for i in range(n)]


SERVING_RESOLUTIONS = ((720, 1280), (1080, 1920), (2160, 3840))
SERVING_WEIGHTS = (0.3, 0.5, 0.2)
SERVING_CLOSE_RANGES = (128, 192, 256)


def serving_requests(n: int, pool_sizes=(32, 32, 32), seed: int = 5000, rate: float = 120.0):
    """The request stream of the serving workload: Poisson arrivals at `rate` per second,
    resolution drawn with SERVING_WEIGHTS, an image pair drawn from that resolution's
    pool, 1..200 boxes sized as the batch frames scaled by W / 1920, close range
    0..D-1 with D drawn from SERVING_CLOSE_RANGES, far range 0..31.

    Returns dicts with rid, arrival (s), res (index), pool (index), boxes (int32 [n, 5]),
    params."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n):
        t += float(rng.exponential(1.0 / rate))
        ri = int(rng.choice(len(SERVING_RESOLUTIONS), p=SERVING_WEIGHTS))
        H, W = SERVING_RESOLUTIONS[ri]
        nb = int(rng.integers(1, 201))
        planes = random_boxes(rng, H, W, nb, scale=W / 1920, tau_s=64 * W / 1920)
        boxes = np.array([[p[0], p[1], p[2], p[3], BOX_RANGE] for p in planes],
                         dtype=np.int32).reshape(-1, 5)
        D = int(rng.choice(SERVING_CLOSE_RANGES))
        params = params_for(5, width=W)
        params["close"] = dict(params["close"], dmax=D - 1)
        out.append(dict(rid=rid, arrival=t, res=ri, pool=int(rng.integers(0, pool_sizes[ri])),
                        boxes=boxes, params=params))
    return out
