"""Host-side accounting of the work of a whole-frame call, for measurement.

`census_tiles` lists the 64 x 32 level-pixel tiles whose descriptors a whole-frame or
batch call makes: by default those that meet a range some ranged box's search reads (the
rule stated with `ocsr_range_frame` in the C header), with the full-census option all of
them. `census_pixels` counts the level pixels of those tiles that lie in the image, the
unit the census kernel's work is priced in.
"""
from __future__ import annotations

import numpy as np

TILE_X, TILE_Y = 64, 32
BOX_RANGE = 1


def _cdiv(a: int, s: int) -> int:
    return -(-a // s)


def _levels(W: int, H: int, params: dict):
    s = params["close_scale"]
    return [(W, H, 1, params["far"]), (W // s, H // s, s, params["close"])]


def census_tiles(W: int, H: int, boxes, params: dict, full: bool = False) -> set:
    """(level, view, tile x, tile y) of every tile a call makes (view 0 = left)."""
    out = set()
    sx, sy = params["sx"], params["sy"]
    boxes = np.asarray(boxes).reshape(-1, 5)
    for level, (Wl, Hl, s, ph) in enumerate(_levels(W, H, params)):
        ntx, nty = _cdiv(Wl, TILE_X), _cdiv(Hl, TILE_Y)
        if full:
            out |= {(level, v, tx, ty) for v in (0, 1) for tx in range(ntx) for ty in range(nty)}
            continue
        dlo = ph["dmin"] // s
        dhi = dlo + _cdiv(ph["dmax"] - ph["dmin"] + 1, s) - 1
        # level vertical offsets (0, 0 without a vertical range)
        eylo, eyhi = params.get("dy_min", 0) // s, _cdiv(params.get("dy_max", 0), s)
        ey = eyhi - eylo
        for x0, y0, x1, y1, flags in boxes.tolist():
            cx0, cy0, cx1, cy1 = max(x0, 0), max(y0, 0), min(x1, W), min(y1, H)
            if not (flags & BOX_RANGE) or cx0 >= cx1 or cy0 >= cy1:
                continue
            if (0 if max(cx1 - cx0, cy1 - cy0) < params["tau_s"] else 1) != level:
                continue
            lx0, lx1 = max(_cdiv(cx0, s), sx), min(_cdiv(cx1, s), Wl - sx)
            ly0, ly1 = max(_cdiv(cy0, s), sy), min(_cdiv(cy1, s), Hl - sy)
            if lx0 >= lx1 or ly0 >= ly1:
                continue
            for view, (a, b, ya, yb) in enumerate(
                    ((lx0 - (dhi - dlo), lx1 + (dhi - dlo), ly0 - ey, ly1 + ey),
                     (lx0 - dhi, lx1 - dlo, ly0 + eylo, ly1 + eyhi))):
                a, b = max(a, 0), min(b, ntx * TILE_X)
                ya, yb = max(ya, 0), min(yb, nty * TILE_Y)
                if a >= b or ya >= yb:
                    continue
                for ty in range(ya // TILE_Y, (yb - 1) // TILE_Y + 1):
                    for tx in range(a // TILE_X, (b - 1) // TILE_X + 1):
                        out.add((level, view, tx, ty))
    return out


def census_pixels(W: int, H: int, tiles: set, params: dict) -> int:
    """Level pixels inside the image of the given tiles."""
    n = 0
    lv = _levels(W, H, params)
    for level, _, tx, ty in tiles:
        Wl, Hl = lv[level][0], lv[level][1]
        n += (min(Wl, (tx + 1) * TILE_X) - tx * TILE_X) * (min(Hl, (ty + 1) * TILE_Y) - ty * TILE_Y)
    return n
