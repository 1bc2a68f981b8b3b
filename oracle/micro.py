"""NumPy / pure-Python micro-oracle for tiny inputs (test infrastructure only).

A second, independently written statement of the same method, used to
cross-check the C oracle by brute force on small scenes. It enumerates every
candidate explicitly and favours directness over speed: census by shifted
whole-image comparisons, block costs by Python loops over points, dense costs
by full cost volumes.
"""
from __future__ import annotations

import numpy as np

MODE_TILED, MODE_GRID = 0, 1
AGG_SEGMENT, AGG_TRIM = 0, 1


def census(img: np.ndarray, sx: int, sy: int, s: int, sentinel: int) -> np.ndarray:
    """Census equation of Sec. 4.3.1 on the level image I_s(x, y) = I(s x, s y)."""
    H, W = img.shape
    Hs, Ws = H // s, W // s
    lv = img[: Hs * s: s, : Ws * s: s].astype(np.int32)
    assert lv.shape == (Hs, Ws)
    n = (2 * sx + 1) * (2 * sy + 1)
    code = np.zeros((Hs, Ws), dtype=np.uint64)
    pad = np.full((Hs + 2 * sy, Ws + 2 * sx), -1, dtype=np.int32)
    pad[sy:sy + Hs, sx:sx + Ws] = lv
    t = 0
    for i in range(-sx, sx + 1):          # x offset: outer (Alg. 1)
        for j in range(-sy, sy + 1):      # y offset: inner
            nb = pad[sy + j: sy + j + Hs, sx + i: sx + i + Ws]
            bit = (nb > lv).astype(np.uint64)
            code |= bit << np.uint64(n - 1 - t)   # first comparison lands highest
            t += 1
    if sentinel:
        code |= np.uint64(1) << np.uint64(n)
    ys, xs = np.mgrid[0:Hs, 0:Ws]
    defined = (xs >= sx) & (xs < Ws - sx) & (ys >= sy) & (ys < Hs - sy)
    code[~defined] = 0
    return code


def _get(img, x, y):
    H, W = img.shape
    if 0 <= x < W and 0 <= y < H:
        return int(img[y, x])
    return 0


def _ham(a: int, b: int) -> int:
    return bin(a ^ b).count("1")


def _clip(b, W, H):
    x0, y0, x1, y1 = max(b[0], 0), max(b[1], 0), min(b[2], W), min(b[3], H)
    return (x0, y0, x1, y1) if (x0 < x1 and y0 < y1) else None


def _cdiv(a, s):
    return -((-a) // s)


def match_boxes(levels: dict, W: int, H: int, boxes, p: dict):
    """levels: {1: (L, R), s: (L, R)} python-int-friendly uint64 arrays.

    Returns (per-box list of dicts, per-block list of dicts) in the block order
    box, row of blocks, column of blocks.
    """
    boxes = [tuple(int(v) for v in b) for b in np.asarray(boxes).reshape(-1, 5)]
    clips = [_clip(b, W, H) for b in boxes]
    res, blocks = [], []
    total = 0
    for i, b in enumerate(boxes):
        r = dict(reason=None, disparity=0.0, depth=0.0, valid=0, n_blocks=0, n_eligible=0,
                 n_valid=0, n_used=0)
        res.append(r)
        if not (b[4] & 1):
            r["reason"] = 1
            continue
        c = clips[i]
        if c is None:
            r["reason"] = 2
            continue
        far = max(c[2] - c[0], c[3] - c[1]) < p["tau_s"]
        path = p["far"] if far else p["close"]
        s = 1 if far else p["close_scale"]
        Lv, Rv = levels[s]
        Hs, Ws = Lv.shape
        dlo = path["dmin"] // s
        nd = _cdiv(path["dmax"] - path["dmin"] + 1, s)
        # level vertical offsets: the fewest whose s-multiples cover [dy_min, dy_max]
        dylo, dyhi = p.get("dy_min", 0) // s, _cdiv(p.get("dy_max", 0), s)
        # level box
        xs_all = [x for x in range(Ws) if c[0] <= s * x < c[2] and p["sx"] <= x < Ws - p["sx"]]
        ys_all = [y for y in range(Hs) if c[1] <= s * y < c[3] and p["sy"] <= y < Hs - p["sy"]]
        if not xs_all or not ys_all:
            r["reason"] = 3
            continue
        lx0, lw, ly0, lh = xs_all[0], len(xs_all), ys_all[0], len(ys_all)
        tiles = []
        if path["mode"] == MODE_TILED:
            bw, bh = min(path["bw"], lw), min(path["bh"], lh)
            nbx, nby = max(1, lw // path["bw"]), max(1, lh // path["bh"])
            ox = lx0 + (lw - nbx * bw) // 2
            oy = ly0 + (lh - nby * bh) // 2
            for v in range(nby):
                for u in range(nbx):
                    tiles.append((u, v, [ox + u * bw + k for k in range(bw)],
                                  [oy + v * bh + k for k in range(bh)]))
        else:
            nx, ny = min(path["n_side"], lw), min(path["n_side"], lh)
            # sample at the centre of each of nx x ny equal cells of the level box
            xs = [lx0 + int(np.floor((k + 0.5) * lw / nx)) for k in range(nx)]
            ys = [ly0 + int(np.floor((k + 0.5) * lh / ny)) for k in range(ny)]
            tiles.append((0, 0, xs, ys))
        # the method sets no per-box limit; a caller may impose one
        if p.get("max_blocks_per_box", 0) > 0 and len(tiles) > p["max_blocks_per_box"]:
            r["reason"] = 7
            continue
        total += len(tiles)
        r["n_blocks"] = len(tiles)
        occ = [j for j in range(len(boxes)) if j != i and clips[j] is not None
               and clips[j][0] < c[2] and c[0] < clips[j][2] and clips[j][1] < c[3]
               and c[1] < clips[j][3] and clips[j][3] > c[3]]
        vals = []
        for (u, v, xs, ys) in tiles:
            pts = []
            for y in ys:
                for x in xs:
                    hid = any(clips[j][0] <= s * x < clips[j][2] and clips[j][1] <= s * y < clips[j][3]
                              for j in occ)
                    pts.append((x, y, not hid))
            used = [(x, y) for (x, y, keep) in pts if keep]
            elig = len(used) > 0 and 100 * len(used) >= p["min_point_pct"] * len(pts)
            blk = dict(box=i, u=u, v=v, px0=xs[0], py0=ys[0], nx=len(xs), ny=len(ys),
                       mask=sum(1 << k for k, t in enumerate(pts) if t[2]), eligible=int(elig))
            blocks.append(blk)
            if not elig:
                continue
            r["n_eligible"] += 1
            # every (d, e) candidate; min over (cost, d, e) puts ties on the smallest d,
            # then the smallest e
            es = range(dylo, dyhi + 1)
            fall = {(d, e): sum(_ham(_get(Lv, x, y), _get(Rv, x - d, y + e)) for (x, y) in used)
                    for d in range(dlo, dlo + nd) for e in es}
            _, d_f, e_f = min((c, d, e) for (d, e), c in fall.items())
            kf = d_f - dlo
            fwd = [fall[(d, e_f)] for d in range(dlo, dlo + nd)]
            if 0 < kf < nd - 1:
                a, cc, bb = fwd[kf - 1], fwd[kf], fwd[kf + 1]
                dsub = np.float32(d_f) + np.float32(np.float32(a - bb) / np.float32(2 * (a + bb - 2 * cc)))
            else:
                dsub = np.float32(d_f)
            # backward from the matched right point (x - d_f, y + e_f): left at (+d, -e)
            ball = {(d, e): sum(_ham(_get(Rv, x - d_f, y + e_f), _get(Lv, x - d_f + d, y + e_f - e))
                                for (x, y) in used)
                    for d in range(dlo, dlo + nd) for e in es}
            _, d_b, e_b = min((c, d, e) for (d, e), c in ball.items())
            bwd = [ball[(d, e_b)] for d in range(dlo, dlo + nd)]
            ok = abs(d_b - d_f) <= p["lr_tol"]
            blk.update(d_f=d_f, d_b=d_b, dy_f=e_f, dy_b=e_b, lr_ok=int(ok), d_sub=float(dsub),
                       cost_f=fwd, cost_b=bwd)
            if ok:
                vals.append(np.float32(s) * np.float32(dsub))
        r["n_valid"] = len(vals)
        if r["n_eligible"] == 0:
            r["reason"] = 3
            continue
        if not vals:
            r["reason"] = 4
            continue
        vals = sorted(vals)
        if far and len(tiles) == 1:
            # Alg. 2: a FAR object matched as one block takes that block's result
            dbox = vals[0]
            r["n_used"] = 1
        elif p["agg_mode"] == AGG_SEGMENT:
            runs, cur = [], [vals[0]]
            for a, bnext in zip(vals[:-1], vals[1:]):
                if np.float32(bnext - a) < np.float32(p["tau_d"]):
                    cur.append(bnext)
                else:
                    runs.append(cur)
                    cur = [bnext]
            runs.append(cur)
            best = max(runs, key=len)  # max() keeps the first of equal lengths
            r["n_used"] = len(best)
            if len(best) < p["n_min"]:
                r["reason"] = 5
                continue
            dbox = _median(best)
        else:
            t = (p["trim_pct"] * len(vals)) // 100
            kept = vals[t: len(vals) - t]
            r["n_used"] = len(kept)
            if len(kept) < max(p["n_min"], 1):
                r["reason"] = 5
                continue
            dbox = _median(kept)
        r["disparity"] = float(dbox)
        if not dbox > p["d_eps"]:
            r["reason"] = 6
            continue
        fb = np.float32(p["focal_px"]) * np.float32(p["baseline_m"])
        r["depth"] = float(np.float32(fb / np.float32(dbox)))
        r["valid"] = 1
        r["reason"] = 0
    return res, blocks, total


def _median(v):
    m = len(v)
    if m % 2:
        return np.float32(v[(m - 1) // 2])
    return np.float32(np.float32(v[m // 2 - 1] + v[m // 2]) * np.float32(0.5))


def dense_volume(CL, CR, dmin, dmax, radius):
    """Full cost volume C[d, y, x] of the dense counterpart (tiny inputs only)."""
    H, W = CL.shape
    nd = dmax - dmin + 1
    vol = np.zeros((nd, H, W), dtype=np.int64)
    for k, d in enumerate(range(dmin, dmax + 1)):
        sh = np.zeros_like(CR)
        if d < W:
            sh[:, d:] = CR[:, : W - d]
        c = np.bitwise_count(CL ^ sh).astype(np.int64)
        pad = np.zeros((H + 2 * radius, W + 2 * radius), dtype=np.int64)
        pad[radius:radius + H, radius:radius + W] = c
        acc = np.zeros((H, W), dtype=np.int64)
        for v in range(2 * radius + 1):
            for u in range(2 * radius + 1):
                acc += pad[v:v + H, u:u + W]
        vol[k] = acc
    return vol


def dense(CL, CR, dmin, dmax, radius, lr_tol):
    vol = dense_volume(CL, CR, dmin, dmax, radius)
    nd, H, W = vol.shape
    dl = dmin + np.argmin(vol, axis=0)
    dr = np.full((H, W), -1, dtype=np.int64)
    for y in range(H):
        for xr in range(W):
            best, bc = -1, None
            for k in range(nd):
                xl = xr + dmin + k
                if 0 <= xl < W and (bc is None or vol[k, y, xl] < bc):
                    best, bc = dmin + k, vol[k, y, xl]
            dr[y, xr] = best
    out = np.full((H, W), -1, dtype=np.int16)
    for y in range(H):
        for x in range(W):
            d = dl[y, x]
            xr = x - d
            if xr >= 0 and dr[y, xr] >= 0 and abs(d - dr[y, xr]) <= lr_tol:
                out[y, x] = d
    return out, dr.astype(np.int16)
