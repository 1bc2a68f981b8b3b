"""Census tiles of whole-frame and batch calls.

By default a call makes the descriptors of only those 64 x 32 tiles that some ranged
box's search reads (the rule stated with ocsr_range_frame in the C header, restated on
the host by paper_2604_07980_amd.accounting). These tests fill the workspace with a
byte pattern first, so a tile the kernels left alone still holds the pattern, and check:
* the set of tiles made is exactly the rule's;
* every tile made holds the oracle's census;
* the box results equal the oracle's, so no search read a tile that was not made;
* with OCSR_OPTION_FULL_CENSUS every tile is made.
"""
import numpy as np
import pytest
import torch

from paper_2604_07980_amd import accounting, synth
from test_gpu_parity import assert_results_match, _cuda, _params

pytestmark = pytest.mark.gpu

PATTERN = 0xA5
TX, TY = accounting.TILE_X, accounting.TILE_Y


def _a256(v):
    return (v + 255) // 256 * 256


def _ws_levels(buf, shapes, s):
    """The descriptor images at the start of a workspace: per frame L0, R0, L1, R1."""
    out, off = [], 0
    for H, W in shapes:
        imgs = []
        for h, w in ((H, W), (H, W), (H // s, W // s), (H // s, W // s)):
            n = h * w * 8
            imgs.append(buf[off:off + n].cpu().numpy().view(np.uint64).reshape(h, w))
            off += _a256(n)
        out.append(imgs)
    return out


def _tiles_made(imgs):
    pat = np.uint64(int.from_bytes(bytes([PATTERN]) * 8, "little"))
    made = set()
    for k, img in enumerate(imgs):
        level, view = k // 2, k % 2
        h, w = img.shape
        for ty in range(-(-h // TY)):
            for tx in range(-(-w // TX)):
                t = img[ty * TY:(ty + 1) * TY, tx * TX:(tx + 1) * TX]
                if not (t == pat).all():
                    made.add((level, view, tx, ty))
    return made


def _check_tiles(orc, imgs, made, left, right, p):
    s = p["close_scale"]
    for k, img in enumerate(imgs):
        level, view = k // 2, k % 2
        want = orc.census(right if view else left, p["sx"], p["sy"], s if level else 1, p["sentinel"])
        for lv, vw, tx, ty in made:
            if (lv, vw) != (level, view):
                continue
            sl = (slice(ty * TY, (ty + 1) * TY), slice(tx * TX, (tx + 1) * TX))
            assert (img[sl] == want[sl]).all(), (level, view, tx, ty)


def _edge_boxes(H, W, tau):
    """Boxes at the four image edges, one of each type, plus an occluder."""
    big, small = max(tau + 8, 40), max(tau // 2, 10)
    return np.array([
        [0, 10, big, 10 + big, 1],                      # close, at the left edge
        [W - small, 5, W, 5 + small, 1],                # far, at the right edge
        [W // 2, H - small, W // 2 + small, H, 1],      # far, at the bottom
        [-20, -20, 12, 12, 1],                          # far, clipped at the corner
        [W // 3, H // 3, W // 3 + big, H // 3 + big, 0],  # occluder only
        [W - big, H - big, W + 7, H + 9, 1],            # close, past the corner
    ], np.int32)


def _frame(lib, orc, left, right, boxes, p, full=False, listed=True):
    H, W = left.shape
    ws = lib.Workspace()
    # a one-frame batch workspace has the whole-frame layout and size
    nbytes = lib.batch_workspace_bytes([(H, W, boxes.shape[0])], p, lib.DEFAULT_CAP_BLOCKS)
    buf = ws.get(nbytes, torch.device("cuda:0"))
    buf.fill_(PATTERN)
    lib.set_option(lib.OPTION_FULL_CENSUS, 1 if full else 0)
    lib.set_option(lib.OPTION_CENSUS_TILE_LIST, 1 if listed else 0)
    try:
        got = lib.results_to_numpy(lib.range_frame(_cuda(left), _cuda(right), _cuda(boxes), p,
                                                   workspace=ws))
    finally:
        lib.set_option(lib.OPTION_FULL_CENSUS, 0)
        lib.set_option(lib.OPTION_CENSUS_TILE_LIST, 1)
    torch.cuda.synchronize()
    want = orc.run_scene(left, right, p, boxes)[1][0]
    assert_results_match(got, want)
    imgs = _ws_levels(buf, [(H, W)], p["close_scale"])[0]
    made = _tiles_made(imgs)
    assert made == accounting.census_tiles(W, H, boxes, p, full=full)
    _check_tiles(orc, imgs, made, left, right, p)
    return made


@pytest.mark.parametrize("listed", [True, False], ids=["list_allowed", "per_tile"])
@pytest.mark.parametrize("variant", ["tiled_trim", "tiled_seg_lr0", "win5x5"])
@pytest.mark.parametrize("seed", [1, 2])
def test_frame_makes_the_tiles_boxes_read(lib, orc, variant, seed, listed):
    p = _params(variant)
    sc = synth.scene_small(500 + 10 * seed + len(variant), H=200, W=360, n_planes=6)
    made = _frame(lib, orc, sc.left, sc.right, sc.boxes, p, listed=listed)
    assert made, "the scene's boxes read some tile"


@pytest.mark.parametrize("listed", [True, False], ids=["listed", "per_tile"])
@pytest.mark.parametrize("dy,scale", [((-3, 2), 2), ((1, 4), 2), ((-5, 4), 3)])
def test_frame_tiles_with_vertical_range(lib, orc, dy, scale, listed):
    """A vertical range widens the rows the searches read: the tiles made follow the
    widened rule, edge boxes included, and the results still equal the oracle's."""
    p = _params("tiled_trim")
    p["dy_min"], p["dy_max"] = dy
    p["close_scale"] = scale
    sc = synth.scene_small(830 + dy[0], H=160, W=300, n_planes=4)
    boxes = np.concatenate([sc.boxes.reshape(-1, 5), _edge_boxes(160, 300, p["tau_s"])]).astype(np.int32)
    right = synth.drift_rows(sc.right, dy[0])
    _frame(lib, orc, sc.left, right, boxes, p, listed=listed)


@pytest.mark.parametrize("listed", [True, False], ids=["listed", "per_tile"])
@pytest.mark.parametrize("variant", ["tiled_trim", "wide_range"])
def test_frame_tiles_at_image_edges(lib, orc, variant, listed):
    p = _params(variant)
    sc = synth.scene_small(811, H=160, W=300, n_planes=3)
    boxes = _edge_boxes(160, 300, p["tau_s"])
    _frame(lib, orc, sc.left, sc.right, boxes, p, listed=listed)


def test_frame_without_ranged_boxes_makes_no_tile(lib, orc):
    p = _params("tiled_trim")
    sc = synth.scene_small(812, H=128, W=192, n_planes=3)
    boxes = sc.boxes.copy()
    boxes[:, 4] = 0
    assert _frame(lib, orc, sc.left, sc.right, boxes, p) == set()


@pytest.mark.parametrize("listed", [True, False], ids=["listed", "per_tile"])
def test_full_census_option_makes_every_tile(lib, orc, listed):
    p = _params("tiled_trim")
    sc = synth.scene_small(813, H=150, W=260, n_planes=4)
    _frame(lib, orc, sc.left, sc.right, sc.boxes, p, full=True, listed=listed)


@pytest.mark.parametrize("listed", [True, False], ids=["listed", "per_tile"])
def test_realistic_frame_tiles(lib, orc, listed):
    """The 1920x1080 frame the benchmark times: about a fifth of the tiles are made (2550
    tiles, more than the persistent grid, so the listed form shares them out)."""
    p = synth.params_for(2)
    sc = synth.scene_realistic()
    made = _frame(lib, orc, sc.left, sc.right, sc.boxes, p, listed=listed)
    H, W = sc.left.shape
    n_all = len(accounting.census_tiles(W, H, sc.boxes, p, full=True))
    assert 0 < len(made) < n_all


@pytest.mark.parametrize("large", [False, True], ids=["small_per_tile", "large_listed"])
@pytest.mark.parametrize("listed", [True, False], ids=["list_allowed", "per_tile"])
def test_batch_makes_each_frames_tiles(lib, orc, large, listed):
    """Small frames take the per-tile launch; four 1920x1200 frames (11400 tiles, at
    least 8 per resident workgroup) the persistent workgroups over tile lists, unless
    lists are switched off."""
    p = synth.params_for(3)
    if large:
        scenes = [synth.scene_batch_frame(f) for f in range(4)]
    else:
        scenes = [synth.scene_small(900 + k, H=h, W=w, n_planes=5)
                  for k, (h, w) in enumerate([(160, 256), (120, 200), (200, 330)])]
    lib.set_option(lib.OPTION_CENSUS_TILE_LIST, 1 if listed else 0)
    try:
        _batch_tiles(lib, orc, p, scenes)
    finally:
        lib.set_option(lib.OPTION_CENSUS_TILE_LIST, 1)


def _batch_tiles(lib, orc, p, scenes):
    frames = [(_cuda(s.left), _cuda(s.right), s.boxes.shape[0]) for s in scenes]
    boxes = _cuda(np.concatenate([s.boxes for s in scenes]))
    ws = lib.Workspace()
    shapes = [(s.left.shape[0], s.left.shape[1], s.boxes.shape[0]) for s in scenes]
    buf = ws.get(lib.batch_workspace_bytes(shapes, p), torch.device("cuda:0"))
    buf.fill_(PATTERN)
    got = lib.results_to_numpy(lib.range_batch(frames, boxes, p, workspace=ws))
    torch.cuda.synchronize()
    per = _ws_levels(buf, [sh[:2] for sh in shapes], p["close_scale"])
    off = 0
    for s, imgs in zip(scenes, per):
        n = s.boxes.shape[0]
        assert_results_match(got[off:off + n], orc.run_scene(s.left, s.right, p, s.boxes)[1][0])
        off += n
        H, W = s.left.shape
        made = _tiles_made(imgs)
        assert made == accounting.census_tiles(W, H, s.boxes, p)
        _check_tiles(orc, imgs, made, s.left, s.right, p)
