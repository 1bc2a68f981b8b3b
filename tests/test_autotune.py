"""Host-side logic of the autotuner and the kernel-variant query: path shapes, table
persistence and validation. No GPU."""
import os

import pytest

from paper_2604_07980_amd import autotune, ocsr, synth


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(ocsr.LIB_PATH):
        from paper_2604_07980_amd import build
        build.build()
    return ocsr.load()


def test_path_shapes_of_the_workloads():
    # realistic frame: far 4x4 blocks over 0..31 at s=1, close 8x8 over 0..191 at s=2
    assert autotune.path_shapes(synth.params_for(2)) == [(4, 4, 32), (8, 8, 96)]
    # tiny frame: far 8x8 over 0..63; the close path is configured the same as the base
    shapes = autotune.path_shapes(synth.params_for(1))
    assert shapes[0] == (8, 8, 64)


def test_variant_candidates_cover_the_shape(built):
    for bw, bh, nd in [(4, 4, 32), (8, 8, 96), (8, 8, 64), (8, 8, 128), (5, 5, 40), (4, 4, 1)]:
        cands = ocsr.variant_candidates(bw, bh, nd)
        assert cands, (bw, bh, nd)
        for rows, cpl, passes in cands:
            if rows == 0:      # the generic kernel: any block of up to 64 points
                assert bw * bh <= 64 and 64 * cpl >= nd and passes == 1
            elif rows == 1:    # four blocks of up to 4 x 4 per wave, 16 candidate groups
                assert bw <= 4 and bh <= 4 and 16 * cpl >= nd and passes == 1
            elif rows == 2:    # two row halves of an up to 8 x 8 block, 32 candidate groups
                assert bw <= 8 and bh <= 8 and 32 * cpl >= nd and passes == 1
            else:
                assert rows in (4, 8) and bh <= rows and bw <= rows
                assert (64 // rows) * cpl * passes >= nd
    # blocks wider than 8 (up to 64 points) run only in the generic kernel; nothing
    # covers more than 256 candidates
    assert ocsr.variant_candidates(16, 4, 32) == [(0, 4, 1)]
    assert ocsr.variant_candidates(9, 8, 32) == []
    assert ocsr.variant_candidates(8, 8, 257) == []
    # 4x4 blocks can also run in the 8-row kernels
    assert (8, 4, 1) in ocsr.variant_candidates(4, 4, 32)
    # fewer candidates per lane in several passes
    assert (8, 4, 3) in ocsr.variant_candidates(8, 8, 96)
    # the defaults: four 4x4 blocks per wave, row halves for 8x8 blocks
    assert ocsr.variant_candidates(4, 4, 32)[0] == (1, 2, 1)
    assert ocsr.variant_candidates(8, 8, 96)[0] == (2, 3, 1)
    assert ocsr.variant_candidates(8, 8, 128)[0] == (2, 4, 1)


def test_table_round_trip(built):
    t = autotune.Table(arch="gfx950", variants={"4x4/32": [4, 2, 1], "8x8/96": [8, 4, 3]},
                       blocks_per_wave=2, match_wgs_per_cu=8, level_launches=2, timings_ms={"a": 1.5})
    back = autotune.from_json(autotune.to_json(t))
    assert back == t


@pytest.mark.parametrize("bad", [
    '{"arch": "gfx950", "variants": {"8x8/96": [8, 8, 1]}, "blocks_per_wave": 1, "match_wgs_per_cu": 16}',
    '{"arch": "gfx950", "variants": {"8x8/96": [4, 16, 1]}, "blocks_per_wave": 1, "match_wgs_per_cu": 16}',
    '{"arch": "gfx950", "variants": {"8x8/96": [8, 12]}, "blocks_per_wave": 1, "match_wgs_per_cu": 16}',
    '{"arch": "gfx950", "variants": {}, "blocks_per_wave": 9, "match_wgs_per_cu": 16}',
    '{"arch": "gfx950", "variants": {}, "blocks_per_wave": 1, "match_wgs_per_cu": 0}',
    '{"arch": "gfx950", "variants": {}, "blocks_per_wave": 1, "match_wgs_per_cu": 16, "level_launches": 3}',
])
def test_invalid_tables_rejected(built, bad):
    with pytest.raises(ValueError):
        autotune.from_json(bad)


def test_tune_keeps_the_current_setting_within_the_margin(monkeypatch):
    """The search over a simulated library: a setting replaces the current one only when
    it is faster by more than the margin, so noise-level differences keep the defaults."""
    state = {"variant": {}, "opts": {}}
    cands = {(4, 4, 32): [(1, 2, 1), (1, 4, 1)], (8, 8, 96): [(2, 3, 1), (2, 4, 1), (8, 12, 1)]}
    monkeypatch.setattr(autotune.ocsr, "variant_candidates", lambda bw, bh, nd, device=None: cands[(bw, bh, nd)])
    monkeypatch.setattr(autotune.ocsr, "set_variant",
                        lambda bw, bh, nd, r, c, p, device=None: state["variant"].__setitem__((bw, bh, nd), (r, c, p)))
    monkeypatch.setattr(autotune.ocsr, "set_option",
                        lambda o, v, device=None: state["opts"].__setitem__(o, v))
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")
    monkeypatch.setattr(autotune, "path_shapes", lambda params: [(4, 4, 32), (8, 8, 96)])
    monkeypatch.setattr(autotune, "_snapshot", lambda r: r)

    import numpy as np

    def run():
        return np.zeros(4)

    def cost():
        v = state["variant"]
        o = state["opts"]
        ms = 1.0
        ms -= 0.005 if v.get((4, 4, 32)) == (1, 4, 1) else 0.0     # within the margin: kept out
        ms -= 0.10 if v.get((8, 8, 96)) == (8, 12, 1) else 0.0     # a clear win: taken
        ms -= 0.05 if o.get(ocsr.OPTION_BLOCKS_PER_WAVE) == 4 else 0.0
        ms -= 0.004 if o.get(ocsr.OPTION_LEVEL_LAUNCHES) == 2 else 0.0
        return ms

    monkeypatch.setattr(autotune, "_time_ms", lambda run, reps, warmup: cost())
    table = autotune.tune(run, {}, reps=1, warmup=0)
    assert table.variants == {"4x4/32": [1, 2, 1], "8x8/96": [8, 12, 1]}
    assert table.blocks_per_wave == 4
    assert table.match_wgs_per_cu == autotune.DEFAULT_MATCH_WGS_PER_CU
    assert table.level_launches == 0
    # the installed configuration is the table's
    assert state["variant"][(8, 8, 96)] == (8, 12, 1) and state["opts"][ocsr.OPTION_LEVEL_LAUNCHES] == 0
    # with no margin the small gains are taken too
    table0 = autotune.tune(run, {}, reps=1, warmup=0, margin=0.0)
    assert table0.variants["4x4/32"] == [1, 4, 1] and table0.level_launches == 2
