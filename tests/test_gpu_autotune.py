"""Every matching kernel variant, blocks-per-wave and grid setting gives the same
results (and the oracle's); the tuner picks among them and its table applies."""
import os

import numpy as np
import pytest
import torch

from paper_2604_07980_amd import autotune, synth
from test_gpu_parity import assert_results_match, _cuda

pytestmark = pytest.mark.gpu


def _workload(lib):
    p = synth.params_for(2)
    p["tau_s"] = 40
    scenes = [synth.scene_small(600 + k, H=200, W=320, n_planes=7) for k in range(4)]
    frames = [(_cuda(sc.left), _cuda(sc.right), len(sc.boxes)) for sc in scenes]
    boxes = _cuda(np.concatenate([sc.boxes for sc in scenes]).astype(np.int32))
    ws = lib.Workspace()
    out = torch.empty((boxes.shape[0], 8), dtype=torch.int32, device="cuda:0")

    def run():
        lib.range_batch(frames, boxes, p, workspace=ws, out=out)
        return out
    return p, scenes, run


def test_every_setting_same_results(lib, orc):
    p, scenes, run = _workload(lib)
    want = np.concatenate([orc.run_scene(sc.left, sc.right, p, sc.boxes)[1][0] for sc in scenes])
    try:
        for bw, bh, nd in autotune.path_shapes(p):
            for rows, cpl, passes in lib.variant_candidates(bw, bh, nd):
                lib.set_variant(bw, bh, nd, rows, cpl, passes)
                # one launch for both levels where a pair kernel is built, and one per level
                for bpw, mode in ((1, 0), (3, 0), (1, 1), (1, 2)):
                    lib.set_option(lib.OPTION_BLOCKS_PER_WAVE, bpw)
                    lib.set_option(lib.OPTION_LEVEL_LAUNCHES, mode)
                    assert_results_match(lib.results_to_numpy(run()), want)
                lib.set_option(lib.OPTION_LEVEL_LAUNCHES, 0)
                lib.set_variant(bw, bh, nd, 0, 0, 0)
        for g in (1, 4, 32):
            lib.set_option(lib.OPTION_MATCH_WGS_PER_CU, g)
            assert_results_match(lib.results_to_numpy(run()), want)
    finally:
        autotune.reset(p)


def test_tune_save_load_apply(lib, orc, tmp_path):
    p, scenes, run = _workload(lib)
    want = np.concatenate([orc.run_scene(sc.left, sc.right, p, sc.boxes)[1][0] for sc in scenes])
    try:
        table = autotune.tune(run, p, reps=3, warmup=1, blocks_per_wave=(1, 2),
                              match_wgs_per_cu=(8, 16))
        assert set(table.variants) == {autotune.shape_key(*s) for s in autotune.path_shapes(p)}
        path = os.path.join(tmp_path, "tune.json")
        autotune.save(table, path)
        autotune.reset(p)
        autotune.apply(autotune.load(path))
        assert_results_match(lib.results_to_numpy(run()), want)
    finally:
        autotune.reset(p)
