"""Batched ranging (many frames, uneven box counts, one launch sequence): identical to
one call per frame, and to the CPU oracle."""
import numpy as np
import pytest
import torch

from paper_2604_07980_amd import synth
from test_gpu_parity import assert_results_match, lib_options, _cuda

pytestmark = pytest.mark.gpu


def _batch_inputs(scenes):
    frames = [(_cuda(sc.left), _cuda(sc.right), len(sc.boxes)) for sc in scenes]
    boxes = _cuda(np.concatenate([sc.boxes.reshape(-1, 5) for sc in scenes]).astype(np.int32))
    return frames, boxes


def _oracle(orc, scenes, p):
    return np.concatenate([orc.run_scene(sc.left, sc.right, p, sc.boxes)[1][0] for sc in scenes])


def _small_batch(n, H=160, W=224, seed=0):
    rng = np.random.default_rng(seed)
    scenes = []
    for k in range(n):
        scenes.append(synth.scene_small(500 + 17 * seed + k, H=H, W=W,
                                        n_planes=int(rng.integers(0, 9))))
    return scenes


@pytest.mark.parametrize("fused", [True, False])
def test_batch_equals_per_frame_and_oracle(lib, orc, fused):
    p = synth.base_params()
    p["tau_s"] = 40
    p["far"].update(dmax=15)
    p["close"].update(dmax=63)
    scenes = _small_batch(7, seed=1)
    frames, boxes = _batch_inputs(scenes)
    with lib_options(lib, fused=fused):
        got = lib.results_to_numpy(lib.range_batch(frames, boxes, p))
        per = np.concatenate([lib.results_to_numpy(
            lib.range_frame(f[0], f[1], _cuda(sc.boxes.reshape(-1, 5).astype(np.int32)), p))
            for f, sc in zip(frames, scenes) if len(sc.boxes)] or [np.zeros(0, got.dtype)])
    assert (got.view(np.int32) == per.view(np.int32)).all()
    assert_results_match(got, _oracle(orc, scenes, p))


def test_batch_mixed_resolutions(lib, orc):
    p = synth.params_for(2)
    scenes = [synth.scene_small(900, H=180, W=320, n_planes=5),
              synth.scene_small(901, H=96, W=128, n_planes=2),
              synth.scene_small(902, H=240, W=300, n_planes=8),
              synth.scene_small(903, H=64, W=64, n_planes=0)]
    frames, boxes = _batch_inputs(scenes)
    for fused in (True, False):
        with lib_options(lib, fused=fused):
            got = lib.results_to_numpy(lib.range_batch(frames, boxes, p))
        assert_results_match(got, _oracle(orc, scenes, p))


def test_batch_config3_16_frames(lib, orc):
    """The batching workload: 16 frames of 1920x1200, Poisson(40) boxes of 12..512 px."""
    p = synth.params_for(3)
    scenes = [synth.scene_batch_frame(f) for f in range(16)]
    frames, boxes = _batch_inputs(scenes)
    want = _oracle(orc, scenes, p)
    got = lib.results_to_numpy(lib.range_batch(frames, boxes, p))
    assert_results_match(got, want)
    # the persistent kernel is built for single-pass close variants
    lib.set_variant(8, 8, 96, 8, 12, 1)
    try:
        with lib_options(lib, fused=True):
            got2 = lib.results_to_numpy(lib.range_batch(frames, boxes, p))
    finally:
        lib.set_variant(8, 8, 96, 0, 0, 0)
    assert (got.view(np.int32) == got2.view(np.int32)).all()
    assert got["valid"].sum() > 0.5 * len(got)


def test_batch_validation(lib):
    p = synth.params_for(2)
    L = torch.zeros((64, 64), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(ValueError):
        lib.range_batch([(L, L, 1)] * 17, torch.zeros((17, 5), dtype=torch.int32, device="cuda:0"), p)
    with pytest.raises(ValueError):
        lib.range_batch([(L, L, 2)], torch.zeros((1, 5), dtype=torch.int32, device="cuda:0"), p)
