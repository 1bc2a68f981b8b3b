"""Dense counterpart (every pixel, every disparity, clipped (2r+1)^2 Hamming sums,
winner-take-all both ways, left/right check) through the C ABI against the oracle:
bit-exact on small images spanning several strips and bands with ragged tails, and on
sampled pixels of the full 1920x1080 frame with 192 disparities."""
import numpy as np
import pytest
import torch

from paper_2604_07980_amd import synth
from test_gpu_parity import _cuda

pytestmark = pytest.mark.gpu


def _desc(orc, sc):
    return orc.census(sc.left), orc.census(sc.right)


def _gpu(a):
    return _cuda(a.view(np.int64))


CASES = [  # (H, W, dmin, dmax, radius)
    (37, 150, 0, 23, 2),
    (70, 131, 3, 40, 2),
    (45, 260, 0, 191, 2),
    (33, 97, 0, 15, 1),
    (29, 140, 5, 60, 3),
    (20, 70, 0, 255, 2),     # range wider than the image
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_d{c[2]}-{c[3]}_r{c[4]}" for c in CASES])
def test_dense_parity_small(lib, orc, case):
    H, W, dmin, dmax, r = case
    sc = synth.scene_small(4000 + H + W, H=H, W=W, n_planes=3)
    CL, CR = _desc(orc, sc)
    want, want_r = orc.dense(CL, CR, dmin, dmax, r, 1)
    got, got_r = lib.dense(_gpu(CL), _gpu(CR), dmin, dmax, r, 1, right=True)
    got_r = got_r.cpu().numpy()
    assert (got_r == want_r).all(), np.argwhere(got_r != want_r)[:10]
    got = got.cpu().numpy()
    assert (got == want).all(), np.argwhere(got != want)[:10]


def test_dense_lr_tolerance_zero(lib, orc):
    sc = synth.scene_small(4100, H=40, W=120, n_planes=4)
    CL, CR = _desc(orc, sc)
    want, _ = orc.dense(CL, CR, 0, 31, 2, 0)
    got = lib.dense(_gpu(CL), _gpu(CR), 0, 31, 2, 0).cpu().numpy()
    assert (got == want).all()


def test_dense_random_words(lib, orc):
    """Uniform random descriptors: many exact cost ties, which the smallest-d rule breaks."""
    rng = np.random.default_rng(5)
    H, W = 26, 90
    CL = rng.integers(0, 1 << 63, size=(H, W), dtype=np.int64).astype(np.uint64)
    CR = rng.integers(0, 1 << 63, size=(H, W), dtype=np.int64).astype(np.uint64)
    CL[:, :7] = 0                      # runs of equal words
    CR[:, 40:50] = CR[:, 30:40]
    want, want_r = orc.dense(CL, CR, 0, 47, 2, 1)
    got, got_r = lib.dense(_gpu(CL), _gpu(CR), 0, 47, 2, 1, right=True)
    assert (got_r.cpu().numpy() == want_r).all()
    assert (got.cpu().numpy() == want).all()


def test_dense_config4_sampled(lib, orc):
    """The dense workload at full size: the realistic 1920x1080 pair, d = 0..191, 5x5."""
    sc = synth.scene_realistic()
    L = _cuda(sc.left)
    R = _cuda(sc.right)
    CL, CR = lib.census_many([L, R], [1, 1])
    got = lib.dense(CL, CR, 0, 191, 2, 1).cpu().numpy()
    CLh = CL.cpu().numpy().view(np.uint64)
    CRh = CR.cpu().numpy().view(np.uint64)
    H, W = sc.left.shape
    rng = np.random.default_rng(9)
    xs = np.concatenate([rng.integers(0, W, 1500), [0, 1, 2, W - 1, W - 2, 191, 192, 57, 1000]])
    ys = np.concatenate([rng.integers(0, H, 1500), [0, H - 1, 1, H - 2, 540, 3, H - 3, 0, 16]])
    xy = np.stack([xs, ys], axis=1).astype(np.int32)
    want = orc.dense_at(CLh, CRh, xy, 0, 191, 2, 1)
    assert (got[ys, xs] == want).all()
    assert (got >= 0).mean() > 0.5        # most pixels pass the check on this texture


def test_dense_rejects(lib):
    z = torch.zeros((8, 8), dtype=torch.int64, device="cuda:0")
    with pytest.raises(lib.OcsrError):
        lib.dense(z, z, 0, 10, 4, 1)      # radius not built
    with pytest.raises(lib.OcsrError):
        lib.dense(z, z, 5, 4, 2, 1)       # empty range
    with pytest.raises(lib.OcsrError):
        lib.dense(z, z, 0, 300, 2, 1)     # more than 256 candidates
