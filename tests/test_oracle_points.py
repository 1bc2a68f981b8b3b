"""Pins of the oracle's per-box 3D point and covariance (Sec. 4.3.6 Q-matrix equation,
Sec. 4.3.7 depth variance and covariance rotation) against facts fixed elsewhere:
Eq. 1's depth for the standard rectified Q, the pinhole back-projection, a rotation by a
right angle written out by hand, a finite-difference derivative of depth, and the
eigenvalues of a rotated diagonal covariance."""
import numpy as np
import pytest

F, B, CX, CY = 1800.0, 0.35, 950.0, 530.0


def _q(f=F, b=B, cx=CX, cy=CY, cx2=CX):
    # rectified pair, right camera at -b along x: W = (d - (cx - cx2)) / b
    return np.array([[1, 0, 0, -cx], [0, 1, 0, -cy], [0, 0, 0, f], [0, 0, 1 / b, -(cx - cx2) / b]])


def _geom(Q=None, R=None, t=(0, 0, 0), var_d=0.25, var_x=0.04, var_y=0.09, W=1920, H=1080):
    return dict(width=W, height=H, Q=_q() if Q is None else Q, R=np.eye(3) if R is None else R, t=t,
                focal_px=F, baseline_m=B, var_d=var_d, var_x=var_x, var_y=var_y)


def _results(orc, disp, valid=None):
    r = np.zeros(len(disp), dtype=orc.BOX_RESULT_DT)
    r["disparity"] = disp
    r["valid"] = 1 if valid is None else valid
    return r


def _boxes(rng, n, W=1920, H=1080):
    x0 = rng.integers(-40, W - 10, n)
    y0 = rng.integers(-40, H - 10, n)
    w = rng.integers(1, 400, n)
    h = rng.integers(1, 300, n)
    return np.stack([x0, y0, x0 + w, y0 + h, np.ones(n, int)], 1).astype(np.int32)


def test_depth_is_eq1_and_backprojection(orc):
    rng = np.random.default_rng(1)
    boxes = _boxes(rng, 200)
    d = rng.uniform(0.5, 190.0, 200).astype(np.float32)
    p = orc.box_points(boxes, _results(orc, d), _geom())
    assert p["valid"].all()
    Z = F * B / d.astype(np.float64)
    assert np.allclose(p["p_cam"][:, 2], Z, rtol=1e-12)
    cx0, cy0 = np.maximum(boxes[:, 0], 0), np.maximum(boxes[:, 1], 0)
    cx1, cy1 = np.minimum(boxes[:, 2], 1920), np.minimum(boxes[:, 3], 1080)
    u, v = (cx0 + cx1 - 1) / 2.0, (cy0 + cy1 - 1) / 2.0
    assert np.allclose(p["p_cam"][:, 0], (u - CX) * Z / F, rtol=1e-12, atol=1e-12)
    assert np.allclose(p["p_cam"][:, 1], (v - CY) * Z / F, rtol=1e-12, atol=1e-12)


def test_identity_and_right_angle_transforms(orc):
    rng = np.random.default_rng(2)
    boxes = _boxes(rng, 50)
    res = _results(orc, rng.uniform(1, 100, 50).astype(np.float32))
    p0 = orc.box_points(boxes, res, _geom())
    assert np.array_equal(p0["p_imu"], p0["p_cam"])
    # 90 degrees about z, then a shift: (x, y, z) -> (-y + 1, x - 2, z + 3)
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], float)
    p1 = orc.box_points(boxes, res, _geom(R=Rz, t=(1, -2, 3)))
    c = p1["p_cam"]
    want = np.stack([-c[:, 1] + 1, c[:, 0] - 2, c[:, 2] + 3], 1)
    assert np.allclose(p1["p_imu"], want, rtol=0, atol=1e-12)
    # the rotated diagonal swaps the lateral variances
    cov = p1["cov_imu"]
    assert np.allclose(cov[:, 0], 0.09) and np.allclose(cov[:, 3], 0.04)
    assert np.allclose(cov[:, 5], p1["var_z"]) and np.allclose(cov[:, [1, 2, 4]], 0)


def test_depth_variance_is_the_squared_derivative(orc):
    d = np.array([2.0, 7.5, 33.0, 150.0], np.float32)
    boxes = np.array([[500, 300, 540, 340, 1]] * 4, np.int32)
    p = orc.box_points(boxes, _results(orc, d), _geom(var_d=0.3))
    h = 1e-3
    zp = orc.box_points(boxes, _results(orc, d + np.float32(h)), _geom())["p_cam"][:, 2]
    zm = orc.box_points(boxes, _results(orc, d - np.float32(h)), _geom())["p_cam"][:, 2]
    dd = (d + np.float32(h)).astype(np.float64) - (d - np.float32(h)).astype(np.float64)
    dz = (zp - zm) / dd
    assert np.allclose(p["var_z"], dz * dz * 0.3, rtol=1e-5)


def test_rotated_covariance_keeps_its_eigenvalues(orc):
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 3))
    Rr, _ = np.linalg.qr(A)
    boxes = _boxes(rng, 20)
    res = _results(orc, rng.uniform(1, 100, 20).astype(np.float32))
    p = orc.box_points(boxes, res, _geom(R=Rr, var_x=0.02, var_y=0.5))
    for rec in p:
        xx, xy, xz, yy, yz, zz = rec["cov_imu"]
        S = np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])
        ev = np.sort(np.linalg.eigvalsh(S))
        assert np.allclose(ev, np.sort([0.02, 0.5, rec["var_z"]]), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("case", ["invalid_result", "clipped_empty", "w_zero"])
def test_points_that_do_not_exist(orc, case):
    boxes = np.array([[10, 10, 50, 50, 1]], np.int32)
    d, valid, Q = [12.0], [1], _q()
    if case == "invalid_result":
        valid = [0]
    elif case == "clipped_empty":
        boxes = np.array([[1920, 10, 1960, 50, 1]], np.int32)
    else:
        d = [0.0]
    p = orc.box_points(boxes, _results(orc, np.float32(d), valid), _geom(Q=Q))
    assert p["valid"][0] == 0
    assert not p["p_cam"].any() and not p["cov_imu"].any() and p["var_z"][0] == 0
