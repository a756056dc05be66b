"""Pins of the oracle's EWA projection (Sec. 3: Sigma = R S S^T R^T, EWA
splatting to a 2D Gaussian) against closed forms, finite differences and a
Monte-Carlo estimate that share nothing with its code."""

import math

import numpy as np
import pytest

import oracle
import synth
from oracle.project import covariance3d


def _cam(R=None, t=(0.0, 0.0, 3.0), f=100.0, W=200, H=160):
    R = np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32)
    return synth.Camera(R, np.asarray(t, np.float32), f, f * 1.1, W / 2, H / 2, W, H, 0.2)


def test_quaternion_about_z_is_textbook_rotation():
    th = 0.7
    q = np.array([[math.cos(th / 2), 0, 0, math.sin(th / 2)]])
    R = oracle.quat_to_rot(q)[0]
    want = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    np.testing.assert_allclose(R, want, atol=1e-15)


def test_quaternion_about_x_and_unnormalised_input():
    th = -1.1
    q = 3.0 * np.array([[math.cos(th / 2), math.sin(th / 2), 0, 0]])
    R = oracle.quat_to_rot(q)[0]
    want = np.array([[1, 0, 0], [0, math.cos(th), -math.sin(th)], [0, math.sin(th), math.cos(th)]])
    np.testing.assert_allclose(R, want, atol=1e-15)


def test_random_rotations_are_proper_orthonormal():
    q = np.random.default_rng(0).standard_normal((100, 4))
    R = oracle.quat_to_rot(q)
    np.testing.assert_allclose(R @ np.swapaxes(R, 1, 2), np.broadcast_to(np.eye(3), R.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)


def test_covariance_eigenvalues_are_squared_scales():
    rng = np.random.default_rng(1)
    s = rng.uniform(0.1, 2.0, (50, 3))
    q = rng.standard_normal((50, 4))
    S = covariance3d(s, q)
    ev = np.linalg.eigvalsh(S)
    np.testing.assert_allclose(np.sort(ev, 1), np.sort(s * s, 1), rtol=1e-12)


def test_on_axis_isotropic_closed_form():
    # Gaussian at the world origin, camera 3 units in front: z = 3, u = cx
    sig = 0.05
    cam = _cam(f=100.0)
    prm = oracle.RenderParams()
    pr = oracle.project(np.zeros((1, 3)), np.full((1, 3), sig), np.array([[0.3, 0.1, -0.5, 0.8]]),
                        np.array([0.9]), cam, prm)
    u, v = pr["means2d"][0]
    assert u == pytest.approx(cam.cx) and v == pytest.approx(cam.cy)
    sx = (cam.fx * sig / 3.0) ** 2 + prm.dilation
    sy = (cam.fy * sig / 3.0) ** 2 + prm.dilation
    a, b, c = pr["conic"][0]
    assert a == pytest.approx(1.0 / sx, rel=1e-12)
    assert c == pytest.approx(1.0 / sy, rel=1e-12)
    assert b == pytest.approx(0.0, abs=1e-15)
    assert pr["depth"][0] == pytest.approx(3.0)


@pytest.mark.parametrize("xz,yz", [(2.0, 0.5), (-0.4, -1.5), (1.2, 1.0), (0.3, -0.2)])
def test_guard_band_clamps_the_jacobian(xz, yz):
    """Isotropic Gaussian (s = 0.4) at camera-space x/z, y/z with R_cw = I and
    z = 3: Sigma2D = s^2 J J^T + dilation I, where J is formed with x/z and
    y/z clamped to guard x the half field of view of their own axis
    (1.3 x 100 / 100 = 1.3 horizontally, 1.3 x 80 / 110 = 0.945 vertically
    for this 200 x 160 camera with fx = 100, fy = 110). The cases clamp x
    only, y only (at the negative limit), y only where swapping the image
    sides (H for W) or the focal lengths would change which axis clamps, and
    neither."""
    cam = _cam(f=100.0)
    prm = oracle.RenderParams()
    z, s = 3.0, 0.4
    pr = oracle.project(np.array([[xz * z, yz * z, 0.0]]), np.full((1, 3), s), np.array([[1.0, 0.0, 0.0, 0.0]]),
                        np.array([0.9]), cam, prm)
    lim_x = 1.3 * (cam.width / 2) / cam.fx
    lim_y = 1.3 * (cam.height / 2) / cam.fy
    xh, yh = min(max(xz, -lim_x), lim_x), min(max(yz, -lim_y), lim_y)
    fx, fy = cam.fx, cam.fy
    sxx = s * s * (fx / z) ** 2 * (1.0 + xh * xh) + prm.dilation
    sxy = s * s * (fx * fy / (z * z)) * xh * yh
    syy = s * s * (fy / z) ** 2 * (1.0 + yh * yh) + prm.dilation
    np.testing.assert_allclose(pr["cov2d"][0], [sxx, sxy, syy], rtol=1e-10)
    det = sxx * syy - sxy * sxy
    np.testing.assert_allclose(pr["conic"][0], [syy / det, -sxy / det, sxx / det], rtol=1e-10)
    # the mean itself is projected without the clamp
    np.testing.assert_allclose(pr["means2d"][0], [fx * xz + cam.cx, fy * yz + cam.cy], rtol=1e-12)


def _pinhole(p, cam):
    return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])


def test_off_axis_covariance_matches_finite_difference_jacobian():
    rng = np.random.default_rng(2)
    yaw = 0.4
    R = np.array([[math.cos(yaw), 0, -math.sin(yaw)], [0, 1, 0], [math.sin(yaw), 0, math.cos(yaw)]])
    cam = _cam(R=R, t=(0.2, -0.1, 4.0))
    prm = oracle.RenderParams(dilation=0.0)
    mu = np.array([[0.5, 0.3, 0.2]])
    s = np.array([[0.05, 0.02, 0.09]])
    q = rng.standard_normal((1, 4))
    pr = oracle.project(mu, s, q, np.array([0.8]), cam, prm)
    R = np.asarray(cam.R_cw, np.float64)  # the camera stores float32
    pc = R @ mu[0] + np.array(cam.t, np.float64)
    h = 1e-6
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (_pinhole(pc + e, cam) - _pinhole(pc - e, cam)) / (2 * h)
    S_cam = R @ covariance3d(s, q)[0] @ R.T
    cov = J @ S_cam @ J.T
    got = pr["cov2d"][0]
    np.testing.assert_allclose(got, [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(pr["means2d"][0], _pinhole(pc, cam), rtol=1e-14)
    a, b, c = pr["conic"][0]
    np.testing.assert_allclose(np.array([[a, b], [b, c]]) @ cov, np.eye(2), atol=1e-9)


def test_ewa_matches_monte_carlo_projection():
    """Small Gaussians: the EWA 2D covariance is the covariance of projected
    samples (to first order in sigma/z)."""
    rng = np.random.default_rng(3)
    yaw, pitch = 0.5, -0.2
    cam = synth.look_camera((0.3, -2.5, 0.4), yaw + math.pi / 2, pitch, 320, 240, 300.0, 280.0, 160, 120)
    prm = oracle.RenderParams(dilation=0.0)
    mu = np.array([[0.4, 0.2, 0.1]])
    s = np.array([[0.01, 0.004, 0.007]])
    q = rng.standard_normal((1, 4))
    pr = oracle.project(mu, s, q, np.array([0.8]), cam, prm)
    X = rng.multivariate_normal(mu[0], covariance3d(s, q)[0], size=400_000)
    P = X @ np.asarray(cam.R_cw, np.float64).T + np.asarray(cam.t, np.float64)
    uv = np.stack([cam.fx * P[:, 0] / P[:, 2] + cam.cx, cam.fy * P[:, 1] / P[:, 2] + cam.cy], 1)
    C = np.cov(uv.T)
    sxx, sxy, syy = pr["cov2d"][0]
    scale = math.sqrt(sxx * syy)
    np.testing.assert_allclose([C[0, 0], C[1, 1]], [sxx, syy], rtol=0.015)
    assert abs(C[0, 1] - sxy) < 0.015 * scale


def test_culling_rules():
    cam = _cam()
    prm = oracle.RenderParams()
    mu = np.array([[0, 0, -2.85], [0, 0, 0], [0, 0, 0], [50.0, 0, 0]])
    s = np.full((4, 3), 0.05)
    q = np.tile([1.0, 0, 0, 0], (4, 1))
    o = np.array([0.9, 0.9, 0.5 / 255.0, 0.9])
    pr = oracle.project(mu, s, q, o, cam, prm)
    # behind the near plane, visible, too transparent, off screen
    assert pr["visible"].tolist() == [False, True, False, False]
    assert pr["tiles_touched"].tolist()[0] == 0 and pr["tiles_touched"].tolist()[2] == 0


def test_footprint_covers_every_pixel_on_the_ray_and_is_tight():
    """The tile rectangle holds every pixel whose alpha' >= alpha_min, and each
    of its edge tile rows/columns holds a pixel centre of the ellipse's box."""
    sc = synth.make_tiny(7, n=300)
    cam = synth.tiny_camera(96)
    prm = oracle.RenderParams()
    pr = oracle.project(sc.means, sc.scales, sc.quats, sc.opacity, cam, prm)
    ys, xs = np.mgrid[0:96, 0:96]
    checked = 0
    for g in np.nonzero(pr["visible"])[0]:
        u, v = pr["means2d"][g]
        a, b, c = pr["conic"][g]
        dx, dy = xs + 0.5 - u, ys + 0.5 - v
        alpha = np.minimum(prm.alpha_max, pr["opacity"][g] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)))
        on = alpha >= prm.alpha_min
        tx0, ty0, tx1, ty1 = pr["rect"][g]
        tiles_x = xs[on] // 16
        tiles_y = ys[on] // 16
        assert np.all((tiles_x >= tx0) & (tiles_x < tx1) & (tiles_y >= ty0) & (tiles_y < ty1))
        sxx, _, syy = pr["cov2d"][g]
        r2 = 2 * math.log(pr["opacity"][g] / prm.alpha_min)
        hx, hy = math.sqrt(r2 * sxx), math.sqrt(r2 * syy)
        inbox = (np.abs(xs + 0.5 - u) <= hx) & (np.abs(ys + 0.5 - v) <= hy)
        assert inbox.any()
        assert (xs[inbox] // 16).min() == tx0 and (xs[inbox] // 16).max() == tx1 - 1
        assert (ys[inbox] // 16).min() == ty0 and (ys[inbox] // 16).max() == ty1 - 1
        checked += 1
    assert checked > 200
