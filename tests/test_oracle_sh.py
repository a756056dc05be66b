"""Pins of the spherical-harmonic colour oracle: the basis is orthonormal on
the sphere (a product Gauss-Legendre x trapezoid quadrature, exact for these
polynomial degrees), each degree-l function is a homogeneous harmonic of
degree l (Laplacian zero, checked by finite differences of its extension
r^l Y_lm), each function equals its definition from scipy's complex
harmonics (which carry the Condon-Shortley phase; this fixes every sign and
index the first two pins leave free), the colour of a degree-0 scene is
0.5 + k / (2 sqrt(pi)), and the view direction runs from the camera centre
-R^T t to the mean."""

import math

import numpy as np
import pytest

import oracle
import synth
from scipy.special import sph_harm_y


def _sphere_quadrature(n_theta=12, n_phi=24):
    u, wu = np.polynomial.legendre.leggauss(n_theta)  # u = cos(theta)
    phi = np.arange(n_phi) * (2 * math.pi / n_phi)
    U, PHI = np.meshgrid(u, phi, indexing="ij")
    s = np.sqrt(1 - U * U)
    d = np.stack([s * np.cos(PHI), s * np.sin(PHI), U], axis=-1).reshape(-1, 3)
    w = (wu[:, None] * np.full(n_phi, 2 * math.pi / n_phi)[None, :]).ravel()
    return d, w


def test_basis_is_orthonormal():
    d, w = _sphere_quadrature()
    B = oracle.sh_basis(d, 3)
    G = (B * w[:, None]).T @ B
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_solid_harmonics_are_harmonic():
    rng = np.random.default_rng(0)
    p = rng.standard_normal((20, 3))
    h = 1e-3
    degs = [0] + [1] * 3 + [2] * 5 + [3] * 7

    def solid(q):
        r = np.linalg.norm(q, axis=1, keepdims=True)
        B = oracle.sh_basis(q / r, 3)
        return B * r ** np.array(degs)[None, :]

    lap = np.zeros((20, 16))
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        lap += (solid(p + e) - 2 * solid(p) + solid(p - e)) / (h * h)
    np.testing.assert_allclose(lap, 0.0, atol=2e-4)


def test_degree_zero_colour():
    cam = synth.tiny_camera(32)
    mu = np.random.default_rng(1).uniform(-1, 1, (10, 3))
    sh = np.zeros((10, 16, 3))
    sh[:, 0, :] = [0.3, -2.0, 1.0]
    rgb = oracle.sh_to_rgb(mu, sh, cam, 0)
    want = np.maximum(0.5 + np.array([0.3, -2.0, 1.0]) / (2 * math.sqrt(math.pi)), 0.0)
    np.testing.assert_allclose(rgb, np.tile(want, (10, 1)), atol=1e-15)


def test_basis_matches_complex_harmonics():
    """Y_lm = sqrt(2) Re Y_l^m (m > 0), Y_l^0, sqrt(2) Im Y_l^|m| (m < 0) at
    random directions (theta polar from +z, phi azimuth from +x)."""
    rng = np.random.default_rng(3)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    B = oracle.sh_basis(d, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            want = Y.real if m == 0 else math.sqrt(2) * (Y.real if m > 0 else Y.imag)
            np.testing.assert_allclose(B[:, l * l + l + m], want, atol=1e-13, err_msg=str((l, m)))


def test_view_direction_from_camera_centre():
    """One degree-1 coefficient on Y_1,0 (the z harmonic): a mean straight
    above the camera centre (in world z) gets 0.5 + k sqrt(3 / (4 pi)) and one
    below it 0.5 - k sqrt(3 / (4 pi)); the camera is translated and rotated so
    that a wrong centre or a transposed rotation changes the result."""
    ang = 0.4
    R = np.array([[1, 0, 0], [0, math.cos(ang), -math.sin(ang)], [0, math.sin(ang), math.cos(ang)]])
    c = np.array([0.3, -0.2, 0.5])
    cam = synth.tiny_camera(32)
    cam.R_cw, cam.t = R, -R @ c
    mu = np.array([c + [0, 0, 2.0], c - [0, 0, 1.5], c + [1.0, 0, 0]])
    sh = np.zeros((3, 4, 3))
    sh[:, 2, :] = 0.25
    rgb = oracle.sh_to_rgb(mu, sh, cam, 1)
    k = 0.25 * math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(rgb[:, 0], [0.5 + k, 0.5 - k, 0.5], atol=1e-14)
