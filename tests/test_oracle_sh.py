"""Pins of the spherical-harmonic colour oracle: the basis is orthonormal on
the sphere (a product Gauss-Legendre x trapezoid quadrature, exact for these
polynomial degrees), each degree-l function is a homogeneous harmonic of
degree l (Laplacian zero, checked by finite differences of its extension
r^l Y_lm), and the colour of a degree-0 scene is 0.5 + k / (2 sqrt(pi))."""

import math

import numpy as np
import pytest

import oracle
import synth


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
