"""View-dependent RGB from spherical-harmonic coefficients (the colour model
of the 3D-GS scenes the paper renders with Q-Render in its RGB experiment,
Appendix "Rendering RGB"), FP64. TEST INFRASTRUCTURE ONLY.

Per Gaussian and view: d = (mu - c) / |mu - c| with c the camera centre
(c = -R_cw^T t); colour_ch = sum_{l <= L, |m| <= l} k[l, m, ch] Y_lm(d) + 1/2,
clipped below at 0 (the 3D-GS convention), with Y_lm the real, orthonormal
spherical harmonics of degree L <= 3 in the order m = -l .. l that carry the
Condon-Shortley phase (-1)^m, the sign convention of 3D-GS's coefficients:
Y_lm = sqrt(2) Re Y_l^m for m > 0, Y_l^0 for m = 0 and sqrt(2) Im Y_l^|m| for
m < 0, Y_l^m the complex harmonics with that phase. Written out below as the
standard real forms (Y_00 = 1 / (2 sqrt(pi)), Y_1,(-1,0,1) = sqrt(3 / (4 pi))
(y, z, x), ...) times (-1)^m. Coefficients are indexed l^2 + l + m. A mean at
the camera centre takes d = 0.
"""

from __future__ import annotations

import math

import numpy as np


def sh_basis(d, degree: int) -> np.ndarray:
    """[n, (degree+1)^2] real orthonormal spherical harmonics at unit vectors d [n, 3]."""
    d = np.asarray(d, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    cols = [np.full_like(x, 0.5 / math.sqrt(pi))]
    if degree >= 1:
        k = math.sqrt(3.0 / (4.0 * pi))
        cols += [k * y, k * z, k * x]
    if degree >= 2:
        cols += [0.5 * math.sqrt(15.0 / pi) * x * y,
                 0.5 * math.sqrt(15.0 / pi) * y * z,
                 0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0),
                 0.5 * math.sqrt(15.0 / pi) * x * z,
                 0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)]
    if degree >= 3:
        cols += [0.25 * math.sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y),
                 0.5 * math.sqrt(105.0 / pi) * x * y * z,
                 0.25 * math.sqrt(21.0 / (2.0 * pi)) * y * (5.0 * z * z - 1.0),
                 0.25 * math.sqrt(7.0 / pi) * (5.0 * z ** 3 - 3.0 * z),
                 0.25 * math.sqrt(21.0 / (2.0 * pi)) * x * (5.0 * z * z - 1.0),
                 0.25 * math.sqrt(105.0 / pi) * z * (x * x - y * y),
                 0.25 * math.sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y)]
    B = np.stack(cols, axis=1)
    # Condon-Shortley phase: (-1)^m on the column of order m
    m = np.concatenate([np.arange(-l, l + 1) for l in range(degree + 1)])
    return B * np.where(m % 2 == 0, 1.0, -1.0)


def sh_to_rgb(means3d, sh, camera, degree: int) -> np.ndarray:
    """[n, 3] colours of Gaussians with coefficients sh [n, (degree+1)^2, 3]
    seen from `camera` (R_cw, t as in the projection)."""
    R = np.asarray(camera.R_cw, np.float64).reshape(3, 3)
    t = np.asarray(camera.t, np.float64)
    c = -R.T @ t
    d = np.asarray(means3d, np.float64) - c
    r = np.linalg.norm(d, axis=1, keepdims=True)
    d = np.divide(d, r, out=np.zeros_like(d), where=r > 0)
    B = sh_basis(d, degree)
    rgb = np.einsum("nk,nkc->nc", B, np.asarray(sh, np.float64)[:, : B.shape[1]]) + 0.5
    return np.maximum(rgb, 0.0)
