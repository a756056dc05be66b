"""EWA projection of 3D Gaussians to 2D conics and tile footprints (FP64).

Follows Sec. 3 of the paper (the 3D-GS preliminaries): each Gaussian has a
mean mu, a covariance Sigma = R S S^T R^T built from its scale s and rotation
quaternion r, and an opacity alpha; it is splatted with EWA to a 2D Gaussian
G(u) evaluated at pixel u. The paper defers the formulas to 3D-GS and EWA;
the reading taken here is their standard form:

* camera space p = R_cw mu + t (x right, y down, z forward); Gaussians with
  p_z <= z_near are culled;
* image-plane mean u = fx p_x / p_z + cx, v = fy p_y / p_z + cy, with pixel
  (px, py) sampled at its centre (px + 0.5, py + 0.5);
* Jacobian of the pinhole map J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]
  with x/z and y/z clamped to guard x the half field of view;
* Sigma_2D = J R_cw Sigma R_cw^T J^T + dilation I, conic = Sigma_2D^-1
  stored as (a, b, c) = (Syy, -Sxy, Sxx) / det; det <= 0 is culled.

Footprint (reading): a Gaussian belongs to a pixel's ray list exactly when
alpha' = min(alpha_max, o G) >= alpha_min, i.e. when the Mahalanobis form
q = d^T conic d satisfies q <= r^2 = 2 ln(o / alpha_min). Its footprint is the
bounding box of that ellipse, half-widths sqrt(r^2 Sxx) and sqrt(r^2 Syy),
clipped to the image and rounded out to 16 x 16 tiles (half-open rectangle).
Gaussians with o < alpha_min or an empty box are culled.
"""

from __future__ import annotations

import numpy as np

from .params import RenderParams


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [N,3,3] from quaternions (w, x, y, z), normalised."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def covariance3d(scales: np.ndarray, quats: np.ndarray) -> np.ndarray:
    """Sigma = R S S^T R^T with S = diag(s)."""
    R = quat_to_rot(quats)
    S = np.asarray(scales, dtype=np.float64)
    M = R * S[..., None, :]  # R @ diag(s)
    return M @ np.swapaxes(M, -1, -2)


def project(means, scales, quats, opacity, cam, params: RenderParams = RenderParams()):
    """Project N Gaussians; returns a dict of float64/int arrays.

    Keys: means2d [N,2], conic [N,3] (a, b, c), opacity [N], depth [N],
    cov2d [N,3] (Sxx, Sxy, Syy), rect [N,4] int (tx0, ty0, tx1, ty1),
    tiles_touched [N] int, visible [N] bool. Culled Gaussians have
    tiles_touched = 0 and rect = 0.
    """
    mu = np.asarray(means, dtype=np.float64)
    o = np.asarray(opacity, dtype=np.float64)
    n = mu.shape[0]
    Rcw = np.asarray(cam.R_cw, dtype=np.float64).reshape(3, 3)
    tcw = np.asarray(cam.t, dtype=np.float64).reshape(3)
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    W, H = int(cam.width), int(cam.height)
    tile = params.tile

    p = mu @ Rcw.T + tcw
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    in_front = z > cam.z_near
    zs = np.where(in_front, z, 1.0)

    u = fx * x / zs + cx
    v = fy * y / zs + cy

    lim_x = params.guard * (W / 2.0) / fx
    lim_y = params.guard * (H / 2.0) / fy
    tx = np.clip(x / zs, -lim_x, lim_x) * zs
    ty = np.clip(y / zs, -lim_y, lim_y) * zs
    J = np.zeros((n, 2, 3))
    J[:, 0, 0] = fx / zs
    J[:, 0, 2] = -fx * tx / (zs * zs)
    J[:, 1, 1] = fy / zs
    J[:, 1, 2] = -fy * ty / (zs * zs)

    Sigma = covariance3d(scales, quats)
    T = J @ Rcw  # [N,2,3]
    cov = T @ Sigma @ np.swapaxes(T, 1, 2)
    sxx = cov[:, 0, 0] + params.dilation
    sxy = cov[:, 0, 1]
    syy = cov[:, 1, 1] + params.dilation
    det = sxx * syy - sxy * sxy
    ok_det = det > 0
    dets = np.where(ok_det, det, 1.0)
    a = syy / dets
    b = -sxy / dets
    c = sxx / dets

    ok_o = o >= params.alpha_min
    r2 = 2.0 * np.log(np.where(ok_o, o, 1.0) / params.alpha_min)
    hx = np.sqrt(np.maximum(r2 * sxx, 0.0))
    hy = np.sqrt(np.maximum(r2 * syy, 0.0))

    visible = in_front & ok_det & ok_o
    px0 = np.full(n, 0, dtype=np.int64)
    px1 = np.full(n, -1, dtype=np.int64)
    py0 = np.full(n, 0, dtype=np.int64)
    py1 = np.full(n, -1, dtype=np.int64)
    vi = np.nonzero(visible)[0]
    # pixel centres px + 0.5 inside [u - hx, u + hx] (same along y)
    px0[vi] = np.maximum(np.ceil(u[vi] - hx[vi] - 0.5), 0).astype(np.int64)
    px1[vi] = np.minimum(np.floor(u[vi] + hx[vi] - 0.5), W - 1).astype(np.int64)
    py0[vi] = np.maximum(np.ceil(v[vi] - hy[vi] - 0.5), 0).astype(np.int64)
    py1[vi] = np.minimum(np.floor(v[vi] + hy[vi] - 0.5), H - 1).astype(np.int64)
    nonempty = (px1 >= px0) & (py1 >= py0)
    visible &= nonempty

    rect = np.zeros((n, 4), dtype=np.int64)
    rect[visible, 0] = px0[visible] // tile
    rect[visible, 1] = py0[visible] // tile
    rect[visible, 2] = px1[visible] // tile + 1
    rect[visible, 3] = py1[visible] // tile + 1
    touched = (rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1])

    return dict(
        means2d=np.stack([u, v], 1),
        conic=np.stack([a, b, c], 1),
        opacity=o.copy(),
        depth=z.copy(),
        cov2d=np.stack([sxx, sxy, syy], 1),
        rect=rect,
        tiles_touched=touched,
        visible=visible,
    )
