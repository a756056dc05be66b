"""Seeded synthetic Gaussian scenes and pinhole cameras.

The paper measures on pre-optimised 3DGS scenes of ScanNet rooms (640x480 and
1296x968 frames, fx = 577) with 512-D CLIP features; none of those are
available here, so these generators stand in for them with the same image
shapes, focal lengths and feature width, and room-like geometry (most
Gaussians lying on floor and wall planes, the rest scattered in the volume).

Everything here is random-number drawing (numpy PCG64 ``default_rng``) and
camera-pose construction. Gaussians are returned as float32 structure-of-arrays
columns: means [N,3], linear scales [N,3], quaternions [N,4] as (w, x, y, z),
activated opacity [N] and features [N, D].
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    A world point X maps to camera space as R_cw @ X + t. Pixel (px, py)
    covers [px, px+1) x [py, py+1); the principal point is (cx, cy).
    """

    R_cw: np.ndarray  # float32 [3, 3], row-major
    t: np.ndarray  # float32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.2


@dataclasses.dataclass
class Scene:
    means: np.ndarray  # float32 [N, 3]
    scales: np.ndarray  # float32 [N, 3], linear (not log)
    quats: np.ndarray  # float32 [N, 4], (w, x, y, z), not necessarily unit
    opacity: np.ndarray  # float32 [N], activated, in (0, 1)
    features: np.ndarray  # float32 [N, D]

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def dim(self) -> int:
        return int(self.features.shape[1])


def _sigmoid(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def look_camera(position, yaw: float, pitch: float, width: int, height: int,
                fx: float, fy: float, cx: float, cy: float,
                z_near: float = 0.2) -> Camera:
    """Camera at `position` (world, z up) looking along yaw/pitch, no roll."""
    c = np.asarray(position, dtype=np.float64)
    fwd = np.array([math.cos(pitch) * math.cos(yaw),
                    math.cos(pitch) * math.sin(yaw),
                    math.sin(pitch)])
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float64)
    t = -R @ c
    return Camera(R.astype(np.float32), t.astype(np.float32), float(fx), float(fy),
                  float(cx), float(cy), int(width), int(height), float(z_near))


# ----------------------------------------------------------------------------
# Tiny scene: 1,000 Gaussians in [-1,1]^3, 64x64 camera at distance 3.
# ----------------------------------------------------------------------------

def make_tiny(seed: int = 0, n: int = 1000, dim: int = 16) -> Scene:
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (n, 3)).astype(np.float32)
    log_s = rng.uniform(math.log(0.01), math.log(0.1), (n, 3))
    scales = np.exp(log_s).astype(np.float32)
    quats = _unit_quats(rng, n)
    opacity = _sigmoid(rng.standard_normal(n)).astype(np.float32)
    features = rng.standard_normal((n, dim), dtype=np.float32)
    return Scene(means, scales, quats, opacity, features)


def tiny_camera(size: int = 64, fov_deg: float = 60.0) -> Camera:
    f = (size / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    R = np.eye(3, dtype=np.float32)
    t = np.array([0.0, 0.0, 3.0], dtype=np.float32)  # camera centre (0,0,-3)
    return Camera(R, t, f, f, size / 2.0, size / 2.0, size, size, 0.2)


# ----------------------------------------------------------------------------
# Room scene: a 6 x 6 x 3 m box, 70% of Gaussians near floor/wall planes.
# ----------------------------------------------------------------------------

ROOM = (6.0, 6.0, 3.0)


def make_room(n: int, seed: int, dim: int = 512, normalise: bool = True,
              with_features: bool = True) -> Scene:
    rng = np.random.default_rng(seed)
    lx, ly, lz = ROOM
    n_plane = int(round(0.7 * n))
    n_free = n - n_plane
    # planes: floor (area 36) and four walls (18 each), chosen by area
    areas = np.array([lx * ly, ly * lz, ly * lz, lx * lz, lx * lz])
    plane = rng.choice(5, size=n_plane, p=areas / areas.sum())
    a = rng.uniform(0.0, 1.0, n_plane)
    b = rng.uniform(0.0, 1.0, n_plane)
    off = rng.uniform(0.0, 0.05, n_plane)
    pts = np.empty((n_plane, 3))
    # floor z = 0
    m = plane == 0
    pts[m] = np.stack([a[m] * lx, b[m] * ly, off[m]], 1)
    # wall x = 0 and x = lx
    m = plane == 1
    pts[m] = np.stack([off[m], a[m] * ly, b[m] * lz], 1)
    m = plane == 2
    pts[m] = np.stack([lx - off[m], a[m] * ly, b[m] * lz], 1)
    # wall y = 0 and y = ly
    m = plane == 3
    pts[m] = np.stack([a[m] * lx, off[m], b[m] * lz], 1)
    m = plane == 4
    pts[m] = np.stack([a[m] * lx, ly - off[m], b[m] * lz], 1)
    free = rng.uniform(0.0, 1.0, (n_free, 3)) * np.array(ROOM)
    means = np.concatenate([pts, free]).astype(np.float32)
    scales = np.exp(rng.uniform(math.log(0.005), math.log(0.05), (n, 3))).astype(np.float32)
    quats = _unit_quats(rng, n)
    opacity = _sigmoid(rng.normal(1.0, 1.5, n)).astype(np.float32)
    if with_features:
        feats = rng.standard_normal((n, dim), dtype=np.float32)
        if normalise:
            feats /= np.linalg.norm(feats, axis=1, keepdims=True)
    else:
        feats = np.zeros((n, 0), np.float32)
    return Scene(means, scales, quats, opacity, feats)


def room_camera(seed: int, width: int = 640, height: int = 480,
                fx: float = 577.0) -> Camera:
    rng = np.random.default_rng(seed)
    pos = np.array([rng.uniform(1, 5), rng.uniform(1, 5), rng.uniform(1, 2)])
    yaw = rng.uniform(0.0, 2 * math.pi)
    pitch = math.radians(rng.uniform(-15.0, 15.0))
    return look_camera(pos, yaw, pitch, width, height, fx, fx, width / 2.0, height / 2.0)


def room_poses(seeds, width: int = 640, height: int = 480, fx: float = 577.0):
    return [room_camera(s, width, height, fx) for s in seeds]


# ----------------------------------------------------------------------------
# Finite-difference sub-case: 2,000 tiny-generator Gaussians, 32x32, 512-D.
# ----------------------------------------------------------------------------

def make_fd_case(seed: int = 5, n: int = 2000, dim: int = 512, size: int = 32):
    scene = make_tiny(seed, n=n, dim=dim)
    return scene, tiny_camera(size)


# ----------------------------------------------------------------------------
# Batched form: several room scenes of uneven size, many views each.
# ----------------------------------------------------------------------------

def make_batched(sizes=(300_000, 800_000, 1_500_000, 3_000_000),
                 scene_seeds=(10, 11, 12, 13), views_per_scene: int = 8,
                 first_view_seed: int = 300, width: int = 1280, height: int = 720,
                 fx: float = 1154.0, dim: int = 512):
    scenes, cams, scene_of_view = [], [], []
    seed = first_view_seed
    for si, (n, s) in enumerate(zip(sizes, scene_seeds)):
        scenes.append(make_room(n, s, dim=dim))
        for _ in range(views_per_scene):
            cams.append(room_camera(seed, width, height, fx))
            scene_of_view.append(si)
            seed += 1
    return scenes, cams, scene_of_view


# Named workloads with their seeds and shapes.
CONFIGS = {
    "tiny": dict(n=1000, seed=0, dim=16, size=64, K=8),
    "room": dict(n=200_000, seed=1, dim=512, width=640, height=480, fx=577.0,
                 pose_seeds=list(range(100, 116)), K=8),
    "precision": dict(n=1_000_000, seed=2, dim=512, width=1296, height=968,
                      fx=577.0 * 1296 / 640, pose_seeds=list(range(200, 204)),
                      Ks=(4, 8, 16)),
    "diff": dict(n=500_000, seed=3, dim=512, width=640, height=480, fx=577.0,
                 pose_seeds=[400], target_seed=4, fd_seed=5, K=8),
}


def sh_coefficients(n: int, degree: int = 3, seed: int = 0) -> np.ndarray:
    """float32 [n, 16, 3] spherical-harmonic colour coefficients: the
    constant term uniform in [-1.4, 1.4] per channel (base colours spread
    over roughly [0.1, 0.9]), degree l >= 1 terms normal with standard
    deviation 0.3 / l, columns past (degree+1)^2 zero."""
    rng = np.random.default_rng(seed)
    k = np.zeros((n, 16, 3), np.float32)
    k[:, 0] = rng.uniform(-1.4, 1.4, (n, 3))
    for l in range(1, degree + 1):
        k[:, l * l:(l + 1) * (l + 1)] = rng.normal(0.0, 0.3 / l, (n, 2 * l + 1, 3))
    return k
