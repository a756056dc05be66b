"""Brute-force per-pixel rendering over every Gaussian of the scene (no tiles).

For one pixel: evaluate alpha' of every visible Gaussian, keep those with
alpha' >= alpha_min (the ray list I of Sec. 4.2), order them by (depth, id)
and run the scalar recurrences of Eq. 1 and Algorithm 1 in plain Python.
This is independent of tiling and of the tile-list sort, so a tiled renderer
that bins, orders or culls wrongly disagrees with it.
"""

from __future__ import annotations

import numpy as np

from .params import RenderParams


def ray_alphas(proj, px: int, py: int, params: RenderParams):
    """(alpha' list, gid list) of pixel (px, py), in ray order."""
    u = np.asarray(proj["means2d"], np.float64)
    con = np.asarray(proj["conic"], np.float64)
    o = np.asarray(proj["opacity"], np.float64)
    vis = np.asarray(proj["visible"], bool)
    depth = np.asarray(proj["depth"])
    dx = px + 0.5 - u[:, 0]
    dy = py + 0.5 - u[:, 1]
    power = -0.5 * (con[:, 0] * dx * dx + 2.0 * con[:, 1] * dx * dy + con[:, 2] * dy * dy)
    alpha = np.minimum(params.alpha_max, o * np.exp(power))
    keep = np.nonzero(vis & (alpha >= params.alpha_min))[0]
    order = sorted(keep.tolist(), key=lambda g: (float(depth[g]), g))
    return [float(alpha[g]) for g in order], order


def ray_dense(alphas, feats, T_eps, D):
    """Eq. 1 on one ray with the early stop; returns (C, T_final, n_blended)."""
    C = [0.0] * D
    T = 1.0
    n = 0
    for a, f in zip(alphas, feats):
        T_test = T * (1.0 - a)
        if T_test < T_eps:
            break
        w = a * T
        for d in range(D):
            C[d] += w * f[d]
        T = T_test
        n += 1
    return C, T, n


def ray_quantile(alphas, feats, K, D):
    """Algorithm 1 on one ray; returns (f~Q, T^Q, [selected list indices])."""
    T, TQ = 1.0, 1.0
    fQ = [0.0] * D
    k = 0
    chosen = []

    def thr(m):  # 1 - m/(K+1); m = K+1 gives 0
        return 1.0 - m / (K + 1.0)

    for i, (a, f) in enumerate(zip(alphas, feats)):
        T_test = T * (1.0 - a)
        if T_test < thr(k + 1):
            k += 1
            w = TQ * a
            for d in range(D):
                fQ[d] += w * f[d]
            TQ *= (1.0 - a)
            chosen.append(i)
            while T_test < thr(k + 1):
                k += 1
        if T_test < 1.0 / (K + 1.0):
            break
        T = T_test
    if not chosen:
        return [0.0] * D, TQ, chosen
    Z = 1.0 - TQ
    return [x / Z for x in fQ], TQ, chosen


def brute_force_render(proj, features, width, height, params: RenderParams = RenderParams(),
                       K=None, pixels=None):
    """Per-pixel render. K=None gives the dense blend, else Quantile with K.

    Returns dict with out [H,W,D] (NaN where not evaluated), T [H,W]
    (T_final for dense, T^Q for quantile) and n [H,W] (blended/selected count).
    """
    F = np.asarray(features, dtype=np.float64)
    D = F.shape[1]
    out = np.full((height, width, D), np.nan)
    Tm = np.full((height, width), np.nan)
    nm = np.full((height, width), -1, dtype=np.int64)
    if pixels is None:
        pixels = [(x, y) for y in range(height) for x in range(width)]
    for (px, py) in pixels:
        alphas, order = ray_alphas(proj, px, py, params)
        feats = [F[g].tolist() for g in order]
        if K is None:
            C, T, n = ray_dense(alphas, feats, params.T_eps, D)
            out[py, px] = C
            Tm[py, px] = T
            nm[py, px] = n
        else:
            f, TQ, chosen = ray_quantile(alphas, feats, K, D)
            out[py, px] = f
            Tm[py, px] = TQ
            nm[py, px] = len(chosen)
    return dict(out=out, T=Tm, n=nm)

