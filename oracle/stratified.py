"""Stratified-K: the adaptive-threshold variant of Quantile Rendering
(Appendix, "Stratified-sampling"), FP64. TEST INFRASTRUCTURE ONLY.

The variant keeps Algorithm 1 but replaces the uniform thresholds
t_m = 1 - m/(K+1) by thresholds placed by the ray's own transmittance
statistics: the mean mu and standard deviation sigma of the transmittance
values along the ray are estimated in a first pass; the interval is cut
uniformly in z-score space under the Gaussian N(mu, sigma^2) and mapped back,
i.e. the m-th threshold sits where that Gaussian leaves probability
1 - m/(K+1) above it:

    t_m = mu + sigma * Phi^{-1}(1 - m/(K+1)),   m = 1..K,

so that thresholds crowd where the transmittance values are concentrated.
The second pass is Algorithm 1 with these thresholds.

Readings (the appendix gives no formula):
  * the transmittance values of the first pass are T_0 = 1 and the
    transmittance after every Gaussian the dense blend (Eq. 1, with its
    3D-GS early stop at T_eps) composites on the ray; T_0 makes sigma > 0 for
    any ray with an on-ray Gaussian (a ray with none selects nothing);
  * sigma is the population standard deviation;
  * thresholds are clipped to [0, 1]; crossings compare with "<" as in
    Algorithm 1; the second pass examines the Gaussians the first pass
    sampled (it ends where the dense blend stops, at T_test < T_eps, like
    the first pass) and ends earlier once all K thresholds are consumed (the
    counterpart of Algorithm 1's stop test);
  * the output is normalised by 1 - T^Q as in Sec. 4.2 (0 if nothing is
    selected).
Phi^{-1} is scipy.special.ndtri (a library step).
"""

from __future__ import annotations

import numpy as np
from scipy.special import ndtri

from .params import RenderParams
from .render import _alpha, _as_f64_proj, _rel, _tile_pixels


def transmittance_stats(alphas, T_eps: float):
    """(mu, sigma) of T_0 = 1 and the transmittance after each Gaussian the
    dense blend composites, for the on-ray opacities ``alphas`` in order."""
    T = 1.0
    vals = [1.0]
    for a in alphas:
        T_test = T * (1.0 - a)
        if T_test < T_eps:
            break
        T = T_test
        vals.append(T)
    v = np.asarray(vals)
    return float(v.mean()), float(v.std())


def stratified_thresholds(mu: float, sigma: float, K: int) -> np.ndarray:
    """t_m = clip(mu + sigma Phi^{-1}(1 - m/(K+1)), 0, 1), m = 1..K (descending)."""
    p = np.array([1.0 - m / (K + 1.0) for m in range(1, K + 1)])
    return np.clip(mu + sigma * ndtri(p), 0.0, 1.0)


def render_stratified(proj, sorted_gid, tile_offsets, features, width, height, K,
                      params: RenderParams = RenderParams(), tiles=None, bias=0.0):
    """Stratified-K render of every pixel's ray list. Returns dict: out [H,W,D],
    T_q [H,W], n_sel [H,W], sel_gid [H,W,K] (-1 padded), sel_w [H,W,K],
    mu [H,W], sigma [H,W], margin [H,W] (smallest relative distance of a
    decision of the second pass - alpha' vs alpha_min, T_test vs a threshold
    - to its boundary, and of the first pass's T_test vs T_eps). ``bias``
    moves every boundary (alpha_min, T_eps, each threshold) by the factor
    (1 + bias), as in render.py, to produce the result a lower-precision
    walk may legitimately give where a margin is tiny."""
    proj = _as_f64_proj(proj)
    F = np.asarray(features, dtype=np.float64)
    D = F.shape[1]
    tile = params.tile
    tiles_x = (width + tile - 1) // tile
    tiles_y = (height + tile - 1) // tile
    out = np.full((height, width, D), np.nan)
    T_q = np.full((height, width), np.nan)
    n_sel = np.full((height, width), -1, dtype=np.int64)
    sel_gid = np.full((height, width, K), -1, dtype=np.int64)
    sel_w = np.zeros((height, width, K))
    mu_out = np.full((height, width), np.nan)
    sd_out = np.full((height, width), np.nan)
    margin = np.full((height, width), np.nan)
    a_min = params.alpha_min * (1.0 + bias)
    t_eps = params.T_eps * (1.0 + bias)
    if tiles is None:
        tiles = range(tiles_x * tiles_y)
    for t in tiles:
        xs, ys = _tile_pixels(t, tiles_x, width, height, tile)
        lo, hi = int(tile_offsets[t]), int(tile_offsets[t + 1])
        gids = [int(sorted_gid[pos]) for pos in range(lo, hi)]
        A = np.array([_alpha(proj, g, xs, ys, params) for g in gids]).reshape(len(gids), xs.size)
        for j in range(xs.size):
            a_all = A[:, j]
            on = a_all >= a_min
            marg = np.min(_rel(a_all, params.alpha_min)) if a_all.size else np.inf
            # pass 1: transmittance statistics along the ray
            T = 1.0
            vals = [1.0]
            for a in a_all[on]:
                T_test = T * (1.0 - a)
                marg = min(marg, abs(T_test - params.T_eps) / params.T_eps)
                if T_test < t_eps:
                    break
                T = T_test
                vals.append(T)
            mu, sd = float(np.mean(vals)), float(np.std(vals))
            thr = np.append(stratified_thresholds(mu, sd, K), -1.0)  # t_{K+1}: never crossed
            thr_b = thr * (1.0 + bias)
            # pass 2: Algorithm 1 with the ray's thresholds
            T, TQ, k, ns = 1.0, 1.0, 0, 0
            fQ = np.zeros(D)
            for i in np.nonzero(on)[0]:
                a = a_all[i]
                T_test = T * (1.0 - a)
                if T_test < t_eps:  # the dense stop ends the sampled ray
                    break
                live = thr[:K][thr[:K] > 0.0]
                if live.size:
                    marg = min(marg, float(np.min(np.abs(T_test - live) / live)))
                if T_test < thr_b[k]:
                    k += 1
                    w = TQ * a
                    fQ += w * F[gids[i]]
                    TQ *= 1.0 - a
                    sel_gid[ys[j], xs[j], ns] = gids[i]
                    sel_w[ys[j], xs[j], ns] = w
                    ns += 1
                    while T_test < thr_b[k]:
                        k += 1
                T = T_test
                if k == K:
                    break
            out[ys[j], xs[j]] = fQ / (1.0 - TQ) if ns > 0 else 0.0
            T_q[ys[j], xs[j]] = TQ
            n_sel[ys[j], xs[j]] = ns
            mu_out[ys[j], xs[j]] = mu
            sd_out[ys[j], xs[j]] = sd
            margin[ys[j], xs[j]] = marg
    return dict(out=out, T_q=T_q, n_sel=n_sel, sel_gid=sel_gid, sel_w=sel_w, mu=mu_out,
                sigma=sd_out, margin=margin)
