"""Dense alpha-blending (Eq. 1) and Quantile Rendering (Algorithm 1), FP64.

Both renderers walk each tile's depth-sorted list one entry at a time, with
the state of the tile's (up to) 256 rays held side by side in arrays; every
ray's arithmetic is exactly the scalar recurrence of the paper.

Per pixel p (centre (px + 0.5, py + 0.5)) and list entry i:
  d = centre - mean_i,  power = -1/2 (a dx^2 + 2 b dx dy + c dy^2),
  alpha'_i = min(alpha_max, o_i exp(power))                       (Eq. 1)
and entries with alpha'_i < alpha_min are not on that pixel's ray list I.

Dense (Eq. 1): T_1 = 1, w_i = T_i alpha'_i, C = sum_i w_i f_i,
T_{i+1} = T_i (1 - alpha'_i). Reading: the 3D-GS early stop - an entry whose
T_test = T (1 - alpha') would fall below T_eps is not blended and the ray
ends; T_eps = 0 blends every Gaussian on the ray. No background term.

Quantile (Algorithm 1), thresholds t_m = 1 - m/(K+1), m = 1..K:
  T = 1, T^Q = 1, f^Q = 0, k = 0
  for i in I:  T_test = T (1 - alpha'_i)
     if T_test < t_{k+1}:  k += 1; w^Q = T^Q alpha'_i; f^Q += w^Q f_i;
                           T^Q *= (1 - alpha'_i)
                           while T_test < t_{k+1}: k += 1
     if T_test < 1/(K+1): stop
     T = T_test
  output f^Q / (1 - T^Q).
Readings: "<" is strict (T_test equal to a threshold does not cross); the
threshold after the last is t_{K+1} = 0, which no T_test crosses, so k never
exceeds K and the while loop ends there; when no Gaussian is
selected (T^Q = 1, a 0/0) the output is the zero vector.

Decision margins. Each ray also reports the smallest relative distance of any
discrete decision it took (alpha' vs alpha_min, T_test vs T_eps, T_test vs a
threshold) to its boundary. A lower-precision implementation may legitimately
take a different branch where that margin is tiny; ``bias`` moves every
boundary by the factor (1 + bias) so such alternative results can be produced.
"""

from __future__ import annotations

import numpy as np

from .params import RenderParams


def quantile_thresholds(K: int) -> np.ndarray:
    """t_m = 1 - m/(K+1) for m = 1..K (index m-1)."""
    return np.array([1.0 - (m / (K + 1.0)) for m in range(1, K + 1)])


def _tile_pixels(t, tiles_x, W, H, tile):
    ty, tx = divmod(int(t), tiles_x)
    ys, xs = np.meshgrid(np.arange(ty * tile, (ty + 1) * tile),
                         np.arange(tx * tile, (tx + 1) * tile), indexing="ij")
    xs, ys = xs.ravel(), ys.ravel()
    inside = (xs < W) & (ys < H)
    return xs[inside], ys[inside]


def _alpha(proj, g, xs, ys, params):
    u, v = proj["means2d"][g]
    a, b, c = proj["conic"][g]
    o = proj["opacity"][g]
    dx = xs + 0.5 - u
    dy = ys + 0.5 - v
    power = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy)
    return np.minimum(params.alpha_max, o * np.exp(power))


def _dense_weight(alpha, T_before, T_after):
    """Eq. 1's weight of an entry: its opacity times the transmittance in
    front of it (T_after = T_before (1 - alpha) is the transmittance behind
    it, which the weight must not use)."""
    return alpha * T_before


def _rel(x, bound):
    return np.abs(x - bound) / bound


def _as_f64_proj(proj):
    return dict(means2d=np.asarray(proj["means2d"], np.float64),
                conic=np.asarray(proj["conic"], np.float64),
                opacity=np.asarray(proj["opacity"], np.float64))


def render_dense(proj, sorted_gid, tile_offsets, features, width, height,
                 params: RenderParams = RenderParams(), tiles=None, bias=0.0):
    """Dense alpha-blend over each pixel's ray list.

    ``proj`` holds means2d [N,2], conic [N,3] (a, b, c), opacity [N].
    Returns dict: out [H,W,D], T_final [H,W], n_contrib [H,W] (list position
    + 1 of the last blended entry, 0 if none), n_on [H,W] (on-ray entries
    examined), margin [H,W]. With ``tiles``
    only those tile ids are evaluated; other pixels are NaN / -1.
    """
    proj = _as_f64_proj(proj)
    F = np.asarray(features, dtype=np.float64)
    D = F.shape[1]
    tile = params.tile
    tiles_x = (width + tile - 1) // tile
    tiles_y = (height + tile - 1) // tile
    out = np.full((height, width, D), np.nan)
    T_final = np.full((height, width), np.nan)
    n_contrib = np.full((height, width), -1, dtype=np.int64)
    n_on = np.full((height, width), -1, dtype=np.int64)
    margin = np.full((height, width), np.nan)
    a_min = params.alpha_min * (1.0 + bias)
    t_eps = params.T_eps * (1.0 + bias)
    if tiles is None:
        tiles = range(tiles_x * tiles_y)
    for t in tiles:
        xs, ys = _tile_pixels(t, tiles_x, width, height, tile)
        m = xs.size
        T = np.ones(m)
        C = np.zeros((m, D))
        done = np.zeros(m, dtype=bool)
        ncon = np.zeros(m, dtype=np.int64)
        non = np.zeros(m, dtype=np.int64)
        marg = np.full(m, np.inf)
        lo, hi = int(tile_offsets[t]), int(tile_offsets[t + 1])
        for pos in range(lo, hi):
            if done.all():
                break
            g = int(sorted_gid[pos])
            alpha = _alpha(proj, g, xs, ys, params)
            live = ~done
            marg[live] = np.minimum(marg[live], _rel(alpha[live], params.alpha_min))
            on_ray = live & (alpha >= a_min)
            non += on_ray
            T_test = T * (1.0 - alpha)
            if params.T_eps > 0:
                marg[on_ray] = np.minimum(marg[on_ray], _rel(T_test[on_ray], params.T_eps))
            stop = on_ray & (T_test < t_eps)
            blend = on_ray & ~stop
            w = np.where(blend, _dense_weight(alpha, T, T_test), 0.0)
            C += w[:, None] * F[g][None, :]
            T = np.where(blend, T_test, T)
            ncon[blend] = pos - lo + 1
            done |= stop
        out[ys, xs] = C
        T_final[ys, xs] = T
        n_contrib[ys, xs] = ncon
        n_on[ys, xs] = non
        margin[ys, xs] = marg
    return dict(out=out, T_final=T_final, n_contrib=n_contrib, n_on=n_on, margin=margin)


def render_quantile(proj, sorted_gid, tile_offsets, features, width, height, K,
                    params: RenderParams = RenderParams(), tiles=None, bias=0.0):
    """Quantile Rendering (Algorithm 1) of every pixel's ray list.

    Returns dict: out [H,W,D] (normalised f~Q), T_q [H,W] (T^Q), n_sel [H,W]
    (number of selected Gaussians), k [H,W] (thresholds consumed), T_final
    [H,W] (Algorithm 1's full transmittance T when the walk ends: the stop
    test breaks before T takes the stopping entry's T_test), n_steps
    [H,W] (list position + 1 of the last on-ray entry examined, the stopping
    entry included), n_on [H,W] (on-ray entries examined),
    sel_gid [H,W,K] (-1 padded, in selection order), sel_w [H,W,K] (w^Q),
    sel_pos [H,W,K] (position in the tile list), margin [H,W].
    """
    proj = _as_f64_proj(proj)
    F = np.asarray(features, dtype=np.float64)
    D = F.shape[1]
    tile = params.tile
    tiles_x = (width + tile - 1) // tile
    tiles_y = (height + tile - 1) // tile
    thr = quantile_thresholds(K)
    # t_{K+1} = 1 - (K+1)/(K+1) = 0: once k = K no threshold can be crossed
    thr_b = np.append(thr, 0.0) * (1.0 + bias)
    stop_b = (1.0 / (K + 1.0)) * (1.0 + bias)
    a_min = params.alpha_min * (1.0 + bias)

    out = np.full((height, width, D), np.nan)
    T_q = np.full((height, width), np.nan)
    n_sel = np.full((height, width), -1, dtype=np.int64)
    k_out = np.full((height, width), -1, dtype=np.int64)
    T_fin = np.full((height, width), np.nan)
    n_steps = np.full((height, width), -1, dtype=np.int64)
    n_on = np.full((height, width), -1, dtype=np.int64)
    sel_gid = np.full((height, width, K), -1, dtype=np.int64)
    sel_w = np.zeros((height, width, K))
    sel_pos = np.full((height, width, K), -1, dtype=np.int64)
    margin = np.full((height, width), np.nan)
    if tiles is None:
        tiles = range(tiles_x * tiles_y)
    for t in tiles:
        xs, ys = _tile_pixels(t, tiles_x, width, height, tile)
        m = xs.size
        T = np.ones(m)
        TQ = np.ones(m)
        fQ = np.zeros((m, D))
        k = np.zeros(m, dtype=np.int64)
        ns = np.zeros(m, dtype=np.int64)
        steps = np.zeros(m, dtype=np.int64)
        non = np.zeros(m, dtype=np.int64)
        done = np.zeros(m, dtype=bool)
        sg = np.full((m, K), -1, dtype=np.int64)
        sw = np.zeros((m, K))
        sp = np.full((m, K), -1, dtype=np.int64)
        marg = np.full(m, np.inf)
        lo, hi = int(tile_offsets[t]), int(tile_offsets[t + 1])
        for pos in range(lo, hi):
            if done.all():
                break
            g = int(sorted_gid[pos])
            alpha = _alpha(proj, g, xs, ys, params)
            live = ~done
            marg[live] = np.minimum(marg[live], _rel(alpha[live], params.alpha_min))
            on_ray = live & (alpha >= a_min)
            steps[on_ray] = pos - lo + 1
            non += on_ray
            T_test = T * (1.0 - alpha)
            if on_ray.any():
                d_thr = np.min(_rel(T_test[on_ray][:, None], thr[None, :]), axis=1)
                marg[on_ray] = np.minimum(marg[on_ray], d_thr)
            # sampling a quantile Gaussian: the first threshold not yet consumed
            crossed = on_ray & (T_test < thr_b[k])
            for p in np.nonzero(crossed)[0]:
                k[p] += 1
                w = TQ[p] * alpha[p]
                fQ[p] += w * F[g]
                TQ[p] *= (1.0 - alpha[p])
                sg[p, ns[p]] = g
                sw[p, ns[p]] = w
                sp[p, ns[p]] = pos - lo
                ns[p] += 1
                while T_test[p] < thr_b[k[p]]:
                    k[p] += 1
            stop = on_ray & (T_test < stop_b)
            T = np.where(on_ray & ~stop, T_test, T)
            done |= stop
        res = np.zeros((m, D))
        nz = ns > 0
        res[nz] = fQ[nz] / (1.0 - TQ[nz])[:, None]
        out[ys, xs] = res
        T_q[ys, xs] = TQ
        n_sel[ys, xs] = ns
        k_out[ys, xs] = k
        T_fin[ys, xs] = T
        n_steps[ys, xs] = steps
        n_on[ys, xs] = non
        sel_gid[ys, xs] = sg
        sel_w[ys, xs] = sw
        sel_pos[ys, xs] = sp
        margin[ys, xs] = marg
    return dict(out=out, T_q=T_q, n_sel=n_sel, k=k_out, T_final=T_fin, n_steps=n_steps, n_on=n_on,
                sel_gid=sel_gid, sel_w=sel_w, sel_pos=sel_pos, margin=margin)
