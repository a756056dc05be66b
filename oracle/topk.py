"""Top-K selection, the alternative sampler the paper compares Quantile
Rendering with inside its own renderer (Sec. 4.2 and the complexity table:
keep the K Gaussians of largest contribution on the ray, O(N log K + KC)),
FP64. TEST INFRASTRUCTURE ONLY.

Readings (the paper names the strategy but not its details):
* "contribution" is the dense blending weight w_i = T_i alpha'_i of Eq. 1,
  with the same ray list I (alpha' >= alpha_min) and the same T_eps stop as
  the dense blend: the candidates are exactly the Gaussians the dense blend
  composites;
* the K largest weights win; equal weights are ranked by list position
  (earlier first);
* the selected Gaussians keep their dense weights and the output is
  normalised by their sum, sum_sel w_i f_i / sum_sel w_i (the analogue of
  Alg. 1's division by 1 - T^Q = sum of the w^Q); T_q reports 1 - sum_sel w_i;
  a ray with no candidate gives the zero vector.

Margins: as the dense oracle's (alpha' vs alpha_min, T_test vs T_eps), plus
the relative gap between the K-th and (K+1)-th largest weights, where a float32
ranking may legitimately differ. ``bias`` moves alpha_min and T_eps as in the
dense oracle; ``swap_kth`` keeps the (K+1)-th largest weight instead of the
K-th on every ray with more than K candidates (the other ranking a float32
comparison may take where the two are nearly equal).
"""

from __future__ import annotations

import numpy as np

from .params import RenderParams
from .render import _alpha, _as_f64_proj, _rel, _tile_pixels


def render_topk(proj, sorted_gid, tile_offsets, features, width, height, K,
                params: RenderParams = RenderParams(), tiles=None, bias=0.0, swap_kth=False):
    """Top-K rendering of every pixel's ray.

    Returns dict: out [H,W,D], T_q [H,W] (1 - sum of the selected weights),
    n_sel [H,W], sel_gid / sel_w / sel_pos [H,W,K] (in list order, -1 / 0
    padded), n_cand [H,W] (Gaussians the dense blend composites), margin [H,W].
    """
    proj = _as_f64_proj(proj)
    F = np.asarray(features, dtype=np.float64)
    D = F.shape[1]
    tile = params.tile
    tiles_x = (width + tile - 1) // tile
    tiles_y = (height + tile - 1) // tile
    a_min = params.alpha_min * (1.0 + bias)
    t_eps = params.T_eps * (1.0 + bias)

    out = np.full((height, width, D), np.nan)
    T_q = np.full((height, width), np.nan)
    n_sel = np.full((height, width), -1, dtype=np.int64)
    n_cand = np.full((height, width), -1, dtype=np.int64)
    sel_gid = np.full((height, width, K), -1, dtype=np.int64)
    sel_w = np.zeros((height, width, K))
    sel_pos = np.full((height, width, K), -1, dtype=np.int64)
    margin = np.full((height, width), np.nan)
    if tiles is None:
        tiles = range(tiles_x * tiles_y)
    for t in tiles:
        xs, ys = _tile_pixels(t, tiles_x, width, height, tile)
        m = xs.size
        lo, hi = int(tile_offsets[t]), int(tile_offsets[t + 1])
        # the dense walk: every pixel's blended (position, weight) pairs
        T = np.ones(m)
        done = np.zeros(m, dtype=bool)
        marg = np.full(m, np.inf)
        cands = [[] for _ in range(m)]
        for pos in range(lo, hi):
            if done.all():
                break
            g = int(sorted_gid[pos])
            alpha = _alpha(proj, g, xs, ys, params)
            live = ~done
            marg[live] = np.minimum(marg[live], _rel(alpha[live], params.alpha_min))
            on_ray = live & (alpha >= a_min)
            T_test = T * (1.0 - alpha)
            if params.T_eps > 0:
                marg[on_ray] = np.minimum(marg[on_ray], _rel(T_test[on_ray], params.T_eps))
            stop = on_ray & (T_test < t_eps)
            blend = on_ray & ~stop
            for p in np.nonzero(blend)[0]:
                cands[p].append((pos - lo, g, T[p] * alpha[p]))
            T = np.where(blend, T_test, T)
            done |= stop
        # the K largest weights, ties to the earlier position
        for p in range(m):
            c = cands[p]
            y, x = ys[p], xs[p]
            n_cand[y, x] = len(c)
            if not c:
                out[y, x] = 0.0
                T_q[y, x] = 1.0
                n_sel[y, x] = 0
                margin[y, x] = marg[p]
                continue
            posv = np.array([e[0] for e in c])
            gv = np.array([e[1] for e in c])
            wv = np.array([e[2] for e in c])
            rank = np.lexsort((posv, -wv))  # weight descending, then position
            if len(c) > K:
                wk, wk1 = wv[rank[K - 1]], wv[rank[K]]
                marg[p] = min(marg[p], (wk - wk1) / wk)
                if swap_kth:
                    rank[[K - 1, K]] = rank[[K, K - 1]]
            keep = np.sort(rank[:K])  # back to list order
            s = wv[keep].sum()
            out[y, x] = (wv[keep][:, None] * F[gv[keep]]).sum(axis=0) / s
            T_q[y, x] = 1.0 - s
            n_sel[y, x] = keep.size
            sel_gid[y, x, :keep.size] = gv[keep]
            sel_w[y, x, :keep.size] = wv[keep]
            sel_pos[y, x, :keep.size] = posv[keep]
            margin[y, x] = marg[p]
    return dict(out=out, T_q=T_q, n_sel=n_sel, n_cand=n_cand, sel_gid=sel_gid, sel_w=sel_w,
                sel_pos=sel_pos, margin=margin)
