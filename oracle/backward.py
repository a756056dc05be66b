"""Analytic gradients of the dense blend (Eq. 1) and of Quantile Rendering
(Algorithm 1), FP64, one pixel at a time.

The paper trains through the renderer (Sec. 4.2: gradients flow from the
image-space loss back to the per-Gaussian features) but prints no backward
formulas; these are the derivatives of the forward definitions in
``render.py``. The discrete decisions (which entries are on the ray, where
the walk stops, which entries are selected) are piecewise constant and pass
no gradient; a clamped alpha' (= alpha_max) passes none to o or the geometry.

With g = dL/d(output), d_i = <g, f_i>:

Dense, w_i = T_i alpha'_i:
  dL/df_i      = w_i g
  dL/dalpha'_i = T_i d_i - (sum_{l>i} w_l d_l) / (1 - alpha'_i)

Quantile, over the selected entries j (in order), w_j = T^Q_j alpha'_j,
Z = 1 - T^Q (final), output f~ = (sum_j w_j f_j) / Z:
  dL/df_j      = (w_j / Z) g
  dL/dalpha'_j = [T^Q_j d_j - (sum_{l>j} w_l d_l)/(1 - alpha'_j)] / Z
                 - <g, f~> T^Q / ((1 - alpha'_j) Z)

Then alpha' = o G with G = exp(power), power = -1/2 (a dx^2 + 2 b dx dy +
c dy^2), dx = px + 0.5 - u, dy = py + 0.5 - v:
  dalpha'/do = G, dalpha'/dpower = alpha',
  dpower/da = -dx^2/2, dpower/db = -dx dy, dpower/dc = -dy^2/2,
  dpower/du = a dx + b dy, dpower/dv = b dx + c dy.
The conic is parameterised by (a, b, c) with b the single off-diagonal entry.

Magnitudes (``magnitude=True``, for tolerances only): alongside each gradient
the oracle returns, per element, a bound on the sum of the absolute values
of the terms that a finite-precision evaluation adds up to form it - every
dot product <g, f> replaced by sum |g| |f|, every tail sum by the whole
ray's sum of w_l sum |g| |f_l| (an evaluation may form tail sums as a total
minus a prefix), and each chain-rule factor by its absolute value. A
float32 evaluation of the same sums errs by at most a small multiple of its
unit roundoff times this bound, element by element.
"""

from __future__ import annotations

import numpy as np

from .params import RenderParams
from .render import quantile_thresholds


def _entries(proj, lst, px, py, params):
    """On-ray entries of pixel (px, py): (gid, alpha', G, dx, dy, clamped)."""
    out = []
    for g in lst:
        u, v = proj["means2d"][g]
        a, b, c = proj["conic"][g]
        o = proj["opacity"][g]
        dx = px + 0.5 - u
        dy = py + 0.5 - v
        power = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy)
        G = np.exp(power)
        raw = o * G
        alpha = min(params.alpha_max, raw)
        if alpha < params.alpha_min:
            continue
        out.append((int(g), float(alpha), float(G), float(dx), float(dy),
                    bool(raw >= params.alpha_max)))
    return out


def _chain(grads, proj, e, dL_dalpha, mag=None, mag_dalpha=0.0):
    g, alpha, G, dx, dy, clamped = e
    if clamped:
        return
    a, b, c = proj["conic"][g]
    if mag is not None:
        m = abs(mag_dalpha)
        mag["opacity"][g] += m * G
        mp = m * alpha
        mag["conic"][g, 0] += mp * 0.5 * dx * dx
        mag["conic"][g, 1] += mp * abs(dx * dy)
        mag["conic"][g, 2] += mp * 0.5 * dy * dy
        mag["means2d"][g, 0] += mp * (abs(a * dx) + abs(b * dy))
        mag["means2d"][g, 1] += mp * (abs(b * dx) + abs(c * dy))
    grads["opacity"][g] += dL_dalpha * G
    dpow = dL_dalpha * alpha
    grads["conic"][g, 0] += dpow * (-0.5 * dx * dx)
    grads["conic"][g, 1] += dpow * (-dx * dy)
    grads["conic"][g, 2] += dpow * (-0.5 * dy * dy)
    grads["means2d"][g, 0] += dpow * (a * dx + b * dy)
    grads["means2d"][g, 1] += dpow * (b * dx + c * dy)


def _new_grads(n, D):
    return dict(features=np.zeros((n, D)), opacity=np.zeros(n),
                conic=np.zeros((n, 3)), means2d=np.zeros((n, 2)))


def _proj64(proj):
    return dict(means2d=np.asarray(proj["means2d"], np.float64),
                conic=np.asarray(proj["conic"], np.float64),
                opacity=np.asarray(proj["opacity"], np.float64))


def _pixels_of_tiles(width, height, tile, tiles=None):
    tiles_x = (width + tile - 1) // tile
    tiles_y = (height + tile - 1) // tile
    for t in (range(tiles_x * tiles_y) if tiles is None else tiles):
        ty, tx = divmod(t, tiles_x)
        for py in range(ty * tile, min((ty + 1) * tile, height)):
            for px in range(tx * tile, min((tx + 1) * tile, width)):
                yield t, px, py


def dense_backward(proj, sorted_gid, tile_offsets, features, width, height, grad_out,
                   params: RenderParams = RenderParams(), tiles=None, magnitude=False):
    """Gradients of the dense blend; with ``tiles`` only those tiles' pixels
    contribute (as if grad_out were zero elsewhere). With ``magnitude`` the
    result also holds "abs", the per-element term magnitudes (module doc)."""
    proj = _proj64(proj)
    F = np.asarray(features, np.float64)
    gout = np.asarray(grad_out, np.float64)
    grads = _new_grads(F.shape[0], F.shape[1])
    mag = _new_grads(F.shape[0], F.shape[1]) if magnitude else None
    for t, px, py in _pixels_of_tiles(width, height, params.tile, tiles):
        lst = sorted_gid[int(tile_offsets[t]):int(tile_offsets[t + 1])]
        T = 1.0
        blended = []
        for e in _entries(proj, lst, px, py, params):
            T_test = T * (1.0 - e[1])
            if T_test < params.T_eps:
                break
            blended.append((e, T))
            T = T_test
        gp = gout[py, px]
        d = [float(F[e[0]] @ gp) for e, _ in blended]
        if mag is not None:
            dabs = [float(np.abs(F[e[0]]) @ np.abs(gp)) for e, _ in blended]
            ray_abs = sum(Tj * e[1] * da for (e, Tj), da in zip(blended, dabs))
        suffix = 0.0
        for j in range(len(blended) - 1, -1, -1):
            e, Tj = blended[j]
            w = Tj * e[1]
            grads["features"][e[0]] += w * gp
            dL_da = Tj * d[j] - suffix / (1.0 - e[1])
            m_da = 0.0
            if mag is not None:
                mag["features"][e[0]] += w * np.abs(gp)
                m_da = Tj * dabs[j] + ray_abs / (1.0 - e[1])
            _chain(grads, proj, e, dL_da, mag, m_da)
            suffix += w * d[j]
    if mag is not None:
        grads["abs"] = mag
    return grads


def quantile_backward(proj, sorted_gid, tile_offsets, features, width, height, K, grad_out,
                      params: RenderParams = RenderParams(), tiles=None, magnitude=False):
    """Gradients of Quantile Rendering; ``tiles`` and ``magnitude`` as in
    dense_backward."""
    proj = _proj64(proj)
    F = np.asarray(features, np.float64)
    gout = np.asarray(grad_out, np.float64)
    grads = _new_grads(F.shape[0], F.shape[1])
    mag = _new_grads(F.shape[0], F.shape[1]) if magnitude else None
    thr = np.append(quantile_thresholds(K), 0.0)
    for t, px, py in _pixels_of_tiles(width, height, params.tile, tiles):
        lst = sorted_gid[int(tile_offsets[t]):int(tile_offsets[t + 1])]
        T, TQ, k = 1.0, 1.0, 0
        sel = []
        for e in _entries(proj, lst, px, py, params):
            T_test = T * (1.0 - e[1])
            if T_test < thr[k]:
                k += 1
                sel.append((e, TQ))
                TQ *= (1.0 - e[1])
                while T_test < thr[k]:
                    k += 1
            if T_test < 1.0 / (K + 1.0):
                break
            T = T_test
        if not sel:
            continue
        Z = 1.0 - TQ
        gp = gout[py, px]
        fsum = sum(TQj * e[1] * F[e[0]] for e, TQj in sel)
        gf = float(gp @ (fsum / Z))
        d = [float(F[e[0]] @ gp) for e, _ in sel]
        if mag is not None:
            dabs = [float(np.abs(F[e[0]]) @ np.abs(gp)) for e, _ in sel]
            ray_abs = sum(TQj * e[1] * da for (e, TQj), da in zip(sel, dabs))
        suffix = 0.0
        for j in range(len(sel) - 1, -1, -1):
            e, TQj = sel[j]
            w = TQj * e[1]
            grads["features"][e[0]] += (w / Z) * gp
            dL_da = (TQj * d[j] - suffix / (1.0 - e[1])) / Z \
                - gf * TQ / ((1.0 - e[1]) * Z)
            m_da = 0.0
            if mag is not None:
                mag["features"][e[0]] += (w / Z) * np.abs(gp)
                m_da = (TQj * dabs[j] + ray_abs / (1.0 - e[1])) / Z \
                    + (ray_abs / Z) * TQ / ((1.0 - e[1]) * Z)
            _chain(grads, proj, e, dL_da, mag, m_da)
            suffix += w * d[j]
    if mag is not None:
        grads["abs"] = mag
    return grads
