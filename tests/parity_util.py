"""Comparison helpers for GPU-vs-oracle parity tests.

Discrete decisions (alpha' vs alpha_min, T vs T_eps, T vs a threshold) are
taken in float32 on the GPU and in float64 by the oracle; each oracle pixel
reports the smallest relative distance of any of its decisions to its
boundary (its margin). Pixels are compared in three tiers:

* margin > DECISION_WINDOW (1e-4): must match the oracle within the float32
  tolerance, with identical selections;
* STRICT_WINDOW < margin <= DECISION_WINDOW, the band between the 1e-6
  window that the selection contract names and 1e-4: counted, and each
  pixel either matches the oracle (counted as a match) or matches an oracle
  run with every boundary moved by +-1e-4 (counted as a band mismatch and
  reported, never absorbed silently);
* margin <= STRICT_WINDOW: must match the oracle or a boundary-moved run.
A pixel that matches none of the runs is unexplained; none is allowed.
Float32 can legitimately disagree in the band: alpha' carries a relative
error of a few ulps times |power| (up to about 11 at the footprint edge,
i.e. about 3e-6), and the transmittance chain one or two roundings per
entry.
"""

from __future__ import annotations

import numpy as np

# float32 kernels vs the float64 oracle (per-pixel relative L2 error)
FP32_TOL = 1e-4
# boundary shift of the alternative oracle runs
DECISION_WINDOW = 1e-4
# window within which selections may differ without being reported
STRICT_WINDOW = 1e-6


def pixel_rel_err(x, y, floor=1e-6):
    """e_p = ||x_p - y_p|| / max(||y_p||, floor) over the last axis."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    num = np.linalg.norm(x - y, axis=-1)
    den = np.maximum(np.linalg.norm(y, axis=-1), floor)
    return num / den


def proj_for_oracle(pr_gpu):
    """Oracle input dict from GPU projection outputs (same float32 values)."""
    co = pr_gpu["conic_opacity"].astype(np.float64)
    return dict(means2d=pr_gpu["means2d"].astype(np.float64), conic=co[:, :3], opacity=co[:, 3])


def _tiers(margin, mask):
    clean = mask & (margin > DECISION_WINDOW)
    band = mask & (margin > STRICT_WINDOW) & (margin <= DECISION_WINDOW)
    tight = mask & (margin <= STRICT_WINDOW)
    return clean, band, tight


def compare_render(gpu_out, oracle_res, oracle_alt, evaluated=None, tol=FP32_TOL,
                   max_unexplained=0):
    """Checks a GPU map against the oracle in the three tiers above.

    Returns a stats dict: pixels, clean / band / tight counts, band and tight
    pixels that differ from the unshifted oracle (explained by a shifted run),
    the unexplained count (asserted <= max_unexplained, default 0) and the
    error statistics over clean pixels."""
    ref = oracle_res["out"]
    mask = ~np.isnan(ref[..., 0]) if evaluated is None else evaluated
    e = pixel_rel_err(gpu_out, ref)
    clean, band, tight = _tiers(oracle_res["margin"], mask)
    stats = dict(pixels=int(mask.sum()), clean=int(clean.sum()), band=int(band.sum()),
                 tight=int(tight.sum()),
                 max_err_clean=float(e[clean].max()) if clean.any() else 0.0,
                 p99_err_clean=float(np.percentile(e[clean], 99)) if clean.any() else 0.0,
                 mean_err_clean=float(e[clean].mean()) if clean.any() else 0.0)
    stats["bad_clean"] = int((clean & (e > tol)).sum())
    near = band | tight
    match0 = e <= tol
    alt_ok = np.zeros_like(near)
    for alt in oracle_alt:
        alt_ok |= near & (pixel_rel_err(gpu_out, alt["out"]) <= tol)
    stats["band_mismatch"] = int((band & ~match0).sum())
    stats["tight_mismatch"] = int((tight & ~match0).sum())
    stats["unexplained"] = int((near & ~match0 & ~alt_ok).sum())
    assert stats["bad_clean"] == 0, stats
    assert stats["unexplained"] <= max_unexplained * max(stats["pixels"], 1), stats
    return stats


def compare_selection(gpu_sel, gpu_ns, oracle_res, oracle_alt, evaluated=None):
    """Selected Gaussian ids (in ray order, -1 padded to K) and counts:
    identical to the oracle on clean pixels; on band and tight pixels
    identical to the oracle or to a boundary-moved run (band differences
    counted). Returns a stats dict."""
    K = oracle_res["sel_gid"].shape[-1]
    mask = ~np.isnan(oracle_res["out"][..., 0]) if evaluated is None else evaluated
    gsel = np.asarray(gpu_sel)[..., :K]
    clean, band, tight = _tiers(oracle_res["margin"], mask)
    np.testing.assert_array_equal(gsel[clean], oracle_res["sel_gid"][clean])
    np.testing.assert_array_equal(np.asarray(gpu_ns)[clean], oracle_res["n_sel"][clean])
    near = band | tight
    same = np.all(gsel == oracle_res["sel_gid"], axis=-1)
    ok = same.copy()
    for alt in oracle_alt:
        ok |= np.all(gsel == alt["sel_gid"], axis=-1)
    stats = dict(sel_band_mismatch=int((band & ~same).sum()),
                 sel_tight_mismatch=int((tight & ~same).sum()),
                 sel_unexplained=int((near & ~ok).sum()))
    assert stats["sel_unexplained"] == 0, stats
    return stats
