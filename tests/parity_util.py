"""Comparison helpers for GPU-vs-oracle parity tests."""

from __future__ import annotations

import numpy as np

# float32 kernels vs the float64 oracle (per-pixel relative L2 error)
FP32_TOL = 1e-4
# relative margin of a discrete decision below which a float32 walk may take
# the other branch (see oracle.render: margin / bias)
DECISION_WINDOW = 1e-4


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


def compare_render(gpu_out, oracle_res, oracle_alt, evaluated=None, tol=FP32_TOL,
                   window=DECISION_WINDOW, max_unexplained=0.0):
    """Checks GPU output against the oracle.

    Pixels whose every decision is further than `window` (relative) from its
    boundary must agree within `tol`. Flagged pixels must agree with the
    oracle or with one of the runs in `oracle_alt` (boundaries moved by
    +-window); the fraction that matches none may not exceed
    `max_unexplained`. Returns a stats dict.
    """
    ref = oracle_res["out"]
    mask = ~np.isnan(ref[..., 0]) if evaluated is None else evaluated
    e = pixel_rel_err(gpu_out, ref)
    flagged = (oracle_res["margin"] <= window) & mask
    clean = mask & ~flagged
    stats = dict(pixels=int(mask.sum()), flagged=int(flagged.sum()),
                 max_err_clean=float(e[clean].max()) if clean.any() else 0.0,
                 p99_err_clean=float(np.percentile(e[clean], 99)) if clean.any() else 0.0,
                 mean_err_clean=float(e[clean].mean()) if clean.any() else 0.0)
    bad_clean = clean & (e > tol)
    stats["bad_clean"] = int(bad_clean.sum())
    unexplained = 0
    for idx in zip(*np.nonzero(flagged)):
        ok = e[idx] <= tol
        for alt in oracle_alt:
            ok = ok or pixel_rel_err(gpu_out[idx], alt["out"][idx]) <= tol
        unexplained += 0 if ok else 1
    stats["unexplained_flagged"] = unexplained
    assert stats["bad_clean"] == 0, stats
    assert unexplained <= max_unexplained * max(stats["pixels"], 1), stats
    return stats
