"""De-voxelisation of network predictions to per-Gaussian features (the step
of the paper's pipeline that produces the feature table the renderer reads;
Appendix, de-voxelisation), FP64. TEST INFRASTRUCTURE ONLY.

Every Gaussian g owns a contiguous run [offsets[g], offsets[g+1]) of voxel
slots; slot m refers to unique voxel voxel_unique[m], whose prediction row is
unique_pred[voxel_unique[m]]. The Gaussian's feature is the elementwise
reduction (max, or mean) of its slots' rows.

Readings (the appendix shows the step only as a code listing, which is
inconsistent in two places): expanding unique-voxel predictions to all voxel
slots is a gather through the slot -> unique-voxel map; the segment offsets
start at 0 (G+1 entries); an empty segment gives the zero row (and no
argmax, -1); ties in max go to the first slot of the segment.
Backward: max routes each output element's gradient to the unique voxel row
of its argmax slot; mean spreads grad / count over the segment's slots (both
accumulated over slots that share a unique voxel).
"""

from __future__ import annotations

import numpy as np


def devoxelize(offsets, voxel_unique, unique_pred, reduce: str = "max"):
    """Returns (out [G, C], argmax [G, C] slot indices or -1; None for mean)."""
    offsets = np.asarray(offsets, np.int64)
    vu = np.asarray(voxel_unique, np.int64)
    P = np.asarray(unique_pred, np.float64)
    G, C = offsets.size - 1, P.shape[1]
    out = np.zeros((G, C))
    arg = np.full((G, C), -1, dtype=np.int64) if reduce == "max" else None
    for g in range(G):
        lo, hi = int(offsets[g]), int(offsets[g + 1])
        if hi == lo:
            continue
        rows = P[vu[lo:hi]]
        if reduce == "max":
            best = rows[0].copy()
            bi = np.full(C, lo, dtype=np.int64)
            for m in range(1, hi - lo):
                better = rows[m] > best  # strict: ties keep the first slot
                best[better] = rows[m][better]
                bi[better] = lo + m
            out[g], arg[g] = best, bi
        else:
            out[g] = rows.sum(axis=0) / (hi - lo)
    return out, arg


def devoxelize_backward(offsets, voxel_unique, n_unique, grad_out, reduce: str = "max", argmax=None):
    """dL/d(unique_pred) [U, C] for dL/d(out) = grad_out [G, C]."""
    offsets = np.asarray(offsets, np.int64)
    vu = np.asarray(voxel_unique, np.int64)
    g_out = np.asarray(grad_out, np.float64)
    G, C = g_out.shape
    grad = np.zeros((n_unique, C))
    for g in range(G):
        lo, hi = int(offsets[g]), int(offsets[g + 1])
        if hi == lo:
            continue
        if reduce == "max":
            for c in range(C):
                grad[vu[argmax[g, c]], c] += g_out[g, c]
        else:
            for m in range(lo, hi):
                grad[vu[m]] += g_out[g] / (hi - lo)
    return grad
