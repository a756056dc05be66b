"""Tile binning: depth-ordered per-tile Gaussian lists (plain Python sort).

The ray list S_r of Eq. 1 is an ordered sequence of the Gaussians on the ray;
3D-GS builds it per 16 x 16 tile by sorting (tile, depth) pairs. Reading:
depth is the camera-space z of the Gaussian's mean (one depth per Gaussian,
not per pixel), and equal depths are ordered by Gaussian index.

Given each visible Gaussian's half-open tile rectangle and depth, this emits
one (tile, depth, gid) triple per covered tile, sorts the triples with
Python's ``sorted`` and returns the gid column plus CSR offsets
``tile_offsets[t]`` = number of pairs whose tile id is below t.
Tile id = ty * tiles_x + tx.
"""

from __future__ import annotations

import numpy as np


def bin_sort(rect, depth, tiles_x: int, tiles_y: int):
    """Returns (sorted_gid int64[P], tile_offsets int64[n_tiles+1], keys list).

    ``rect`` is int [N,4] (tx0, ty0, tx1, ty1), empty for culled Gaussians;
    ``depth`` is the per-Gaussian sort depth (compared as given).
    ``keys`` is the sorted list of (tile, depth, gid) triples.
    """
    rect = np.asarray(rect)
    depth = np.asarray(depth)
    triples = []
    for gid in range(rect.shape[0]):
        tx0, ty0, tx1, ty1 = (int(v) for v in rect[gid])
        d = float(depth[gid])
        for ty in range(ty0, ty1):
            for tx in range(tx0, tx1):
                triples.append((ty * tiles_x + tx, d, gid))
    triples = sorted(triples)
    n_tiles = tiles_x * tiles_y
    offsets = np.zeros(n_tiles + 1, dtype=np.int64)
    for tile, _, _ in triples:
        offsets[tile + 1] += 1
    offsets = np.cumsum(offsets)
    gids = np.array([g for _, _, g in triples], dtype=np.int64)
    return gids, offsets, triples


def depth_bits_key(tile: int, depth32: np.float32) -> int:
    """64-bit sort key used by GPU binning: tile in the high 32 bits, the
    IEEE-754 bits of the (positive) float32 depth in the low 32 bits. For
    positive floats the bit pattern orders like the value, so sorting these
    keys stably in gid order equals sorting (tile, depth, gid)."""
    bits = int(np.asarray(depth32, dtype=np.float32).view(np.uint32))
    return (int(tile) << 32) | bits
