"""Pins of the oracle's tile binning: depth-ordered per-tile lists (the
ordered ray sequence S_r of Eq. 1) against an independent per-tile
enumeration, and the 64-bit key form used on the GPU."""

import numpy as np

import oracle
from oracle.binning import depth_bits_key


def _random_rects(rng, n, tiles_x, tiles_y):
    tx0 = rng.integers(0, tiles_x, n)
    ty0 = rng.integers(0, tiles_y, n)
    tx1 = np.minimum(tx0 + rng.integers(0, 4, n), tiles_x)
    ty1 = np.minimum(ty0 + rng.integers(0, 3, n), tiles_y)
    return np.stack([tx0, ty0, tx1, ty1], 1)


def test_bin_sort_matches_per_tile_enumeration():
    rng = np.random.default_rng(0)
    tiles_x, tiles_y, n = 7, 5, 400
    rect = _random_rects(rng, n, tiles_x, tiles_y)
    # few distinct depths so that ties (broken by gid) occur
    depth = rng.integers(1, 30, n).astype(np.float32) * np.float32(0.25)
    gids, offs, _ = oracle.bin_sort(rect, depth, tiles_x, tiles_y)
    assert offs[0] == 0 and offs[-1] == gids.size
    assert np.all(np.diff(offs) >= 0)
    assert gids.size == int(np.sum((rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1])))
    for t in range(tiles_x * tiles_y):
        ty, tx = divmod(t, tiles_x)
        cover = np.nonzero((rect[:, 0] <= tx) & (tx < rect[:, 2]) & (rect[:, 1] <= ty) & (ty < rect[:, 3]))[0]
        want = cover[np.lexsort((cover, depth[cover]))]
        np.testing.assert_array_equal(gids[offs[t]:offs[t + 1]], want)


def test_empty_rects_and_empty_tiles():
    rect = np.array([[0, 0, 0, 0], [1, 1, 2, 2], [0, 0, 0, 3]])
    gids, offs, _ = oracle.bin_sort(rect, np.array([1.0, 2.0, 3.0], np.float32), 3, 3)
    assert gids.tolist() == [1]
    assert offs.tolist() == [0, 0, 0, 0, 0, 1, 1, 1, 1, 1]


def test_stable_sort_of_bit_keys_equals_triple_sort():
    rng = np.random.default_rng(1)
    tiles_x, tiles_y, n = 9, 4, 300
    rect = _random_rects(rng, n, tiles_x, tiles_y)
    depth = rng.uniform(0.2, 50.0, n).astype(np.float32)
    depth[::7] = depth[0]  # ties
    gids, offs, _ = oracle.bin_sort(rect, depth, tiles_x, tiles_y)
    keys, vals = [], []
    for g in range(n):  # emitted in gid order, as the GPU does
        for ty in range(rect[g, 1], rect[g, 3]):
            for tx in range(rect[g, 0], rect[g, 2]):
                keys.append(depth_bits_key(ty * tiles_x + tx, depth[g]))
                vals.append(g)
    order = sorted(range(len(keys)), key=lambda i: keys[i])  # Python sort is stable
    np.testing.assert_array_equal(np.array(vals)[order], gids)
