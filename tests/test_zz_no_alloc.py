"""The static-workspace binning (qr_bin_sort_noalloc) against qr_bin_sort on
the same projected scenes: bit-identical keys, order, offsets and pair
count, on two calls in a row, the second on a smaller scene (the scratch
array keeps the first call's contents)."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qr():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2512_20927_amd as qr
    return qr


def _bins_both(qr, sc, cam):
    from paper_2512_20927_amd import _lib as L
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pr = qr.project(t(sc.means), t(sc.scales), t(sc.quats), t(sc.opacity), cam)
    ref = qr.bin_sort(pr, cam.width, cam.height, keep_keys=True)
    cap = ref.capacity
    n = pr.depth.shape[0]
    tx, ty = (cam.width + 15) // 16, (cam.height + 15) // 16
    i32 = dict(dtype=torch.int32, device="cuda")
    # outputs pre-filled with garbage so that nothing is taken for written
    offs = torch.full((tx * ty + 1,), -7, **i32)
    gid = torch.full((max(cap, 1),), -7, **i32)
    keys = torch.full((max(cap, 1),), -7, dtype=torch.int64, device="cuda")
    total = torch.full((1,), -7, **i32)
    L.qr_bin_sort_noalloc(n, tx, ty, pr.tile_rect, pr.tiles_touched, pr.depth, cap, gid, keys,
                          offs, total)
    torch.cuda.synchronize()
    return ref, (offs, gid, keys, total)


def _assert_same(ref, got):
    offs, gid, keys, total = got
    P = int(ref.total_pairs.item())
    assert int(total.item()) == P
    assert torch.equal(offs, ref.tile_offsets)
    assert torch.equal(gid[:P], ref.sorted_gid[:P])
    assert torch.equal(keys[:P], ref.sorted_keys[:P])


def test_bin_sort_noalloc_matches_bin_sort_twice(qr):
    # first call: room scene, 200k Gaussians (about 150k pairs over 1,200 tiles)
    sc1, cam1 = synth.make_room(200_000, 1, dim=16), synth.room_camera(100)
    ref1, got1 = _bins_both(qr, sc1, cam1)
    print("noalloc call 1: pairs", int(ref1.total_pairs.item()), flush=True)
    _assert_same(ref1, got1)
    # second call, smaller: a ragged 100x75 image of 3,000 Gaussians
    sc2, cam2 = synth.make_tiny(3, n=3000, dim=16), synth.tiny_camera(100)
    cam2.height = 75
    cam2.cy = 37.5
    ref2, got2 = _bins_both(qr, sc2, cam2)
    print("noalloc call 2: pairs", int(ref2.total_pairs.item()), flush=True)
    _assert_same(ref2, got2)
    assert int(ref2.total_pairs.item()) < int(ref1.total_pairs.item())


def test_bin_sort_noalloc_long_lists(qr):
    """Tile lists past the LDS sort (6,000 keys) take the radix sort through
    the scratch array's second segment."""
    n = 6000
    rng = np.random.default_rng(8)
    means = np.zeros((n, 3), np.float32)
    means[:, :2] = rng.uniform(-0.2, 0.2, (n, 2))
    means[:, 2] = rng.integers(0, 50, n) * np.float32(0.01)
    sc = synth.Scene(means, np.full((n, 3), 0.6, np.float32), np.tile(np.float32([1, 0, 0, 0]), (n, 1)),
                     np.full(n, 0.5, np.float32), rng.standard_normal((n, 16)).astype(np.float32))
    ref, got = _bins_both(qr, sc, synth.tiny_camera())
    print("noalloc long lists: pairs", int(ref.total_pairs.item()), flush=True)
    _assert_same(ref, got)
