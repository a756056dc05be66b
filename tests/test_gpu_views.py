"""Multi-view front: qr_project_views and qr_bin_sort_views over a batch of
cameras must reproduce, bit for bit, the single-view projection and binning
of every camera (already checked against the oracle), and the renders made
from their per-view slices must equal the single-view renders."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_20927_amd as qr
    return qr


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _scene(n=30_000, seed=21, dim=32):
    sc = synth.make_room(n, seed, dim=dim)
    return sc, [_t(sc.means), _t(sc.scales), _t(sc.quats), _t(sc.opacity)]


@pytest.mark.parametrize("n_views", [3, 37])  # 37: two launches of at most 32 cameras
def test_project_views_matches_per_view(qr, n_views):
    sc, s = _scene()
    W, H = 200, 150
    cams = [synth.room_camera(500 + v, W, H, 180.0) for v in range(n_views)]
    pv = qr.project_views(*s, cams)
    n = sc.n
    for v, cam in enumerate(cams):
        one = qr.project(*s, cam)
        sl = slice(v * n, (v + 1) * n)
        for name in ("means2d", "conic_opacity", "depth", "tile_rect", "tiles_touched"):
            # bit patterns: culled records may hold non-finite conics in both
            a, b = getattr(pv, name)[sl], getattr(one, name)
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (v, name)


def test_bin_sort_views_matches_per_view(qr):
    sc, s = _scene()
    W, H = 200, 150  # ragged: 13 x 10 tiles, last row and column partial
    cams = [synth.room_camera(600 + v, W, H, 180.0) for v in range(5)]
    pv = qr.project_views(*s, cams)
    total = qr.count_pairs(pv)
    vb = qr.ViewsBinner(len(cams), sc.n, W, H, total + 16, keep_keys=True)
    bins = vb(pv)
    torch.cuda.synchronize()
    assert int(bins.total_pairs.item()) == total
    offs = bins.tile_offsets.cpu().numpy().astype(np.int64)
    gids = bins.sorted_gid.cpu().numpy()
    keys = bins.sorted_keys.cpu().numpy().view(np.uint64)
    T = vb.tiles_per_view
    for v, cam in enumerate(cams):
        one = qr.bin_sort(qr.project(*s, cam), W, H, keep_keys=True)
        torch.cuda.synchronize()
        p = int(one.total_pairs.item())
        o1 = one.tile_offsets.cpu().numpy().astype(np.int64)
        ov = offs[v * T:(v + 1) * T + 1]
        np.testing.assert_array_equal(ov - ov[0], o1)
        np.testing.assert_array_equal(gids[ov[0]:ov[-1]], one.sorted_gid.cpu().numpy()[:p])
        k1 = one.sorted_keys.cpu().numpy().view(np.uint64)[:p]
        np.testing.assert_array_equal(keys[ov[0]:ov[-1]] - np.uint64((v * T) << 32), k1)


def test_bin_sort_views_reports_overflow(qr):
    sc, s = _scene(n=5_000)
    cams = [synth.room_camera(700 + v, 128, 96, 120.0) for v in range(3)]
    pv = qr.project_views(*s, cams)
    total = qr.count_pairs(pv)
    assert total > 10
    vb = qr.ViewsBinner(len(cams), sc.n, 128, 96, total // 2)
    bins = vb(pv)
    torch.cuda.synchronize()
    assert int(bins.total_pairs.item()) == total  # more than the capacity: caller must retry


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_renders_from_view_slices_match_single_view(qr, storage):
    from paper_2512_20927_amd import _lib as L
    from paper_2512_20927_amd.batched import BatchedQuantile
    sc, s = _scene(dim=48)
    W, H, K = 160, 128, 8
    cams = [synth.room_camera(800 + v, W, H, 150.0) for v in range(4)]
    f32 = _t(sc.features)
    feats, scale = (f32, None) if storage == "f32" else qr.quantize(f32, storage)
    pv = qr.project_views(*s, cams)
    vb = qr.ViewsBinner(len(cams), sc.n, W, H, qr.count_pairs(pv) + 16)
    vb(pv)
    views = []
    for v, cam in enumerate(cams):
        pr1 = qr.project(*s, cam)
        b1 = qr.bin_sort(pr1, W, H)
        ref_q = qr.render_quantile(pr1, b1, feats, W, H, K, feature_scale=scale)
        ref_d = qr.render_dense(pr1, b1, feats, W, H, feature_scale=scale)
        prv, bv = vb.view(pv, v)
        got_q = qr.render_quantile(prv, bv, feats, W, H, K, feature_scale=scale)
        got_d = qr.render_dense(prv, bv, feats, W, H, feature_scale=scale)
        for k in ref_q:
            assert torch.equal(got_q[k], ref_q[k]), (v, k)
        for k in ref_d:
            assert torch.equal(got_d[k], ref_d[k]), (v, k)
        views.append((dict(tile_offsets=bv.tile_offsets, sorted_gid=bv.sorted_gid,
                           means2d=prv.means2d, conic_opacity=prv.conic_opacity, features=feats,
                           feature_scale=scale, out=torch.full_like(ref_q["out"], float("nan")),
                           T_q=torch.full_like(ref_q["T_q"], float("nan")),
                           n_sel=torch.full_like(ref_q["n_sel"], -7), width=W, height=H), ref_q))
    code = L.QR_F32 if storage == "f32" else L.QR_BF16
    bq = BatchedQuantile([v for v, _ in views], K, 48, code, qr.RenderParams().c())
    for w in (0, 2):
        bq.render("natural", w)
        torch.cuda.synchronize()
        for v, ref in views:
            assert torch.equal(v["out"], ref["out"]) and torch.equal(v["n_sel"], ref["n_sel"])
