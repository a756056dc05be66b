"""The dense blend (Eq. 1): single-view maps against the FP64 oracle at
feature widths of the narrow tile kernels (16: one column tile; 48 and 64:
one permuted group) and of the strip kernel (144: partial groups; 528: a
second 512-column pass), with every feature storage;
and the batched launch over (view, tile) items (every launch shape) bit for
bit against the single-view kernel on views of uneven scenes and image
shapes."""

import numpy as np
import pytest
import torch

import synth
from tests.test_gpu_parity import check_all, decoded_features, gpu_pipeline, oracle_renders

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_20927_amd as qr
    return qr


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("dim,storage", [(16, "f32"), (16, "bf16"), (16, "fp8"), (48, "f32"),
                                         (48, "bf16"), (64, "fp8"), (144, "f32"), (528, "f32"),
                                         (144, "bf16"), (528, "fp8")])
def test_dense_matches_oracle_feature_widths(qr, dim, storage):
    """100x75 (ragged tiles and strips that lie partly or wholly below the
    image), 3,000 Gaussians."""
    sc = synth.make_tiny(5, n=3000, dim=dim)
    cam = synth.tiny_camera(100)
    cam.height, cam.cy = 75, 37.5
    res = gpu_pipeline(qr, sc, cam, 8, storage=storage)
    feats = decoded_features(qr, sc, res, storage)
    ors = oracle_renders(res, feats, 100, 75, 8)
    st = check_all(res, ors, 100, 75)
    assert st["d"]["clean"] > 0.9 * st["d"]["pixels"]


def _make_views(qr, storage, dim):
    scenes = [synth.make_tiny(1, n=2500, dim=dim), synth.make_room(30_000, 9, dim=dim)]
    cams = [synth.tiny_camera(64), synth.room_camera(120, 100, 75, 120.0), synth.tiny_camera(80)]
    cams[2].height, cams[2].cy = 48, 24.0
    scene_of = [0, 1, 0]
    feats = []
    for sc in scenes:
        f = _t(sc.features)
        feats.append((f, None) if storage == "f32" else qr.quantize(f, storage))
    views, single = [], []
    for cam, si in zip(cams, scene_of):
        sc = scenes[si]
        pr = qr.project(_t(sc.means), _t(sc.scales), _t(sc.quats), _t(sc.opacity), cam)
        bins = qr.bin_sort(pr, cam.width, cam.height)
        f, s = feats[si]
        ref = qr.render_dense(pr, bins, f, cam.width, cam.height, feature_scale=s)
        single.append(ref)
        views.append(dict(tile_offsets=bins.tile_offsets, sorted_gid=bins.sorted_gid,
                          means2d=pr.means2d, conic_opacity=pr.conic_opacity, features=f,
                          feature_scale=s,
                          out=torch.full_like(ref["out"], float("nan")),
                          T_q=torch.full_like(ref["T_final"], float("nan")),
                          n_sel=torch.full_like(ref["n_contrib"], -7),
                          width=cam.width, height=cam.height, _pr=pr, _bins=bins))
    return views, single


@pytest.mark.parametrize("storage,dim", [("f32", 16), ("bf16", 16), ("fp8", 16), ("f32", 32),
                                         ("f32", 528), ("bf16", 144), ("fp8", 64)])
def test_batched_dense_matches_single_view(qr, storage, dim):
    from paper_2512_20927_amd import _lib as L
    from paper_2512_20927_amd.batched import BatchedDense
    views, single = _make_views(qr, storage, dim)
    code = L.DTYPE_CODE[views[0]["features"].dtype]
    bd = BatchedDense(views, dim, code, qr.RenderParams().c())
    for kind, w in (("natural", 0), ("heavy", 0), ("natural", 3), ("heavy", 8)):
        for v in views:
            v["out"].fill_(float("nan"))
            v["T_q"].fill_(float("nan"))
            v["n_sel"].fill_(-7)
        bd.render(kind, w)
        torch.cuda.synchronize()
        for v, ref in zip(views, single):
            assert torch.equal(v["out"], ref["out"]), (kind, w)
            assert torch.equal(v["T_q"], ref["T_final"]), (kind, w)
            assert torch.equal(v["n_sel"], ref["n_contrib"]), (kind, w)


def test_batched_dense_autotune(qr, tmp_path):
    from paper_2512_20927_amd import _lib as L
    from paper_2512_20927_amd.batched import BatchedDense, autotune
    views, single = _make_views(qr, "f32", 32)
    bd = BatchedDense(views, 32, L.QR_F32, qr.RenderParams().c())
    cfg, timings = autotune(bd, wg_per_cu=(0, 2), reps=2, cache_path=str(tmp_path / "t.json"))
    assert cfg["ms"] == min(timings.values()) and len(timings) == 4
    torch.cuda.synchronize()
    for v, ref in zip(views, single):  # outputs of the last timed launch
        assert torch.equal(v["out"], ref["out"])
