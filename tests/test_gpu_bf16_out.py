"""Q-Render with bfloat16 feature maps (qr_params.out_dtype = QR_BF16): the
map must be the float32 map rounded to nearest even, bit for bit (the same
kernel arithmetic, rounded only at the store), for one view and for every
batched launch shape; per-pixel scalars are unchanged. The dense blend
rejects the option."""

import numpy as np
import pytest
import torch

import synth
from tests.test_gpu_batched import _make_views

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_20927_amd as qr
    return qr


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("storage", ["f32", "bf16", "fp8"])
def test_single_view_bf16_maps_are_rounded_f32_maps(qr, storage):
    from paper_2512_20927_amd import _lib as L
    sc = synth.make_tiny(5, n=3000, dim=48)  # dim 48: a partial column pass
    cam = synth.tiny_camera(100)
    cam.height, cam.cy = 75, 37.5  # ragged tiles
    pr = qr.project(_t(sc.means), _t(sc.scales), _t(sc.quats), _t(sc.opacity), cam)
    bins = qr.bin_sort(pr, cam.width, cam.height)
    f32 = _t(sc.features)
    feats, scale = (f32, None) if storage == "f32" else qr.quantize(f32, storage)
    ref = qr.render_quantile(pr, bins, feats, cam.width, cam.height, 8, feature_scale=scale)
    prm = qr.RenderParams(out_dtype=L.QR_BF16)
    got = qr.render_quantile(pr, bins, feats, cam.width, cam.height, 8, params=prm, feature_scale=scale)
    torch.cuda.synchronize()
    assert got["out"].dtype == torch.bfloat16
    assert torch.equal(got["out"].view(torch.int16), ref["out"].to(torch.bfloat16).view(torch.int16))
    assert torch.equal(got["T_q"], ref["T_q"]) and torch.equal(got["n_sel"], ref["n_sel"])
    with pytest.raises(L.QRError):
        qr.render_dense(pr, bins, feats, cam.width, cam.height, params=prm, feature_scale=scale)


def test_batched_bf16_maps_every_launch_shape(qr):
    from paper_2512_20927_amd import _lib as L
    from paper_2512_20927_amd.batched import BatchedQuantile
    views, single = _make_views(qr, "f32")
    for v in views:
        v["out"] = torch.full(v["out"].shape, float("nan"), dtype=torch.bfloat16, device="cuda")
    bq = BatchedQuantile(views, 8, 32, L.QR_F32, qr.RenderParams(out_dtype=L.QR_BF16).c())
    for kind in ("natural", "heavy"):
        for w in (0, 3):
            for v in views:
                v["out"].fill_(float("nan"))
            bq.render(kind, w)
            torch.cuda.synchronize()
            for v, ref in zip(views, single):
                want = ref["out"].to(torch.bfloat16).view(torch.int16)
                assert torch.equal(v["out"].view(torch.int16), want), (kind, w)
