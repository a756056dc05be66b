"""Host-side validation of batched view records (no GPU needed): every
mismatch between a view's buffers and the batch's K, feature width, feature
dtype or output dtype is refused before any pointer reaches the device table
that the batched kernels read."""

import pytest
import torch

from paper_2512_20927_amd import _lib as L
from paper_2512_20927_amd.batched import validate_views


def _view(W=40, H=24, n=50, dim=32, feat_dtype=torch.float32, out_dtype=torch.float32, scale=False):
    tiles = ((W + 15) // 16) * ((H + 15) // 16)
    return dict(tile_offsets=torch.zeros(tiles + 1, dtype=torch.int32),
                sorted_gid=torch.zeros(8, dtype=torch.int32),
                means2d=torch.zeros(n, 2), conic_opacity=torch.zeros(n, 4),
                features=torch.zeros(n, dim, dtype=feat_dtype),
                feature_scale=torch.ones(n) if scale else None,
                out=torch.zeros(H, W, dim, dtype=out_dtype),
                T_q=torch.zeros(H, W), n_sel=torch.zeros(H, W, dtype=torch.int32),
                width=W, height=H)


def _params(out_dtype=L.QR_F32):
    return L.make_params(out_dtype=out_dtype)


def test_good_views_pass():
    validate_views([_view(), _view(W=17, H=5, n=9)], 8, 32, L.QR_F32, _params())
    validate_views([_view(feat_dtype=torch.uint8, scale=True)], 8, 32, L.QR_FP8_E4M3, _params())
    validate_views([_view(out_dtype=torch.bfloat16)], 64, 32, L.QR_F32, _params(L.QR_BF16))
    v = _view()
    v["T_q"] = v["n_sel"] = None  # optional outputs
    validate_views([v], 8, 32, L.QR_F32, _params())


@pytest.mark.parametrize("mutate,exc,msg", [
    (lambda v: v.update(out=torch.zeros(23, 40, 32)), ValueError, "view 1: out"),
    (lambda v: v.update(out=torch.zeros(24, 40, 32, dtype=torch.bfloat16)), TypeError, "view 1: out"),
    (lambda v: v.update(features=torch.zeros(50, 48)), ValueError, "view 1: features"),
    (lambda v: v.update(features=torch.zeros(50, 32, dtype=torch.bfloat16)), TypeError, "view 1: features"),
    (lambda v: v.update(T_q=torch.zeros(10)), ValueError, "view 1: T_q"),
    (lambda v: v.update(n_sel=torch.zeros(24, 40)), TypeError, "view 1: n_sel"),
    (lambda v: v.update(tile_offsets=torch.zeros(6, dtype=torch.int32)), ValueError, "view 1: tile_offsets"),
    (lambda v: v.update(means2d=torch.zeros(49, 2)), ValueError, "view 1: means2d"),
    (lambda v: v.update(conic_opacity=torch.zeros(50, 4)[:, :3]), ValueError, "view 1: conic_opacity"),
])
def test_bad_view_is_refused(mutate, exc, msg):
    views = [_view(), _view()]
    mutate(views[1])
    with pytest.raises(exc, match=msg):
        validate_views(views, 8, 32, L.QR_F32, _params())


def test_fp8_needs_scale_and_k_range():
    with pytest.raises(ValueError, match="feature_scale"):
        validate_views([_view(feat_dtype=torch.uint8)], 8, 32, L.QR_FP8_E4M3, _params())
    with pytest.raises(ValueError, match="K = 0"):
        validate_views([_view()], 0, 32, L.QR_F32, _params())
    with pytest.raises(ValueError, match="K = %d" % (L.QR_MAX_K + 1)):
        validate_views([_view()], L.QR_MAX_K + 1, 32, L.QR_F32, _params())
