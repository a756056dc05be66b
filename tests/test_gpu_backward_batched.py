"""Q-Render backward over many views in one launch: for views of two scenes
(one scene seen by two views that share its gradient arrays), every launch
shape must accumulate the sum of the single-view backward calls (already
checked against the oracle). Float atomics add in an unspecified order, so
the comparison is to float32 rounding (relative L2 <= 1e-5 per array).
Also: a feature width wider than one 512-column pass, and the backward with
only some of the gradient arrays requested."""

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


def _rel(a, b):
    a, b = a.double(), b.double()
    return float((a - b).norm() / max(float(b.norm()), 1e-30))


def _single_backward(qr, v, K, g, grads):
    qr._lib.qr_render_quantile_backward(v["width"], v["height"], qr.RenderParams().c(), K,
                                        v["tile_offsets"], v["sorted_gid"], v["means2d"],
                                        v["conic_opacity"], v["features"], v["feature_scale"], g,
                                        grads[0], grads[1], grads[2])


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_batched_backward_matches_sum_of_single_views(qr, storage):
    from paper_2512_20927_amd import _lib as L
    from paper_2512_20927_amd.batched import BatchedQuantile
    K, dim = 8, 32
    views, _ = _make_views(qr, storage, dim=dim, K=K)
    scene_of = [0, 1, 0]
    n_of = [v["features"].shape[0] for v in views]
    rng = np.random.default_rng(3)
    gouts = [_t(rng.standard_normal((v["height"], v["width"], dim)).astype(np.float32)) for v in views]

    def zeros():
        return [[torch.zeros(n_of[si], dim, device="cuda"), torch.zeros(n_of[si], 2, device="cuda"),
                 torch.zeros(n_of[si], 4, device="cuda")] for si in (0, 1)]

    ref = zeros()
    for v, si, g in zip(views, scene_of, gouts):
        _single_backward(qr, v, K, g, ref[si])
    torch.cuda.synchronize()
    code = {"f32": L.QR_F32, "bf16": L.QR_BF16}[storage]
    bq = BatchedQuantile(views, K, dim, code, qr.RenderParams().c())
    for kind in ("natural", "heavy"):
        for w in (0, 2):
            got = zeros()
            bq.set_grads([dict(grad_out=g, grad_features=got[si][0], grad_means2d=got[si][1],
                               grad_conic_opacity=got[si][2]) for g, si in zip(gouts, scene_of)])
            bq.backward(kind, w)
            torch.cuda.synchronize()
            for si in (0, 1):
                for a, b in zip(got[si], ref[si]):
                    assert float(b.abs().sum()) > 0
                    assert _rel(a, b) <= 1e-5, (kind, w, si)


def test_backward_wide_features_and_partial_outputs(qr):
    """dim = 640: a full 512-column pass plus a partial one. Requesting only
    the feature gradient, or only the geometric ones, gives the same arrays
    as requesting all three."""
    K, dim = 8, 640
    sc = synth.make_tiny(4, n=1200, dim=dim)
    cam = synth.tiny_camera(48)
    pr = qr.project(_t(sc.means), _t(sc.scales), _t(sc.quats), _t(sc.opacity), cam)
    bins = qr.bin_sort(pr, cam.width, cam.height)
    f = _t(sc.features)
    v = dict(width=cam.width, height=cam.height, tile_offsets=bins.tile_offsets,
             sorted_gid=bins.sorted_gid, means2d=pr.means2d, conic_opacity=pr.conic_opacity,
             features=f, feature_scale=None)
    g = _t(np.random.default_rng(8).standard_normal((cam.height, cam.width, dim)).astype(np.float32))
    n = sc.n

    def run(which):
        out = [torch.zeros(n, dim, device="cuda") if "f" in which else None,
               torch.zeros(n, 2, device="cuda") if "g" in which else None,
               torch.zeros(n, 4, device="cuda") if "g" in which else None]
        _single_backward(qr, v, K, g, out)
        torch.cuda.synchronize()
        return out

    full, feat_only, geo_only = run("fg"), run("f"), run("g")
    assert float(full[0].abs().sum()) > 0 and float(full[1].abs().sum()) > 0
    assert _rel(feat_only[0], full[0]) <= 1e-6
    assert _rel(geo_only[1], full[1]) <= 1e-6 and _rel(geo_only[2], full[2]) <= 1e-6
