"""RGB use of Q-Render (Appendix, "Rendering RGB"): spherical-harmonic colours
on the GPU against the FP64 oracle, and the colour table rendered by both
renderers against the oracle renders of the same table."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.parity_util import DECISION_WINDOW, compare_render, proj_for_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_20927_amd as qr
    return qr


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_sh_colours_match_oracle(qr, degree):
    from paper_2512_20927_amd import _lib as L
    rng = np.random.default_rng(degree)
    n = 5000
    mu = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    sh = (rng.standard_normal((n, 16, 3)) * 0.4).astype(np.float32)
    cam = synth.tiny_camera(64)
    out = torch.full((n, 16), float("nan"), device="cuda")
    L.qr_sh_to_rgb(_t(mu), _t(sh), degree, cam, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = oracle.sh_to_rgb(mu.astype(np.float64), sh.astype(np.float64), cam, degree)
    np.testing.assert_allclose(got[:, :3], want, atol=2e-6)
    assert np.all(got[:, 3:] == 0.0)


def test_rgb_render_parity(qr):
    """The colour table (degree 3, 13 zero columns to the renderers' width of
    16) through both renderers against the oracle renders of the GPU's own
    colours, projection and bins."""
    from paper_2512_20927_amd import _lib as L
    sc = synth.make_tiny(2, n=2000, dim=16)
    cam = synth.tiny_camera(64)
    rng = np.random.default_rng(5)
    sh = (rng.standard_normal((sc.n, 16, 3)) * 0.3).astype(np.float32)
    rgb = torch.empty(sc.n, 16, device="cuda")
    L.qr_sh_to_rgb(_t(sc.means), _t(sh), 3, cam, rgb)
    pr = qr.project(_t(sc.means), _t(sc.scales), _t(sc.quats), _t(sc.opacity), cam)
    bins = qr.bin_sort(pr, 64, 64)
    q = qr.render_quantile(pr, bins, rgb, 64, 64, 8)
    d = qr.render_dense(pr, bins, rgb, 64, 64)
    torch.cuda.synchronize()
    P = int(bins.total_pairs.item())
    proj = proj_for_oracle(dict(means2d=pr.means2d.cpu().numpy(), conic_opacity=pr.conic_opacity.cpu().numpy()))
    gids = bins.sorted_gid.cpu().numpy()[:P].astype(np.int64)
    offs = bins.tile_offsets.cpu().numpy().astype(np.int64)
    F = rgb.cpu().numpy().astype(np.float64)
    for name, got, fn in (("q", q, lambda b: oracle.render_quantile(proj, gids, offs, F, 64, 64, 8, bias=b)),
                          ("d", d, lambda b: oracle.render_dense(proj, gids, offs, F, 64, 64, bias=b))):
        ref = fn(0.0)
        print(name, compare_render(got["out"].cpu().numpy(), ref, [fn(DECISION_WINDOW), fn(-DECISION_WINDOW)]))


@pytest.mark.parametrize("n_views,degree,out_dim,stride", [(3, 3, 16, 16), (37, 3, 16, 16), (3, 0, 4, 1),
                                                           (5, 2, 20, 9)])
def test_sh_colours_views_match_per_view(qr, n_views, degree, out_dim, stride):
    """The batched colour kernel against the single-camera one (same
    arithmetic, coefficients read once) and the oracle; 37 cameras take two
    launches of at most 32; out_dim / 4 = 1, 4 and 5 lanes per Gaussian;
    coefficient rows exactly (degree + 1)^2 long."""
    from paper_2512_20927_amd import _lib as L
    rng = np.random.default_rng(11 + degree)
    n = 3001
    mu = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    sh = (rng.standard_normal((n, stride, 3)) * 0.4).astype(np.float32)
    cams = [synth.room_camera(900 + v, 64, 48, 50.0) for v in range(n_views)]
    out = torch.full((n_views, n, out_dim), float("nan"), device="cuda")
    L.qr_sh_to_rgb_views(_t(mu), _t(sh), degree, cams, out)
    one = torch.empty(n, out_dim, device="cuda")
    for v in (0, n_views // 2, n_views - 1):
        L.qr_sh_to_rgb(_t(mu), _t(sh), degree, cams[v], one)
        torch.cuda.synchronize()
        np.testing.assert_allclose(out[v].cpu().numpy(), one.cpu().numpy(), rtol=0, atol=1e-6)
        want = oracle.sh_to_rgb(mu.astype(np.float64), sh.astype(np.float64), cams[v], degree)
        np.testing.assert_allclose(out[v, :, :3].cpu().numpy(), want, atol=2e-6)
    assert torch.all(out[:, :, 3:] == 0)
