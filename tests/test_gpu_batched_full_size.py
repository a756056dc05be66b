"""The batched Q-Render launch at the shapes it is timed at.

* room: 200k Gaussians, 16 poses at 640x480, 512-D float32 features, K = 8,
  projected by one multi-camera launch and binned over one stacked tile grid
  exactly as the benchmark step does. Every launch shape the autotuner
  chooses among (one workgroup per item, persistent workgroups on per-XCD
  queues; natural and longest-list-first order) must reproduce the
  single-view kernel bit for bit on every pose (maps, T^Q and selection
  counts), and the batched maps of two poses match the FP64 oracle on
  sampled tiles (the longest list among them).
* batched (reduced): four room scenes of uneven size (75k, 200k, 375k and
  750k Gaussians, a quarter of the full batched workload's), two views each
  at 1280x720, 512-D e4m3 features with per-Gaussian scales, K = 8: forward
  bit-identical to the single-view kernel; the backward of all eight views in
  one launch equals the sum of the single-view backward calls per scene up
  to float32 rounding of the atomic additions.
"""

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


def _front(qr, sc_t, cams, W, H):
    """Projection of one scene into all its cameras (one launch) and binning
    over the stacked grid, as the benchmark's front does."""
    n = sc_t["means"].shape[0]
    pv = qr.project_views(sc_t["means"], sc_t["scales"], sc_t["quats"], sc_t["opacity"], cams)
    vb = qr.ViewsBinner(len(cams), n, W, H, int(qr.count_pairs(pv) * 1.05) + 1024)
    vb(pv)
    return pv, vb


def _scene_t(sc):
    return dict(means=_t(sc.means), scales=_t(sc.scales), quats=_t(sc.quats), opacity=_t(sc.opacity))


def _view(pr, b, feats, scale, W, H, D, out_dtype=torch.float32):
    return dict(tile_offsets=b.tile_offsets, sorted_gid=b.sorted_gid, means2d=pr.means2d,
                conic_opacity=pr.conic_opacity, features=feats, feature_scale=scale,
                out=torch.full((H, W, D), float("nan"), dtype=out_dtype, device="cuda"),
                T_q=torch.full((H, W), float("nan"), device="cuda"),
                n_sel=torch.full((H, W), -7, dtype=torch.int32, device="cuda"), width=W, height=H)


SHAPES = [("heavy", 3), ("natural", 0), ("natural", 3), ("heavy", 8)]


def test_room_batched_launch_matches_single_view_and_oracle(qr):
    from paper_2512_20927_amd import _lib as L
    from paper_2512_20927_amd.batched import BatchedQuantile
    cfg = synth.CONFIGS["room"]
    W, H, D, K = cfg["width"], cfg["height"], cfg["dim"], 8
    sc = synth.make_room(cfg["n"], cfg["seed"], dim=D)
    cams = synth.room_poses(cfg["pose_seeds"], W, H, cfg["fx"])
    st = _scene_t(sc)
    feats = _t(sc.features)
    pv, vb = _front(qr, st, cams, W, H)
    per_view = [vb.view(pv, v) for v in range(len(cams))]
    views = [_view(pr, b, feats, None, W, H, D) for pr, b in per_view]
    bq = BatchedQuantile(views, K, D, L.QR_F32, qr.RenderParams().c())
    for kind, w in SHAPES:
        print("room batched launch", kind, w, flush=True)
        for v in views:
            v["out"].fill_(float("nan"))
            v["T_q"].fill_(float("nan"))
            v["n_sel"].fill_(-7)
        bq.render(kind, w)
        for i, (pr, b) in enumerate(per_view):
            ref = qr.render_quantile(pr, b, feats, W, H, K)
            torch.cuda.synchronize()
            assert torch.equal(views[i]["out"], ref["out"]), (kind, w, i)
            assert torch.equal(views[i]["T_q"], ref["T_q"]), (kind, w, i)
            assert torch.equal(views[i]["n_sel"], ref["n_sel"]), (kind, w, i)
            del ref
    # the maps of the last launch (persistent, longest list first) against the oracle
    for i in (0, 7):
        pr, b = per_view[i]
        offs = b.tile_offsets.cpu().numpy().astype(np.int64)
        lo, hi = int(offs[0]), int(offs[-1])
        gids = b.sorted_gid[lo:hi].cpu().numpy().astype(np.int64)
        offs = offs - lo
        lens = np.diff(offs)
        rng = np.random.default_rng(40 + i)
        tiles = [int(np.argmax(lens))] + [int(t) for t in rng.choice(np.nonzero(lens > 0)[0], 5, replace=False)]
        proj = proj_for_oracle(dict(means2d=pr.means2d.cpu().numpy(), conic_opacity=pr.conic_opacity.cpu().numpy()))
        ors = [oracle.render_quantile(proj, gids, offs, sc.features, W, H, K, tiles=tiles, bias=bb)
               for bb in (0.0, DECISION_WINDOW, -DECISION_WINDOW)]
        ev = ~np.isnan(ors[0]["out"][..., 0])
        out = views[i]["out"].cpu().numpy()
        st_ = compare_render(out, ors[0], ors[1:], evaluated=ev)
        clean = ev & (ors[0]["margin"] > DECISION_WINDOW)
        np.testing.assert_array_equal(views[i]["n_sel"].cpu().numpy()[clean], ors[0]["n_sel"][clean])
        np.testing.assert_allclose(views[i]["T_q"].cpu().numpy()[clean], ors[0]["T_q"][clean],
                                   rtol=1e-4, atol=1e-6)
        print("pose", i, "tiles", tiles, st_)


def test_reduced_batched_workload_fp8_forward_and_backward(qr):
    from paper_2512_20927_amd import _lib as L
    from paper_2512_20927_amd.batched import BatchedQuantile
    W, H, D, K = 1280, 720, 512, 8
    sizes, seeds, per = (75_000, 200_000, 375_000, 750_000), (10, 11, 12, 13), 2
    prm = qr.RenderParams().c()
    views, per_view, scene_of, scenes = [], [], [], []
    for si, (n, sd) in enumerate(zip(sizes, seeds)):
        sc = synth.make_room(n, sd, dim=D)
        st = _scene_t(sc)
        codes, scale = qr.quantize(_t(sc.features), "fp8")
        del sc
        cams = [synth.room_camera(300 + 8 * si + k, W, H, 1154.0) for k in range(per)]
        pv, vb = _front(qr, st, cams, W, H)
        scenes.append(dict(n=n, codes=codes, scale=scale, pv=pv, vb=vb))
        for k in range(per):
            pr, b = vb.view(pv, k)
            per_view.append((pr, b))
            scene_of.append(si)
            views.append(_view(pr, b, codes, scale, W, H, D))
    bq = BatchedQuantile(views, K, D, L.QR_FP8_E4M3, prm)
    for kind, w in (("heavy", 3), ("natural", 0)):
        print("reduced batched forward", kind, w, flush=True)
        for v in views:
            v["out"].fill_(float("nan"))
        bq.render(kind, w)
        for i, (pr, b) in enumerate(per_view):
            s = scenes[scene_of[i]]
            ref = qr.render_quantile(pr, b, s["codes"], W, H, K, feature_scale=s["scale"])
            torch.cuda.synchronize()
            assert torch.equal(views[i]["out"], ref["out"]), (kind, w, i)
            assert torch.equal(views[i]["T_q"], ref["T_q"]) and torch.equal(views[i]["n_sel"], ref["n_sel"])
            del ref
    # backward: one dL/d(out) buffer per view, gradients per scene
    gen = torch.Generator(device="cuda").manual_seed(5)
    gouts = [torch.randn(H, W, D, device="cuda", generator=gen) for _ in views]

    def zeros():
        return [[torch.zeros(s["n"], D, device="cuda"), torch.zeros(s["n"], 2, device="cuda"),
                 torch.zeros(s["n"], 4, device="cuda")] for s in scenes]

    ref = zeros()
    for i, (pr, b) in enumerate(per_view):
        s = scenes[scene_of[i]]
        g = ref[scene_of[i]]
        L.qr_render_quantile_backward(W, H, prm, K, b.tile_offsets, b.sorted_gid, pr.means2d,
                                      pr.conic_opacity, s["codes"], s["scale"], gouts[i], g[0], g[1], g[2])
    torch.cuda.synchronize()
    for kind, w in (("heavy", 2), ("natural", 0)):
        print("reduced batched backward", kind, w, flush=True)
        got = zeros()
        bq.set_grads([dict(grad_out=gouts[i], grad_features=got[si][0], grad_means2d=got[si][1],
                           grad_conic_opacity=got[si][2]) for i, si in enumerate(scene_of)])
        bq.backward(kind, w)
        torch.cuda.synchronize()
        for si in range(len(scenes)):
            for a, b in zip(got[si], ref[si]):
                assert float(b.abs().sum()) > 0
                a64, b64 = a.double(), b.double()
                rel = float((a64 - b64).norm() / b64.norm())
                # element-wise: the atomic additions reorder float32 sums of
                # terms no larger than the largest accumulated value
                worst = float((a64 - b64).abs().max() / b64.abs().max())
                assert rel <= 1e-5 and worst <= 1e-5, (kind, w, si, rel, worst)
        del got


def test_room_batched_dense_matches_single_view_and_oracle(qr):
    """The dense blend over the same 16 room poses, items and launch shapes
    as the batched Q-Render launch the benchmark times: bit-identical to the
    single-view dense kernel per pose; two poses' maps against the oracle on
    sampled tiles (with the longest list)."""
    from paper_2512_20927_amd import _lib as L
    from paper_2512_20927_amd.batched import BatchedDense
    cfg = synth.CONFIGS["room"]
    W, H, D = cfg["width"], cfg["height"], cfg["dim"]
    sc = synth.make_room(cfg["n"], cfg["seed"], dim=D)
    cams = synth.room_poses(cfg["pose_seeds"], W, H, cfg["fx"])
    st = _scene_t(sc)
    feats = _t(sc.features)
    pv, vb = _front(qr, st, cams, W, H)
    per_view = [vb.view(pv, v) for v in range(len(cams))]
    views = [_view(pr, b, feats, None, W, H, D) for pr, b in per_view]
    bd = BatchedDense(views, D, L.QR_F32, qr.RenderParams().c())
    for kind, w in SHAPES:
        print("room batched dense launch", kind, w, flush=True)
        for v in views:
            v["out"].fill_(float("nan"))
            v["T_q"].fill_(float("nan"))
            v["n_sel"].fill_(-7)
        bd.render(kind, w)
        for i, (pr, b) in enumerate(per_view):
            ref = qr.render_dense(pr, b, feats, W, H)
            torch.cuda.synchronize()
            assert torch.equal(views[i]["out"], ref["out"]), (kind, w, i)
            assert torch.equal(views[i]["T_q"], ref["T_final"]), (kind, w, i)
            assert torch.equal(views[i]["n_sel"], ref["n_contrib"]), (kind, w, i)
            del ref
    for i in (0, 7):
        pr, b = per_view[i]
        offs = b.tile_offsets.cpu().numpy().astype(np.int64)
        lo = int(offs[0])
        gids = b.sorted_gid[lo:int(offs[-1])].cpu().numpy().astype(np.int64)
        offs = offs - lo
        lens = np.diff(offs)
        rng = np.random.default_rng(60 + i)
        tiles = [int(np.argmax(lens))] + [int(t) for t in rng.choice(np.nonzero(lens > 0)[0], 4, replace=False)]
        proj = proj_for_oracle(dict(means2d=pr.means2d.cpu().numpy(), conic_opacity=pr.conic_opacity.cpu().numpy()))
        ors = [oracle.render_dense(proj, gids, offs, sc.features, W, H, tiles=tiles, bias=bb)
               for bb in (0.0, DECISION_WINDOW, -DECISION_WINDOW)]
        ev = ~np.isnan(ors[0]["out"][..., 0])
        st_ = compare_render(views[i]["out"].cpu().numpy(), ors[0], ors[1:], evaluated=ev)
        clean = ev & (ors[0]["margin"] > DECISION_WINDOW)
        np.testing.assert_array_equal(views[i]["n_sel"].cpu().numpy()[clean], ors[0]["n_contrib"][clean])
        np.testing.assert_allclose(views[i]["T_q"].cpu().numpy()[clean], ors[0]["T_final"][clean],
                                   rtol=1e-4, atol=1e-7)
        print("dense pose", i, "tiles", tiles, st_)
