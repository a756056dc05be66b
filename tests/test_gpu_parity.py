"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

* projection: float32 GPU vs float64 oracle, within rounding;
* binning: bit-exact sorted keys, Gaussian order and tile offsets when the
  oracle is fed the GPU's own float32 tile rectangles and depths;
* rendering: the oracle is fed the GPU's projected float32 records and its
  bins; per-pixel relative L2 error <= 1e-4 for float32 features on every
  pixel whose decisions are clear of their boundaries, identical quantile
  selections there, and agreement with a boundary-shifted oracle run on the
  few pixels with a decision within 1e-4 (relative) of its boundary.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.binning import depth_bits_key
from tests.parity_util import (DECISION_WINDOW, FP32_TOL, compare_render, compare_selection,
                               pixel_rel_err, proj_for_oracle)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_20927_amd as qr
    return qr


def _t(a, dtype=None):
    x = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        x = x.to(dtype)
    return x.cuda()


def gpu_pipeline(qr, sc, cam, K, storage="f32", dense=True, debug=True):
    W, H = cam.width, cam.height
    pr = qr.project(_t(sc.means), _t(sc.scales), _t(sc.quats), _t(sc.opacity), cam)
    bins = qr.bin_sort(pr, W, H, keep_keys=True)
    f32 = _t(sc.features)
    scale = None
    feats = f32
    if storage != "f32":
        feats, scale = qr.quantize(f32, storage)
    q = qr.render_quantile(pr, bins, feats, W, H, K, feature_scale=scale, debug=debug)
    d = qr.render_dense(pr, bins, feats, W, H, feature_scale=scale) if dense else None
    torch.cuda.synchronize()
    cpu = lambda t: t.cpu().numpy()
    P = int(bins.total_pairs.item())
    res = dict(
        pr=dict(means2d=cpu(pr.means2d), conic_opacity=cpu(pr.conic_opacity), depth=cpu(pr.depth),
                rect=cpu(pr.tile_rect), touched=cpu(pr.tiles_touched)),
        P=P, gids=cpu(bins.sorted_gid)[:P].astype(np.int64),
        keys=cpu(bins.sorted_keys)[:P].view(np.uint64), offs=cpu(bins.tile_offsets).astype(np.int64),
        q={k: cpu(v) for k, v in q.items()},
        feats=feats, scale=scale)
    if dense:
        res["d"] = {k: cpu(v) for k, v in d.items()}
    return res


def decoded_features(qr, sc, res, storage):
    if storage == "f32":
        return sc.features.astype(np.float64)
    if storage == "bf16":
        return oracle.quant.bf16_decode(res["feats"].view(torch.int16).cpu().numpy().view(np.uint16))
    return oracle.quant.e4m3_dequantize(res["feats"].cpu().numpy(), res["scale"].cpu().numpy())


def oracle_renders(res, feats, W, H, K, tiles=None, dense=True):
    proj = proj_for_oracle(res["pr"])
    out = {}
    for b in (0.0, DECISION_WINDOW, -DECISION_WINDOW):
        out[("q", b)] = oracle.render_quantile(proj, res["gids"], res["offs"], feats, W, H, K, tiles=tiles, bias=b)
        if dense:
            out[("d", b)] = oracle.render_dense(proj, res["gids"], res["offs"], feats, W, H, tiles=tiles, bias=b)
    return out


def check_selection(res, ors, evaluated):
    """Selections, their weights and T^Q against the oracle: identical ids
    on clean pixels, ids of the oracle or of a boundary-moved run on the
    others (parity_util.compare_selection); weights and T^Q on clean pixels
    within float32 rounding."""
    orq = ors[("q", 0.0)]
    st = compare_selection(res["q"]["sel_gid"], res["q"]["n_sel"], orq,
                           [ors[("q", DECISION_WINDOW)], ors[("q", -DECISION_WINDOW)]], evaluated)
    clean = evaluated & (orq["margin"] > DECISION_WINDOW)
    K = orq["sel_w"].shape[-1]
    w = res["q"]["sel_w"][clean][:, :K]
    np.testing.assert_allclose(w, orq["sel_w"][clean], rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(res["q"]["T_q"][clean], orq["T_q"][clean], rtol=1e-4, atol=1e-6)
    if "T_final" in res["q"]:  # Algorithm 1's T when the walk ends, last examined position
        np.testing.assert_allclose(res["q"]["T_final"][clean], orq["T_final"][clean], rtol=1e-4, atol=1e-6)
        np.testing.assert_array_equal(res["q"]["last_pos"][clean], orq["n_steps"][clean])
        st["T_final_checked"] = int(clean.sum())
    return st


def check_all(res, ors, W, H, tiles=None, dense=True):
    orq = ors[("q", 0.0)]
    ev = ~np.isnan(orq["out"][..., 0])
    st = {}
    st["q"] = compare_render(res["q"]["out"], orq, [ors[("q", DECISION_WINDOW)], ors[("q", -DECISION_WINDOW)]],
                             evaluated=ev)
    st["q"].update(check_selection(res, ors, ev))
    if dense:
        ord_ = ors[("d", 0.0)]
        st["d"] = compare_render(res["d"]["out"], ord_, [ors[("d", DECISION_WINDOW)], ors[("d", -DECISION_WINDOW)]],
                                 evaluated=ev)
        clean = ev & (ord_["margin"] > DECISION_WINDOW)
        np.testing.assert_allclose(res["d"]["T_final"][clean], ord_["T_final"][clean], rtol=1e-4, atol=1e-7)
        np.testing.assert_array_equal(res["d"]["n_contrib"][clean], ord_["n_contrib"][clean])
    print("parity stats", st)
    return st


# ---------------------------------------------------------------------------

def test_projection_matches_oracle(qr):
    for sc, cam in [(synth.make_tiny(0), synth.tiny_camera()),
                    (synth.make_room(200_000, 1, dim=16), synth.room_camera(100))]:
        res = gpu_pipeline(qr, sc, cam, 8, dense=False, debug=False)
        o = oracle.project(sc.means, sc.scales, sc.quats, sc.opacity, cam)
        g = res["pr"]
        vis = o["visible"] & (g["touched"] > 0)
        # visibility agrees except where a float32/float64 boundary straddles
        assert np.mean(o["visible"] != (g["touched"] > 0)) < 1e-3
        np.testing.assert_allclose(g["means2d"][vis], o["means2d"][vis], rtol=1e-5, atol=2e-3)
        np.testing.assert_allclose(g["depth"][vis], o["depth"][vis], rtol=2e-6, atol=1e-6)
        ec = np.linalg.norm(g["conic_opacity"][vis, :3] - o["conic"][vis], axis=1) / np.linalg.norm(o["conic"][vis], axis=1)
        assert np.median(ec) < 1e-6 and ec.max() < 1e-3, (np.median(ec), ec.max())
        rect_diff = np.abs(g["rect"][vis] - o["rect"][vis])
        assert rect_diff.max() <= 1
        assert np.mean(np.any(rect_diff > 0, axis=1)) < 1e-3


@pytest.mark.parametrize("case", ["tiny", "ragged", "room", "many_tiles"])
def test_bin_sort_bit_exact(qr, case):
    """"many_tiles" (3840 x 2400: 36,000 tiles) takes the multi-workgroup
    scan of the tile counters; the other images the single-workgroup one."""
    if case == "tiny":
        sc, cam = synth.make_tiny(0), synth.tiny_camera()
    elif case == "ragged":
        sc, cam = synth.make_tiny(3, n=3000, dim=16), synth.tiny_camera(100)
        cam.height = 75
        cam.cy = 37.5
    elif case == "room":
        sc, cam = synth.make_room(200_000, 1, dim=16), synth.room_camera(100)
    else:
        sc, cam = synth.make_room(20_000, 4, dim=16), synth.room_camera(101, 3840, 2400, 3462.0)
    res = gpu_pipeline(qr, sc, cam, 8, dense=False, debug=False)
    tx, ty = (cam.width + 15) // 16, (cam.height + 15) // 16
    g = res["pr"]
    gids, offs, triples = oracle.bin_sort(g["rect"], g["depth"], tx, ty)
    assert res["P"] == gids.size == int(g["touched"].sum())
    np.testing.assert_array_equal(res["gids"], gids)
    np.testing.assert_array_equal(res["offs"], offs)
    want_keys = np.array([depth_bits_key(t, np.float32(d)) for t, d, _ in triples], dtype=np.uint64)
    np.testing.assert_array_equal(res["keys"], want_keys)


@pytest.mark.parametrize("n", [1500, 6000])
def test_bin_sort_long_tile_lists(qr, n):
    """n large Gaussians over a 64x64 image put ~n entries in every tile
    list: 1,500 is longer than one key per thread and takes the tile's LDS
    bitonic sort; 6,000 is longer than the LDS holds and takes the per-tile
    radix sort through global scratch. Ties in depth are forced."""
    rng = np.random.default_rng(8)
    means = np.zeros((n, 3), np.float32)
    means[:, :2] = rng.uniform(-0.2, 0.2, (n, 2))
    means[:, 2] = rng.integers(0, 50, n) * np.float32(0.01)  # repeated depths
    sc = synth.Scene(means, np.full((n, 3), 0.6, np.float32), np.tile(np.float32([1, 0, 0, 0]), (n, 1)),
                     np.full(n, 0.5, np.float32), rng.standard_normal((n, 16)).astype(np.float32))
    cam = synth.tiny_camera()
    res = gpu_pipeline(qr, sc, cam, 8, dense=True, debug=True)
    g = res["pr"]
    gids, offs, triples = oracle.bin_sort(g["rect"], g["depth"], 4, 4)
    longest = np.diff(offs).max()
    assert (longest > 2048) if n > 2048 else (256 < longest <= 2048)
    np.testing.assert_array_equal(res["gids"], gids)
    np.testing.assert_array_equal(res["offs"], offs)
    want_keys = np.array([depth_bits_key(t, np.float32(d)) for t, d, _ in triples], dtype=np.uint64)
    np.testing.assert_array_equal(res["keys"], want_keys)
    ors = oracle_renders(res, sc.features.astype(np.float64), 64, 64, 8, tiles=[0, 5, 15])
    check_all(res, ors, 64, 64, tiles=[0, 5, 15])


def test_render_parity_tiny(qr):
    sc, cam = synth.make_tiny(0), synth.tiny_camera()
    res = gpu_pipeline(qr, sc, cam, 8)
    ors = oracle_renders(res, sc.features.astype(np.float64), 64, 64, 8)
    check_all(res, ors, 64, 64)


@pytest.mark.parametrize("dim,K", [(16, 8), (16, 32), (48, 8), (128, 8), (128, 32), (144, 8), (144, 32), (1040, 4)])
def test_render_parity_feature_widths(qr, dim, K):
    """Rows of at most 128 features take the gather that blends all groups of
    a wave side by side (4, 16 or 32 lanes per group); 144 takes the
    column-pass gather with a partial pass, 1040 three passes. K = 32 puts
    groups past the distinct-selection capacity onto the per-pixel path."""
    sc = synth.make_tiny(5, n=3000, dim=dim)
    cam = synth.tiny_camera(100)
    cam.height, cam.cy = 75, 37.5
    res = gpu_pipeline(qr, sc, cam, K, dense=False)
    ors = oracle_renders(res, sc.features.astype(np.float64), 100, 75, K, dense=False)
    check_all(res, ors, 100, 75, dense=False)
    if K == 32:  # some 4-pixel groups (x = 4k .. 4k+3 of a row) exceed 16 distinct selections
        sg = ors[("q", 0.0)]["sel_gid"][:, :96].reshape(75, 24, 4 * K)
        distinct = np.array([[len(set(r[r >= 0].tolist())) for r in row] for row in sg])
        assert (distinct > 16).sum() > 10, (distinct > 16).sum()


@pytest.mark.parametrize("K", [1, 4, 32, 40, 50, 64])
def test_render_parity_ragged_image(qr, K):
    """K = 40 is the paper's trained setting, 50 the top of its K sweep, 64
    the largest the library takes."""
    sc = synth.make_tiny(3, n=3000, dim=32)
    cam = synth.tiny_camera(100)
    cam.height, cam.cy = 75, 37.5
    res = gpu_pipeline(qr, sc, cam, K)
    ors = oracle_renders(res, sc.features.astype(np.float64), 100, 75, K)
    check_all(res, ors, 100, 75)
    assert res["q"]["n_sel"].max() <= K


@pytest.mark.parametrize("dim", [48, 80])
def test_render_parity_feature_width_not_multiple_of_64(qr, dim):
    """Feature widths that leave a partial staged column chunk."""
    sc = synth.make_tiny(12, n=2500, dim=dim)
    cam = synth.tiny_camera(72)
    res = gpu_pipeline(qr, sc, cam, 8)
    ors = oracle_renders(res, sc.features.astype(np.float64), 72, 72, 8)
    check_all(res, ors, 72, 72)


def test_render_parity_many_distinct_selections(qr):
    """30,000 pixel-sized, nearly opaque Gaussians: every pixel selects its
    own few, so a tile holds hundreds of distinct selected Gaussians - more
    than the per-tile LDS staging takes - and the direct gather is used."""
    rng = np.random.default_rng(21)
    n = 30_000
    sc = synth.Scene(rng.uniform(-1.0, 1.0, (n, 3)).astype(np.float32),
                     np.full((n, 3), 0.004, np.float32), synth.scenes._unit_quats(rng, n),
                     rng.uniform(0.5, 0.99, n).astype(np.float32),
                     rng.standard_normal((n, 32)).astype(np.float32))
    cam = synth.tiny_camera(64)
    res = gpu_pipeline(qr, sc, cam, 8)
    uniq = [len(set(res["q"]["sel_gid"][y:y + 16, x:x + 16].ravel()) - {-1})
            for y in range(0, 64, 16) for x in range(0, 64, 16)]
    assert max(uniq) > 128, uniq
    ors = oracle_renders(res, sc.features.astype(np.float64), 64, 64, 8)
    check_all(res, ors, 64, 64)


@pytest.fixture(scope="module")
def room_res(qr):
    sc = synth.make_room(200_000, 1, dim=512)
    cam = synth.room_camera(100)
    res = gpu_pipeline(qr, sc, cam, 8)
    return sc, cam, res


def _sample_tiles(res, n, seed):
    lens = np.diff(res["offs"])
    rng = np.random.default_rng(seed)
    heavy = int(np.argmax(lens))
    others = rng.choice(np.nonzero(lens > 0)[0], n - 1, replace=False)
    return [heavy] + [int(t) for t in others]


def test_render_parity_room_full_size_sampled_tiles(qr, room_res):
    """640x480, 200k Gaussians, 512-D float32, K=8: the full frame on the GPU
    in the benchmark's launch configuration; the oracle on sampled tiles,
    the tile with the longest list among them."""
    sc, cam, res = room_res
    tiles = _sample_tiles(res, 10, 0)
    ors = oracle_renders(res, sc.features, cam.width, cam.height, 8, tiles=tiles)
    check_all(res, ors, cam.width, cam.height, tiles=tiles)
    # whole-frame properties that hold at any size
    q = res["q"]
    assert q["n_sel"].max() <= 8 and q["n_sel"].min() >= 0
    has = q["n_sel"] > 0
    assert np.all(q["out"][~has] == 0)
    d = res["d"]
    assert np.all((d["T_final"] >= 1e-4 * (1 - 1e-6)) & (d["T_final"] <= 1.0))
    assert np.all(np.isfinite(q["out"])) and np.all(np.isfinite(d["out"]))


@pytest.mark.parametrize("scale", [1.0, 0.3711])
def test_fp8_decode_of_every_code(qr, scale):
    """One Gaussian whose feature row holds every finite e4m3 code (all but
    0x7F and 0xFF). A pixel that selects only this Gaussian has
    out = (alpha f) / alpha = f, so Q-Render and the dense blend must
    return the decoded row times the scale: each code's value against the
    format definition (oracle table), byte order in the 4-byte loads
    included."""
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)] + [0, 0], np.uint8)
    sc = synth.Scene(np.zeros((1, 3), np.float32), np.full((1, 3), 0.3, np.float32),
                     np.float32([[1, 0, 0, 0]]), np.float32([0.9]), np.zeros((1, 256), np.float32))
    cam = synth.tiny_camera(32)
    pr = qr.project(_t(sc.means), _t(sc.scales), _t(sc.quats), _t(sc.opacity), cam)
    bins = qr.bin_sort(pr, 32, 32)
    feats = _t(codes[None, :])
    sc_t = torch.tensor([scale], dtype=torch.float32, device="cuda")
    q = qr.render_quantile(pr, bins, feats, 32, 32, 8, feature_scale=sc_t)
    d = qr.render_dense(pr, bins, feats, 32, 32, feature_scale=sc_t)
    torch.cuda.synchronize()
    want = oracle.quant.e4m3_decode(codes) * np.float64(np.float32(scale))
    nz = want != 0
    assert int(q["n_sel"][16, 16].item()) == 1

    def check(got, spread):
        # every code decoded exactly: got = want * (common factor), up to the
        # roundings of the products that follow the decode
        assert np.all(got[~nz] == 0)
        ratio = got[nz] / want[nz]
        assert np.ptp(ratio) <= spread * np.abs(ratio).max(), np.ptp(ratio)
        assert abs(ratio.mean() - 1.0) < 1e-4

    # Q-Render: float32 scale, weight and normalisation products
    check(q["out"][16, 16].cpu().numpy().astype(np.float64), 6e-7)
    # dense: out = alpha f with T_final = 1 - alpha; its bf16 hi/lo split
    # product is exact to below 2^-16 relative
    alpha = 1.0 - float(d["T_final"][16, 16].item())
    check(d["out"][16, 16].cpu().numpy().astype(np.float64) / alpha, 2.0 ** -15)


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_quantized_storage(qr, storage):
    """Storage codes are bit-exact with the oracle's encoder; the kernels on
    decoded features match the oracle to float32 tolerance (kernel error);
    the error from storage itself is measured against float32 features."""
    sc = synth.make_room(200_000, 1, dim=512)
    cam = synth.room_camera(101)
    res = gpu_pipeline(qr, sc, cam, 8, storage=storage)
    f = sc.features
    if storage == "bf16":
        codes = res["feats"].view(torch.int16).cpu().numpy().view(np.uint16)
        np.testing.assert_array_equal(codes, oracle.quant.bf16_encode(f))
    else:
        want_codes, want_scale = oracle.quant.e4m3_quantize(f)
        np.testing.assert_array_equal(res["scale"].cpu().numpy(), want_scale)
        np.testing.assert_array_equal(res["feats"].cpu().numpy(), want_codes)
    tiles = _sample_tiles(res, 6, 1)
    dec = decoded_features(qr, sc, res, storage)
    ors = oracle_renders(res, dec, cam.width, cam.height, 8, tiles=tiles)
    check_all(res, ors, cam.width, cam.height, tiles=tiles)
    # storage error against the float32 features (reported; bound only for bf16)
    orig = oracle.render_quantile(proj_for_oracle(res["pr"]), res["gids"], res["offs"], f,
                                  cam.width, cam.height, 8, tiles=tiles)
    ev = ~np.isnan(orig["out"][..., 0]) & (orig["n_sel"] > 0)
    e = pixel_rel_err(res["q"]["out"][ev], orig["out"][ev])
    print("%s storage error vs float32 features: max %.3e p99 %.3e mean %.3e" % (storage, e.max(), np.percentile(e, 99), e.mean()))
    if storage == "bf16":
        assert e.max() < 1e-2


def test_forward_is_deterministic(qr):
    sc, cam = synth.make_tiny(4, n=5000, dim=64), synth.tiny_camera(128)
    a = gpu_pipeline(qr, sc, cam, 8)
    b = gpu_pipeline(qr, sc, cam, 8)
    for k in ("out", "T_q", "n_sel", "sel_gid", "sel_w"):
        np.testing.assert_array_equal(a["q"][k], b["q"][k])
    for k in ("out", "T_final", "n_contrib"):
        np.testing.assert_array_equal(a["d"][k], b["d"][k])
    np.testing.assert_array_equal(a["gids"], b["gids"])


def test_edge_cases(qr):
    # every Gaussian culled (camera looking away): empty bins, zero maps
    sc = synth.make_tiny(0)
    cam = synth.tiny_camera()
    cam.t = np.array([0.0, 0.0, -3.0], np.float32)  # scene behind the camera
    res = gpu_pipeline(qr, sc, cam, 8)
    assert res["P"] == 0 and np.all(res["offs"] == 0)
    assert np.all(res["q"]["out"] == 0) and np.all(res["q"]["n_sel"] == 0)
    assert np.all(res["d"]["out"] == 0) and np.all(res["d"]["T_final"] == 1)
    # a single Gaussian: dense = alpha' f, quantile = f where selected
    one = synth.Scene(np.zeros((1, 3), np.float32), np.full((1, 3), 0.3, np.float32),
                      np.array([[1, 0, 0, 0]], np.float32), np.array([0.9], np.float32),
                      np.arange(16, dtype=np.float32)[None, :])
    res = gpu_pipeline(qr, one, synth.tiny_camera(), 1)
    d, q = res["d"], res["q"]
    alpha = 1 - d["T_final"]
    np.testing.assert_allclose(d["out"], alpha[..., None] * one.features[0], rtol=1e-4, atol=1e-5)
    sel = q["n_sel"] == 1
    assert sel.any() and np.all(q["n_sel"] <= 1)
    np.testing.assert_allclose(q["out"][sel], np.broadcast_to(one.features[0], q["out"][sel].shape), rtol=1e-6)
    # K=1 on a one-Gaussian ray selects iff alpha' > 1/2
    np.testing.assert_array_equal(sel, alpha > 0.5)
    # N = 0
    empty = synth.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                        np.zeros((0, 4), np.float32), np.zeros(0, np.float32), np.zeros((0, 16), np.float32))
    res = gpu_pipeline(qr, empty, synth.tiny_camera(), 8)
    assert res["P"] == 0 and np.all(res["q"]["out"] == 0) and np.all(res["d"]["out"] == 0)


def test_hip_graph_replay_matches_eager(qr):
    """The whole frame (project, bin_sort, both renderers) captured in one HIP
    graph: every replay, with other eager work and output scrambling in
    between, reproduces the eager result bit for bit."""
    from paper_2512_20927_amd import _lib as L
    sc = synth.make_room(20_000, 5, dim=64)
    cam = synth.room_camera(130, 160, 120, 144.0)
    W, H = cam.width, cam.height
    s = [_t(a) for a in (sc.means, sc.scales, sc.quats, sc.opacity)]
    feats = _t(sc.features)
    pr = qr.project(*s, cam)
    binner = qr.Binner(sc.n, W, H, qr.count_pairs(pr) + 1024)
    prm, camc = qr.RenderParams().c(), L.make_camera(cam)
    outq = torch.empty(H, W, 64, device="cuda")
    outd = torch.empty(H, W, 64, device="cuda")
    tq = torch.empty(H, W, device="cuda")
    ns = torch.empty(H, W, dtype=torch.int32, device="cuda")

    def frame():
        L.qr_project(*s, camc, prm, pr.means2d, pr.conic_opacity, pr.depth, pr.tile_rect, pr.tiles_touched)
        b = binner(pr)
        L.qr_render_quantile(W, H, prm, 8, b.tile_offsets, b.sorted_gid, pr.means2d, pr.conic_opacity,
                             feats, None, outq, tq, ns)
        L.qr_render_dense(W, H, prm, b.tile_offsets, b.sorted_gid, pr.means2d, pr.conic_opacity,
                          feats, None, outd, None, None)

    frame()
    torch.cuda.synchronize()
    ref = [outq.clone(), outd.clone(), tq.clone(), ns.clone()]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        frame()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        frame()
    other = synth.room_camera(131, 160, 120, 144.0)
    for i in range(3):
        for t in (outq, outd, tq):
            t.fill_(float("nan"))
        ns.fill_(-1)
        # eager work between replays: another view rendered with fresh buffers
        qr.render_quantile(qr.project(*s, other), qr.bin_sort(qr.project(*s, other), W, H),
                           feats, W, H, 8)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((outq, outd, tq, ns), ref):
            assert torch.equal(a, b), i


def test_render_parity_precision_full_size_sampled_tiles(qr):
    """1M Gaussians, 1296x968, 512-D bf16 storage, K = 8: full frame on the
    GPU, oracle on sampled tiles with the decoded features (kernel error),
    storage error against the float32 features reported."""
    cfg = synth.CONFIGS["precision"]
    sc = synth.make_room(cfg["n"], cfg["seed"], dim=cfg["dim"])
    cam = synth.room_poses(cfg["pose_seeds"][:1], cfg["width"], cfg["height"], cfg["fx"])[0]
    res = gpu_pipeline(qr, sc, cam, 8, storage="bf16")
    tiles = _sample_tiles(res, 5, 3)
    dec = decoded_features(qr, sc, res, "bf16")
    ors = oracle_renders(res, dec, cam.width, cam.height, 8, tiles=tiles)
    check_all(res, ors, cam.width, cam.height, tiles=tiles)
    orig = oracle.render_quantile(proj_for_oracle(res["pr"]), res["gids"], res["offs"], sc.features,
                                  cam.width, cam.height, 8, tiles=tiles)
    ev = ~np.isnan(orig["out"][..., 0]) & (orig["n_sel"] > 0)
    e = pixel_rel_err(res["q"]["out"][ev], orig["out"][ev])
    print("precision config bf16 storage error: max %.3e mean %.3e" % (e.max(), e.mean()))
    assert e.max() < 1e-2
