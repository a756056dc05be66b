"""Pins of the oracle renderers: dense alpha-blend (Eq. 1) and Quantile
Rendering (Algorithm 1, Sec. 4.2) against hand-worked rays, brute force,
closed forms, invariants and the interval form of the selection."""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from oracle.render import quantile_thresholds

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "alg1_hand_examples.json")


def ray_case(alphas, D=None):
    """One 1x1 image whose single tile list is the given ray: every Gaussian has
    a zero conic, so alpha' = min(alpha_max, o) at the pixel."""
    n = len(alphas)
    D = n if D is None else D
    proj = dict(means2d=np.zeros((n, 2)), conic=np.zeros((n, 3)),
                opacity=np.asarray(alphas, np.float64))
    feats = np.eye(n, D)
    return proj, np.arange(n), np.array([0, n]), feats


def _frac(s):
    return float(Fraction(s))


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_hand_worked_examples(ex):
    K = ex["K"]
    proj, gids, offs, feats = ray_case(ex["alphas"])
    q = oracle.render_quantile(proj, gids, offs, feats, 1, 1, K)
    n = len(ex["selected"])
    assert q["n_sel"][0, 0] == n
    assert q["sel_pos"][0, 0, :n].tolist() == ex["selected"]
    np.testing.assert_allclose(q["sel_w"][0, 0, :n], [_frac(w) for w in ex["weights"]], rtol=1e-14)
    assert q["T_q"][0, 0] == pytest.approx(_frac(ex["T_q"]), rel=1e-14)
    np.testing.assert_allclose(q["out"][0, 0], [_frac(v) for v in ex["output"]], rtol=1e-14, atol=1e-15)
    # the scalar brute-force walk and the interval form agree
    f, TQ, chosen = brute.ray_quantile(ex["alphas"], feats.tolist(), K, feats.shape[1])
    assert chosen == ex["selected"]
    assert oracle.interval_selection(ex["alphas"], K) == ex["selected"]
    if "dense_output" in ex:
        d = oracle.render_dense(proj, gids, offs, feats, 1, 1)
        np.testing.assert_allclose(d["out"][0, 0], [_frac(v) for v in ex["dense_output"]], rtol=1e-14)
        assert d["T_final"][0, 0] == pytest.approx(_frac(ex["dense_T_final"]), rel=1e-14)


def test_thresholds():
    np.testing.assert_allclose(quantile_thresholds(3), [0.75, 0.5, 0.25])
    assert quantile_thresholds(1).tolist() == [0.5]


def _check_tiled_equals_brute(sc, cam, K, prm=oracle.RenderParams()):
    pr = oracle.project(sc.means, sc.scales, sc.quats, sc.opacity, cam, prm)
    tx = (cam.width + 15) // 16
    ty = (cam.height + 15) // 16
    gids, offs, _ = oracle.bin_sort(pr["rect"], pr["depth"], tx, ty)
    d = oracle.render_dense(pr, gids, offs, sc.features, cam.width, cam.height, prm)
    q = oracle.render_quantile(pr, gids, offs, sc.features, cam.width, cam.height, K, prm)
    bd = oracle.brute_force_render(pr, sc.features, cam.width, cam.height, prm)
    bq = oracle.brute_force_render(pr, sc.features, cam.width, cam.height, prm, K=K)
    np.testing.assert_allclose(d["out"], bd["out"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(d["T_final"], bd["T"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(q["out"], bq["out"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(q["T_q"], bq["T"], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(q["n_sel"], bq["n"])
    return d, q


def test_tiled_equals_brute_force_tiny(tiny_case):
    sc, cam = tiny_case["scene"], tiny_case["cam"]
    d, q = _check_tiled_equals_brute(sc, cam, 8)
    assert np.nanmean(d["n_contrib"]) > 5 and np.nanmean(q["n_sel"]) > 1


def test_tiled_equals_brute_force_ragged_image():
    sc = synth.make_tiny(11, n=400, dim=8)
    cam = synth.Camera(np.eye(3, dtype=np.float32), np.array([0.1, -0.2, 3.0], np.float32),
                       40.0, 44.0, 25.0, 18.5, 50, 37, 0.2)
    _check_tiled_equals_brute(sc, cam, 4)


# Algorithm 1's full transmittance T when the walk ends and the position of
# the last entry it examined, walked by hand on the golden rays (the stop test
# breaks before T takes the stopping entry's T_test):
#   A (K=3, 0.5 x4): T 1 -> 1/2 -> 1/4; entry 2 crosses t_3 = 1/4 and stops -> T = 1/4, 3 entries
#   B (K=3, 0.2 x8): entry 6 (T_test = 0.2097152) stops; T = 0.8^6 = 0.262144, 7 entries
#   C (K=3, 0.9, ...): entry 0 crosses all three thresholds and stops -> T = 1, 1 entry
#   D (K=1, 0.3 x4): entry 1 (T_test = 0.49 < 1/2) stops -> T = 0.7, 2 entries
#   F (K=3, 0.1): no stop, the list ends -> T = 0.9, 1 entry
HAND_T_FINAL = {"A_strict_threshold": ("1/4", 3), "B_residual_transmittance": ("4096/15625", 7),
                "C_one_step_crosses_all": ("1", 1), "D_median_K1": ("7/10", 2),
                "F_nothing_selected": ("9/10", 1)}


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_hand_worked_final_transmittance(ex):
    if ex["name"] not in HAND_T_FINAL:
        pytest.skip("no hand value")
    T_fin, last = HAND_T_FINAL[ex["name"]]
    proj, gids, offs, feats = ray_case(ex["alphas"])
    q = oracle.render_quantile(proj, gids, offs, feats, 1, 1, ex["K"])
    assert q["T_final"][0, 0] == pytest.approx(_frac(T_fin), rel=1e-14)
    assert q["n_steps"][0, 0] == last


def test_final_transmittance_of_unstopped_rays_is_the_full_product(tiny_case):
    """A ray that never takes the stop test (k < K at the end of its list)
    has T = the product of (1 - alpha') over its whole list: the dense blend
    with T_eps = 0 (no stop) gives the same value; a stopped ray ends with
    T >= 1/(K+1) (T before the stopping entry passed the stop test)."""
    tc = tiny_case
    K = 8
    feats = tc["scene"].features
    q = oracle.render_quantile(tc["proj"], tc["gids"], tc["offs"], feats, 64, 64, K, tc["params"])
    prm0 = oracle.RenderParams(T_eps=0.0)
    d = oracle.render_dense(tc["proj"], tc["gids"], tc["offs"], feats, 64, 64, prm0)
    unstopped = q["k"] < K
    assert unstopped.mean() > 0.2 and (~unstopped).mean() > 0.1
    np.testing.assert_allclose(q["T_final"][unstopped], d["T_final"][unstopped], rtol=1e-12)
    assert np.all(q["T_final"][~unstopped] >= 1.0 / (K + 1) * (1 - 1e-12))
    assert np.all(q["T_final"][unstopped] <= 1.0)


def test_partition_of_unity_and_constant_features(tiny_case):
    """Sum_i w_i + T_final = 1, hence a constant feature c renders (1-T_final) c
    densely; quantile weights satisfy sum w^Q + T^Q = 1, so Q renders c."""
    tc = tiny_case
    n = tc["scene"].n
    c = np.array([[0.5, -2.0, 3.0]])
    feats = np.repeat(c, n, 0)
    d = oracle.render_dense(tc["proj"], tc["gids"], tc["offs"], feats, 64, 64, tc["params"])
    np.testing.assert_allclose(d["out"], (1 - d["T_final"])[..., None] * c, atol=1e-13)
    q = oracle.render_quantile(tc["proj"], tc["gids"], tc["offs"], feats, 64, 64, 8, tc["params"])
    has = q["n_sel"] > 0
    np.testing.assert_allclose(q["out"][has], np.broadcast_to(c, q["out"][has].shape), rtol=1e-12)
    assert np.all(q["out"][~has] == 0)
    assert np.all(q["n_sel"] <= 8) and np.all(q["n_sel"] <= q["k"])
    np.testing.assert_allclose(q["sel_w"].sum(-1) + q["T_q"], 1.0, atol=1e-13)
    assert has.mean() > 0.3


def test_single_and_two_gaussian_closed_forms():
    a1, a2 = 0.3, 0.6
    proj, gids, offs, feats = ray_case([a1])
    d = oracle.render_dense(proj, gids, offs, feats, 1, 1)
    assert d["out"][0, 0, 0] == pytest.approx(a1)
    proj, gids, offs, feats = ray_case([a1, a2])
    d = oracle.render_dense(proj, gids, offs, feats, 1, 1)
    np.testing.assert_allclose(d["out"][0, 0], [a1, (1 - a1) * a2], rtol=1e-15)
    assert d["T_final"][0, 0] == pytest.approx((1 - a1) * (1 - a2))
    # K = 2 (t = 2/3, 1/3): 0.7 -> no; 0.28 crosses both; only entry 1 selected
    q = oracle.render_quantile(proj, gids, offs, feats, 1, 1, 2)
    assert q["sel_pos"][0, 0].tolist() == [1, -1]
    np.testing.assert_allclose(q["out"][0, 0], [0.0, 1.0])


def test_interval_form_equals_algorithm_on_random_rays():
    rng = np.random.default_rng(42)
    mism = 0
    for r in range(100_000):
        n = int(rng.integers(0, 30))
        K = int(rng.integers(1, 17))
        kind = r % 3
        if kind == 0:
            al = rng.uniform(1 / 255, 0.99, n)
        elif kind == 1:
            al = rng.beta(0.5, 3.0, n) * 0.99
        else:
            al = np.full(n, rng.choice([0.5, 0.25, 0.75]))  # exact binary steps, ties
        _, _, chosen = brute.ray_quantile(al.tolist(), [[]] * n, K, 0)
        if chosen != oracle.interval_selection(al, K):
            mism += 1
        assert len(chosen) <= K
    assert mism == 0


def test_K1_selects_the_median_crossing():
    rng = np.random.default_rng(5)
    for _ in range(200):
        al = rng.uniform(0.05, 0.6, 12)
        T = np.cumprod(1 - al)
        first = int(np.argmax(T < 0.5)) if np.any(T < 0.5) else None
        _, _, chosen = brute.ray_quantile(al.tolist(), [[]] * 12, 1, 0)
        assert chosen == ([] if first is None else [first])


def test_large_K_limit_selects_every_entry():
    """If every step lowers T by more than 1/(K+1), each step crosses a
    threshold: Q-Render selects all entries and equals the dense blend
    normalised by its opacity, C / (1 - T_final) (with T_eps = 0)."""
    al = [0.3, 0.25, 0.4, 0.35, 0.3]
    K = 30
    T = np.concatenate([[1.0], np.cumprod(1 - np.array(al))])
    assert np.all(-np.diff(T) > 1 / (K + 1))
    proj, gids, offs, feats = ray_case(al, D=4)
    feats = np.random.default_rng(0).standard_normal((5, 4))
    prm = oracle.RenderParams(T_eps=0.0)
    q = oracle.render_quantile(proj, gids, offs, feats, 1, 1, K, prm)
    d = oracle.render_dense(proj, gids, offs, feats, 1, 1, prm)
    assert q["n_sel"][0, 0] == 5
    np.testing.assert_allclose(q["out"][0, 0], d["out"][0, 0] / (1 - d["T_final"][0, 0]), rtol=1e-13)


def test_alpha_min_filter_and_clamp():
    prm = oracle.RenderParams()
    # o below alpha_min: not on the ray; o above alpha_max: clamped
    proj, gids, offs, feats = ray_case([0.5 / 255, 1.0])
    d = oracle.render_dense(proj, gids, offs, feats, 1, 1, prm)
    np.testing.assert_allclose(d["out"][0, 0], [0.0, 0.99])


# -- planted mistakes: each must make one of the pins above fail -------------

def _expect_failure(fn):
    with pytest.raises(AssertionError):
        fn()


def test_planted_mistakes_are_caught(monkeypatch, tiny_case):
    import oracle.render as R
    ex = {e["name"]: e for e in _golden()}
    # (1) "<=" instead of "<" at a threshold
    orig_thr = R.quantile_thresholds
    monkeypatch.setattr(R, "quantile_thresholds", lambda K: np.nextafter(orig_thr(K), 2.0))
    _expect_failure(lambda: test_hand_worked_examples(ex["A_strict_threshold"]))
    monkeypatch.setattr(R, "quantile_thresholds", orig_thr)
    # (2) wrong sign of the conic's off-diagonal term
    orig_alpha = R._alpha

    def bad_alpha(proj, g, xs, ys, params):
        p2 = dict(proj)
        p2["conic"] = proj["conic"] * np.array([1.0, -1.0, 1.0])
        return orig_alpha(p2, g, xs, ys, params)
    monkeypatch.setattr(R, "_alpha", bad_alpha)
    _expect_failure(lambda: test_tiled_equals_brute_force_tiny(tiny_case))
    monkeypatch.setattr(R, "_alpha", orig_alpha)
    # (3) transmittance updated before the weight is taken: w = alpha T_{i+1}
    orig_w = R._dense_weight
    monkeypatch.setattr(R, "_dense_weight", lambda alpha, T_before, T_after: alpha * T_after)
    _expect_failure(lambda: test_partition_of_unity_and_constant_features(tiny_case))
    monkeypatch.setattr(R, "_dense_weight", orig_w)
