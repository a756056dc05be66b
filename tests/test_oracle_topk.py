"""Pins of the Top-K oracle: hand-worked single rays (exact binary
fractions, including a tie in weight and a ray where ranking by alpha' would
pick differently), brute force over every K-subset of a ray's candidates on
random rays, the limit of a K no smaller than the candidate count (the dense
blend normalised by 1 - T_final, the dense oracle being pinned on its own),
and invariants (constant features, empty rays)."""

import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle.params import RenderParams


def _ray(alphas):
    """One pixel (a 1x1 image) whose ray meets Gaussians of alpha' = alphas
    in this order (zero conic: alpha' = min(alpha_max, opacity))."""
    n = len(alphas)
    proj = dict(means2d=np.full((n, 2), 0.5), conic=np.zeros((n, 3)), opacity=np.asarray(alphas, np.float64))
    return proj, np.arange(n), np.array([0, n])


def _one_hot(n):
    return np.eye(n)


def test_hand_example_half_alphas():
    proj, gid, offs = _ray([0.5] * 4)  # w = 1/2, 1/4, 1/8, 1/16
    r = oracle.render_topk(proj, gid, offs, _one_hot(4), 1, 1, 2)
    assert r["n_sel"][0, 0] == 2
    np.testing.assert_array_equal(r["sel_pos"][0, 0], [0, 1])
    np.testing.assert_array_equal(r["sel_w"][0, 0], [0.5, 0.25])
    np.testing.assert_allclose(r["out"][0, 0], [2 / 3, 1 / 3, 0, 0], atol=1e-15)
    assert r["T_q"][0, 0] == 0.25


def test_hand_example_weight_not_alpha():
    proj, gid, offs = _ray([0.6, 0.7])  # w = 0.6, 0.28: by alpha' the second would win
    r = oracle.render_topk(proj, gid, offs, _one_hot(2), 1, 1, 1)
    np.testing.assert_array_equal(r["sel_pos"][0, 0], [0])
    np.testing.assert_allclose(r["out"][0, 0], [1, 0], atol=1e-15)
    np.testing.assert_allclose(r["T_q"][0, 0], 0.4, atol=1e-15)


def test_hand_example_tie_goes_to_the_earlier():
    proj, gid, offs = _ray([0.5, 0.25, 1 / 3])  # w = 1/2, 1/8, 1/8 exactly in float64
    r = oracle.render_topk(proj, gid, offs, _one_hot(3), 1, 1, 2)
    np.testing.assert_array_equal(r["sel_pos"][0, 0], [0, 1])
    np.testing.assert_allclose(r["out"][0, 0], [0.8, 0.2, 0], atol=1e-15)
    assert r["margin"][0, 0] == 0.0  # an exact tie is a boundary decision


def test_dense_stop_and_alpha_min_define_the_candidates():
    # alpha' below alpha_min is not on the ray; after 0.99 twice T = 1e-4 and the
    # third entry would take T below T_eps: it is not blended, so not a candidate
    proj, gid, offs = _ray([0.001, 0.99, 0.99, 0.99])
    r = oracle.render_topk(proj, gid, offs, _one_hot(4), 1, 1, 8)
    assert r["n_cand"][0, 0] == 2
    np.testing.assert_array_equal(r["sel_pos"][0, 0, :2], [1, 2])


def test_empty_ray_is_zero():
    proj, gid, offs = _ray([0.001, 0.002])
    r = oracle.render_topk(proj, gid, offs, _one_hot(2), 1, 1, 4)
    assert r["n_sel"][0, 0] == 0 and r["T_q"][0, 0] == 1.0
    np.testing.assert_array_equal(r["out"][0, 0], [0, 0])


def test_brute_force_over_subsets():
    """The selected set is the K-subset of the candidates of largest total
    weight, the earliest positions among equal totals; the candidates' weights
    are read from a run with K at least their count, which the large-K pin
    ties to the dense blend."""
    rng = np.random.default_rng(17)
    for trial in range(150):
        n = int(rng.integers(1, 10))
        alphas = rng.uniform(0.0, 0.95, n)
        alphas[rng.random(n) < 0.15] = 0.002  # off the ray
        if trial % 5 == 0:
            alphas[:] = np.round(alphas * 4) / 4  # coarse values: ties in weight
        proj, gid, offs = _ray(alphas)
        F = rng.standard_normal((n, 3))
        full = oracle.render_topk(proj, gid, offs, F, 1, 1, 16)
        nc = int(full["n_cand"][0, 0])
        pos_all = full["sel_pos"][0, 0, :nc]
        w_all = full["sel_w"][0, 0, :nc]
        for K in range(1, 6):
            r = oracle.render_topk(proj, gid, offs, F, 1, 1, K)
            k = min(K, nc)
            best = None
            for sub in itertools.combinations(range(nc), k):
                key = (-sum(w_all[list(sub)]), tuple(pos_all[list(sub)]))
                if best is None or key < best[0]:
                    best = (key, sub)
            want = pos_all[list(best[1])] if nc else np.zeros(0, np.int64)
            got = r["sel_pos"][0, 0, :r["n_sel"][0, 0]]
            np.testing.assert_array_equal(got, want, err_msg=str((trial, K, alphas)))
            if nc:
                sw = w_all[list(best[1])]
                np.testing.assert_allclose(r["out"][0, 0], (sw[:, None] * F[gid[want]]).sum(0) / sw.sum(),
                                           rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 3])
def test_large_K_is_the_normalised_dense_blend(seed):
    sc = synth.make_tiny(seed, n=600, dim=8)
    cam = synth.tiny_camera(32)
    pr = oracle.project(sc.means, sc.scales, sc.quats, sc.opacity, cam)
    gids, offs, _ = oracle.bin_sort(pr["rect"], pr["depth"], 2, 2)
    proj = dict(means2d=pr["means2d"], conic=pr["conic"], opacity=pr["opacity"])
    F = sc.features.astype(np.float64)
    d = oracle.render_dense(proj, gids, offs, F, 32, 32)
    r = oracle.render_topk(proj, gids, offs, F, 32, 32, 4096)
    lit = d["T_final"] < 1.0
    assert lit.mean() > 0.5
    np.testing.assert_allclose(r["out"][lit], d["out"][lit] / (1.0 - d["T_final"][lit])[:, None],
                               rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r["T_q"], d["T_final"], atol=1e-12)
    np.testing.assert_array_equal(r["out"][~lit], 0.0)
    # fewer: K-th selection set is a subset of the (K+1)-th, constant features stay constant
    r2 = oracle.render_topk(proj, gids, offs, np.ones((sc.n, 2)), 32, 32, 3)
    np.testing.assert_allclose(r2["out"][lit], 1.0, atol=1e-12)
    assert (r2["n_sel"] <= 3).all()


def test_params_alpha_max_respected():
    proj, gid, offs = _ray([1.5, 0.5])  # opacity above 1: alpha' = alpha_max = 0.99
    r = oracle.render_topk(proj, gid, offs, _one_hot(2), 1, 1, 2, params=RenderParams())
    np.testing.assert_allclose(r["sel_w"][0, 0], [0.99, 0.01 * 0.5], atol=1e-15)
