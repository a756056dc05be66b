"""Pins of the oracle's analytic gradients (dense blend and Algorithm 1)
against central finite differences of the oracle's own forward renderers,
on the 2,000-Gaussian 32x32 512-D sub-case; plus closed-form special cases.

A perturbation that changes a discrete decision (an entry entering or leaving
a ray, the dense stop, the quantile selection) makes the forward function
non-smooth there; such parameters are detected and skipped, and their count
is bounded."""

import numpy as np
import pytest

import oracle
import synth

K = 8


@pytest.fixture(scope="module")
def fd_case():
    sc, cam = synth.make_fd_case(seed=5)
    prm = oracle.RenderParams()
    pr = oracle.project(sc.means, sc.scales, sc.quats, sc.opacity, cam, prm)
    gids, offs, _ = oracle.bin_sort(pr["rect"], pr["depth"], 2, 2)
    rng = np.random.default_rng(99)
    gout = rng.standard_normal((32, 32, sc.dim))
    proj = dict(means2d=pr["means2d"].copy(), conic=pr["conic"].copy(), opacity=pr["opacity"].copy())
    return dict(sc=sc, cam=cam, prm=prm, pr=pr, proj=proj, gids=gids, offs=offs, gout=gout)


def _tiles_of(c, g):
    tx0, ty0, tx1, ty1 = c["pr"]["rect"][g]
    return [ty * 2 + tx for ty in range(ty0, ty1) for tx in range(tx0, tx1)]


def _forward(c, proj, feats, tiles, quantile):
    if quantile:
        r = oracle.render_quantile(proj, c["gids"], c["offs"], feats, 32, 32, K, c["prm"], tiles=tiles)
        key = (r["sel_gid"], r["k"], r["n_on"])
    else:
        r = oracle.render_dense(proj, c["gids"], c["offs"], feats, 32, 32, c["prm"], tiles=tiles)
        key = (r["n_contrib"], r["n_on"])
    m = ~np.isnan(r["out"][..., 0])
    return float(np.sum(r["out"][m] * c["gout"][m])), key


def _same(k1, k2):
    return all(np.array_equal(a, b) for a, b in zip(k1, k2))


def _fd(c, quantile, group, g, j, h):
    tiles = _tiles_of(c, g)
    feats = c["sc"].features.astype(np.float64)
    base = _forward(c, c["proj"], feats, tiles, quantile)[1]
    vals, keys = [], []
    for sgn in (1.0, -1.0):
        proj = {k: v.copy() for k, v in c["proj"].items()}
        f = feats
        if group == "features":
            f = feats.copy()
            f[g, j] += sgn * h
        elif group == "opacity":
            proj["opacity"][g] += sgn * h
        else:
            proj[group][g, j] += sgn * h
        L, key = _forward(c, proj, f, tiles, quantile)
        vals.append(L)
        keys.append(key)
    smooth = _same(base, keys[0]) and _same(base, keys[1])
    return (vals[0] - vals[1]) / (2 * h), smooth


@pytest.mark.parametrize("quantile", [False, True], ids=["dense", "quantile"])
def test_gradients_match_finite_differences(fd_case, quantile):
    c = fd_case
    args = (c["proj"], c["gids"], c["offs"], c["sc"].features, 32, 32)
    if quantile:
        gr = oracle.quantile_backward(*args, K, c["gout"], c["prm"])
    else:
        gr = oracle.dense_backward(*args, c["gout"], c["prm"])
    rng = np.random.default_rng(7)
    # Gaussians that actually contribute somewhere
    active = np.nonzero(np.abs(gr["opacity"]) > 1e-6)[0]
    assert active.size > 50
    steps = {"features": 1e-3, "opacity": 1e-6, "means2d": 1e-5, "conic": 1e-7}
    for group, h in steps.items():
        got, want, skipped = [], [], 0
        for g in rng.choice(active, 8, replace=False):
            j = int(rng.integers(0, {"features": 512, "opacity": 1, "means2d": 2, "conic": 3}[group]))
            fd, smooth = _fd(c, quantile, group, int(g), j, h)
            if not smooth:
                skipped += 1
                continue
            a = gr[group][g] if group == "opacity" else gr[group][g, j]
            got.append(a)
            want.append(fd)
        got, want = np.array(got), np.array(want)
        assert skipped <= 3, (group, skipped)
        rel = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-12)
        assert rel < 1e-5, (group, rel, got, want)


def test_single_selected_entry_has_no_geometric_gradient():
    """With one selected Gaussian, f~Q = f_j exactly, whatever its alpha'."""
    from tests.test_oracle_render import ray_case
    proj, gids, offs, feats = ray_case([0.3, 0.3, 0.3, 0.3])
    feats = np.random.default_rng(0).standard_normal((4, 5))
    gout = np.random.default_rng(1).standard_normal((1, 1, 5))
    gr = oracle.quantile_backward(proj, gids, offs, feats, 1, 1, 1, gout)
    for k in ("opacity", "conic", "means2d"):
        np.testing.assert_allclose(gr[k], 0.0, atol=1e-12)
    np.testing.assert_allclose(gr["features"][1], gout[0, 0])
    assert np.all(gr["features"][[0, 2, 3]] == 0)


def test_dense_single_gaussian_closed_form():
    """C = alpha' f: dL/df = alpha' g and dL/dalpha' = <g, f>."""
    from tests.test_oracle_render import ray_case
    proj, gids, offs, _ = ray_case([0.4])
    f = np.array([[1.0, -2.0, 0.5]])
    g = np.array([[[0.3, 0.1, -1.0]]])
    gr = oracle.dense_backward(proj, gids, offs, f, 1, 1, g)
    np.testing.assert_allclose(gr["features"][0], 0.4 * g[0, 0])
    # zero conic: G = 1, so dL/do = dL/dalpha'
    assert gr["opacity"][0] == pytest.approx(float(g[0, 0] @ f[0]))


@pytest.mark.parametrize("quantile", [False, True])
def test_term_magnitudes_bound_the_gradients(fd_case, quantile):
    """The magnitudes (a tolerance scale) bound every gradient entry from
    above, leave the gradients themselves unchanged, and equal the feature
    gradient exactly when every term is non-negative (g >= 0: the feature
    terms are w g / Z >= 0)."""
    c = fd_case
    feats = c["sc"].features.astype(np.float64)
    tiles = [0, 3]
    call = ((lambda g, **kw: oracle.quantile_backward(c["proj"], c["gids"], c["offs"], feats, 32, 32, K, g,
                                                     tiles=tiles, **kw))
            if quantile else
            (lambda g, **kw: oracle.dense_backward(c["proj"], c["gids"], c["offs"], feats, 32, 32, g,
                                                   tiles=tiles, **kw)))
    plain = call(c["gout"])
    r = call(c["gout"], magnitude=True)
    for k in ("features", "opacity", "conic", "means2d"):
        np.testing.assert_array_equal(r[k], plain[k])
        assert np.all(r["abs"][k] >= np.abs(r[k]) * (1 - 1e-12)), k
        assert np.all(r["abs"][k] >= 0)
    assert np.count_nonzero(r["abs"]["means2d"]) > 0
    pos = call(np.abs(c["gout"]), magnitude=True)
    np.testing.assert_allclose(pos["abs"]["features"], pos["features"], rtol=1e-12, atol=0)
