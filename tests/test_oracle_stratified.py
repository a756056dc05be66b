"""Pins of the Stratified-K oracle (Appendix, adaptive variants) against
facts that do not come from the oracle itself: the defining property of the
thresholds (Gaussian tail mass, evaluated with math.erf rather than the
inverse the oracle uses), hand-computed transmittance statistics, the closed
interval form of the selection with the ray's own thresholds (written out
here from the cumulative product of (1 - alpha')), and the blend's
invariants."""

import math

import numpy as np
import pytest

import oracle


def _phi(z):
    return 0.5 * (1.0 + math.erf(z / math.sqrt(2.0)))


@pytest.mark.parametrize("K", [1, 2, 7, 8, 32])
def test_thresholds_leave_equal_gaussian_mass(K):
    rng = np.random.default_rng(K)
    for _ in range(50):
        mu, sd = rng.uniform(0.05, 0.95), rng.uniform(0.01, 0.4)
        t = oracle.stratified_thresholds(mu, sd, K)
        assert np.all(np.diff(t) <= 0.0)  # descending, as transmittance falls
        for m in range(1, K + 1):
            want = 1.0 - m / (K + 1.0)
            tm = t[m - 1]
            if 0.0 < tm < 1.0:
                assert abs((1.0 - _phi((tm - mu) / sd)) - (1.0 - want)) < 1e-12 or \
                    abs(_phi((tm - mu) / sd) - want) < 1e-12
            else:  # clipped: the unclipped point lies outside [0, 1]
                z = (tm - mu) / sd
                assert (tm == 0.0 and _phi((0.0 - mu) / sd) >= want - 1e-12) or \
                    (tm == 1.0 and _phi((1.0 - mu) / sd) <= want + 1e-12)


def test_transmittance_stats_hand_example():
    # alpha' = 0.5 four times: T values 1, 1/2, 1/4, 1/8, 1/16
    mu, sd = oracle.transmittance_stats([0.5] * 4, T_eps=1e-4)
    v = [1.0, 0.5, 0.25, 0.125, 0.0625]
    m = sum(v) / 5.0
    assert mu == pytest.approx(1.9375 / 5.0, abs=1e-15) and mu == pytest.approx(m)
    assert sd == pytest.approx(math.sqrt(sum((x - m) ** 2 for x in v) / 5.0), abs=1e-15)
    # the dense early stop ends the list: 0.5^14 < 1e-4 is not composited
    mu2, _ = oracle.transmittance_stats([0.5] * 20, T_eps=1e-4)
    v2 = [0.5 ** i for i in range(14)]
    assert mu2 == pytest.approx(sum(v2) / len(v2), abs=1e-15)


def _one_ray_case(alphas, dim=3, seed=0):
    """A 1x1 image whose ray meets Gaussians centred on the pixel: alpha' =
    opacity (below alpha_max)."""
    n = len(alphas)
    proj = dict(means2d=np.full((n, 2), 0.5), conic=np.tile([1.0, 0.0, 1.0], (n, 1)),
                opacity=np.asarray(alphas, np.float64))
    feats = np.random.default_rng(seed).standard_normal((n, dim))
    return proj, np.arange(n), np.array([0, n]), feats


def _interval_selection(alphas, thr, T_eps):
    """Closed form: entry i is selected iff a threshold lies in (T_after_i,
    T_before_i]; the walk ends after the entry that consumes the last one, or
    at the first entry whose T_after falls below T_eps (not examined)."""
    a = np.asarray(alphas, np.float64)
    T_after = np.cumprod(1.0 - a)
    T_before = np.concatenate([[1.0], T_after[:-1]])
    sel, consumed = [], 0
    for i in range(a.size):
        if consumed == len(thr) or T_after[i] < T_eps:
            break
        hit = [m for m in range(len(thr)) if T_after[i] < thr[m] <= T_before[i]]
        if hit:
            sel.append(i)
        consumed = sum(1 for t in thr if T_after[i] < t)
    return sel


@pytest.mark.parametrize("K", [1, 3, 8])
def test_selection_matches_interval_form_with_the_rays_thresholds(K):
    rng = np.random.default_rng(100 + K)
    prm = oracle.RenderParams()
    for trial in range(60):
        n = int(rng.integers(1, 40))
        alphas = rng.uniform(0.02, 0.6, n) if trial % 2 else rng.uniform(0.3, 0.95, n)
        proj, gids, offs, feats = _one_ray_case(alphas, seed=trial)
        r = oracle.render_stratified(proj, gids, offs, feats, 1, 1, K, prm)
        # statistics written out independently: T_0 = 1 and the composited T
        T = np.concatenate([[1.0], np.cumprod(1.0 - alphas)])
        keep = np.concatenate([[True], T[1:] >= prm.T_eps])
        last = np.argmin(keep) if not keep.all() else T.size
        vals = T[:last]
        thr = oracle.stratified_thresholds(vals.mean(), vals.std(), K)
        want = _interval_selection(alphas, list(thr), prm.T_eps)
        got = [int(g) for g in r["sel_gid"][0, 0] if g >= 0]
        assert got == want, (trial, alphas, thr)
        assert r["n_sel"][0, 0] <= K
        # w^Q sum to 1 - T^Q; a constant feature renders itself
        assert r["sel_w"][0, 0].sum() + r["T_q"][0, 0] == pytest.approx(1.0, abs=1e-12)
        if got:
            c = np.full_like(feats, 0.7)
            rc = oracle.render_stratified(proj, gids, offs, c, 1, 1, K, prm)
            np.testing.assert_allclose(rc["out"][0, 0], 0.7, rtol=1e-12)


def test_empty_ray_selects_nothing():
    proj, gids, offs, feats = _one_ray_case([0.001, 0.002])  # below alpha_min = 1/255
    r = oracle.render_stratified(proj, gids, offs, feats, 1, 1, 4)
    assert r["n_sel"][0, 0] == 0 and np.all(r["out"][0, 0] == 0.0) and r["T_q"][0, 0] == 1.0
