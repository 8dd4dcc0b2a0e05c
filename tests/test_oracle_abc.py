"""Pins of the oracle's ABC / PMC steps and its Philox generator.

Philox4x32-10 is checked against the known-answer vectors published with
the generator (Salmon et al., SC'11, Random123 distribution); the tolerance
rule against numpy's inverted-CDF quantile; the weighted covariance against
numpy.cov; the Beaumont weights against a mixture density built from
scipy.stats; prior draws and Box-Muller normals against their moments.
"""
import numpy as np
import pytest

from oracle import abc, philox


@pytest.mark.parametrize("ctr,key,out", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, out):
    got = philox.philox4x32(np.array(ctr, dtype=np.uint64).astype(np.uint32),
                            np.array(key, dtype=np.uint64).astype(np.uint32))
    assert tuple(int(v) for v in got) == out


def test_uniforms_open_interval_and_moments():
    u = philox.uniforms(123, 0, np.arange(200000, dtype=np.uint64), 0)
    assert u.min() > 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 3e-3 and abs(u.var() - 1 / 12) < 2e-3


def test_tolerance_is_inverted_cdf_quantile():
    rng = np.random.Generator(np.random.PCG64(1))
    d = rng.exponential(size=4096)
    for q in (0.05, 0.1, 0.25, 0.5):
        assert abs(abc.tolerance(d, q) - np.quantile(d, q, method="inverted_cdf")) == 0
    # failed runs (d = inf) are rejected and excluded from the percentile
    d[::7] = np.inf
    nf = int(np.isfinite(d).sum())
    assert abc.tolerance(d, 0.05) == np.quantile(d[np.isfinite(d)], 0.05, method="inverted_cdf")
    assert abc.accept(d, abc.tolerance(d, 0.05)).sum() == int(np.ceil(0.05 * nf))
    assert abc.accept(d, abc.tolerance(d, 1.0)).sum() == nf
    # no completed run: nothing is accepted
    assert abc.tolerance(np.full(5, np.inf), 0.5) == np.inf
    assert not abc.accept(np.full(5, np.inf), np.inf).any()


def test_distance_definition():
    data = np.zeros((50, 2))
    obs = np.full((3, 50, 2), 0.5)
    obs[1] = 0.0
    obs[2, 3, 1] = np.nan
    d = abc.distance(obs, data)
    assert d[0] == 0.5 and d[1] == 0.0 and d[2] == np.inf


def test_weighted_cov_matches_numpy():
    rng = np.random.Generator(np.random.PCG64(2))
    th = rng.standard_normal((500, 3)) * [1, 0.1, 100]
    w = rng.uniform(size=500)
    mu, S = abc.weighted_cov(th, w)
    np.testing.assert_allclose(S, np.cov(th.T, aweights=w, bias=True), rtol=1e-12)
    np.testing.assert_allclose(mu, np.average(th, axis=0, weights=w), rtol=1e-12)


def test_prior_draw_in_box_and_uniform():
    lo, hi = np.array([0.0, 0.01, 1e2]), np.array([10.0, 1.0, 1e4])
    th = abc.prior_draw(7, 100000, lo, hi)
    assert np.all(th >= lo) and np.all(th <= hi)
    np.testing.assert_allclose(th.mean(0), (lo + hi) / 2, rtol=1e-2)


def test_box_muller_moments():
    u = philox.uniforms(9, 3, np.arange(100000, dtype=np.uint64), 0)
    z0, z1 = abc.box_muller(u[:, 0], u[:, 1])
    for z in (z0, z1):
        assert abs(z.mean()) < 0.02 and abs(z.var() - 1) < 0.02
    assert abs(np.mean(z0 * z1)) < 0.02


def test_pmc_weights_match_scipy_mixture_density():
    """w_i proportional to 1 / sum_j w_j N(theta_i; theta_j, 2 Sigma), with the
    Gaussian density from scipy.stats."""
    from scipy.stats import multivariate_normal
    rng = np.random.Generator(np.random.PCG64(3))
    prev = rng.standard_normal((40, 3)) * [0.5, 0.05, 200] + [2.0, 0.1, 1000.0]
    pw = rng.uniform(size=40)
    pw /= pw.sum()
    th = rng.standard_normal((25, 3)) * [0.5, 0.05, 200] + [2.0, 0.1, 1000.0]
    acc = rng.uniform(size=25) < 0.7
    w = abc.pmc_weights(th, acc, prev, pw)
    _, S = abc.weighted_cov(prev, pw)
    dens = np.array([sum(pw[j] * multivariate_normal(prev[j], 2 * S).pdf(t) for j in range(40))
                     for t in th[acc]])
    ref = 1 / dens
    np.testing.assert_allclose(w, ref / ref.sum(), rtol=1e-9)


def test_pmc_proposals_stay_in_box_and_follow_parents():
    lo, hi = np.array([0.0, 0.01, 1e2]), np.array([10.0, 1.0, 1e4])
    rng = np.random.Generator(np.random.PCG64(4))
    prev = lo + (hi - lo) * rng.uniform(size=(200, 3)) * 0.1 + [4.0, 0.3, 3000.0]
    w = rng.uniform(size=200)
    w /= w.sum()
    th = abc.pmc_propose(11, 1, 400, prev, w, lo, hi)
    assert np.all(th >= lo) and np.all(th <= hi)
    mu, _ = abc.weighted_cov(prev, w)
    assert np.all(np.abs(th.mean(0) - mu) < 0.25 * (hi - lo))
