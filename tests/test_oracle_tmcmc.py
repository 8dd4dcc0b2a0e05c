"""Pins of the TMCMC oracle (Sec. 2.3, Algorithm TMCMC; likelihood eqs.
(likelihood)-(fitness)) against what the mathematics fixes: the Gaussian
density of scipy, the coefficient-of-variation criterion, a Gaussian
posterior and its evidence in closed form, a constant likelihood (one stage,
exact evidence), and zero-likelihood regions entering the evidence as the
completed fraction."""
import numpy as np
import pytest
from scipy import stats

from oracle import abc, tmcmc


def test_gauss_loglik_is_the_isotropic_normal_density():
    rng = np.random.Generator(np.random.PCG64(1))
    D = rng.normal(size=100)
    g = D[None] + rng.normal(scale=0.01, size=(5, 100))
    sig = np.array([0.005, 0.01, 0.02, 0.1, 1.0])
    ll = tmcmc.gauss_loglik(g, D, sig)
    for i in range(5):
        ref = stats.multivariate_normal(mean=g[i], cov=sig[i] ** 2 * np.eye(100)).logpdf(D)
        assert abs(ll[i] - ref) <= 1e-9 * abs(ref)
    g[2, 7] = np.nan
    assert np.isneginf(tmcmc.gauss_loglik(g, D, sig)[2])


def test_next_q_meets_the_cv_target():
    rng = np.random.Generator(np.random.PCG64(2))
    logl = -0.5 * rng.chisquare(3, size=4000) * 50.0
    logl[::7] = -np.inf
    q1 = tmcmc.next_q(logl, 0.0, 1.0)
    assert 0.0 < q1 < 1.0
    assert abs(tmcmc.weight_cv(logl, q1) - 1.0) < 1e-9
    # a flat likelihood moves straight to q = 1
    assert tmcmc.next_q(np.full(100, -3.0), 0.3, 1.0) == 1.0
    # a larger target allows a larger step
    assert tmcmc.next_q(logl, 0.0, 2.0) > q1


def test_resample_counts():
    rng = np.random.Generator(np.random.PCG64(3))
    w = rng.uniform(size=500)
    w[::5] = 0.0
    w /= w.sum()
    c = tmcmc.resample_counts(9, 2, w, 2000)
    assert c.sum() == 2000 and np.all(c[::5] == 0)
    # frequencies follow the weights (chi-square over the drawn support)
    e = 2000 * w[w > 0]
    chi2 = np.sum((c[w > 0] - e) ** 2 / e)
    assert chi2 < stats.chi2.ppf(0.999, (w > 0).sum() - 1)


def test_gaussian_posterior_and_evidence():
    """L = N(theta; mu0, diag(s0^2)) normalized, prior uniform on a box that
    holds mu0 +- 10 s0: the posterior is that normal and the evidence is
    1/vol(box) (the mass outside the box is below 1e-20).  TMCMC's short
    chains leave strongly correlated final samples (an effective size of a
    few dozen per run at 2000 samples), so four seeds are pooled: the pooled
    mean within 0.2 s0, each run's mean within 0.4 s0 and spread within 20 %,
    the evidence within 1 in log (a dropped term of the estimator moves it by
    the log of the peak likelihood, about 5 here)."""
    mu0 = np.array([1.0, -2.0, 0.5, 3.0])
    s0 = np.array([0.1, 0.3, 0.05, 0.2])
    lo, hi = mu0 - 10 * s0, mu0 + 10 * s0
    mvn = stats.multivariate_normal(mean=mu0, cov=np.diag(s0 ** 2))

    def loglik(th):
        return mvn.logpdf(np.atleast_2d(th))

    means = []
    for seed in (11, 12, 13, 14):
        r = tmcmc.tmcmc(loglik, lo, hi, 2000, seed=seed)
        assert r["q"][-1] == 1.0 and np.all(np.diff(r["q"]) > 0)
        assert np.all(np.abs(r["cv"][:-1] - 1.0) < 1e-9)
        th = r["theta"]
        assert np.all(np.abs(th.mean(0) - mu0) < 0.4 * s0), seed
        assert np.all(np.abs(th.std(0) / s0 - 1) < 0.2), seed
        assert abs(r["log_evidence"] + np.sum(np.log(hi - lo))) < 1.0, seed
        assert np.allclose(r["logl"], loglik(th))
        means.append(th.mean(0))
    assert np.all(np.abs(np.mean(means, 0) - mu0) < 0.2 * s0)


def test_constant_likelihood_takes_one_stage():
    lo, hi = np.zeros(3), np.array([1.0, 2.0, 3.0])
    r = tmcmc.tmcmc(lambda th: np.full(len(th), -4.5), lo, hi, 500, seed=5)
    assert list(r["q"]) == [0.0, 1.0]
    assert r["log_evidence"] == pytest.approx(-4.5, abs=1e-12)
    # a flat target accepts every proposal that stays in the box
    assert np.all((r["theta"] >= lo) & (r["theta"] <= hi))


def test_zero_likelihood_region_enters_the_evidence():
    """L = e^c where theta_0 < 1/2 and 0 elsewhere (runs that fail): the
    evidence estimate is e^c times the fraction of prior samples in the
    support, which is a binomial estimate of 1/2."""
    lo, hi = np.zeros(2), np.ones(2)
    c = -2.0

    def loglik(th):
        th = np.atleast_2d(th)
        return np.where(th[:, 0] < 0.5, c, -np.inf)

    n = 1000
    p_hat = np.mean(abc.prior_draw(8, n, lo, hi)[:, 0] < 0.5)
    r = tmcmc.tmcmc(loglik, lo, hi, n, seed=8)
    assert list(r["q"]) == [0.0, 1.0]
    assert r["log_evidence"] == pytest.approx(c + np.log(p_hat), abs=1e-12)
    assert abs(p_hat - 0.5) < 3 * np.sqrt(0.25 / n)
    assert np.all(r["theta"][:, 0] < 0.5)


def test_two_level_loglik_is_the_diagonal_normal_density():
    rng = np.random.Generator(np.random.PCG64(21))
    m = 40
    D = rng.normal(size=m)
    g = D[None] + rng.normal(scale=0.02, size=(4, m))
    sa = np.array([0.01, 0.02, 0.05, 0.3])
    sb = np.array([0.03, 0.02, 0.001, 1.0])
    ll = tmcmc.gauss_loglik2(g, D, sa, sb)
    for i in range(4):
        sd = np.where(np.arange(m) % 2 == 0, sa[i], sb[i])
        ref = stats.multivariate_normal(mean=g[i], cov=np.diag(sd ** 2)).logpdf(D)
        assert abs(ll[i] - ref) <= 1e-10 * abs(ref)
    # one level: the isotropic density
    assert np.allclose(tmcmc.gauss_loglik2(g, D, sa, sa), tmcmc.gauss_loglik(g, D, sa), rtol=1e-13, atol=0)
    g[1, 3] = np.nan
    out = tmcmc.gauss_loglik2(g, D, sa, np.array([0.03, 0.02, 0.0, 1.0]))
    assert np.isneginf(out[1]) and np.isneginf(out[2]) and np.isfinite(out[0])
