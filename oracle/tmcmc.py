"""Transitional Markov chain Monte Carlo (Sec. 2.3, Algorithm TMCMC, after
Ching and Chen 2007) and the Gaussian likelihood of eqs. (likelihood) and
(fitness), in plain numpy FP64 -- test infrastructure only.

The sampler moves from the prior f_0 = pi to the posterior through
f_j ~ p(D|theta)^{q_j} pi(theta), 0 = q_0 < q_1 < ... < q_lambda = 1.  At each
stage the plausibility weights w = p(D|theta)^{q_{j+1} - q_j} of the current
samples give the mean weight S_j, the normalized weights and the scaled
weighted covariance b^2 sum_k wbar_k (theta_k - mu_j)(theta_k - mu_j)^T; the
next generation resamples the current one by the normalized weights, and each
distinct resampled point starts a Metropolis chain, with Gaussian proposals of
that covariance, as long as the number of times it was drawn.  The product of
the S_j estimates the evidence.

Readings of the text (each also listed in the design notes):
* Sigma = sigma^2 I: sigma is the standard deviation of the observation noise
  (the data model D_k = g_k + sigma eps_k with unit-variance eps_k), sampled
  as the last parameter, so
  log p = -m/2 log(2 pi) - m log(sigma) - |D - g|^2 / (2 sigma^2).
* q_{j+1}: the largest increment dq in (0, 1 - q_j] whose weights have a
  coefficient of variation (population standard deviation over mean) of at
  most cv_target, found by BISECT_ITERS bisection steps; q_{j+1} = 1 ends the
  run after one more resampling stage.
* mu_j is the weighted mean; the chains target f_{j+1}, the distribution the
  new generation represents.
* a chain of length n takes n Metropolis steps from its point; its samples are
  the states after each step.  Proposals outside the prior box are rejected
  without a likelihood evaluation.
* forward runs that do not complete have zero likelihood in every stage: they
  take no part in the coefficient of variation (the criterion is applied to
  the completed runs), are never resampled, and count as zero weights in S_j,
  so the evidence carries the completed fraction of the prior samples.
* a weighted covariance without full rank (all weight on fewer than d + 1
  points) gets 1e-12 (hi - lo)^2 added to its diagonal before the Cholesky
  factorization.

Random numbers come from Philox4x32-10 (oracle/philox.py), key = seed:
  prior sample i:                     stream 0, draws 0 and 1 (abc.prior_draw)
  resampling draw k at stage j:       stream 1000 + 2j, index k, draw 0 -> u[0]
  chain c (in increasing order of its starting sample), step s (1-based),
  at stage j:                         stream 1001 + 2j, index c,
                                      draws 3(s-1), 3(s-1)+1, 3(s-1)+2 -> u0..u5;
                                      Box-Muller (u0, u1) -> z0, z1 and
                                      (u2, u3) -> z2, z3; u4 decides acceptance
"""
import numpy as np

from . import abc, philox

BISECT_ITERS = 80


def gauss_loglik(g, D, sigma):
    """Log-likelihood of eqs. (likelihood)-(fitness) with Sigma = sigma^2 I.
    g: (P, m) model outputs (a row with a non-finite entry: failed run, -inf);
    D: (m,); sigma: (P,)."""
    g = np.asarray(g, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64).ravel()
    sigma = np.asarray(sigma, dtype=np.float64)
    g = g.reshape(g.shape[0], -1)
    m = D.size
    J = np.sum((D[None, :] - g) ** 2, axis=1) / sigma ** 2
    ll = -0.5 * m * np.log(2.0 * np.pi) - m * np.log(sigma) - 0.5 * J
    ll[~np.all(np.isfinite(g), axis=1)] = -np.inf
    return ll


def gauss_loglik2(g, D, sigma_a, sigma_b):
    """Log-likelihood of eqs. (likelihood)-(fitness) with the diagonal
    covariance of Sec. 4.3: entries 0, 2, 4, ... (odd in 1-based numbering)
    have standard deviation sigma_a, the others sigma_b.  g: (P, m) model
    outputs (a row with a non-finite entry: -inf); D: (m,); sigma_a,
    sigma_b: (P,) (a level that is not > 0: -inf)."""
    g = np.asarray(g, dtype=np.float64)
    g = g.reshape(g.shape[0], -1)
    D = np.asarray(D, dtype=np.float64).ravel()
    sa = np.asarray(sigma_a, dtype=np.float64)
    sb = np.asarray(sigma_b, dtype=np.float64)
    r2 = (D[None, :] - g) ** 2
    Ja, Jb = r2[:, 0::2].sum(axis=1), r2[:, 1::2].sum(axis=1)
    ma, mb = D[0::2].size, D[1::2].size
    with np.errstate(divide="ignore", invalid="ignore"):
        ll = (-0.5 * (ma + mb) * np.log(2.0 * np.pi) - ma * np.log(sa) - mb * np.log(sb)
              - 0.5 * Ja / sa ** 2 - 0.5 * Jb / sb ** 2)
    ll[~np.all(np.isfinite(g), axis=1) | ~(sa > 0) | ~(sb > 0)] = -np.inf
    return ll


def weight_cv(logl, dq):
    """Coefficient of variation of the weights exp(dq (l - max l)) over the
    finite log-likelihoods."""
    f = np.asarray(logl, dtype=np.float64)
    f = f[np.isfinite(f)]
    w = np.exp(dq * (f - f.max()))
    m = w.mean()
    return np.sqrt(np.mean((w - m) ** 2)) / m


def next_q(logl, q, cv_target):
    """q_{j+1} for the samples' log-likelihoods at q_j = q."""
    dmax = 1.0 - q
    if weight_cv(logl, dmax) <= cv_target:
        return 1.0
    lo, hi = 0.0, dmax
    for _ in range(BISECT_ITERS):
        mid = 0.5 * (lo + hi)
        if weight_cv(logl, mid) > cv_target:
            hi = mid
        else:
            lo = mid
    return q + lo


def stage_statistics(theta, logl, dq, b):
    """Normalized weights (zero for failed runs), log S_j, weighted mean and the
    proposal covariance b^2 sum wbar (theta - mu)(theta - mu)^T."""
    theta = np.asarray(theta, dtype=np.float64)
    logl = np.asarray(logl, dtype=np.float64)
    fin = np.isfinite(logl)
    lmax = logl[fin].max()
    w = np.zeros(logl.size)
    w[fin] = np.exp(dq * (logl[fin] - lmax))
    log_s = dq * lmax + np.log(w.sum() / logl.size)
    wbar = w / w.sum()
    mu = wbar @ theta
    dv = theta - mu
    cov = b * b * ((dv * wbar[:, None]).T @ dv)
    return wbar, log_s, mu, cov


def resample_counts(seed, stage, wbar, n):
    """How many of the n draws of stage `stage` pick each sample."""
    cdf = np.cumsum(np.asarray(wbar, dtype=np.float64))
    u = philox.uniforms(seed, 1000 + 2 * stage, np.arange(n, dtype=np.uint64), 0)[:, 0]
    idx = np.minimum(np.searchsorted(cdf, u * cdf[-1], side="right"), cdf.size - 1)
    return np.bincount(idx, minlength=cdf.size)


def proposal_factor(cov, lo, hi):
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    try:
        return np.linalg.cholesky(cov)
    except np.linalg.LinAlgError:
        return np.linalg.cholesky(cov + np.diag(1e-12 * (hi - lo) ** 2))


def chain_normals(seed, stage, chain, step):
    """z0..z3 and the acceptance uniform of chain `chain`, step `step` (1-based)."""
    base = 3 * (step - 1)
    u01 = philox.uniforms(seed, 1001 + 2 * stage, np.uint64(chain), base)
    u23 = philox.uniforms(seed, 1001 + 2 * stage, np.uint64(chain), base + 1)
    u45 = philox.uniforms(seed, 1001 + 2 * stage, np.uint64(chain), base + 2)
    z0, z1 = abc.box_muller(u01[0], u01[1])
    z2, z3 = abc.box_muller(u23[0], u23[1])
    return np.array([z0, z1, z2, z3]), u45[0]


def metropolis_stage(seed, stage, theta, logl, counts, L, q_next, lo, hi, loglik_fn):
    """Chains from every sample drawn at least once, run step by step across all
    chains (one batched likelihood call per step).  Returns the new generation
    (chain by chain, step by step), its log-likelihoods, the accepted moves and
    the likelihood evaluations."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    d = lo.size
    starts = np.flatnonzero(counts)
    lengths = counts[starts]
    cur = np.asarray(theta, float)[starts].copy()
    lcur = np.asarray(logl, float)[starts].copy()
    out_theta = [np.empty((n, d)) for n in lengths]
    out_logl = [np.empty(n) for n in lengths]
    accepted = evals = 0
    for s in range(1, int(lengths.max()) + 1):
        active = np.flatnonzero(lengths >= s)
        prop = np.empty((active.size, d))
        uacc = np.empty(active.size)
        for a, c in enumerate(active):
            z, u = chain_normals(seed, stage, int(c), s)
            prop[a] = cur[c] + L @ z[:d]
            uacc[a] = u
        inbox = np.all(prop >= lo, axis=1) & np.all(prop <= hi, axis=1)
        lprop = np.full(active.size, -np.inf)
        if inbox.any():
            lprop[inbox] = loglik_fn(prop[inbox])
            evals += int(inbox.sum())
        for a, c in enumerate(active):
            if inbox[a] and np.log(uacc[a]) < q_next * (lprop[a] - lcur[c]):
                cur[c] = prop[a]
                lcur[c] = lprop[a]
                accepted += 1
            out_theta[c][s - 1] = cur[c]
            out_logl[c][s - 1] = lcur[c]
    return np.concatenate(out_theta), np.concatenate(out_logl), accepted, evals


def tmcmc(loglik_fn, lo, hi, n, seed, cv_target=1.0, b=0.2, max_stages=50):
    """Full run.  loglik_fn(theta (P, d)) -> (P,) log-likelihoods (-inf: failed
    run).  Returns the final generation and the stage record."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    theta = abc.prior_draw(seed, n, lo, hi)
    logl = np.asarray(loglik_fn(theta), dtype=np.float64)
    evals = n
    if not np.isfinite(logl).any():
        raise RuntimeError("no prior sample has a finite likelihood")
    q = 0.0
    qs, log_s, acc, cvs = [0.0], [], [], []
    for stage in range(max_stages):
        q_next = next_q(logl, q, cv_target)
        wbar, ls, _, cov = stage_statistics(theta, logl, q_next - q, b)
        cvs.append(weight_cv(logl, q_next - q))
        log_s.append(ls)
        counts = resample_counts(seed, stage, wbar, n)
        L = proposal_factor(cov, lo, hi)
        theta, logl, a, e = metropolis_stage(seed, stage, theta, logl, counts, L, q_next, lo, hi, loglik_fn)
        acc.append(a)
        evals += e
        q = q_next
        qs.append(q)
        if q >= 1.0:
            break
    return dict(theta=theta, logl=logl, q=np.array(qs), log_evidence=float(np.sum(log_s)), log_s=np.array(log_s),
                accepted=np.array(acc), evaluations=evals, cv=np.array(cvs))
