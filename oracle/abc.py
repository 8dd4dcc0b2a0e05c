"""ABC rejection and population-Monte-Carlo steps in plain numpy FP64
(test infrastructure only).

The paper samples its posterior with TMCMC (Sec. 3.2); the workloads here use
approximate Bayesian computation around the same forward model g(theta|M) of
eq. (model_err).  Definitions used:

* distance  d_i = sqrt( mean over the n_obs head samples and both coordinates
  of (obs_i - data)^2 );  a failed forward run has d_i = +inf.
* tolerance tol = the k-th smallest finite distance, k = ceil(q * P_f)
  (1-based), P_f the number of forward runs that completed (finite d_i):
  failed runs are rejected and take no part in the percentile.  With no
  completed run tol = +inf.  accept d_i <= tol for finite d_i (ties
  accepted).
* prior: uniform box on (alpha, S_b, S_s), linear scale.
* PMC (Beaumont, Cornuet, Marin & Robert 2009): proposals resample the previous
  accepted population by its normalized weights and perturb with a Gaussian of
  covariance 2 x the weighted sample covariance; perturbations that leave the
  prior box are redrawn.  New weights w_i = pi(theta_i) / sum_j w_j N(theta_i;
  theta_j, 2 Sigma), normalized over the accepted particles.

Random numbers come from Philox4x32-10 (oracle/philox.py):
  prior draw of particle i:       stream 0, draws 0 and 1 -> u[0..3]
  PMC attempt a of particle i:    stream 1 + generation, draws 3a, 3a+1, 3a+2
                                  -> u0 (resample), Box-Muller (u1,u2), (u3,u4)
"""
import numpy as np

from . import philox

MAX_ATTEMPTS = 10000


def distance(obs, data):
    """obs: (P, n_obs, 2) (NaN rows = failed run); data: (n_obs, 2)."""
    obs = np.asarray(obs, dtype=np.float64)
    d = np.sqrt(np.mean((obs - np.asarray(data, dtype=np.float64)[None]) ** 2, axis=(1, 2)))
    d[~np.isfinite(d)] = np.inf
    return d


def tolerance(d, q):
    """k-th smallest finite distance with k = ceil(q P_f)."""
    d = np.asarray(d, dtype=np.float64)
    f = np.sort(d[np.isfinite(d)])
    if f.size == 0:
        return float("inf")
    k = int(np.ceil(q * f.size))
    k = min(max(k, 1), f.size)
    return float(f[k - 1])


def accept(d, tol):
    d = np.asarray(d)
    return np.isfinite(d) & (d <= tol)


def prior_draw(seed, n, lo, hi):
    """theta_i = lo + (hi - lo) * u, u from Philox stream 0."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    idx = np.arange(n, dtype=np.uint64)
    u = np.concatenate([philox.uniforms(seed, 0, idx, 0), philox.uniforms(seed, 0, idx, 1)], axis=-1)
    return lo[None] + (hi - lo)[None] * u[:, : lo.size]


def weighted_cov(theta, w):
    """Weighted mean and covariance sum_j w_j (theta_j - mu)(theta_j - mu)^T, w normalized."""
    theta = np.asarray(theta, float)
    w = np.asarray(w, float) / np.sum(w)
    mu = w @ theta
    dv = theta - mu
    return mu, (dv * w[:, None]).T @ dv


def box_muller(u, v):
    r = np.sqrt(-2.0 * np.log(u))
    return r * np.cos(2.0 * np.pi * v), r * np.sin(2.0 * np.pi * v)


def pmc_propose(seed, generation, n, prev_theta, prev_w, lo, hi):
    """n proposals for PMC generation `generation` (>= 1)."""
    prev_theta = np.asarray(prev_theta, float)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    w = np.asarray(prev_w, float)
    cdf = np.cumsum(w)
    _, S = weighted_cov(prev_theta, w)
    L = np.linalg.cholesky(2.0 * S)
    out = np.empty((n, lo.size))
    stream = 1 + generation
    for i in range(n):
        for a in range(MAX_ATTEMPTS):
            u01 = philox.uniforms(seed, stream, np.uint64(i), 3 * a)
            u23 = philox.uniforms(seed, stream, np.uint64(i), 3 * a + 1)
            u45 = philox.uniforms(seed, stream, np.uint64(i), 3 * a + 2)
            j = int(np.searchsorted(cdf, u01[0] * cdf[-1], side="right"))
            j = min(j, prev_theta.shape[0] - 1)
            z0, z1 = box_muller(u01[1], u23[0])
            z2, _ = box_muller(u23[1], u45[0])
            cand = prev_theta[j] + L @ np.array([z0, z1, z2])[: lo.size]
            if np.all(cand >= lo) and np.all(cand <= hi):
                out[i] = cand
                break
        else:
            raise RuntimeError("PMC proposal could not be placed inside the prior box")
    return out


def pmc_weights(theta, acc, prev_theta, prev_w):
    """Beaumont weights for the accepted proposals (uniform prior inside the box).
    Returns normalized weights over theta[acc]."""
    theta = np.asarray(theta, float)[np.asarray(acc, bool)]
    prev_theta = np.asarray(prev_theta, float)
    pw = np.asarray(prev_w, float) / np.sum(prev_w)
    _, S = weighted_cov(prev_theta, pw)
    K = 2.0 * S
    Kinv = np.linalg.inv(K)
    dv = theta[:, None, :] - prev_theta[None, :, :]
    quad = np.einsum("ijk,kl,ijl->ij", dv, Kinv, dv)
    dens = np.exp(-0.5 * quad) @ pw
    w = 1.0 / dens
    return w / np.sum(w)
