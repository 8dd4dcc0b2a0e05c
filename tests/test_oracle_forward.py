"""Pins of the oracle's forward model (forces -> velocity sum -> forward
Euler, Sec. 2.1 and the Appendix's numerical-algorithm paragraph).

Absolute trajectories of this filament model are not printed in the paper
(parity unpinned for absolute values); the pins are structural: translation
and mirror equivariance, rest states, energy decay with a frozen beat, the
Stokes limit, and a brute-force 40-digit re-computation of a tiny run.
"""
import mpmath as mp
import numpy as np
import pytest

from paper_1910_12007_amd import inputs

pytestmark = pytest.mark.usefixtures("reading_blob_module")


def _run(core, N=24, steps=40, dt=1e-4, obs_every=10, **kw):
    P = inputs.param_rows(1, **kw)
    return core.forward(P, N, steps, dt, obs_every)


def test_translation_equivariance(oracle_core):
    a = _run(oracle_core, alpha=1.5)
    b = _run(oracle_core, alpha=1.5, x0=0.25, y0=-0.5)
    np.testing.assert_allclose(b["obs"][..., 0] - 0.25, a["obs"][..., 0], atol=1e-13)
    np.testing.assert_allclose(b["obs"][..., 1] + 0.5, a["obs"][..., 1], atol=1e-13)


def test_mirror_equivariance(oracle_core):
    """y -> -y flips the signed curvature, so b -> -b mirrors the run."""
    a = _run(oracle_core, alpha=0.8, b=0.1)
    b = _run(oracle_core, alpha=0.8, b=-0.1)
    np.testing.assert_allclose(b["obs"][..., 0], a["obs"][..., 0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(b["obs"][..., 1], -a["obs"][..., 1], rtol=0, atol=1e-14)


def test_straight_filament_without_beat_stays_at_rest(oracle_core):
    r = _run(oracle_core, alpha=2.0, b=0.0)
    N = 24
    assert np.all(np.abs(r["x"] - np.arange(N) / (N - 1)) < 1e-12)
    assert np.all(r["y"] == 0.0)


def test_frozen_beat_energy_decreases(oracle_core):
    """With omega = 0 the preferred shape is fixed and the flow only
    dissipates: the energy is non-increasing for a small step."""
    N, b, phase = 24, 0.1, 0.4
    k0 = oracle_core.kappa0(N, b, 2 * np.pi, 0.0, phase, 0.0)
    E = []
    for steps in [1, 20, 40, 80, 160]:
        r = _run(oracle_core, N=N, steps=steps, dt=2e-5, alpha=1.0, omega=0.0, phase=phase, b=b)
        E.append(oracle_core.energy(r["x"], r["y"], 0.1, 1e3, k0))
    assert all(E[i + 1] < E[i] for i in range(len(E) - 1)), E


def test_stokes_limit_of_trajectory(oracle_core):
    a = _run(oracle_core, alpha=0.0)
    b = _run(oracle_core, alpha=1e-7)
    np.testing.assert_allclose(b["obs"], a["obs"], rtol=0, atol=1e-12)


def test_single_workload_runs_stably(oracle_core):
    """N = 64, 2000 steps of dt = 1e-4, alpha in {1, 0}."""
    for alpha in (1.0, 0.0):
        r = oracle_core.forward(inputs.param_rows(1, alpha=alpha), 64, 2000, 1e-4, 100)
        assert r["status"] == 0
        assert np.all(np.isfinite(r["obs"])) and 0 < r["speed"][0] < 1.0


def test_blowup_is_reported(oracle_core):
    """Forward Euler beyond its stability bound (S_b = 1 at N = 128,
    dt = 5e-5) reports a failed status instead of garbage."""
    r = oracle_core.forward(inputs.param_rows(1, alpha=2.0, Sb=1.0, Ss=1e4), 128, 400, 5e-5, 100)
    assert r["status"] in (1, 2)
    assert np.isnan(r["speed"][0])


def _mp_run(N, steps, dt, alpha, Sb, Ss, b, kw, om, eps_ds):
    """Brute force at 40 digits: energy gradient by mpmath differentiation,
    kernel by the closed form with mpmath Bessel functions."""
    mp.mp.dps = 40
    ds = mp.mpf(1) / (N - 1)
    eps = mp.mpf(eps_ds) * ds
    alpha = mp.mpf(alpha)
    X = [mp.mpf(i) * ds for i in range(N)] + [mp.mpf(0)] * N

    def energy(V, t):
        x, y = V[:N], V[N:]
        E = mp.mpf(0)
        for k in range(N - 1):
            l = mp.sqrt((x[k + 1] - x[k]) ** 2 + (y[k + 1] - y[k]) ** 2)
            E += Ss * (l / ds - 1) ** 2 * ds
        for k in range(1, N - 1):
            a = (x[k + 1] - x[k - 1]) / (2 * ds)
            bb = (y[k + 1] - y[k - 1]) / (2 * ds)
            p = (x[k + 1] - 2 * x[k] + x[k - 1]) / ds ** 2
            q = (y[k + 1] - 2 * y[k] + y[k - 1]) / ds ** 2
            kap = (q * a - p * bb) / (a * a + bb * bb) ** mp.mpf(1.5)
            k0 = -kw * kw * b * mp.sin(kw * k * ds - om * t)
            E += Sb * (kap - k0) ** 2 * ds
        return E

    z0 = alpha * eps
    c = 1 / (z0 * mp.besselk(1, z0))

    def H(t2):
        if t2 == 0:
            return c * mp.besselk(0, z0) / (4 * mp.pi), 1 / (8 * mp.pi * eps ** 2)
        R = mp.sqrt(t2 + eps ** 2)
        z = alpha * R
        g = -c * mp.besselk(0, z) / (2 * mp.pi)
        M = c * (z * mp.besselk(1, z) - z0 * mp.besselk(1, z0)) / (2 * mp.pi * alpha ** 2)
        return M / t2 - g, (g - 2 * M / t2) / t2

    for n in range(steps):
        t = n * mp.mpf(dt)
        F = []
        for m in range(2 * N):
            F.append(-mp.diff(lambda v: energy(X[:m] + [v] + X[m + 1:], t), X[m]))
        U = [mp.mpf(0)] * (2 * N)
        for i in range(N):
            for j in range(N):
                dx, dy = X[i] - X[j], X[N + i] - X[N + j]
                h1, h2 = H(dx * dx + dy * dy)
                fd = F[j] * dx + F[N + j] * dy
                U[i] += h1 * F[j] + h2 * fd * dx
                U[N + i] += h1 * F[N + j] + h2 * fd * dy
        X = [X[m] + mp.mpf(dt) * U[m] for m in range(2 * N)]
    return np.array([float(v) for v in X])


@pytest.mark.slow
def test_tiny_run_matches_brute_force_40_digits(oracle_core):
    N, steps, dt = 4, 3, 1e-3
    pars = dict(alpha=1.3, Sb=0.2, Ss=50.0, b=0.3, k=2 * np.pi, omega=2 * np.pi)
    r = oracle_core.forward(inputs.param_rows(1, **pars), N, steps, dt, 1)
    ref = _mp_run(N, steps, dt, pars["alpha"], pars["Sb"], pars["Ss"], pars["b"], pars["k"],
                  pars["omega"], 1.5)
    got = np.concatenate([r["x"], r["y"]])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
