"""Pins of the oracle's elastic energy and forces (Appendix eqs. EFB, curva,
EFT; F = -dE/dX, eq. Fenergy).

Checks: closed-form energies of a uniformly stretched rod and of points on a
circle (whose centred-difference curvature is 2/(rho (1 + cos theta)) for an
angular step theta), the forces as the central-difference gradient of the
energy, zero net force and torque (the energy is invariant under translation
and rotation, so the swimmer is force- and torque-free, Sec. 2), and a
straight, unforced filament feeling no force.
"""
import numpy as np
import pytest


def _shape(N, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.linspace(0, 1, N)
    x = s + 0.01 * rng.standard_normal(N)
    y = 0.1 * np.sin(2 * np.pi * s + rng.uniform(0, 6)) + 0.01 * rng.standard_normal(N)
    k0 = rng.uniform(-3, 3, N)
    return x, y, k0


def test_uniform_stretch_energy(oracle_core):
    N, lam, Ss = 17, 1.013, 750.0
    ds = 1.0 / (N - 1)
    x = lam * ds * np.arange(N)
    y = np.zeros(N)
    E = oracle_core.energy(x, y, 0.3, Ss, np.zeros(N))
    assert abs(E - Ss * (lam - 1) ** 2) < 1e-14 * Ss


def test_circle_bending_energy(oracle_core):
    N, rho, Sb = 21, 0.37, 0.8
    theta = 0.11
    ang = theta * np.arange(N)
    x, y = rho * np.cos(ang), rho * np.sin(ang)
    ds = 1.0 / (N - 1)
    kap = 2.0 / (rho * (1 + np.cos(theta)))
    k0 = np.linspace(-1, 2, N)
    seg = 2 * rho * np.sin(theta / 2)
    Es = 40.0 * (N - 1) * (seg / ds - 1) ** 2 * ds
    Eb = Sb * np.sum((kap - k0[1:-1]) ** 2) * ds
    E = oracle_core.energy(x, y, Sb, 40.0, k0)
    assert abs(E - (Es + Eb)) < 1e-12 * (Es + Eb)


@pytest.mark.parametrize("N", [3, 4, 5, 8, 13])
def test_forces_are_energy_gradient(oracle_core, N):
    x, y, k0 = _shape(N, N)
    Sb, Ss = 0.37, 120.0
    fx, fy = oracle_core.forces(x, y, Sb, Ss, k0)
    h = 1e-6
    for arr, f in ((x, fx), (y, fy)):
        for k in range(N):
            ap, am = arr.copy(), arr.copy()
            ap[k] += h
            am[k] -= h
            if arr is x:
                Ep, Em = oracle_core.energy(ap, y, Sb, Ss, k0), oracle_core.energy(am, y, Sb, Ss, k0)
            else:
                Ep, Em = oracle_core.energy(x, ap, Sb, Ss, k0), oracle_core.energy(x, am, Sb, Ss, k0)
            g = (Ep - Em) / (2 * h)
            assert abs(f[k] + g) < 2e-6 * (1 + np.abs(fx).max() + np.abs(fy).max()), (k, f[k], -g)


@pytest.mark.parametrize("N", [5, 64, 128])
def test_net_force_and_torque_vanish(oracle_core, N):
    x, y, k0 = _shape(N, 100 + N)
    fx, fy = oracle_core.forces(x, y, 0.1, 1e3, k0)
    scale = np.abs(fx).sum() + np.abs(fy).sum()
    assert abs(fx.sum()) < 1e-13 * scale
    assert abs(fy.sum()) < 1e-13 * scale
    tq = np.sum(x * fy - y * fx)
    assert abs(tq) < 1e-13 * scale * (1 + np.abs(x).max())


def test_energy_invariant_under_rigid_motion(oracle_core):
    x, y, k0 = _shape(33, 5)
    E0 = oracle_core.energy(x, y, 0.2, 300.0, k0)
    c, s = np.cos(0.7), np.sin(0.7)
    xr, yr = c * x - s * y + 3.0, s * x + c * y - 1.0
    assert abs(oracle_core.energy(xr, yr, 0.2, 300.0, k0) / E0 - 1) < 1e-12


def test_straight_unforced_filament_feels_no_force(oracle_core):
    N = 40
    x = np.linspace(0, 1, N)
    y = np.zeros(N)
    fx, fy = oracle_core.forces(x, y, 0.5, 1e4, np.zeros(N))
    assert np.all(np.abs(fx) < 1e-9) and np.all(fy == 0.0)


def test_preferred_curvature(oracle_core):
    N = 9
    k0 = oracle_core.kappa0(N, 0.1, 2 * np.pi, 2 * np.pi, 0.3, 0.125)
    s = np.arange(N) / (N - 1)
    np.testing.assert_allclose(k0, -(2 * np.pi) ** 2 * 0.1 * np.sin(2 * np.pi * s - 2 * np.pi * 0.125 + 0.3),
                               rtol=1e-14, atol=1e-14)
