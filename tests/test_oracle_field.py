"""Pins of the oracle's flow and pressure at arbitrary points (Sec. 2.1,
eqs. BrFlow, BrV, BrP) for the blob of the kernel reading:

* the blob mass inside r, m(r) = 2 pi int_0^r s phi ds (closed form, with a
  series near contact), against quadrature of the blob itself; m -> 1;
* the field satisfies the regularized Brinkman equations at points between
  the forces: Delta v - alpha^2 v = grad p - sum F_i phi(x - X_i) and
  div v = 0, by high-order finite differences;
* far from the forces the pressure is that of point forces,
  sum F . x / (2 pi r^2);
* at a force point, the field's velocity is the velocity sum of the forward
  model.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import core

pytestmark = pytest.mark.usefixtures("reading_blob_module")


@pytest.mark.parametrize("alpha", [0.0, 0.4, 3.0, 10.0])
def test_blob_mass_is_the_integral_of_the_blob(alpha):
    eps = 0.03
    t = np.array([1e-10, 1e-5, 0.2 * eps ** 2, 0.3 * eps ** 2, 4 * eps ** 2, 0.5])
    phi, m = core.blob(alpha, eps, t)
    for ti, mi in zip(t, m):
        r = np.sqrt(ti)
        q, _ = integrate.quad(lambda s: 2 * np.pi * s * core.blob(alpha, eps, [s * s])[0][0], 0, r, epsabs=0,
                              epsrel=1e-13, limit=200)
        assert abs(mi * ti - q) <= 1e-12 * q
    _, m_far = core.blob(alpha, eps, [1e6])
    assert abs(m_far[0] * 1e6 - 1.0) < 1e-9


def fd_check(alpha, seed):
    eps = 0.05
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = rng.uniform(-0.1, 0.1, 6), rng.uniform(-0.1, 0.1, 6)
    FX, FY = rng.normal(size=6), rng.normal(size=6)
    x0, y0 = 0.02, 0.11    # between and near the forces
    h = 0.04 * eps

    def f(dx, dy):
        u, v, p = core.field(X, Y, FX, FY, alpha, eps, np.array([x0 + dx]), np.array([y0 + dy]))
        return np.array([u[0], v[0], p[0]])

    def d1(axis, hh):  # fourth-order first derivative
        e = np.array([hh, 0.0]) if axis == 0 else np.array([0.0, hh])
        return (-f(*(2 * e)) + 8 * f(*e) - 8 * f(*(-e)) + f(*(-2 * e))) / (12 * hh)

    def lap(hh):
        c = f(0, 0)
        return (f(hh, 0) + f(-hh, 0) + f(0, hh) + f(0, -hh) - 4 * c) / hh ** 2
    L = (4 * lap(h / 2) - lap(h)) / 3   # Richardson: fourth order
    c = f(0, 0)
    gx, gy = d1(0, h), d1(1, h)
    phi, _ = core.blob(alpha, eps, (x0 - X) ** 2 + (y0 - Y) ** 2)
    res_x = L[0] - alpha ** 2 * c[0] - gx[2] + np.sum(FX * phi)
    res_y = L[1] - alpha ** 2 * c[1] - gy[2] + np.sum(FY * phi)
    scale = max(abs(L[0]), abs(L[1]), abs(gx[2]), abs(gy[2]))
    div = gx[0] + gy[1]
    return res_x / scale, res_y / scale, div / max(abs(gx[0]), abs(gy[1]))


@pytest.mark.parametrize("alpha,seed", [(0.0, 1), (0.7, 2), (6.0, 3)])
def test_field_solves_the_regularized_brinkman_equations(alpha, seed):
    rx, ry, div = fd_check(alpha, seed)
    assert abs(rx) < 1e-5 and abs(ry) < 1e-5, (rx, ry)
    assert abs(div) < 1e-5  # fourth-order differences at h = 0.04 eps: (h/eps)^4 ~ 3e-6


def test_far_pressure_is_that_of_point_forces():
    rng = np.random.Generator(np.random.PCG64(9))
    X, Y = rng.uniform(-0.05, 0.05, 5), rng.uniform(-0.05, 0.05, 5)
    FX, FY = rng.normal(size=5), rng.normal(size=5)
    tx, ty = np.array([40.0, -3.0, 0.0]), np.array([0.0, 35.0, -50.0])
    for alpha, tol in ((0.0, 1e-5), (2.0, 1e-12)):
        _, _, p = core.field(X, Y, FX, FY, alpha, 0.01, tx, ty)
        ref = np.array([np.sum((FX * (a - X) + FY * (b - Y)) / (2 * np.pi * ((a - X) ** 2 + (b - Y) ** 2)))
                        for a, b in zip(tx, ty)])
        np.testing.assert_allclose(p, ref, rtol=tol)


def test_field_velocity_at_force_points_is_the_velocity_sum():
    rng = np.random.Generator(np.random.PCG64(10))
    X, Y = rng.uniform(0, 1, 30), rng.uniform(0, 0.2, 30)
    FX, FY = rng.normal(size=30), rng.normal(size=30)
    for alpha in (0.0, 1.5):
        u, v, _ = core.field(X, Y, FX, FY, alpha, 0.03, X, Y)
        ux, uy = core.velocity(X, Y, FX, FY, alpha, 0.03)
        np.testing.assert_allclose(u, ux, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(v, uy, rtol=1e-13, atol=1e-14)
