"""Pins of the oracle's regularized-Brinkmanlet kernel (eq. BrV, Sec. 2.1).

Each test checks the oracle against something other than itself: an
independent special-function library (mpmath), the governing equation
(BrFlow) and the incompressibility it implies, textbook limits (singular
Brinkmanlet far field, regularized Stokeslet as alpha -> 0), and a published
closed form (Cortez 2001) for the assembly of H1, H2 from G.
"""
import mpmath as mp
import numpy as np
import pytest

pytestmark = pytest.mark.usefixtures("reading_blob_module")

EPS64 = 1.5 / 63      # blob width at N = 64
EPS512 = 1.5 / 511    # blob width at N = 512


def mpf(x):
    return mp.mpf(float(x))


def blob(alpha, eps, r):
    """Blob of the kernel reading: phi = c eps^2/(2 pi) [a^2 K0(aR)/R^2 + 2 a K1(aR)/R^3],
    c = 1/(a eps K1(a eps)); at alpha = 0 it is eps^2/(pi R^4)."""
    alpha, eps, r = mpf(alpha), mpf(eps), mp.mpf(r)
    R = mp.sqrt(r * r + eps * eps)
    if alpha == 0:
        return eps ** 2 / (mp.pi * R ** 4)
    c = 1 / (alpha * eps * mp.besselk(1, alpha * eps))
    return c * eps ** 2 / (2 * mp.pi) * (alpha ** 2 * mp.besselk(0, alpha * R) / R ** 2
                                         + 2 * alpha * mp.besselk(1, alpha * R) / R ** 3)


def test_bessel_matches_mpmath(oracle_core):
    mp.mp.dps = 40
    z = np.logspace(-9, np.log10(120.0), 97)
    k0, k1, q = oracle_core.bessel(z)
    for i, zi in enumerate(z):
        Z = mpf(zi)
        assert abs(k0[i] / float(mp.besselk(0, Z)) - 1) < 4e-16
        assert abs(k1[i] / float(mp.besselk(1, Z)) - 1) < 4e-16
        assert abs(q[i] / float(Z * mp.besselk(1, Z) - 1) - 1) < 1e-15


@pytest.mark.parametrize("alpha", [0.3, 1.0, 10.0])
def test_blob_is_positive_unit_mass(alpha):
    mp.mp.dps = 30
    eps = EPS64
    mass = mp.quad(lambda r: 2 * mp.pi * r * blob(alpha, eps, r), [0, eps, 10 * eps, 1, mp.inf])
    assert abs(mass - 1) < 1e-20
    for r in [0, 0.3 * eps, eps, 5 * eps, 0.5, 3.0]:
        assert blob(alpha, eps, r) > 0


def test_blob_tends_to_stokes_blob():
    mp.mp.dps = 30
    for r in [0, EPS64, 0.3]:
        a = blob(1e-7, EPS64, r)
        b = blob(0.0, EPS64, r)
        assert abs(a / b - 1) < 1e-10


def _closed_form_mp(alpha, eps, t):
    """The kernel closed form evaluated in 60-digit arithmetic."""
    mp.mp.dps = 60
    alpha, eps, t = mpf(alpha), mpf(eps), mpf(t)
    R = mp.sqrt(t + eps ** 2)
    if alpha == 0:
        d = t / eps ** 2
        return ((-mp.log(R) + mp.log1p(d) / (2 * d) - mp.mpf(1) / 2) / (4 * mp.pi),
                (1 / (2 * t) - mp.log1p(d) / (2 * t * d)) / (2 * mp.pi))
    z0 = alpha * eps
    c = 1 / (z0 * mp.besselk(1, z0))
    z = alpha * R
    g = -c * mp.besselk(0, z) / (2 * mp.pi)
    M = c * (z * mp.besselk(1, z) - z0 * mp.besselk(1, z0)) / (2 * mp.pi * alpha ** 2)
    return M / t - g, (g - 2 * M / t) / t


@pytest.mark.parametrize("alpha", [0.0, 1e-8, 1e-3, 0.5, 2.0, 10.0, 40.0])
@pytest.mark.parametrize("eps", [EPS64, EPS512])
def test_kernel_rounding_accuracy(oracle_core, alpha, eps):
    """The oracle's extended-precision evaluation (closed form, or its Taylor
    series near contact) agrees with the closed form at 60 digits."""
    dl = np.array([1e-7, 1e-3, 0.2, 0.249, 0.251, 0.44, 1.78, 10.0, 1e3, 1e5])
    H1, H2 = oracle_core.kernel(alpha, eps, eps ** 2 * dl)
    for i, d in enumerate(dl):
        a, b = _closed_form_mp(alpha, eps, eps ** 2 * d)
        scale1 = max(abs(float(a)), 1e-3)
        assert abs(H1[i] - float(a)) / scale1 < 2e-15, (d, H1[i], float(a))
        assert abs(H2[i] / float(b) - 1) < 2e-15, (d, H2[i], float(b))


def _fd(f, r, h):
    fp2, fp1, f0, fm1, fm2 = f(r + 2 * h), f(r + h), f(r), f(r - h), f(r - 2 * h)
    d1 = (-fp2 + 8 * fp1 - 8 * fm1 + fm2) / (12 * h)
    d2 = (-fp2 + 16 * fp1 - 30 * f0 + 16 * fm1 - fm2) / (12 * h * h)
    return f0, d1, d2


@pytest.mark.parametrize("alpha", [0.0, 0.5, 2.0, 10.0])
def test_velocity_field_is_divergence_free(oracle_core, alpha):
    """div v = (F.x) [H1'/r + r H2' + 3 H2] must vanish (Brinkman flow is
    incompressible, eq. BrFlow)."""
    eps = EPS64
    H1f = lambda r: oracle_core.kernel(alpha, eps, np.array([r * r]))[0][0]
    H2f = lambda r: oracle_core.kernel(alpha, eps, np.array([r * r]))[1][0]
    for r in [0.7 * eps, 1.3 * eps, 4 * eps, 0.2, 0.9]:
        h = 0.01 * min(r, eps)
        h1, dh1, _ = _fd(H1f, r, h)
        h2, dh2, _ = _fd(H2f, r, h)
        div = dh1 / r + r * dh2 + 3 * h2
        scale = abs(dh1 / r) + abs(r * dh2) + abs(3 * h2)
        assert abs(div) < 1e-7 * scale, (r, div, scale)


@pytest.mark.parametrize("alpha", [0.0, 0.5, 2.0, 10.0])
def test_velocity_field_solves_brinkman(oracle_core, alpha):
    """With H1 = -B'', H2 = (r B'' - B')/r^3, the function g = Delta B =
    -2 H1 - r^2 H2 must satisfy (Delta - alpha^2) g = phi (eq. BrFlow with
    the regularized force F phi)."""
    mp.mp.dps = 30
    eps = EPS64

    def g(r):
        H1, H2 = oracle_core.kernel(alpha, eps, np.array([r * r]))
        return -2 * H1[0] - r * r * H2[0]

    for r in [0.5 * eps, eps, 3 * eps, 0.15, 0.6]:
        h = 0.01 * min(r, eps)
        f0, d1, d2 = _fd(g, r, h)
        lhs = d2 + d1 / r - alpha ** 2 * f0
        rhs = float(blob(alpha, eps, r))
        scale = abs(d2) + abs(d1 / r) + alpha ** 2 * abs(f0) + abs(rhs)
        assert abs(lhs - rhs) < 2e-7 * scale, (r, lhs, rhs)


@pytest.mark.parametrize("alpha", [1.0, 3.0, 10.0])
def test_far_field_is_singular_brinkmanlet(oracle_core, alpha):
    """For alpha r >> 1: H1 r^2 -> -1/(2 pi alpha^2), H2 r^4 -> 1/(pi alpha^2)."""
    r = 45.0 / alpha
    H1, H2 = oracle_core.kernel(alpha, EPS64, np.array([r * r]))
    assert abs(H1[0] * r * r / (-1 / (2 * np.pi * alpha ** 2)) - 1) < 1e-13
    assert abs(H2[0] * r ** 4 / (1 / (np.pi * alpha ** 2)) - 1) < 1e-13


def test_stokes_limit(oracle_core):
    """As alpha -> 0, H2 -> the Stokes H2, and H1 - H1_Stokes tends to the
    r-independent constant -(ln(alpha/2) + gamma)/(4 pi)."""
    eps = EPS64
    t = eps ** 2 * np.array([0.01, 0.44, 3.0, 100.0, 1500.0])
    H1s, H2s = oracle_core.kernel(0.0, eps, t)
    for alpha, tol in [(1e-4, 1e-6), (1e-6, 1e-10)]:
        H1, H2 = oracle_core.kernel(alpha, eps, t)
        np.testing.assert_allclose(H2, H2s, rtol=tol)
        const = -(np.log(alpha / 2) + np.euler_gamma) / (4 * np.pi)
        np.testing.assert_allclose(H1 - H1s, const, rtol=tol)


def test_values_at_contact(oracle_core):
    """H1(0) = c K0(alpha eps)/(4 pi), H2(0) = 1/(8 pi eps^2); Stokes H1(0) = -ln(eps)/(4 pi)."""
    mp.mp.dps = 30
    eps = EPS64
    for alpha in [0.0, 0.7, 9.0]:
        H1, H2 = oracle_core.kernel(alpha, eps, np.array([0.0]))
        if alpha == 0:
            h1 = -np.log(eps) / (4 * np.pi)
        else:
            z0 = mpf(alpha) * mpf(eps)
            h1 = float(mp.besselk(0, z0) / (z0 * mp.besselk(1, z0)) / (4 * mp.pi))
        assert abs(H1[0] / h1 - 1) < 1e-15
        assert abs(H2[0] * 8 * np.pi * eps ** 2 - 1) < 1e-15


def test_assembly_reproduces_cortez_2001():
    """The route H1 = M/r^2 - G, H2 = (G - 2 M/r^2)/r^2 with M = int_0^r s G ds,
    fed the Stokes G of the paper's own blob (eq. eqnblob), reproduces the
    published 2D regularized Stokeslet of Cortez (2001):
      H1 = -[ln(R+e) - e(R+2e)/(R(R+e))]/(4 pi),  H2 = (R+2e)/(4 pi R (R+e)^2).
    In 2D Stokes flow a uniform velocity is a homogeneous solution, so H1 is
    fixed only up to an additive constant: H1 is compared through differences."""
    mp.mp.dps = 40
    e = mp.mpf("0.045")
    G = lambda r: (mp.log(mp.sqrt(r * r + e * e) + e) - e / mp.sqrt(r * r + e * e)) / (2 * mp.pi)
    # Delta G equals the paper's blob 3 e^3 / (2 pi R^5)
    for r in [mp.mpf("0.01"), mp.mpf("0.2")]:
        lap = mp.diff(G, r, 2) + mp.diff(G, r, 1) / r
        assert abs(lap - 3 * e ** 3 / (2 * mp.pi * (r * r + e * e) ** mp.mpf(2.5))) < mp.mpf(10) ** -30
    def route(r):
        M = mp.quad(lambda s: s * G(s), [0, r])
        return M / r ** 2 - G(r), (G(r) - 2 * M / r ** 2) / r ** 2

    def cortez(r):
        R = mp.sqrt(r * r + e * e)
        return (-(mp.log(R + e) - e * (R + 2 * e) / (R * (R + e))) / (4 * mp.pi),
                (R + 2 * e) / (4 * mp.pi * R * (R + e) ** 2))

    r0 = mp.mpf("0.02")
    a0, c0 = route(r0)[0], cortez(r0)[0]
    for r in [mp.mpf("0.003"), mp.mpf("0.05"), mp.mpf("0.7")]:
        (H1, H2), (C1, C2) = route(r), cortez(r)
        assert abs((H1 - a0) - (C1 - c0)) < mp.mpf(10) ** -28
        assert abs(H2 - C2) < mp.mpf(10) ** -28


def test_mobility_is_symmetric_positive_definite(oracle_core):
    """A positive blob gives an SPD mobility (the regularized flow dissipates
    energy); symmetry follows from H depending on |x_i - X_j| only."""
    from paper_1910_12007_amd import inputs
    N = 24
    x, y = inputs.filament_geometry(N, seed=7)
    for alpha in [0.0, 2.0]:
        Mmat = np.zeros((2 * N, 2 * N))
        for j in range(2 * N):
            f = np.zeros(2 * N)
            f[j] = 1.0
            ux, uy = oracle_core.velocity(x, y, f[:N], f[N:], alpha, 1.5 / (N - 1))
            Mmat[:, j] = np.concatenate([ux, uy])
        np.testing.assert_allclose(Mmat, Mmat.T, atol=1e-15 * np.abs(Mmat).max())
        np.linalg.cholesky(0.5 * (Mmat + Mmat.T))
