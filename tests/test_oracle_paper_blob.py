"""Pins of the oracle's kernel for the paper's own blob, phi = 3 eps^3 /
(2 pi (r^2 + eps^2)^(5/2)) (eq. eqnblob), in the Stokes limit:

* H2 equals the published regularized Stokeslet of this blob (Cortez,
  Fauci & Medovikov 2005, 2D), H1 equals it up to the constant -1/(8 pi)
  that the 2D H1 leaves free (the oracle's route H1 = M/r^2 - G fixes it);
* the blob has unit mass (the paper's normalization int r phi dr = 1/(2 pi)),
  and the mass inside r, 1 - eps^3/R^3, equals the integral of the blob;
* velocity and pressure of a few forces satisfy the regularized Stokes
  equations Delta v = grad p - sum F phi(x - X_i), div v = 0, at field
  points (fourth-order differences).
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import core

import test_oracle_field as tof


def test_matches_the_published_regularized_stokeslet():
    eps = 0.03
    t = np.concatenate([[0.0, 1e-9, 1e-6], np.geomspace(1e-5, 100.0, 60)])
    with core.paper_blob():
        H1, H2 = core.kernel(0.0, eps, t)
    R = np.sqrt(t + eps ** 2)
    H1c = -(np.log(R + eps) - eps * (R + 2 * eps) / (R * (R + eps))) / (4 * np.pi)
    H2c = (R + 2 * eps) / (4 * np.pi * R * (R + eps) ** 2)
    np.testing.assert_allclose(H2, H2c, rtol=2e-15, atol=0)
    np.testing.assert_allclose(H1, H1c - 1 / (8 * np.pi), rtol=2e-15, atol=1e-17)


def test_blob_mass():
    eps = 0.05
    with core.paper_blob():
        phi, m = core.blob(0.0, eps, [1e-6, 0.1 * eps ** 2, eps ** 2, 9 * eps ** 2, 1.0])
        total, _ = integrate.quad(lambda r: r * core.blob(0.0, eps, [r * r])[0][0], 0, np.inf, epsabs=0,
                                  epsrel=1e-12, limit=400)
        for tt, mm in zip([1e-6, 0.1 * eps ** 2, eps ** 2, 9 * eps ** 2, 1.0], m):
            q, _ = integrate.quad(lambda s: 2 * np.pi * s * core.blob(0.0, eps, [s * s])[0][0], 0, np.sqrt(tt),
                                  epsabs=0, epsrel=1e-13, limit=200)
            assert abs(mm * tt - q) <= 1e-12 * q
            R = np.sqrt(tt + eps ** 2)
            assert abs(mm * tt - (1 - eps ** 3 / R ** 3)) <= 1e-14
        phi0, _ = core.blob(0.0, eps, [0.0])
    assert abs(total - 1 / (2 * np.pi)) < 1e-12
    assert phi0[0] == pytest.approx(3 / (2 * np.pi * eps ** 2), rel=1e-15)


@pytest.mark.parametrize("seed", [1, 2])
def test_field_solves_the_regularized_stokes_equations(seed):
    with core.paper_blob():
        rx, ry, div = tof.fd_check(0.0, seed)
    assert abs(rx) < 1e-5 and abs(ry) < 1e-5, (rx, ry)
    assert abs(div) < 1e-5
