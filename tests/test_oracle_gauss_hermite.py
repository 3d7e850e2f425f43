"""Pins of the oracle's Gauss-Hermite line-of-sight kernels (paper section 1:
absorption-line kinematics from long-slit and integral-field spectra; reading:
the LOSVD of a bin is expanded about the Gaussian (V_b, sigma_b) given with the
data, van der Marel & Franx 1993).

Moment code 2 + m (m = 1..4) of a particle with v_los in bin b is
K = 2 sqrt(pi) alpha(nu) H_m(nu), nu = (v_los - V_b)/sigma_b.  Pinned to
  - the normalised Hermite polynomials H_m = Hp_m / sqrt(2^m m!) of numpy's
    physicists' Hermite series;
  - quadrature: the expectation of K under a Gauss-Hermite LOSVD with
    coefficients h3, h4 about (V_b, sigma_b) is (0, 0, h3, h4) for m = 1..4
    (orthonormality of the H_m under alpha^2), and a plain Gaussian of another
    width gives the closed forms of its h2, h4.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import hermite as H
from scipy import integrate

import oracle


def layout(V, sig):
    """One annulus [0.5, 2) around the line of sight z (LOS velocity = vz), binned
    twice: h1, h2 and h3, h4 (at most three moments per binning)."""
    gh = np.array([[V], [sig]])
    return {"incl": 0.0, "binnings": [
        {"kind": "annulus", "edges": np.array([0.5, 2.0]), "moments": (3, 4), "gh": gh},
        {"kind": "annulus", "edges": np.array([0.5, 2.0]), "moments": (5, 6), "gh": gh}]}


def kernel_values(lay, v):
    """The oracle's kernel entries of a particle at R = 1 with v_los = v."""
    ent = oracle.kernel_entries(lay, (1.0, 0.0, 0.3, 0.0, 0.0, v))
    return np.array([K for _, K in ent])


def test_normalised_hermite_polynomials():
    lay = layout(0.0, 1.0)
    for nu in (-2.7, -1.0, -0.3, 0.0, 0.45, 1.3, 3.1):
        got = kernel_values(lay, nu)
        want = [math.sqrt(2.0) * math.exp(-0.5 * nu * nu) * H.hermval(nu, np.eye(m + 1)[m]) /
                math.sqrt(2.0 ** m * math.factorial(m)) for m in (1, 2, 3, 4)]
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)


def test_kernel_expectation_is_the_gauss_hermite_coefficient():
    V, sig, h3, h4 = 0.3, 0.8, 0.07, -0.05
    lay = layout(V, sig)

    def losvd(v):
        w = (v - V) / sig
        a = math.exp(-0.5 * w * w) / math.sqrt(2.0 * math.pi)
        H3 = (2 * w ** 3 - 3 * w) / math.sqrt(3.0)
        H4 = (4 * w ** 4 - 12 * w ** 2 + 3) / math.sqrt(24.0)
        return a / sig * (1.0 + h3 * H3 + h4 * H4)

    got = [integrate.quad(lambda v: losvd(v) * kernel_values(lay, v)[m], V - 12 * sig, V + 12 * sig,
                          epsabs=1e-13, epsrel=1e-12, limit=200)[0] for m in range(4)]
    np.testing.assert_allclose(got, [0.0, 0.0, h3, h4], atol=2e-11)


def test_plain_gaussian_of_another_width():
    """A Gaussian of dispersion s read with sigma_b = 1: h1 = h3 = 0 and the closed
    forms h2 = (s^2 - 1)/(1 + s^2)^(3/2), h4 = (sqrt(3)/2) (s^2 - 1)^2/(1 + s^2)^(5/2),
    from E[nu^2k exp(-nu^2/2)] = (2k-1)!! s^2k / (1 + s^2)^(k + 1/2) under N(0, s^2)."""
    s = 1.4
    lay = layout(0.0, 1.0)
    g = lambda v: math.exp(-0.5 * v * v / (s * s)) / (s * math.sqrt(2 * math.pi))
    got = [integrate.quad(lambda v: g(v) * kernel_values(lay, v)[m], -15 * s, 15 * s, epsabs=1e-13,
                          epsrel=1e-12, limit=200)[0] for m in range(4)]
    h2 = (s * s - 1) / (1 + s * s) ** 1.5
    h4 = math.sqrt(3.0) / 2.0 * (s * s - 1) ** 2 / (1 + s * s) ** 2.5
    np.testing.assert_allclose(got, [0.0, h2, 0.0, h4], atol=2e-11)
