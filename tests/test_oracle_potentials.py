"""Pins of the oracle's potentials, circular-orbit angular momentum and leapfrog.

The paper (section 2) evolves particles in a potential that is fixed a priori or
self-consistent; the analytic forms and the kick-drift-kick integrator are
readings.  They are pinned here to closed forms (Hernquist 1990; the logarithmic
potential's Poisson density; NFW enclosed mass), finite differences and
time-reversibility, none of which reuse the oracle's own formulas.
"""
import numpy as np
import pytest

import oracle
from synth import configs, galaxy

HERN = {"kind": "hernquist", "G": 1.0, "M": 1.0, "a": 1.0}
LOG = {"kind": "log", "v0": 1.0, "Rc": 0.1, "q": 0.8}
HNFW = {"kind": "hernquist_nfw", "G": 1.0, "M": 1.0, "a": 1.0, "Mh": 5.0, "rs": 4.0}


def fd_grad(pot, x, h=1e-5):
    g = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        g[k] = (oracle.potential(pot, *(x + e))[0] - oracle.potential(pot, *(x - e))[0]) / (2 * h)
    return g


@pytest.mark.parametrize("pot", [HERN, LOG, HNFW])
def test_acceleration_is_minus_gradient(pot):
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.normal(0, 2.0, 3)
        phi, ax, ay, az = oracle.potential(pot, *x)
        np.testing.assert_allclose([ax, ay, az], -fd_grad(pot, x), rtol=1e-7, atol=1e-9)


def test_hernquist_closed_form():
    for r in [0.01, 0.5, 1.0, 7.0, 100.0]:
        phi = oracle.potential(HERN, 0.0, 0.0, r)[0]
        assert phi == pytest.approx(-1.0 / (r + 1.0), rel=1e-15)
    assert oracle.potential(HERN, 0.0, 0.0, 0.0)[1:] == (0.0, 0.0, 0.0)


def test_log_potential_poisson_density():
    """Laplacian of the oracle's Phi (finite differences) equals 4 pi G rho_L."""
    rng = np.random.default_rng(2)
    h = 1e-3
    for _ in range(10):
        x = rng.normal(0, 1.0, 3)
        lap = 0.0
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            lap += (oracle.potential(LOG, *(x + e))[0] - 2 * oracle.potential(LOG, *x)[0]
                    + oracle.potential(LOG, *(x - e))[0]) / h ** 2
        rho = galaxy.log_density(x[0] ** 2 + x[1] ** 2, x[2] ** 2, 1.0, 0.1, 0.8)
        assert lap == pytest.approx(4 * np.pi * rho, rel=2e-5)


def test_hnfw_enclosed_mass():
    """Gauss's law: -r^2 a_r / G = M_hernquist(r) + M_NFW(r)."""
    for r in [0.1, 1.0, 3.0, 20.0]:
        _, ax, ay, az = oracle.potential(HNFW, r, 0.0, 0.0)
        m = -ax * r * r
        expect = galaxy.hernquist_mass(r) + galaxy.nfw_mass(r, 5.0, 4.0)
        assert m == pytest.approx(expect, rel=1e-12)


def test_circular_L_hernquist_closed_form():
    """u = r_c + a solves 2E u^2 + GM u + GM a = 0; Lc = r_c sqrt(GM r_c)/(r_c + a)."""
    for E in [-0.95, -0.7, -0.5, -0.2, -0.01]:
        u = (1.0 + np.sqrt(1.0 - 8.0 * E)) / (-4.0 * E)
        rc = u - 1.0
        Lc = rc * np.sqrt(rc) / (rc + 1.0)
        assert oracle.circular_L(HERN, E) == pytest.approx(Lc, rel=1e-12)


def test_circular_L_log_closed_form():
    """For Phi_log: v_c^2 = v0^2 R^2/(Rc^2 + R^2); E_c = (v0^2/2)[R^2/(Rc^2+R^2) + ln(Rc^2+R^2)]."""
    for R in [0.01, 0.1, 0.7, 3.0, 9.0]:
        s = 0.01 + R * R
        E = 0.5 * (R * R / s + np.log(s))
        Lc = R * R / np.sqrt(s)
        assert oracle.circular_L(LOG, E) == pytest.approx(Lc, rel=1e-10)


def test_leapfrog_time_reversible():
    ics = configs.make_inputs(configs.cfg1(N=200))["ics"]
    fwd = oracle.leapfrog(HERN, ics, 500, 0.01)
    fwd[3:] *= -1
    back = oracle.leapfrog(HERN, fwd, 500, 0.01)
    back[3:] *= -1
    np.testing.assert_allclose(back, ics, rtol=0, atol=1e-10)


def test_leapfrog_circular_orbit_period():
    """Circular orbit at r = 1 in the Hernquist potential: v_c = 1/2, period 4 pi."""
    dt = 0.001
    n = int(round(4 * np.pi / dt))
    ics = np.array([[1.0], [0.0], [0.0], [0.0], [0.5], [0.0]])
    out = oracle.leapfrog(HERN, ics, n, dt)
    assert np.hypot(out[0, 0], out[1, 0]) == pytest.approx(1.0, abs=1e-6)
    assert abs(np.arctan2(out[1, 0], out[0, 0])) < 4 * np.pi * (4 * np.pi - n * dt) + 1e-4


@pytest.mark.slow
def test_leapfrog_energy_drift_cfg1():
    """Hernquist ICs, dt = 0.01, 2000 steps: median |dE/E| < 1e-4, 99th percentile < 1e-2,
    no secular growth (second-half maximum within 2x of the first-half maximum)."""
    inp = configs.make_inputs(configs.cfg1(N=4000))
    ics = inp["ics"]
    E0 = oracle.energies(HERN, ics)
    half = oracle.leapfrog(HERN, ics, 1000, 0.01)
    E1 = oracle.energies(HERN, half)
    full = oracle.leapfrog(HERN, half, 1000, 0.01)
    E2 = oracle.energies(HERN, full)
    d1 = np.abs((E1 - E0) / E0)
    d2 = np.abs((E2 - E0) / E0)
    assert np.median(d2) < 1e-4
    assert np.percentile(d2, 99) < 1e-2
    assert np.percentile(d2, 99) < 2 * max(np.percentile(d1, 99), 1e-12)
