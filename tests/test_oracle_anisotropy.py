"""Pins of the oracle's shell velocity moments (paper section 3, Fig. 1: the
anisotropy beta(r) = 1 - (<v_theta^2> + <v_phi^2>) / (2 <v_r^2>) recovered for a
spherical target).

Particles are placed at chosen spherical coordinates (r, theta, phi) with chosen
spherical velocity components (v_r, v_theta, v_phi), turned into Cartesian
vectors with the textbook trigonometric unit vectors -- a construction the
oracle's cross-product basis does not share -- and the sums must come back.
"""
import numpy as np

import oracle


def spherical_particles(r, th, ph, vr, vt, vp):
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    er = np.stack([st * cp, st * sp, ct])
    et = np.stack([ct * cp, ct * sp, -st])
    ep = np.stack([-sp, cp, np.zeros_like(ph)])
    return np.vstack([r * er, vr * er + vt * et + vp * ep])


def test_spherical_components_come_back():
    rng = np.random.default_rng(12)
    n = 400
    r = rng.uniform(0.2, 5.0, n)
    th = np.arccos(rng.uniform(-0.99, 0.99, n))
    ph = rng.uniform(0.0, 2 * np.pi, n)
    vr, vt, vp = rng.normal(0, 1.0, (3, n))
    w = rng.uniform(0.1, 2.0, n)
    ics = spherical_particles(r, th, ph, vr, vt, vp)
    edges = np.array([0.5, 1.0, 2.0, 4.0])
    got = oracle.shell_moments(ics, w, edges)
    k = np.searchsorted(edges, r, side="right") - 1
    ok = (k >= 0) & (k < 3)
    want = np.stack([np.bincount(k[ok], weights=(w * q)[ok], minlength=3) for q in (1.0 + 0 * r, vr ** 2, vt ** 2, vp ** 2)])
    np.testing.assert_allclose(got, want, rtol=1e-12)


def test_radial_and_circular_orbits():
    """Purely radial motion gives beta = 1; purely tangential motion gives no v_r; unit
    velocities along the three axes at each position (an orthonormal set of
    directions) give beta = 0."""
    r = np.array([1.0, 1.0, 1.0])
    th = np.array([0.3, 1.2, 2.5])
    ph = np.array([0.1, 2.0, 4.0])
    one = np.ones(3)
    rad = oracle.shell_moments(spherical_particles(r, th, ph, 2.0 * one, 0 * one, 0 * one), one, [0.5, 2.0])
    assert abs(rad[2, 0]) < 1e-28 and abs(rad[3, 0]) < 1e-28
    assert rad[1, 0] == 12.0
    circ = oracle.shell_moments(spherical_particles(r, th, ph, 0 * one, one, one), one, [0.5, 2.0])
    assert abs(circ[1, 0]) < 1e-28
    np.testing.assert_allclose(circ[2:, 0], [3.0, 3.0], rtol=1e-14)
    x = np.array([[1, 0, 0], [0, 1, 0], [0, 0.6, 0.8]], dtype=float).T * 1.5
    ics = np.vstack([np.repeat(x, 3, axis=1), np.tile(np.eye(3), 3)])
    m = oracle.shell_moments(ics, np.ones(9), [1.0, 2.0])
    assert abs(1.0 - (m[2, 0] + m[3, 0]) / (2 * m[1, 0])) < 1e-14


def test_half_open_shells_and_axis():
    """r exactly at an inner edge belongs to the outer shell; r = edges[-1] to none;
    on the z axis v_phi = 0 and the whole tangential motion is v_theta."""
    ics = np.array([[0.0, 0.0, 1.0, 0.3, 0.4, 0.5],     # r = 1: shell 0, on the axis
                    [0.0, 0.0, 2.0, 0.0, 0.0, 1.0],     # r = 2 = outer edge: no shell
                    [0.0, 0.0, 1.5, 0.8, 0.0, 0.0]]).T  # r = 1.5 = inner edge of shell 1
    m = oracle.shell_moments(ics, np.array([1.0, 2.0, 4.0]), [1.0, 1.5, 2.0])
    np.testing.assert_allclose(m[0], [1.0, 4.0])
    np.testing.assert_allclose(m[:, 0], [1.0, 0.25, 0.09 + 0.16, 0.0])
    np.testing.assert_allclose(m[:, 1], [4.0, 0.0, 4 * 0.64, 0.0])
