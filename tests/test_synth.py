"""Pins of the seeded input generators (initial particle models and targets).

These fix the synthetic galaxies to textbook closed forms: the Hernquist (1990)
isotropic distribution function and mass profile, the isotropic Hernquist
dispersion, and the Poisson density of the logarithmic potential.
"""
import numpy as np
import pytest
from scipy import integrate

from synth import configs, galaxy, targets


def test_hernquist_df_normalisation():
    for r in [0.1, 1.0, 4.0]:
        phi = galaxy.hernquist_phi(r)
        vesc = np.sqrt(-2 * phi)
        val, _ = integrate.quad(lambda v: 4 * np.pi * v * v * galaxy.hernquist_df(phi + 0.5 * v * v),
                                0, vesc * (1 - 1e-12), limit=200)
        assert val == pytest.approx(galaxy.hernquist_density(r), rel=1e-8)


@pytest.mark.slow
def test_hernquist_ics_shell_masses_and_dispersion():
    """N = 1e6 sampled ICs: shell counts within 3.5 sigma (Poisson) of M(r), and the
    isotropic sigma_r^2 closed form (Hernquist 1990, eq. 10) within 2% in three shells."""
    N = 1_000_000
    ics = galaxy.hernquist_isotropic_ics(N, 99)
    r = np.linalg.norm(ics[:3], axis=0)
    e = np.geomspace(0.05, 20.0, 31)
    cnt = np.histogram(r, e)[0]
    expect = np.diff(galaxy.hernquist_mass(e)) * N
    assert np.all(np.abs(cnt - expect) < 3.5 * np.sqrt(expect))
    vr = np.sum(ics[:3] * ics[3:], axis=0) / r
    for lo, hi in [(0.4, 0.6), (0.9, 1.1), (2.5, 3.5)]:
        sel = (r > lo) & (r < hi)
        x = r[sel]
        s2 = (1 / 12.0) * (12 * x * (1 + x) ** 3 * np.log((1 + x) / x)
                           - x / (1 + x) * (25 + 52 * x + 42 * x * x + 12 * x ** 3))
        assert np.mean(vr[sel] ** 2) == pytest.approx(np.mean(s2), rel=2e-2)


def test_om_projected_dispersion_reference_values():
    """Projected LOS dispersion of the Hernquist model (isotropic and Osipkov-Merritt
    r_a = 1) at R = 0.1, 0.5, 3, 10 against independent quadrature values."""
    def Sigma(R):
        s = np.asarray(R, float)
        X = np.where(s < 1, np.arccosh(1 / np.minimum(s, 1)) / np.sqrt(np.abs(1 - s * s) + 1e-300),
                     np.arccos(1 / np.maximum(s, 1)) / np.sqrt(np.abs(s * s - 1) + 1e-300))
        return 1 / (2 * np.pi * (1 - s * s) ** 2) * ((2 + s * s) * X - 3)
    R = np.array([0.1, 0.5, 3.0, 10.0])
    iso = np.sqrt(targets.om_projected_sigma2_sigma(R, np.inf) / Sigma(R))
    om = np.sqrt(targets.om_projected_sigma2_sigma(R, 1.0) / Sigma(R))
    np.testing.assert_allclose(iso, [0.30974, 0.30676, 0.20179, 0.12342], atol=2e-5)
    np.testing.assert_allclose(om, [0.34360, 0.34929, 0.14831, 0.07553], atol=2e-5)


def test_isotropic_jeans_matches_closed_form():
    lr, P = targets.om_rho_sigr2_table(np.inf)
    for x in [0.05, 0.5, 2.0, 10.0]:
        s2 = np.exp(np.interp(np.log(x), lr, np.log(P))) / galaxy.hernquist_density(x)
        exact = (1 / 12.0) * (12 * x * (1 + x) ** 3 * np.log((1 + x) / x)
                              - x / (1 + x) * (25 + 52 * x + 42 * x * x + 12 * x ** 3))
        assert s2 == pytest.approx(exact, rel=1e-6)


def test_projected_mass_closed_form():
    for R in [0.1, 0.5, 2.0, 7.0]:
        f = lambda r: 4 * np.pi * r * r * galaxy.hernquist_density(r) * (1 - np.sqrt(max(0.0, 1 - (R / r) ** 2)))
        val = integrate.quad(f, 0, R, limit=400)[0] + integrate.quad(f, R, np.inf, limit=400)[0]
        assert targets.hernquist_projected_mass(np.array([R]))[0] == pytest.approx(val, rel=1e-6)


def test_log_sampler_density():
    """Sampled log-model positions: mass in spherical shells matches the 2D quadrature
    of rho_L (within 4 sigma Poisson)."""
    rng = np.random.default_rng(5)
    pos = galaxy.log_positions(rng, 200_000)
    r = np.linalg.norm(pos, axis=0)
    assert r.max() <= 10.0
    e = np.array([0.0, 0.1, 0.5, 1.0, 3.0, 10.0])
    cnt = np.histogram(r, e)[0]
    tot = galaxy.log_mass_within_sphere()
    frac = np.diff([galaxy.log_mass_within_sphere(rm) if rm > 0 else 0.0 for rm in e]) / tot
    assert np.all(np.abs(cnt - frac * r.size) < 4 * np.sqrt(frac * r.size))


def test_rotating_target_keeps_density_and_energy():
    ics = galaxy.log_isotropic_ics(20000, 3)
    rot = galaxy.make_rotating(ics, 0.8, 4)
    np.testing.assert_array_equal(rot[:3], ics[:3])
    np.testing.assert_allclose(np.sum(rot[3:] ** 2, axis=0), np.sum(ics[3:] ** 2, axis=0), rtol=1e-12)
    Lz = rot[0] * rot[4] - rot[1] * rot[3]
    assert np.mean(Lz > 0) > 0.85


def test_noise_is_seeded_and_sized():
    lay = configs.layout_cfg1()
    Yt, Mb = targets.hernquist_om_target(lay)
    Y1, s1 = targets.add_noise(lay, Yt, Mb, 0.05, 1)
    Y2, s2 = targets.add_noise(lay, Yt, Mb, 0.05, 1)
    np.testing.assert_array_equal(Y1, Y2)
    np.testing.assert_allclose(s1[:30], 0.05 * Yt[:30])
    np.testing.assert_allclose(s1[30:], 0.1 * Yt[30:])
    assert np.all(s1 > 0)


# ------------------------------------------- anisotropic initial models (NEXT-1)
def test_om_df_reduces_to_isotropic_closed_form():
    """Osipkov-Merritt inversion with ra -> infinity is the isotropic Hernquist DF."""
    df = galaxy.OMDF(1e6)
    E = -np.array([0.05, 0.2, 0.5, 0.8, 0.95])
    np.testing.assert_allclose(df(-E), galaxy.hernquist_df(E), rtol=1e-3)


@pytest.mark.parametrize("ra", [1.0, 0.6])
def test_om_df_reproduces_density(ra):
    """4 pi / (1 + r^2/ra^2) int w^2 f(Psi - w^2/2) dw = rho(r) (the OM velocity
    integral with w = (v_r, v_t sqrt(1 + r^2/ra^2)))."""
    from scipy import integrate
    df = galaxy.OMDF(ra)
    for r in (0.1, 1.0, 4.0):
        psi = 1.0 / (1.0 + r)
        I = integrate.quad(lambda w: w * w * df(psi - 0.5 * w * w), 0.0, np.sqrt(2 * psi), limit=400)[0]
        rho = 4.0 * np.pi * I / (1.0 + r * r / (ra * ra))
        assert rho == pytest.approx(galaxy.hernquist_density(r), rel=2e-3)


def test_tangential_df_reproduces_density():
    """2 pi^2 r int_0^Psi (Psi - e) g(e) de = rho(r) for f = L g(e)."""
    from scipy import integrate
    for r in (0.1, 1.0, 4.0):
        psi = 1.0 / (1.0 + r)
        I = integrate.quad(lambda e: (psi - e) * galaxy.tangential_g(e), 0.0, psi, limit=200)[0]
        assert 2 * np.pi ** 2 * r * I == pytest.approx(galaxy.hernquist_density(r), rel=1e-10)


def test_sampled_anisotropy_profiles():
    """Sampled models carry the anisotropy they are built with: OM beta(r) =
    r^2/(r^2 + ra^2) (shell averages), beta = -1/2, and 0 for the isotropic DF."""
    edges = np.array([0.5, 1.0, 2.0, 4.0])
    n = 100000
    rm = np.sqrt(edges[1:] * edges[:-1])
    om = galaxy.hernquist_om_ics(n, 11, 0.6)
    np.testing.assert_allclose(galaxy.anisotropy_profile(om, np.ones(n), edges), rm ** 2 / (rm ** 2 + 0.36), atol=0.04)
    tg = galaxy.hernquist_tangential_ics(n, 12)
    np.testing.assert_allclose(galaxy.anisotropy_profile(tg, np.ones(n), edges), -0.5, atol=0.04)
    iso = galaxy.hernquist_isotropic_ics(n, 13)
    np.testing.assert_allclose(galaxy.anisotropy_profile(iso, np.ones(n), edges), 0.0, atol=0.04)


def test_om_exact_target():
    """The exact Osipkov-Merritt line-of-sight sums: annulus masses against the
    closed-form projected mass, annulus v_los^2 against the Jeans quadrature,
    h3 = 0 by symmetry, and h4 against a 2^20-particle realisation of the DF
    within 4 standard errors of its shot noise."""
    los = targets.OMLineOfSight(1.0)
    e = configs.layout_cfg1()["binnings"][1]["edges"]
    sums = np.array([los.annulus_sums(e[i], e[i + 1], [lambda v: 1.0 + 0.0 * v, lambda v: v * v])
                     for i in range(len(e) - 1)])
    np.testing.assert_allclose(sums[:, 0], np.diff(targets.hernquist_projected_mass(e, 1.0, 1.0)), rtol=1e-5)
    np.testing.assert_allclose(sums[:, 1], targets.hernquist_om_annulus_moment2(e, 1.0), rtol=2e-5)
    lay = configs.layout_fig1()
    Y, Mb, gh = targets.hernquist_om_exact_target(lay, 1.0)
    nb = len(e) - 1
    assert np.all(np.abs(Y[30 + nb:30 + 2 * nb]) <= 1e-10 * Mb[30 + nb:30 + 2 * nb])
    n = 1 << 20
    real = galaxy.hernquist_om_ics(n, 21, 1.0)
    k, _ = targets._bin_index(lay["binnings"][1], real, 0.0)
    ok = k >= 0
    K = targets.gauss_hermite_kernel(4, real[5, ok] / gh[1][1][k[ok]])
    h4 = np.bincount(k[ok], weights=K, minlength=nb) / n
    se = np.sqrt(np.bincount(k[ok], weights=K * K, minlength=nb)) / n
    assert np.all(np.abs(h4 - Y[30 + 2 * nb:]) <= 4.0 * se + 1e-12), (h4 - Y[30 + 2 * nb:]) / se
