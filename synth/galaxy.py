"""Initial particle models (positions, velocities) for the synthetic galaxies.

The paper (section 2) evolves an N-body particle system in a galaxy potential and
starts from weights 1/N (section 2.1).  It names no particular galaxy model, so
the workloads use textbook models:

* Hernquist (1990, ApJ 356, 359) sphere, G = M = a = 1: isotropic distribution
  function f(E), mass profile M(r) = M r^2/(r+a)^2.
* Axisymmetric logarithmic potential Phi = v0^2/2 ln(Rc^2 + R^2 + z^2/q^2)
  (Binney & Tremaine 2008, eq. 2.71), with its Poisson density, truncated at r<=10.
* Hernquist stars in a Hernquist + NFW total potential, velocities from the
  spherical Jeans equation.

Every sampler is seeded; arrays are float64 structure-of-arrays (x, y, z, vx, vy, vz).
"""
import numpy as np
from scipy import integrate, interpolate

SEED_BASE = 12076403


def seed_for(cfg_index, offset=0):
    """Seed of configuration ``cfg_index`` (1..5): base + 1000*k, +1 for target
    noise, +2 for MLP initialisation and training subsets."""
    return SEED_BASE + 1000 * cfg_index + offset


# ---------------------------------------------------------------- Hernquist
def hernquist_mass(r, M=1.0, a=1.0):
    return M * r * r / (r + a) ** 2


def hernquist_phi(r, G=1.0, M=1.0, a=1.0):
    return -G * M / (r + a)


def hernquist_density(r, M=1.0, a=1.0):
    return M * a / (2.0 * np.pi * r * (r + a) ** 3)


def hernquist_df(E, G=1.0, M=1.0, a=1.0):
    """Isotropic Hernquist distribution function f(E) (Hernquist 1990, eq. 17)."""
    q2 = -a * E / (G * M)
    q = np.sqrt(q2)
    vg = np.sqrt(G * M / a)
    pref = M / (8.0 * np.sqrt(2.0) * np.pi ** 3 * a ** 3 * vg ** 3)
    return pref * (1 - q2) ** -2.5 * (3 * np.arcsin(q) + q * np.sqrt(1 - q2) * (1 - 2 * q2)
                                      * (8 * q2 * q2 - 8 * q2 - 3))


def _isotropic_directions(rng, n):
    ct = rng.uniform(-1.0, 1.0, n)
    st = np.sqrt(1.0 - ct * ct)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    return st * np.cos(ph), st * np.sin(ph), ct


def hernquist_positions(rng, n, a=1.0, rmax=None):
    """Radii by inverting M(r)/M = u: r = a sqrt(u)/(1 - sqrt(u))."""
    umax = 1.0 if rmax is None else hernquist_mass(rmax, 1.0, a)
    u = rng.uniform(0.0, umax, n)
    su = np.sqrt(u)
    r = a * su / (1.0 - su)
    ex, ey, ez = _isotropic_directions(rng, n)
    return r * ex, r * ey, r * ez


def hernquist_isotropic_ics(n, seed, G=1.0, M=1.0, a=1.0):
    """Positions from M(r); speeds by rejection from v^2 f(Phi + v^2/2) on [0, v_esc]."""
    rng = np.random.default_rng(seed)
    x, y, z = hernquist_positions(rng, n, a)
    r = np.sqrt(x * x + y * y + z * z)
    phi = hernquist_phi(r, G, M, a)
    vesc = np.sqrt(-2.0 * phi)
    # per-particle envelope: max of p(v) on a grid dense near v = 0, times a margin
    s = np.linspace(0.0, 1.0, 129)[1:-1]
    bound = np.zeros(n)
    for k in range(0, n, 65536):
        sl = slice(k, k + 65536)
        v = vesc[sl, None] * s[None, :] ** 2
        p = v * v * hernquist_df(phi[sl, None] + 0.5 * v * v, G, M, a)
        bound[sl] = 1.5 * p.max(axis=1)
    speed = np.empty(n)
    todo = np.arange(n)
    worst = 0.0
    while todo.size:
        v = rng.uniform(0.0, 1.0, todo.size) * vesc[todo]
        p = v * v * hernquist_df(phi[todo] + 0.5 * v * v, G, M, a)
        worst = max(worst, float(np.max(p / bound[todo])))
        acc = rng.uniform(0.0, 1.0, todo.size) * bound[todo] < p
        speed[todo[acc]] = v[acc]
        todo = todo[~acc]
    if worst > 1.0:
        raise RuntimeError("rejection envelope too low (%.3f)" % worst)
    ex, ey, ez = _isotropic_directions(rng, n)
    return np.stack([x, y, z, speed * ex, speed * ey, speed * ez])


# ------------------------------------------------- anisotropic Hernquist models
# Initial models of the convergence experiment (paper section 3), G = M = a = 1, in
# terms of the relative potential Psi = -Phi = 1/(1 + r) (r = (1 - Psi)/Psi) and
# the binding energy eps = Psi - v^2/2.
#
# Osipkov-Merritt (anisotropy radius ra): f = f(Q), Q = eps - L^2/(2 ra^2), from the
# Eddington inversion of rho_Q = (1 + r^2/ra^2) rho, which for the Hernquist
# sphere is rho_Q(Psi) = [Psi^4/(1 - Psi) + (Psi^2 - Psi^3)/ra^2] / (2 pi):
#   f(Q) = 1/(sqrt(8) pi^2) int_0^Q rho_Q''(Psi) dPsi / sqrt(Q - Psi)
# (d rho_Q/d Psi vanishes at Psi = 0); beta(r) = r^2/(r^2 + ra^2).
#
# Tangential, constant beta = -1/2: f = L g(eps).  Then rho/r = 2 pi^2
# int_0^Psi (Psi - e) g(e) de, so g = (rho/r)''/(2 pi^2) with
# rho/r = Psi^5/(2 pi (1 - Psi)^2).

def om_rhoq_pp(psi, ra):
    """Second derivative of rho_Q(Psi) of the Osipkov-Merritt Hernquist model."""
    u = 1.0 - psi
    app = 12.0 * psi ** 2 / u + 2.0 * psi ** 3 * (4.0 - 3.0 * psi) / u ** 3
    bpp = (2.0 - 6.0 * psi) / (ra * ra)
    return (app + bpp) / (2.0 * np.pi)


def om_df_table(ra, n=1200):
    """f(Q) of the Osipkov-Merritt Hernquist model on Q in (0, 1): the Eddington
    integral with Psi = Q - u^2 (dPsi / sqrt(Q - Psi) = 2 du), by adaptive
    quadrature.  Returns (Q, f); galaxy.OMDF interpolates ln f in ln Q."""
    # geometric in Q towards 0 and in 1 - Q towards 1
    Q = np.concatenate([np.geomspace(1e-7, 0.5, n // 2, endpoint=False), 1.0 - np.geomspace(0.5, 1e-7, n // 2)])
    f = np.empty(Q.size)
    for k, q in enumerate(Q):
        f[k] = integrate.quad(lambda u: 2.0 * om_rhoq_pp(q - u * u, ra), 0.0, np.sqrt(q),
                              epsabs=0.0, epsrel=1e-10, limit=400)[0]
    return Q, f / (np.sqrt(8.0) * np.pi ** 2)


class OMDF:
    """Interpolated f(Q) of the Osipkov-Merritt Hernquist model (0 for Q <= 0)."""

    def __init__(self, ra):
        self.ra = ra
        Q, f = om_df_table(ra)
        if np.any(f < 0):
            raise ValueError("Osipkov-Merritt Hernquist model with ra=%g is unphysical (f < 0)" % ra)
        self._x = np.log(Q)
        self._y = np.log(np.maximum(f, 1e-300))

    def __call__(self, Q):
        Q = np.asarray(Q, dtype=np.float64)
        out = np.zeros(Q.shape)
        ok = (Q > 0) & (Q < 1)
        out[ok] = np.exp(np.interp(np.log(Q[ok]), self._x, self._y))
        return out


def tangential_g(eps):
    """g(eps) of the beta = -1/2 Hernquist model f = L g(eps): (rho/r)''/(2 pi^2)."""
    eps = np.asarray(eps, dtype=np.float64)
    u = 1.0 - eps
    cpp = 20.0 * eps ** 3 / u ** 2 + 20.0 * eps ** 4 / u ** 3 + 6.0 * eps ** 5 / u ** 4
    return np.where((eps > 0) & (eps < 1), cpp / (4.0 * np.pi ** 3), 0.0)


def _rejection(rng, n, bound, sample, density):
    """Rejection sampling of n values with per-item envelopes `bound` (proposal
    sample(idx) on the item's support, unnormalised density(values, idx))."""
    out = np.empty(n)
    todo = np.arange(n)
    worst = 0.0
    while todo.size:
        v = sample(todo)
        p = density(v, todo)
        worst = max(worst, float(np.max(p / bound[todo])))
        acc = rng.uniform(0.0, 1.0, todo.size) * bound[todo] < p
        out[todo[acc]] = v[acc]
        todo = todo[~acc]
    if worst > 1.0:
        raise RuntimeError("rejection envelope too low (%.3f)" % worst)
    return out


def _envelope(n, dens_on_grid):
    s = np.linspace(0.0, 1.0, 257)[1:-1]
    b = np.zeros(n)
    for k in range(0, n, 32768):
        sl = slice(k, k + 32768)
        b[sl] = 1.5 * dens_on_grid(s, sl).max(axis=1)
    return b


def _tangential_frame(x, y, z, rng):
    """Unit vectors r_hat and two tangential directions per particle."""
    r = np.sqrt(x * x + y * y + z * z)
    er = np.stack([x, y, z]) / r
    a = rng.normal(0.0, 1.0, (3, x.size))
    e1 = a - er * (a * er).sum(axis=0)
    e1 /= np.linalg.norm(e1, axis=0)
    e2 = np.cross(er.T, e1.T).T
    return r, er, e1, e2


def hernquist_om_ics(n, seed, ra):
    """Osipkov-Merritt Hernquist initial model: positions from M(r); velocities with
    w = (v_r, v_t sqrt(1 + r^2/ra^2)) isotropic and |w| drawn from w^2 f(Psi - w^2/2)."""
    rng = np.random.default_rng(seed)
    df = OMDF(ra)
    x, y, z = hernquist_positions(rng, n)
    r, er, e1, e2 = _tangential_frame(x, y, z, rng)
    psi = 1.0 / (1.0 + r)
    wmax = np.sqrt(2.0 * psi)
    dens = lambda w, idx: w * w * df(psi[idx] - 0.5 * w * w)
    bound = _envelope(n, lambda s, sl: (wmax[sl, None] * s) ** 2 * df(psi[sl, None] * (1.0 - s * s)))
    w = _rejection(rng, n, bound, lambda idx: rng.uniform(0.0, 1.0, idx.size) * wmax[idx], dens)
    ct = rng.uniform(-1.0, 1.0, n)
    st = np.sqrt(1.0 - ct * ct)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    vr = w * ct
    vt = w * st / np.sqrt(1.0 + (r / ra) ** 2)
    v = er * vr + (e1 * np.cos(ph) + e2 * np.sin(ph)) * vt
    return np.concatenate([np.stack([x, y, z]), v])


def hernquist_tangential_ics(n, seed):
    """beta = -1/2 Hernquist initial model f = L g(eps): positions from M(r); speed
    from v^3 g(Psi - v^2/2), angle eta to r_hat from sin^2(eta)."""
    rng = np.random.default_rng(seed)
    x, y, z = hernquist_positions(rng, n)
    r, er, e1, e2 = _tangential_frame(x, y, z, rng)
    psi = 1.0 / (1.0 + r)
    vmax = np.sqrt(2.0 * psi)
    dens = lambda v, idx: v ** 3 * tangential_g(psi[idx] - 0.5 * v * v)
    bound = _envelope(n, lambda s, sl: (vmax[sl, None] * s) ** 3 * tangential_g(psi[sl, None] * (1.0 - s * s)))
    v = _rejection(rng, n, bound, lambda idx: rng.uniform(0.0, 1.0, idx.size) * vmax[idx], dens)
    eta = _rejection(rng, n, np.ones(n), lambda idx: rng.uniform(0.0, np.pi, idx.size),
                     lambda e, idx: np.sin(e) ** 2)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    vel = er * (v * np.cos(eta)) + (e1 * np.cos(ph) + e2 * np.sin(ph)) * (v * np.sin(eta))
    return np.concatenate([np.stack([x, y, z]), vel])


def anisotropy_profile(ics, w, edges):
    """beta(r) = 1 - (sigma_theta^2 + sigma_phi^2)/(2 sigma_r^2) of a weighted
    particle model in radial shells (second moments about zero: the models are
    non-rotating)."""
    x, y, z, vx, vy, vz = ics
    r = np.sqrt(x * x + y * y + z * z)
    vr = (x * vx + y * vy + z * vz) / r
    v2 = vx * vx + vy * vy + vz * vz
    k = np.digitize(r, edges) - 1
    ok = (k >= 0) & (k < len(edges) - 1)
    nb = len(edges) - 1
    sr = np.bincount(k[ok], weights=(w * vr * vr)[ok], minlength=nb)
    st = np.bincount(k[ok], weights=(w * (v2 - vr * vr))[ok], minlength=nb)
    return 1.0 - st / (2.0 * sr)


# ---------------------------------------------------------- logarithmic potential
def log_density(R2, z2, v0=1.0, Rc=0.1, q=0.8, G=1.0):
    """Poisson density of Phi = v0^2/2 ln(Rc^2 + R^2 + z^2/q^2)."""
    num = (2 * q * q + 1) * Rc * Rc + R2 + (2 - 1.0 / (q * q)) * z2
    den = (Rc * Rc + R2 + z2 / (q * q)) ** 2
    return v0 * v0 / (4 * np.pi * G * q * q) * num / den


def log_positions(rng, n, v0=1.0, Rc=0.1, q=0.8, rmax=10.0):
    """Rejection sampling of rho_L inside r <= rmax.  Proposal: spherical density
    proportional to 1/(r^2 + Rc^2), radii by inverting r - Rc atan(r/Rc)."""
    rt = np.linspace(0.0, rmax, 200001)
    cdf = rt - Rc * np.arctan(rt / Rc)
    inv = interpolate.interp1d(cdf / cdf[-1], rt)
    # envelope constant: max of rho_L (r^2 + Rc^2) over a (r, cos theta) grid
    rr = np.concatenate([[0.0], np.geomspace(1e-4, rmax, 400)])
    ct = np.linspace(-1.0, 1.0, 201)
    R2 = (rr[:, None] ** 2) * (1 - ct[None, :] ** 2)
    z2 = (rr[:, None] ** 2) * ct[None, :] ** 2
    ratio = log_density(R2, z2, v0, Rc, q) * (rr[:, None] ** 2 + Rc * Rc)
    cmax = 1.05 * ratio.max()
    out = np.empty((3, n))
    filled = 0
    worst = 0.0
    while filled < n:
        m = int((n - filled) * 2.2) + 1024
        r = inv(rng.uniform(0.0, 1.0, m))
        ex, ey, ez = _isotropic_directions(rng, m)
        x, y, z = r * ex, r * ey, r * ez
        rat = log_density(x * x + y * y, z * z, v0, Rc, q) * (r * r + Rc * Rc) / cmax
        worst = max(worst, float(rat.max()))
        acc = rng.uniform(0.0, 1.0, m) < rat
        k = min(int(acc.sum()), n - filled)
        idx = np.nonzero(acc)[0][:k]
        out[0, filled:filled + k] = x[idx]
        out[1, filled:filled + k] = y[idx]
        out[2, filled:filled + k] = z[idx]
        filled += k
    if worst > 1.0:
        raise RuntimeError("rejection envelope too low (%.3f)" % worst)
    return out


def log_isotropic_ics(n, seed, v0=1.0, Rc=0.1, q=0.8, rmax=10.0):
    """Positions from rho_L (r <= rmax); isotropic Gaussian velocities, sigma = v0/sqrt(2)."""
    rng = np.random.default_rng(seed)
    pos = log_positions(rng, n, v0, Rc, q, rmax)
    vel = rng.normal(0.0, v0 / np.sqrt(2.0), (3, n))
    return np.concatenate([pos, vel])


def make_rotating(ics, frac, seed):
    """Flip the azimuthal velocity to v_phi -> |v_phi| for a random fraction of the
    particles.  f(E, Lz) stays a function of the integrals, so the model stays
    stationary while acquiring net rotation."""
    rng = np.random.default_rng(seed)
    x, y, z, vx, vy, vz = ics
    R = np.sqrt(x * x + y * y)
    R = np.where(R > 0, R, 1.0)
    vR = (x * vx + y * vy) / R
    vphi = (x * vy - y * vx) / R
    sel = rng.uniform(0.0, 1.0, x.size) < frac
    vphi = np.where(sel, np.abs(vphi), vphi)
    out = ics.copy()
    out[3] = (x * vR - y * vphi) / R
    out[4] = (y * vR + x * vphi) / R
    return out


# -------------------------------------------------------------------------- NFW
def nfw_mass(r, Mh, rs):
    xx = r / rs
    return Mh * (np.log1p(xx) - xx / (1.0 + xx))


def nfw_phi(r, Mh, rs, G=1.0):
    return -G * Mh * np.log1p(r / rs) / r


def hernquist_nfw_jeans_sigma(r_eval, G=1.0, M=1.0, a=1.0, Mh=0.0, rs=1.0):
    """Isotropic Jeans dispersion of Hernquist tracers in the Hernquist + NFW potential:
    rho sigma_r^2(r) = int_r^inf rho(r') G M_tot(r') / r'^2 dr'."""
    lr = np.linspace(np.log(1e-5), np.log(1e5), 40001)
    rr = np.exp(lr)
    integrand = hernquist_density(rr, M, a) * G * (hernquist_mass(rr, M, a) + nfw_mass(rr, Mh, rs)) / rr ** 2 * rr
    # cumulative integral from the outside in (trapezoid on ln r)
    seg = 0.5 * (integrand[1:] + integrand[:-1]) * np.diff(lr)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    sig2 = tail / hernquist_density(rr, M, a)
    return np.sqrt(np.interp(np.log(r_eval), lr, sig2))


def hernquist_nfw_ics(n, seed, G=1.0, M=1.0, a=1.0, Mh=0.0, rs=1.0, vmax_frac=0.95):
    """Hernquist positions; isotropic Gaussian velocities with the local Jeans sigma_r,
    redrawn above vmax_frac of the local escape speed."""
    rng = np.random.default_rng(seed)
    x, y, z = hernquist_positions(rng, n, a, rmax=200.0 * a)
    r = np.sqrt(x * x + y * y + z * z)
    sig = hernquist_nfw_jeans_sigma(r, G, M, a, Mh, rs)
    phi = hernquist_phi(r, G, M, a) + (nfw_phi(r, Mh, rs, G) if Mh > 0 else 0.0)
    vlim = vmax_frac * np.sqrt(-2.0 * phi)
    vel = np.empty((3, n))
    todo = np.arange(n)
    while todo.size:
        v = rng.normal(0.0, 1.0, (3, todo.size)) * sig[todo]
        ok = np.sqrt((v * v).sum(axis=0)) < vlim[todo]
        vel[:, todo[ok]] = v[:, ok]
        todo = todo[~ok]
    return np.concatenate([np.stack([x, y, z]), vel])


def log_mass_within_sphere(rmax=10.0, v0=1.0, Rc=0.1, q=0.8, G=1.0):
    """Mass of rho_L inside the sphere r <= rmax (2D quadrature over r, cos theta)."""
    def inner(r):
        f = lambda c: log_density(r * r * (1 - c * c), r * r * c * c, v0, Rc, q, G)
        return 2 * np.pi * r * r * integrate.quad(f, -1.0, 1.0, epsabs=0, epsrel=1e-11)[0]
    return integrate.quad(inner, 0.0, rmax, epsabs=0, epsrel=1e-10, limit=200)[0]
