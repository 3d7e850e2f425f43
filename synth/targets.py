"""Target observables Y_j with errors sigma_j for the synthetic galaxies.

The paper (section 2) fits observables of a target galaxy that come with
observational errors; the data types are photometry and line-of-sight
kinematics (section 1).  Here a target is either

* analytic: Hernquist shell masses and projected second LOS moments of an
  Osipkov-Merritt (r_a = 1) Hernquist model from the spherical Jeans equation, or
* a realisation: an independent particle model observed on the sky plane
  (surface density, first and second LOS moments),

and then perturbed once by Gaussian noise of relative size f.

A "layout" is a dict: ``incl`` (radians) and a list ``binnings``; each binning is
one of ``{"kind": "shell", "edges": ...}``, ``{"kind": "annulus", "edges": ...}`` or
``{"kind": "grid", "nx", "ny", "x0", "x1", "y0", "y1"}`` and carries ``moments``, a
tuple drawn from (0, 1, 2): mass, sum of w*v_los, sum of w*v_los^2, and 3..6: the
Gauss-Hermite moments h1..h4 of the line-of-sight velocity distribution about the
Gaussian (V_b, sigma_b) of each bin, which such a binning carries as ``gh``
(array [2, nb]: V_b, sigma_b; measured from the target, as an observer's
Gaussian fit would be).  Observable j runs over binnings in order, then over the
listed moments, then over bins.
"""
import numpy as np

from . import galaxy


def layout_size(layout):
    J = 0
    for b in layout["binnings"]:
        J += len(b["moments"]) * binning_nbins(b)
    return J


def binning_nbins(b):
    if b["kind"] in ("shell", "annulus"):
        return len(b["edges"]) - 1
    return b["nx"] * b["ny"]


def observable_kinds(layout):
    """Per observable: (moment, binning index, bin index)."""
    out = []
    for ib, b in enumerate(layout["binnings"]):
        nb = binning_nbins(b)
        for m in b["moments"]:
            for k in range(nb):
                out.append((m, ib, k))
    return out


# ------------------------------------------------------------ analytic Hernquist OM
def hernquist_projected_mass(R, M=1.0, a=1.0):
    """M_p(R) = M s^2 (X(s) - 1)/(1 - s^2), s = R/a (Hernquist 1990, eq. 37)."""
    s = np.asarray(R, dtype=float) / a
    out = np.empty_like(s)
    lo = s < 1.0
    hi = s > 1.0
    X = np.empty_like(s)
    X[lo] = np.arccosh(1.0 / s[lo]) / np.sqrt(1.0 - s[lo] ** 2)
    X[hi] = np.arccos(1.0 / s[hi]) / np.sqrt(s[hi] ** 2 - 1.0)
    one = ~(lo | hi)
    X[one] = 1.0
    out[lo | hi] = M * s[lo | hi] ** 2 * (X[lo | hi] - 1.0) / (1.0 - s[lo | hi] ** 2)
    out[one] = M / 3.0
    return out


def om_rho_sigr2_table(ra, G=1.0, M=1.0, a=1.0):
    """rho sigma_r^2 of a Hernquist model with Osipkov-Merritt anisotropy
    beta = r^2/(r^2 + ra^2) from the spherical Jeans equation:
    rho sigma_r^2 (r) = (1 + r^2/ra^2)^-1 int_r^inf (1 + r'^2/ra^2) rho G M(r')/r'^2 dr'.
    ra = inf gives the isotropic model.  Returns (ln r grid, rho sigma_r^2)."""
    lr = np.linspace(np.log(1e-7), np.log(1e7), 56001)
    r = np.exp(lr)
    fac = 1.0 + (r / ra) ** 2 if np.isfinite(ra) else np.ones_like(r)
    integrand = fac * galaxy.hernquist_density(r, M, a) * G * galaxy.hernquist_mass(r, M, a) / r ** 2 * r
    seg = 0.5 * (integrand[1:] + integrand[:-1]) * np.diff(lr)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    return lr, tail / fac


def om_projected_sigma2_sigma(R, ra, G=1.0, M=1.0, a=1.0, nu=6000):
    """Sigma(R) sigma_p^2(R) = 2 int_R^inf (1 - beta R^2/r^2) rho sigma_r^2 r dr / sqrt(r^2 - R^2),
    with r = R cosh(u) to remove the end-point singularity."""
    lr, P = om_rho_sigr2_table(ra, G, M, a)
    lP = np.log(np.maximum(P, 1e-300))
    R = np.atleast_1d(np.asarray(R, dtype=float))
    out = np.empty_like(R)
    for i, Ri in enumerate(R):
        umax = np.arccosh(1e7 / Ri)
        u = np.linspace(0.0, umax, nu)
        r = Ri * np.cosh(u)
        beta = r * r / (r * r + ra * ra) if np.isfinite(ra) else np.zeros_like(r)
        Pr = np.exp(np.interp(np.log(r), lr, lP))
        f = (1.0 - beta * Ri * Ri / (r * r)) * Pr * Ri * np.cosh(u)
        out[i] = 2.0 * np.trapezoid(f, u)
    return out


def hernquist_om_annulus_moment2(edges, ra, G=1.0, M=1.0, a=1.0, per_bin=161):
    """Y2_b = int_{R_b}^{R_b+1} 2 pi R Sigma sigma_p^2 dR (Simpson in ln R)."""
    out = np.empty(len(edges) - 1)
    for b in range(len(edges) - 1):
        lR = np.linspace(np.log(edges[b]), np.log(edges[b + 1]), per_bin)
        R = np.exp(lR)
        g = om_projected_sigma2_sigma(R, ra, G, M, a)
        f = 2 * np.pi * R * R * g
        h = lR[1] - lR[0]
        out[b] = h / 3.0 * (f[0] + f[-1] + 4 * f[1:-1:2].sum() + 2 * f[2:-1:2].sum())
    return out


class OMLineOfSight:
    """Exact line-of-sight kinematics of the Osipkov-Merritt Hernquist model
    (G = M = a = 1), line of sight along z.

    At a point at radius r the DF is f_Q(Psi - v_r^2/2 - s^2 v_t^2/2) with
    s^2 = 1 + r^2/r_a^2; in u = (v_r, s v_t) it is isotropic, so the velocity
    along a unit vector n has the density (1/(s^2 k)) G(Psi - v^2/(2 k^2)), where
    k^2 = n_r^2 + n_t^2/s^2 and G(q) = 2 pi int_0^q f_Q (the one-dimensional
    marginal of an isotropic distribution).  By Eddington's formula
    int_0^q f_Q = (1/(sqrt(8) pi^2)) int_0^q rho_Q'(Psi) dPsi / sqrt(q - Psi), so
    G(q) = (sqrt(2)/pi) sqrt(q) int_0^1 rho_Q'(q (1 - s^2)) ds needs no f_Q.  An
    annulus's sum of K(v_los) is the integral over R (Gauss-Legendre in ln R),
    z = R tan(theta) and t = sqrt(2 Psi) sin(phi) of (1/s^2) K(k t) G(Psi - t^2/2)."""

    def __init__(self, ra, nR=24, ntheta=96, nphi=64, qmax=0.95, ntab=40001):
        self.ra = ra
        xs, ws = np.polynomial.legendre.leggauss(64)
        s = 0.5 * (xs + 1.0)
        self._q = np.linspace(0.0, qmax, ntab)
        psi = self._q[:, None] * (1.0 - s[None, :] ** 2)
        self._G = np.sqrt(2.0) / np.pi * np.sqrt(self._q) * (0.5 * ws[None, :] * self.rhoq_p(psi)).sum(axis=1)
        self._gl = [np.polynomial.legendre.leggauss(n) for n in (nR, ntheta, nphi)]

    def rhoq_p(self, psi):
        """d rho_Q / d Psi, rho_Q = [Psi^4/(1 - Psi) + (Psi^2 - Psi^3)/r_a^2] / (2 pi)."""
        u = 1.0 - psi
        return ((4.0 * psi ** 3 * u + psi ** 4) / (u * u) + (2.0 * psi - 3.0 * psi ** 2) / self.ra ** 2) / (2.0 * np.pi)

    def G(self, q):
        return np.interp(q, self._q, self._G)

    def annulus_sums(self, R1, R2, kernels):
        """[len(kernels)] sums of K(v_los) over the annulus R1 <= R < R2, each kernel
        a function of v_los (vectorised)."""
        (xr, wr), (xt, wt), (xp, wp) = self._gl
        lR = 0.5 * (np.log(R2) - np.log(R1)) * xr + 0.5 * (np.log(R2) + np.log(R1))
        R = np.exp(lR)[:, None, None]
        wR = (0.5 * (np.log(R2) - np.log(R1)) * wr * 2.0 * np.pi * np.exp(2 * lR))[:, None, None]
        th = (0.25 * np.pi * (xt + 1.0))[None, :, None]
        wth = (0.25 * np.pi * wt)[None, :, None]
        ph = (0.5 * np.pi * xp)[None, None, :]
        wph = (0.5 * np.pi * wp)[None, None, :]
        z = R * np.tan(th)
        dz = R / np.cos(th) ** 2
        r = np.sqrt(R * R + z * z)
        psi = 1.0 / (1.0 + r)
        s2 = 1.0 + r * r / (self.ra * self.ra)
        nr2 = (z / r) ** 2
        k = np.sqrt(nr2 + (1.0 - nr2) / s2)
        t = np.sqrt(2.0 * psi) * np.sin(ph)
        base = 2.0 * wR * wth * dz * wph * np.sqrt(2.0 * psi) * np.cos(ph) * self.G(psi * np.cos(ph) ** 2) / s2
        return np.array([np.sum(base * K(k * t)) for K in kernels])


def hernquist_om_exact_target(layout, ra=1.0):
    """Idealised data of the Osipkov-Merritt Hernquist target (G = M = a = 1, line
    of sight z): exact shell and annulus masses (closed forms) and, per annulus,
    the exact sums of v_los, v_los^2 and the Gauss-Hermite kernels about
    V_b = 0 and sigma_b = the annulus's exact dispersion.  Returns (Y, M_b, gh)
    with gh per binning ([2, nb] or None); fills b["gh"] of the layout."""
    los = OMLineOfSight(ra)
    Y, Mb_list, gh = [], [], []
    for b in layout["binnings"]:
        e = np.asarray(b["edges"], dtype=float)
        nb = len(e) - 1
        if b["kind"] == "shell":
            mass = np.diff(galaxy.hernquist_mass(e, 1.0, 1.0))
            if any(m != 0 for m in b["moments"]):
                raise ValueError("shells carry masses only")
            Y += [mass] * len(b["moments"])
            Mb_list += [mass] * len(b["moments"])
            gh.append(None)
            continue
        if b["kind"] != "annulus":
            raise ValueError("exact target supports shells and annuli only")
        mass = np.diff(hernquist_projected_mass(e, 1.0, 1.0))
        v2 = np.array([los.annulus_sums(e[i], e[i + 1], [lambda v: v * v])[0] for i in range(nb)])
        sig = np.sqrt(v2 / mass)
        g = np.stack([np.zeros(nb), sig]) if any(m >= 3 for m in b["moments"]) else None
        if g is not None:
            b["gh"] = g
        gh.append(g)
        for m in b["moments"]:
            if m == 0:
                Y.append(mass)
            elif m == 1:
                Y.append(np.zeros(nb))
            elif m == 2:
                Y.append(v2)
            else:
                Y.append(np.array([los.annulus_sums(e[i], e[i + 1],
                                                    [lambda v, i=i: gauss_hermite_kernel(m - 2, v / sig[i])])[0]
                                   for i in range(nb)]))
            Mb_list.append(mass)
    return np.concatenate(Y), np.concatenate(Mb_list), gh


def hernquist_om_target(layout, ra=1.0, G=1.0, M=1.0, a=1.0):
    """True (noise-free) observables of the OM Hernquist target for a layout made of
    shells (moment 0) and annuli (moment 0 or 2; the mean LOS velocity is zero)."""
    Y = []
    Mb_list = []
    for b in layout["binnings"]:
        e = np.asarray(b["edges"], dtype=float)
        if b["kind"] == "shell":
            mass = np.diff(galaxy.hernquist_mass(e, M, a))
            proj = None
        elif b["kind"] == "annulus":
            mass = np.diff(hernquist_projected_mass(e, M, a))
            proj = hernquist_om_annulus_moment2(e, ra, G, M, a)
        else:
            raise ValueError("analytic target supports shells and annuli only")
        for m in b["moments"]:
            if m == 0:
                Y.append(mass)
            elif m == 1:
                Y.append(np.zeros_like(mass))
            else:
                if proj is None:
                    raise ValueError("second moment needs a projected binning")
                Y.append(proj)
            Mb_list.append(mass)
    return np.concatenate(Y), np.concatenate(Mb_list)


# ----------------------------------------------------------------- realisations
def _bin_index(b, ics, inc):
    """Bin of every particle of a realisation in binning b (-1 outside) and nb."""
    x, y, z = ics[0], ics[1], ics[2]
    X = x
    Ysky = y * np.cos(inc) - z * np.sin(inc)
    if b["kind"] == "grid":
        ix = np.floor((X - b["x0"]) / (b["x1"] - b["x0"]) * b["nx"]).astype(np.int64)
        iy = np.floor((Ysky - b["y0"]) / (b["y1"] - b["y0"]) * b["ny"]).astype(np.int64)
        ok = (ix >= 0) & (ix < b["nx"]) & (iy >= 0) & (iy < b["ny"])
        return np.where(ok, iy * b["nx"] + ix, -1), b["nx"] * b["ny"]
    rad = np.sqrt(x * x + y * y + z * z) if b["kind"] == "shell" else np.sqrt(X * X + Ysky * Ysky)
    e = np.asarray(b["edges"])
    k = np.searchsorted(e, rad, side="right") - 1
    return np.where((k >= 0) & (k < len(e) - 1), k, -1), len(e) - 1


def gh_parameters(b, ics, inc, zero_mean=False):
    """The Gaussian each bin's line-of-sight velocities are expanded about: the
    mass-weighted mean V_b (0 when zero_mean) and dispersion sigma_b of the
    realisation's v_los in the bin; [2, nb]."""
    vlos = ics[4] * np.sin(inc) + ics[5] * np.cos(inc)
    k, nb = _bin_index(b, ics, inc)
    ok = k >= 0
    n = np.maximum(np.bincount(k[ok], minlength=nb), 1)
    m1 = np.bincount(k[ok], weights=vlos[ok], minlength=nb) / n
    m2 = np.bincount(k[ok], weights=vlos[ok] ** 2, minlength=nb) / n
    V = np.zeros(nb) if zero_mean else m1
    sig = np.sqrt(np.maximum(m2 - V * V, 1e-12))
    return np.stack([V, sig])


def gauss_hermite_kernel(m, nu):
    """2 sqrt(pi) alpha(nu) H_m(nu) of the van der Marel & Franx expansion, m = 1..4
    (alpha = exp(-nu^2/2)/sqrt(2 pi); H_1 = sqrt(2) nu, H_2 = (2 nu^2 - 1)/sqrt(2),
    H_3 = (2 nu^3 - 3 nu)/sqrt(3), H_4 = (4 nu^4 - 12 nu^2 + 3)/sqrt(24))."""
    h = {1: np.sqrt(2.0) * nu, 2: (2 * nu ** 2 - 1) / np.sqrt(2.0), 3: (2 * nu ** 3 - 3 * nu) / np.sqrt(3.0),
         4: (4 * nu ** 4 - 12 * nu ** 2 + 3) / np.sqrt(24.0)}[m]
    return np.sqrt(2.0) * np.exp(-0.5 * nu * nu) * h


def observe_realisation(layout, ics, mass):
    """Observe a particle realisation of the target galaxy (equal masses) on the
    layout's bins.  Returns (Y_true, M_b) where M_b is the binned mass that goes with
    each observable (used to size kinematic errors)."""
    x, y, z, vx, vy, vz = ics
    inc = layout["incl"]
    X = x
    Ysky = y * np.cos(inc) - z * np.sin(inc)
    vlos = vy * np.sin(inc) + vz * np.cos(inc)
    out, mb = [], []
    for b in layout["binnings"]:
        if b["kind"] == "grid":
            ix = np.floor((X - b["x0"]) / (b["x1"] - b["x0"]) * b["nx"]).astype(np.int64)
            iy = np.floor((Ysky - b["y0"]) / (b["y1"] - b["y0"]) * b["ny"]).astype(np.int64)
            ok = (ix >= 0) & (ix < b["nx"]) & (iy >= 0) & (iy < b["ny"])
            idx = (iy * b["nx"] + ix)[ok]
            nb = b["nx"] * b["ny"]
        else:
            rad = np.sqrt(x * x + y * y + z * z) if b["kind"] == "shell" else np.sqrt(X * X + Ysky * Ysky)
            e = np.asarray(b["edges"])
            k = np.searchsorted(e, rad, side="right") - 1
            ok = (k >= 0) & (k < len(e) - 1)
            idx = k[ok]
            nb = len(e) - 1
        vv = vlos[ok]
        mass_b = np.bincount(idx, minlength=nb) * mass
        for m in b["moments"]:
            if m <= 2:
                w = mass * vv ** m
            else:
                gh = np.asarray(b["gh"])
                w = mass * gauss_hermite_kernel(m - 2, (vv - gh[0][idx]) / gh[1][idx])
            out.append(np.bincount(idx, weights=w, minlength=nb))
            mb.append(mass_b)
    return np.concatenate(out), np.concatenate(mb)


# ------------------------------------------------------------------------ noise
def add_noise(layout, Y_true, M_b, f, seed, f_gh=None):
    """One fixed Gaussian noise draw.  Mass-type observables: sigma = f |Y|;
    first moments: sigma = f sqrt(M_b Y2) (f on the rms LOS velocity);
    second moments: sigma = 2 f Y2 (f on the dispersion); Gauss-Hermite moments:
    sigma = f_gh M_b (an error f_gh on h_m; f_gh = f when not given).  Zero errors
    (empty bins) are raised to the smallest positive error of the same group."""
    f_gh = f if f_gh is None else f_gh
    rng = np.random.default_rng(seed)
    kinds = observable_kinds(layout)
    moment = np.array([k[0] for k in kinds])
    sigma = np.empty_like(Y_true)
    # second moment of each first-moment bin: look it up in the same binning
    start = 0
    for b in layout["binnings"]:
        nb = binning_nbins(b)
        y2 = None
        for mi, m in enumerate(b["moments"]):
            if m == 2:
                y2 = Y_true[start + mi * nb: start + (mi + 1) * nb]
        for mi, m in enumerate(b["moments"]):
            sl = slice(start + mi * nb, start + (mi + 1) * nb)
            if m == 0:
                sigma[sl] = f * np.abs(Y_true[sl])
            elif m == 1:
                if y2 is None:
                    raise ValueError("first moment needs the second moment in the same binning")
                sigma[sl] = f * np.sqrt(np.maximum(M_b[sl] * y2, 0.0))
            elif m == 2:
                sigma[sl] = 2.0 * f * np.abs(Y_true[sl])
            else:
                sigma[sl] = f_gh * M_b[sl]
            s = sigma[sl]
            pos = s[s > 0]
            floor = pos.min() if pos.size else 1.0
            sigma[sl] = np.where(s > 0, s, floor)
        start += len(b["moments"]) * nb
    g = rng.normal(0.0, 1.0, Y_true.size)
    del moment
    return Y_true + sigma * g, sigma


def discrete_tracers(layout, ib, ics, n, dv, seed):
    """Discrete tracers (planetary-nebula-like) drawn from a target realisation:
    n of its particles at random, each with its bin in binning ib (those outside
    the binning are skipped) and its line-of-sight velocity plus a Gaussian error
    of dispersion dv.  Returns (bin, v) of the kept tracers."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(ics.shape[1], size=n, replace=False)
    sub = ics[:, idx]
    k, _ = _bin_index(layout["binnings"][ib], sub, layout["incl"])
    inc = layout["incl"]
    vlos = sub[4] * np.sin(inc) + sub[5] * np.cos(inc)
    ok = k >= 0
    return k[ok].astype(np.int32), vlos[ok] + dv * rng.standard_normal(int(ok.sum()))
