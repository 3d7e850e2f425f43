"""Guard bands of the FP32 prior-cell decisions (section 2.1: the moving prior
averages over cells of the integrals of motion E and L/Lc(E) or Lz/Lc(E)).

The fused kernel computes each particle's cell coordinates in FP32 and
re-decides an axis in FP64 when its coordinate lies within the guard band of
an edge.  The guards are twice per-particle bounds on the FP32 error (u = 2^-24):
  energy: |E32 - E| <= u (4 KE + 25 |phi| + 3 v0^2), carried into
      fE = (E - Emin) sE with the rounded Emin and sE;
  L/Lc or Lz/Lc: the rounding of L or Lz over Lc, plus the relative error of
      the tabulated Lc(E) (the table's interpolation bound, the energy error and
      the index rounding through the slope of ln Lc, the rounding of the
      interpolation and of exp) times the distance from the axis origin.
These tests restate that FP32 arithmetic with numpy float32, with and without
contraction into fused multiply-adds, modelling each hardware transcendental
(log, exp, reciprocal, square root, and ln(1 + x) in Goldberg's form from the
hardware log) as the correctly rounded result moved at random by up to one ulp
(two for the square root, six for ln(1 + x): their measured bounds on gfx950
are 1.6u and 6u relative).  On particles placed within
a few 1e-5 cells of both an energy edge and an edge of the second axis, in the
three analytic potentials, no decision the guard calls sure may differ from
the oracle's FP64 cell of the same FP32 particle, and a guard ten (for
Hernquist + NFW thirty) times narrower must be wrong somewhere (the sample
reaches the region the bounds are about).
"""
import numpy as np
import pytest

import oracle
from synth import configs

F32 = np.float32
U = 2.0 ** -24
LCE = 2048
FLOOR = 1e-6


class Hw:
    """FP32 operations with a random error of up to `ulps` ulp on the hardware
    transcendentals (the basic operations are IEEE round-to-nearest)."""

    def __init__(self, rng):
        self.rng = rng

    def _wiggle(self, v, ulps):
        v = np.asarray(v, dtype=F32)
        k = self.rng.integers(-ulps, ulps + 1, v.shape)
        out = v.copy()
        for step in range(1, ulps + 1):
            up, dn = k >= step, k <= -step
            out = np.where(up, np.nextafter(out, F32(np.inf)), out)
            out = np.where(dn, np.nextafter(out, F32(-np.inf)), out)
        return out.astype(F32)

    def log(self, s):     # log2 in hardware, times ln 2
        l2 = self._wiggle(np.log2(s.astype(np.float64)).astype(F32), 1)
        return (l2 * F32(np.log(2.0))).astype(F32)

    def exp(self, l):     # exp2 in hardware of l log2(e)
        y = (l * F32(np.log2(np.e))).astype(F32)
        return self._wiggle(np.exp2(y.astype(np.float64)).astype(F32), 1)

    def rcp(self, v):
        return self._wiggle((1.0 / v.astype(np.float64)).astype(F32), 1)

    def sqrt(self, v):
        return self._wiggle(np.sqrt(v.astype(np.float64)).astype(F32), 2)

    def log1p(self, v):
        return self._wiggle(np.log1p(v.astype(np.float64)).astype(F32), 6)


def fma(a, b, c):
    """One rounding after the exact a b + c (the product of two FP32 values is
    exact in FP64)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def sumsq(a, b, c, fused):
    if fused:
        return fma(c, c, fma(b, b, (a * a).astype(F32)))
    return (((a * a).astype(F32) + (b * b).astype(F32)).astype(F32) + (c * c).astype(F32)).astype(F32)


def pot32(pot, x, y, z, hw, fused):
    """The kernel's FP32 potential Phi(x)."""
    k = pot["kind"]
    if k == "log":
        v2, Rc2, iq2 = F32(pot["v0"] ** 2), F32(pot["Rc"] ** 2), F32(1.0 / pot["q"] ** 2)
        if fused:
            s = fma((z * z).astype(F32), np.full_like(z, iq2), fma(y, y, fma(x, x, np.full_like(x, Rc2))))
        else:
            s = (((Rc2 + (x * x).astype(F32)).astype(F32) + (y * y).astype(F32)).astype(F32) +
                 ((z * z).astype(F32) * iq2).astype(F32)).astype(F32)
        return (F32(0.5) * v2 * hw.log(s)).astype(F32)
    GM, a = F32(pot.get("G", 1.0) * pot.get("M", 1.0)), F32(pot.get("a", 1.0))
    r = hw.sqrt(sumsq(x, y, z, fused))
    ph = -(GM * hw.rcp((r + a).astype(F32))).astype(F32)
    if k == "hernquist_nfw":
        GMh, irs = F32(pot.get("G", 1.0) * pot["Mh"]), F32(1.0 / pot["rs"])
        l1 = hw.log1p((r * irs).astype(F32))
        t = (-GMh * l1).astype(F32)
        ir = hw.rcp(r)          # one hardware reciprocal of r
        ph = fma(t, ir, ph) if fused else (ph + (t * ir).astype(F32)).astype(F32)
    return ph


def lc_table(pot, Emin, Emax):
    """The host's uniform-E table: (ln Lc, interpolation bound) at kLcE energies."""
    W = Emax - Emin
    lo, hi = Emin - 0.25 * W, Emax + 0.25 * W
    if pot["kind"] != "log" and hi >= 0.0:
        hi = -1e-3 * abs(Emin)
    h = (hi - lo) / (LCE - 1)
    L = np.array([oracle.circular_L(pot, lo + k * h) for k in range(LCE)])
    tab = np.zeros((LCE, 2))
    tab[:, 0] = np.where(L > 0, np.log(np.maximum(L, 1e-300)), -1e30)
    tab[:, 1] = 1.0
    for k in range(LCE - 1):
        if L[k] > 0 and L[k + 1] > 0:
            l0, l1 = np.log(L[k]), np.log(L[k + 1])
            dev = 0.0
            for f in (0.25, 0.5, 0.75):
                ex = oracle.circular_L(pot, lo + (k + f) * h)
                dev = max(dev, abs(np.exp(l0 + f * (l1 - l0)) - ex) / ex)
            tab[k, 1] = min(1.0, 4.0 * dev + 1e-7)
    return tab.astype(F32), F32(lo), F32(1.0 / h)


def cell_fp32(pot, prior, Erange, tab, E0, invh, xv, hw, fused, scale=1.0):
    """The kernel's FP32 cell coordinates and guards: (iE, i2, sure_E, sure_2)."""
    n0, n1 = prior["shape"][0], prior["shape"][1]
    ax2 = 0 if prior["axes"][1] == "L/Lc" else 1
    x, y, z, vx, vy, vz = xv
    phi = pot32(pot, x, y, z, hw, fused)
    KE = (F32(0.5) * sumsq(vx, vy, vz, fused)).astype(F32)
    E = (KE + phi).astype(F32)
    v2 = F32(pot.get("v0", 0.0) ** 2)
    eE = (F32(U) * (F32(4) * KE + F32(25) * np.abs(phi) + F32(3) * v2)).astype(F32)
    xvy, yvx = (x * vy).astype(F32), (y * vx).astype(F32)
    Lz = fma(x, vy, -yvx) if fused else (xvy - yvx).astype(F32)
    dL = (F32(2 * U) * (np.abs(xvy) + np.abs(yvx))).astype(F32)
    L = np.zeros_like(x)
    if ax2 == 0:
        yvz, zvy, zvx, xvz = (y * vz).astype(F32), (z * vy).astype(F32), (z * vx).astype(F32), (x * vz).astype(F32)
        Lx = fma(y, vz, -zvy) if fused else (yvz - zvy).astype(F32)
        Ly = fma(z, vx, -xvz) if fused else (zvx - xvz).astype(F32)
        L = hw.sqrt(sumsq(Lx, Ly, Lz, fused))
        dL = (dL + F32(2 * U) * (np.abs(yvz) + np.abs(zvy) + np.abs(zvx) + np.abs(xvz)) + F32(4 * U) * L).astype(F32)
    # the table
    d = (E - E0).astype(F32)
    t = (d * invh).astype(F32)
    have = (t >= 0) & (t < LCE - 1)
    k = np.clip(np.where(have, t, 0).astype(np.int64), 0, LCE - 2)
    f = (t - k.astype(F32)).astype(F32)
    a0, a1, b0 = tab[k, 0], tab[k, 1], tab[k + 1, 0]
    dlt = (b0 - a0).astype(F32)
    l = fma(f, dlt, a0) if fused else (a0 + (f * dlt).astype(F32)).astype(F32)
    Lc = hw.exp(l)
    dl = (a1 + np.abs(dlt) * invh * (eE + F32(U) * (np.abs(E0) + F32(3) * np.abs(d))) +
          F32(U) * (F32(4) * np.abs(l) + F32(3))).astype(F32)
    have &= Lc > 0
    # coordinates
    Emin, Emax = F32(Erange[0]), F32(Erange[1])
    sE = (F32(n0) / (Emax - Emin).astype(F32)).astype(F32)
    fE = ((E - Emin).astype(F32) * sE).astype(F32)
    iLc = hw.rcp(Lc)
    s2 = F32(n1) if ax2 == 0 else F32(0.5 * n1)
    f2 = ((L * iLc).astype(F32) * F32(n1)).astype(F32) if ax2 == 0 else \
        (((Lz * iLc).astype(F32) + F32(1)).astype(F32) * s2).astype(F32)
    # guards
    e0 = F32(2 * sE * U * abs(float(Emin)) + FLOOR)
    e1 = F32(2 * sE)
    e2 = F32(2 * U * (4 + (abs(float(Emin)) + abs(float(Emax))) / (float(Emax) - float(Emin))))
    gE = F32(scale) * (e0 + e1 * eE + e2 * np.abs(fE))
    c2 = F32(0) if ax2 == 0 else s2
    g2 = F32(scale) * (F32(2) * (s2 * dL * iLc + np.abs(f2 - c2) * (dl + F32(3 * U)) + F32(2 * U) * np.abs(f2)) +
                       F32(FLOOR))

    def near(v, n, g):
        inside = (v > -g) & (v < F32(n) + g)
        fr = v - np.floor(v)
        return inside & ((fr < g) | (fr > F32(1) - g))

    sure_E = ~near(fE, n0, gE)
    sure_2 = have & ~near(f2, n1, g2)
    iE = np.clip(np.floor(fE), 0, n0 - 1).astype(np.int64)
    i2 = np.clip(np.floor(np.nan_to_num(f2, nan=0.0)), 0, n1 - 1).astype(np.int64)
    return iE, i2, sure_E, sure_2


def _near_edge_sample(pot, prior, Erange, n, rng):
    """Particles with E within 4e-5 cells of an energy edge and the second axis
    within 4e-5 cells of one of its edges, at random positions."""
    n0, n1 = prior["shape"][0], prior["shape"][1]
    ax2 = 0 if prior["axes"][1] == "L/Lc" else 1
    Emin, Emax = Erange
    fE = rng.integers(0, n0 + 1, n) + rng.uniform(-4e-5, 4e-5, n)
    E = Emin + fE * (Emax - Emin) / n0
    r = np.exp(rng.uniform(np.log(0.05), np.log(20.0), n))
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0)
    x, y, z = u * r
    phi = np.array([oracle.potential(pot, *p)[0] for p in zip(x, y, z)])
    Lc = np.array([oracle.circular_L(pot, e) if e < (0 if pot["kind"] != "log" else np.inf) else 0.0 for e in E])
    v2 = 2 * (E - phi)
    ok = (v2 > 0) & (Lc > 0)
    v = np.sqrt(np.maximum(v2, 0))
    f2 = rng.integers(0, n1 + 1, n) + rng.uniform(-4e-5, 4e-5, n)
    R = np.hypot(x, y)
    if ax2 == 1:
        Lz = (f2 / n1 * 2 - 1) * Lc
        vphi = Lz / np.maximum(R, 1e-12)
        ok &= np.abs(vphi) < v
        rest = np.sqrt(np.maximum(v * v - vphi * vphi, 0))
        ang = rng.uniform(0, 2 * np.pi, n)
        vR, vz = rest * np.cos(ang), rest * np.sin(ang)
        cph, sph = x / np.maximum(R, 1e-12), y / np.maximum(R, 1e-12)
        vx, vy = vR * cph - vphi * sph, vR * sph + vphi * cph
    else:
        Lt = f2 / n1 * Lc                      # |L| = r v_t
        vt = Lt / r
        ok &= vt < v
        vr = np.sqrt(np.maximum(v * v - vt * vt, 0)) * rng.choice([-1.0, 1.0], n)
        # a unit vector orthogonal to the position
        w = rng.normal(size=(3, n))
        w -= u * np.sum(w * u, axis=0)
        w /= np.linalg.norm(w, axis=0)
        vx, vy, vz = u * vr + w * vt
    xv = np.array([x, y, z, vx, vy, vz])[:, ok]
    return xv.astype(F32)


# (name, potential, prior, sample size, the narrower guard that must be wrong
# somewhere: the bounds are within 3-10x of the worst error seen for the log and
# Hernquist potentials, 10-30x for Hernquist + NFW)
CASES = [
    ("log", configs.LOG_POT, {"kind": "hist", "axes": ("E", "Lz/Lc"), "shape": (32, 32), "period": 1}, 60000, 0.1),
    ("log_L", configs.LOG_POT, {"kind": "hist", "axes": ("E", "L/Lc"), "shape": (32, 32), "period": 1}, 60000,
     0.1),
    ("hernquist", configs.HERN_POT, {"kind": "hist", "axes": ("E", "L/Lc"), "shape": (20, 20), "period": 1}, 60000,
     0.1),
    ("hernquist_nfw", {"kind": "hernquist_nfw", "G": 1.0, "M": 1.0, "a": 1.0, "Mh": 5.0, "rs": 4.0},
     {"kind": "hist", "axes": ("E", "Lz/Lc"), "shape": (20, 20), "period": 1}, 150000, 0.03),
]


@pytest.mark.parametrize("name,pot,prior,nsample,narrow", CASES, ids=[c[0] for c in CASES])
def test_cell_guards_are_sound(name, pot, prior, nsample, narrow):
    rng = np.random.default_rng(abs(hash(name)) % (1 << 31))
    cfg = configs.cfg2(N=20000) if pot["kind"] == "log" else configs.cfg1(N=20000)
    cfg = dict(cfg, potential=pot, prior=prior, precision="f32")
    inp = configs.make_inputs(cfg)
    Erange = oracle.energy_range(cfg, inp["ics"].astype(F32).astype(np.float64))
    tab, E0, invh = lc_table(pot, *Erange)
    xv = _near_edge_sample(pot, prior, Erange, nsample, rng)
    ref = oracle.Model(cfg, xv.astype(np.float64), np.ones(xv.shape[1]), inp["Y"], inp["sigma"],
                       Erange=Erange).cells()
    n1, n2 = prior["shape"][1], 1
    rE, r2 = ref // (n1 * n2), (ref // n2) % n1
    bad = wrong_narrow = 0
    for fused in (False, True):
        hw = Hw(np.random.default_rng(7 + fused))
        iE, i2, sE, s2 = cell_fp32(pot, prior, Erange, tab, E0, invh, xv, hw, fused)
        bad += int(np.sum(sE & (iE != rE))) + int(np.sum(s2 & (i2 != r2)))
        iE, i2, sE, s2 = cell_fp32(pot, prior, Erange, tab, E0, invh, xv, hw, fused, scale=narrow)
        wrong_narrow += int(np.sum(sE & (iE != rE))) + int(np.sum(s2 & (i2 != r2)))
    assert bad == 0, "%s: %d sure FP32 cell decisions differ from FP64" % (name, bad)
    assert wrong_narrow > 0, "%s: a guard %g times as wide is never wrong" % (name, narrow)
