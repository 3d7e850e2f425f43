"""Pins of the oracle's self-consistent step order, its interpolation between
multipole nodes and its prior-cell axes in the logarithmic potential.

Self-consistent potential (paper sections 1-2: the potential is computed from the
particles while they move).  The oracle's reading is a kick-drift-kick step whose
second kick uses coefficients rebuilt from the drifted positions and the updated
weights.  Pinned here by:
  - massless probe particles, whose kicks must equal the force of a direct O(N^2)
    sum of the truncated addition-theorem series over the massive particles at
    the right positions and weights (exact where no massive particle shares a
    probe's node interval);
  - time reversibility of the frozen-weight self-consistent system;
  - the step reproduced from the separately pinned coefficient and field routines
    called in that order;
each shown to reject the plausible mistakes (a stale second kick, the weights of
the old step).

Node interpolation (reading R-12: coefficients linear in ln r between nodes):
the field between nodes equals the truncated series summed in the test from the
interpolated tables, and the exact expansion within the bound set by the mass in
the node interval.

Prior cells (section 2.1: priors over integrals of motion E, L, Lz): the cells
of the (E, Lz/Lc) and (E, L/Lc, Lz/L) grids in the logarithmic potential against
cells computed here with a circular-orbit Lc(E) solved in the test, and O(N^2)
cell means.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy import optimize, special

import oracle
from synth import configs

G_GRAV = 1.0


# ---------------------------------------------------------------- direct sums
def _legendre_and_derivative(lmax, mu):
    """P_l(mu) and P_l'(mu), l = 0..lmax, from the Legendre series (numpy)."""
    P = np.empty((lmax + 1,) + np.shape(mu))
    dP = np.empty_like(P)
    for l in range(lmax + 1):
        c = np.zeros(l + 1)
        c[l] = 1.0
        P[l] = npleg.legval(mu, c)
        dP[l] = npleg.legval(mu, npleg.legder(c)) if l > 0 else 0.0
    return P, dP


def direct_field(src, m, pt, lmax, G=G_GRAV):
    """Phi and a = -grad Phi at point pt of the truncated series
    Phi = -G sum_k m_k sum_{l<=lmax} r<^l / r>^(l+1) P_l(cos gamma_k), by direct
    summation over the sources src [3, K] with masses m [K]."""
    r = np.linalg.norm(pt)
    rk = np.linalg.norm(src, axis=0)
    xh = pt / r
    xk = src / rk
    mu = np.clip(xh @ xk, -1.0, 1.0)
    P, dP = _legendre_and_derivative(lmax, mu)
    inside = rk < r
    phi = 0.0
    grad = np.zeros(3)
    tang = xk - mu * xh[:, None]            # (d mu / d x) * r
    for l in range(lmax + 1):
        f_in = rk ** l / r ** (l + 1)        # r_k < r
        f_out = r ** l / rk ** (l + 1)       # r_k >= r
        f = np.where(inside, f_in, f_out)
        phi += np.sum(m * f * P[l])
        dr = np.where(inside, -(l + 1) * f_in / r, (l * r ** (l - 1) / rk ** (l + 1)) if l > 0 else 0.0)
        grad += (m * dr * P[l]) @ np.tile(xh, (rk.size, 1)) + (tang * (m * f * dP[l] / r)).sum(axis=1)
    return -G * phi, G * grad


def node_interval(pot, r):
    """Node interval [r_k, r_k+1) of radius r (node radii as defined: exp(ln rmin + k dl))."""
    lr0 = np.log(pot["rmin"])
    dl = (np.log(pot["rmax"]) - lr0) / (pot["nodes"] - 1)
    k = int(np.floor((np.log(r) - lr0) / dl))
    while k > 0 and r < np.exp(lr0 + k * dl):
        k -= 1
    while k < pot["nodes"] - 2 and r >= np.exp(lr0 + (k + 1) * dl):
        k += 1
    return k, np.exp(lr0 + k * dl), np.exp(lr0 + (k + 1) * dl)


# ----------------------------------------------------- self-consistent model
def probe_system(n_mass=100, n_probe=300, seed=21):
    """Massive particles of a rotating, flattened cloud, plus probes of negligible mass."""
    rng = np.random.default_rng(seed)
    pos = rng.normal(0.0, 1.0, (3, n_mass)) * np.array([[1.0], [0.8], [0.5]])
    vel = rng.normal(0.0, 0.4, (3, n_mass)) + np.array([[0.0], [0.0], [0.0]])
    vel[0] += -0.5 * pos[1]
    vel[1] += 0.5 * pos[0]
    ppos = rng.normal(0.0, 1.2, (3, n_probe))
    pvel = rng.normal(0.0, 0.5, (3, n_probe))
    ics = np.concatenate([np.concatenate([pos, vel]), np.concatenate([ppos, pvel])], axis=1)
    w = np.concatenate([np.full(n_mass, 1.0 / n_mass), np.full(n_probe, 1e-20)])
    return ics, w


def mp_cfg(nodes, eps, lmax=8, dt=0.005):
    c = configs.cfg1(N=10)
    c.update(precision="f64", dt=dt, eps=eps, mu=0.0, tau=0.5, update="exp",
             potential={"kind": "multipole", "G": G_GRAV, "lmax": lmax, "nodes": nodes, "rmin": 1e-3,
                        "rmax": 100.0, "Mtot": 1.0},
             prior={"kind": "flat"})
    return c


def mp_model(cfg, ics, w):
    J = 50
    rng = np.random.default_rng(3)
    Y = rng.uniform(0.0, 0.05, J)
    return oracle.Model(cfg, ics, w, Y, np.full(J, 0.01))


def test_step_kicks_probes_with_direct_forces_at_drifted_positions():
    """One self-consistent step: every probe's position and velocity equal a
    kick-drift-kick written here with direct O(N^2) truncated-series forces of the
    massive particles -- the first kick from their positions and weights of step
    n, the second from their drifted positions and updated weights w(n+1) --
    wherever no massive particle lies in the probe's node interval (there the
    interpolated coefficients are exact).  A second kick with the old positions,
    or with the old weights, misses the bar by orders of magnitude."""
    nm = 100
    cfg = mp_cfg(nodes=2000, eps=0.02)
    ics, w = probe_system(nm)
    m = mp_model(cfg, ics, w)
    m.run(1)
    assert m.status == 0
    new = m.ics()
    w1 = m.w.copy()
    dt = cfg["dt"]
    pot = cfg["potential"]
    src0, m0 = ics[:3, :nm], w[:nm] * pot["Mtot"]
    src1, m1 = new[:3, :nm], w1[:nm] * pot["Mtot"]
    # the update really moved the massive weights (so w(n) and w(n+1) differ visibly)
    assert np.max(np.abs(w1[:nm] / w[:nm] - 1.0)) > 1e-3
    r0m, r1m = np.linalg.norm(src0, axis=0), np.linalg.norm(src1, axis=0)
    checked, err_x, err_v, err_stale, err_oldw = 0, 0.0, 0.0, 0.0, 0.0
    for i in range(nm, ics.shape[1]):
        x0, v0 = ics[:3, i], ics[3:, i]
        _, lo0, hi0 = node_interval(pot, np.linalg.norm(x0))
        _, a0 = direct_field(src0, m0, x0, pot["lmax"])
        vh = v0 + 0.5 * dt * a0
        x1 = x0 + dt * vh
        _, lo1, hi1 = node_interval(pot, np.linalg.norm(x1))
        if np.any((r0m >= lo0) & (r0m < hi0)) or np.any((r1m >= lo1) & (r1m < hi1)):
            continue
        _, a1 = direct_field(src1, m1, x1, pot["lmax"])
        v1 = vh + 0.5 * dt * a1
        scale = np.abs(0.5 * dt * a1).max()
        err_x = max(err_x, np.abs(new[:3, i] - x1).max() / (dt * dt * np.abs(a0).max()))
        err_v = max(err_v, np.abs(new[3:, i] - v1).max() / scale)
        # the plausible mistakes: the tables of step n, or drifted positions with the old weights
        _, a_st = direct_field(src0, m0, x1, pot["lmax"])
        _, a_ow = direct_field(src1, w[:nm] * pot["Mtot"], x1, pot["lmax"])
        err_stale = max(err_stale, np.abs(new[3:, i] - (vh + 0.5 * dt * a_st)).max() / scale)
        err_oldw = max(err_oldw, np.abs(new[3:, i] - (vh + 0.5 * dt * a_ow)).max() / scale)
        checked += 1
    assert checked >= 150, checked
    assert err_x < 1e-9, err_x
    assert err_v < 1e-9, err_v
    assert err_stale > 1e-6 and err_oldw > 1e-6, (err_stale, err_oldw)


def _kdk_composed(cfg, ics, w0, w1, stale=False):
    """One step of the particles from the separately pinned coefficient and field
    routines: kick with the tables of (x_n, w_n), drift, tables of (x_n+1, w1),
    kick (or, stale, the first tables again)."""
    pot, dt = cfg["potential"], cfg["dt"]
    x, v = ics[:3].copy(), ics[3:].copy()
    A, B = oracle.mp_coeffs(pot, x, w0)
    _, ax, ay, az = oracle.mp_eval(pot, A, B, x)
    v = v + 0.5 * dt * np.stack([ax, ay, az])
    x = x + dt * v
    if not stale:
        A, B = oracle.mp_coeffs(pot, x, w1)
    _, ax, ay, az = oracle.mp_eval(pot, A, B, x)
    v = v + 0.5 * dt * np.stack([ax, ay, az])
    return np.concatenate([x, v])


def test_step_equals_kick_drift_rebuild_kick_of_pinned_parts():
    """The oracle's step reproduces, bitwise, the order kick (tables of x_n, w_n) ->
    drift -> rebuild (x_n+1, w_n+1) -> kick built here from the coefficient and
    field routines (each pinned against the addition theorem elsewhere); the stale
    second kick does not."""
    cfg = mp_cfg(nodes=200, eps=40.0)
    rng = np.random.default_rng(4)
    ics = np.concatenate([rng.normal(0, 1.0, (3, 150)), rng.normal(0, 0.5, (3, 150))])
    w = rng.uniform(0.5, 1.5, 150)
    w /= w.sum()
    m = mp_model(cfg, ics, w)
    m.run(1)
    ref = _kdk_composed(cfg, ics, w, m.w)
    np.testing.assert_array_equal(m.ics(), ref)
    stale = _kdk_composed(cfg, ics, w, m.w, stale=True)
    assert np.abs(stale[3:] - ref[3:]).max() > 1e-6 * np.abs(ref[3:]).max()


def _reverse_error(cfg, ics, w, nsteps, composed_stale=False):
    if composed_stale:
        x = ics.copy()
        for _ in range(nsteps):
            x = _kdk_composed(cfg, x, w, w, stale=True)
        x[3:] *= -1.0
        for _ in range(nsteps):
            x = _kdk_composed(cfg, x, w, w, stale=True)
        back = x
    else:
        m = mp_model(cfg, ics, w)
        m.run(nsteps)
        assert m.status == 0
        fwd = m.ics()
        fwd[3:] *= -1.0
        m2 = mp_model(cfg, fwd, m.w)
        m2.run(nsteps)
        back = m2.ics()
    back[3:] *= -1.0
    return np.abs(back - ics).max() / np.abs(ics).max()


def test_frozen_weight_self_consistent_system_is_time_reversible():
    """eps = 0: 100 self-consistent steps, velocities flipped, 100 steps back return
    to the start within 1e-10 (kick-drift-kick with the second kick's coefficients
    rebuilt from the drifted positions is time-symmetric); a stale second kick is
    not (its return error is > 1e-6)."""
    cfg = mp_cfg(nodes=200, eps=0.0)
    rng = np.random.default_rng(6)
    n = 200
    pos = rng.normal(0, 1.0, (3, n))
    vel = rng.normal(0, 0.3, (3, n))
    ics = np.concatenate([pos, vel])
    w = np.full(n, 1.0 / n)
    err = _reverse_error(cfg, ics, w, 100)
    assert err < 1e-10, err
    err_stale = _reverse_error(cfg, ics, w, 100, composed_stale=True)
    assert err_stale > 1e-6, err_stale


# ------------------------------------------------------- node interpolation
def _interp_tables(pot, A, B, r):
    k, lo, hi = node_interval(pot, r)
    t = (np.log(r) - np.log(lo)) / (np.log(hi) - np.log(lo))
    return A[k] + t * (A[k + 1] - A[k]), B[k] + t * (B[k + 1] - B[k]), k, t


def series_from_tables(Ar, Br, pt, lmax, G=G_GRAV):
    """Phi = -G sum_lm c_lm P_l^m(cos th)[cos(m ph)(Ac r^-(l+1) + Bc r^l) +
    sin(m ph)(As r^-(l+1) + Bs r^l)], c_lm = (2 - d_m0)(l-m)!/(l+m)! (the addition
    theorem with the Condon-Shortley associated Legendre functions), table index
    l^2 (m = 0), l^2 + 2m - 1 (cos), l^2 + 2m (sin)."""
    x, y, z = pt
    r = np.sqrt(x * x + y * y + z * z)
    ct, ph = z / r, np.arctan2(y, x)
    s = 0.0
    for l in range(lmax + 1):
        for mm in range(l + 1):
            c = (1.0 if mm == 0 else 2.0) * special.factorial(l - mm) / special.factorial(l + mm)
            plm = special.lpmv(mm, l, ct)
            jc = l * l if mm == 0 else l * l + 2 * mm - 1
            term = np.cos(mm * ph) * (Ar[jc] * r ** -(l + 1) + Br[jc] * r ** l)
            if mm > 0:
                term += np.sin(mm * ph) * (Ar[jc + 1] * r ** -(l + 1) + Br[jc + 1] * r ** l)
            s += c * plm * term
    return -G * s


def test_field_between_nodes_is_linear_in_ln_r_of_the_tables():
    """At points between nodes with particles inside their node interval (where
    the interpolation matters): Phi equals the series of the tables interpolated
    here, A_k + t (A_k+1 - A_k) with t the position in ln r, within 1e-12; the
    force equals minus its gradient with the tables held fixed; Phi differs from
    the exact expansion by no more than the node interval's particles can move
    it.  Interpolating from the wrong node, or with 1 - t, fails the first bar."""
    MP = {"kind": "multipole", "G": G_GRAV, "lmax": 8, "nodes": 40, "rmin": 1e-2, "rmax": 10.0, "Mtot": 1.0}
    rng = np.random.default_rng(17)
    pos = rng.normal(0, 1.0, (3, 400))
    w = rng.uniform(0.5, 1.5, 400)
    w /= w.sum()
    A, B = oracle.mp_coeffs(MP, pos, w)
    rk = np.linalg.norm(pos, axis=0)
    done = 0
    for trial in range(200):
        d = rng.normal(0, 1, 3)
        r = np.exp(rng.uniform(np.log(0.3), np.log(3.0)))
        pt = d / np.linalg.norm(d) * r
        Ar, Br, k, t = _interp_tables(MP, A, B, r)
        _, lo, hi = node_interval(MP, r)
        inbr = (rk >= lo) & (rk < hi)
        if not inbr.any() or not (0.15 < t < 0.4 or 0.6 < t < 0.85):
            continue
        phi, ax, ay, az = (v[0] for v in oracle.mp_eval(MP, A, B, pt[:, None]))
        want = series_from_tables(Ar, Br, pt, 8)
        assert phi == pytest.approx(want, rel=1e-12), (phi, want)
        # the mistakes are far off: 1 - t, or the next node interval
        bad_t = series_from_tables(A[k] + (1 - t) * (A[k + 1] - A[k]), B[k] + (1 - t) * (B[k + 1] - B[k]), pt, 8)
        bad_k = series_from_tables(A[k + 1] + t * (A[k + 2] - A[k + 1]), B[k + 1] + t * (B[k + 2] - B[k + 1]), pt, 8)
        assert abs(bad_t - want) > 1e-9 * abs(want)
        assert abs(bad_k - want) > 1e-9 * abs(want)
        # force = -grad Phi with the interpolated tables held fixed
        h = 1e-5
        g = np.zeros(3)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            g[c] = (series_from_tables(Ar, Br, pt + e, 8) - series_from_tables(Ar, Br, pt - e, 8)) / (2 * h)
        np.testing.assert_allclose([ax, ay, az], -g, rtol=1e-6, atol=1e-8 * np.abs(g).max())
        # against the exact expansion: only the interval's particles j differ, by
        # m_j (t - [r_j < r]) sum_l (r_j^l / r^(l+1) - r^l / r_j^(l+1)) P_l(cos g_j),
        # each degree at most m_j e^(l dl) (1/r + 1/r_j) with dl the node spacing
        ex = oracle.mp_exact(MP, pos, w, pt)[0]
        dl = np.log(hi / lo)
        bound = G_GRAV * np.sum(w[inbr] * (1.0 / r + 1.0 / rk[inbr])) * np.sum(np.exp(dl * np.arange(9)))
        assert abs(phi - ex) <= bound, (phi, ex, bound)
        done += 1
        if done >= 12:
            break
    assert done >= 12


# ------------------------------------------------------- log-potential cells
def log_lc(E, v0=1.0, Rc=0.1):
    """Lc(E) of the circular orbit in the equatorial plane of the logarithmic
    potential Phi = v0^2/2 ln(Rc^2 + R^2 + z^2/q^2): E_c(R) = v0^2/2 ln(Rc^2 + R^2)
    + v_c^2/2 with v_c^2 = v0^2 R^2/(Rc^2 + R^2), solved for R by bracketing."""
    def Ec(R):
        return 0.5 * v0 ** 2 * np.log(Rc ** 2 + R ** 2) + 0.5 * v0 ** 2 * R ** 2 / (Rc ** 2 + R ** 2)
    out = np.empty(np.size(E))
    for i, e in enumerate(np.atleast_1d(E)):
        R = optimize.brentq(lambda R: Ec(R) - e, 1e-12, 1e8, xtol=1e-300, rtol=1e-15, maxiter=500)
        out[i] = R * v0 * R / np.sqrt(Rc ** 2 + R ** 2)
    return out


def log_integrals(ics, q=0.8, v0=1.0, Rc=0.1):
    x, y, z, vx, vy, vz = ics
    E = 0.5 * (vx * vx + vy * vy + vz * vz) + 0.5 * v0 ** 2 * np.log(Rc ** 2 + x * x + y * y + z * z / q ** 2)
    Lx, Ly, Lz = y * vz - z * vy, z * vx - x * vz, x * vy - y * vx
    L = np.sqrt(Lx * Lx + Ly * Ly + Lz * Lz)
    return E, L, Lz


def cells_here(ics, Erange, shape, second):
    """Cell of each particle: E uniform over Erange (clamped), then L/Lc in [0, 1]
    or Lz/Lc in [-1, 1], then (3 axes) Lz/L in [-1, 1]; returns the cell and the
    smallest distance (in cells) of any coordinate to an interior edge."""
    E, L, Lz = log_integrals(ics)
    Lc = log_lc(E)
    f0 = (E - Erange[0]) / (Erange[1] - Erange[0]) * shape[0]
    f1 = (L / Lc) * shape[1] if second == "L/Lc" else (Lz / Lc + 1.0) * 0.5 * shape[1]
    fs = [f0, f1]
    if len(shape) > 2:
        fs.append((np.where(L > 0, Lz / np.where(L > 0, L, 1.0), 0.0) + 1.0) * 0.5 * shape[2])
    idx = [np.clip(np.floor(f), 0, n - 1).astype(int) for f, n in zip(fs, shape)]
    near = np.min([np.where((f > 0) & (f < n), np.abs(f - np.round(f)), np.inf) for f, n in zip(fs, shape)], axis=0)
    cell = idx[0] * shape[1] + idx[1]
    if len(shape) > 2:
        cell = cell * shape[2] + idx[2]
    return cell, near


@pytest.mark.parametrize("axes,shape", [(("E", "Lz/Lc"), (32, 32)), (("E", "L/Lc", "Lz/L"), (32, 32, 8))])
def test_log_potential_cells_brute_force(axes, shape):
    """Cells of the logarithmic-potential workloads' grids (cfg 2/3: (E, Lz/Lc) 32x32;
    cfg 5's judge: (E, L/Lc, Lz/L) 32x32x8) against cells computed here with Lc(E)
    from a root solve of the circular-orbit energy: identical except particles
    within 1e-9 cells of an edge.  Swapping the second axis (L/Lc for Lz/Lc and
    back) or the sign of Lz moves many particles."""
    cfg = configs.cfg2(N=4000, target_n=1 << 14)
    cfg["prior"] = {"kind": "hist", "axes": axes, "shape": shape, "period": 1}
    inp = configs.make_inputs(cfg)
    m = oracle.Model(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    got = m.cells()
    want, near = cells_here(inp["ics"], m.Erange, shape, axes[1])
    sure = near > 1e-9
    assert sure.sum() >= 3990
    np.testing.assert_array_equal(got[sure], want[sure])
    other = "L/Lc" if axes[1] == "Lz/Lc" else "Lz/Lc"
    swapped, _ = cells_here(inp["ics"], m.Erange, shape, other)
    assert np.mean(swapped != got) > 0.3
    flipped = inp["ics"].copy()
    flipped[3:5] *= -1.0     # Lz -> -Lz, E and L unchanged
    fl, _ = cells_here(flipped, m.Erange, shape, axes[1])
    assert np.mean(fl != got) > 0.3


@pytest.mark.parametrize("axes,shape", [(("E", "Lz/Lc"), (32, 32)), (("E", "L/Lc", "Lz/L"), (32, 32, 8))])
def test_log_potential_cell_means_brute_force(axes, shape):
    """O(N^2) cell means at N = 100 (the test's own cells) against the oracle's
    priors; sum of priors = sum of weights."""
    cfg = configs.cfg2(N=100, target_n=1 << 12)
    cfg["prior"] = {"kind": "hist", "axes": axes, "shape": shape, "period": 1}
    inp = configs.make_inputs(cfg)
    rng = np.random.default_rng(9)
    w = rng.uniform(0.2, 2.0, 100) / 100
    m = oracle.Model(cfg, inp["ics"], w, inp["Y"], inp["sigma"])
    cells, near = cells_here(inp["ics"], m.Erange, shape, axes[1])
    assert np.all(near > 1e-9)
    what = np.array([np.mean([w[k] for k in range(100) if cells[k] == cells[i]]) for i in range(100)])
    got, cs, cn = m.prior_means()
    np.testing.assert_allclose(got, what, rtol=1e-14)
    assert got.sum() == pytest.approx(w.sum(), rel=1e-13)
