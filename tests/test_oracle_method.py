"""Pins of the oracle's M2M arithmetic: observables, smoothing, chi^2, entropy,
weight update and moving prior.

Paper anchors: eq. (1) F = -chi^2/2 + mu S and eq. (2) S = -sum w ln(w/what)
(section 2); flat priors what = 1/N and initial weights 1/N (section 2.1); moving
priors from the weight distribution over integrals of motion (section 2.1).  The
remaining rules are readings; each test fixes one with an independent route:
closed-form recurrences, exact special cases and brute force on tiny inputs.
"""
import copy

import numpy as np
import pytest

import oracle
from synth import configs

HERN = {"kind": "hernquist", "G": 1.0, "M": 1.0, "a": 1.0}


def small_cfg(**kw):
    c = configs.cfg1(N=100)
    c.update(kw)
    return c


# ------------------------------------------------------------------ observables
def brute_K(layout, z):
    """Dense kernel row written from the bin definitions (explicit edge comparisons)."""
    x, y, zz, vx, vy, vz = z
    inc = layout["incl"]
    X, Ys = x, y * np.cos(inc) - zz * np.sin(inc)
    vl = vy * np.sin(inc) + vz * np.cos(inc)
    row = []
    for b in layout["binnings"]:
        if b["kind"] == "grid":
            hx = (b["x1"] - b["x0"]) / b["nx"]
            hy = (b["y1"] - b["y0"]) / b["ny"]
            ind = np.zeros(b["nx"] * b["ny"])
            for iy in range(b["ny"]):
                for ix in range(b["nx"]):
                    if (b["x0"] + ix * hx <= X < b["x0"] + (ix + 1) * hx
                            and b["y0"] + iy * hy <= Ys < b["y0"] + (iy + 1) * hy):
                        ind[iy * b["nx"] + ix] = 1.0
        else:
            rad = np.sqrt(x * x + y * y + zz * zz) if b["kind"] == "shell" else np.hypot(X, Ys)
            e = b["edges"]
            ind = np.array([1.0 if e[k] <= rad < e[k + 1] else 0.0 for k in range(len(e) - 1)])
        for m in b["moments"]:
            row.append(ind * vl ** m)
    return np.concatenate(row)


@pytest.mark.parametrize("layout", [configs.layout_cfg1(), configs.layout_cfg3()])
def test_observe_matches_dense_brute_force(layout):
    rng = np.random.default_rng(3)
    N = 100
    ics = np.concatenate([rng.normal(0, 1.5, (3, N)), rng.normal(0, 0.7, (3, N))])
    w = rng.uniform(0.5, 1.5, N) / N
    c = small_cfg(layout=layout)
    J = sum(len(b["moments"]) * (len(b["edges"]) - 1 if b["kind"] != "grid" else b["nx"] * b["ny"])
            for b in layout["binnings"])
    m = oracle.Model(c, ics, w, np.ones(J), np.ones(J), Erange=(-1, 0))
    Kd = np.stack([brute_K(layout, ics[:, i]) for i in range(N)])   # [N, J]
    np.testing.assert_allclose(m.observe(), w @ Kd, rtol=1e-13, atol=1e-18)


def test_observe_all_in_one_bin():
    """Every particle in one pixel: y = sum w, sum w v, sum w v^2 for that bin only."""
    layout = configs.layout_cfg2()
    rng = np.random.default_rng(4)
    N = 1000
    inc = layout["incl"]
    ics = np.zeros((6, N))
    ics[0] = rng.uniform(0.01, 0.15, N)               # X in pixel column 32 (width 10/64)
    ics[1] = rng.uniform(0.01, 0.05, N) / np.cos(inc)  # Y = y cos i when z = 0
    ics[3:] = rng.normal(0, 1, (3, N))
    w = rng.uniform(0.1, 1.0, N)
    c = small_cfg(layout=layout)
    J = 4096 + 800
    m = oracle.Model(c, ics, w, np.ones(J), np.ones(J), Erange=(-1, 0))
    y = m.observe()
    vl = ics[4] * np.sin(inc) + ics[5] * np.cos(inc)
    pix = 32 * 64 + 32
    kin = 10 * 20 + 10
    assert y[pix] == pytest.approx(w.sum(), rel=1e-14)
    assert y[4096 + kin] == pytest.approx((w * vl).sum(), rel=1e-12)
    assert y[4096 + 400 + kin] == pytest.approx((w * vl ** 2).sum(), rel=1e-13)
    mask = np.ones(J, bool)
    mask[[pix, 4096 + kin, 4096 + 400 + kin]] = False
    assert np.all(y[mask] == 0.0)


def test_sky_projection_special_cases():
    """Inclination 0: sky (x, y), v_los = vz.  Inclination 90 deg: sky (x, -z), v_los = vy."""
    z = [0.3, 0.2, -0.1, 0.5, 0.7, -0.4]
    lay = {"incl": 0.0, "binnings": [{"kind": "grid", "nx": 2, "ny": 2, "x0": -1, "x1": 1, "y0": -1, "y1": 1,
                                      "moments": (1,)}]}
    (j, K), = oracle.kernel_entries(lay, z)
    assert (j, K) == (3, -0.4)
    lay["incl"] = np.pi / 2
    (j, K), = oracle.kernel_entries(lay, z)
    assert j == 3 and K == pytest.approx(0.7, rel=1e-15)
    z[2] = 0.1
    (j, K), = oracle.kernel_entries(lay, z)
    assert j == 1


# -------------------------------------------------------------- smoothing, chi^2
def test_ema_impulse_response_and_fixed_point():
    """Frozen particles, eps = 0: a constant input is a fixed point; after the weights
    jump once, ys(n) = yB + (yA - yB)(1 - dt/tau)^(n-1) for n >= 1."""
    c = configs.cfg1(N=300)
    c.update(frozen=True, eps=0.0)
    inp = configs.make_inputs(c)
    m = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    m.run(1)
    yA = m.arr["ys"].copy()
    np.testing.assert_array_equal(yA, m.observe())
    m.run(3)
    np.testing.assert_allclose(m.arr["ys"], yA, rtol=1e-15)
    m.arr["w"][:] *= np.linspace(0.5, 1.5, c["N"])
    yB = m.observe()
    g = c["dt"] / c["tau"]
    for n in range(1, 30):
        m.run(1)
        np.testing.assert_allclose(m.arr["ys"], yB + (yA - yB) * (1 - g) ** n, rtol=1e-12, atol=1e-18)


def test_chi2_and_entropy_definitions():
    """chi^2 = sum ((ys - Y)/sigma)^2 (eq. 1); S(0) = 0 exactly for w = what = 1/N (eq. 2,
    section 2.1); F = -chi^2/2 + mu S."""
    c = configs.cfg1(N=500)
    c["prior"] = {"kind": "flat"}
    inp = configs.make_inputs(c)
    m = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    y0 = m.observe()
    st = m.run(1)[0]
    assert st[0] == pytest.approx(np.sum(((y0 - inp["Y"]) / inp["sigma"]) ** 2), rel=1e-13)
    assert st[2] == 0.0
    assert st[3] == pytest.approx(-0.5 * st[0], rel=1e-15)


def test_entropy_hand_values():
    """S = -sum w ln(w/what) on a two-particle example."""
    c = configs.cfg1(N=2)
    c.update(frozen=True, eps=0.0, mu=0.3)
    c["prior"] = {"kind": "external"}
    ics = np.array([[0.5, -0.5], [0, 0], [0, 0], [0, 0], [0.1, 0.1], [0, 0]], dtype=float)
    m = oracle.Model(c, ics, np.array([0.5, 0.5]), np.ones(50), np.ones(50))
    m.set_what(np.array([0.25, 0.75]))
    st = m.run(1)[0]
    S = -(0.5 * np.log(2.0) + 0.5 * np.log(0.5 / 0.75))
    assert st[2] == pytest.approx(S, rel=1e-15)
    assert st[3] == pytest.approx(-0.5 * st[0] + 0.3 * S, rel=1e-14)


# ----------------------------------------------------------------- update law
@pytest.mark.parametrize("law", ["exp", "euler"])
def test_update_entropy_only_closed_form(law):
    """Frozen particles, chi^2 switched off (huge sigma), one prior cell with equal
    weights (what = w): G = -mu, so w_n = w_0 exp(-eps dt mu n) or w_0 (1 - eps dt mu)^n."""
    c = configs.cfg1(N=200)
    c.update(frozen=True, eps=0.05, mu=0.5, update=law)
    c["prior"] = {"kind": "hist", "axes": ("E", "L/Lc"), "shape": (1, 1), "period": 1}
    inp = configs.make_inputs(c)
    m = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], np.full(50, 1e300))
    a = c["eps"] * c["dt"] * c["mu"]
    for n in range(1, 50):
        m.run(1)
        expect = (1.0 / 200) * (np.exp(-a * n) if law == "exp" else (1 - a) ** n)
        np.testing.assert_allclose(m.w, expect, rtol=1e-13)


@pytest.mark.parametrize("law", ["exp", "euler"])
def test_update_single_bin_recurrence(law):
    """One shell holding every particle, mu = 0, tau = dt (no smoothing):
    W_n+1 = W_n exp(-eps dt (W_n - Y)/sigma^2) (or W_n (1 - eps dt (W_n - Y)/sigma^2))."""
    c = configs.cfg1(N=64)
    c.update(frozen=True, eps=2e-4, mu=0.0, tau=0.01, update=law)
    c["layout"] = {"incl": 0.0, "binnings": [{"kind": "shell", "edges": np.array([0.0, 1e9]),
                                              "moments": (0,)}]}
    c["prior"] = {"kind": "flat"}
    inp = configs.make_inputs(c)
    Y, sig = np.array([0.7]), np.array([0.05])
    m = oracle.Model(c, inp["ics"], inp["w"], Y, sig)
    W = 1.0
    for n in range(40):
        m.run(1)
        f = c["eps"] * c["dt"] * (W - Y[0]) / sig[0] ** 2
        W = W * (np.exp(-f) if law == "exp" else 1 - f)
        assert m.w.sum() == pytest.approx(W, rel=1e-12)


def test_chi2_monotone_with_frozen_particles():
    """mu = 0, no smoothing, frozen particles, small eps dt: chi^2 never rises."""
    c = configs.cfg1(N=2000)
    c.update(frozen=True, eps=2e-5, mu=0.0, tau=0.01)
    c["prior"] = {"kind": "flat"}
    inp = configs.make_inputs(c)
    m = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    chi = m.run(300)[:, 0]
    assert np.all(np.diff(chi) <= 1e-12 * chi[:-1])
    assert chi[-1] < 0.5 * chi[0]


@pytest.mark.slow
def test_cfg1_chi2_falls_and_weights_stay_positive():
    """Moving particles, cfg 1 settings: smoothed chi^2 falls by 20x within 1000 steps
    and stays down (every 100-step sample after step 500 below chi^2(0)/10); w > 0."""
    c = configs.cfg1(N=20000, steps=1000)
    inp = configs.make_inputs(c)
    m = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    st = m.run(1000)
    assert m.status == 0
    chi = st[:, 0]
    assert chi[-1] < chi[0] / 20
    assert np.all(chi[500::100] < chi[0] / 10)
    assert np.all(st[:, 5] > 0)


def test_nonpositive_weight_is_reported():
    """Euler law with eps dt G < -1 for some particle stops with status 4 at step 0."""
    c = configs.cfg1(N=2000)
    c.update(update="euler", eps=1.0)
    inp = configs.make_inputs(c)
    m = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    m.run(5)
    assert m.status == 4 and m.s.bad_step == 0


# --------------------------------------------------------------- moving prior
def brute_cells(cfg, ics, Erange):
    """Cell index of each particle from E, L and the closed-form Hernquist Lc(E)."""
    x, y, z, vx, vy, vz = ics
    r = np.sqrt(x * x + y * y + z * z)
    E = 0.5 * (vx * vx + vy * vy + vz * vz) - 1.0 / (r + 1.0)
    L = np.sqrt((y * vz - z * vy) ** 2 + (z * vx - x * vz) ** 2 + (x * vy - y * vx) ** 2)
    u = (1.0 + np.sqrt(1.0 - 8.0 * E)) / (-4.0 * E)
    rc = u - 1.0
    Lc = rc * np.sqrt(rc) / (rc + 1.0)
    nE, nL = cfg["prior"]["shape"]
    iE = np.clip(np.floor((E - Erange[0]) / (Erange[1] - Erange[0]) * nE), 0, nE - 1).astype(int)
    iL = np.clip(np.floor(L / Lc * nL), 0, nL - 1).astype(int)
    return iE * nL + iL


def test_prior_cells_and_means_brute_force():
    """O(N^2) cell means at N = 100 against the oracle's what; sum what = sum w."""
    c = configs.cfg1(N=100)
    inp = configs.make_inputs(c)
    rng = np.random.default_rng(5)
    w = rng.uniform(0.2, 2.0, 100) / 100
    m = oracle.Model(c, inp["ics"], w, inp["Y"], inp["sigma"])
    cells = brute_cells(c, inp["ics"], m.Erange)
    np.testing.assert_array_equal(m.cells(), cells)
    what = np.array([np.mean([w[k] for k in range(100) if cells[k] == cells[i]]) for i in range(100)])
    got, cs, cn = m.prior_means()
    np.testing.assert_allclose(got, what, rtol=1e-14)
    assert got.sum() == pytest.approx(w.sum(), rel=1e-13)
    assert cn.sum() == 100


def test_prior_equal_weights_in_cell_give_w():
    c = configs.cfg2(N=5000, target_n=1 << 14)
    inp = configs.make_inputs(c)
    m = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    cells = m.cells()
    w = (1.0 + cells % 7) / 5000.0
    m.arr["w"][:] = w
    what, _, _ = m.prior_means()
    np.testing.assert_allclose(what, w, rtol=1e-14)


def test_checkpoint_restart_is_bitwise():
    """State (x, v, w, ys, what, n) copied after 7 steps continues bitwise."""
    c = configs.cfg1(N=500)
    inp = configs.make_inputs(c)
    a = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    a.run(7)
    snap = {k: v.copy() for k, v in a.arr.items()}
    b = oracle.Model(c, a.ics(), snap["w"], inp["Y"], inp["sigma"], Erange=a.Erange)
    for k in ("ys", "what"):
        b.arr[k][:] = snap[k]
    b.s.n = a.s.n
    sa = a.run(9)
    sb = b.run(9)
    np.testing.assert_array_equal(sa, sb)
    np.testing.assert_array_equal(a.w, b.w)
    np.testing.assert_array_equal(a.ics(), b.ics())


def test_batched_models_are_independent():
    """A model's trajectory does not depend on which other models exist (cfg 4 is a set
    of independent M2M runs)."""
    c = configs.cfg4(n_models=2, nmin=300, nmax=400, steps=5)
    inp = configs.make_inputs(c)
    n0 = int(c["model_sizes"][0])
    m = oracle.Model(c, inp["ics"][:, :n0], inp["w"][:n0], inp["Y"], inp["sigma"], model=0)
    st = m.run(5)
    m2 = oracle.Model(copy.deepcopy(c), inp["ics"][:, :n0].copy(), inp["w"][:n0].copy(), inp["Y"],
                      inp["sigma"], model=0)
    np.testing.assert_array_equal(st, m2.run(5))
