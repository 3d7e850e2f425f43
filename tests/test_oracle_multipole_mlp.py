"""Pins of the oracle's self-consistent multipole potential, learned prior and
counter-based generator.

Self-consistent potential (paper sections 1-2): pinned to the Legendre addition
theorem summed by brute force, the exact monopole, finite differences and a sampled
Hernquist sphere.  Learned prior (reading of section 2.1's moving priors): pinned to
central finite differences, the first Adam step's closed form and a learnable
linear target.  Philox4x32-10: pinned to published known-answer vectors.
"""
import os

import numpy as np
import pytest
from scipy import special

import oracle
from oracle import mlp
from synth import galaxy

GOLD = os.path.join(os.path.dirname(__file__), "golden")
MP = {"kind": "multipole", "G": 1.0, "lmax": 8, "nodes": 200, "rmin": 1e-3, "rmax": 100.0, "Mtot": 1.0}


def cloud(n, seed=7):
    rng = np.random.default_rng(seed)
    pos = rng.normal(0, 1.0, (3, n)) * np.array([[1.0], [0.7], [0.5]]) + np.array([[0.2], [0.0], [-0.1]])
    w = rng.uniform(0.5, 1.5, n)
    return pos, w / w.sum()


def test_legendre_matches_scipy():
    for x in [-0.9, -0.3, 0.0, 0.4, 0.99]:
        P = oracle.legendre(8, x)
        for l in range(9):
            for m in range(l + 1):
                assert P[l, m] == pytest.approx(special.lpmv(m, l, x), rel=1e-12, abs=1e-14)


def brute_phi(pos, w, pt, lmax, G=1.0):
    """-G sum_k m_k sum_l r<^l / r>^(l+1) P_l(cos gamma_k) (addition theorem, truncated)."""
    r = np.linalg.norm(pos, axis=0)
    rp = np.linalg.norm(pt)
    cg = (pos.T @ pt) / (r * rp)
    rl, rg = np.minimum(r, rp), np.maximum(r, rp)
    s = 0.0
    for l in range(lmax + 1):
        s += np.sum(w * rl ** l / rg ** (l + 1) * special.eval_legendre(l, cg))
    return -G * s


def test_exact_expansion_matches_addition_theorem():
    pos, w = cloud(100)
    rng = np.random.default_rng(8)
    for _ in range(10):
        pt = rng.normal(0, 1.2, 3)
        phi = oracle.mp_exact(MP, pos, w, pt)[0]
        assert phi == pytest.approx(brute_phi(pos, w, pt, 8), rel=1e-11)


def test_exact_expansion_force_is_minus_gradient():
    pos, w = cloud(100)
    r = np.sort(np.linalg.norm(pos, axis=0))
    rng = np.random.default_rng(9)
    h = 1e-6
    done = 0
    while done < 8:
        pt = rng.normal(0, 1.2, 3)
        rp = np.linalg.norm(pt)
        if np.min(np.abs(r - rp)) < 1e-3:
            continue
        _, ax, ay, az = oracle.mp_exact(MP, pos, w, pt)
        g = np.zeros(3)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            g[k] = (oracle.mp_exact(MP, pos, w, pt + e)[0] - oracle.mp_exact(MP, pos, w, pt - e)[0]) / (2 * h)
        np.testing.assert_allclose([ax, ay, az], -g, rtol=1e-6, atol=1e-8)
        done += 1


@pytest.mark.parametrize("pt", [(0.0, 0.0, 0.7), (0.0, 0.0, -1.3), (1e-7, 0.0, 0.9)])
def test_force_on_the_polar_axis_is_minus_gradient(pt):
    """On (and next to) the z axis the spherical angles are singular but the force is
    not: central differences of Phi in x, y, z give it."""
    pos, w = cloud(100)
    pt = np.array(pt)
    _, ax, ay, az = oracle.mp_exact(MP, pos, w, pt)
    h = 1e-5
    g = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        g[k] = (oracle.mp_exact(MP, pos, w, pt + e)[0] - oracle.mp_exact(MP, pos, w, pt - e)[0]) / (2 * h)
    scale = np.abs(g).max()
    np.testing.assert_allclose([ax, ay, az], -g, rtol=0, atol=1e-6 * scale)


def test_node_tables_equal_exact_at_node_radii():
    pos, w = cloud(100)
    A, B = oracle.mp_coeffs(MP, pos, w)
    lr = np.linspace(np.log(1e-3), np.log(100.0), 200)
    rng = np.random.default_rng(10)
    for k in [60, 100, 120, 140, 170]:
        d = rng.normal(0, 1, 3)
        pt = d / np.linalg.norm(d) * np.exp(lr[k])
        node = [v[0] for v in oracle.mp_eval(MP, A, B, pt[:, None])]
        exact = oracle.mp_exact(MP, pos, w, pt)
        np.testing.assert_allclose(node, exact, rtol=1e-9, atol=1e-12)


def test_monopole_is_exact_for_lmax0():
    pos, w = cloud(100)
    mp0 = dict(MP, lmax=0)
    r = np.linalg.norm(pos, axis=0)
    for rp in [0.3, 1.0, 2.5]:
        pt = np.array([0.0, rp, 0.0])
        phi, ax, ay, az = oracle.mp_exact(mp0, pos, w, pt)
        inside = r < rp
        assert phi == pytest.approx(-(w[inside].sum() / rp + np.sum(w[~inside] / r[~inside])), rel=1e-13)
        assert ay == pytest.approx(-w[inside].sum() / rp ** 2, rel=1e-12)


@pytest.mark.slow
def test_sampled_hernquist_potential():
    """N = 2e5 Hernquist sphere: Phi within 1% of -1/(r+1) at r in [0.3, 10]."""
    rng = np.random.default_rng(11)
    x, y, z = galaxy.hernquist_positions(rng, 200000, rmax=1e4)
    pos = np.stack([x, y, z])
    w = np.full(x.size, 1.0 / x.size)
    mp = dict(MP, rmax=1e4, Mtot=galaxy.hernquist_mass(1e4))
    A, B = oracle.mp_coeffs(mp, pos, w)
    d = rng.normal(0, 1, (3, 40))
    rr = np.geomspace(0.3, 10.0, 40)
    pts = d / np.linalg.norm(d, axis=0) * rr
    phi, ax, ay, az = oracle.mp_eval(mp, A, B, pts)
    np.testing.assert_allclose(phi, -1.0 / (rr + 1.0), rtol=1e-2)
    ar = (ax * pts[0] + ay * pts[1] + az * pts[2]) / rr
    # l = 1..8 shot noise of 2e5 particles perturbs the force by a few per cent
    np.testing.assert_allclose(ar, -1.0 / (rr + 1.0) ** 2, rtol=6e-2)
    # the monopole alone is accurate to the Poisson noise of the enclosed particles
    mp0 = dict(mp, lmax=0)
    A0, B0 = oracle.mp_coeffs(mp0, pos, w)
    phi0, ax0, ay0, az0 = oracle.mp_eval(mp0, A0, B0, pts)
    ar0 = (ax0 * pts[0] + ay0 * pts[1] + az0 * pts[2]) / rr
    np.testing.assert_allclose(phi0, -1.0 / (rr + 1.0), rtol=5e-3)
    np.testing.assert_allclose(ar0, -1.0 / (rr + 1.0) ** 2, rtol=1.5e-2)


# ------------------------------------------------------------------------ MLP
def rand_theta(seed=0, scale=0.5):
    return np.random.default_rng(seed).normal(0, scale, mlp.NPARAM)


def test_mlp_parameter_count():
    assert mlp.NPARAM == 4481


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(12)
    u = rng.uniform(-1, 1, (32, 3))
    t = rng.normal(0, 1, 32)
    th = rand_theta()
    _, g = mlp.loss_grad(th, u, t)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [0, 191, 192, 255, 4480, 4479]])
    h = 1e-4
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        # fourth-order central difference
        fd = (8 * (mlp.loss(th + e, u, t) - mlp.loss(th - e, u, t))
              - (mlp.loss(th + 2 * e, u, t) - mlp.loss(th - 2 * e, u, t))) / (12 * h)
        assert g[k] == pytest.approx(fd, rel=1e-7, abs=1e-10)


def test_adam_first_step_closed_form():
    """After one step from zero moments, m_hat/sqrt(v_hat) = sign(g): theta - lr sign(g)."""
    th = rand_theta(1)
    g = np.random.default_rng(2).normal(0, 1, mlp.NPARAM)
    new, m, v = mlp.adam(th, g, np.zeros_like(th), np.zeros_like(th), 1, 1e-3, 0.9, 0.999, 0.0)
    np.testing.assert_allclose(new, th - 1e-3 * np.sign(g), rtol=1e-13, atol=1e-16)


@pytest.mark.slow
def test_mlp_learns_linear_target():
    rng = np.random.default_rng(13)
    a, b = np.array([0.3, -0.5, 0.2]), 0.1
    th = rng.normal(0, 0.3, mlp.NPARAM)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for t in range(1, 3001):
        u = rng.uniform(-1, 1, (256, 3))
        _, g = mlp.loss_grad(th, u, u @ a + b)
        th, m, v = mlp.adam(th, g, m, v, t, 3e-3, 0.9, 0.999, 1e-8)
    u = rng.uniform(-1, 1, (4096, 3))
    assert mlp.loss(th, u, u @ a + b) < 1e-4


def test_priors_rescaled_to_weight_sum():
    rng = np.random.default_rng(14)
    u = rng.uniform(-1, 1, (500, 3))
    w = rng.uniform(0.1, 1.0, 500)
    what = mlp.priors(rand_theta(3), u, w)
    assert what.sum() == pytest.approx(w.sum(), rel=1e-13)
    assert np.all(what > 0)


# ---------------------------------------------------------------------- Philox
def test_philox_known_answers():
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        assert oracle.philox4x32(v[0:4], v[4:6]) == v[6:10]


def test_subset_indices_in_range_and_uniform():
    idx = oracle.subset(12345, 3, 1 << 16, 1000)
    assert idx.min() >= 0 and idx.max() < 1000
    counts = np.bincount(idx, minlength=1000)
    assert counts.std() < 3 * np.sqrt(65.536)


# ---------------------------------------------------- learned prior: refreshes
def small_mlp_model(N=3000, **prior):
    from synth import configs
    cfg = configs.cfg5(N=N, target_n=1 << 14)
    cfg["prior"].update(prior)
    inp = configs.make_inputs(cfg)
    m = oracle.Model(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    pr = cfg["prior"]
    lp = mlp.LearnedPrior(pr["mlp_init"], pr["lr"], pr["beta1"], pr["beta2"], pr["adam_eps"], pr["seed"],
                          pr["subset"], pr["batch"], pr["fallback"])
    return cfg, m, lp


def test_circular_orbit_has_L_equal_Lc():
    """Integrals of a circular orbit in the equatorial plane of the logarithmic
    potential: L = Lc(E) (the feature 2 L/Lc - 1 = 1) and Lz = L."""
    from synth import configs
    cfg, m, _ = small_mlp_model(N=8)
    lp = configs.LOG_POT
    R = np.array([0.05, 0.3, 1.0, 4.0])
    vc = lp["v0"] * R / np.sqrt(lp["Rc"] ** 2 + R * R)
    ics = np.zeros((6, R.size))
    ics[0], ics[4] = R, vc
    mc = oracle.Model(cfg, ics, np.full(R.size, 0.25), np.zeros(m.J), np.ones(m.J), Erange=m.Erange)
    E, L, Lz, Lc = mc.integrals()
    np.testing.assert_allclose(L, Lc, rtol=1e-10)
    np.testing.assert_allclose(Lz, L, rtol=1e-14)
    np.testing.assert_allclose(E, 0.5 * vc ** 2 + 0.5 * lp["v0"] ** 2 * np.log(lp["Rc"] ** 2 + R * R), rtol=1e-14)


def test_refresh_with_zero_threshold_gives_the_histogram_prior():
    cfg, m, lp = small_mlp_model(subset=512, batch=128, fallback=0.0)
    E, L, Lz, Lc = m.integrals()
    u = mlp.features(E, L, Lz, Lc, *m.Erange)
    hist = m.prior_means()[0]
    what = lp.refresh(0, oracle.subset(lp.seed, 0, lp.subset, u.shape[0]), u, m.w, hist)
    assert lp.used_fallback and lp.last_judge > 0
    np.testing.assert_array_equal(what, hist)


def test_refresh_counts_adam_steps_and_normalises():
    cfg, m, lp = small_mlp_model(subset=512, batch=128, fallback=1e9)
    E, L, Lz, Lc = m.integrals()
    u = mlp.features(E, L, Lz, Lc, *m.Erange)
    hist = m.prior_means()[0]
    th0 = lp.theta.copy()
    what = lp.refresh(0, oracle.subset(lp.seed, 0, lp.subset, u.shape[0]), u, m.w, hist)
    assert lp.t == 4 and not lp.used_fallback
    assert np.sum(what) == pytest.approx(np.sum(m.w), rel=1e-12)
    # Adam's step bound (Kingma & Ba, section 2.1): |step| <= lr (1 - b1)/sqrt(1 - b2)
    # when 1 - b1 > sqrt(1 - b2)
    assert np.max(np.abs(lp.theta - th0)) <= 4 * lp.lr * (1 - lp.beta1) / np.sqrt(1 - lp.beta2)
    lp.refresh(1, oracle.subset(lp.seed, 1, lp.subset, u.shape[0]), u, m.w, hist)
    assert lp.t == 8


def test_first_adam_step_moves_each_parameter_by_lr():
    """One minibatch per refresh: the first Adam step is lr g / (|g| + eps) per parameter."""
    cfg, m, lp = small_mlp_model(subset=256, batch=256, fallback=1e9)
    E, L, Lz, Lc = m.integrals()
    u = mlp.features(E, L, Lz, Lc, *m.Erange)
    idx = oracle.subset(lp.seed, 0, lp.subset, u.shape[0])
    _, g = mlp.loss_grad(lp.theta, u[idx], np.log(m.w[idx]))
    th0 = lp.theta.copy()
    lp.refresh(0, idx, u, m.w, m.prior_means()[0])
    np.testing.assert_allclose(th0 - lp.theta, lp.lr * g / (np.abs(g) + lp.eps), rtol=1e-9, atol=1e-15)


def test_refresh_training_lowers_the_loss():
    """Training on the refresh's own sample lowers the loss on it."""
    cfg, m, lp = small_mlp_model(N=4000, subset=4096, batch=256, fallback=1e9)
    E, L, Lz, Lc = m.integrals()
    u = mlp.features(E, L, Lz, Lc, *m.Erange)
    rng = np.random.default_rng(3)
    w = m.w * np.exp(0.3 * u[:, 0] - 0.2 * u[:, 1] + 0.05 * rng.normal(size=u.shape[0]))
    idx = oracle.subset(lp.seed, 0, lp.subset, u.shape[0])
    before = mlp.loss(lp.theta, u[idx], np.log(w[idx]))
    for q in range(4):
        lp.refresh(q, idx, u, w, m.prior_means()[0])
    assert mlp.loss(lp.theta, u[idx], np.log(w[idx])) < 0.5 * before
