"""GPU parity of the self-consistent multipole model (sections 1-2: the potential
computed from the particles) against the FP64 oracle, through the C ABI.

Bars:
  node tables -- each coefficient within rtol * scale, scale = sum over the same
    particles of m_i r_i^l (or r_i^-(l+1)) times max |P_l^m| (so that coefficients
    that cancel to ~0 are judged against the size of their terms): rtol 1e-12 for
    FP64 (summation order only); FP32, same coordinates on both sides (the initial
    state): 2e-6 (FP32 terms, per-lane FP32 sums of 16 particles and a 64-lane
    butterfly, FP64 above: each under 2e-7 of the scale in a numpy restatement,
    3.4e-7 measured); FP32 after steps: 2e-5 (the two sides' coordinates then
    differ by the FP32 rounding of the orbit integration, which dominates);
  FP64 steps -- weights, coordinates and statistics within 1e-10 relative after a
    few steps (FP64 atomics make the summation order, and so the last bits of the
    coefficients, vary);
  FP32 steps -- one step: weights within 2e-6 relative, coordinates within 2e-6
    relative plus 2e-6 of their largest magnitude; observables as the fused-kernel
    tests (particles within 1e-5 of a bin edge may land on either side).
"""
import numpy as np
import pytest

import oracle
from synth import configs
from tests import helpers as H

pytestmark = pytest.mark.gpu

m2m = pytest.importorskip("paper_1207_6403_amd")


def pmax(lmax):
    """max over x in [-1, 1] of |P_l^m(x)| (oracle Legendre on a fine grid)."""
    xs = np.linspace(-1.0, 1.0, 2001)
    return np.max(np.abs(np.stack([oracle.legendre(lmax, x) for x in xs])), axis=0)


def node_radii(pot):
    lr0 = np.log(pot["rmin"])
    return np.exp(lr0 + np.arange(pot["nodes"]) * (np.log(pot["rmax"]) - lr0) / (pot["nodes"] - 1))


def radii(ics):
    x, y, z = np.asarray(ics[:3], dtype=np.float64)
    return np.sqrt(x * x + y * y + z * z)


def coefficient_rows(pot):
    """(l, column indices) of the coefficients of degree l."""
    return [(l, [l * l] + [l * l + 2 * mm - 1 + s for mm in range(1, l + 1) for s in (0, 1)])
            for l in range(pot["lmax"] + 1)]


def table_scale(pot, r, m):
    """Per-node, per-coefficient size of the terms summed into A (particles below the
    node radius) and B (the rest): m_i r_i^l (or r_i^-(l+1)) times max |P_l^m|.
    Prefix sums for A and suffix sums for B, both accumulated from the small terms
    up, so that neither loses the nodes' partial sums to cancellation."""
    nn, nlm = pot["nodes"], (pot["lmax"] + 1) ** 2
    P = pmax(pot["lmax"])
    order = np.argsort(r)
    rs, ms = r[order], m[order]
    cut = np.searchsorted(rs, node_radii(pot), side="left")    # particles with r < r_k
    SA = np.zeros((nn, nlm))
    SB = np.zeros((nn, nlm))
    for l, cols in coefficient_rows(pot):
        pre = np.concatenate([[0.0], np.cumsum(ms * rs ** l)])
        with np.errstate(divide="ignore"):
            tb = np.where(rs > 0, ms / rs ** (l + 1), 0.0)
        suf = np.concatenate([np.cumsum(tb[::-1])[::-1], [0.0]])
        for j in cols:
            mm = (j - l * l + 1) // 2
            SA[:, j] = pre[cut] * P[l, mm]
            SB[:, j] = suf[cut] * P[l, mm]
    return SA, SB


def flip_allowance(pot, r, m, r_other):
    """Terms of the particles counted below node k by one side and above it by the
    other (radii r and r_other on different sides of r_k), added to both tables."""
    nn, nlm = pot["nodes"], (pot["lmax"] + 1) ** 2
    P = pmax(pot["lmax"])
    rk = node_radii(pot)
    ka = np.searchsorted(rk, r, side="right")
    kb = np.searchsorted(rk, r_other, side="right")
    XA = np.zeros((nn, nlm))
    XB = np.zeros((nn, nlm))
    idx = np.nonzero(ka != kb)[0]
    for i in idx:
        ks = slice(min(ka[i], kb[i]), max(ka[i], kb[i]))
        for l, cols in coefficient_rows(pot):
            for j in cols:
                mm = (j - l * l + 1) // 2
                XA[ks, j] += m[i] * r[i] ** l * P[l, mm]
                XB[ks, j] += m[i] / r[i] ** (l + 1) * P[l, mm]
    return XA, XB, idx.size


def check_tables(ctx, pot, om, ics, w, rtol, ics_gpu=None):
    """GPU node tables against the oracle's, each coefficient within rtol times its
    scale.  When the two sides' particles differ (after steps), a particle whose two
    radii lie on different sides of a node radius is counted below that node by one
    side only: its terms are added to that node's allowance."""
    lmax, nn = pot["lmax"], pot["nodes"]
    nlm = (lmax + 1) ** 2
    A, B = m2m.m2m_multipole_tables(ctx, nn, lmax)
    Ao = om.arr["mpA"].reshape(nn, nlm)
    Bo = om.arr["mpB"].reshape(nn, nlm)
    r = radii(ics)
    m = np.asarray(w, dtype=np.float64) * pot["Mtot"]
    SA, SB = table_scale(pot, r, m)
    XA, XB, nflip = (np.zeros_like(SA), np.zeros_like(SB), 0) if ics_gpu is None else \
        flip_allowance(pot, r, m, radii(ics_gpu))
    ea = np.abs(A - Ao) / np.maximum(rtol * SA + XA, 1e-300)
    eb = np.abs(B - Bo) / np.maximum(rtol * SB + XB, 1e-300)
    H.flush("tables: max error / allowance A %.3g B %.3g; max error / scale A %.3g B %.3g; "
            "particles across a node radius: %d" % (
                ea.max(), eb.max(), (np.abs(A - Ao) / np.maximum(SA, 1e-300)).max(),
                (np.abs(B - Bo) / np.maximum(SB, 1e-300)).max(), nflip))
    assert np.all(np.abs(A - Ao) <= rtol * SA + XA + 1e-300)
    assert np.all(np.abs(B - Bo) <= rtol * SB + XB + 1e-300)


def small(N, precision):
    cfg = configs.cfg3(N=N, target_n=1 << 18)
    cfg["precision"] = precision
    return cfg


def start(cfg, launch=None):
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case %s %s N=%d launch=%s" % (cfg["name"], cfg["precision"], cfg["N"], launch))
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    if launch:
        m2m.m2m_set_launch(ctx, **launch)
    (om,) = H.oracle_models(cfg, inp, er)
    return inp, ctx, om


@pytest.mark.parametrize("precision,rtol", [("f64", 1e-12), ("f32", 2e-6)])
def test_tables_of_the_initial_state(precision, rtol):
    cfg = small(30011, precision)
    inp, ctx, om = start(cfg)
    check_tables(ctx, cfg["potential"], om, inp["ics"], inp["w"], rtol)


@pytest.mark.parametrize("nsteps", [1, 3])
def test_fp64_steps_match_oracle(nsteps):
    cfg = small(20000, "f64")
    inp, ctx, om = start(cfg)
    st = m2m.m2m_step(ctx, nsteps)[0]
    ost = om.run(nsteps)[-1]
    tol = 1e-10
    np.testing.assert_allclose(m2m.m2m_weights(ctx), om.w, rtol=tol)
    np.testing.assert_allclose(m2m.m2m_particles(ctx), om.ics(), rtol=tol, atol=tol)
    for k, name in enumerate(["chi2", "chi2_inst", "S", "F", "sum_w", "min_w", "sum_w2"]):
        assert st[name] == pytest.approx(ost[k], rel=tol, abs=1e-12 if name == "S" else 1e-300), name
    check_tables(ctx, cfg["potential"], om, om.ics(), om.w, 1e-11, ics_gpu=m2m.m2m_particles(ctx))
    obs = m2m.m2m_observables(ctx, 0)
    np.testing.assert_allclose(obs["y"], om.observe(), rtol=1e-9, atol=1e-18)
    assert m2m.m2m_step_index(ctx) == nsteps


@pytest.mark.parametrize("launch", [None, {"threads": 256, "ilp": 2, "blocks_per_cu": 2}])
def test_fp32_single_step(launch):
    cfg = small(40007, "f32")
    inp, ctx, om = start(cfg, launch)
    st = m2m.m2m_step(ctx, 1)[0]
    ost = om.run(1)[-1]
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=2e-6)
    xg = m2m.m2m_particles(ctx).astype(np.float64)
    xo = om.ics()
    np.testing.assert_allclose(xg, xo, rtol=2e-6, atol=2e-6 * np.abs(xo).max())
    assert st["chi2"] == pytest.approx(ost[0], rel=1e-6)
    assert st["sum_w"] == pytest.approx(ost[4], rel=1e-6)
    check_tables(ctx, cfg["potential"], om, xo, om.w, 2e-5, ics_gpu=xg)
    obs = m2m.m2m_observables(ctx, 0)
    y1 = om.observe()
    amb = H.edge_distance(cfg["layout"], xo) < 1e-5
    scale = H.moment_scale(cfg, xo, om.w)
    wk = np.max(np.abs(om.w[amb]) * (1 + np.sum(xo[3:5, amb] ** 2, axis=0))) if amb.any() else 0.0
    H.compare_observables(obs["y"], y1, scale, int(amb.sum()), wk, 1e-6)


def test_fp32_ten_steps_chi2():
    """Ten FP32 steps: chi^2 within 1e-4 of the FP64 oracle; the weights within 1e-5
    except for at most 0.1% of the particles (those whose FP32 bin or cell decision
    fell on the other side of an edge in some step: each such flip moves ln w by at
    most 2 eps dt max|G| <= 0.2)."""
    cfg = small(30000, "f32")
    inp, ctx, om = start(cfg)
    st = m2m.m2m_step(ctx, 10)[0]
    ost = om.run(10)[-1]
    assert st["chi2"] == pytest.approx(ost[0], rel=1e-4)
    err = np.abs(np.log(m2m.m2m_weights(ctx).astype(np.float64) / om.w))
    H.flush("ten steps: |ln w| error median %.3g p99.9 %.3g max %.3g" % (
        np.median(err), np.percentile(err, 99.9), err.max()))
    assert np.mean(err > 1e-5) <= 1e-3
    assert err.max() <= 0.2


def test_frozen_model_keeps_particles_and_tables():
    cfg = small(5000, "f64")
    cfg["frozen"] = True
    inp, ctx, om = start(cfg)
    m2m.m2m_step(ctx, 2)
    om.run(2)
    np.testing.assert_array_equal(m2m.m2m_particles(ctx), inp["ics"])
    np.testing.assert_allclose(m2m.m2m_weights(ctx), om.w, rtol=1e-11)
    # neither side rebuilds the tables of a frozen model: those of the initial state
    check_tables(ctx, cfg["potential"], om, inp["ics"], inp["w"], 1e-12)


def test_full_size_one_step():
    """The multipole workload at full size (2^23 particles, FP32): one step against
    the oracle's whole step -- every weight, every coordinate, chi^2 and the node
    tables of the new state."""
    cfg = configs.cfg3()
    inp, ctx, om = start(cfg)
    st = m2m.m2m_step(ctx, 1)[0]
    H.flush("gpu step done; oracle step")
    ost = om.run(1)[-1]
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=2e-6)
    xg = m2m.m2m_particles(ctx).astype(np.float64)
    xo = om.ics()
    np.testing.assert_allclose(xg, xo, rtol=2e-6, atol=2e-6 * np.abs(xo).max())
    assert st["chi2"] == pytest.approx(ost[0], rel=1e-6)
    check_tables(ctx, cfg["potential"], om, xo, om.w, 2e-5, ics_gpu=xg)


@pytest.mark.parametrize("precision,lmax,nodes,period", [("f64", 4, 50, 1), ("f32", 4, 50, 3), ("f32", 8, 120, 2)])
def test_other_expansions_and_prior_periods(precision, lmax, nodes, period):
    """Other truncations and node counts (the terms above lmax stay zero in the
    tables), and a histogram prior refreshed every P steps: weights and tables
    after three steps against the oracle."""
    cfg = small(20011, precision)
    cfg["potential"] = dict(cfg["potential"], lmax=lmax, nodes=nodes)
    cfg["prior"] = dict(cfg["prior"], period=period)
    inp, ctx, om = start(cfg)
    m2m.m2m_step(ctx, 3)
    om.run(3)
    f64 = precision == "f64"
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=1e-10 if f64 else 1e-5)
    xg = m2m.m2m_particles(ctx).astype(np.float64)
    check_tables(ctx, cfg["potential"], om, om.ics(), om.w, 1e-11 if f64 else 4e-5, ics_gpu=xg)
