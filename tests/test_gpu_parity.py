"""GPU parity of the fused M2M step (C ABI, HIP path) against the FP64 oracle.

Bars:
  FP64 path: every output within 1e-11 relative of the oracle after one step and
             within 1e-8 after 50 steps (rounding order only).
  FP32 path: one step -- weights and coordinates within 1e-6 relative (coordinates
             absolute 1e-6 * scale), observables within 1e-6 of sum |w K| except bins
             explained by particles within 1e-5 of a bin edge, chi^2 within 1e-6
             relative; end of run -- chi^2 within 1e-3, every bin within
             max(1e-3, 3 x the spread of an oracle run started one FP32 ulp away).
  Batched FP32 path: weights within max(2e-6, 6e-7 L), L the largest total change
             of a log-weight over the run (sum over steps of |ln w_n+1 / w_n|): the
             FP32 update exponent carries a relative error of a few ulp, so each
             step's error in ln w is ~6e-8 times a small multiple of its change.
"""
import numpy as np
import pytest

import oracle
from synth import configs
from tests import helpers as H
from tests.golden import derive_eps

pytestmark = pytest.mark.gpu

m2m = pytest.importorskip("paper_1207_6403_amd")


def run_both(cfg, nsteps, launch=None, er=None):
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp) if er is None else er
    H.flush("case %s N=%d steps=%d launch=%s" % (cfg["name"], cfg["N"], nsteps, launch))
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    if launch:
        m2m.m2m_set_launch(ctx, **launch)
    ors = H.oracle_models(cfg, inp, er)
    return inp, ctx, ors


def test_prologue_observables_fp64():
    cfg = configs.cfg1(N=3000)
    inp, ctx, (om,) = run_both(cfg, 0)
    obs = m2m.m2m_observables(ctx, 0)
    y0 = om.observe()
    np.testing.assert_allclose(obs["y"], y0, rtol=1e-12, atol=1e-18)
    np.testing.assert_array_equal(obs["y_smooth"], obs["y"])
    chi2 = np.sum(((y0 - inp["Y"]) / inp["sigma"]) ** 2)
    assert obs["chi2"] == pytest.approx(chi2, rel=1e-12)
    what, cells = m2m.m2m_priors(ctx)
    o_what, o_cs, o_cn = om.prior_means()
    np.testing.assert_allclose(what, o_what, rtol=1e-12)
    np.testing.assert_allclose(cells[0], np.where(o_cn > 0, o_cs / np.maximum(o_cn, 1), 0), rtol=1e-12)


@pytest.mark.parametrize("nsteps", [1, 2, 50])
def test_cfg1_fp64_matches_oracle(nsteps):
    cfg = configs.cfg1(N=5000)
    inp, ctx, (om,) = run_both(cfg, nsteps)
    st = m2m.m2m_step(ctx, nsteps)[0]
    ost = om.run(nsteps)[-1]
    tol = 1e-11 if nsteps <= 2 else 1e-8
    np.testing.assert_allclose(m2m.m2m_weights(ctx), om.w, rtol=tol)
    np.testing.assert_allclose(m2m.m2m_particles(ctx), om.ics(), rtol=tol, atol=tol)
    for k, name in enumerate(["chi2", "chi2_inst", "S", "F", "sum_w", "min_w", "sum_w2"]):
        # S(0) = 0 exactly (w = what); its rounding noise is ~1e-16 of sum w |ln w|
        assert st[name] == pytest.approx(ost[k], rel=tol, abs=1e-12 if name == "S" else 1e-300), name
    assert st["step"] == nsteps - 1
    # the context already observed the state of step nsteps; the oracle observes it
    # at the start of its next step
    obs = m2m.m2m_observables(ctx, 0)
    y_next = om.observe()
    np.testing.assert_allclose(obs["y"], y_next, rtol=max(tol, 1e-10), atol=1e-18)
    assert m2m.m2m_step_index(ctx) == nsteps


def test_fp32_bin_reduction_bound():
    """The FP32 path's observables of the initial state (no step: the same FP32
    coordinates on both sides, every bin decision exact) at the benchmark size and
    launch shape.  Each block sums its particles' w K in FP64 in LDS and rounds the
    sum to FP32 once in its partial slot; the slots are added in FP64.  So a mass
    bin (K = 1, w exact) is off by at most 2^-24 of sum |w K|, and a moment bin
    adds the FP32 rounding of K itself (v_los from one fused multiply-add, then
    its square: a few units of 2^-24)."""
    from synth import targets
    cfg = configs.cfg2()
    inp, ctx, (om,) = run_both(cfg, 0, launch={"threads": 1024, "ilp": 1, "blocks_per_cu": 1})
    y = m2m.m2m_observables(ctx, 0)["y"]
    yo = om.observe()
    scale = H.moment_scale(cfg, om.ics(), om.w)
    mom = np.array([k[0] for k in targets.observable_kinds(cfg["layout"])])
    err = np.abs(y - yo) / np.maximum(scale, 1e-300)
    H.flush("initial-state observables, error / sum |w K|: mass %.3g, v %.3g, v^2 %.3g" % (
        err[mom == 0].max(), err[mom == 1].max(), err[mom == 2].max()))
    u = 2.0 ** -24
    assert err[mom == 0].max() <= 1.0 * u
    assert err[mom == 1].max() <= 3.0 * u
    assert err[mom == 2].max() <= 5.0 * u


def test_cfg2_fp32_single_step():
    cfg = configs.cfg2(N=50000)
    inp, ctx, (om,) = run_both(cfg, 1)
    m2m.m2m_step(ctx, 1)
    om.run(1)
    wg = m2m.m2m_weights(ctx).astype(np.float64)
    np.testing.assert_allclose(wg, om.w, rtol=1e-6)
    xg = m2m.m2m_particles(ctx).astype(np.float64)
    xo = om.ics()
    np.testing.assert_allclose(xg, xo, rtol=1e-6, atol=1e-6 * np.abs(xo).max())
    obs = m2m.m2m_observables(ctx, 0)
    y1 = om.observe()
    amb = H.edge_distance(cfg["layout"], xo) < 1e-5
    scale = H.moment_scale(cfg, xo, om.w)
    wk = np.max(np.abs(om.w[amb]) * (1 + np.sum(xo[3:5, amb] ** 2, axis=0))) if amb.any() else 0.0
    H.compare_observables(obs["y"], y1, scale, int(amb.sum()), wk, 1e-6)


@pytest.mark.parametrize("launch", [{"threads": 256, "ilp": 1, "blocks_per_cu": 1},
                                    {"threads": 1024, "ilp": 2, "blocks_per_cu": 1},
                                    {"threads": 512, "ilp": 2, "blocks_per_cu": 4}])
def test_cfg2_fp32_launch_shapes_agree(launch):
    """Ragged tiles (N = 40,007 is not a multiple of any tile) in several launch shapes."""
    cfg = configs.cfg2(N=40007)
    inp, ctx, (om,) = run_both(cfg, 3, launch=launch)
    st = m2m.m2m_step(ctx, 3)[0]
    ost = om.run(3)[-1]
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=2e-6)
    assert st["chi2"] == pytest.approx(ost[0], rel=2e-6)
    assert st["S"] == pytest.approx(ost[2], rel=1e-4, abs=1e-9)
    assert st["sum_w"] == pytest.approx(ost[4], rel=1e-6)


def smoothed_next(cfg, om):
    """Oracle smoothed observables of its current state (those the context holds)."""
    g = cfg["dt"] / cfg["tau"]
    ys = om.arr["ys"]
    return ys + g * (om.observe() - ys)


def one_particle_share(layout, ics, w, scale):
    """Per observable, the largest |w_i K_ij| of one particle over sum_i |w_i K_ij|."""
    big = np.zeros(scale.size)
    for i in range(w.size):
        for j, K in oracle.kernel_entries(layout, ics[:, i]):
            big[j] = max(big[j], abs(w[i] * K))
    return big / np.maximum(scale, 1e-300)


def end_of_run(cfg, nsteps, launch=None):
    """Run the GPU path and the oracle nsteps from the same inputs (and, when some
    bin differs by more than 1e-3, a second oracle run whose initial coordinates
    are one FP32 ulp away: the spread that FP32 coordinates alone cause in an
    orbit integration of this length).
    Asserts chi^2 within 1e-3 of the oracle's, and every bin's smoothed
    observable within max(1e-3, 3 x the largest one-ulp spread) of the scale
    sum |w K| of its bin, or, in a bin beyond that, within twice the largest
    share of one particle in it; returns the errors."""
    inp, ctx, (om,) = run_both(cfg, nsteps, launch=launch)
    st = m2m.m2m_step(ctx, nsteps)[0]
    ost = om.run(nsteps)[-1]
    obs = m2m.m2m_observables(ctx, 0)
    ys_o = smoothed_next(cfg, om)
    scale = H.moment_scale(cfg, om.ics(), om.w)
    big = scale > 1e-3 * scale.max()
    err = np.abs(obs["y_smooth"] - ys_o)[big] / scale[big]
    chi_err = abs(st["chi2"] - ost[0]) / ost[0]
    floor = None
    if err.max() > 1e-3:
        # only needed when the bins are not all within 1e-3
        ulp = H.oracle_models(cfg, dict(inp, ics=np.nextafter(inp["ics"], np.float32(np.inf))),
                              H.erange(cfg, inp))[0]
        ulp.run(nsteps)
        floor = np.abs(smoothed_next(cfg, ulp) - ys_o)[big] / scale[big]
    H.flush("%s N=%d %d steps: chi2 GPU %.8g oracle %.8g rel %.3g; bins max %.3g p99 %.3g; one-ulp floor %s" % (
        cfg["name"], cfg["N"], nsteps, st["chi2"], ost[0], chi_err, err.max(), np.percentile(err, 99),
        "not needed" if floor is None else "max %.3g p99 %.3g" % (floor.max(), np.percentile(floor, 99))))
    assert chi_err <= 1e-3
    bound = max(1e-3, 0.0 if floor is None else 3 * floor.max())
    if err.max() > bound:
        # sparse bins: one particle on the other side of an edge moves the bin by its
        # own share of sum |w K| (the orbits of FP32 and FP64 coordinates part in time)
        share = one_particle_share(cfg["layout"], om.ics(), om.w, scale)[big]
        over = err > bound
        H.flush("%d bins beyond %.3g, each within twice its largest one-particle share: %s" % (
            over.sum(), bound, np.all(err[over] <= 2 * share[over])))
        assert np.all(err[over] <= 2 * share[over])
    m2m.m2m_destroy(ctx)
    return chi_err, err, floor


def test_cfg2_fp32_end_of_run():
    """200 steps of N = 2e4."""
    end_of_run(configs.cfg2(N=20000), 200)


def test_cfg2_fp32_end_of_run_full_size():
    """The benchmark's 2^20 particles in its launch shape, 500 steps."""
    end_of_run(configs.cfg2(), 500, launch={"threads": 1024, "ilp": 1, "blocks_per_cu": 1})


def test_cfg3_multipole_end_of_run():
    """The self-consistent multipole model, 2^18 particles, 200 steps (its rate derived
    at this size as for the full workload)."""
    cfg = configs.cfg3(N=1 << 18)
    cfg["eps"] = 0.1 / (cfg["dt"] * derive_eps.max_abs_G(cfg))
    end_of_run(cfg, 200)


def test_cfg5_learned_prior_end_of_run():
    """The learned prior, 2^18 particles, 300 steps (three refreshes)."""
    cfg = configs.cfg5(N=1 << 18)
    cfg["eps"] = 0.1 / (cfg["dt"] * derive_eps.max_abs_G(cfg))
    end_of_run(cfg, 300)


def test_cfg1_fp64_full_run_chi2():
    """cfg 1 at its full size and length (N = 20,000, 2000 steps): chi^2 of the FP64 GPU
    path within 1e-6 of the oracle, the final weights within 1e-6."""
    cfg = configs.cfg1()
    inp, ctx, (om,) = run_both(cfg, 2000)
    st = m2m.m2m_step(ctx, 2000)[0]
    ost = om.run(2000)[-1]
    assert st["chi2"] == pytest.approx(ost[0], rel=1e-6)
    np.testing.assert_allclose(m2m.m2m_weights(ctx), om.w, rtol=1e-6)


def test_cfg2_full_size_one_step():
    """N = 2^20 in the benchmark's launch shape: one step against the oracle."""
    cfg = configs.cfg2()
    inp, ctx, (om,) = run_both(cfg, 1, launch={"threads": 1024, "ilp": 1, "blocks_per_cu": 1})
    st = m2m.m2m_step(ctx, 1)[0]
    ost = om.run(1)[-1]
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=1e-6)
    assert st["chi2"] == pytest.approx(ost[0], rel=1e-6)
    obs = m2m.m2m_observables(ctx, 0)
    chi2_next = np.sum(((smoothed_next(cfg, om) - inp["Y"]) / inp["sigma"]) ** 2)
    assert obs["chi2"] == pytest.approx(chi2_next, rel=1e-6)


def test_nonpositive_weight_keeps_last_state():
    cfg = configs.cfg1(N=2000)
    cfg.update(update="euler", eps=1.0)
    inp, ctx, (om,) = run_both(cfg, 1)
    with pytest.raises(m2m.M2MError) as e:
        m2m.m2m_step(ctx, 3)
    assert e.value.status == 4
    assert m2m.m2m_step_index(ctx) == 0
    np.testing.assert_array_equal(m2m.m2m_weights(ctx), inp["w"])
    with pytest.raises(m2m.M2MError):
        m2m.m2m_step(ctx, 1)


def test_batched_models_match_oracle():
    cfg = configs.cfg4(n_models=5, nmin=1500, nmax=6000, steps=4)
    cfg["eps"] = 1e-3   # small models: the cfg-1 rate keeps the weights positive and moves them visibly
    inp, ctx, ors = run_both(cfg, 4, launch={"threads": 256, "ilp": 2, "blocks_per_cu": 1})
    rows = m2m.m2m_step(ctx, 4)
    offs = np.concatenate([[0], np.cumsum(cfg["model_sizes"])])
    wg = m2m.m2m_weights(ctx).astype(np.float64)
    for m, om in enumerate(ors):
        L = np.zeros(om.w.size)
        for n in range(4):
            w0 = om.w.copy()
            ost = om.run(1)[-1]
            L += np.abs(np.log(om.w / w0))
        tol = max(2e-6, 6e-7 * L.max())
        H.flush("model %d: largest total |d ln w| %.3g, bar %.3g, error %.3g" % (
            m, L.max(), tol, np.max(np.abs(wg[offs[m]:offs[m + 1]] / om.w - 1))))
        np.testing.assert_allclose(wg[offs[m]:offs[m + 1]], om.w, rtol=tol)
        assert rows[m]["chi2"] == pytest.approx(ost[0], rel=tol)
        assert rows[m]["model"] == m


@pytest.mark.parametrize("prec,period,nsteps,tol", [("f64", 3, 7, 1e-11), ("f32", 4, 9, 5e-6)])
def test_periodic_hist_prior(prec, period, nsteps, tol):
    """Histogram prior refreshed every P > 1 steps (priors stored per particle between
    refreshes): weights, chi^2 and S against the oracle across several refreshes."""
    cfg = configs.cfg1(N=3000) if prec == "f64" else configs.cfg2(N=30000)
    cfg["prior"] = dict(cfg["prior"], period=period)
    inp, ctx, (om,) = run_both(cfg, nsteps)
    m2m.m2m_step(ctx, nsteps)
    orows = om.run(nsteps)
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=tol)
    hist = m2m.m2m_history(ctx)
    assert [r["step"] for r in hist] == list(range(nsteps))
    for r, o in zip(hist, orows):
        assert r["chi2"] == pytest.approx(o[0], rel=tol)
        # S is a sum of terms of both signs (S(0) = 0): compare it on the scale of sum w |ln w|
        assert r["S"] == pytest.approx(o[2], abs=tol * 30.0 * o[4])


@pytest.mark.parametrize("period,nsteps", [(1, 4), (3, 7)])
def test_large_hist_prior_cells_apart(period, nsteps):
    """A 32x32x8 (E, L/Lc, Lz/L) histogram prior next to the 4896 observables (more
    than the fused kernel's LDS holds): the cells are summed by their own kernel and
    the priors gathered before each step.  Weights, chi^2 and the priors against the
    oracle at the FP32 bar of the periodic prior."""
    cfg = configs.cfg2(N=30000)
    cfg["prior"] = {"kind": "hist", "axes": ("E", "L/Lc", "Lz/L"), "shape": (32, 32, 8), "period": period}
    inp, ctx, (om,) = run_both(cfg, nsteps)
    m2m.m2m_step(ctx, nsteps)
    orows = om.run(nsteps)
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=5e-6)
    for r, o in zip(m2m.m2m_history(ctx), orows):
        assert r["chi2"] == pytest.approx(o[0], rel=5e-6)
    # priors of the next step: the oracle's cell means of the current state
    what, cells = m2m.m2m_priors(ctx)
    if (nsteps % period) == 0:
        o_what = om.prior_means()[0]
        np.testing.assert_allclose(what.astype(np.float64), o_what, rtol=5e-6)


def test_batched_full_size_sampled_models():
    """The 64-model batch at its full size (sum N_m ~ 67M, one launch per step, the
    benchmark's launch shape): chi^2 and weights of sampled models after two steps
    against the oracle run on each of those models alone."""
    cfg = configs.cfg4()
    H.flush("case batched 64 models N=%d: generating inputs" % cfg["N"])
    inp = configs.make_inputs(cfg, dtype=np.float32)
    er = H.erange(cfg, inp)
    offs = np.concatenate([[0], np.cumsum(cfg["model_sizes"])])
    H.flush("case batched 64 models N=%d: create + 2 steps" % cfg["N"])
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    m2m.m2m_step(ctx, 2)
    hist = m2m.m2m_history(ctx)
    wg = m2m.m2m_weights(ctx)
    assert len(hist) == 2 * 64
    for m in (0, 17, 63):
        sl = slice(offs[m], offs[m + 1])
        om = oracle.Model(cfg, inp["ics"][:, sl].astype(np.float64), inp["w"][sl].astype(np.float64), inp["Y"],
                          inp["sigma"], Erange=tuple(er[2 * m:2 * m + 2]), model=m)
        rows = om.run(2)
        for n in (0, 1):
            g = [r for r in hist if r["model"] == m and r["step"] == n][0]
            assert g["chi2"] == pytest.approx(rows[n][0], rel=2e-6), (m, n)
            assert g["sum_w"] == pytest.approx(rows[n][4], rel=1e-6), (m, n)
        np.testing.assert_allclose(wg[sl].astype(np.float64), om.w, rtol=2e-6)


def test_frozen_entropy_recurrence_gpu():
    """Frozen particles, one prior cell, chi^2 off: w_n = w_0 exp(-eps dt mu n) (FP64)."""
    cfg = configs.cfg1(N=700)
    cfg.update(frozen=True, eps=0.05, mu=0.5)
    cfg["prior"] = {"kind": "hist", "axes": ("E", "L/Lc"), "shape": (1, 1), "period": 1}
    inp = H.inputs(cfg)
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], np.full(50, 1e300), Erange=np.array([-1.0, 0.0]))
    m2m.m2m_step(ctx, 40)
    a = cfg["eps"] * cfg["dt"] * cfg["mu"]
    np.testing.assert_allclose(m2m.m2m_weights(ctx), np.exp(-a * 40) / 700, rtol=1e-13)


def test_single_particle_and_empty_bins():
    """N = 1 (one ragged tile, most bins empty) in FP32 and FP64."""
    for prec in ("f64", "f32"):
        cfg = configs.cfg1(N=1)
        cfg["precision"] = prec
        ics = np.array([[0.3], [0.1], [0.2], [0.1], [-0.2], [0.3]])
        w = np.array([1.0])
        inp = configs.make_inputs(configs.cfg1(N=10))
        ctx = m2m.m2m_create(cfg, ics, w, inp["Y"], inp["sigma"], Erange=np.array([-1.0, 0.0]))
        st = m2m.m2m_step(ctx, 2)[0]
        om = oracle.Model(cfg, ics, w, inp["Y"], inp["sigma"], Erange=(-1.0, 0.0))
        ost = om.run(2)[-1]
        tol = 1e-11 if prec == "f64" else 2e-6
        assert st["chi2"] == pytest.approx(ost[0], rel=tol)
        np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=tol)


def test_graphs_match_direct_launches():
    cfg = configs.cfg2(N=30000)
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    a = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    b = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    m2m.m2m_set_launch(b, graph_steps=8)
    sa = m2m.m2m_step(a, 21)[0]
    sb = m2m.m2m_step(b, 21)[0]
    assert sb["step"] == sa["step"] == 20
    np.testing.assert_allclose(m2m.m2m_weights(b), m2m.m2m_weights(a), rtol=1e-6)
    assert sb["chi2"] == pytest.approx(sa["chi2"], rel=1e-6)
    hist = m2m.m2m_history(b)
    assert [r["step"] for r in hist] == list(range(21))


def test_autotune_restores_state():
    cfg = configs.cfg2(N=30000)
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    a = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    m2m.m2m_step(a, 2)
    w_before = m2m.m2m_weights(a).copy()
    chosen = m2m.m2m_autotune(a, 3)
    assert chosen["threads"] in (256, 512, 1024)
    np.testing.assert_array_equal(m2m.m2m_weights(a), w_before)
    assert m2m.m2m_step_index(a) == 2
    m2m.m2m_step(a, 1)
