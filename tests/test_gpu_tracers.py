"""GPU parity of the discrete-velocity likelihood (paper section 1: PNe
velocities among the data; reading: each tracer's likelihood is the model's
line-of-sight velocity density at its velocity in its bin, lambda times the
summed log joins the merit function) against the FP64 oracle, through the C ABI.

Workload: the cfg 1 model (Hernquist potential, moving (E, L/Lc) prior, shells
and annuli) with discrete tracers drawn from its Osipkov-Merritt target and binned
in the annuli.  Bars as for the binned data: FP64 1e-11 after 1-2 steps and 1e-8
after 50 (weights, chi^2, log-likelihood and the smoothed sums); FP32 one step
1e-6; FP32 end of run (200 steps) chi^2 and log-likelihood within 1e-3.
"""
import numpy as np
import pytest

from synth import configs
from tests import helpers as H
from tests.golden import derive_eps

pytestmark = pytest.mark.gpu

m2m = pytest.importorskip("paper_1207_6403_amd")


def setup(N, T, precision, lam=1.0):
    cfg = configs.cfg_pne(N=N, n_tracers=T, precision=precision, lam=lam)
    cfg["eps"] = 0.1 / (cfg["dt"] * derive_eps.max_abs_G(cfg))
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case tracers %s N=%d T=%d eps %.3g" % (precision, N, T, cfg["eps"]))
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    (om,) = H.oracle_models(cfg, inp, er)
    return cfg, inp, ctx, om


def oracle_now(cfg, om, first):
    """The oracle's smoothed sums and log-likelihood of its current state (the one
    the GPU holds after the same number of steps)."""
    L, M = om.tracer_observe()
    if not first:
        g = cfg["dt"] / cfg["tau"]
        L = om.arr["tL"][:L.size] + g * (L - om.arr["tL"][:L.size])
        M = om.arr["tM"] + g * (M - om.arr["tM"])
    ll = np.sum(np.log(L / M[cfg["tracers"]["bin"]]))
    return ll, L, M


def nbins(cfg):
    return len(cfg["layout"]["binnings"][cfg["tracers"]["binning"]]["edges"]) - 1


@pytest.mark.parametrize("nsteps", [0, 1, 2, 50])
def test_fp64_matches_oracle(nsteps):
    cfg, inp, ctx, om = setup(5000, 300, "f64")
    if nsteps:
        st = m2m.m2m_step(ctx, nsteps)[0]
        ost = om.run(nsteps)[-1]
        tol = 1e-11 if nsteps <= 2 else 1e-8
        np.testing.assert_allclose(m2m.m2m_weights(ctx), om.w, rtol=tol)
        assert st["chi2"] == pytest.approx(ost[0], rel=tol)
    else:
        tol = 1e-12
    ll, L, M = m2m.m2m_tracer_state(ctx, nbins(cfg))
    oll, oL, oM = oracle_now(cfg, om, nsteps == 0)
    H.flush("loglike GPU %.12g oracle %.12g" % (ll, oll))
    assert ll == pytest.approx(oll, rel=tol)
    np.testing.assert_allclose(L, oL, rtol=max(tol, 1e-12))
    np.testing.assert_allclose(M, oM, rtol=max(tol, 1e-12))


def test_fp32_single_step():
    cfg, inp, ctx, om = setup(50000, 2000, "f32")
    st = m2m.m2m_step(ctx, 1)[0]
    ost = om.run(1)[-1]
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=1e-6)
    assert st["chi2"] == pytest.approx(ost[0], rel=1e-6)
    ll, L, M = m2m.m2m_tracer_state(ctx, nbins(cfg))
    oll, oL, oM = oracle_now(cfg, om, False)
    H.flush("loglike GPU %.10g oracle %.10g" % (ll, oll))
    assert ll == pytest.approx(oll, rel=1e-6)
    np.testing.assert_allclose(L, oL, rtol=1e-5)


def test_fp32_end_of_run():
    cfg, inp, ctx, om = setup(20000, 1000, "f32")
    st = m2m.m2m_step(ctx, 200)[0]
    ost = om.run(200)[-1]
    ll = m2m.m2m_tracer_state(ctx, nbins(cfg))[0]
    oll = oracle_now(cfg, om, False)[0]
    H.flush("200 steps: chi2 GPU %.8g oracle %.8g; loglike GPU %.8g oracle %.8g" % (st["chi2"], ost[0], ll, oll))
    assert st["chi2"] == pytest.approx(ost[0], rel=1e-3)
    assert ll == pytest.approx(oll, rel=1e-3)


def test_likelihood_term_raises_the_likelihood():
    """The same run with and without the likelihood term (lambda 1 and 0): with it,
    the tracers' log-likelihood ends higher."""
    lls = []
    for lam in (0.0, 1.0):
        cfg, inp, ctx, om = setup(20000, 1000, "f32", lam=lam)
        m2m.m2m_step(ctx, 500)
        lls.append(m2m.m2m_tracer_state(ctx, nbins(cfg))[0])
    H.flush("loglike after 500 steps: lambda 0 %.6g, lambda 1 %.6g" % tuple(lls))
    assert lls[1] > lls[0]


def test_tracer_arguments_checked():
    cfg = configs.cfg_pne(N=1000, n_tracers=50)
    inp = H.inputs(cfg)
    plain = {k: v for k, v in cfg.items() if k != "tracers"}
    ctx = m2m.m2m_create(plain, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    tr = cfg["tracers"]
    for bad in (dict(tr, binning=5), dict(tr, bin=np.full(len(tr["bin"]), 99)), dict(tr, dv=np.zeros(len(tr["v"])), h=0.0)):
        with pytest.raises(m2m.M2MError) as e:
            m2m.m2m_set_tracers(ctx, bad)
        assert e.value.status == 1
    m2m.m2m_step(ctx, 1)
    with pytest.raises(m2m.M2MError) as e:
        m2m.m2m_set_tracers(ctx, tr)
    assert e.value.status == 1
    m2m.m2m_destroy(ctx)
    b4 = configs.cfg4(n_models=2, nmin=500, nmax=600, steps=1)
    inp4 = H.inputs(b4)
    ctx4 = m2m.m2m_create(b4, inp4["ics"], inp4["w"], inp4["Y"], inp4["sigma"])
    with pytest.raises(m2m.M2MError) as e:
        m2m.m2m_set_tracers(ctx4, tr)
    assert e.value.status == 6
    m2m.m2m_destroy(ctx4)
