"""GPU parity of the learned moving prior (section 2.1: priors over integrals of
motion that follow the weight distribution; learned form) against the FP64
oracle's refresh schedule, through the C ABI.

Bars: the GPU trains in FP32 (features from FP64 integrals of motion, FP32
network and Adam) and the oracle in FP64 on the same sample:
  parameters after a refresh within 2e-5 absolute plus 1e-3 relative (Adam
    normalises each step to about lr, so FP32 gradient noise moves a parameter
    by at most a few lr * 1e-5);
  priors within 1e-4 relative, the judge within 1e-4 relative and the same
    fallback decision;
  weights after the step within 2e-6 relative (the FP32 update bar of the
    fused kernel, widened by the priors' error through mu dt eps).
"""
import numpy as np
import pytest

import oracle
from oracle import mlp
from synth import configs
from tests import helpers as H
from tests.golden import derive_eps

pytestmark = pytest.mark.gpu

m2m = pytest.importorskip("paper_1207_6403_amd")


def setup(N, subset, batch, period, fallback=0.5, target_n=1 << 16, full=False):
    cfg = configs.cfg5() if full else configs.cfg5(N=N, target_n=target_n)
    cfg["prior"].update(subset=subset, batch=batch, period=period, fallback=fallback)
    if not full:
        # the rate of a small model, derived as for the full-size workloads:
        # eps dt max|G(0)| = 0.1 (G is far larger when few particles meet the target)
        cfg["eps"] = 0.1 / (cfg["dt"] * derive_eps.max_abs_G(cfg))
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case %s N=%d subset=%d batch=%d period=%d fallback=%g" % (cfg["name"], cfg["N"], subset, batch,
                                                                      period, fallback))
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    (om,) = H.oracle_models(cfg, inp, er)
    pr = cfg["prior"]
    lp = mlp.LearnedPrior(pr["mlp_init"], pr["lr"], pr["beta1"], pr["beta2"], pr["adam_eps"], pr["seed"],
                          pr["subset"], pr["batch"], pr["fallback"])
    return cfg, ctx, om, lp


def compare(ctx, om, lp, what_rtol=1e-4):
    st = m2m.m2m_mlp_state(ctx)
    dth = np.abs(st["theta"].astype(np.float64) - lp.theta)
    H.flush("theta: max |d| %.3g, judge GPU %.8g oracle %.8g, fallback GPU %s oracle %s" % (
        dth.max(), st["judge"], lp.last_judge, st["used_fallback"], lp.used_fallback))
    assert np.all(dth <= 2e-5 + 1e-3 * np.abs(lp.theta))
    assert st["judge"] == pytest.approx(lp.last_judge, rel=1e-4)
    assert st["used_fallback"] == lp.used_fallback
    what, _ = m2m.m2m_priors(ctx)
    err = np.abs(what.astype(np.float64) / om.arr["what"] - 1)
    H.flush("priors: max rel err %.3g" % err.max())
    assert err.max() <= what_rtol
    return st


def test_one_refresh_and_step():
    cfg, ctx, om, lp = setup(20011, 4096, 512, 4)
    m2m.m2m_step(ctx, 1)
    mlp.run(om, lp, cfg["prior"], 1, oracle.subset)
    st = compare(ctx, om, lp)
    assert st["refreshes"] == 1
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=2e-6)


def test_three_refreshes():
    """Steps 0..8 with period 4: refreshes at steps 0, 4 and 8, Adam state carried over."""
    cfg, ctx, om, lp = setup(12007, 2048, 256, 4)
    m2m.m2m_step(ctx, 9)
    mlp.run(om, lp, cfg["prior"], 9, oracle.subset)
    st = compare(ctx, om, lp, what_rtol=3e-4)
    assert st["refreshes"] == 3
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=1e-5)


def test_learned_priors_without_fallback():
    """A threshold no judge reaches: the network's priors are used and compared."""
    cfg, ctx, om, lp = setup(20011, 4096, 512, 3, fallback=1e9)
    m2m.m2m_step(ctx, 4)
    mlp.run(om, lp, cfg["prior"], 4, oracle.subset)
    st = compare(ctx, om, lp)
    assert not st["used_fallback"] and st["refreshes"] == 2
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=1e-5)


def test_zero_threshold_falls_back_to_the_histogram_prior():
    cfg, ctx, om, lp = setup(8000, 1024, 256, 2, fallback=0.0)
    m2m.m2m_step(ctx, 1)
    mlp.run(om, lp, cfg["prior"], 1, oracle.subset)
    st = compare(ctx, om, lp, what_rtol=2e-6)
    assert st["used_fallback"]


def test_full_size_refresh():
    """The learned-prior workload at full size: 2^22 particles, a sample of 2^20 in
    128 minibatches of 8192; one refresh and step, with a threshold no judge
    reaches so that the network's priors are the ones compared (the fallback path
    is covered at small sizes)."""
    cfg, ctx, om, lp = setup(0, 1 << 20, 8192, 100, fallback=1e9, full=True)
    m2m.m2m_step(ctx, 1)
    H.flush("gpu step done; oracle refresh")
    mlp.run(om, lp, cfg["prior"], 1, oracle.subset)
    compare(ctx, om, lp, what_rtol=3e-4)
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=2e-6)
