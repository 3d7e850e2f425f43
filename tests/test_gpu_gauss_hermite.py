"""GPU parity of the Gauss-Hermite line-of-sight kernels (paper section 1:
absorption-line kinematics from long-slit and integral-field spectra; reading:
each bin's LOSVD expanded about its Gaussian (V_b, sigma_b), van der Marel &
Franx 1993) against the FP64 oracle, through the C ABI.

Workloads: the log-potential model fitted to surface density, v, v^2 and h3, h4
on the kinematic grid (FP32; the layout has no compiled signature, so the generic
kernels run); the spherical Hernquist model fitted to shell masses and v^2, h3,
h4 in annuli (FP64).  Bars as for the other moments: FP64 1e-11 after 1-2 steps,
1e-8 after 50; FP32 one step 1e-6 (weights, chi^2, observables on the scale of
sum |w K|); FP32 end of run (200 steps) chi^2 within 1e-3.
"""
import numpy as np
import pytest

from synth import configs
from tests import helpers as H
from tests.golden import derive_eps

pytestmark = pytest.mark.gpu

m2m = pytest.importorskip("paper_1207_6403_amd")


def _eps(cfg):
    return 0.1 / (cfg["dt"] * derive_eps.max_abs_G(cfg))


def run_both(cfg):
    inp = H.inputs(cfg)
    er = H.erange(cfg, inp)
    H.flush("case %s N=%d J=%d" % (cfg["name"], cfg["N"], inp["Y"].size))
    ctx = m2m.m2m_create(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=er)
    (om,) = H.oracle_models(cfg, inp, er)
    return inp, ctx, om


def test_gh_fp32_single_step():
    cfg = configs.cfg2gh(N=50000, target_n=1 << 20)
    configs.make_inputs(cfg)        # the layout's (V_b, sigma_b) come with the target
    cfg["eps"] = _eps(cfg)
    inp, ctx, om = run_both(cfg)
    st = m2m.m2m_step(ctx, 1)[0]
    ost = om.run(1)[-1]
    np.testing.assert_allclose(m2m.m2m_weights(ctx).astype(np.float64), om.w, rtol=1e-6)
    assert st["chi2"] == pytest.approx(ost[0], rel=1e-6)
    obs = m2m.m2m_observables(ctx, 0)
    y1 = om.observe()
    xo = om.ics()
    amb = H.edge_distance(cfg["layout"], xo) < 1e-5
    scale = H.moment_scale(cfg, xo, om.w)
    wk = np.max(np.abs(om.w[amb]) * (1.5 + np.sum(xo[3:5, amb] ** 2, axis=0))) if amb.any() else 0.0
    H.compare_observables(obs["y"], y1, scale, int(amb.sum()), wk, 1e-6)


@pytest.mark.parametrize("nsteps", [1, 2, 50])
def test_gh_fp64_matches_oracle(nsteps):
    cfg = configs.cfg_fig1(N=5000, target_n=1 << 18, ics="tangential")
    configs.make_inputs(cfg)
    cfg["eps"] = _eps(cfg)
    inp, ctx, om = run_both(cfg)
    st = m2m.m2m_step(ctx, nsteps)[0]
    ost = om.run(nsteps)[-1]
    tol = 1e-11 if nsteps <= 2 else 1e-8
    np.testing.assert_allclose(m2m.m2m_weights(ctx), om.w, rtol=tol)
    assert st["chi2"] == pytest.approx(ost[0], rel=tol)
    np.testing.assert_allclose(m2m.m2m_observables(ctx, 0)["y"], om.observe(), rtol=max(tol, 1e-10), atol=1e-18)


def test_gh_fp32_end_of_run():
    """200 steps of N = 2e4: chi^2 within 1e-3 of the FP64 oracle."""
    cfg = configs.cfg2gh(N=20000, target_n=1 << 20)
    configs.make_inputs(cfg)
    cfg["eps"] = _eps(cfg)
    inp, ctx, om = run_both(cfg)
    st = m2m.m2m_step(ctx, 200)[0]
    ost = om.run(200)[-1]
    H.flush("chi2 GPU %.10g oracle %.10g rel %.3g" % (st["chi2"], ost[0], abs(st["chi2"] - ost[0]) / ost[0]))
    assert st["chi2"] == pytest.approx(ost[0], rel=1e-3)


def test_gh_moments_need_their_gaussians():
    """A Gauss-Hermite binning without (V_b, sigma_b), or with sigma_b <= 0, is
    rejected before any device work."""
    cfg = configs.cfg_fig1(N=200, target_n=1 << 14)
    inp = configs.make_inputs(cfg)
    bad = dict(cfg["layout"]["binnings"][1])
    bad["gh"] = np.array(bad["gh"]) * np.array([[1.0], [0.0]])
    cfg2 = dict(cfg, layout={"incl": 0.0, "binnings": [cfg["layout"]["binnings"][0], bad]})
    with pytest.raises(m2m.M2MError) as e:
        m2m.m2m_create(cfg2, inp["ics"], inp["w"], inp["Y"], inp["sigma"], Erange=np.array([-1.0, 0.0]))
    assert e.value.status == 1
