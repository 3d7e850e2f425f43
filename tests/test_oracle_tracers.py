"""Pins of the oracle's discrete-velocity likelihood (paper section 1: PNe
velocities among the data; reading: each tracer's likelihood is the model's
line-of-sight velocity density at its velocity in its bin, and lambda times the
summed log-likelihood joins the merit function).

  - L_t and M_b against a brute-force restatement (projected radius, bin edges,
    normal density written out here);
  - the update's tracer term equals lambda d(loglike)/dw_i, by central finite
    differences of the log-likelihood of the observed sums (step 0: the smoothed
    sums are the observed ones);
  - lambda = 0 reproduces the run without tracers bit for bit;
  - with frozen particles, weights driven by the likelihood alone (errors so wide
    that chi^2 does not act, no entropy) climb it: the log-likelihood of the
    smoothed sums does not fall over the run.
"""
import numpy as np

import oracle
from synth import configs


def small(N=400, T=40, lam=1.0):
    cfg = configs.cfg_pne(N=N, n_tracers=T, lam=lam)
    inp = configs.make_inputs(cfg)
    return cfg, inp


def brute(cfg, ics, w):
    tr = cfg["tracers"]
    b = cfg["layout"]["binnings"][tr["binning"]]
    e = np.asarray(b["edges"])
    x, y, z, vx, vy, vz = ics
    inc = cfg["layout"]["incl"]
    R = np.hypot(x, y * np.cos(inc) - z * np.sin(inc))
    vl = vy * np.sin(inc) + vz * np.cos(inc)
    k = np.searchsorted(e, R, side="right") - 1
    k[(R < e[0]) | (R >= e[-1])] = -1
    s = np.sqrt(np.asarray(tr["dv"]) ** 2 + tr["h"] ** 2)
    L = np.zeros(len(tr["v"]))
    for t in range(L.size):
        inb = k == tr["bin"][t]
        L[t] = np.sum(w[inb] * np.exp(-0.5 * ((vl[inb] - tr["v"][t]) / s[t]) ** 2) / (np.sqrt(2 * np.pi) * s[t]))
    M = np.array([w[k == j].sum() for j in range(len(e) - 1)])
    return L, M, k


def test_sums_against_brute_force():
    cfg, inp = small()
    m = oracle.Model(cfg, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    L, M = m.tracer_observe()
    Lb, Mb, _ = brute(cfg, inp["ics"], inp["w"])
    np.testing.assert_allclose(L, Lb, rtol=1e-12)
    np.testing.assert_allclose(M, Mb, rtol=1e-12)
    assert np.all(L > 0)


def loglike_of(cfg, ics, w):
    L, M, _ = brute(cfg, ics, w)
    return np.sum(np.log(L / M[cfg["tracers"]["bin"]]))


def test_update_term_is_the_likelihood_gradient():
    cfg, inp = small()
    c = dict(cfg, eps=1e-9, mu=0.0, frozen=True, update="exp")
    c0 = dict(c, tracers=dict(cfg["tracers"], **{"lambda": 0.0}))
    ma = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    mb = oracle.Model(c0, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    w0 = inp["w"].copy()
    ma.run(1)
    mb.run(1)
    lam = cfg["tracers"]["lambda"]
    G = (np.log(ma.w / w0) - np.log(mb.w / w0)) / (c["eps"] * c["dt"])
    assert abs(ma.loglike - loglike_of(cfg, inp["ics"], w0)) < 1e-10 * abs(ma.loglike)
    _, _, k = brute(cfg, inp["ics"], w0)
    picks = [int(np.flatnonzero(k == j)[0]) for j in np.unique(k[k >= 0])[:6]] + [int(np.flatnonzero(k < 0)[0])]
    for i in picks:
        h = 1e-6 * w0[i]
        wp, wm = w0.copy(), w0.copy()
        wp[i] += h
        wm[i] -= h
        fd = (loglike_of(cfg, inp["ics"], wp) - loglike_of(cfg, inp["ics"], wm)) / (2 * h)
        assert abs(G[i] - lam * fd) <= 1e-5 * max(1.0, abs(lam * fd)), (i, G[i], lam * fd)
    assert G[picks[-1]] == 0.0   # a particle outside the tracers' binning


def test_zero_lambda_is_the_plain_run():
    cfg, inp = small()
    c0 = dict(cfg, tracers=dict(cfg["tracers"], **{"lambda": 0.0}))
    plain = {k: v for k, v in cfg.items() if k != "tracers"}
    ma = oracle.Model(c0, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    mb = oracle.Model(plain, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    sa, sb = ma.run(20), mb.run(20)
    np.testing.assert_array_equal(ma.w, mb.w)
    np.testing.assert_array_equal(sa, sb)


def test_likelihood_climbs_when_it_alone_drives_the_weights():
    cfg, inp = small(N=2000, T=200)
    c = dict(cfg, eps=2e-4, mu=0.0, frozen=True)
    m = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], 1e12 * inp["sigma"])
    ll = []
    for _ in range(30):
        m.run(1)
        ll.append(m.loglike)
    ll = np.array(ll)
    assert np.all(np.diff(ll) >= -1e-9 * np.abs(ll[:-1]))
    assert ll[-1] > ll[0] + 0.1
