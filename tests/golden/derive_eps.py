"""Derive the weight-adaptation rate eps of the log-potential workloads.

Reading of the update law: eps is set once from the initial state so that
eps * dt * max_i |G_i(0)| = 0.1, where G_i = dF/dw_i with the priors held fixed.
G_i(0) is read off one oracle step with a negligible rate (w1 = w0 exp(e dt G)).
The batched workload shares one rate over its 64 models: the maximum is taken over
all of them at their full sizes.  Calls only the oracle and the input generators;
prints the values recorded in synth/configs.py (EPS_CFG2, EPS_CFG3, EPS_CFG4,
EPS_PNE of the discrete-velocity workload, and EPS_FIG1 of the Fig. 1 experiment,
whose runs take eps dt max|G(0)| = 3).

    python tests/golden/derive_eps.py
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle  # noqa: E402
from synth import configs  # noqa: E402


def max_abs_G(cfg):
    inp = configs.make_inputs(cfg)
    c = dict(cfg, eps=1e-12, update="exp", frozen=True)
    m = oracle.Model(c, inp["ics"], inp["w"], inp["Y"], inp["sigma"])
    w0 = m.w.copy()
    m.run(1)
    G = np.log(m.w / w0) / (c["eps"] * c["dt"])
    return float(np.max(np.abs(G)))


def max_abs_G_batched(cfg):
    inp = configs.make_inputs(cfg)
    offs = np.concatenate([[0], np.cumsum(cfg["model_sizes"])])
    c = dict(cfg, eps=1e-12, update="exp", frozen=True)
    g = 0.0
    for k in range(len(cfg["model_sizes"])):
        sl = slice(offs[k], offs[k + 1])
        m = oracle.Model(c, inp["ics"][:, sl].copy(), inp["w"][sl].copy(), inp["Y"], inp["sigma"], model=k)
        w0 = m.w.copy()
        m.run(1)
        g = max(g, float(np.max(np.abs(np.log(m.w / w0) / (c["eps"] * c["dt"])))))
    return g


if __name__ == "__main__":
    which = sys.argv[1:] or ["EPS_CFG2", "EPS_CFG3", "EPS_CFG4", "EPS_PNE", "EPS_FIG1"]
    if "EPS_FIG1" in which:
        which.remove("EPS_FIG1")
        # the Fig. 1 runs adapt 30 times faster: eps dt max|G(0)| = 3, per initial model
        for ics in ("isotropic", "radial", "tangential"):
            c = configs.cfg_fig1_run(ics, eps=1.0)
            g = max_abs_G(c)
            print("EPS_FIG1[%r] = %.4e   # max|G(0)| = %.4e" % (ics, float("%.3e" % (3.0 / (c["dt"] * g))), g))
    cases = {"EPS_CFG2": lambda: max_abs_G(configs.cfg2(N=1 << 20)),
             "EPS_CFG3": lambda: max_abs_G(configs.cfg3(N=1 << 20)),
             "EPS_CFG4": lambda: max_abs_G_batched(configs.cfg4()),
             "EPS_PNE": lambda: max_abs_G(configs.cfg_pne(N=1 << 20, n_tracers=1000, precision="f32"))}
    dts = {"EPS_CFG2": configs.cfg2(N=16)["dt"], "EPS_CFG3": configs.cfg3(N=16)["dt"], "EPS_CFG4": 0.01,
           "EPS_PNE": configs.cfg_pne(N=16, n_tracers=16)["dt"]}
    for name in which:
        g = cases[name]()
        cfg = {"dt": dts[name]}
        eps = 0.1 / (cfg["dt"] * g)
        print("%s = %.3e   # max|G(0)| = %.4e" % (name, float("%.2e" % eps), g))
