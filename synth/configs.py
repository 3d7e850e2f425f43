"""The five synthetic workloads and their reduced-size variants.

Each configuration is a plain dict that both the HIP path and the CPU oracle read:

  N, precision ("f64" | "f32"), potential (dict, or a list of dicts when batched),
  model_sizes (batched only), layout (see ``synth.targets``), prior (dict),
  dt, eps, mu, tau, steps, seeds.

``make_inputs(cfg)`` draws the initial particle model and the noisy target and
returns a dict of float64 numpy arrays: ics [6, N], w [N], Y [J], sigma [J].
Weights start at 1/N (per model when batched), as in paper section 2.1.
"""
import numpy as np

from . import galaxy, targets
from .galaxy import seed_for

DEG = np.pi / 180.0


def _log_edges(lo, hi, n):
    return np.geomspace(lo, hi, n + 1)


def layout_cfg1():
    """30 log shells in r over [0.05, 20] (mass) + 20 log annuli in R over [0.1, 10]
    (second LOS moment); line of sight along z."""
    return {"incl": 0.0, "binnings": [
        {"kind": "shell", "edges": _log_edges(0.05, 20.0, 30), "moments": (0,)},
        {"kind": "annulus", "edges": _log_edges(0.1, 10.0, 20), "moments": (2,)},
    ]}


def layout_cfg2():
    """64x64 sky pixels over [-5,5]^2 (mass) + 20x20 kinematic bins over [-2,2]^2
    (first and second LOS moments), inclination 60 degrees."""
    return {"incl": 60.0 * DEG, "binnings": [
        {"kind": "grid", "nx": 64, "ny": 64, "x0": -5.0, "x1": 5.0, "y0": -5.0, "y1": 5.0,
         "moments": (0,)},
        {"kind": "grid", "nx": 20, "ny": 20, "x0": -2.0, "x1": 2.0, "y0": -2.0, "y1": 2.0,
         "moments": (1, 2)},
    ]}


def layout_cfg3():
    lay = layout_cfg2()
    lay["binnings"].append({"kind": "shell", "edges": _log_edges(0.05, 10.0, 50), "moments": (0,)})
    return lay


LOG_POT = {"kind": "log", "v0": 1.0, "Rc": 0.1, "q": 0.8}
HERN_POT = {"kind": "hernquist", "G": 1.0, "M": 1.0, "a": 1.0}


def cfg1(N=20000, steps=2000):
    return {"name": "hernquist_fp64_N%d" % N, "index": 1, "N": N, "precision": "f64",
            "potential": dict(HERN_POT), "layout": layout_cfg1(),
            "prior": {"kind": "hist", "axes": ("E", "L/Lc"), "shape": (20, 20), "period": 1},
            "dt": 0.01, "eps": 1e-3, "mu": 1e-2, "tau": 0.5, "steps": steps,
            "target": {"kind": "hernquist_om", "ra": 1.0, "noise": 0.05}}


def cfg2(N=1 << 20, steps=5000, target_n=1 << 23):
    return {"name": "log_fp32_N%d" % N, "index": 2, "N": N, "precision": "f32",
            "potential": dict(LOG_POT), "layout": layout_cfg2(),
            "prior": {"kind": "hist", "axes": ("E", "Lz/Lc"), "shape": (32, 32), "period": 1},
            "dt": 0.005, "eps": EPS_CFG2, "mu": 5e-3, "tau": 0.5, "steps": steps,
            "target": {"kind": "log_rotating", "n": target_n, "rot_frac": 0.8, "noise": 0.03}}


def cfg3(N=1 << 23, steps=2000, target_n=1 << 23):
    c = cfg2(N, steps, target_n)
    c.update({"name": "multipole_fp32_N%d" % N, "index": 3, "layout": layout_cfg3(),
              "potential": {"kind": "multipole", "G": 1.0, "lmax": 8, "nodes": 200,
                            "rmin": 1e-3, "rmax": 100.0, "Mtot": LOG_MASS_R10},
              "eps": EPS_CFG3})
    # prior cells measured in the analytic potential the particles were drawn from
    c["prior"] = dict(c["prior"], ref_potential=dict(LOG_POT))
    return c


def cfg4(n_models=64, nmin=100_000, nmax=2_000_000, steps=3000):
    rng = np.random.default_rng(seed_for(4, 3))
    sizes = rng.integers(nmin, nmax + 1, n_models)
    ratio = np.linspace(0.0, 10.0, 8)
    rs = np.linspace(1.0, 10.0, 8)
    pots = []
    for m in range(n_models):
        pots.append({"kind": "hernquist_nfw", "G": 1.0, "M": 1.0, "a": 1.0,
                     "Mh": float(ratio[(m // 8) % 8]), "rs": float(rs[m % 8])})
    return {"name": "batched_hnfw_%dmodels" % n_models, "index": 4, "N": int(sizes.sum()),
            "model_sizes": sizes.astype(np.int64), "precision": "f32", "potential": pots,
            "layout": layout_cfg1(),
            "prior": {"kind": "hist", "axes": ("E", "L/Lc"), "shape": (20, 20), "period": 1},
            "dt": 0.01, "eps": EPS_CFG4, "mu": 1e-2, "tau": 0.5, "steps": steps,
            "target": {"kind": "hernquist_om", "ra": 1.0, "noise": 0.05, "seed_cfg": 1}}


def layout_cfg2_gh():
    """The cfg 2 layout plus the kinematic grid again with the Gauss-Hermite moments
    h3 and h4 (integral-field kinematics); the bins' Gaussians (V_b, sigma_b) come
    from the target (filled in by make_inputs)."""
    lay = layout_cfg2()
    kin = dict(lay["binnings"][1])
    kin.update(moments=(5, 6), gh=None)
    lay["binnings"].append(kin)
    return lay


def cfg2gh(N=1 << 20, steps=5000, target_n=1 << 23):
    """Log-potential model fitted to surface density, v, v^2 and Gauss-Hermite h3,
    h4 of a rotating target (errors 3% on density and velocities, 0.01 on h_m)."""
    c = cfg2(N, steps, target_n)
    c.update({"name": "log_gh_fp32_N%d" % N, "index": 6, "layout": layout_cfg2_gh()})
    c["target"] = dict(c["target"], noise_gh=0.01, seed_cfg=2)
    return c


def layout_fig1():
    """The cfg 1 shells, and the annuli with the second moment and the
    Gauss-Hermite h3, h4 about the target's own dispersion (V_b = 0: non-rotating)."""
    lay = layout_cfg1()
    lay["binnings"][1] = dict(lay["binnings"][1], moments=(2, 5, 6), gh=None, gh_zero_mean=True)
    return lay


def cfg_fig1(N=20000, steps=2000, ics="isotropic", target_n=None, precision="f64", noise=0.01, noise_gh=0.005):
    """The convergence experiment of the paper's Fig. 1: the cfg 1 model (Hernquist
    potential, moving (E, L/Lc) priors) fitted to idealised line-of-sight data of
    an Osipkov-Merritt r_a = 1 target -- shell masses, and per annulus v^2, h3 and
    h4 -- with errors `noise` (masses, dispersions) and `noise_gh` (h_m), no noise
    drawn.  The data are the model's exact moments (target_n None) or those of a
    realisation of target_n particles.  Initial particle models 'isotropic',
    'radial' (Osipkov-Merritt r_a = 0.6) or 'tangential' (beta = -1/2)."""
    c = cfg1(N, steps)
    c.update({"name": "fig1_%s_N%d" % (ics, N), "index": 7, "layout": layout_fig1(), "precision": precision,
              "ics": ics})
    if target_n is None:
        c["target"] = {"kind": "hernquist_om_exact", "ra": 1.0, "noise": noise, "noise_gh": noise_gh, "draw": False}
    else:
        c["target"] = {"kind": "hernquist_om_realisation", "ra": 1.0, "n": target_n, "noise": noise,
                       "noise_gh": noise_gh, "draw": False}
    return c


def cfg_fig1_run(ics, prior="moving", eps=None):
    """One fit of the Fig. 1 experiment as run on the GPU: 2^21 particles (FP32) of
    the initial model `ics`, exact target data with errors 0.3% (masses,
    dispersions) and 0.0015 (h_m), entropy weight mu = 1e3 with the moving (E,
    L/Lc) prior or constant priors (prior="flat"), 150,000 steps; eps from
    EPS_FIG1 (eps dt max|G(0)| = 3) unless given."""
    c = cfg_fig1(N=1 << 21, steps=150_000, ics=ics, precision="f32", noise=0.003, noise_gh=0.0015)
    c.update({"name": "fig1_%s_%s" % (ics, prior), "mu": 1e3, "eps": EPS_FIG1[ics] if eps is None else eps})
    if prior == "flat":
        c["prior"] = {"kind": "flat"}
    return c


_PNE_CACHE = {}


def _pne_tracers(n, dv):
    """(bin, v) of n tracers drawn from the 2^20-particle Osipkov-Merritt
    realisation (memoised: the realisation takes seconds)."""
    if (n, dv) not in _PNE_CACHE:
        if "real" not in _PNE_CACHE:
            _PNE_CACHE["real"] = galaxy.hernquist_om_ics(1 << 20, seed_for(1, 8), 1.0)
        _PNE_CACHE[(n, dv)] = targets.discrete_tracers(layout_cfg1(), 1, _PNE_CACHE["real"], n, dv, seed_for(1, 9))
    return _PNE_CACHE[(n, dv)]


def cfg_pne(N=20000, steps=2000, n_tracers=2000, precision="f64", lam=1.0, dv=0.05, h=0.05):
    """Discrete line-of-sight velocities (planetary-nebula-like tracers) added to
    the cfg 1 model: n_tracers drawn from a 2^20-particle realisation of its
    Osipkov-Merritt target, each binned in the annuli (binning 1) with a velocity
    error dv; kernel width sqrt(dv^2 + h^2); weight lam of the log-likelihood in
    the merit function."""
    c = cfg1(N, steps)
    c.update({"name": "pne_%s_N%d_T%d" % (precision, N, n_tracers), "precision": precision})
    b, v = _pne_tracers(n_tracers, dv)
    c["tracers"] = {"binning": 1, "bin": b, "v": v, "dv": np.full(b.size, dv), "h": h, "lambda": lam}
    return c


def mlp_init(seed):
    """Initial parameters of the 3-64-64-1 prior network (FP32): weights normal
    with variance 1/fan-in, biases zero; W1[64,3], b1, W2[64,64], b2, W3[1,64], b3."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0.0, 1.0 / np.sqrt(3.0), (64, 3)), np.zeros(64), rng.normal(0.0, 1.0 / 8.0, (64, 64)),
             np.zeros(64), rng.normal(0.0, 1.0 / 8.0, (1, 64)), np.zeros(1)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def cfg5(N=1 << 22, steps=5000, target_n=1 << 23):
    c = cfg2(N, steps, target_n)
    seed = seed_for(5, 2)
    c.update({"name": "mlp_prior_fp32_N%d" % N, "index": 5,
              "prior": {"kind": "mlp", "axes": ("E", "L/Lc", "Lz/L"), "shape": (32, 32, 8),
                        "period": 100, "hidden": 64, "subset": 1 << 20, "batch": 8192,
                        "lr": 1e-3, "beta1": 0.9, "beta2": 0.999, "adam_eps": 1e-8,
                        "fallback": 0.5, "seed": seed, "mlp_init": mlp_init(seed), "mfma": True},
              "eps": EPS_CFG2})
    return c


# Values fixed once from the initial state so that eps*dt*max_i |G_i(0)| <= 0.1;
# written by tests/golden/derive_eps.py, which calls only the oracle.
EPS_CFG2 = 1.8e-6
EPS_CFG3 = 1.85e-6
# The 64-model batch shares one rate: the maximum of |G(0)| over its models at
# their full sizes (1.1e8, from the halo-heavy models' outer shells).
EPS_CFG4 = 8.98e-8
# The discrete-velocity workload (cfg_pne at 2^20 particles, 1000 tracers, FP32).
EPS_PNE = 7.04e-05
# The Fig. 1 runs (cfg_fig1_run), one rate per initial model.
EPS_FIG1 = {"isotropic": 7.448e-06, "radial": 2.764e-05, "tangential": 6.088e-06}
# Mass of the truncated (r <= 10) logarithmic-potential density: the self-consistent
# form weights its particles by w_i * Mtot (galaxy.log_mass_within_sphere()).
LOG_MASS_R10 = 9.999142073415042


_TARGET_CACHE = {}


def _layout_key(lay):
    return repr({"incl": lay["incl"], "binnings": [{k: v for k, v in b.items() if k != "gh"}
                                                   for b in lay["binnings"]]})


def cached_target(cfg):
    """make_target(cfg), memoised on the target recipe and the layout (with the
    Gauss-Hermite parameters it fills into the layout)."""
    key = (cfg["index"], repr(cfg["target"]), _layout_key(cfg["layout"]))
    if key not in _TARGET_CACHE:
        _TARGET_CACHE[key] = make_target(cfg)
    Y, sigma, gh = _TARGET_CACHE[key]
    for b, g in zip(cfg["layout"]["binnings"], gh):
        if g is not None:
            b["gh"] = g
    return Y, sigma


def make_inputs(cfg, dtype=np.float64, cache_target=True):
    """Initial particle model, weights 1/N (per model), noisy target."""
    idx = cfg["index"]
    seed = seed_for(idx)
    pot = cfg["potential"]
    if "model_sizes" in cfg:
        parts, ws = [], []
        for m, (n, p) in enumerate(zip(cfg["model_sizes"], pot)):
            parts.append(galaxy.hernquist_nfw_ics(int(n), seed + 7 * m, p["G"], p["M"], p["a"],
                                                  p["Mh"], p["rs"]))
            ws.append(np.full(int(n), 1.0 / int(n)))
        ics = np.concatenate(parts, axis=1)
        w = np.concatenate(ws)
    elif pot["kind"] == "hernquist":
        kind = cfg.get("ics", "isotropic")
        if kind == "isotropic":
            ics = galaxy.hernquist_isotropic_ics(cfg["N"], seed, pot["G"], pot["M"], pot["a"])
        elif kind == "radial":
            ics = galaxy.hernquist_om_ics(cfg["N"], seed + 3, 0.6)
        elif kind == "tangential":
            ics = galaxy.hernquist_tangential_ics(cfg["N"], seed + 4)
        else:
            raise ValueError("unknown initial model %r" % kind)
        w = np.full(cfg["N"], 1.0 / cfg["N"])
    else:
        lp = LOG_POT
        ics = galaxy.log_isotropic_ics(cfg["N"], seed, lp["v0"], lp["Rc"], lp["q"])
        w = np.full(cfg["N"], 1.0 / cfg["N"])
    if cache_target:
        Y, sigma = cached_target(cfg)
    else:
        Y, sigma, gh = make_target(cfg)
        for b, g in zip(cfg["layout"]["binnings"], gh):
            if g is not None:
                b["gh"] = g
    return {"ics": ics.astype(dtype), "w": w.astype(dtype), "Y": Y.copy(), "sigma": sigma.copy()}


def make_target(cfg):
    """(Y, sigma, gh): the noisy target and, per binning, the Gauss-Hermite
    parameters (V_b, sigma_b) measured from the target (None for binnings without
    Gauss-Hermite moments)."""
    t = cfg["target"]
    lay = cfg["layout"]
    sidx = t.get("seed_cfg", cfg["index"])
    gh = [None] * len(lay["binnings"])
    if t["kind"] == "hernquist_om":
        Yt, Mb = targets.hernquist_om_target(lay, ra=t["ra"])
    elif t["kind"] == "hernquist_om_exact":
        Yt, Mb, gh = targets.hernquist_om_exact_target(lay, ra=t["ra"])
    else:
        if t["kind"] == "hernquist_om_realisation":
            real = galaxy.hernquist_om_ics(t["n"], seed_for(sidx, 5), t["ra"])
        else:
            lp = LOG_POT
            real = galaxy.log_isotropic_ics(t["n"], seed_for(sidx, 5), lp["v0"], lp["Rc"], lp["q"])
            real = galaxy.make_rotating(real, t["rot_frac"], seed_for(sidx, 6))
        for ib, b in enumerate(lay["binnings"]):
            if any(m >= 3 for m in b["moments"]):
                gh[ib] = targets.gh_parameters(b, real, lay["incl"], zero_mean=b.get("gh_zero_mean", False))
                b["gh"] = gh[ib]
        Yt, Mb = targets.observe_realisation(lay, real, 1.0 / t["n"])
    Y, sigma = targets.add_noise(lay, Yt, Mb, t["noise"], seed_for(sidx, 1), f_gh=t.get("noise_gh"))
    if not t.get("draw", True):
        Y = Yt   # idealised data: the errors are given, no noise is drawn
    return Y, sigma, gh
