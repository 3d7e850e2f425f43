"""Shared helpers of the GPU parity tests: run the same seeded workload through the
C ABI (HIP path) and through the oracle, and compare with the bars stated in each
test.  The oracle decides in FP64; the FP32 path decides bins and cells in FP32, so
a particle within a few FP32 ulp of a bin or cell edge may legitimately land on
either side (such particles are counted, not ignored)."""
import sys

import numpy as np

import oracle
from synth import configs


def flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def inputs(cfg):
    inp = configs.make_inputs(cfg)
    if cfg["precision"] == "f32":
        inp["ics"] = inp["ics"].astype(np.float32)
        inp["w"] = inp["w"].astype(np.float32)
    return inp


def erange(cfg, inp):
    if cfg["prior"]["kind"] == "flat":
        return None
    if "model_sizes" in cfg:
        offs = np.concatenate([[0], np.cumsum(cfg["model_sizes"])])
        er = []
        for m in range(len(cfg["model_sizes"])):
            er += list(oracle.energy_range(cfg, inp["ics"].astype(np.float64), slice(offs[m], offs[m + 1]), model=m))
        return np.array(er)
    return np.array(oracle.energy_range(cfg, inp["ics"].astype(np.float64)))


def oracle_models(cfg, inp, er):
    """One oracle Model per model of the configuration (FP64 copies of the inputs)."""
    ics = inp["ics"].astype(np.float64)
    w = inp["w"].astype(np.float64)
    if "model_sizes" not in cfg:
        return [oracle.Model(cfg, ics, w, inp["Y"], inp["sigma"], Erange=None if er is None else tuple(er))]
    offs = np.concatenate([[0], np.cumsum(cfg["model_sizes"])])
    out = []
    for m in range(len(cfg["model_sizes"])):
        sl = slice(offs[m], offs[m + 1])
        out.append(oracle.Model(cfg, ics[:, sl].copy(), w[sl].copy(), inp["Y"], inp["sigma"],
                                Erange=tuple(er[2 * m:2 * m + 2]), model=m))
    return out


def edge_distance(layout, ics):
    """Smallest relative distance of each particle's binned coordinates to a bin edge."""
    x, y, z, vx, vy, vz = ics.astype(np.float64)
    inc = layout["incl"]
    X, Ys = x, y * np.cos(inc) - z * np.sin(inc)
    d = np.full(x.size, np.inf)
    for b in layout["binnings"]:
        if b["kind"] == "grid":
            for v, lo, hi, n in ((X, b["x0"], b["x1"], b["nx"]), (Ys, b["y0"], b["y1"], b["ny"])):
                f = (v - lo) / (hi - lo) * n
                d = np.minimum(d, np.abs(f - np.round(f)) / n)
        else:
            r = np.sqrt(x * x + y * y + z * z) if b["kind"] == "shell" else np.hypot(X, Ys)
            e = np.asarray(b["edges"])
            k = np.clip(np.searchsorted(e, r), 1, len(e) - 1)
            d = np.minimum(d, np.minimum(np.abs(r - e[k - 1]), np.abs(r - e[k])) / np.maximum(r, 1e-30))
    return d


def compare_observables(y_gpu, y_or, scale, n_ambiguous, wk_max, rtol):
    """Bins agree within rtol * scale (scale = sum |w K| per bin); the bins that do not
    are at most 6 per ambiguous particle and each differs by at most 2 wk_max."""
    bad = np.abs(y_gpu - y_or) > rtol * scale + 1e-300
    nbad = int(bad.sum())
    assert nbad <= 6 * n_ambiguous, "%d bins differ beyond %.1e (ambiguous particles: %d); worst %s" % (
        nbad, rtol, n_ambiguous, np.max(np.abs(y_gpu - y_or) / np.maximum(scale, 1e-300)))
    if nbad:
        assert np.all(np.abs(y_gpu - y_or)[bad] <= 2.0 * wk_max + rtol * scale[bad])
    return nbad


def abs_moment_scale(cfg, ics, w):
    """sum_i |w_i K_j(z_i)| per observable (oracle kernels, FP64)."""
    layout = cfg["layout"]
    m = oracle.Model(dict(cfg, prior={"kind": "flat"}), ics.astype(np.float64), np.abs(w).astype(np.float64),
                     np.zeros(sum_J(layout)), np.ones(sum_J(layout)))
    yabs = m.observe()
    # odd moments: sum |w v| needs |v|; observe with |v_los| by flipping velocities is not
    # possible per bin, so use sqrt(M_b * Y2) >= |sum w v| as the scale for first moments
    return np.abs(yabs)


def sum_J(layout):
    J = 0
    for b in layout["binnings"]:
        nb = len(b["edges"]) - 1 if b["kind"] != "grid" else b["nx"] * b["ny"]
        J += len(b["moments"]) * nb
    return J


def moment_scale(cfg, ics, w):
    """Per-observable magnitude sum_i |w_i K_j| (first moments bounded by sqrt(M_b Y2_b))."""
    layout = cfg["layout"]
    base = abs_moment_scale(cfg, ics, w)
    out = base.copy()
    start = 0
    for b in layout["binnings"]:
        nb = len(b["edges"]) - 1 if b["kind"] != "grid" else b["nx"] * b["ny"]
        mom = list(b["moments"])
        # mass of the binning (moment 0 needs to be computed even if not fitted)
        lay1 = {"incl": layout["incl"], "binnings": [{k: v for k, v in dict(b, moments=(0, 2)).items()
                                                      if k not in ("gh", "gh_zero_mean")}]}
        c1 = dict(cfg, layout=lay1, prior={"kind": "flat"})
        mm = oracle.Model(c1, ics.astype(np.float64), np.abs(w).astype(np.float64), np.zeros(2 * nb), np.ones(2 * nb))
        y = mm.observe()
        M_b, Y2 = y[:nb], y[nb:]
        for k, mo in enumerate(mom):
            if mo == 1:
                out[start + k * nb:start + (k + 1) * nb] = np.sqrt(M_b * Y2)
            elif mo >= 3:
                # Gauss-Hermite kernels: |sqrt(2) exp(-nu^2/2) H_m(nu)| < 1.5
                out[start + k * nb:start + (k + 1) * nb] = 1.5 * M_b
        start += len(mom) * nb
    return out
