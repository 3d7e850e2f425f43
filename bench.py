"""Benchmark: particle-steps per second of the M2M step on one MI355X.

Workloads (--workload):
  logpot     the headline: the plain method at scale -- N = 2^20 particles in the
             axisymmetric logarithmic potential (v0 = 1, Rc = 0.1, q = 0.8), FP32,
             64x64 sky pixels plus 20x20 kinematic bins (first and second LOS
             moments, J = 4896), moving (E, Lz/Lc) prior on 32x32 cells every step,
             dt = 0.005;
  batched    64 Hernquist+NFW models, sum N_m ~ 7e7, one launch per step;
  multipole  2^23 particles in their own multipole potential (lmax 8, 200 nodes),
             the logpot observables plus 50 density shells;
  mlp        2^22 particles with the learned prior (refreshed every 100 steps on a
             2^20 sample, judged against a 32x32x8 histogram prior);
  pne        2^20 Hernquist-potential particles with 833 discrete line-of-sight
             velocities (their log-likelihood in the merit function).
One step = weight update + push + observe + smoothing, deviations, chi^2 and
prior, all on the GPU.

Prints one JSON line.  The timed region starts with the particles resident in
HBM; in a second timed region HIP events attached to the dominant kernel's
launches (on the context's stream) take its own start and end times, which give
the roofline figure.

    python bench.py [--workload W] [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
    python bench.py --copy-calibration MIB   # plain device copy, for HBM counter scaling
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_PARTICLE_STEP = 56      # read x y z vx vy vz w (7 x 4 B), write the same
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3           # MI355X vector FP32 (published; packed FP32 counts twice)


def mp_flops_per_particle(lmax=8):
    """Algorithmic FP32 operations (an FMA counts 2) of the multipole
    update/kick/drift kernel per particle: per (l, m >= 0) term 12 to interpolate
    the four node coefficients (a + t (b - a) each), 12 for the potential (the two
    normalised radial combinations P and their sum against Y_lm), 28 for the
    gradient (9 each for the doubled x and y ladder sums, 5 for z, 5 for the radial
    term) and 8 for the harmonic recurrence; per degree l 5 for the radial powers
    and the radial sum; 60 for the set-up of the expansion point, the final
    scaling of the gradient, the weight update, the kick and the drift."""
    terms = (lmax + 1) * (lmax + 2) // 2
    return terms * (12 + 12 + 28 + 8) + (lmax + 1) * 5 + 60


def kernel_sources_sha256():
    """Digest of the sources the fused step kernel is compiled from."""
    h = hashlib.sha256()
    for f in ("step.hip", "particle.h", "device.h", "runtime.h"):
        with open(os.path.join(ROOT, "paper_1207_6403_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n):
    """HBM bytes per launch of the fused kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a plain copy), or None
    when the kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "step_kernel_logpot_N1M_counters.txt")
    if n != 1 << 20 or not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return float(kv["hbm_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    """Model name of the host CPU and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def _oracle_model(cfg, inp, er, sl=None, model=0):
    import oracle
    ics = inp["ics"].astype(np.float64)
    w = inp["w"].astype(np.float64)
    if sl is not None:
        ics, w = ics[:, sl].copy(), w[sl].copy()
    return oracle.Model(cfg, ics, w, inp["Y"], inp["sigma"], Erange=tuple(er), model=model)


def _oracle_run(cfg, m, nsteps):
    import oracle
    from oracle import mlp
    if cfg["prior"]["kind"] == "mlp":
        pr = cfg["prior"]
        lp = mlp.LearnedPrior(pr["mlp_init"], pr["lr"], pr["beta1"], pr["beta2"], pr["adam_eps"], pr["seed"],
                              pr["subset"], pr["batch"], pr["fallback"])
        return mlp.run(m, lp, pr, nsteps, oracle.subset)
    return m.run(nsteps)


def cpu_baseline(cfg, inp, er, nsteps, steps_1core, sl=None, model=0):
    """The FP64 oracle, as it is, on the host cores: a bounded sample of the workload
    on all of them, and a shorter one on one core.  Returns the baseline record, the
    oracle's statistics rows and its model after the all-core sample."""
    import oracle
    cpu_model, ncores = host_cpu()
    n = cfg["N"] if sl is None else sl.stop - sl.start
    m1 = _oracle_model(cfg, inp, er, sl, model)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    _oracle_run(cfg, m1, steps_1core)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(ncores)
    m = _oracle_model(cfg, inp, er, sl, model)
    t0 = time.perf_counter()
    st = _oracle_run(cfg, m, nsteps)
    dt = time.perf_counter() - t0
    what = "N=%d particles" % n if sl is None else "model %d alone (N=%d)" % (model, n)
    rec = {"value": n * nsteps / dt, "unit": "particle-steps/s", "cores": oracle.threads(), "kind": "oracle",
           "sample": "%s x %d steps of the same workload (%.1f s)" % (what, nsteps, dt),
           "value_1core": n * steps_1core / dt1,
           "sample_1core": "%s x %d steps on one core (%.1f s)" % (what, steps_1core, dt1),
           "cpu_model": cpu_model}
    return rec, st, m


def obs_rel_err(cfg, ys_gpu, ys_or):
    """Largest error of the smoothed observables relative to the largest value of
    the same binning and moment."""
    err, j = 0.0, 0
    for b in cfg["layout"]["binnings"]:
        nb = b["nx"] * b["ny"] if b["kind"] == "grid" else len(b["edges"]) - 1
        for _ in b["moments"]:
            o, g = ys_or[j:j + nb], ys_gpu[j:j + nb]
            err = max(err, float(np.max(np.abs(g - o)) / max(np.max(np.abs(o)), 1e-300)))
            j += nb
    return err


def smoothed_next(cfg, om):
    """The oracle's smoothed observables of its current state (those a context holds
    after the same number of steps)."""
    g = cfg["dt"] / cfg["tau"]
    ys = om.arr["ys"]
    return ys + g * (om.observe() - ys)


def batched_checks(m2m, cfg, inp, xv, w, launch, cpu_steps, steps_1core, sample=(0, 31, 63)):
    """Batched workload: the full 64-model run for cpu_steps steps against the oracle
    run on sampled models alone -- the first sampled model for all cpu_steps steps
    (also the oracle's rate), the others for two -- and the chi^2 errors."""
    import oracle
    offs = np.concatenate([[0], np.cumsum(cfg["model_sizes"])])
    ics64 = inp["ics"].astype(np.float64)
    er = []
    for m in range(len(cfg["model_sizes"])):
        er += list(oracle.energy_range(cfg, ics64, slice(offs[m], offs[m + 1]), model=m))
    ctx2 = m2m.m2m_create(cfg, xv, w, inp["Y"], inp["sigma"], Erange=np.array(er), device_ptrs=True)
    m2m.m2m_set_launch(ctx2, threads=launch["threads"], ilp=launch["ilp"], blocks_per_cu=launch["blocks_per_cu"])
    m2m.m2m_step(ctx2, cpu_steps)
    hist = m2m.m2m_history(ctx2)
    m2m.m2m_destroy(ctx2)
    errs, cpu = [], None
    for m in sample:
        sl = slice(int(offs[m]), int(offs[m + 1]))
        if cpu is None:
            cpu, rows, _ = cpu_baseline(cfg, inp, er[2 * m:2 * m + 2], cpu_steps, steps_1core, sl=sl, model=m)
            n = cpu_steps - 1
        else:
            rows = _oracle_model(cfg, inp, er[2 * m:2 * m + 2], sl, m).run(2)
            n = 1
        g = [r for r in hist if r["model"] == m and r["step"] == n][0]
        errs.append(abs(g["chi2"] - rows[n][0]) / rows[n][0])
        log("model %d: chi2 step %d GPU %.10g oracle %.10g" % (m, n, g["chi2"], rows[n][0]))
    return cpu, errs


WORKLOADS = {
    "logpot": ("log-potential M2M at scale: N=%d FP32 particles, J=4896 observables (64x64 sky pixels "
               "+ 20x20 kinematic bins x 2 LOS moments), 32x32 (E, Lz/Lc) moving prior every step, dt=0.005"),
    "batched": ("64 Hernquist+NFW models (halo mass ratio x scale radius grid), sum N_m=%d FP32 particles, "
                "30 shells + 20 annuli (LOS second moment) per model, (E, L/Lc) 20x20 moving prior per "
                "model every step, dt=0.01, one launch per step for all models"),
    "multipole": ("self-consistent multipole model: N=%d FP32 particles, lmax=8 at 200 log-spaced nodes "
                  "rebuilt every step, J=4896 + 50 density shells, 32x32 (E, Lz/Lc) prior in the analytic "
                  "log potential every step, dt=0.005"),
    "mlp": ("learned prior: N=%d FP32 particles in the log potential, 3-64-64-1 network retrained every 100 "
            "steps on a 2^20 sample (128 Adam minibatches of 8192), judged against a 32x32x8 (E, L/Lc, Lz/L) "
            "histogram prior, J=4896, dt=0.005"),
    "pne": ("discrete-velocity likelihood: N=%d FP32 particles in the Hernquist potential, 30 shells + 20 "
            "annuli (LOS second moment), the line-of-sight velocities of the 833 of 1000 drawn tracers that "
            "fall in the annuli (lambda=1, kernel width 0.071), (E, L/Lc) 20x20 moving prior every step, dt=0.01"),
}
# oracle steps of the CPU sample: about 10-15 s on 16 host threads
DEFAULT_CPU_STEPS = {"logpot": 96, "batched": 220, "multipole": 6, "mlp": 150, "pne": 20}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=1 << 20, help="particles of the logpot workload")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="logpot",
                    help="logpot (the headline), batched, multipole, mlp or pne (discrete velocities)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0, help="oracle steps of the CPU baseline (0: per workload)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate launch shapes first (the default shape is the tuned one)")
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--inputs-cache", default="", metavar="DIR",
                    help="keep the generated inputs in DIR and reuse them (repeated profiler runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 60 times (the reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters, and its bandwidth at that footprint) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(each model's particles would shard over GPUs with an all-reduce of the partial "
              "histograms per step); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(50):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 50
        print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 60, "ms_per_copy": ms,
                          "read_plus_write_GBps": 2 * 4 * n / (ms * 1e-3) / 1e9}))
        return

    import paper_1207_6403_amd as m2m
    from synth import configs

    wl = args.workload
    batched = wl == "batched"
    cfg = {"logpot": lambda: configs.cfg2(N=args.n), "batched": configs.cfg4, "multipole": configs.cfg3,
           "mlp": configs.cfg5,
           "pne": lambda: dict(configs.cfg_pne(N=args.n, n_tracers=1000, precision="f32"), eps=configs.EPS_PNE)}[wl]()
    cpu_steps = args.cpu_steps or DEFAULT_CPU_STEPS[wl]
    cache = os.path.join(args.inputs_cache, "%s_%d.npz" % (wl, cfg["N"])) if args.inputs_cache else None
    if cache and os.path.exists(cache):
        log("loading inputs (N=%d) from %s" % (cfg["N"], cache))
        with np.load(cache) as z:
            inp = {k: z[k] for k in ("ics", "w", "Y", "sigma")}
    else:
        log("generating inputs (N=%d)" % cfg["N"])
        inp = configs.make_inputs(cfg, dtype=np.float32)
        if cache:
            os.makedirs(args.inputs_cache, exist_ok=True)
            np.savez(cache, **inp)
    dev = torch.device("cuda:0")
    xv = torch.from_numpy(np.ascontiguousarray(inp["ics"])).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(inp["w"])).to(dev)
    ctx = m2m.m2m_create(cfg, xv, w, inp["Y"], inp["sigma"], device_ptrs=True)
    launch = m2m.m2m_get_launch(ctx)
    if args.autotune:
        launch = m2m.m2m_autotune(ctx, 20)
        log("autotuned launch: %s" % launch)
    log("warmup %d steps" % args.warmup)
    m2m.m2m_step(ctx, args.warmup)
    torch.cuda.synchronize()

    # timed region 1 (the throughput): K steps as the library runs them, from
    # HIP graphs of G steps each where the step sequence allows (both step
    # parities' graphs built beforehand)
    # (graphs hold an even number of steps, at most K, so that K steps replay whole
    # graphs where K allows)
    G = min(args.graph_steps, args.steps - args.steps % 2) if args.steps >= 2 else 0
    m2m.m2m_set_launch(ctx, timing=0, graph_steps=G)
    if G:
        m2m.m2m_step(ctx, 2 * G)
    torch.cuda.synchronize()
    log("timing %d steps (graphs of %d)" % (args.steps, G))
    t0 = time.perf_counter()
    last = m2m.m2m_step(ctx, args.steps)[0]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = cfg["N"] * args.steps / wall

    # timed region 2 (the roofline): the same K steps launched one by one, HIP
    # events attached to the dominant kernel's launches on the context's stream
    m2m.m2m_set_launch(ctx, timing=1, graph_steps=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    m2m.m2m_step(ctx, args.steps)
    torch.cuda.synchronize()
    wall_ev = time.perf_counter() - t1
    k_ms, k_n = m2m.m2m_kernel_time(ctx)
    if wl == "multipole":
        flops = mp_flops_per_particle() * cfg["N"]
        achieved = flops / (k_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                "kernel": "mp_kick_kernel (second kick: the l <= 8 field from the node tables in LDS, stored for "
                          "the next step's first kick)",
                "kernel_us": k_ms * 1e3, "flops_per_launch": flops}
    else:
        # (the learned prior, or the tracers' term of G, is read per particle)
        bpp = BYTES_PER_PARTICLE_STEP + (4 if wl in ("mlp", "pne") else 0)
        achieved = bpp * cfg["N"] / (k_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(cfg["N"]) if wl == "logpot" else None,
                "kernel": "step_kernel (fused update + push + observe + prior cells)",
                "kernel_us": k_ms * 1e3, "bytes_per_launch": bpp * cfg["N"]}
    roof["timing"] = ("HIP events attached to each of %d one-by-one launches (the kernel's own start and end)"
                      % k_n)
    log("throughput: %.2f us/step (%.3g particle-steps/s); one by one: %.2f us/step, dominant kernel %.2f us (%d launches)"
        % (wall / args.steps * 1e6, value, wall_ev / args.steps * 1e6, k_ms * 1e3, k_n))

    # chi^2 (and the smoothed observables) against the oracle at the end of the
    # oracle's CPU sample: a second context from the same initial state runs the
    # same number of steps
    chi2_err = None
    parity = None
    cpu = None
    steps_1core = max(1, cpu_steps // 16)
    if batched and not args.no_cpu_baseline:
        cpu, errs = batched_checks(m2m, cfg, inp, xv, w, launch, cpu_steps, steps_1core)
        chi2_err = errs[0]
        parity = {"chi2_rel_err_model0_end_of_sample": errs[0], "chi2_rel_err_sampled_models_step1": errs[1:],
                  "steps": cpu_steps}
    elif not args.no_cpu_baseline:
        import oracle
        er = oracle.energy_range(cfg, inp["ics"].astype(np.float64))
        ctx2 = m2m.m2m_create(cfg, xv, w, inp["Y"], inp["sigma"], Erange=np.array(er), device_ptrs=True)
        m2m.m2m_set_launch(ctx2, threads=launch["threads"], ilp=launch["ilp"], blocks_per_cu=launch["blocks_per_cu"])
        g_last = m2m.m2m_step(ctx2, cpu_steps)[0]
        ys_gpu = m2m.m2m_observables(ctx2, 0)["y_smooth"]
        trc = cfg.get("tracers")
        if trc:
            nb = len(cfg["layout"]["binnings"][trc["binning"]]["edges"]) - 1
            ll_gpu = m2m.m2m_tracer_state(ctx2, nb)[0]
        m2m.m2m_destroy(ctx2)
        log("cpu baseline: %d oracle steps of N=%d (and %d on one core)" % (cpu_steps, cfg["N"], steps_1core))
        cpu, ost, om = cpu_baseline(cfg, inp, er, cpu_steps, steps_1core)
        chi2_err = abs(g_last["chi2"] - ost[-1][0]) / ost[-1][0]
        parity = {"steps": cpu_steps, "chi2_rel_err": chi2_err,
                  "obs_max_rel_err": obs_rel_err(cfg, ys_gpu, smoothed_next(cfg, om))}
        if trc:
            # the oracle's tracer log-likelihood of its current state (smoothed sums)
            g = cfg["dt"] / cfg["tau"]
            L, M = om.tracer_observe()
            L = om.arr["tL"][:L.size] + g * (L - om.arr["tL"][:L.size])
            M = om.arr["tM"] + g * (M - om.arr["tM"])
            ll = float(np.sum(np.log(L / M[trc["bin"]])))
            parity["loglike_rel_err"] = abs(ll_gpu - ll) / abs(ll)
        log("parity after %d steps: chi2 %.3g, smoothed observables %.3g" % (
            cpu_steps, chi2_err, parity["obs_max_rel_err"]))

    config = {"workload": WORKLOADS[wl] % cfg["N"], "N": cfg["N"], "launch": launch}
    if batched:
        config.update(models=len(cfg["model_sizes"]), J=50, prior_cells=400)
    elif wl == "pne":
        config.update(J=50, prior_cells=400, tracers=len(cfg["tracers"]["v"]))
    else:
        config.update(J=4946 if wl == "multipole" else 4896,
                      prior_cells=8192 if wl == "mlp" else 1024)
    graphs = G and (cfg["prior"]["kind"] == "flat" or cfg["prior"].get("period", 1) == 1)
    replayed = (args.steps // G) * G if graphs else 0
    out = {
        "metric": "particle-steps/sec at 1M particles (push+observe+update); chi2 rel. err vs oracle",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
        "roofline": roof,
        "timing": {"value": ("%d steps: %d replayed from HIP graphs of %d steps, %d launched one by one"
                             % (args.steps, replayed, G, args.steps - replayed)) if graphs
                   else "%d steps launched one by one (the step sequence changes between refreshes)" % args.steps,
                   "one_by_one_value": cfg["N"] * args.steps / wall_ev,
                   "one_by_one_ms_per_step": wall_ev / args.steps * 1e3},
        "chi2_rel_err_vs_oracle": chi2_err,
        "parity_vs_oracle": parity,
        "chi2_final": last["chi2"],
        "cpu_baseline": cpu,
    }
    m2m.m2m_destroy(ctx)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
