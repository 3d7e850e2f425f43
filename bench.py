"""Benchmark: particle-steps per second of the fused M2M step on one MI355X.

Workload: the plain method at scale -- N = 2^20 particles in the axisymmetric
logarithmic potential (v0 = 1, Rc = 0.1, q = 0.8), FP32 particle arithmetic,
64x64 sky pixels plus 20x20 kinematic bins (first and second LOS moments,
J = 4896 observables), moving (E, Lz/Lc) prior on 32x32 cells refreshed every
step, dt = 0.005.  One step = weight update + leapfrog push + observe + smoothing,
deviations, chi^2 and prior cell means, all on the GPU.

Prints one JSON line (see the keys below).  The timed region starts with the
particles resident in HBM; each fused step kernel is bracketed by HIP events on
the context's stream, which gives the roofline figure.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--n N] [--no-cpu-baseline]
    python bench.py --copy-calibration MIB   # plain device copy, for HBM counter scaling
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_PARTICLE_STEP = 56      # read x y z vx vy vz w (7 x 4 B), write the same
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, inp, er, nsteps):
    """The FP64 oracle, as it is, on the host cores: a bounded sample of the workload."""
    import oracle
    m = oracle.Model(cfg, inp["ics"].astype(np.float64), inp["w"].astype(np.float64), inp["Y"], inp["sigma"],
                     Erange=tuple(er))
    t0 = time.perf_counter()
    st = m.run(nsteps)
    dt = time.perf_counter() - t0
    return {"value": cfg["N"] * nsteps / dt, "unit": "particle-steps/s", "cores": oracle.threads(),
            "kind": "oracle", "sample": "N=%d particles x %d steps of the same workload (%.1f s)" % (cfg["N"], nsteps, dt)}, st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device 10 times (the reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 10}))
        return

    import paper_1207_6403_amd as m2m
    from synth import configs

    cfg = configs.cfg2(N=args.n)
    log("generating inputs (N=%d)" % args.n)
    inp = configs.make_inputs(cfg, dtype=np.float32)
    # prior energy grid: [min E(0), max E(0)] in the model potential, from the synthetic model
    from synth import galaxy  # noqa: F401
    dev = torch.device("cuda:0")
    xv = torch.from_numpy(np.ascontiguousarray(inp["ics"])).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(inp["w"])).to(dev)
    ctx = m2m.m2m_create(cfg, xv, w, inp["Y"], inp["sigma"], device_ptrs=True)
    launch = m2m.m2m_get_launch(ctx)
    if not args.no_autotune:
        launch = m2m.m2m_autotune(ctx, 20)
        log("autotuned launch: %s" % launch)
    # timed region: every fused step kernel bracketed by HIP events on the
    # context's stream (direct launches: event records inside a HIP graph cannot
    # be timed)
    m2m.m2m_set_launch(ctx, timing=1, graph_steps=0)
    log("warmup %d steps" % args.warmup)
    m2m.m2m_step(ctx, args.warmup)
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = m2m.m2m_step(ctx, args.steps)[0]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms, k_n = m2m.m2m_kernel_time(ctx)
    # the same steps replayed from HIP graphs of G steps (no per-kernel events)
    graph_value = None
    G = args.graph_steps
    if G:
        steps_g = max(G, args.steps // G * G)
        m2m.m2m_set_launch(ctx, timing=0, graph_steps=G)
        m2m.m2m_step(ctx, 2 * G)   # builds both parities' graphs
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m2m.m2m_step(ctx, steps_g)
        torch.cuda.synchronize()
        graph_value = cfg["N"] * steps_g / (time.perf_counter() - t1)
        log("graph replay: %.3g particle-steps/s" % graph_value)
    value = cfg["N"] * args.steps / wall
    achieved = BYTES_PER_PARTICLE_STEP * cfg["N"] / (k_ms * 1e-3) / 1e9
    log("wall %.3f s, %.2f us/step, fused kernel %.2f us (%d launches)" % (wall, wall / args.steps * 1e6, k_ms * 1e3, k_n))

    # chi^2 relative error against the oracle: one step from the initial state
    er = None
    chi2_err = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        er = oracle.energy_range(cfg, inp["ics"].astype(np.float64))
        ctx2 = m2m.m2m_create(cfg, xv, w, inp["Y"], inp["sigma"], Erange=np.array(er), device_ptrs=True)
        m2m.m2m_set_launch(ctx2, threads=launch["threads"], ilp=launch["ilp"], blocks_per_cu=launch["blocks_per_cu"])
        g1 = m2m.m2m_step(ctx2, 2)[0]
        log("cpu baseline: %d oracle steps of N=%d" % (args.cpu_steps, cfg["N"]))
        cpu, ost = cpu_baseline(cfg, inp, er, args.cpu_steps)
        chi2_err = abs(g1["chi2"] - ost[1][0]) / ost[1][0]
        m2m.m2m_destroy(ctx2)

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
        "config": {"workload": "log-potential M2M at scale: N=%d FP32 particles, J=4896 observables "
                               "(64x64 sky pixels + 20x20 kinematic bins x 2 LOS moments), "
                               "32x32 (E, Lz/Lc) moving prior every step, dt=0.005" % cfg["N"],
                   "N": cfg["N"], "J": 4896, "prior_cells": 1024, "launch": launch},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "step_kernel<float,float,1,ILP>", "kernel_us": k_ms * 1e3,
                     "bytes_per_launch": BYTES_PER_PARTICLE_STEP * cfg["N"]},
        "graph_replay_value": graph_value,
        "chi2_rel_err_vs_oracle": chi2_err,
        "chi2_final": last["chi2"],
        "cpu_baseline": cpu,
    }
    m2m.m2m_destroy(ctx)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
