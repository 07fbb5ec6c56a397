"""Throughput of the PIC-MCC diode hot path on one MI355X.

A step is one pass of the whole hot path for every diode of the workload:
cell re-sort (every K steps), gather + push + absorption + null-collision MCC +
fixed-point deposit, sources (ionisation products, thermionic emission, pair
replenishment), Poisson solve and field.  Inputs are resident in HBM before
the timed region; the metric is live particle-steps per second.

Prints one JSON line.  Options: --gpus (must be 1), --steps, --warmup,
--workload {large,bench,tiny,sweep,paper,paperscan,surrogate} (default large: the 16384-cell,
16.4M-per-species diode, the one configuration whose per-step working set
exceeds the 256 MB last-level cache), --no-cpu-baseline.  --copy-probe BYTES
runs a plain device copy of that size instead (counter calibration).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_PARTICLE_STEP = 28      # z r/w 16 B + v_z r/w 8 B + free-flight counter read 4 B
HBM_PEAK_GBS = 8000.0
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_particles_large_diode_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2605_07083_amd", "csrc", "pic_kernels.hip")


def measured_traffic():
    """Counter-measured HBM bytes per particle-kernel launch of the large diode,
    if the committed profile was taken with the current kernel source."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = dict(ln.split(": ", 1) for ln in text.splitlines() if ln.startswith(("traffic_bytes", "source_sha")))
    if fields.get("source_sha256", "").strip() != src:
        return None
    return float(fields["traffic_bytes_per_launch"])


def workload(name):
    from paper_2605_07083_amd import presets
    if name == "bench":
        return "2048-cell helium diode, 409.6k macro-particles per species, emission 7.25e19 m^-2 s^-1", [presets.bench()]
    if name == "tiny":
        return "256-cell helium diode, 25.6k macro-particles per species, emission 1e19 m^-2 s^-1", [presets.tiny()]
    if name == "large":
        return "16384-cell collisional helium diode, 16.4M macro-particles per species", [presets.large()]
    if name == "sweep":
        return "32-diode emission sweep 1e19-1.2e20 m^-2 s^-1, 100-600k per species", presets.sweep()
    if name == "paper":
        return ("the paper's benchmark diode (10 cm helium gap, 4096 cells, 40 V), 4.1M macro-particles per "
                "species, emission 7.25e19 m^-2 s^-1", [presets.paper()])
    if name == "paperscan":
        from paper_2605_07083_amd import fluxscan
        return ("the paper's eleven-flux scan as one batch of its benchmark diode, 409.6k macro-particles per "
                "species per diode", fluxscan.configs(100))
    raise SystemExit("unknown workload " + name)


def _host():
    """Host CPU model and the cores this process may use."""
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return model, cores


def _oracle_rate(cfg, seconds, omp):
    from oracle import oracle as O
    s = O.Sim(cfg, omp=omp)
    s.load()
    s.step(2)
    live = sum(s.count(sp) for sp in range(3))
    t0 = time.perf_counter()
    steps = 0
    ps = 0
    while time.perf_counter() - t0 < seconds:
        ps += sum(s.count(sp) for sp in range(3))
        s.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    return ps / dt, steps, live, O.threads(omp)


def cpu_baseline(cfg, seconds=12.0):
    """The FP64 oracle on a bounded sample of the same diode: its OpenMP build
    on every host core (the reported value) and its single-threaded build."""
    model, cores = _host()
    v1, n1, live, _ = _oracle_rate(cfg, seconds, omp=False)
    vp, npar, _, threads = _oracle_rate(cfg, seconds, omp=True)
    return {"value": vp, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": "%d steps of the same diode from its initial load (%d live particles), FP64, "
                      "OpenMP build on %d threads" % (npar, live, threads),
            "host_cores": cores, "cpu_model": model,
            "single_thread": {"value": v1, "unit": "particle-steps/s", "cores": 1,
                              "sample": "%d steps of the same sample, single-threaded build" % n1}}


# FLOPs of one surrogate training step per position: forward and weight
# gradients 2 * 88000 each (88000 = multiply-adds of the six layers per
# position), input gradients of layers 1-5 2 * 82880.
# model flops per position and training step (real channels, not the padding):
# forward and weight gradients 2 x 99520 each, input gradients of layers 1-5
# 2 x (4 x 64 x 64 x 5 + 39 x 64 x 5) = 2 x 94400
SUR_FLOP_PER_POSITION = 2 * 99520 + 2 * 99520 + 2 * 94400
MFMA_BF16_PEAK_TFLOPS = 2500.0


def surrogate_bench(args):
    """Training throughput of the warm-start surrogate (batch 32 x 2048 cells)."""
    import numpy as np
    import torch
    from paper_2605_07083_amd import presets
    from paper_2605_07083_amd.surrogate import Surrogate
    B, X = 32, 2048
    q = presets.surrogate_params(B, presets.SURROGATE_TRAIN_SEED)
    P = torch.tensor(np.stack([q["gamma_emit"], q["T_K"], q["V"], q["ng"]], 1), dtype=torch.float32,
                     device="cuda:0")
    u = np.linspace(0.5 / X, 1 - 0.5 / X, X)
    def target(k):
        rows = [u * (1 + 0.01 * k), np.log(0.3 + u), np.log(1.3 - u)]
        rows += [0.3 * ((c - 3) % 9 - 4) + 0.2 * np.sin(3 * u + c + k) for c in range(3, 39)]
        return np.stack(rows)
    T = torch.tensor(np.stack([target(k) for k in range(B)]), dtype=torch.float32, device="cuda:0")
    net = Surrogate(B, X, seed=1)
    for _ in range(args.warmup):
        net.train_step(P, T, 1e-3, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(P, T, 1e-3, want_loss=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t1 = time.perf_counter()
    for _ in range(args.steps):
        net.forward(P)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t1) / args.steps
    step_s = wall / args.steps
    achieved = SUR_FLOP_PER_POSITION * B * X / step_s / 1e12
    out = {"metric": "surrogate training samples/s", "value": B * args.steps / wall, "unit": "samples/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16 x bf16 -> f32 (f32 master weights)", "data": "synthetic smooth targets",
           "config": {"workload": "warm-start surrogate, 6 conv1d layers k=5, 64 channels, batch 32 x 2048 cells",
                      "batch": B, "cells": X, "forward_ms_batch32": fwd * 1e3},
           "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": None,
                        "kernel": "sur_train_step (all kernels of one step)",
                        "flop_per_step": SUR_FLOP_PER_POSITION * B * X}}
    if not args.no_cpu_baseline:
        from oracle import surrogate_oracle as SO
        W, b = presets.surrogate_test_weights(1)
        Bs = 2
        f = SO.features(P[:Bs].double().cpu().numpy(), X)
        tg = T[:Bs].double().cpu().numpy()
        zeros = lambda L: [np.zeros_like(x, dtype=np.float64) for x in L]
        t2 = time.perf_counter()
        n = 0
        while time.perf_counter() - t2 < args.cpu_seconds:
            SO.train_step(W, b, zeros(W), zeros(W), zeros(b), zeros(b), 1, f, tg, 1e-3)
            n += 1
        dt = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": Bs * n / dt, "unit": "samples/s", "cores": torch.get_num_threads(),
                               "kind": "oracle", "sample": "%d FP64 training steps of %d samples x %d cells "
                                                          "(torch CPU conv1d + autograd)" % (n, Bs, X)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4096)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--copy-probe", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-steps", type=int, default=192)
    ap.add_argument("--schedule", default="", help="ppt,grid,sort_period,use_graph: fixed schedule, no autotuning")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1:
        raise SystemExit("bench.py measures one GPU only: the library has no multi-GPU path "
                         "(the design notes describe how it would shard)")

    import torch
    from paper_2605_07083_amd import pic

    if args.copy_probe:
        n = args.copy_probe // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda:0")
        a.fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "launches": 3}), flush=True)
        return

    if args.workload == "surrogate":
        surrogate_bench(args)
        return

    desc, cfgs = workload(args.workload)
    print("bench: workload %s, %d diode(s), warmup %d, steps %d" % (args.workload, len(cfgs), args.warmup,
                                                                    args.steps), file=sys.stderr, flush=True)
    h = pic.Handle(cfgs, device="cuda:0")
    h.step(args.warmup)
    if args.schedule:
        ppt, grid, K, g = (int(x) for x in args.schedule.split(","))
        h.set_tuning(ppt=ppt, grid=grid, sort_period=K, use_graph=g)
        h.step(2 * K)
        tune = h.tuning()
    else:
        tune = h.autotune(trial_steps=args.tune_steps) if args.tune_steps > 0 else h.tuning()
    print("bench: schedule %s" % tune, file=sys.stderr, flush=True)
    K = tune["sort_period"]

    def align():
        # position the schedule so that the timed steps end at a re-sort
        # boundary: they then hold floor(steps / K) whole re-sort periods, each
        # with its re-sort, after the last steps of the period before them
        t = h.tally(0)["step"]
        h.step((K - (t + args.steps) % K) % K)

    # untimed: two passes of the same length from the same schedule position
    # as the timed pass.  Each re-sort flips the particle buffer, and the
    # graphs are captured per buffer: the timed pass starts on the buffer of
    # one of the two passes (the sequence repeats if both started on the
    # same), so every graph it replays is captured before it starts.
    for _ in range(2):
        align()
        h.step_timed(args.steps)
    align()
    h.sync()
    live0 = h.live_total()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = h.step_timed(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h.sync()
    live = 0.5 * (live0 + h.live_total())
    value = live * args.steps / wall
    if not (r["particle_kernel_ms"] > 0.0 and math.isfinite(r["particle_kernel_ms"])):
        raise SystemExit("bench: the particle kernel was not timed (%r)" % r)
    kern_s = r["particle_kernel_ms"] * 1e-3
    achieved = BYTES_PER_PARTICLE_STEP * live / kern_s / 1e9
    step_gbs = BYTES_PER_PARTICLE_STEP * live * args.steps / wall / 1e9
    out = {
        "metric": "particle-steps/s (push+MCC+deposit) on 1 GPU",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 positions / f32 velocities / int64 deposit",
        "data": "synthetic (seeded Philox load of the stated diode)",
        "config": {"workload": desc, "n_diodes": len(cfgs), "cells": cfgs[0]["N"],
                   "particles_per_species": cfgs[0]["n_load"], "live_particles": live,
                   "schedule": {k: tune[k] for k in ("ppt", "grid", "sort_period", "use_graph")},
                   "timed_window": "ends at a re-sort boundary: floor(steps / sort_period) re-sorts inside, "
                                   "after the last steps % sort_period steps of the period before them",
                   "events_ms": r["total_ms"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if args.workload == "large" else None,
                     "traffic_unit": "bytes per launch",
                     "algorithmic_bytes_per_launch": BYTES_PER_PARTICLE_STEP * live,
                     "kernel": "k_particles", "kernel_ms": r["particle_kernel_ms"],
                     "bytes_per_particle_step": BYTES_PER_PARTICLE_STEP,
                     "whole_step_achieved": step_gbs, "whole_step_frac": step_gbs / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline and len(cfgs) == 1:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfgs[0], args.cpu_seconds)
    print(json.dumps(out, allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
