"""Throughput of the polar-cap PIC step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2] [--no-cpu-baseline]

A step is one whole PIC cycle of the tube: push + deposit, field update +
SCLF injection, and the periodic cell sort.  Inputs are seeded synthetic
tubes shaped like the paper's frame-dragging runs and are resident in HBM
before the timed region.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec + % HBM roofline, FP64 plain vs FP32-bulk; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_PARTICLE_FP64 = 32   # x, u read + written per particle-step

WORKLOADS = {
    "c1": "c1: flat-space SCLF tube, 1024 cells, cold start (~3e3 particles), dt=dz/2",
    "c2": "c2: frame-dragging tube (kappa=0.15, R*=10R), 65536 cells, ~4.0e7 warm particles, "
          "gamma up to ~6e6, dt=dz/2, cell sort every 16 steps",
    "c4": "c4: 64-knot frame-dragging tube, 4096 cells, ~1e6 warm particles",
    "c5": "c5: frame-dragging tube, 2^20 cells, L=100R, ~2.5e8 warm particles",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--push", default="64:2:nt", help="push launch shape threads:slots-per-thread[:nt]")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1011_6330_amd import Tube, synth

    cfg = synth.preset(args.config)
    params = synth.tube_params(cfg)
    log("config", args.config, "cells", cfg["n_cells"], "warm particles", cfg["warm"])
    x, u = synth.warm_start(cfg)
    torch.cuda.set_device(0)
    tube = Tube(params, device="cuda:0")
    if len(x):
        tube.inject(x, u)
    log("injected", len(x))
    parts = args.push.split(":")
    pb, pp, pnt = int(parts[0]), int(parts[1]), len(parts) > 2 and parts[2] == "nt"
    tube.set_push_config(pb, pp, pnt)
    tube.step(args.warmup)
    tube.sync()
    d0 = tube.diagnostics(fields=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tim = tube.step_timed(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d1 = tube.diagnostics(fields=False)
    elapsed = t1 - t0
    alive_avg = 0.5 * (d0["n_alive"] + d1["n_alive"])
    particle_steps = alive_avg * args.steps
    value = particle_steps / elapsed
    push_avg_s = tim["push_ms"] / max(tim["push_launches"], 1) / 1e3
    achieved_gbs = BYTES_PER_PARTICLE_FP64 * alive_avg / push_avg_s / 1e9
    log(f"elapsed {elapsed:.4f}s, push avg {push_avg_s * 1e6:.1f} us, field {tim['field_ms'] / args.steps * 1e3:.1f} us/step,"
        f" sort {tim['sort_ms'] / max(tim['sort_launches'], 1) * 1e3:.1f} us/launch")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded warm-start beam shaped like the paper's frame-dragging runs)",
        "config": {"workload": WORKLOADS[args.config], "n_cells": int(cfg["n_cells"]),
                   "particles": int(alive_avg), "sort_every": int(cfg["sort_every"]),
                   "push": f"fp64 {pb}x{pp}{' nt' if pnt else ''}"},
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_push_f64", "avg_launch_us": push_avg_s * 1e6,
                     "bytes_per_launch": BYTES_PER_PARTICLE_FP64 * alive_avg},
        "breakdown_ms_per_step": {"push": tim["push_ms"] / args.steps, "field": tim["field_ms"] / args.steps,
                                  "sort": tim["sort_ms"] / args.steps},
    }
    tube.close()
    del tube
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth(torch)
    result["roofline"]["achievable_copy_gbs"] = copy_gbs
    result["roofline"]["frac_of_copy"] = achieved_gbs / copy_gbs
    log(f"copy kernel {copy_gbs:.0f} GB/s; push {achieved_gbs:.0f} GB/s")

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(cfg, x, u, args.cpu_seconds)
    print(json.dumps(result), flush=True)


def copy_bandwidth(torch, nbytes=2 << 30, reps=20):
    """Achievable HBM bandwidth of a plain device copy (bytes read + written per second)."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / s / 1e9


def cpu_baseline(cfg, x, u, seconds):
    """The oracle, as it stands, on the same warm tube for a bounded number of steps."""
    from oracle.oracle import OracleTube
    from paper_1011_6330_amd import synth
    p = {k: v for k, v in synth.tube_params(cfg).items() if k not in ("sort_every", "max_bins", "precision")}
    o = OracleTube(p)
    if len(x):
        o.inject(x, u)
    done = 0
    ps = 0.0
    t0 = time.perf_counter()
    while True:
        n = o.n
        o.step(1)
        ps += 0.5 * (n + o.n)
        done += 1
        if time.perf_counter() - t0 > seconds and done >= 2:
            break
    el = time.perf_counter() - t0
    log(f"oracle: {done} steps in {el:.1f}s")
    return {"value": ps / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"the same warm tube ({int(o.n)} particles), first {done} steps, single-threaded FP64 oracle"}


if __name__ == "__main__":
    main()
