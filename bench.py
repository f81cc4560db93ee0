"""Throughput of the polar-cap PIC step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]
                    [--push 128:2:nt] [--push32 128:4:nt] [--tune]
                    [--no-fp32] [--no-ensemble] [--no-adjoint] [--no-cpu-baseline]

A step is one whole PIC cycle of the tube: push + deposit, field update +
SCLF injection, and the periodic cell sort.  Inputs are seeded synthetic
tubes shaped like the paper's frame-dragging runs and are resident in HBM
before the timed region.  The throughput is timed over K plain steps (no
events between the kernels); the per-kernel durations come from K further
steps of the same tube with HIP events around every push, field update and
sort on the tube's stream.  Prints one JSON line:

  value          particle-steps/s of the plain FP64 step on the configured tube
  roofline       of the dominant kernel (the FP64 push), HIP-event timed; its
                 "traffic" is the counter-measured HBM bytes per launch from
                 profiles/k_push_f64_c2_hbm_traffic.txt when that summary was
                 taken on the current push sources and launch shape (else null)
  fp32_bulk      the same tube with the FP32-bulk push (f32 momentum below
                 gamma = 1e6, f64 above), with its own roofline (traffic from
                 profiles/k_push_f32_c2_hbm_traffic.txt); low_gamma: the
                 same geometry with a beam below 1e6, FP64 against FP32-bulk
  gr_alpha       the same tube with the full-GR lapse (PIC_GR_ALPHA), FP64, with
                 the push's VALU busy time from
                 profiles/k_push_f64_gr_c2_sq_counters.txt (same source rule)
  large_tube     the 2^20-cell tube with 2.5e8 particles in FP64 and FP32-bulk,
                 with the Gauss residual at the end
  ensemble       256 tubes of uneven size, one graph launch per round (FP32-bulk;
                 fp64: the same tubes in FP64), with the roofline of the batched
                 push (particle streams plus the kick read and current write
                 per cell; traffic from profiles/k_batch_push_c3_hbm_traffic.txt)
  plausibility   flat-space SCLF over a = omega_p R / c (sec. 3, Table 2): gamma
                 behind the front and the oscillation amplitude per a
  full_step      the whole step's rate against the push's 32 B per particle-step
  pcie_inclusive the rate with the host-to-device copy of the initial particles
                 (pic_inject from host memory) counted in, over the K timed steps
                 and over a 20,000-step run; never the value
  diagnostics    one pic_diagnostics call (fields, Gauss residual, profile)
  small_tubes    C1 (and C4) as time per step: cache-resident, latency-bound
  cpu_baseline   the FP64 oracle on the same tube on every usable host core
                 (threaded oracle step), with the single-threaded rate beside it
The roofline also carries the rate of torch's device copy and of the library's
plain 16-byte nontemporal copy (the achievable stream rate, pic_stream_copy).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec + % HBM roofline, FP64 plain vs FP32-bulk; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
B_FP64 = 32                    # x, u (f64) read + written per particle-step
B_F32_LOW = 24                 # cell, offset, u (f32)
B_F32_HIGH = 24                # position word (4 B), u (f64); the per-group header is 4 B per 256 slots
B_GRID_PUSH = 16               # per cell and push: the kick (E_z) read, the current written
DEFAULT_PUSH = "128:2:nt"      # FP64 push launch shape: threads, slots per thread, nontemporal
DEFAULT_PUSH32 = "128:4:nt"    # FP32-bulk push launch shape


def shape_of(text):
    """A launch shape "threads:slots[:nt]" as (threads, slots, nontemporal)."""
    parts = text.split(":")
    return (int(parts[0]), int(parts[1]), len(parts) > 2 and parts[2] == "nt")

WORKLOADS = {
    "c1": "c1: flat-space SCLF tube, 1024 cells, cold start (~3e3 particles), dt=dz/2",
    "c2": "c2: frame-dragging tube (kappa=0.15, R*=10R, a=6878), 65536 cells, ~4.0e7 warm particles, "
          "gamma up to ~6e6, dt=dz/2, cell sort every 64 steps",
    "c4": "c4: 64-knot frame-dragging tube, 4096 cells, ~1e6 warm particles",
    "c5": "c5: frame-dragging tube (a=6809), 2^20 cells, L=100R, ~2.5e8 warm particles, sort every 16",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def run_tube(cfg, x, u, precision, steps, warmup, push=None, tune=True, diag=None, time_diag=False):
    """Warm a tube up (tuning its push shape), then time `steps` steps."""
    import torch

    from paper_1011_6330_amd import Tube, autotune, synth
    tube = Tube(dict(synth.tube_params(cfg), precision=precision), device="cuda:0")
    inject_s = 0.0
    if len(x):
        # from host memory: the particle streams cross PCIe here, before any timed region
        torch.cuda.synchronize()
        ti = time.perf_counter()
        tube.inject(x, u)
        tube.sync()
        inject_s = time.perf_counter() - ti
    if push is not None:
        tube.set_push_config(*push)
        shape = push
    elif tune:
        b, p, nt, _ = autotune.tune_tube(tube, steps=max(4, warmup // 4), use_cache=False)
        shape = (b, p, nt)
    else:
        shape = None
    tube.step(warmup)
    tube.sync()
    d0 = tube.diagnostics(fields=False)
    # throughput: `steps` plain steps, nothing recorded between the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tube.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d1 = tube.diagnostics(fields=False)
    # kernel durations: `steps` more steps with HIP events around every push,
    # field update and sort, on the tube's own stream
    tim = tube.step_timed(steps)
    d2 = tube.diagnostics(fields=False, **(diag or {}))
    if time_diag:
        # a full diagnostics call (fields, Gauss residual, 64-bin profile, host
        # copies included), averaged over 5 calls after an untimed one
        tube.diagnostics(n_bins=64, gauss=True, fields=True)
        t2 = time.perf_counter()
        for _ in range(5):
            tube.diagnostics(n_bins=64, gauss=True, fields=True)
        tim["diag_ms"] = (time.perf_counter() - t2) / 5 * 1e3
    tim["alive"] = 0.5 * (d1["n_alive"] + d2["n_alive"])
    tim["inject_ms"] = inject_s * 1e3
    tim["gauss_max"], tim["gauss_l2"] = d2["gauss_max"], d2["gauss_l2"]
    tim["alive_high"] = 0.5 * (d1["n_slots_high"] + d2["n_slots_high"])
    tube.close()
    del tube
    torch.cuda.empty_cache()
    return d0, d1, tim, t1 - t0, shape


def roofline_of(bytes_per_launch, tim, kernel):
    push_avg_s = tim["push_ms"] / max(tim["push_launches"], 1) / 1e3
    gbs = bytes_per_launch / push_avg_s / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": None, "kernel": kernel, "avg_launch_us": push_avg_s * 1e6,
            "bytes_per_launch": bytes_per_launch}


CSRC = "paper_1011_6330_amd/csrc/"
PUSH_SOURCES = tuple(CSRC + f for f in ("k_push.hip", "push_body.h", "push_common.h", "short_math.h", "wave.h"))
PUSH32_SOURCES = tuple(CSRC + f for f in ("k_push32.hip", "push_body.h", "push_common.h", "short_math.h", "wave.h"))
BATCH_SOURCES = tuple(CSRC + f for f in ("k_batch.hip", "push_body.h", "push_common.h", "short_math.h", "wave.h"))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_push_f64_c2_hbm_traffic.txt")
TRAFFIC32_FILE = os.path.join(ROOT, "profiles", "k_push_f32_c2_hbm_traffic.txt")
TRAFFIC_BATCH_FILE = os.path.join(ROOT, "profiles", "k_batch_push_c3_hbm_traffic.txt")
GR_SQ_FILE = os.path.join(ROOT, "profiles", "k_push_f64_gr_c2_sq_counters.txt")


def push_source_hash(sources=PUSH_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def shape_text(shape):
    return f"{shape[0]}:{shape[1]}:{'nt' if shape[2] else 'plain'}" if shape else None


def measured_traffic(shape, path=None, sources=PUSH_SOURCES, key="traffic_bytes_per_launch"):
    """HBM bytes per launch of a kernel from a committed counter summary (default:
    the FP64 push's), if it was taken on the current kernel sources and this
    launch shape; else None."""
    path = path or TRAFFIC_FILE
    try:
        with open(path) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(" "))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != push_source_hash(sources) or kv.get("push_shape") != shape_text(shape):
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--push", default=DEFAULT_PUSH, help="FP64 push shape threads:slots[:nt]")
    ap.add_argument("--push32", default=DEFAULT_PUSH32, help="FP32-bulk push shape threads:4[:nt]")
    ap.add_argument("--tune", action="store_true", help="autotune the push shapes instead")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=512)
    ap.add_argument("--ensemble-dense", action="store_true",
                    help="also run the ensemble control of 256 equal dense tubes (FP32-bulk)")
    ap.add_argument("--ensemble-shape", default=None,
                    help="FP32-bulk ensemble launch shape threads:slots instead of the autotuner's "
                         "(a fixed shape for counter runs)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 2^20-cell, 2.5e8-particle tube")
    ap.add_argument("--large-steps", type=int, default=200)
    ap.add_argument("--no-small", action="store_true", help="skip the C1 time-per-step leg")
    ap.add_argument("--no-gr", action="store_true", help="skip the full-GR (PIC_GR_ALPHA) leg")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="seconds per CPU-baseline leg")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(no sharding of a tube across GPUs, no collectives)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1011_6330_amd import synth

    torch.cuda.set_device(0)
    cfg = synth.preset(args.config)
    log("config", args.config, "cells", cfg["n_cells"], "warm particles", cfg["warm"])
    x, u = synth.warm_start(cfg)
    push = None if args.tune else shape_of(args.push)
    push32 = None if args.tune else shape_of(args.push32)

    # ---- plain FP64 step: the headline value ----
    d0, d1, tim, elapsed, shape = run_tube(cfg, x, u, 0, args.steps, args.warmup, push=push, time_diag=True)
    alive = 0.5 * (d0["n_alive"] + d1["n_alive"])
    value = alive * args.steps / elapsed
    roof = roofline_of(B_FP64 * tim["alive"], tim, "k_push_f64")
    roof["traffic"] = measured_traffic(shape)
    log(f"fp64: {elapsed / args.steps * 1e3:.3f} ms/step, push {roof['avg_launch_us']:.1f} us "
        f"({roof['achieved']:.0f} GB/s), shape {shape}")
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
        "config": {"workload": WORKLOADS[args.config], "n_cells": int(cfg["n_cells"]), "particles": int(alive),
                   "sort_every": int(cfg["sort_every"]), "push_shape": list(shape) if shape else None},
        "roofline": roof,
        "breakdown_ms_per_step": {"push": tim["push_ms"] / args.steps, "field": tim["field_ms"] / args.steps,
                                  "sort": tim["sort_ms"] / args.steps},
        # the whole step (push, field update, injection, sort) against the push's 32 B per particle-step
        "full_step": {"achieved": B_FP64 * value / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": B_FP64 * value / 1e9 / HBM_PEAK_GBS},
        "device": device_info(torch),
        # not the value: the same K steps with the host-to-device copy of the initial particles
        # (pic_inject from NumPy arrays in pageable host memory) counted in
        "pcie_inclusive": {"inject_ms": tim["inject_ms"],
                           "value": alive * args.steps / (elapsed + tim["inject_ms"] / 1e3),
                           "value_20000_steps": alive / (elapsed / args.steps + tim["inject_ms"] / 1e3 / 20000)},
    }
    # diagnostics (fields, Gauss residual, profile) are taken every K steps, not every step
    result["diagnostics"] = {"ms_per_call": tim["diag_ms"], "ms_per_step_at_k100": tim["diag_ms"] / 100,
                             "what": "pic_diagnostics on the same tube with E_z, E_r, B_phi, the Gauss residual "
                                     "and a 64-bin signed-gamma profile, host copies included"}
    log(f"diagnostics: {tim['diag_ms']:.2f} ms per call")

    # ---- FP32-bulk push on the same tube ----
    if not args.no_fp32:
        f0, f1, ftim, fel, fshape = run_tube(cfg, x, u, 1, args.steps, args.warmup, push=push32)
        falive = 0.5 * (f0["n_alive"] + f1["n_alive"])
        fhigh = 0.5 * (f0["n_slots_high"] + f1["n_slots_high"])
        froof = roofline_of(B_F32_LOW * max(ftim["alive"] - ftim["alive_high"], 0.0) + B_F32_HIGH * ftim["alive_high"],
                            ftim, "k_push_f32")
        froof["traffic"] = measured_traffic(fshape, TRAFFIC32_FILE, PUSH32_SOURCES)
        result["fp32_bulk"] = {"value": falive * args.steps / fel, "unit": "particle-steps/s",
                               "ms_per_step": fel / args.steps * 1e3, "dtype": "f32+f64",
                               "high_stream_fraction": fhigh / max(falive, 1.0), "push_shape": list(fshape),
                               "roofline": froof, "vs_fp64": (falive * args.steps / fel) / value}
        log(f"fp32-bulk: {fel / args.steps * 1e3:.3f} ms/step, push {froof['avg_launch_us']:.1f} us "
            f"({froof['achieved']:.0f} GB/s), high-stream fraction {fhigh / max(falive, 1):.3f}")

        # the same geometry with a beam below gamma_fp64 (a = 430, gamma up to ~3e4):
        # every particle in the f32-momentum stream, 24 B per particle-step
        lcfg = dict(cfg, q_over_m=synth.q_over_m_for(430.0))
        lx, lu = synth.warm_start(lcfg)
        l0, l1, ltim, lel, _ = run_tube(lcfg, lx, lu, 0, args.steps, args.warmup, push=push)
        m0, m1, mtim, mel, _ = run_tube(lcfg, lx, lu, 1, args.steps, args.warmup, push=push32)
        del lx, lu
        lval = 0.5 * (l0["n_alive"] + l1["n_alive"]) * args.steps / lel
        mval = 0.5 * (m0["n_alive"] + m1["n_alive"]) * args.steps / mel
        mroof = roofline_of(B_F32_LOW * max(mtim["alive"] - mtim["alive_high"], 0.0) + B_F32_HIGH * mtim["alive_high"],
                            mtim, "k_push_f32")
        result["fp32_bulk"]["low_gamma"] = {
            "workload": "the c2 tube geometry with a = 430 (q/m = -a^2/4pi): gamma up to ~3e4, all particles "
                        "in the f32-momentum stream",
            "fp64": {"value": lval, "ms_per_step": lel / args.steps * 1e3,
                     "push_us": ltim["push_ms"] / max(ltim["push_launches"], 1) * 1e3},
            "fp32_bulk": {"value": mval, "ms_per_step": mel / args.steps * 1e3, "roofline": mroof,
                          "high_stream_fraction": mtim["alive_high"] / max(mtim["alive"], 1.0)},
            "fp32_over_fp64": mval / lval}
        log(f"fp32-bulk, low gamma: {mel / args.steps * 1e3:.3f} ms/step (push {mroof['avg_launch_us']:.1f} us) vs "
            f"fp64 {lel / args.steps * 1e3:.3f} ms/step")

    # ---- the same tube with the full-GR lapse factors (PIC_GR_ALPHA), FP64 ----
    if not args.no_gr and args.config == "c2":
        from paper_1011_6330_amd import GR_ALPHA
        gcfg = dict(cfg, flags=int(cfg.get("flags", 0)) | GR_ALPHA, rg_over_rstar=0.4)
        g0, g1, gtim, gel, _ = run_tube(gcfg, x, u, 0, args.steps, args.warmup, push=push)
        gval = 0.5 * (g0["n_alive"] + g1["n_alive"]) * args.steps / gel
        groof = roofline_of(B_FP64 * gtim["alive"], gtim, "k_push_f64<128, 2, 1, 1>")
        result["gr_alpha"] = {"value": gval, "unit": "particle-steps/s", "ms_per_step": gel / args.steps * 1e3,
                              "roofline": groof, "vs_flat": gval / value,
                              "workload": "the c2 tube with the lapse alpha (r_g/R_* = 0.4) in Maxwell's equations "
                                          "and the equation of motion (PIC_GR_ALPHA), FP64"}
        # the full-GR push is launched at 128 x 2 whatever the configured shape
        busy = measured_traffic((128, 2, True), GR_SQ_FILE, PUSH_SOURCES, key="valu_busy_us")
        if busy is not None:
            result["gr_alpha"]["valu"] = {
                "busy_us": busy, "frac_of_push": busy / groof["avg_launch_us"],
                "source": "SQ_ACTIVE_INST_VALU x 4 cycles over 1024 SIMDs at 2.4 GHz, from "
                          "profiles/k_push_f64_gr_c2_sq_counters.txt (taken on these kernel sources)"}
        log(f"gr alpha: {gel / args.steps * 1e3:.3f} ms/step, push {groof['avg_launch_us']:.1f} us "
            f"({groof['achieved']:.0f} GB/s), {gval / value:.3f} of the flat step")

    # ---- the large tube: 2^20 cells, 2.5e8 particles, FP64 and FP32-bulk ----
    if not args.no_large and args.config == "c2":
        result["large_tube"] = run_large(args.large_steps, push, push32)

    # ---- ensemble: 256 tubes, one graph launch per round ----
    if not args.no_ensemble:
        result["ensemble"] = run_ensemble(args.ensemble_steps, precision=1, shape=args.ensemble_shape)
        e64 = run_ensemble(args.ensemble_steps, precision=0)
        result["ensemble"]["fp64"] = {k: e64[k] for k in ("value", "ms_per_step", "launch", "dtype", "roofline",
                                                          "breakdown_ms_per_step")}
        if args.ensemble_dense:
            ed = run_ensemble(args.ensemble_steps, precision=1, dense=True, shape=args.ensemble_shape)
            result["ensemble"]["dense_control"] = {k: ed[k] for k in ("value", "ms_per_step", "launch", "roofline",
                                                                      "particles", "cells", "workload")}

    if not args.no_adjoint:
        adj = run_adjoint_leg(args.adjoint_steps)
        result["adjoint"] = adj
        result["adjoint_forward_ratio"] = adj["backward_over_plain_forward"]

    copy_gbs = copy_bandwidth(torch)
    result["roofline"]["torch_copy_gbs"] = copy_gbs
    ach = stream_copy_bandwidth(torch)
    result["roofline"]["achievable_copy_gbs"] = ach
    result["roofline"]["frac_of_achievable"] = result["roofline"]["achieved"] / ach
    log(f"copy: torch {copy_gbs:.0f} GB/s, 16-byte nontemporal stream {ach:.0f} GB/s")

    if args.config == "c2" and not args.no_small:
        result["small_tubes"] = run_small()
        if "adjoint" in result:
            result["small_tubes"]["c4"] = {
                "us_per_step": result["adjoint"]["plain_forward_ms"] * 1e3 / result["adjoint"]["steps"],
                "steps": result["adjoint"]["steps"],
                "workload": "c4 plain forward of the adjoint leg (4096 cells, ~1e6 particles, 16 MB of state)"}

    if not args.no_sweep:
        from paper_1011_6330_amd import sweep
        rows = sweep.run_convergence([3.5, 5.5, 11.0, 30.0])
        result["plausibility"] = {"workload": "flat-space SCLF from empty tubes, L = 40R, one grid for all a "
                                              "(24 cells per plasma wavelength of the largest a, at least 50 per R), "
                                              "profiles read at the first whole R of light travel after the front reaches 30R; the "
                                              "same on a grid twice "
                                              "as fine ('fine', and the relative changes)",
                                  "rows": [{k: r[k] for k in ("a", "n_cells", "gamma_plateau", "gamma_peak",
                                                              "gamma_sclf", "gamma_paper", "amplitude", "returning",
                                                              "e_surf_ratio", "fine", "change_plateau",
                                                              "change_peak")} for r in rows]}
        log("plausibility: " + "; ".join(f"a={r['a']:g}: peak {r['gamma_peak']:.2f} (fine {r['fine']['gamma_peak']:.2f})"
                                           f" vs sqrt2 a {r['gamma_paper']:.2f}, ampl {r['amplitude']:.2f}"
                                           for r in rows))
        inc = sweep.run_inclination((0.1, 0.5))
        result["plausibility"]["inclination"] = {
            "workload": "Fig. 6: one star (frame dragging, redshift, inclination term of eq. 6; surface density "
                        "cos i) at i = 0.1 and 0.5 rad, a = 100, empty tubes, profiles read at front 8R",
            "rows": [{k: r[k] for k in ("incl", "gamma_plateau", "gamma_peak", "amplitude", "front")} for r in inc]}
        log("inclination: " + "; ".join(f"i={r['incl']:g}: plateau {r['gamma_plateau']:.1f}, peak "
                                          f"{r['gamma_peak']:.1f}" for r in inc))

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(cfg, x, u, args.cpu_seconds)
    print(json.dumps(result), flush=True)


def run_large(steps, push, push32):
    """C5: the 2^20-cell, L = 100R frame-dragging tube with 2.5e8 warm particles,
    cell sort every 16 steps, in FP64 and in FP32-bulk; the Gauss residual of
    eq. (2) at the end of each run, evaluated in FP64."""
    import gc

    from paper_1011_6330_amd import synth
    cfg = synth.preset("c5")
    x, u = synth.warm_start(cfg)
    out = {"workload": WORKLOADS["c5"], "steps": steps}
    for prec, key, shape, bpp in ((0, "fp64", push, B_FP64), (1, "fp32_bulk", push32, None)):
        t0 = time.perf_counter()
        d0, d1, tim, el, sh = run_tube(cfg, x, u, prec, steps, 16, push=shape, tune=False,
                                       diag=dict(gauss=True))
        alive = 0.5 * (d0["n_alive"] + d1["n_alive"])
        if bpp is None:
            nbytes = B_F32_LOW * max(tim["alive"] - tim["alive_high"], 0.0) + B_F32_HIGH * tim["alive_high"]
        else:
            nbytes = bpp * tim["alive"]
        roof = roofline_of(nbytes, tim, "k_push_f64" if prec == 0 else "k_push_f32")
        out[key] = {"value": alive * steps / el, "unit": "particle-steps/s", "ms_per_step": el / steps * 1e3,
                    "particles": int(alive), "roofline": roof, "gauss_max": tim["gauss_max"],
                    "gauss_l2": tim["gauss_l2"], "high_stream_fraction": tim["alive_high"] / max(tim["alive"], 1.0)}
        log(f"large tube {key}: {el / steps * 1e3:.3f} ms/step for {alive:.3g} particles, push "
            f"{roof['avg_launch_us']:.1f} us ({roof['achieved']:.0f} GB/s), Gauss max {tim['gauss_max']:.2e} "
            f"({time.perf_counter() - t0:.1f} s)")
    del x, u
    gc.collect()
    return out


def run_ensemble(steps, precision=1, dense=False, shape=None):
    """C3: 256 tubes of uneven size, autotuned, `steps` plain steps (rounds replayed
    from their graphs), then `steps` more with HIP events around every batched
    kernel for the roofline of the batched push.  dense: the control of equal,
    dense tubes (synth.ensemble).  shape: "threads:slots" in place of the tuner."""
    import torch

    from paper_1011_6330_amd import Batch, autotune, synth
    cfgs = synth.ensemble(n_tubes=256, seed=0, precision=precision, dense=dense)
    b = Batch([synth.tube_params(c) for c in cfgs], device="cuda:0")
    for t, c in enumerate(cfgs):
        x, u = synth.warm_start(c, seed=t)
        b.tubes[t].inject(x, u)
    log("ensemble loaded")
    if shape:
        blk, ppt = (int(v) for v in shape.split(":")[:2])
        b.set_config(blk, ppt)
    else:
        autotune.tune_batch(b, use_cache=False)
    b.step(32)
    b.sync()
    n0 = sum(t.diagnostics(fields=False)["n_alive"] for t in b.tubes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    b.sync()
    d1 = [t.diagnostics(fields=False) for t in b.tubes]
    tim = b.step_timed(steps)
    d2 = [t.diagnostics(fields=False) for t in b.tubes]
    n1 = sum(d["n_alive"] for d in d1)
    cfg = b.get_config()
    b.close()
    del b
    torch.cuda.empty_cache()
    alive = 0.5 * (n0 + n1)
    cells = int(sum(c["n_cells"] for c in cfgs))
    # algorithmic bytes of one batched push: the particle streams (as the single-tube
    # pushes) plus, per cell, the kick (E_z) read and the current written once
    t_alive = 0.5 * sum(a["n_alive"] + c["n_alive"] for a, c in zip(d1, d2))
    t_high = 0.5 * sum(a["n_slots_high"] + c["n_slots_high"] for a, c in zip(d1, d2))
    if precision:
        pbytes = B_F32_LOW * max(t_alive - t_high, 0.0) + B_F32_HIGH * t_high
    else:
        pbytes = B_FP64 * t_alive
    gbytes = B_GRID_PUSH * cells
    kern = f"k_batch_push<{cfg['block']}, {cfg['per_thread']}, 1, {precision}>"
    roof = roofline_of(pbytes + gbytes, tim, kern)
    roof["particle_bytes_per_launch"] = pbytes
    roof["grid_bytes_per_launch"] = gbytes
    shape = (cfg["block"], cfg["per_thread"], True)
    roof["traffic"] = measured_traffic(shape, TRAFFIC_BATCH_FILE, BATCH_SOURCES) if precision else None
    steps_t = max(tim["push_launches"], 1)
    log(f"ensemble ({'fp32-bulk' if precision else 'fp64'}{', dense control' if dense else ''}): "
        f"{el / steps * 1e3:.3f} ms/step for {alive:.3g} "
        f"particles in 256 tubes, shape {cfg}; push {roof['avg_launch_us']:.1f} us ({roof['achieved']:.0f} GB/s), "
        f"field + work list {tim['field_ms'] / steps_t * 1e3:.1f} us per step")
    return {"value": alive * steps / el, "unit": "particle-steps/s", "ms_per_step": el / steps * 1e3,
            "tubes": 256, "cells": cells, "particles": int(alive),
            "dtype": "f32+f64" if precision else "f64", "launch": cfg, "steps": steps, "roofline": roof,
            "breakdown_ms_per_step": {"push": tim["push_ms"] / steps_t, "field": tim["field_ms"] / steps_t,
                                      "sort": tim["sort_ms"] / steps_t},
            "high_stream_fraction": t_high / max(t_alive, 1.0),
            "workload": ("256 frame-dragging tubes of 2048 cells and 2.2e5 particles each (the control: dense "
                         "tubes, about 107 particles per cell), FP32-bulk, one graph launch per 64-step round"
                         if dense else
                         "256 frame-dragging tubes, cells log-uniform 2048-65536, particles log-uniform 1e4-1e6, "
                         "kappa 0.05-0.2, rho_GJ amplitude 0.3-3, FP32-bulk (fp64: the same tubes in FP64), "
                         "one graph launch per 64-step round (steps and cell sort)")}


def run_adjoint_leg(steps, ckpt=50):
    """C4: the hand-written adjoint of `steps` steps (checkpoints every `ckpt`)
    against a plain forward of the same steps on the same tube: the recorded
    forward (pic_adjoint_forward) and the reverse sweep (pic_backward) timed
    apart.  `rate_variant` is the same tube cut to its first 256 cells (same
    cell size and density), where electrons injected during the run reach the
    top, so that the injection-rate gradient is not 0."""
    out = _adjoint_case(synth_preset("c4"), steps, ckpt)
    out["workload"] = ("c4: 64-knot frame-dragging tube, 4096 cells, ~1e6 warm particles, loss = mean exit gamma, "
                       f"{steps} steps, checkpoint every {ckpt}, FP64")
    c = synth_preset("c4")
    n = 256
    c.update(n_cells=n, length=c["length"] * n / c["n_cells"], warm=int(c["ppc"] * n),
             capacity=int(c["ppc"] * n * 8))   # the beam leaves and is replaced about twice
    rv = _adjoint_case(c, steps, ckpt)
    rv["workload"] = (f"the c4 tube's first 256 cells (L = {c['length']:.3f} R, same cell size and density, "
                      f"{c['warm']} warm particles), {steps} steps, checkpoint every {ckpt}: injected electrons "
                      "reach the top")
    out["rate_variant"] = rv
    log(f"adjoint rate variant: dL/drate {rv['g_rate']:.6g}, backward / plain forward "
        f"{rv['backward_over_plain_forward']:.2f}")
    return out


def synth_preset(name):
    from paper_1011_6330_amd import synth
    return synth.preset(name)


def _adjoint_case(cfg, steps, ckpt, reps=3):
    """Plain forward, and recorded forward + reverse sweep, `reps` times each on
    fresh tubes; the medians are reported (the reverse sweep's two streams make
    single runs vary by tens of percent on these short kernels)."""
    import statistics

    import torch

    from paper_1011_6330_amd import Tube, synth
    x, u = synth.warm_start(cfg)
    p = synth.tube_params(cfg)
    fwds, recs, bwds = [], [], []
    for _ in range(reps):
        # the plain forward: the same steps launched back to back, nothing recorded
        # between them, timed from the host around a device synchronisation
        t = Tube(p, device="cuda:0")
        t.inject(x, u)
        t.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t.step(steps)
        t.sync()
        fwds.append((time.perf_counter() - t0) * 1e3)
        t.close()
        t = Tube(p, device="cuda:0")
        t.inject(x, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = t.adjoint_forward(steps, ckpt)
        r = t.backward()
        el = time.perf_counter() - t0
        recs.append(f["forward_ms"])
        bwds.append(r["backward_ms"])
        t.close()
        del t
        torch.cuda.empty_cache()
    fwd, rec, bwd = statistics.median(fwds), statistics.median(recs), statistics.median(bwds)
    log(f"adjoint: plain forward {fwd:.1f} ms, checkpointed forward {rec:.1f} ms, "
        f"backward {bwd:.1f} ms (medians of {reps}; backward runs {', '.join(f'{b:.1f}' for b in bwds)} ms), "
        f"loss {r['loss']:.6g} over {r['n_exit']} exits, dL/drate {r['g_rate']:.4g}")
    return {"steps": steps, "checkpoint_every": ckpt, "plain_forward_ms": fwd,
            "checkpointed_forward_ms": rec, "backward_ms": bwd, "repeats": reps,
            "backward_ms_runs": bwds, "plain_forward_ms_runs": fwds,
            "backward_over_plain_forward": bwd / fwd if fwd > 0 else None,
            "backward_over_checkpointed_forward": bwd / rec if rec > 0 else None,
            "loss": r["loss"], "n_exit": r["n_exit"], "tape_bytes": f["tape_bytes"], "wall_s": el,
            "g_kappa": r["g_kappa"], "g_rate": r["g_rate"]}


def copy_bandwidth(torch, nbytes=2 << 30, reps=20):
    """HBM bandwidth of torch's device copy_ (bytes read + written per second): context
    for the push's figure, not a ceiling (the push itself moves its bytes faster)."""
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


def stream_copy_bandwidth(torch, nbytes=2 << 30, reps=20):
    """HBM bandwidth (bytes read + written per second) of the library's plain
    16-byte nontemporal copy kernel: the achievable rate of a simple stream."""
    import ctypes

    from paper_1011_6330_amd import _binding
    lib = _binding.load()
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def once():
        rc = lib.pic_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes, stream)
        if rc != 0:
            raise RuntimeError("pic_stream_copy: " + lib.pic_last_error().decode())

    for _ in range(3):
        once()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    if not torch.equal(src[:4096], dst[:4096]) or not torch.equal(src[-4096:], dst[-4096:]):
        raise RuntimeError("pic_stream_copy did not copy")
    s = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / s / 1e9


def device_info(torch):
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "memory_gib": p.total_memory / 2 ** 30}


def run_small(steps=2000):
    """C1: the 1024-cell flat-space SCLF tube from empty, 2000 steps.  Its state
    is a few hundred kB and stays in cache, so it is reported as time per step
    (launch latency of two kernels a step), not against the HBM roofline."""
    import torch

    from paper_1011_6330_amd import Tube, synth
    cfg = synth.preset("c1")
    tube = Tube(synth.tube_params(cfg), device="cuda:0")
    tube.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tube.step(steps)
    tube.sync()
    el = time.perf_counter() - t0
    n = tube.diagnostics(fields=False)["n_alive"]
    tube.close()
    log(f"c1: {el / steps * 1e6:.1f} us/step over {steps} steps from empty, {n} particles at the end")
    return {"c1": {"us_per_step": el / steps * 1e6, "steps": steps, "particles_end": int(n),
                   "workload": WORKLOADS["c1"]}}


def host_cpu():
    """nproc, the cores this process may run on, and the CPU model of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": model}


def cpu_baseline(cfg, x, u, seconds):
    """The oracle on the same warm tube for a bounded number of steps: on every
    core this process may use (orc_step_par: the oracle's own steps with the
    particles split over OpenMP threads, bit-identical to the serial oracle),
    and single-threaded (orc_step), each for about `seconds` seconds."""
    from oracle.oracle import OracleTube
    from paper_1011_6330_amd import synth
    host = host_cpu()
    threads = host["usable_cores"]
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = max(1, min(threads, int(os.environ["OMP_NUM_THREADS"])))
    p = {k: v for k, v in synth.tube_params(cfg).items()
         if k not in ("sort_every", "max_bins", "precision", "gamma_fp64")}
    legs = {}
    for key, nthreads in (("all_cores", threads), ("serial", 1)):
        o = OracleTube(p)
        if len(x):
            o.inject(x, u)
        done, ps = 0, 0.0
        t0 = time.perf_counter()
        while True:
            n = o.n
            if nthreads == 1:
                o.step(1)
            else:
                o.step_par(1, nthreads)
            ps += 0.5 * (n + o.n)
            done += 1
            if time.perf_counter() - t0 > seconds and done >= 2:
                break
        el = time.perf_counter() - t0
        legs[key] = {"value": ps / el, "steps": done, "seconds": el, "threads": nthreads}
        log(f"oracle ({key}, {nthreads} threads): {done} steps in {el:.1f}s, {ps / el:.3g} particle-steps/s")
        del o
    a = legs["all_cores"]
    adj = cpu_adjoint_ratio()
    others = cpu_other_configs(threads)
    return {"value": a["value"], "unit": "particle-steps/s", "cores": a["threads"], "kind": "oracle",
            "adjoint": adj, "other_configs": others,
            "sample": f"the same warm tube ({len(x)} particles at the start), first {a['steps']} steps, FP64 "
                      f"oracle on {a['threads']} threads (particles split into contiguous slices, integer sums "
                      f"in thread order: the serial oracle's state bit for bit)",
            "serial": {"value": legs["serial"]["value"], "cores": 1, "steps": legs["serial"]["steps"],
                       "sample": f"first {legs['serial']['steps']} steps, single-threaded FP64 oracle"},
            "parallel_speedup": a["value"] / legs["serial"]["value"], **host}


def cpu_other_configs(threads, ens_steps=2):
    """The oracle on the small tube (C1 from empty, all 2000 steps, serial: a time per
    step) and on the ensemble (every tube of C3 from its warm start, `ens_steps`
    steps on `threads` threads: particle-steps/s)."""
    from oracle.oracle import OracleTube
    from paper_1011_6330_amd import synth
    out = {}
    c1 = synth.preset("c1")
    p = {k: v for k, v in synth.tube_params(c1).items()
         if k not in ("sort_every", "max_bins", "precision", "gamma_fp64")}
    o = OracleTube(p)
    t0 = time.perf_counter()
    o.step(2000)
    el = time.perf_counter() - t0
    out["c1"] = {"us_per_step": el / 2000 * 1e6, "steps": 2000, "threads": 1, "particles_end": int(o.n)}
    log(f"oracle c1: {el / 2000 * 1e6:.1f} us/step over 2000 steps (serial)")
    ps, el = 0.0, 0.0
    for t, c in enumerate(synth.ensemble(n_tubes=256, seed=0, precision=0)):
        x, u = synth.warm_start(c, seed=t)
        p = {k: v for k, v in synth.tube_params(c).items()
             if k not in ("sort_every", "max_bins", "precision", "gamma_fp64")}
        o = OracleTube(p)
        o.inject(x, u)
        n = o.n
        t0 = time.perf_counter()
        o.step_par(ens_steps, threads)
        el += time.perf_counter() - t0
        ps += 0.5 * (n + o.n) * ens_steps
        del o
    out["c3"] = {"value": ps / el, "unit": "particle-steps/s", "steps": ens_steps, "threads": threads,
                 "sample": f"all 256 tubes, {ens_steps} steps each from the warm start (tube set-up not timed)"}
    log(f"oracle c3: {ps / el:.3g} particle-steps/s on {threads} threads ({ens_steps} steps of all 256 tubes)")
    return out


def cpu_adjoint_ratio(steps=200):
    """The adjoint/forward time ratio of the oracle on a 1e5-particle downscale of
    the adjoint workload (4096 cells, 24.4 particles per base cell-charge, the same
    density relative to rho_GJ): a plain serial forward of `steps` steps, and the
    oracle's adjoint (the same steps recorded whole, then the reverse sweep)."""
    from oracle.oracle import OracleTube
    from paper_1011_6330_amd import synth
    ppc = 24.4
    cfg = synth.preset("c4", ppc=ppc, warm=int(ppc * 4096), capacity=int(ppc * 4096 * 1.3),
                       macro_charge=-(1.0 - 0.15) * (10.0 / 4096) / ppc)
    x, u = synth.warm_start(cfg)
    p = {k: v for k, v in synth.tube_params(cfg).items()
         if k not in ("sort_every", "max_bins", "precision", "gamma_fp64")}
    o = OracleTube(p)
    o.inject(x, u)
    t0 = time.perf_counter()
    o.step(steps)
    fwd = time.perf_counter() - t0
    o = OracleTube(p)
    o.inject(x, u)
    t0 = time.perf_counter()
    loss, nex, _, _ = o.adjoint(steps)
    adj = time.perf_counter() - t0
    del o
    log(f"oracle adjoint ({len(x)} particles, {steps} steps): plain forward {fwd * 1e3:.0f} ms, recorded forward "
        f"and reverse sweep {adj * 1e3:.0f} ms")
    return {"workload": f"c4 downscaled to {len(x)} particles (4096 cells, ppc {ppc}), {steps} steps, serial FP64 oracle",
            "plain_forward_s": fwd, "adjoint_s": adj, "adjoint_over_plain_forward": adj / fwd,
            "backward_over_plain_forward": (adj - fwd) / fwd, "loss": loss, "n_exit": nex,
            "note": "the oracle records every step (no checkpoints); backward = adjoint run minus a plain forward"}


if __name__ == "__main__":
    main()
