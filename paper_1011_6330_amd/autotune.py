"""Launch-shape autotuner for single tubes and batches.

Every candidate shape gives bit-identical results (integer deposition), so the
tuner only times: it runs a few steps per candidate with per-kernel HIP events
(``pic_step_timed``) and keeps the fastest.  Timing advances the simulation,
so tuning is meant for the warm-up steps of a run.  Results are cached in a
JSON file keyed by device, precision and a log2 bucket of the particle count.
"""
import json
import math
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pcpic_tune.json")

TUBE_SHAPES = [(64, 2, True), (128, 2, True), (256, 2, True), (64, 4, True), (256, 2, False), (128, 4, True)]
TUBE_SHAPES_F32 = [(64, 4, True), (128, 4, True), (256, 4, True), (512, 4, True), (256, 4, False)]
BATCH_SHAPES = [(b, p) for b in (64, 128, 256, 512) for p in (2, 4) if (b, p) != (512, 4)]
BATCH_SHAPES_F32 = [(b, 4) for b in (64, 128, 256, 512)]


def _device_key():
    try:
        import torch
        return torch.cuda.get_device_name(0).replace(" ", "_")
    except Exception:
        return "unknown"


def _bucket(n):
    return int(math.log2(max(n, 1)))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_tube(tube, steps=16, cache_path=DEFAULT_CACHE, use_cache=True):
    """Pick the push shape of a Tube; returns (block, per_thread, nontemporal, times)."""
    f32 = int(tube.cfg.get("precision", 0)) == 1
    n = tube.diagnostics(fields=False)["n_alive"]
    key = f"tube/{_device_key()}/{'f32' if f32 else 'f64'}/{_bucket(n)}"
    cache = _load(cache_path) if use_cache else {}
    if key in cache:
        b, p, nt = cache[key]
        tube.set_push_config(b, p, nt)
        return b, p, nt, {}
    times = {}
    for b, p, nt in (TUBE_SHAPES_F32 if f32 else TUBE_SHAPES):
        tube.set_push_config(b, p, nt)
        t = tube.step_timed(steps)
        times[(b, p, nt)] = t["push_ms"] / max(t["push_launches"], 1)
    best = min(times, key=times.get)
    tube.set_push_config(*best)
    if use_cache:
        cache[key] = list(best)
        _store(cache_path, cache)
    return (*best, times)


def tune_batch(batch, steps=None, cache_path=DEFAULT_CACHE, use_cache=True):
    """Pick the batched-kernel shape of a Batch; returns (block, per_thread, times)."""
    f32 = int(batch.cfgs[0].get("precision", 0)) == 1
    n = sum(t.diagnostics(fields=False)["n_alive"] for t in batch.tubes)
    se = int(batch.cfgs[0].get("sort_every", 16)) or 16
    steps = steps or se
    key = f"batch/{_device_key()}/{'f32' if f32 else 'f64'}/{len(batch)}/{_bucket(n)}"
    cache = _load(cache_path) if use_cache else {}
    if key in cache:
        b, p = cache[key]
        batch.set_config(b, p)
        return b, p, {}
    times = {}
    for b, p in (BATCH_SHAPES_F32 if f32 else BATCH_SHAPES):
        try:
            batch.set_config(b, p)
        except Exception:
            continue
        t = batch.step_timed(steps)
        times[(b, p)] = t["total_ms"] / steps
    best = min(times, key=times.get)
    batch.set_config(*best)
    if use_cache:
        cache[key] = list(best)
        _store(cache_path, cache)
    return (*best, times)
