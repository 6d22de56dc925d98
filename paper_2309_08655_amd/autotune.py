"""Autotuner of the persistent tracing kernels' launch schedule.

Candidates vary the workgroup size (rays per workgroup), the register budget
(one or two waves per SIMD) and the refill policy (idle lanes a wave waits for
before taking new rays from the queue).  Each candidate runs the caller's
workload function on the current stream, timed with HIP events (median of a few
repetitions after a warm-up); the fastest wins.  Results are cached in a JSON
file keyed by device name and a workload key.
"""
from __future__ import annotations

import json
import os

import torch

CANDIDATES = [dict(block=b, occupancy=o, refill_min=r, waves_per_cu=0)
              for o in (2, 1) for r in (1, 4, 16) for b in (256, 64)]

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def _time(fn, reps):
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune(run_with_schedule, key: str, candidates=None, reps: int = 3, use_cache: bool = True, verbose=False):
    """run_with_schedule(schedule_dict) must launch the workload once.  Returns
    (best_schedule, {json(schedule): ms})."""
    dev = torch.cuda.get_device_name()
    ck = f"{dev}|{key}"
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            cache = json.load(open(CACHE))
        except (OSError, ValueError):
            cache = {}
        if ck in cache:
            return cache[ck]["best"], cache[ck]["times"]
    times = {}
    for c in candidates or CANDIDATES:
        run_with_schedule(c)  # warm-up
        torch.cuda.synchronize()
        ms = _time(lambda: run_with_schedule(c), reps)
        times[json.dumps(c, sort_keys=True)] = ms
        if verbose:
            print(f"autotune {key}: {c} -> {ms:.3f} ms", flush=True)
    best = json.loads(min(times, key=times.get))
    cache[ck] = dict(best=best, times=times)
    try:
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return best, times
