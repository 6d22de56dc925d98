"""Autotuner of the persistent tracing kernels' launch schedule.

Candidates vary the workgroup size (rays per workgroup), the register budget
(one or two waves per SIMD), the refill policy (idle lanes a wave waits for
before taking new rays from the queue), the batched launch's queue chunk (list
entries a wave claims at once from its instance's queue) and, for the GJ
density, the number of null-surface restarts a wave batches.  Each candidate
runs the caller's workload function on the current stream, timed with HIP events
(median of several repetitions after a warm-up); the fastest wins.  Results are
cached in a JSON file keyed by device name, a hash of the kernel sources and a
workload key, so a changed kernel is tuned afresh.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))

CANDIDATES = [dict(block=b, occupancy=o, refill_min=r, waves_per_cu=0)
              for o in (2, 1) for r in (1, 4, 16) for b in (256, 64)]

# batched launch: rays per workgroup, occupancy, refill threshold, queue chunk (0: the idle
# lanes' worth per refill) and the null-surface restart batch
BATCHED_CANDIDATES = ([dict(block=256, occupancy=o, refill_min=r, chunk=c, waves_per_cu=0)
                       for o in (2, 1) for r in (4, 16) for c in (0, 64, 256)] +
                      [dict(block=b, occupancy=2, refill_min=4, chunk=0, waves_per_cu=0) for b in (64, 128)] +
                      [dict(block=256, occupancy=2, refill_min=4, chunk=0, cross_batch=x, waves_per_cu=0)
                       for x in (4, 16)])

CACHE = os.path.join(_HERE, "tuning_cache.json")


def kernel_source_hash() -> str:
    """sha256 (first 16 hex digits) of the HIP sources the tracing kernels are built from and
    of the build script that holds their compiler flags"""
    h = hashlib.sha256()
    csrc = os.path.join(_HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    with open(os.path.join(_HERE, "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


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
    ck = f"{dev}|{kernel_source_hash()}|{key}"
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
