"""Autotuner for the execution knobs of a context.

Every knob (see hg_tune in include/hegmm.h) changes only how the work is
scheduled -- which transform kernels run, how inner products are grouped,
how many products share a launch group -- never the result.  The tuner runs
a workload under each candidate setting, checks that the serialised outputs
are bit-identical to those of the first setting, times the candidates with
events on the current stream (bracketing the reps, with a host clock as a
floor), and applies, returns and optionally stores the fastest.

Usage:
    best = autotune(ctx, run_fn, candidates)
where run_fn() enqueues one step of the workload and returns its outputs.
"""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Callable, Dict, Iterable, List, Optional

import numpy as np

DEFAULT_SPACE = {
    "fuse_rows": [0, 64, 256],
    "ip_chunk": [0, 16, 64],
    "ip_order": [0, 1],
    "ntt_radix": [8, 16],
    "half_rows": [0, 128],
    "batch_window": [0, 64, 128],
}


def grid(space: Dict[str, Iterable[int]]) -> List[Dict[str, int]]:
    keys = sorted(space)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(list(space[k]) for k in keys))]


def _time_steps(run_fn: Callable, reps: int):
    """Seconds per call of run_fn (the later of the stream events around the
    calls and the host clock), and the last call's outputs."""
    import torch
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(reps):
        outs = run_fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return max(e0.elapsed_time(e1) * 1e-3, wall) / reps, outs


def autotune(ctx, run_fn: Callable, candidates: List[Dict[str, int]], reps: int = 3,
             cache: Optional[str] = None, tag: str = "") -> Dict[str, object]:
    """Time run_fn under each candidate knob setting; outputs must not change."""
    ref = None
    results = []
    for cand in candidates:
        for k, v in cand.items():
            ctx.tune(k, v)
        run_fn()  # warm-up (plans, workspace growth)
        dt, outs = _time_steps(run_fn, reps)
        words = [o.export() for o in outs[:: max(1, len(outs) // 8)]]
        if ref is None:
            ref = words
        elif not all(np.array_equal(a, b) for a, b in zip(ref, words)):
            raise RuntimeError(f"setting {cand} changed the results")
        results.append({"knobs": cand, "seconds": dt})
    best = min(results, key=lambda r: r["seconds"])
    for k, v in best["knobs"].items():
        ctx.tune(k, v)
    report = {"tag": tag, "best": best, "all": results}
    if cache:
        data = {}
        if os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
        data[tag] = best["knobs"]
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return report


def apply_cached(ctx, cache: str, tag: str) -> bool:
    """Apply a stored setting; returns False when none is stored for tag."""
    if not os.path.exists(cache):
        return False
    with open(cache) as f:
        data = json.load(f)
    if tag not in data:
        return False
    for k, v in data[tag].items():
        ctx.tune(k, v)
    return True
