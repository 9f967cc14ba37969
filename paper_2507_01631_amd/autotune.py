"""Autotuner for the launch shapes of the window step.

The tunables (``_lib.TUNABLES``) decide how each kernel's work is cut across
the 256 compute units: blocks per CU of the grid-stride kernels, the block
count and levels per pass of the binned table adjoint.  ``tune`` times a
caller-given step (HIP events on the current stream, median of ``reps``
runs after ``warmup``) and walks the tunables one at a time over their
candidate values, keeping each value that lowers the step time (coordinate
descent, ``rounds`` sweeps).  The winning table is applied to the library,
and can be saved as JSON and loaded before a step is captured into a graph
(a captured graph keeps the launch shapes it was captured with).

The tuned step must not depend on the tunables for its results beyond
summation order (``mlp_bwd_blocks_per_cu`` changes the order of the weight-
gradient sum); the step callable is free to train (its updates are part of
the cost being timed).
"""
from __future__ import annotations

import json

import torch

from . import _lib as L

CANDIDATES = {
    "hash_fwd_blocks_per_cu": [4, 8, 16, 32],
    "mlp_fwd_blocks_per_cu": [2, 3, 4, 8],
    "mlp_bwd_blocks_per_cu": [1, 2],
    "composite_blocks_per_cu": [4, 8, 16],
    "bin_blocks": [512, 1024, 2048],
    "bin_levels_per_pass": [0, 2, 4],
    "sampler_blocks_per_cu": [8, 16, 32],
    "hash_fwd_superchunk": [0, 1, 2, 4],
}


def current():
    return {k: L.snake_tune_get(k) for k in L.TUNABLES}


def apply(table):
    for k, v in table.items():
        L.snake_tune_set(k, v)


def time_step(step, reps=5, warmup=2):
    """Median milliseconds of one call of ``step`` (HIP events)."""
    for _ in range(warmup):
        step()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune(step, candidates=None, rounds=1, reps=5, warmup=2, log=None):
    """Coordinate descent over the tunables; returns (table, best_ms, trace)."""
    cand = dict(CANDIDATES if candidates is None else candidates)
    best = current()
    apply(best)
    best_ms = time_step(step, reps, warmup)
    trace = [dict(best, ms=best_ms)]
    for _ in range(rounds):
        for name, values in cand.items():
            for v in values:
                if v == best[name]:
                    continue
                trial = dict(best, **{name: v})
                apply(trial)
                ms = time_step(step, reps, warmup)
                trace.append(dict(trial, ms=ms))
                if log:
                    log("  tune %s=%d: %.3f ms (best %.3f)" % (name, v, ms, best_ms))
                if ms < best_ms:
                    best, best_ms = trial, ms
            apply(best)
    return best, best_ms, trace


def save(path, table):
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load(path):
    with open(path) as f:
        table = json.load(f)
    apply(table)
    return table
