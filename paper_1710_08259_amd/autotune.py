"""Autotuner for the launch shape of the neighbour loops.

For a set of cases it times a short run of full steps under every candidate
tuning (particles per work item / threads per workgroup, grid vs persistent
launch, persistent workgroups per compute unit) with HIP events on the
library's stream, and keeps the fastest.  Full steps are nauticle_step for
the SPH models and nauticle_step_law for the pair laws (with the cases' own
attributes).  Results are cached as JSON per workload bucket: model,
dimension, log2 of particles per cell, log2 of the total particle count and
log2 of the number of cases.  The tuning changes only how work is
distributed, never the arithmetic: every candidate gives bitwise the same
results.
"""
from __future__ import annotations

import json
import math
import os
from typing import Optional

import torch

from . import nauticle as N

# Grid launches at three item sizes, and the persistent launch in its
# resident-only form (groups_per_cu = 0: as many workgroups per CU as fit).
# Fewer persistent groups per CU only idle compute units.  The persistent
# launch trailed the grid launch on every workload measured (the 256-case
# batch by 2-9 % per kernel); it stays a candidate for tables whose items
# differ widely in cost, where its cost-ordered queues can balance the load.
CANDIDATES = tuple(N.Tuning(block=b, persistent=p, groups_per_cu=g)
                   for b in (64, 128, 256)
                   for (p, g) in ((0, 4), (1, 0)))


def bucket(cases) -> str:
    n = sum(c.n for c in cases)
    cells = sum(c.n_cells for c in cases)
    ppc = max(n / max(cells, 1), 1e-3)
    model = int(getattr(cases[0], "model", N.MODEL_SUMMATION))
    return (f"m{model}-d{cases[0].dim}-ppc{round(math.log2(ppc))}-n{round(math.log2(max(n, 1)))}"
            f"-c{round(math.log2(len(cases)))}")


def default_cache_path() -> str:
    base = os.environ.get("NAUTICLE_TUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "nauticle", "tuning.json")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_tuning(cases, tuning: N.Tuning, steps: int = 3, warmup: int = 1, device="cuda:0",
                max_nbr: Optional[int] = None) -> float:
    """Mean GPU milliseconds per full step under `tuning`."""
    prob = N.Problem(cases, device=device, tuning=tuning, max_nbr=max_nbr)
    st = prob.state_from_cases()
    if prob.model in (N.MODEL_DEM, N.MODEL_SOCIAL):
        attrs = prob.law_attrs()

        def run(n, events=None):
            prob.step_law(st, attrs, n, events=events)
    elif prob.model in (N.MODEL_SUMMATION, N.MODEL_CONTINUITY):
        def run(n, events=None):
            prob.step(st, n, events=events)
    else:
        raise ValueError("the autotuner times stepping models (SPH and the pair laws)")
    run(warmup)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5 * steps)]
    run(steps, events=ev)
    torch.cuda.synchronize()
    prob.check()
    return sum(ev[5 * k].elapsed_time(ev[5 * k + 4]) for k in range(steps)) / steps


def tune(cases, steps: int = 3, candidates=CANDIDATES, cache_path: Optional[str] = None, device="cuda:0",
         force: bool = False, max_nbr: Optional[int] = None):
    """Best tuning for `cases` (from the cache unless `force`), and the table
    of timings {tuning: ms per step} when it was measured now."""
    path = cache_path or default_cache_path()
    key = bucket(cases)
    cache = _load(path)
    if key in cache and not force:
        return N.Tuning(**cache[key]["tuning"]), None
    timings = {}
    for cand in candidates:
        timings[cand] = time_tuning(cases, cand, steps=steps, device=device, max_nbr=max_nbr)
    best = min(timings, key=timings.get)
    cache[key] = {"tuning": {"block": best.block, "persistent": best.persistent,
                             "groups_per_cu": best.groups_per_cu},
                  "ms_per_step": timings[best]}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return best, timings
