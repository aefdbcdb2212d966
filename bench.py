"""Benchmark of the WCSPH hot path on one MI355X.

A step is one pass of the whole hot path over the 3-D periodic jittered
lattice of 8,388,608 particles (256 x 256 x 128, h = 1.2 dx, ~57
neighbours): neighbour search (keys, radix sort, cell table, reorder,
neighbour lists), density + Tait pressure, accelerations with the fused
semi-implicit Euler update.  Inputs are resident in HBM before timing.

Prints ONE JSON line.  `value` is pair interactions per second over the
whole step (each ordered neighbour pair counted once per step);
`force_pass_interactions_per_s` the same pairs over the force pass alone.  Phase times
come from HIP events recorded on the library's stream between the kernels.
`roofline` is for the dominant kernel (the neighbour-list search);
`extra.roofline_force_pass` for the force kernel.  `cpu_baseline` times the
FP64 oracle on a bounded sample of the same workload (a smaller box of the
same lattice recipe).  `extra` also carries the forward + adjoint step rate
of the 262,144-particle differentiation case (with the oracle's rate on the
same case: the "vs plain" figure), the 256-case batched workload and the
3-D dam-break workload.
"""
import argparse
import json
import os
import tempfile
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per unit (see the design notes):
#  search: per candidate tested, d = off_j - t (3), r^2 (3 mul/fma = 5 flops), compare (1)
#  force pass: per neighbour pair, 40 flops (FMA = 2)
SEARCH_FLOP_PER_CANDIDATE = 9
FORCE_FLOP_PER_PAIR = 40
PEAK_FP32_TFLOPS = 157.3            # published MI355X FP32 vector peak (packed FP32)
PEAK_FP32_TFLOPS_UNPACKED = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz: the kernels are compiled without packed FP32
PEAK_HBM_GBS = 8000.0
# HBM bytes per k_nlist launch from the FETCH_SIZE / WRITE_SIZE counter runs
# summarised in profiles/neighbour_kernels_periodic_3d_8388608_traffic.md
# (scaled by a plain 1 GiB copy); valid only for the search source the
# counters were taken on, reported as null otherwise.
NLIST_TRAFFIC_BYTES = 3.711e9
NLIST_TRAFFIC_SOURCE_SHA256 = "f3f0d4aae76e8902"


# VALU and vector-L1 figures from the counter runs summarised in
# profiles/neighbour_kernels_periodic_3d_8388608_issue.md, guarded the same
# way (by the sources of the kernels they were taken on).  VALU rates are
# wave instructions per SIMD per 4 cycles (SQ_INSTS_VALU over 1024 SIMDs x
# cycles / 4); gfx950 exceeds 1.0 on this measure, so it is a rate, not a
# fraction of a ceiling.
NLIST_VALU_PER_SIMD_4CYC = 1.184
NLIST_VALU_INSTS = 1.274e9    # wave instructions per search launch (SQ_INSTS_VALU)
FORCE_L1_ACCESS_RATE = 1.12   # accesses per CU per clock
# HBM bytes per density / force launch (FETCH_SIZE x2 + WRITE_SIZE, same
# runs and guard as the L1 rate), and the force pass's VALU rate.
DENSITY_TRAFFIC_BYTES = 2.684e9 + 0.403e9
FORCE_TRAFFIC_BYTES = 3.026e9 + 0.369e9
FORCE_VALU_PER_SIMD_4CYC = 0.495
FORCE_SOURCES_SHA256 = "258c56d86fb8744c"


def _digest(*rel):
    import hashlib

    h = hashlib.sha256()
    for r in rel:
        with open(os.path.join(ROOT, "paper_1710_08259_amd", "csrc", r), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def nlist_traffic():
    return NLIST_TRAFFIC_BYTES if _digest("search.hip", "internal.h") == NLIST_TRAFFIC_SOURCE_SHA256 else None


def nlist_valu_rate():
    return NLIST_VALU_PER_SIMD_4CYC if _digest("search.hip", "internal.h") == NLIST_TRAFFIC_SOURCE_SHA256 else None


def nlist_lane_slots_per_candidate(candidates):
    """VALU lane-slots (wave instructions x 64) the search spends per
    candidate it tests, from the counter run; null for other sources."""
    if _digest("search.hip", "internal.h") != NLIST_TRAFFIC_SOURCE_SHA256 or not candidates:
        return None
    return round(NLIST_VALU_INSTS * 64 / candidates, 2)


def force_l1_rate():
    return FORCE_L1_ACCESS_RATE if _digest("sph.hip", "pairs.h", "internal.h") == FORCE_SOURCES_SHA256 else None


def _force_guard(v):
    return v if _digest("sph.hip", "pairs.h", "internal.h") == FORCE_SOURCES_SHA256 else None


# Algorithmic HBM bytes per particle and step (3-D FP32 SoA): density reads
# offsets (12) and writes rho, p, s, 1/rho (16); the force pass with the
# integration reads offsets, velocity, s, 1/rho (32) and writes the new
# cell, offsets, velocity (28) plus a (12); keys, three sort passes, cell
# ranges and the reorder move about 128.
DENSITY_ALGO_BYTES = 28
FORCE_ALGO_BYTES = 72
SORT_REORDER_ALGO_BYTES = 128


def hbm_fractions(n, phase_ms):
    """Measured (counter) and algorithmic HBM rates of the step's phases
    against the 8 TB/s peak."""
    def rate(nbytes, ms):
        if nbytes is None:
            return None
        tbps = nbytes / (ms * 1e-3) / 1e12
        return {"bytes": nbytes, "TB_per_s": round(tbps, 3), "frac": round(tbps * 1e3 / PEAK_HBM_GBS, 4)}

    return {
        "density": {"measured": rate(_force_guard(DENSITY_TRAFFIC_BYTES), phase_ms[2]),
                    "algorithmic": rate(DENSITY_ALGO_BYTES * n, phase_ms[2])},
        "force_pass": {"measured": rate(_force_guard(FORCE_TRAFFIC_BYTES), phase_ms[3]),
                       "algorithmic": rate(FORCE_ALGO_BYTES * n, phase_ms[3]),
                       "valu_per_simd_4_cycles": _force_guard(FORCE_VALU_PER_SIMD_4CYC)},
        "sort_cells_reorder": {"algorithmic": rate(SORT_REORDER_ALGO_BYTES * n, phase_ms[0])},
    }


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="only the main workload")
    ap.add_argument("--cpu-sample", default="256x256x128",
                    help="oracle sample box (lattice sites per axis; the default is the main workload)")
    ap.add_argument("--ex1a-only", action="store_true",
                    help="only the Example 1a dam break (continuity model, symmetric faces)")
    ap.add_argument("--ch-only", action="store_true", help="only the Example 1b Cahn-Hilliard sphere")
    ap.add_argument("--law-only", choices=("dem", "social"), default=None,
                    help="only one pair-law workload (DEM damper or social force room)")
    ap.add_argument("--only", choices=("adjoint", "batched", "dam_break", "paper_shape", "small", "largest"),
                    default=None, help="only one extra workload (for profiling runs)")
    ap.add_argument("--batched-tuning", default=None,
                    help="block/persistent/groups_per_cu for the batched workload instead of the autotuner's pick")
    ap.add_argument("--verlet-only", action="store_true",
                    help="only the main lattice with neighbour lists reused between builds")
    ap.add_argument("--skin-frac", type=float, default=0.1, help="Verlet skin in units of 2h")
    ap.add_argument("--law-tuning", default=None,
                    help="block/persistent/groups_per_cu for the pair-law workloads instead of the autotuner's pick")
    ap.add_argument("--ex1a-scale", type=float, default=87.0,
                    help="resolution factor of the Example 1a dam break (87: 4.1M particles)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB of a plain device copy run before timing (counter calibration runs)")
    return ap.parse_args()


def candidates_per_step(prob, case):
    """Candidates the search tests per step: sum over particles of the
    occupancy of the 3^dim cells around theirs (periodic box)."""
    import torch

    nc = case.ncell
    start = prob.cells.cell_start[: case.n_cells].to(torch.int64)
    end = prob.cells.cell_end[: case.n_cells].to(torch.int64)
    cnt = torch.where(start < 0, torch.zeros_like(start), end - start)
    grid = cnt.reshape(nc[2], nc[1], nc[0]).double()
    s = torch.zeros_like(grid)
    for dz in (-1, 0, 1) if case.dim == 3 else (0,):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                s += torch.roll(grid, shifts=(dz, dy, dx), dims=(0, 1, 2))
    return float((grid * s).sum().item())


def timed_steps(prob, st, steps, warmup, step=None):
    """Runs warmup + steps full steps; returns (wall s, per-phase ms [4], pairs).
    `step(st, events)` runs one step (default: nauticle_step)."""
    import numpy as np
    import torch

    n = prob.n
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(5 * steps)]
    for e in evs:  # create the HIP events before the timed region
        e.record(stream)
    pairs = torch.zeros((), dtype=torch.int64, device=prob.device)

    def body(k):
        if step is None:
            prob.step(st, 1, events=evs[5 * k: 5 * k + 5])
        else:
            step(st, evs[5 * k: 5 * k + 5])
        pairs.add_(prob.cells.nbr_count[:n].sum())  # int32 counts, summed in int64

    for k in range(warmup):  # the timed body itself, so every kernel module is loaded
        body(k % steps)
    torch.cuda.synchronize()
    prob.check()
    pairs.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        body(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prob.check()
    phase = np.zeros(4)
    for k in range(steps):
        e = evs[5 * k: 5 * k + 5]
        phase += [e[i].elapsed_time(e[i + 1]) for i in range(4)]
    return wall, phase / steps, int(pairs.item())


def cpu_single_thread(case):
    """The oracle on one thread: one FP64 step of a 64^3 box of the same
    lattice recipe (about 3 s)."""
    import numpy as np

    from oracle import oracle as O
    from paper_1710_08259_amd import workloads as WL

    sample = WL.lattice_case(3, (64, 64, 64), 0.01, 1.2, 0.05, 0.05, seed=3, c0=case.c0, nu=case.nu, dt=case.dt)
    dom = O.Domain(dim=3, n=sample.ncell, cs=sample.cell_size, origin=sample.origin)
    prm = O.Params(h=sample.h, mass=sample.mass, rho0=sample.rho0, c0=sample.c0, gamma=sample.gamma,
                   nu=sample.nu, dt=sample.dt, g=sample.g)
    x = sample.pos.astype(np.float64)
    v = sample.vel.astype(np.float64)
    _, _, counts = O.density(dom, prm, x, counts=True, nthreads=1)
    t0 = time.perf_counter()
    O.step(dom, prm, x, v, n_steps=1, nthreads=1)
    dt = time.perf_counter() - t0
    return {"value": int(counts.sum()) / dt, "unit": "interactions/s", "cores": 1, "kind": "oracle",
            "steps_per_s": 1.0 / dt, "sample": f"one FP64 step of a 64^3 box ({sample.n} particles), {dt:.2f} s"}


def cpu_baseline(args, case):
    """The oracle, as it stands, on the main workload itself (or a smaller box
    of the same lattice recipe, --cpu-sample): full FP64 steps (density,
    pressure, accelerations, integration) on the host's threads, each from
    the last one's state, until 10 s have passed (at most 8 steps); each step
    is credited with the first step's interaction count."""
    import numpy as np

    from oracle import oracle as O
    from paper_1710_08259_amd import workloads as WL

    side = tuple(int(s) for s in args.cpu_sample.split("x"))
    sample = case if side == (256, 256, 128) else WL.lattice_case(3, side, 0.01, 1.2, 0.05, 0.05, seed=3,
                                                                   c0=case.c0, nu=case.nu, dt=case.dt)
    dom = O.Domain(dim=3, n=sample.ncell, cs=sample.cell_size, origin=sample.origin)
    prm = O.Params(h=sample.h, mass=sample.mass, rho0=sample.rho0, c0=sample.c0, gamma=sample.gamma,
                   nu=sample.nu, dt=sample.dt, g=sample.g)
    threads = O.default_threads()
    x = sample.pos.astype(np.float64)
    v = sample.vel.astype(np.float64)
    _, _, counts = O.density(dom, prm, x, counts=True, nthreads=threads)
    pairs = int(counts.sum())
    dt, steps = 0.0, 0
    while dt < 10.0 and steps < 8:
        t0 = time.perf_counter()
        x, v, _, _, _ = O.step(dom, prm, x, v, n_steps=1, nthreads=threads)
        dt += time.perf_counter() - t0
        steps += 1
    return {"value": pairs * steps / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} FP64 steps of the {side[0]}x{side[1]}x{side[2]} lattice ({sample.n} particles, "
                      f"{pairs} interactions in the first{'' if sample is case else '; a smaller box of the same recipe'}), "
                      f"{dt:.2f} s"}


def adjoint_extra(device):
    """Forward and forward+adjoint steps/s of the 262,144-particle 3-D case
    over a segment of 20 steps, in the rollout's two modes:
      - kept records (the default wherever every step's record fits in half
        the free device memory; a 200-step rollout of this case takes ~31 GB
        of the 288): the forward pass keeps each step's sorted state, lists
        and fields, and the reverse sweep runs the adjoint passes only;
      - checkpoints: plain forward steps, then each segment recomputed with
        its records before the adjoint passes.
    Next to them, the FP64 oracle's forward + adjoint step on the same
    case."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL
    from paper_1710_08259_amd.rollout import Rollout, record_bytes

    case = WL.periodic_3d_262k()
    prob = N.Problem([case], device=device)
    st = prob.state_from_cases()
    K = 20
    prob.step(st, 2)
    torch.cuda.synchronize()
    ck = st.clone()
    lam = {"x": [torch.full((prob.n,), 1e-3, device=device) for _ in range(3)],
           "v": [torch.zeros(prob.n, device=device) for _ in range(3)],
           "ox": [torch.empty(prob.n, device=device) for _ in range(3)],
           "ov": [torch.empty(prob.n, device=device) for _ in range(3)]}
    dnu = torch.zeros(1, dtype=torch.float64, device=device)
    dc0 = torch.zeros(1, dtype=torch.float64, device=device)

    def timed(fn):
        fn()  # warm (allocator, modules)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    def plain_forward():
        cur = ck.clone()
        prob.step(cur, K)

    def recorded_forward():
        cur = ck.clone()
        return Rollout._record_steps(prob, cur, K)

    def sweep(records):
        for rec in reversed(records):
            prob.adjoint(rec.sorted, rec.cells, rec.fields, lam["x"], lam["v"], lam["ox"], lam["ov"], dnu, dc0)
            lam["x"], lam["ox"] = lam["ox"], lam["x"]
            lam["v"], lam["ov"] = lam["ov"], lam["v"]

    t_fwd, _ = timed(plain_forward)
    t_fwd_rec, records = timed(recorded_forward)
    t_adj, _ = timed(lambda: sweep(records))
    t_rev, _ = timed(lambda: sweep(recorded_forward()))  # checkpoint mode: recompute, then sweep
    prob.check()
    # the oracle: one FP64 forward step and one step VJP on the same case
    dom = O.Domain(dim=3, n=case.ncell, cs=case.cell_size, origin=case.origin)
    prm = O.Params(h=case.h, mass=case.mass, rho0=case.rho0, c0=case.c0, gamma=case.gamma, nu=case.nu,
                   dt=case.dt, g=case.g)
    x, v = case.pos.astype(np.float64), case.vel.astype(np.float64)
    threads = O.default_threads()
    t0 = time.perf_counter()
    O.step(dom, prm, x, v, n_steps=1, nthreads=threads)
    O.step_vjp(dom, prm, x, v, np.ones_like(x), np.zeros_like(v), nthreads=threads)
    t_or = time.perf_counter() - t0
    fa_kept = K / (t_fwd_rec + t_adj)
    fa_ckpt = K / (t_fwd + t_rev)
    return {"workload": case.name, "particles": case.n, "segment_steps": K,
            "record_bytes_per_step": record_bytes(prob),
            "forward_steps_per_s": K / t_fwd, "recorded_forward_steps_per_s": K / t_fwd_rec,
            "adjoint_steps_per_s": K / t_adj, "adjoint_over_forward": t_adj / t_fwd,
            "fwd_plus_adjoint_steps_per_s": fa_kept,
            "checkpointed": {"checkpoint_every": K, "adjoint_with_recompute_steps_per_s": K / t_rev,
                             "adjoint_over_forward": t_rev / t_fwd, "fwd_plus_adjoint_steps_per_s": fa_ckpt},
            "oracle_fwd_plus_adjoint_steps_per_s": 1.0 / t_or, "oracle_cores": threads,
            "fwd_plus_adjoint_vs_oracle": fa_kept * t_or}


def batched_extra(device, steps=10, tuning=None):
    """The 256-case batched workload, launch shape picked by the autotuner
    (or the given one)."""
    from paper_1710_08259_amd import autotune
    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    cases = WL.batched_2d()
    if tuning is not None:
        best, timings = tuning, {}
    else:
        cands = (N.Tuning(), N.Tuning(block=128), N.Tuning(block=128, persistent=1, groups_per_cu=0),
                 N.Tuning(block=256, persistent=1, groups_per_cu=0))
        cache = os.environ.get("NAUTICLE_TUNING_CACHE",
                               os.path.join(tempfile.gettempdir(), "nauticle_tuning.json"))
        best, timings = autotune.tune(cases, steps=2, candidates=cands, cache_path=cache, force=True)
    prob = N.Problem(cases, device=device, tuning=best)
    st = prob.state_from_cases()
    wall, phase, pairs = timed_steps(prob, st, steps, 2)
    return {"workload": f"batched_2d_{len(cases)}_cases", "particles": prob.n, "cases": len(cases),
            "tuning": best.__dict__, "steps_per_s": steps / wall, "interactions_per_s": pairs / wall,
            "tuning_ms_per_step": {f"{t.block}/{t.persistent}/{t.groups_per_cu}": round(v, 4)
                                   for t, v in timings.items()}}


def dam_break_extra(device, steps=10):
    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    case = WL.dam_break_3d()
    prob = N.Problem([case], device=device)
    st = prob.state_from_cases()
    wall, phase, pairs = timed_steps(prob, st, steps, 2)
    return {"workload": case.name, "particles": case.n, "fixed": case.n_fixed, "steps_per_s": steps / wall,
            "interactions_per_s": pairs / wall, "ms_per_step": wall * 1e3 / steps}


def small_extra(device, steps=200, per_graph=20):
    """The 4,096-particle 2-D periodic lattice, bound by the latency of its
    kernels rather than by any one of them, in the launch shape the
    autotuner picks: ms per step with one nauticle_step call per step from
    Python, and with per_graph steps captured once in a HIP graph and
    replayed (the library's launches are all capturable)."""
    import torch

    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    from paper_1710_08259_amd import autotune

    case = WL.periodic_2d_4096()
    cache = os.environ.get("NAUTICLE_TUNING_CACHE", os.path.join(tempfile.gettempdir(), "nauticle_tuning.json"))
    best, timings = autotune.tune([case], steps=5, cache_path=cache, device=device, force=True)
    prob = N.Problem([case], device=device, tuning=best)
    st = prob.state_from_cases()
    for _ in range(5):
        prob.step(st, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.step(st, 1)
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / steps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        prob.step(st, per_graph)
    g.replay()
    torch.cuda.synchronize()
    reps = max(steps // per_graph, 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) / (reps * per_graph)
    prob.check()
    pairs = float(prob.cells.nbr_count[: case.n].sum().item())
    return {"workload": case.name, "particles": case.n, "tuning": best.__dict__,
            "tuning_ms_per_step": {f"{t.block}/{t.persistent}/{t.groups_per_cu}": round(v, 4)
                                   for t, v in (timings or {}).items()},
            "eager_ms_per_step": round(eager * 1e3, 4),
            "graph_ms_per_step": round(graph * 1e3, 4), "steps_per_graph": per_graph,
            "graph_steps_per_s": 1.0 / graph, "graph_interactions_per_s": pairs / graph}


def largest_extra(device, steps=5, warmup=2):
    """The largest lattice of the headline recipe under the 26-bit index
    limit of a list entry: 512 x 512 x 255 sites (66,846,720 particles),
    whole steps as the headline line times them, with the device memory
    the table holds."""
    import torch

    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    case = WL.lattice_case(3, (512, 512, 255), 0.01, 1.2, 0.05, 0.05, seed=3, c0=10.0, nu=1e-3, dt=1e-4,
                           name="periodic_3d_66846720")
    torch.cuda.reset_peak_memory_stats()
    prob = N.Problem([case], device=device)
    st = prob.state_from_cases()
    wall, phase, pairs = timed_steps(prob, st, steps, warmup)
    prob.check()
    out = {"workload": case.name, "particles": case.n, "cells": list(case.ncell),
           "ms_per_step": round(wall * 1e3 / steps, 3), "interactions_per_s": pairs / wall,
           "phases": {"sort_reorder_ms": round(phase[0], 4), "neighbour_lists_ms": round(phase[1], 4),
                      "density_ms": round(phase[2], 4), "forces_integrate_ms": round(phase[3], 4)},
           "device_gib": round(torch.cuda.max_memory_allocated() / 2**30, 1)}
    del prob, st
    return out


def paper_shape_extra(device, passes=50):
    """The shape of the paper's performance benchmark: density-summation
    passes (nauticle_sph_density, lists built once) on 3-D periodic lattices
    of 15^3 ... 100^3 sites with h = 1.05 dx, in particles per second per
    pass: event-timed on the library's stream with one call per pass from
    Python, and with the passes captured once in a HIP graph and replayed
    (no host launch per pass).  Beside it, the FP64 oracle's density pass on
    the 15^3 lattice on one host thread.  Context only: the paper's own
    figure is a CPU's, with an evaluation count it does not state."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    out = {"h_over_dx": 1.05, "sizes": []}
    for side in (15, 22, 47, 100):
        case = WL.lattice_case(3, (side,) * 3, 0.01, 1.05, 0.0, 0.0, seed=side, name=f"paper_shape_{side}")
        prob = N.Problem([case], device=device)
        st = prob.state_from_cases()
        prob.build_cells(st)
        for _ in range(3):
            prob.density()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(passes):
            prob.density()
        e1.record(stream)
        torch.cuda.synchronize()
        prob.check()
        ms = e0.elapsed_time(e1) / passes
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(passes):
                prob.density()
        g.replay()
        torch.cuda.synchronize()
        reps = 5
        e0.record(stream)
        for _ in range(reps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        prob.check()
        gms = e0.elapsed_time(e1) / (reps * passes)
        nbr = float(prob.cells.nbr_count[: case.n].sum().item()) / case.n
        out["sizes"].append({"particles": case.n, "ms_per_pass": round(ms, 5),
                             "particles_per_s": case.n / (ms * 1e-3),
                             "graph_ms_per_pass": round(gms, 5), "graph_particles_per_s": case.n / (gms * 1e-3),
                             "neighbours_per_particle": round(nbr, 2)})
        del g
        del prob, st
    case = WL.lattice_case(3, (15,) * 3, 0.01, 1.05, 0.0, 0.0, seed=15)
    dom = O.Domain(dim=3, n=case.ncell, cs=case.cell_size, origin=case.origin)
    prm = O.Params(h=case.h, mass=case.mass, rho0=case.rho0, c0=case.c0, gamma=case.gamma, nu=case.nu,
                   dt=case.dt, g=case.g)
    x = case.pos.astype(np.float64)
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < 1.0:
        O.density(dom, prm, x, nthreads=1)
        reps += 1
    out["oracle_15^3_one_thread"] = {"particles_per_s": case.n * reps / (time.perf_counter() - t0),
                                     "cores": 1, "kind": "oracle"}
    return out


def ex1a_extra(device, scale, steps=10, warmup=2):
    """Example 1a's 2-D dam break (continuity, linear EOS, artificial
    viscosity, symmetric faces), refined by `scale`, from rest, in the launch
    shape the autotuner picks; next to it the FP64 oracle's step on the
    paper's own 558-particle column."""
    import numpy as np

    from oracle import oracle as O
    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    from paper_1710_08259_amd import autotune

    case = WL.ex1a_dam_break(scale)
    cache = os.environ.get("NAUTICLE_TUNING_CACHE", os.path.join(tempfile.gettempdir(), "nauticle_tuning.json"))
    best, timings = autotune.tune([case], steps=3, candidates=(N.Tuning(), N.Tuning(block=128), N.Tuning(block=64)),
                                  cache_path=cache, device=device, force=True)
    prob = N.Problem([case], device=device, tuning=best)
    st = prob.state_from_cases()
    wall, phase, pairs = timed_steps(prob, st, steps, warmup)
    del prob, st
    small = WL.ex1a_dam_break(1.0)
    dom = O.Domain(dim=2, n=small.ncell, cs=small.cell_size, origin=small.origin, periodic=(False,) * 3,
                   symmetric=(True, True, False))
    prm = O.Params(h=small.h, mass=small.mass, rho0=small.rho0, c0=small.c0, gamma=small.gamma, nu=small.nu,
                   dt=small.dt, g=small.g, alpha_av=small.alpha_av)
    x = small.pos.astype(np.float64)
    k_or = 20
    t0 = time.perf_counter()
    O.step_ex1a(dom, prm, x, np.zeros_like(x), small.rho.astype(np.float64), n_steps=k_or, nthreads=1)
    t_or = (time.perf_counter() - t0) / k_or
    return {"workload": case.name, "particles": case.n, "cells": list(case.ncell), "scale": scale,
            "tuning": best.__dict__,
            "tuning_ms_per_step": {f"{t.block}/{t.persistent}/{t.groups_per_cu}": round(v, 4)
                                   for t, v in (timings or {}).items()},
            "steps_per_s": steps / wall, "ms_per_step": round(wall * 1e3 / steps, 4),
            "interactions_per_s": pairs / wall, "neighbours_per_particle": round(pairs / steps / case.n, 2),
            "phases": {"sort_reorder_ms": round(phase[0], 4), "neighbour_lists_ms": round(phase[1], 4),
                       "continuity_ms": round(phase[2], 4), "momentum_integrate_ms": round(phase[3], 4)},
            "oracle_paper_case": {"particles": small.n, "ms_per_step": round(t_or * 1e3, 3), "cores": 1}}


def verlet_extra(device, skin_frac=0.1, steps=100, warmup=5, pairs_2h_per_step=None, plain_ms=None):
    """The main workload's lattice stepped with neighbour lists reused
    between builds: lists reaching 2h + skin (skin = skin_frac 2h, cells
    resized to fit), a build only before a step at whose start a particle
    has moved about skin / 2 since the last one.  Reports the builds, the
    mean step and its phases over the build and the reuse steps."""
    import numpy as np
    import torch

    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    base = WL.periodic_3d_8m()
    skin = skin_frac * 2.0 * base.h
    case = WL.lattice_case(3, (256, 256, 128), 0.01, 1.2, 0.05, 0.05, seed=3, c0=10.0, nu=1e-3, dt=1e-4,
                           skin=skin, name=f"periodic_3d_8388608_skin{skin_frac:g}")
    prob = N.Problem([case], device=device)
    st = prob.state_from_cases()
    prob.step_verlet(st, warmup)  # loads every kernel module
    torch.cuda.synchronize()
    prob.check()
    # the timed run records no events (the next step's first pass is then queued ahead of the
    # host's wait for the rebuild word); a second run with phase events gives the breakdown
    t0 = time.perf_counter()
    builds = prob.step_verlet(st, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prob.check()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(5 * steps)]
    for e in evs:
        e.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prob.step_verlet(st, steps, events=evs)
    torch.cuda.synchronize()
    wall_events = time.perf_counter() - t1
    prob.check()
    per = np.array([[evs[5 * k + i].elapsed_time(evs[5 * k + i + 1]) for i in range(4)] for k in range(steps)])
    built = per[:, 0] + per[:, 1] > 0.02
    entries = float(prob.cells.nbr_count[: case.n].sum(dtype=torch.int64).item())
    out = {"workload": case.name, "particles": case.n, "cells": list(case.ncell), "skin": skin,
           "skin_over_2h": skin_frac, "steps": steps, "builds": builds,
           "ms_per_step": round(wall * 1e3 / steps, 4), "steps_per_s": steps / wall,
           "with_phase_events": {"ms_per_step": round(wall_events * 1e3 / steps, 4),
                                 "gpu_ms_per_step": round(float(per.sum(axis=1).mean()), 4)},
           "list_entries_per_particle": round(entries / case.n, 2),
           "reuse_step_ms": {"density": round(float(per[~built, 2].mean()), 4),
                             "forces_drift": round(float(per[~built, 3].mean()), 4)} if (~built).any() else None,
           "build_step_ms": {"sort_reorder": round(float(per[built, 0].mean()), 4),
                             "neighbour_lists": round(float(per[built, 1].mean()), 4)} if built.any() else None}
    if pairs_2h_per_step:
        out["interactions_per_s"] = pairs_2h_per_step * steps / wall
    if plain_ms:
        out["speedup_vs_build_every_step"] = round(plain_ms / (wall * 1e3 / steps), 3)
    return out


def dem_verlet_extra(device, skin_frac=0.1, steps=100, warmup=5, plain_ms=None):
    """The DEM bed of the pair-law extra (3,889,053 spheres packed at 0.99
    of their diameter) stepped with contact lists reused between builds:
    lists reaching 2R + skin (skin = skin_frac 2R, cells resized to fit)."""
    import torch

    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    skin = skin_frac * 2.0 * 0.004
    case = WL.dem_damper(19, spacing=2 * 0.004 * 0.99, jitter=0.05, skin=skin,
                         name=f"dem_damper_3889053_skin{skin_frac:g}")
    best, _ = law_tuning(case, 32, device, force=False)
    prob = N.Problem([case], device=device, max_nbr=32, tuning=best)
    st = prob.state_from_cases()
    attrs = prob.law_attrs()
    prob.step_verlet(st, warmup, attrs=attrs)
    torch.cuda.synchronize()
    prob.check()
    t0 = time.perf_counter()
    builds = prob.step_verlet(st, steps, attrs=attrs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prob.check()
    out = {"workload": case.name, "particles": case.n, "cells": list(case.ncell), "skin": skin,
           "skin_over_2h": skin_frac, "tuning": best.__dict__, "steps": steps, "builds": builds,
           "ms_per_step": round(wall * 1e3 / steps, 4), "steps_per_s": steps / wall}
    if plain_ms:
        out["speedup_vs_build_every_step"] = round(plain_ms / (wall * 1e3 / steps), 3)
    return out


LAW_TUNING = None  # a fixed launch shape for the pair-law workloads (--law-tuning), else the autotuner's


def law_tuning(case, max_nbr, device, force):
    """The autotuner's launch shape for a pair-law case (measured now when
    `force`, else from its cache when there), and the timings it measured;
    or the shape fixed on the command line."""
    from paper_1710_08259_amd import autotune
    from paper_1710_08259_amd import nauticle as N

    if LAW_TUNING is not None:
        return LAW_TUNING, {}

    cands = (N.Tuning(), N.Tuning(block=128), N.Tuning(block=64), N.Tuning(block=128, persistent=1, groups_per_cu=0))
    cache = os.environ.get("NAUTICLE_TUNING_CACHE", os.path.join(tempfile.gettempdir(), "nauticle_tuning.json"))
    best, timings = autotune.tune([case], steps=3, candidates=cands, cache_path=cache, device=device, force=force,
                                  max_nbr=max_nbr)
    return best, timings or {}


def law_extra(device, which, steps=10, warmup=2):
    """A pair law at scale: Example 2's DEM damper with 19^3 times the
    table's 567 spheres (3,889,053, symmetric faces) packed at 0.99 of their
    diameter (every sphere touching its lattice neighbours, a compressed
    bed), or the social force room of side 800 m (654,394 people, fixed
    walls), in the launch shape the autotuner picks for it; next to it the
    FP64 oracle's step on the paper-size case (the 567 spheres packed the
    same way / a 20 m room)."""
    import numpy as np

    from oracle import oracle as O
    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    packed = dict(spacing=2 * 0.004 * 0.99, jitter=0.05)
    case = WL.dem_damper(19, **packed) if which == "dem" else WL.social_room(width=800.0)
    max_nbr = 32 if which == "dem" else 64
    best, timings = law_tuning(case, max_nbr, device, force=True)
    prob = N.Problem([case], device=device, max_nbr=max_nbr, tuning=best)
    st = prob.state_from_cases()
    attrs = prob.law_attrs()
    wall, phase, pairs = timed_steps(prob, st, steps, warmup,
                                     step=lambda s_, ev: prob.step_law(s_, attrs, 1, events=ev))
    del prob, st
    small = WL.dem_damper(1, **packed) if which == "dem" else WL.social_room(width=20.0)
    dom = O.Domain(dim=small.dim, n=small.ncell, cs=small.cell_size, origin=small.origin,
                   periodic=tuple(b == WL.PERIODIC for b in small.boundary),
                   symmetric=tuple(b == WL.SYMMETRIC for b in small.boundary))
    prm = O.Params(h=small.h, mass=small.mass, rho0=small.rho0, c0=small.c0, gamma=small.gamma, nu=small.nu,
                   dt=small.dt, g=small.g, law=tuple(small.law) + (0.0,) * (4 - len(small.law)))
    k_or = 20
    t0 = time.perf_counter()
    O.step_law(which, dom, prm, small.pos.astype(np.float64), small.vel.astype(np.float64), small.radius,
               small.pmass, small.coef, v0=small.v0, goal=small.goal, fixed=small.fixed_mask(), n_steps=k_or,
               nthreads=1)
    t_or = (time.perf_counter() - t0) / k_or
    return {"workload": case.name, "particles": case.n, "fixed": case.n_fixed, "cells": list(case.ncell),
            "tuning": best.__dict__,
            "tuning_ms_per_step": {f"{t.block}/{t.persistent}/{t.groups_per_cu}": round(v, 4)
                                   for t, v in timings.items()},
            "steps_per_s": steps / wall, "ms_per_step": round(wall * 1e3 / steps, 4),
            "pairs_within_2h_per_s": pairs / wall, "pairs_per_particle": round(pairs / steps / case.n, 2),
            "phases": {"sort_reorder_ms": round(phase[0], 4), "neighbour_lists_ms": round(phase[1], 4),
                       "pair_law_integrate_ms": round(phase[3], 4)},
            "oracle_paper_case": {"particles": small.n, "ms_per_step": round(t_or * 1e3, 3), "cores": 1}}


def ch_extra(device, dx=0.005, steps=20, warmup=3):
    """Example 1b refined: the Cahn-Hilliard equation on a Fibonacci sphere
    of radius 2 m at dx = 0.005 (2,010,619 points; the paper's dx = 0.07
    gives 10,258), lists built once (fixed particles), steps timed with the
    device-side adaptive dt; next to it the FP64 oracle's step at the
    paper's dx."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    case = WL.ch_sphere(dx=dx)
    prob = N.Problem([case], device=device, max_nbr=32)
    st = prob.state_from_cases()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.build_cells(st)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    perm = prob.cells.perm[: case.n].long()
    c = torch.from_numpy(case.coef).to(device)[perm].contiguous()
    clock = torch.tensor([0.0, case.dt], dtype=torch.float64, device=device)
    prob.ch_steps(c, clock, warmup)
    torch.cuda.synchronize()
    pairs = int(prob.cells.nbr_count[: case.n].sum(dtype=torch.int64).item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    prob.ch_steps(c, clock, steps)
    e1.record()
    torch.cuda.synchronize()
    prob.check()
    ms = e0.elapsed_time(e1) / steps
    t_sim, dt_now = clock.cpu().tolist()
    small = WL.ch_sphere()
    dom = O.Domain(dim=3, n=small.ncell, cs=small.cell_size, origin=small.origin, periodic=(True,) * 3)
    prm = O.Params(h=small.h, mass=small.mass, rho0=small.rho0, law=tuple(small.law) + (0.0,))
    k_or = 5
    t0 = time.perf_counter()
    O.ch_steps(dom, prm, small.pos.astype(np.float64), small.coef.astype(np.float64), 0.0, small.dt, k_or,
               nthreads=1)
    t_or = (time.perf_counter() - t0) / k_or
    return {"workload": case.name, "particles": case.n, "cells": list(case.ncell), "dx": dx,
            "ms_per_step": round(ms, 4), "steps_per_s": 1e3 / ms, "pairs_per_particle": round(pairs / case.n, 2),
            "laplacian_pairs_per_s": 2 * pairs / (ms * 1e-3), "lists_built_once_ms": round(t_build * 1e3, 2),
            "sim_time": t_sim, "dt": dt_now,
            "oracle_paper_case": {"particles": small.n, "ms_per_step": round(t_or * 1e3, 3), "cores": 1}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU sharding is "
              f"described in the design notes but not built", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1710_08259_amd import nauticle as N
    from paper_1710_08259_amd import workloads as WL

    device = "cuda:0"
    if args.law_tuning:
        global LAW_TUNING
        b, p, g = (int(v) for v in args.law_tuning.split("/"))
        LAW_TUNING = N.Tuning(block=b, persistent=p, groups_per_cu=g)
    if args.ch_only:
        print(json.dumps({"extra": {"ch": ch_extra(device)}}), flush=True)
        return
    if args.law_only:
        print(json.dumps({"extra": {args.law_only: law_extra(device, args.law_only, args.steps, args.warmup)}}),
              flush=True)
        return
    if args.only:
        tn = None
        if args.batched_tuning:
            b, p, g = (int(v) for v in args.batched_tuning.split("/"))
            tn = N.Tuning(block=b, persistent=p, groups_per_cu=g)
        fn = {"adjoint": lambda: adjoint_extra(device), "batched": lambda: batched_extra(device, tuning=tn),
              "dam_break": lambda: dam_break_extra(device), "paper_shape": lambda: paper_shape_extra(device),
              "small": lambda: small_extra(device), "largest": lambda: largest_extra(device)}[args.only]
        print(json.dumps({"extra": {args.only: fn()}}), flush=True)
        return
    if args.ex1a_only:
        print(json.dumps({"extra": {"ex1a": ex1a_extra(device, args.ex1a_scale, args.steps, args.warmup)}}),
              flush=True)
        return
    if args.verlet_only:
        print(json.dumps({"extra": {"verlet": verlet_extra(device, args.skin_frac, max(args.steps, 20)),
                                    "dem_verlet": dem_verlet_extra(device, args.skin_frac, max(args.steps, 20))}}),
              flush=True)
        return
    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        a = torch.empty(nb // 4, dtype=torch.float32, device=device).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    case = WL.periodic_3d_8m()
    prob = N.Problem([case], device=device)
    st = prob.state_from_cases()
    wall, phase_ms, total_pairs = timed_steps(prob, st, args.steps, args.warmup)
    pairs_per_step = total_pairs / args.steps
    cand = candidates_per_step(prob, case)
    search_s = phase_ms[1] * 1e-3
    force_s = phase_ms[3] * 1e-3
    search_tflops = SEARCH_FLOP_PER_CANDIDATE * cand / search_s / 1e12
    force_tflops = FORCE_FLOP_PER_PAIR * pairs_per_step / force_s / 1e12
    # the kernels are built without packed FP32: the FP32 vector peak that applies is the unpacked one
    roofline = {"bound": "alu", "kernel": "k_nlist (neighbour-list search)",
                "achieved": round(search_tflops, 3), "peak": PEAK_FP32_TFLOPS_UNPACKED, "unit": "TFLOP/s",
                "frac": round(search_tflops / PEAK_FP32_TFLOPS_UNPACKED, 4), "traffic": nlist_traffic(),
                "peak_published_packed_fp32": PEAK_FP32_TFLOPS,
                "valu_per_simd_4_cycles": nlist_valu_rate(),
                "lane_slots_per_candidate": nlist_lane_slots_per_candidate(cand),
                "candidates_per_step": cand, "ms": round(phase_ms[1], 4)}
    line = {
        "metric": "particle-pair interactions/s (SPH force pass) + fwd+adjoint steps/s vs plain",
        "value": total_pairs / wall, "unit": "interactions/s",
        "value_is": "ordered neighbour pairs (FP32 predicate) per whole step (sort, search, density, "
                    "forces + integrate) / wall time of the timed steps",
        "force_pass_interactions_per_s": pairs_per_step / force_s,
        "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": case.name, "particles": case.n, "dim": case.dim, "h_over_dx": 1.2,
                   "neighbours_per_particle": round(pairs_per_step / case.n, 2),
                   "candidates_per_particle": round(cand / case.n, 1),
                   "cells": list(case.ncell), "max_nbr": prob.max_nbr},
        "phases": {"sort_reorder_ms": round(phase_ms[0], 4), "neighbour_lists_ms": round(phase_ms[1], 4),
                   "density_ms": round(phase_ms[2], 4), "forces_integrate_ms": round(phase_ms[3], 4),
                   "gpu_ms_per_step": round(float(phase_ms.sum()), 4),
                   "force_pass_interactions_per_s": pairs_per_step / force_s},
        "roofline": roofline,
        "extra": {"roofline_force_pass": {
            "bound": "alu", "kernel": "k_forces<true> (force pass with fused integration)",
            "achieved": round(force_tflops, 3), "peak": PEAK_FP32_TFLOPS_UNPACKED, "unit": "TFLOP/s",
            "frac": round(force_tflops / PEAK_FP32_TFLOPS_UNPACKED, 4), "ms": round(phase_ms[3], 4),
            "l1_accesses_per_cu_clock": force_l1_rate()},
            "hbm": hbm_fractions(case.n, phase_ms)},
    }
    del prob, st
    torch.cuda.empty_cache()
    if not args.no_extra:
        line["extra"]["adjoint"] = adjoint_extra(device)
        torch.cuda.empty_cache()
        line["extra"]["batched"] = batched_extra(device)
        torch.cuda.empty_cache()
        line["extra"]["dam_break"] = dam_break_extra(device)
        torch.cuda.empty_cache()
        line["extra"]["ex1a"] = ex1a_extra(device, args.ex1a_scale)
        torch.cuda.empty_cache()
        line["extra"]["dem"] = law_extra(device, "dem")
        torch.cuda.empty_cache()
        line["extra"]["social"] = law_extra(device, "social")
        torch.cuda.empty_cache()
        line["extra"]["ch"] = ch_extra(device)
        torch.cuda.empty_cache()
        line["extra"]["paper_shape"] = paper_shape_extra(device)
        torch.cuda.empty_cache()
        line["extra"]["small"] = small_extra(device)
        torch.cuda.empty_cache()
        line["extra"]["largest"] = largest_extra(device)
        torch.cuda.empty_cache()
        line["extra"]["verlet"] = verlet_extra(device, args.skin_frac, pairs_2h_per_step=pairs_per_step,
                                               plain_ms=wall * 1e3 / args.steps)
        torch.cuda.empty_cache()
        line["extra"]["dem_verlet"] = dem_verlet_extra(device, args.skin_frac,
                                                       plain_ms=line["extra"]["dem"]["ms_per_step"])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args, case)
        line["extra"]["cpu_single_thread"] = cpu_single_thread(case)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
