#!/usr/bin/env python3
"""Throughput of the DUWP particle pipeline on one MI355X.

Workload: Mach-8 argon shock, 4000 cells over 200 upstream mean free paths,
5e7 simulated particles (synthetic, seeded).  The timed path stores particles
in FP32 (position relative to its cell) with FP64 cell moments, NS wave update
and absorption fractions; the plain FP64 path is timed on the same workload
beside it.  A step is one full DUWP time step of every stage, replayed as a
captured HIP graph.  Metric: particle-steps per second (particles alive at the
start of each step, summed over the timed steps, over the wall time).

Also reported: the batched form (256 independent uneven shock and Sod cases in
one context, one launch per stage), the roofline of the dominant kernel and the
CPU oracle on the same state.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec on Mach-8 argon shock (FP32+FP64 vs FP64) + % HBM peak"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per particle of the particle-streaming kernels, per
# element size s of the particle arrays (4 in FP32 mode, 8 in FP64 mode): the
# scatter reads x,u,v,w of each particle and writes them to its sorted place;
# absorb_resample reads and writes them once for the cells that absorb or
# resample (counted over all particles of the step, an upper bound).
BYTES_PER_PARTICLE = {
    "scatter": lambda s: 8 * s,
    "absorb_resample": lambda s: 8 * s,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("duwp_kernels.hip", "duwp_physics.hpp", "duwp_device.hpp", "duwp_scan.hpp")


def counted_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE runs, each scaled by a plain copy of known size), or
    None when the kernel sources changed since the counters were taken."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_12071_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        with open(path) as fh:
            d = json.load(fh)
        if d.get("kernel") == kernel and d.get("workload") == workload \
                and d.get("kernel_sources_sha256") == h.hexdigest():
            return d["hbm_bytes_per_launch"], d["particles_per_launch"]
    return None


def run_path(cases, precision, steps, warmup, graph, seed=1, block_cells=0):
    from paper_2305_12071_amd import duwp
    import torch

    sim = duwp.Sim(cases, seed=seed, precision=precision, use_graph=graph, block_cells=block_cells)
    t = time.perf_counter()
    sim.step(warmup)
    log(f"  warmup {warmup} steps in {time.perf_counter() - t:.2f}s, N={sim.total_particles()}")
    sim.particle_steps(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)          # returns after the device finished (error word read back)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ps = sim.particle_steps(reset=True)
    return sim, ps, t1 - t0


def block_size(cases, precision, args):
    """Block size of the per-cell kernels: fixed, tuned now, cached, or 256."""
    from paper_2305_12071_amd import autotune
    if args.block_cells:
        return args.block_cells, "fixed"
    if args.autotune:
        return autotune.tune(cases, precision, path=args.tune_cache, log=log), "tuned"
    bc = autotune.lookup(cases, precision)
    return (bc, "cache") if bc else (256, "default")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cells", type=int, default=4000)
    ap.add_argument("--particles", type=float, default=5e7)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--block-cells", type=int, default=0, help="threads per block of the per-cell kernels")
    ap.add_argument("--autotune", action="store_true", help="time the block-size candidates first")
    ap.add_argument("--tune-cache", default=None, help="file --autotune writes (default: the package cache)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched form")
    ap.add_argument("--batched-cases", type=int, default=256)
    ap.add_argument("--batched-steps", type=int, default=50)
    ap.add_argument("--batched-vs-single", action="store_true",
                    help="also time the batched cases one context per case")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the pipeline would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_12071_amd import duwp
    from paper_2305_12071_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    duwp.lib()
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    case = I.mach8_shock(args.cells, args.particles)
    graph = not args.no_graph

    bc, bc_src = block_size([case], duwp.MIXED, args)
    log(f"mixed FP32+FP64 path: {case.name}, block_cells={bc} ({bc_src})")
    sim, ps, dt = run_path([case], duwp.MIXED, args.steps, args.warmup, graph, block_cells=bc)
    value = ps / dt
    n_now = sim.total_particles()
    log(f"  {args.steps} steps in {dt:.3f}s -> {value:.4e} particle-steps/s")

    # per-kernel device time (HIP events on the library's stream, eager launches)
    kms = sim.profile(args.profile_steps)
    prof_ps = sim.particle_steps(reset=True) / args.profile_steps
    dom = max((k for k in kms if k in BYTES_PER_PARTICLE), key=lambda k: kms[k])
    alg_bytes = BYTES_PER_PARTICLE[dom](4) * prof_ps
    achieved = alg_bytes / (kms[dom] * 1e-3) / 1e9
    kname = {"scatter": "k_scatter<float>", "absorb_resample": "k_absorb_resample<float>"}.get(dom)
    tr = counted_traffic(kname, case.name) if kname else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": tr[0] if tr else None,
                "traffic_per_particle": round(tr[0] / tr[1], 2) if tr else None,
                "bytes_per_particle": BYTES_PER_PARTICLE[dom](4), "particles_per_launch": int(prof_ps),
                "kernel_ms": round(kms[dom], 4)}
    log("  kernels (ms):", json.dumps({k: round(v, 4) for k, v in kms.items()}))

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        log(f"CPU oracle: {args.cpu_steps} steps from the GPU state after warm-up")
        st = sim.get_state()
        sim.close()
        del sim
        orc = O.Oracle(case, seed=1, case_id=0)
        orc.set_state(st)
        n0 = len(st["x"])
        del st
        t = time.perf_counter()
        pst = 0
        for _ in range(args.cpu_steps):
            pst += orc.n
            orc.step(1)
        cdt = time.perf_counter() - t
        cpu = {"value": pst / cdt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"{case.name}: {args.cpu_steps} FP64 oracle steps from the warmed-up state "
                         f"({n0} particles), single thread, {cdt:.1f}s"}
        log(f"  oracle {cpu['value']:.3e} particle-steps/s")
        del orc
    else:
        sim.close()
        del sim

    fp64 = None
    bc64 = None
    if not args.no_fp64:
        bc64, src64 = block_size([case], duwp.FP64, args)
        log(f"plain FP64 path, block_cells={bc64} ({src64})")
        s64, ps64, dt64 = run_path([case], duwp.FP64, args.steps, args.warmup, graph, block_cells=bc64)
        fp64 = ps64 / dt64
        log(f"  {args.steps} steps in {dt64:.3f}s -> {fp64:.4e} particle-steps/s")
        s64.close()

    batched = None
    if not args.no_batched:
        cases = I.batched_cases(args.batched_cases)
        bcb, srcb = block_size(cases, duwp.MIXED, args)
        ncell = sum(c.ncells for c in cases)
        log(f"batched form: {len(cases)} cases, {ncell} cells, block_cells={bcb} ({srcb})")
        sb, psb, dtb = run_path(cases, duwp.MIXED, args.batched_steps, 5, graph, block_cells=bcb)
        batched = {"value": psb / dtb, "unit": "particle-steps/s", "cases": len(cases), "cells": ncell,
                   "particles": sb.total_particles(), "steps": args.batched_steps,
                   "ms_per_step": dtb / args.batched_steps * 1e3,
                   "precision": "fp32 particles + fp64 cells", "block_cells": bcb}
        batched["kernels_ms"] = {k: round(v, 4) for k, v in sb.profile(args.profile_steps).items()}
        sb.close()
        log(f"  {batched['value']:.4e} particle-steps/s, N={batched['particles']}")
        if args.batched_vs_single:
            tot_ps, tot_t = 0, 0.0
            for c in cases:
                s1, p1, t1 = run_path([c], duwp.MIXED, args.batched_steps, 5, graph, block_cells=bcb)
                s1.close()
                tot_ps += p1
                tot_t += t1
            batched["one_context_per_case"] = tot_ps / tot_t
            log(f"  one context per case: {batched['one_context_per_case']:.4e} particle-steps/s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": case.ncells, "particles": n_now,
                   "particles_target": args.particles, "precision": "fp32 particles + fp64 cells",
                   "graph": graph, "gas": "argon VHS omega=0.81", "mach": 8, "block_cells": bc},
        "fp64_value": fp64,
        "mixed_over_fp64": (value / fp64) if fp64 else None,
        "fp64_block_cells": bc64,
        "batched": batched,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
