#!/usr/bin/env python3
"""Throughput of the DUWP particle pipeline on one MI355X.

Headline workload: Mach-8 argon shock, 4000 cells over 200 upstream mean free
paths, 5e7 simulated particles (synthetic, seeded).  The timed path stores
particles in FP32 (position relative to its cell) with FP64 cell moments, NS
wave update and absorption fractions; the plain FP64 path is timed on the same
workload beside it.  A step is one full DUWP time step of every stage, replayed
as a captured HIP graph.  Metric: particle-steps per second (particles alive at
the start of each step, summed over the timed steps, over the wall time).

Also reported (legs): the batched form (256 independent uneven shock and Sod
cases in one context, against the plain FP64 path), the large near-continuum
Mach-10 case (20000 cells, 1e9 particles, most mass in the wave part), the
roofline of the dominant kernel, the step's effective bandwidth, the mixed
path's profile error (its time-averaged rho, U, T against the FP64 path's,
beside the gap between two FP64 seeds) and the CPU oracle on the same state.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec on Mach-8 argon shock (FP32+FP64 vs FP64) + % HBM peak"
HBM_PEAK_GBS = 8000.0
LEGS = ("main", "fp64", "batched", "large", "cpu")

# Algorithmic HBM bytes per particle of the particle-streaming kernels, per
# element size s of the particle arrays (4 in FP32 mode, 8 in FP64 mode): the
# scatter reads x,u,v,w of each particle and writes them to its sorted place;
# absorb_resample reads and writes them once for the cells that absorb or
# resample (counted over all particles of the step, an upper bound).
BYTES_PER_PARTICLE = {
    "scatter": lambda s: 8 * s,
    "absorb_resample": lambda s: 8 * s,
}
# Algorithmic bytes of a whole step per particle when almost nothing is absorbed:
# each particle's state (16 B in FP32 mode, 32 B in FP64 mode) is read and
# written once by the cell pass and once by the sort, four times the state.
STEP_BYTES_PER_PARTICLE = {"mixed": 64, "fp64": 128}
# The counted traffic of a kernel stays valid while its own source and the headers
# it uses are unchanged: the fingerprint covers the kernel's text in
# duwp_kernels.hip (from its template line to the next numbered section) and the
# device and physics headers.
KERNEL_HEADERS = ("duwp_physics.hpp", "duwp_device.hpp")


def kernel_fingerprint(kernel: str) -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_2305_12071_amd", "csrc")
    with open(os.path.join(csrc, "duwp_kernels.hip")) as fh:
        src = fh.read()
    name = kernel.split("<")[0]
    i0 = src.index(f") {name}(")
    i0 = src.rindex("template <typename T", 0, i0) if "<" in kernel else src.rindex("__global__", 0, i0)
    i1 = src.find("\n// ", i0 + 1)
    h = hashlib.sha256(src[i0:i1 if i1 > 0 else len(src)].encode())
    for f in KERNEL_HEADERS:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sources_fingerprint() -> str:
    """sha256 over every source file of the library (the counted traffic of a whole
    step stays valid while none of them changed)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2305_12071_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def counted_step(workload: str):
    """HBM bytes of one whole step (all kernels, FETCH_SIZE + WRITE_SIZE scaled as
    for the dominant kernel) and the particles of that step, from the committed
    counter summary, or None when any library source changed since."""
    import glob
    fp = sources_fingerprint()
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        with open(path) as fh:
            d = json.load(fh)
        if d.get("workload") == workload and d.get("sources_sha256") == fp and "step_hbm_bytes" in d:
            return d["step_hbm_bytes"], d["particles_per_launch"]
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counted_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE runs, each scaled by a plain copy of known size), or
    None when the kernel sources changed since the counters were taken."""
    import glob
    fp = kernel_fingerprint(kernel)
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        with open(path) as fh:
            d = json.load(fh)
        if d.get("kernel") == kernel and d.get("workload") == workload and d.get("kernel_sha256") == fp:
            return d["hbm_bytes_per_launch"], d["particles_per_launch"]
    return None


def run_path(cases, precision, steps, warmup, graph, seed=1, block_cells=0):
    from paper_2305_12071_amd import duwp
    import torch

    sim = duwp.Sim(cases, seed=seed, precision=precision, use_graph=graph, block_cells=block_cells)
    t = time.perf_counter()
    sim.step(warmup)
    log(f"  warmup {warmup} steps in {time.perf_counter() - t:.2f}s, N={sim.total_particles()}")
    sim.reset_average()      # the timed steps' time average (summed inside the step anyway)
    sim.particle_steps(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)          # returns after the device finished (error word read back)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ps = sim.particle_steps(reset=True)
    return sim, ps, t1 - t0


def profile_gap(a, b, R):
    """Gap of two time-averaged (rho, U, T) profiles summed over the cells: for rho
    and T relative to the sum of the second's values, for U relative to the sum
    of its thermal speeds sqrt(R T)."""
    out = {}
    for name, k in (("rho", 0), ("T", 4)):
        den = float(np.abs(b[:, k]).sum())
        out[name] = float(np.abs(a[:, k] - b[:, k]).sum() / den) if den > 0 else 0.0
    den = float(np.sqrt(R * np.abs(b[:, 4])).sum())
    out["U"] = float(np.abs(a[:, 1] - b[:, 1]).sum() / den) if den > 0 else 0.0
    return out


def profile_gap_cases(a, b, cases):
    """profile_gap per case, the largest over the cases."""
    gaps = [profile_gap(x, y, c.R) for x, y, c in zip(a, b, cases)]
    return {k: max(g[k] for g in gaps) for k in gaps[0]}


def block_size(cases, precision, args):
    """Block size of the per-cell kernels: fixed, tuned now, cached, or 256."""
    from paper_2305_12071_amd import autotune
    if args.block_cells:
        return args.block_cells, "fixed"
    if args.autotune:
        return autotune.tune(cases, precision, path=args.tune_cache, log=log), "tuned"
    bc = autotune.lookup(cases, precision)
    return (bc, "cache") if bc else (256, "default")


def roofline_of(sim, profile_steps, workload, block_cells):
    """Dominant particle-streaming kernel: algorithmic bytes over its event-timed duration."""
    kms = sim.profile(profile_steps)
    prof_ps = sim.particle_steps(reset=True) / profile_steps
    dom = max((k for k in kms if k in BYTES_PER_PARTICLE), key=lambda k: kms[k])
    alg_bytes = BYTES_PER_PARTICLE[dom](4) * prof_ps
    achieved = alg_bytes / (kms[dom] * 1e-3) / 1e9
    # the scatter's instance: one-wave blocks get the small-LDS variant
    scat = "k_scatter<float, 1, 2>" if block_cells == 64 else "k_scatter<float, 8, 4>"
    kname = {"scatter": scat, "absorb_resample": "k_absorb_resample<float>"}.get(dom)
    tr = counted_traffic(kname, workload) if kname else None
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": tr[0] if tr else None,
            "traffic_per_particle": round(tr[0] / tr[1], 2) if tr else None,
            "bytes_per_particle": BYTES_PER_PARTICLE[dom](4), "particles_per_launch": int(prof_ps),
            "kernel_ms": round(kms[dom], 4)}
    return roof, {k: round(v, 4) for k, v in kms.items()}


def leg_batched(args, graph, legs):
    from paper_2305_12071_amd import duwp
    from paper_2305_12071_amd import inputs as I
    cases = I.batched_cases(args.batched_cases)
    bcb, srcb = block_size(cases, duwp.MIXED, args)
    ncell = sum(c.ncells for c in cases)
    log(f"batched form: {len(cases)} cases, {ncell} cells, block_cells={bcb} ({srcb})")
    sb, psb, dtb = run_path(cases, duwp.MIXED, args.batched_steps, 5, graph, block_cells=bcb)
    out = {"value": psb / dtb, "unit": "particle-steps/s", "cases": len(cases), "cells": ncell,
           "particles": sb.total_particles(), "steps": args.batched_steps,
           "ms_per_step": dtb / args.batched_steps * 1e3,
           "precision": "fp32 particles + fp64 cells", "block_cells": bcb}
    avg_m = [sb.moments(k, duwp.M_AVG_PRIM) for k in range(len(cases))]
    out["kernels_ms"] = {k: round(v, 4) for k, v in sb.profile(args.profile_steps).items()}
    sb.close()
    log(f"  {out['value']:.4e} particle-steps/s, N={out['particles']}")
    if "fp64" in legs:
        bcf, srcf = block_size(cases, duwp.FP64, args)
        log(f"  batched plain FP64 path, block_cells={bcf} ({srcf})")
        sf, psf, dtf = run_path(cases, duwp.FP64, args.batched_steps, 5, graph, block_cells=bcf)
        avg_f = [sf.moments(k, duwp.M_AVG_PRIM) for k in range(len(cases))]
        sf.close()
        out["fp64_value"] = psf / dtf
        out["mixed_over_fp64"] = out["value"] / out["fp64_value"]
        log(f"  {out['fp64_value']:.4e} particle-steps/s")
        # profile error of the mixed path, as for the headline workload, per case
        sg, _, _ = run_path(cases, duwp.FP64, args.batched_steps, 5, graph, seed=2, block_cells=bcf)
        avg_g = [sg.moments(k, duwp.M_AVG_PRIM) for k in range(len(cases))]
        sg.close()
        out["profile_error"] = {
            "quantity": f"rho, U, T of each case averaged over the {args.batched_steps} timed steps",
            "norm": "sum over cells of |a - b| / sum over cells of |b| (rho, T) or of sqrt(R T) of b (U), the largest over the cases",
            "mixed_vs_fp64": profile_gap_cases(avg_m, avg_f, cases),
            "fp64_seed_to_seed": profile_gap_cases(avg_g, avg_f, cases)}
        log("  profile error:", json.dumps(out["profile_error"]))
    if args.batched_vs_single:
        # the same cases, one context each, plain FP64, one after another
        tot_ps, tot_t = 0, 0.0
        for c in cases:
            s1, p1, t1 = run_path([c], duwp.FP64, args.batched_steps, 5, graph)
            s1.close()
            tot_ps += p1
            tot_t += t1
        out["one_by_one_fp64"] = tot_ps / tot_t
        log(f"  one context per case, FP64: {out['one_by_one_fp64']:.4e} particle-steps/s")
    return out


def leg_large(args, graph):
    from paper_2305_12071_amd import duwp
    from paper_2305_12071_amd import inputs as I
    c = I.mach10_large(n_kept=args.large_particles)
    log(f"large near-continuum case: {c.name}, {args.large_particles:.0e} kept particles")
    sl, psl, dtl = run_path([c], duwp.MIXED, args.large_steps, 3, graph)
    out = {"value": psl / dtl, "unit": "particle-steps/s", "workload": c.name, "cells": c.ncells,
           "particles": sl.total_particles(), "steps": args.large_steps,
           "ms_per_step": dtl / args.large_steps * 1e3, "precision": "fp32 particles + fp64 cells"}
    d = sl.diag()
    out["absorbed_per_step"] = int(d["n_abs"].sum())
    out["resampled_per_step"] = int(d["n_new"].sum())
    out["collision_candidates_per_step"] = int(d["n_cand"].sum())
    wave = sl.moments(0, duwp.M_PSI_W)[:, 0].sum() / sl.moments(0, duwp.M_PSI_T)[:, 0].sum()
    out["wave_mass_fraction"] = round(float(wave), 4)
    out["kernels_ms"] = {k: round(v, 3) for k, v in sl.profile(1).items()}
    sl.close()
    log(f"  {out['value']:.4e} particle-steps/s, {out['ms_per_step']:.1f} ms/step, N={out['particles']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cells", type=int, default=4000)
    ap.add_argument("--particles", type=float, default=5e7)
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma list of " + ",".join(LEGS) + " (main is the headline value)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--block-cells", type=int, default=0, help="threads per block of the per-cell kernels")
    ap.add_argument("--autotune", action="store_true", help="time the block-size candidates first")
    ap.add_argument("--tune-cache", default=None, help="file --autotune writes (default: the package cache)")
    ap.add_argument("--no-fp64", action="store_true", help="leave out the fp64 leg")
    ap.add_argument("--no-batched", action="store_true", help="leave out the batched leg")
    ap.add_argument("--no-large", action="store_true", help="leave out the large leg")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="leave out the cpu leg")
    ap.add_argument("--batched-cases", type=int, default=256)
    ap.add_argument("--batched-steps", type=int, default=50)
    ap.add_argument("--batched-vs-single", action="store_true",
                    help="also time the batched cases one context per case (plain FP64)")
    ap.add_argument("--large-particles", type=float, default=1e9)
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs each context on one GPU "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x]
    for flag, leg in ((args.no_fp64, "fp64"), (args.no_batched, "batched"), (args.no_large, "large"),
                      (args.no_cpu_baseline, "cpu")):
        if flag and leg in legs:
            legs.remove(leg)

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

    value = dt = None
    n_now = None
    roofline = kernels = cpu = fp64 = None
    avg_mixed = prof_err = None
    bc = bc64 = None
    if "main" in legs:
        bc, bc_src = block_size([case], duwp.MIXED, args)
        log(f"mixed FP32+FP64 path: {case.name}, block_cells={bc} ({bc_src})")
        sim, ps, dt = run_path([case], duwp.MIXED, args.steps, args.warmup, graph, block_cells=bc)
        value = ps / dt
        n_now = sim.total_particles()
        avg_mixed = sim.moments(0, duwp.M_AVG_PRIM)
        log(f"  {args.steps} steps in {dt:.3f}s -> {value:.4e} particle-steps/s")
        # per-kernel device time (HIP events on the library's stream, eager launches)
        roofline, kernels = roofline_of(sim, args.profile_steps, case.name, bc)
        log("  kernels (ms):", json.dumps(kernels))
        if "cpu" in legs:
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
    if "fp64" in legs and "main" in legs:
        bc64, src64 = block_size([case], duwp.FP64, args)
        log(f"plain FP64 path, block_cells={bc64} ({src64})")
        s64, ps64, dt64 = run_path([case], duwp.FP64, args.steps, args.warmup, graph, block_cells=bc64)
        fp64 = ps64 / dt64
        log(f"  {args.steps} steps in {dt64:.3f}s -> {fp64:.4e} particle-steps/s")
        avg64 = s64.moments(0, duwp.M_AVG_PRIM)
        s64.close()
        # the profile error of the mixed path: its time-averaged profiles against
        # the FP64 path's over the same steps, beside two FP64 runs that differ
        # only in the seed.  Both paths draw from the same seed, so their samples
        # stay correlated for a while; a gap within the seed-to-seed one says the
        # FP32 particles add nothing that this sample size can resolve
        s64b, _, _ = run_path([case], duwp.FP64, args.steps, args.warmup, graph, seed=2, block_cells=bc64)
        avg64b = s64b.moments(0, duwp.M_AVG_PRIM)
        s64b.close()
        if avg_mixed is not None:
            prof_err = {"quantity": f"rho, U, T averaged over the {args.steps} timed steps",
                        "norm": "sum over cells of |a - b| / sum over cells of |b| (rho, T) or of sqrt(R T) of b (U)",
                        "mixed_vs_fp64": profile_gap(avg_mixed, avg64, case.R),
                        "fp64_seed_to_seed": profile_gap(avg64b, avg64, case.R)}
            log("  profile error:", json.dumps(prof_err))

    extra = {}
    for leg, fn in (("batched", lambda: leg_batched(args, graph, legs)), ("large", lambda: leg_large(args, graph))):
        if leg not in legs:
            extra[leg] = None
            continue
        try:
            extra[leg] = fn()
        except Exception as e:        # a failed extra leg is reported, the headline stays
            log(f"  {leg} leg failed: {e!r}")
            extra[leg] = {"error": repr(e)}
        torch.cuda.empty_cache()

    step_tr = counted_step(case.name) if value is not None else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3 if dt else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": case.ncells, "particles": n_now,
                   "particles_target": args.particles, "precision": "fp32 particles + fp64 cells",
                   "graph": graph, "gas": "argon VHS omega=0.81", "mach": 8, "block_cells": bc},
        "step_effective": None if value is None else {
            "bytes_per_particle_step": STEP_BYTES_PER_PARTICLE["mixed"],
            "gbs": round(STEP_BYTES_PER_PARTICLE["mixed"] * value / 1e9, 1),
            "frac": round(STEP_BYTES_PER_PARTICLE["mixed"] * value / 1e9 / HBM_PEAK_GBS, 4),
            "fp64_gbs": round(STEP_BYTES_PER_PARTICLE["fp64"] * fp64 / 1e9, 1) if fp64 else None,
            "note": "nominal: a cell pass and a sort each read and write every particle; this path "
                    "streams inside the sort and skips the cell pass where nothing is absorbed or "
                    "resampled, so the nominal rate can exceed the HBM peak",
            "counted_bytes_per_particle_step": round(step_tr[0] / step_tr[1], 2) if step_tr else None,
            "counted_gbs": round(step_tr[0] / step_tr[1] * value / 1e9, 1) if step_tr else None},
        "fp64_value": fp64,
        "mixed_over_fp64": (value / fp64) if (fp64 and value) else None,
        "fp64_block_cells": bc64,
        "profile_error": prof_err,
        "kernels_ms": kernels,
        "batched": extra["batched"],
        "large": extra["large"],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
