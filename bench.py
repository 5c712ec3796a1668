#!/usr/bin/env python3
"""Throughput of the DUWP particle pipeline on one MI355X.

Headline workload: Mach-8 argon shock, 4000 cells over 200 upstream mean free
paths, 5e7 simulated particles (synthetic, seeded).  The timed path stores
particles in FP32 (position relative to its cell) with FP64 cell moments, NS
wave update and absorption fractions; the plain FP64 path is timed on the same
workload beside it.  A step is one full DUWP time step of every stage, replayed
as a captured HIP graph.  Metric: particle-steps per second (particles alive at
the start of each step, summed over the timed steps, over the wall time).

Legs beside the headline (each reported in its own field; a failing leg does not
take the headline down):
  fp64       the plain FP64 path on the headline workload
  precision  the mixed path's profile error on the headline workload where it is
             defined: rho, U, T averaged over the last 2500 of 5000 steps, relative
             L2 over the cells against the FP64 path, beside the FP64 seed-to-seed gap
  batched    256 independent uneven shock and Sod cases in one context, mixed and
             FP64, the same cases one context each (FP64), the profile error over
             500 steps, and the oracle over the 256 cases on all host threads
  large      the Mach-10 near-continuum case, 20000 cells, 1e9 particles
  c1         the Mach-3 shock, 100 cells, 2e4 particles, 500 steps (FP64), and the
             oracle's full run
  c2         the Sod Kn sweep, 5 tubes of 1000 cells and 1e6 particles, 2000 steps
             (FP64), and an oracle sample
  cpu        the oracle on the headline workload (one thread: it is serial per case)
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
LEGS = ("main", "fp64", "precision", "batched", "large", "c1", "c2", "cpu")

# Algorithmic HBM bytes per particle of the particle-streaming kernels, per
# element size s of the particle records (4 in FP32 mode, 8 in FP64 mode): the
# scatter reads each particle's record (x,u,v,w) and writes it to its sorted
# place; absorb_resample reads and writes the records of the cells it touches
# (counted over all particles of the step, an upper bound).
BYTES_PER_PARTICLE = {
    "scatter": lambda s: 8 * s,
    "absorb_resample": lambda s: 8 * s,
}
# A simple model of a whole step when almost nothing is absorbed: each
# particle's record read and written once by a cell pass and once by the sort.
STEP_BYTES_PER_PARTICLE = {"mixed": 64, "fp64": 128}
KERNEL_HEADERS = ("duwp_physics.hpp", "duwp_device.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info() -> dict:
    """Host cores and CPU model (the oracle's machine)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"nproc": avail, "cpu_count": os.cpu_count(), "cpu_model": model}


def pool_threads() -> int:
    """Worker threads for the oracle over many cases: the host's share, at most 16."""
    return max(1, min(16, host_info()["nproc"]))


# ---------------------------------------------------------------------------
# Counted traffic (committed rocprofv3 counter summaries)
# ---------------------------------------------------------------------------

def kernel_fingerprint(kernel: str) -> str:
    """sha256 of a kernel's text (from its template line to the next numbered
    section of duwp_kernels.hip) and of the device and physics headers."""
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
    """sha256 over every source file of the library."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2305_12071_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _traffic_files():
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        with open(path) as fh:
            yield json.load(fh)


def counted_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE
    and WRITE_SIZE runs, each scaled by a plain copy), or None when the kernel's
    sources changed since the counters were taken."""
    fp = kernel_fingerprint(kernel)
    for d in _traffic_files():
        if d.get("kernel") == kernel and d.get("workload") == workload and d.get("kernel_sha256") == fp:
            return d["hbm_bytes_per_launch"], d["particles_per_launch"]
    return None


def counted_step(workload: str):
    """HBM bytes of one whole step and its particles from the committed counter
    summary, or None when any library source changed since."""
    fp = sources_fingerprint()
    for d in _traffic_files():
        if d.get("workload") == workload and d.get("sources_sha256") == fp and "step_hbm_bytes" in d:
            return d["step_hbm_bytes"], d["particles_per_launch"]
    return None


# ---------------------------------------------------------------------------
# Running the library
# ---------------------------------------------------------------------------

def config_for(cases, precision, args):
    """(block_cells, tune, source) of the per-cell kernels and tiles: fixed, tuned now,
    from the autotuner's cache (same or nearest shape family), or the defaults."""
    from paper_2305_12071_amd import autotune
    if args.block_cells:
        return args.block_cells, {}, "fixed"
    if args.autotune:
        bc, t = autotune.tune(cases, precision, path=args.tune_cache, log=log)
        return bc, t, "tuned"
    hit = autotune.lookup(cases, precision, path=args.tune_cache or autotune.DEFAULT_CACHE)
    if hit:
        return hit[0], hit[1], f"cache {hit[2]}"
    return 256, {}, "default"


def run_path(cases, precision, steps, warmup, graph, cfg, seed=1):
    from paper_2305_12071_amd import duwp
    import torch

    sim = duwp.Sim(cases, seed=seed, precision=precision, use_graph=graph, block_cells=cfg[0], tune=cfg[1])
    t = time.perf_counter()
    sim.step(warmup)
    log(f"  warmup {warmup} steps in {time.perf_counter() - t:.2f}s, N={sim.total_particles()}")
    sim.reset_average()
    sim.particle_steps(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)          # returns after the device finished (error word read back)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ps = sim.particle_steps(reset=True)
    return sim, ps, t1 - t0


def averaged_profiles(cases, precision, steps, avg_from, cfg, seed):
    """(rho, U, V, W, T) of each case time-averaged over the steps after avg_from."""
    from paper_2305_12071_amd import duwp
    sim = duwp.Sim(cases, seed=seed, precision=precision, use_graph=True, block_cells=cfg[0], tune=cfg[1])
    sim.step(avg_from)
    sim.reset_average()
    sim.step(steps - avg_from)
    out = [sim.moments(k, duwp.M_AVG_PRIM) for k in range(len(cases))]
    sim.close()
    return out


def rel_l2(a, b) -> dict:
    """Relative L2 gap over the cells of profile a from profile b, for rho, U and T."""
    out = {}
    for name, k in (("rho", 0), ("U", 1), ("T", 4)):
        den = float(np.sqrt((b[:, k] ** 2).sum()))
        out[name] = float(np.sqrt(((a[:, k] - b[:, k]) ** 2).sum()) / den) if den > 0 else 0.0
    return out


def leg_roofline(kernel, instance, workload, ms, alg_bytes):
    """A leg's dominant kernel against the HBM peak: its algorithmic bytes per launch,
    and the bytes HBM really moved for it (committed counters, when current)."""
    tr = counted_traffic(instance, workload)
    out = {"bound": "hbm", "kernel": kernel, "instance": instance, "kernel_ms": ms,
           "algorithmic_bytes": int(alg_bytes),
           "achieved": round(alg_bytes / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(alg_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": tr[0] if tr else None}
    if tr:
        out["traffic_gbs"] = round(tr[0] / (ms * 1e-3) / 1e9, 1)
        out["traffic_frac"] = round(tr[0] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def roofline_of(sim, profile_steps, workload, block_cells, scat_items):
    """Dominant particle-streaming kernel: algorithmic bytes over its event-timed duration."""
    kms = sim.profile(profile_steps)
    prof_ps = sim.particle_steps(reset=True) / profile_steps
    dom = max((k for k in kms if k in BYTES_PER_PARTICLE), key=lambda k: kms[k])
    alg_bytes = BYTES_PER_PARTICLE[dom](4) * prof_ps
    achieved = alg_bytes / (kms[dom] * 1e-3) / 1e9
    scat = "k_scatter<float, 1, 2>" if block_cells == 64 else f"k_scatter<float, 8, {scat_items}>"
    kname = {"scatter": scat, "absorb_resample": "k_absorb_resample<float, false>"}.get(dom)
    tr = counted_traffic(kname, workload) if kname else None
    roof = {"bound": "hbm", "kernel": dom, "instance": kname, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": tr[0] if tr else None,
            "traffic_per_particle": round(tr[0] / tr[1], 2) if tr else None,
            "bytes_per_particle": BYTES_PER_PARTICLE[dom](4), "particles_per_launch": int(prof_ps),
            "kernel_ms": round(kms[dom], 4),
            "timing": "HIP events on the context's stream around each launch, eager steps"}
    return roof, {k: round(v, 4) for k, v in kms.items()}


def oracle_pool(cases, states, seed, steps):
    """The oracle over many cases at once, one thread per case at a time (the C calls
    release the interpreter): particle-steps, seconds, threads."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    orcs = []
    for k, (c, st) in enumerate(zip(cases, states)):
        o = O.Oracle(c, seed=seed, case_id=k)
        if st is not None:
            o.set_state(st)
        orcs.append(o)
    nthr = pool_threads()

    def run(o):
        ps = 0
        for _ in range(steps):
            ps += o.n
            o.step(1)
        return ps

    t = time.perf_counter()
    with ThreadPoolExecutor(nthr) as ex:
        ps = sum(ex.map(run, orcs))
    return ps, time.perf_counter() - t, nthr


# ---------------------------------------------------------------------------
# Legs
# ---------------------------------------------------------------------------

def stream_ceiling(nbytes: int = 1600 << 20, reps: int = 20) -> dict:
    """A plain streaming kernel of the scatter's traffic (read nbytes, write nbytes:
    torch's elementwise scale of a float buffer), timed with HIP events: the HBM
    rate a read-once write-once kernel reaches on this device."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_launch": 2 * nbytes, "ms": round(ms, 4), "gbs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1),
            "kernel": "torch elementwise scale (read once, write once)"}


def leg_precision(args, case, cfg_m, cfg_f):
    """The mixed path's profile error where it is defined: rho, U, T time-averaged
    over the last half of the run, relative L2 over the cells against the FP64 path
    with the same seed.  R replicas of the case run side by side in one context per
    precision (case index r keys replica r's random streams, the same in both
    contexts), which gives R same-seed pairs, the FP64 seed-to-seed gap from pairs of
    FP64 replicas, and the gap of the two R-replica means with its noise level (the
    standard error of the mean difference, per cell, over the cells)."""
    from paper_2305_12071_amd import duwp
    S, A, R = args.precision_steps, args.precision_steps // 2, args.precision_replicas
    log(f"precision: {case.name}, {R} replicas a side, {S} steps, average of the last {S - A}")
    t = time.perf_counter()
    m = np.stack(averaged_profiles([case] * R, duwp.MIXED, S, A, cfg_m, 1))
    log(f"  mixed done ({time.perf_counter() - t:.1f}s)")
    f = np.stack(averaged_profiles([case] * R, duwp.FP64, S, A, cfg_f, 1))
    log(f"  fp64 done ({time.perf_counter() - t:.1f}s)")
    q = ("rho", "U", "T")

    def mean_of(gaps):
        return {k: float(np.mean([g[k] for g in gaps])) for k in q}

    same = [rel_l2(m[r], f[r]) for r in range(R)]
    floor = [rel_l2(f[i], f[j]) for i in range(R) for j in range(i + 1, R)]
    mm, fm = m.mean(0), f.mean(0)
    se = np.sqrt(m.var(0, ddof=1) / R + f.var(0, ddof=1) / R)
    noise, bias = {}, {}
    gap = rel_l2(mm, fm)
    for name, k in (("rho", 0), ("U", 1), ("T", 4)):
        den = float(np.sqrt((fm[:, k] ** 2).sum()))
        noise[name] = float(np.sqrt((se[:, k] ** 2).sum()) / den)
        bias[name] = float(np.sqrt(max(gap[name] ** 2 - noise[name] ** 2, 0.0)))
    out = {"workload": case.name, "steps": S, "averaged_steps": S - A, "replicas": R,
           "quantity": f"rho, U, T time-averaged over steps {A + 1}..{S}",
           "norm": "relative L2 over the cells: ||a - b||_2 / ||b||_2",
           "mixed_vs_fp64": mean_of(same),
           "mixed_vs_fp64_per_replica": same,
           "fp64_seed_to_seed": mean_of(floor),
           "replica_means": {"mixed_vs_fp64": gap, "noise": noise, "bias_estimate": bias},
           "target": 1e-3,
           "max_mixed_vs_fp64": max(mean_of(same).values()),
           "seconds": round(time.perf_counter() - t, 1)}
    log("  ", json.dumps(out))
    return out


def leg_batched(args, graph, legs):
    from paper_2305_12071_amd import duwp
    from paper_2305_12071_amd import inputs as I
    cases = I.batched_cases(args.batched_cases)
    cfg_m = config_for(cases, duwp.MIXED, args)
    cfg_f = config_for(cases, duwp.FP64, args)
    ncell = sum(c.ncells for c in cases)
    log(f"batched form: {len(cases)} cases, {ncell} cells; mixed {cfg_m}; fp64 {cfg_f}")
    sb, psb, dtb = run_path(cases, duwp.MIXED, args.batched_steps, 5, graph, cfg_m)
    out = {"value": psb / dtb, "unit": "particle-steps/s", "cases": len(cases), "cells": ncell,
           "particles": sb.total_particles(), "steps": args.batched_steps,
           "ms_per_step": dtb / args.batched_steps * 1e3,
           "precision": "fp32 particles + fp64 cells",
           "config": {"block_cells": cfg_m[0], "tune": cfg_m[1], "source": cfg_m[2]}}
    out["kernels_ms"] = {k: round(v, 4) for k, v in sb.profile(args.profile_steps).items()}
    prof_ps = sb.particle_steps(reset=True) / args.profile_steps
    sb.close()
    out["roofline"] = leg_roofline("scatter", "k_scatter<float, 1, 2>" if cfg_m[0] == 64 else
                                   f"k_scatter<float, 8, {cfg_m[1].get('scatter_items', 4)}>",
                                   "batched256", out["kernels_ms"]["scatter"], BYTES_PER_PARTICLE["scatter"](4) * prof_ps)
    log(f"  mixed {out['value']:.4e} particle-steps/s, N={out['particles']}")
    states = None
    if not args.no_batched_fp64:
        sf, psf, dtf = run_path(cases, duwp.FP64, args.batched_steps, 5, graph, cfg_f)
        out["fp64_value"] = psf / dtf
        out["fp64_config"] = {"block_cells": cfg_f[0], "tune": cfg_f[1], "source": cfg_f[2]}
        out["mixed_over_fp64"] = out["value"] / out["fp64_value"]
        log(f"  fp64 {out['fp64_value']:.4e} particle-steps/s")
        if "cpu" in legs:
            states = [sf.get_state(k) for k in range(len(cases))]
        sf.close()
    # the same cases one context each, plain FP64, one after another (timed steps only)
    if args.single_steps > 0:
        tot_ps, tot_t = 0, 0.0
        for c in cases:
            cfg1 = config_for([c], duwp.FP64, args)
            s1, p1, t1 = run_path([c], duwp.FP64, args.single_steps, 3, graph, cfg1)
            s1.close()
            tot_ps += p1
            tot_t += t1
        out["one_context_per_case_fp64"] = tot_ps / tot_t
        if "fp64_value" in out:
            out["batched_fp64_over_one_by_one"] = out["fp64_value"] / out["one_context_per_case_fp64"]
        out["batched_mixed_over_one_by_one"] = out["value"] / out["one_context_per_case_fp64"]
        log(f"  one context per case, FP64: {out['one_context_per_case_fp64']:.4e} particle-steps/s")
    if args.batched_precision_steps > 0:
        out["profile_error"] = batched_profile_error(args, cases, cfg_m, cfg_f)
    if states is not None:
        n0 = sum(len(s["x"]) for s in states)
        ps, dt, nthr = oracle_pool(cases, states, 1, args.cpu_batched_steps)
        del states
        out["cpu_oracle"] = {"value": ps / dt, "unit": "particle-steps/s", "threads": nthr, **host_info(),
                             "kind": "oracle",
                             "sample": f"{len(cases)} cases, {args.cpu_batched_steps} FP64 oracle steps from the GPU "
                                       f"state after warm-up ({n0} particles), one case per thread at a time, "
                                       f"{dt:.1f}s"}
        log(f"  oracle over the cases: {ps / dt:.3e} particle-steps/s on {nthr} threads")
    return out


def batched_profile_error(args, cases, cfg_m, cfg_f):
    """Per case: rho, U, T averaged over the second half of the run, mixed against FP64
    (same seed), beside FP64 against FP64 (another seed); medians and maxima over the
    cases, and the ratio of the two gaps."""
    from paper_2305_12071_amd import duwp
    S, A = args.batched_precision_steps, args.batched_precision_steps // 2
    pm = averaged_profiles(cases, duwp.MIXED, S, A, cfg_m, 1)
    pf = averaged_profiles(cases, duwp.FP64, S, A, cfg_f, 1)
    pg = averaged_profiles(cases, duwp.FP64, S, A, cfg_f, 2)
    gaps = [rel_l2(a, b) for a, b in zip(pm, pf)]
    floor = [rel_l2(a, b) for a, b in zip(pg, pf)]
    q = ("rho", "U", "T")
    ratio = [max(g[k] for k in q) / max(max(f[k] for k in q), 1e-300) for g, f in zip(gaps, floor)]
    out = {
        "steps": S, "averaged_steps": S - A,
        "norm": "relative L2 over the cells per case, rho U T",
        "mixed_vs_fp64": {"median": {k: float(np.median([g[k] for g in gaps])) for k in q},
                          "max": {k: float(max(g[k] for g in gaps)) for k in q}},
        "fp64_seed_to_seed": {"median": {k: float(np.median([f[k] for f in floor])) for k in q},
                              "max": {k: float(max(f[k] for f in floor)) for k in q}},
        "ratio_to_seed_gap": {"median": float(np.median(ratio)), "max": float(max(ratio))}}
    log("  profile error:", json.dumps(out))
    return out


def leg_large(args, graph):
    from paper_2305_12071_amd import duwp
    from paper_2305_12071_amd import inputs as I
    c = I.mach10_large(ncells=args.large_cells, n_kept=args.large_particles)
    cfg = config_for([c], duwp.MIXED, args)
    log(f"large near-continuum case: {c.name}, {args.large_particles:.0e} kept particles, {cfg}")
    sl, psl, dtl = run_path([c], duwp.MIXED, args.large_steps, 3, graph, cfg)
    out = {"value": psl / dtl, "unit": "particle-steps/s", "workload": c.name, "cells": c.ncells,
           "particles": sl.total_particles(), "steps": args.large_steps,
           "ms_per_step": dtl / args.large_steps * 1e3, "precision": "fp32 particles + fp64 cells",
           "config": {"block_cells": cfg[0], "tune": cfg[1], "source": cfg[2]}}
    d = sl.diag()
    out["absorbed_per_step"] = int(d["n_abs"].sum())
    out["resampled_per_step"] = int(d["n_new"].sum())
    out["collision_candidates_per_step"] = int(d["n_cand"].sum())
    out["accepted_collisions_per_step"] = int(d["n_coll"].sum())
    wave = sl.moments(0, duwp.M_PSI_W)[:, 0].sum() / sl.moments(0, duwp.M_PSI_T)[:, 0].sum()
    out["wave_mass_fraction"] = round(float(wave), 4)
    out["kernels_ms"] = {k: round(v, 3) for k, v in sl.profile(1).items()}
    sl.close()
    # the big-cell collide reads and writes particle records at random inside cells of
    # 0.8 MB: its algorithmic bytes are those records (16 B each: two reads per
    # candidate, two writes per accepted pair); HBM moves whole lines for them
    cand, acc = out["collision_candidates_per_step"], out["accepted_collisions_per_step"]
    inst = f"k_collide_big<float, {cfg[1].get('big_block', 512)}>"
    out["roofline"] = leg_roofline("collide_big", inst, c.name, out["kernels_ms"]["collide_big"],
                                   16.0 * (2 * cand + 2 * acc))
    # its record accesses at random inside the cells: two reads per candidate and two
    # writes per accepted pair, each in a 128-byte line of its own
    out["roofline"]["record_accesses_per_s"] = round((2 * cand + 2 * acc) / (out["kernels_ms"]["collide_big"] * 1e-3), 1)
    log(f"  {out['value']:.4e} particle-steps/s, {out['ms_per_step']:.1f} ms/step, N={out['particles']}")
    return out


def leg_c1(args, graph, legs):
    from paper_2305_12071_amd import duwp
    from paper_2305_12071_amd import inputs as I
    c = I.mach3_small()
    cfg = config_for([c], duwp.FP64, args)
    log(f"c1: {c.name}, FP64, 500 steps, {cfg}")
    s, ps, dt = run_path([c], duwp.FP64, 500, 0, graph, cfg)
    out = {"value": ps / dt, "unit": "particle-steps/s", "workload": c.name, "cells": c.ncells,
           "particles": s.total_particles(), "steps": 500, "ms_per_step": dt / 500 * 1e3, "precision": "fp64",
           "config": {"block_cells": cfg[0], "tune": cfg[1], "source": cfg[2]}}
    s.close()
    log(f"  {out['value']:.4e} particle-steps/s, {out['ms_per_step'] * 1e3:.1f} us/step")
    if "cpu" in legs:
        ps, odt, _ = oracle_pool([c], [None], 1, 500)
        out["cpu_oracle"] = {"value": ps / odt, "unit": "particle-steps/s", "threads": 1, "kind": "oracle",
                             "sample": f"the whole run: 500 FP64 oracle steps from the initial state, {odt:.1f}s"}
        log(f"  oracle {ps / odt:.3e} particle-steps/s")
    return out


def leg_c2(args, graph, legs):
    from paper_2305_12071_amd import duwp
    from paper_2305_12071_amd import inputs as I
    cases = I.sod_kn_sweep()
    cfg = config_for(cases, duwp.FP64, args)
    steps = args.c2_steps
    log(f"c2: Sod Kn sweep, {len(cases)} tubes x {cases[0].ncells} cells, FP64, {steps} steps, {cfg}")
    s, ps, dt = run_path(cases, duwp.FP64, steps, 0, graph, cfg)
    out = {"value": ps / dt, "unit": "particle-steps/s", "workload": "sod_kn_sweep_c1000",
           "kn": [1e-4, 1e-3, 1e-2, 1e-1, 1.0], "cases": len(cases), "cells_per_case": cases[0].ncells,
           "particles": s.total_particles(), "steps": steps, "ms_per_step": dt / steps * 1e3,
           "precision": "fp64", "config": {"block_cells": cfg[0], "tune": cfg[1], "source": cfg[2]}}
    states = [s.get_state(k) for k in range(len(cases))] if "cpu" in legs else None
    s.close()
    log(f"  {out['value']:.4e} particle-steps/s, {out['ms_per_step']:.3f} ms/step")
    if states is not None:
        n0 = sum(len(x["x"]) for x in states)
        ps, odt, nthr = oracle_pool(cases, states, 1, args.cpu_c2_steps)
        out["cpu_oracle"] = {"value": ps / odt, "unit": "particle-steps/s", "threads": nthr, "kind": "oracle",
                             "sample": f"{args.cpu_c2_steps} FP64 oracle steps of the {len(cases)} tubes from the "
                                       f"GPU's final state ({n0} particles), one tube per thread, {odt:.1f}s"}
        log(f"  oracle {ps / odt:.3e} particle-steps/s")
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
    ap.add_argument("--autotune", action="store_true", help="tune each workload's launch shapes first")
    ap.add_argument("--tune-cache", default=None, help="cache file (default: the package's)")
    ap.add_argument("--precision-steps", type=int, default=5000)
    ap.add_argument("--precision-replicas", type=int, default=4)
    ap.add_argument("--batched-cases", type=int, default=256)
    ap.add_argument("--batched-steps", type=int, default=50)
    ap.add_argument("--batched-precision-steps", type=int, default=500, help="0: leave out")
    ap.add_argument("--no-batched-fp64", action="store_true", help="the batched leg without its FP64 path")
    ap.add_argument("--single-steps", type=int, default=20,
                    help="timed steps per case, one context each (0: leave out)")
    ap.add_argument("--large-particles", type=float, default=1e9)
    ap.add_argument("--large-cells", type=int, default=20000,
                    help="cells of the near-continuum case (2500 with 1.25e8 particles: one GPU's share of eight)")
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--c2-steps", type=int, default=2000)
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--cpu-batched-steps", type=int, default=3)
    ap.add_argument("--cpu-c2-steps", type=int, default=4)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run kernels of known traffic on 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs each context on one GPU "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x]

    import torch
    from paper_2305_12071_amd import duwp
    from paper_2305_12071_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    duwp.lib()
    if args.calibrate_copy:
        # kernels of known traffic for the byte counters: a fill writes 1 GiB, a
        # scale reads 1 GiB and writes 1 GiB, a sum reads 1 GiB
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=b)
            float(a.sum())
        torch.cuda.synchronize()
        del a, b
    case = I.mach8_shock(args.cells, args.particles)
    graph = not args.no_graph
    cfg_m = config_for([case], duwp.MIXED, args)
    cfg_f = config_for([case], duwp.FP64, args)

    value = dt = None
    n_now = None
    roofline = kernels = cpu = fp64 = None
    if "main" in legs:
        log(f"mixed FP32+FP64 path: {case.name}, {cfg_m}")
        sim, ps, dt = run_path([case], duwp.MIXED, args.steps, args.warmup, graph, cfg_m)
        value = ps / dt
        n_now = sim.total_particles()
        log(f"  {args.steps} steps in {dt:.3f}s -> {value:.4e} particle-steps/s")
        roofline, kernels = roofline_of(sim, args.profile_steps, case.name, cfg_m[0],
                                        cfg_m[1].get("scatter_items", 4))
        if not args.calibrate_copy:     # (profiling runs keep their kernel list to the step's)
            ceil = stream_ceiling()
            roofline["stream_ceiling_gbs"] = ceil["gbs"]
            roofline["frac_of_stream_ceiling"] = round(roofline["achieved"] / ceil["gbs"], 4)
            log("  streaming ceiling:", json.dumps(ceil))
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
                   **host_info(),
                   "sample": f"{case.name}: {args.cpu_steps} FP64 oracle steps from the warmed-up state "
                             f"({n0} particles), one thread (the oracle is serial within a case), {cdt:.1f}s"}
            log(f"  oracle {cpu['value']:.3e} particle-steps/s")
            del orc
        else:
            sim.close()
            del sim
    if "fp64" in legs:
        log(f"plain FP64 path, {cfg_f}")
        s64, ps64, dt64 = run_path([case], duwp.FP64, args.steps, args.warmup, graph, cfg_f)
        fp64 = ps64 / dt64
        s64.close()
        log(f"  {args.steps} steps in {dt64:.3f}s -> {fp64:.4e} particle-steps/s")

    extra = {}
    for leg, fn in (("precision", lambda: leg_precision(args, case, cfg_m, cfg_f)),
                    ("batched", lambda: leg_batched(args, graph, legs)),
                    ("large", lambda: leg_large(args, graph)),
                    ("c1", lambda: leg_c1(args, graph, legs)),
                    ("c2", lambda: leg_c2(args, graph, legs))):
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
                   "graph": graph, "gas": "argon VHS omega=0.81", "mach": 8,
                   "block_cells": cfg_m[0], "tune": cfg_m[1], "tune_source": cfg_m[2]},
        "step_effective": None if value is None else {
            "counted_bytes_per_particle_step": round(step_tr[0] / step_tr[1], 2) if step_tr else None,
            "counted_gbs": round(step_tr[0] / step_tr[1] * value / 1e9, 1) if step_tr else None,
            "counted_frac": round(step_tr[0] / step_tr[1] * value / 1e9 / HBM_PEAK_GBS, 4) if step_tr else None,
            "model_bytes_per_particle_step": STEP_BYTES_PER_PARTICLE["mixed"],
            "model_gbs": round(STEP_BYTES_PER_PARTICLE["mixed"] * value / 1e9, 1),
            "model_fp64_gbs": round(STEP_BYTES_PER_PARTICLE["fp64"] * fp64 / 1e9, 1) if fp64 else None,
            "note": "counted: every kernel's HBM bytes of one step from the committed counters (null once a "
                    "source changed); model: a cell pass and a sort each reading and writing every record, "
                    "which this path does not do (it streams inside the sort and skips untouched cells), "
                    "so the model figure is no bandwidth and can pass the peak"},
        "fp64_value": fp64,
        "mixed_over_fp64": (value / fp64) if (fp64 and value) else None,
        "fp64_config": {"block_cells": cfg_f[0], "tune": cfg_f[1], "source": cfg_f[2]},
        "profile_error": extra["precision"],
        "kernels_ms": kernels,
        "batched": extra["batched"],
        "large": extra["large"],
        "c1": extra["c1"],
        "c2": extra["c2"],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
