"""Autotuner of the DUWP step's launch shapes.

The knobs are the per-cell kernels' block size (`block_cells`) and the tile
shapes and thresholds of `duwp_tune` (scatter items per thread, the
block-per-cell collide's block and residency, the size from which a cell
collides in that kernel, the cell count up to which a wave per cell runs the
other collisions and the grid of work items beyond it, destinations per block
of the sort's count kernels).  None
of them changes an integer result, so the tuner only times.

`tune` searches one knob at a time (coordinate descent, each knob over its
candidates with the others at their best so far; the size threshold of the
block-per-cell collide before its shape, which matters only for the cells the
threshold sends there), timing graph-replayed steps
of a fresh context per candidate, and stores the winner in a JSON cache under
the workload's shape family: GPU architecture, precision, number of cases,
cells per case and particles per cell (both rounded to powers of two), and
whether most of the mass sits in the wave part.  `lookup` returns the cached
configuration of the same family, else of the nearest family of the same
architecture, precision and wave regime, else None (the library's defaults).
"""
from __future__ import annotations

import json
import math
import os
import time

from . import duwp

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
BLOCK_CELLS = (64, 128, 256, 512)


def _arch() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _wave_regime(cases) -> int:
    """1 when most of the initial mass of the cases goes to the wave part: the
    absorbed fraction of Eq. p, P = 1 - tau/dt, at the two initial states,
    weighted by their mass (0 otherwise).  Shape data only: a property of the
    inputs that decides whether the block-per-cell collide matters."""
    tot = wav = 0.0
    for c in cases:
        for rho, T, L in ((c.rho_L, c.T_L, c.x_split - c.x_lo), (c.rho_R, c.T_R, c.x_hi - c.x_split)):
            w = c.omega
            beta = 15.0 / (2.0 * (5.0 - 2.0 * w) * (7.0 - 2.0 * w))
            lam = c.lambda_ref * c.rho_ref if c.lambda_ref > 0 else c.m_mol / (math.sqrt(2.0) * math.pi * c.d_ref ** 2)
            mu = beta * lam * math.sqrt(2.0 * math.pi * c.R * c.T_ref) * (T / c.T_ref) ** w
            tau = mu / (rho * c.R * T)
            P = max(0.0, 1.0 - tau / c.dt)
            tot += rho * L
            wav += P * rho * L
    return 1 if tot > 0 and wav > 0.5 * tot else 0


def family(cases, precision: int, arch: str | None = None) -> dict:
    """Shape family of a workload (the cache key's fields)."""
    cells = sum(c.ncells for c in cases)
    parts = sum(c.domain_mass() / c.m_particle for c in cases)
    return {"arch": arch or _arch(), "precision": "mixed" if precision == duwp.MIXED else "fp64",
            "cases": len(cases),
            "log2_cells_per_case": int(round(math.log2(max(cells / len(cases), 1.0)))),
            "log2_particles_per_cell": int(round(math.log2(max(parts / max(cells, 1), 1.0)))),
            "wave": _wave_regime(cases)}


def key_of(f: dict) -> str:
    return (f"{f['arch']}|{f['precision']}|cases={f['cases']}|cells~2^{f['log2_cells_per_case']}"
            f"|ppc~2^{f['log2_particles_per_cell']}|wave={f['wave']}")


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _distance(a: dict, b: dict) -> float:
    return (abs(a["log2_cells_per_case"] - b["log2_cells_per_case"])
            + abs(a["log2_particles_per_cell"] - b["log2_particles_per_cell"])
            + abs(math.log2(a["cases"]) - math.log2(b["cases"])))


def lookup(cases, precision: int, path: str = DEFAULT_CACHE, arch: str | None = None):
    """(block_cells, tune dict, family key it came from), or None."""
    f = family(cases, precision, arch)
    cache = load_cache(path)
    e = cache.get(key_of(f))
    if e is None:
        near = [(_distance(f, v["family"]), k) for k, v in cache.items()
                if "family" in v and all(v["family"][x] == f[x] for x in ("arch", "precision", "wave"))]
        if not near:
            return None
        k = min(near)[1]
        e = cache[k]
    else:
        k = key_of(f)
    return int(e["block_cells"]), dict(e.get("tune", {})), k


def _candidates(knob: str, precision: int, ncells: int, has_big: bool):
    if knob == "block_cells":
        return list(BLOCK_CELLS)
    if knob == "scatter_items":
        return [2, 4]
    if knob == "big":
        if not has_big:
            return []
        if precision == duwp.MIXED:
            return [(256, 2), (256, 4), (256, 6), (512, 2), (512, 3), (512, 1), (1024, 1)]
        return [(256, 2), (256, 3), (256, 4), (256, 1), (512, 1), (1024, 1)]
    if knob == "big_min":
        # 2**31 - 1: no block-per-cell collide at all (not even its launch)
        return [256, 1024, 4096, 16384, 2147483647] if has_big else [2147483647]
    if knob == "collide_by_cell_max":
        # a wave per cell, or work items from the candidate list, where both apply
        return [ncells, max(ncells - 1, 1)] if 512 <= ncells <= (1 << 16) else []
    if knob == "count_dests":
        return [64, 256] if ncells >= 8192 else []
    if knob == "collide_blocks_per_cu":
        # the wave collide's grid for work items (the form that more than
        # collide_by_cell_max cells take)
        return [32, 64, 128] if ncells >= 512 else []
    raise KeyError(knob)


def _apply(cfg: dict, knob: str, v) -> dict:
    c = dict(cfg)
    t = dict(c["tune"])
    if knob == "block_cells":
        c["block_cells"] = v
    elif knob == "big":
        t["big_block"], t["big_blocks_per_cu"] = v
    elif knob == "big_min":
        t["big_min_particles"] = t["big_min_candidates"] = v
    else:
        t[knob] = v
    c["tune"] = t
    return c


def time_config(cases, precision: int, cfg: dict, steps: int, warmup: int) -> float:
    """ms per graph-replayed step of a fresh context with configuration cfg."""
    import torch
    sim = duwp.Sim(cases, seed=1, precision=precision, use_graph=True, block_cells=cfg["block_cells"],
                   tune=cfg["tune"])
    try:
        sim.step(warmup)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.step(steps)
        return (time.perf_counter() - t) / steps * 1e3
    finally:
        sim.close()
        torch.cuda.empty_cache()


def _has_big_cells(cases, precision: int) -> bool:
    """Whether any cell draws as many candidates as the lowest threshold of the
    block-per-cell collide after a few steps (candidates per cell from duwp_diag)."""
    sim = duwp.Sim(cases, seed=1, precision=precision, use_graph=False)
    try:
        sim.step(2)
        return any((sim.diag(k)["n_cand"] >= 256).any() for k in range(len(cases)))
    finally:
        sim.close()


def tune(cases, precision: int, steps: int = 20, warmup: int = 5, path: str | None = DEFAULT_CACHE,
         log=None, knobs=("block_cells", "scatter_items", "big_min", "big", "collide_by_cell_max",
                          "collide_blocks_per_cu", "count_dests"), sweeps: int = 2):
    """Coordinate search over the knobs, `sweeps` passes (the knobs interact: the
    size threshold, the collide kernel's shape and the wave-per-cell switch);
    stores and returns (block_cells, tune dict)."""
    ncells = sum(c.ncells for c in cases)
    has_big = _has_big_cells(cases, precision)
    best = {"block_cells": 256, "tune": {}}
    # the first context of a process tends to run a few percent faster than the
    # ones after it (fresh device memory): one throwaway timing puts the default
    # on the same footing as the candidates
    time_config(cases, precision, best, max(1, steps // 4), warmup)
    best_ms = time_config(cases, precision, best, steps, warmup)
    tried = {"default": round(best_ms, 5)}
    if log:
        log(f"  autotune default: {best_ms:.4f} ms/step")
    for sweep in range(sweeps):
        for knob in knobs:
            for v in _candidates(knob, precision, ncells, has_big):
                cfg = _apply(best, knob, v)
                if cfg == best:
                    continue        # the configuration in hand
                if knob == "scatter_items" and cfg["block_cells"] == 64:
                    continue        # one-wave scatter blocks have a fixed depth
                ms = time_config(cases, precision, cfg, steps, warmup)
                tried[f"{knob}={v}" + (f" (pass {sweep + 1})" if sweep else "")] = round(ms, 5)
                if log:
                    log(f"  autotune {knob}={v}: {ms:.4f} ms/step")
                if ms < best_ms:
                    best, best_ms = cfg, ms
    if path:
        f = family(cases, precision)
        cache = load_cache(path)
        cache[key_of(f)] = {"family": f, "block_cells": best["block_cells"], "tune": best["tune"],
                            "ms_per_step": round(best_ms, 5), "tried": tried, "steps": steps}
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return best["block_cells"], best["tune"]
