"""Block-size autotuner for the per-cell kernels of the DUWP step.

The per-cell kernels (cell state, absorb/resample, histogram recount, scatter)
run one block per cell; the best block size depends on the particles per cell
and on the precision.  `tune` times whole graph-replayed steps for each
candidate and keeps the fastest; results are cached in a JSON file keyed by
(GPU architecture, precision, cell count, particle count to two digits).
"""
from __future__ import annotations

import json
import os
import time

from . import duwp

CANDIDATES = (64, 128, 256, 512)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _arch() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def shape_key(cases, precision: int) -> str:
    cells = sum(c.ncells for c in cases)
    mass = sum(c.domain_mass() / c.m_particle for c in cases)
    return f"{_arch()}|{'mixed' if precision == duwp.MIXED else 'fp64'}|cases={len(cases)}|cells={cells}|n={mass:.1e}"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(cases, precision: int, path: str = DEFAULT_CACHE):
    e = load_cache(path).get(shape_key(cases, precision))
    return int(e["block_cells"]) if e else None


def tune(cases, precision: int, steps: int = 20, warmup: int = 5, candidates=CANDIDATES,
         path: str | None = DEFAULT_CACHE, log=None) -> int:
    """Time `steps` graph-replayed steps after `warmup` for each candidate; return the best."""
    import torch
    res = {}
    for bc in candidates:
        sim = duwp.Sim(cases, seed=1, precision=precision, use_graph=True, block_cells=bc)
        sim.step(warmup)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.step(steps)
        res[bc] = (time.perf_counter() - t) / steps * 1e3
        sim.close()
        if log:
            log(f"  autotune block_cells={bc}: {res[bc]:.4f} ms/step")
    best = min(res, key=res.get)
    if path:
        cache = load_cache(path)
        cache[shape_key(cases, precision)] = {"block_cells": best,
                                              "ms_per_step": {str(k): round(v, 5) for k, v in res.items()}}
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return best
