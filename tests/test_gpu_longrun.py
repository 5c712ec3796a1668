"""Long runs: the GPU path's averaged density, velocity and temperature profiles
against the oracle's, within the noise of independent ensembles.

Per-step parity holds only while both sides take the same integer decisions;
over hundreds of steps the few-ulp differences of the transcendental functions
grow through the collisions until decisions differ, so long runs are compared
statistically.  Each side runs its own replicas from seeds the other never
uses; per cell and quantity the difference of the two replica means is
compared with its standard error (a t statistic), with a Bonferroni allowance
over all cells and quantities, and the mean square of the statistics over the
cells must stay near one (a small bias shared by many cells shows there).

- Mach-3 argon shock (100 cells, 2e4 particles, pure DSMC, reservoirs): 500
  steps, time average of the last 250 (the shock structure of Sec. 4.1), 16
  replicas a side, FP64 and FP32+FP64 on the GPU.
- Sod tube at the paper's resolution, Kn = 1e-4 (absorption, resampling and the
  wave flux all active on the left): the ensemble average of 50 replicas at
  t = 0.15 (300 steps), as in Sec. 4.2, FP64 and FP32+FP64 on the GPU.
- Mach-10 shock in the near-continuum regime (cells of 1000 upstream mean free
  paths, nearly all particles absorbed and resampled every step, most of the
  mass in the wave part), 100 cells and 2e4 particles, every cell's
  collisions in the block-per-cell kernel: 200 steps, time average of the last
  100, 16 replicas a side.
"""
import numpy as np
import pytest

import _ensemble as E
from oracle import oracle as O
from paper_2305_12071_amd import duwp
from paper_2305_12071_amd import inputs as I

pytestmark = pytest.mark.gpu


def _gpu_runs(case, nrep, seed, steps, avg_from, prec, tune=None):
    g = duwp.Sim([case] * nrep, seed=seed, precision=prec, use_graph=True, tune=tune)
    if avg_from is None:
        g.step(steps)
        out = np.stack([g.moments(k, duwp.M_PRIM) for k in range(nrep)])
    else:
        g.step(avg_from)
        g.reset_average()
        g.step(steps - avg_from)
        out = np.stack([g.moments(k, duwp.M_AVG_PRIM) for k in range(nrep)])
    g.close()
    return out


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)
    duwp.lib()


_ORACLE = {}


def _oracle_ensemble(key, *args):
    """The oracle side, computed once per module for both GPU precisions."""
    if key not in _ORACLE:
        _ORACLE[key] = E.oracle_runs(*args)
    return _ORACLE[key]


@pytest.mark.parametrize("prec", [duwp.FP64, duwp.MIXED], ids=["fp64", "mixed"])
def test_mach3_time_averaged_profiles_match_oracle_ensemble(prec):
    c = I.mach3_small()
    nrep, steps, avg_from = 16, 500, 250
    E.say("mach3 long run", prec)
    gg = _gpu_runs(c, nrep, 1001, steps, avg_from, prec)
    oo = _oracle_ensemble("mach3", c, nrep, 2002, steps, avg_from)
    rep = E.compare(gg, oo, f"mach3 prec={prec}")
    # the standard error of the difference is about 0.7% of the density: the
    # mean square over the cells sees a shared bias of that size
    assert rep["rho"]["rel_se"] < 1e-2


@pytest.mark.parametrize("prec", [duwp.FP64, duwp.MIXED], ids=["fp64", "mixed"])
def test_sod_ensemble_at_t015_matches_oracle_ensemble(prec):
    c = I.sod_paper(1e-4)
    nrep, steps = 50, 300
    assert abs(steps * c.dt - 0.15) < 1e-12
    E.say("sod ensemble", prec)
    gg = _gpu_runs(c, nrep, 3003, steps, None, prec)
    oo = _oracle_ensemble("sod", c, nrep, 4004, steps, None)
    # the wave part carries most of the left state's mass at this Kn
    g1 = duwp.Sim(c, seed=5, precision=prec)
    g1.step(steps)
    wave = g1.moments(0, duwp.M_PSI_W)[:, 0] / g1.moments(0, duwp.M_PSI_T)[:, 0]
    g1.close()
    assert wave[:20].mean() > 0.5
    E.compare(gg, oo, f"sod Kn1e-4 prec={prec}")


@pytest.mark.parametrize("prec", [duwp.FP64, duwp.MIXED], ids=["fp64", "mixed"])
def test_near_continuum_shock_through_the_block_per_cell_collide(prec):
    c = I.mach10_large(ncells=100, n_kept=2e4)
    # thresholds lowered so that every cell (about 200 particles and 250
    # candidates) collides in the block-per-cell kernel, 256 candidates a chunk:
    # its waiting-candidate rounds and its serial path both run
    tune = {"big_min_particles": 64, "big_min_candidates": 64, "big_block": 256}
    nrep, steps, avg_from = 16, 200, 100
    E.say("near-continuum long run", prec)
    g1 = duwp.Sim(c, seed=7, precision=prec, tune=tune)
    g1.step(20)
    d = g1.diag()
    wave = g1.moments(0, duwp.M_PSI_W)[:, 0].sum() / g1.moments(0, duwp.M_PSI_T)[:, 0].sum()
    g1.close()
    assert wave > 0.9 and d["n_new"].sum() > 0.8 * d["n_abs"].sum() > 0
    gg = _gpu_runs(c, nrep, 5005, steps, avg_from, prec, tune=tune)
    oo = _oracle_ensemble("mach10", c, nrep, 6006, steps, avg_from)
    E.compare(gg, oo, f"mach10 near-continuum prec={prec}")
