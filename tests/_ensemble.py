"""Comparison of two independent replica ensembles of averaged profiles (rho, U, T
per cell): Welch t statistics with a Bonferroni allowance, and the mean square
of the statistics over the cells."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy import stats

from oracle import oracle as O

QUANT = {"rho": 0, "U": 1, "T": 4}
ALPHA = 1e-3            # family-wise false-alarm rate of the per-cell tests


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def threads():
    return max(1, min(16, os.cpu_count() or 1))


def oracle_runs(case, nrep, seed, steps, avg_from):
    """nrep oracle replicas (case ids 0..nrep-1 of `seed`), in parallel threads (the
    C calls release the interpreter); returns (nrep, C, 5) primitive profiles:
    time-averaged over the steps after avg_from, or the last state when
    avg_from is None."""
    def run(k):
        o = O.Oracle(case, seed=seed, case_id=k)
        if avg_from is None:
            o.step(steps)
            return o.cells()["prim"]
        o.step(avg_from)
        o.reset_average()
        o.step(steps - avg_from)
        s, n = o.average()
        return O.prim_from_psi(s / n, case.R)
    with ThreadPoolExecutor(threads()) as ex:
        return np.stack(list(ex.map(run, range(nrep))))


def compare(a, b, label):
    """Welch t statistics per cell and quantity of two replica sets (nrep, C, 5)."""
    na, nb = a.shape[0], b.shape[0]
    worst, report = 0.0, {}
    tcrit = None
    for name, q in QUANT.items():
        ma, mb = a[:, :, q].mean(0), b[:, :, q].mean(0)
        va, vb = a[:, :, q].var(0, ddof=1) / na, b[:, :, q].var(0, ddof=1) / nb
        se = np.sqrt(va + vb)
        keep = se > 0
        t = np.zeros_like(se)
        t[keep] = (ma[keep] - mb[keep]) / se[keep]
        assert np.all(ma[~keep] == mb[~keep]), (label, name)
        # Welch-Satterthwaite degrees of freedom (the smallest over the cells)
        dof = np.min((va + vb)[keep] ** 2 / (va[keep] ** 2 / (na - 1) + vb[keep] ** 2 / (nb - 1)))
        ntests = len(QUANT) * a.shape[1]
        tcrit = stats.t.ppf(1.0 - ALPHA / (2 * ntests), dof)
        report[name] = dict(max_t=float(np.abs(t).max()), mean_t2=float((t[keep] ** 2).mean()),
                            tcrit=float(tcrit), rel_se=float(np.median(se[keep] / np.maximum(np.abs(mb[keep]), 1e-300))))
        worst = max(worst, float(np.abs(t).max()) / tcrit)
        assert np.abs(t).max() < tcrit, (label, name, report[name])
        # the mean square of t over the cells: about dof/(dof-2) for unbiased sides
        assert report[name]["mean_t2"] < 2.0, (label, name, report[name])
    say(label, report)
    return report


