"""duwp_moments_noalloc (the entry point for callers that cannot allocate) against
duwp_moments on the same state, through the C ABI: two calls in a row, the second
on a smaller case, for every kind of moment and both precisions."""
import sys

import numpy as np
import pytest

from paper_2305_12071_amd import duwp
from paper_2305_12071_amd import inputs as I

pytestmark = pytest.mark.gpu

WHATS = [duwp.M_PRIM, duwp.M_PSI_T, duwp.M_PSI_W, duwp.M_PSI_P, duwp.M_AVG_PRIM, duwp.M_AVG_SUM,
         duwp.M_STRESS_HEAT]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", [duwp.FP64, duwp.MIXED])
def test_noalloc_moments_equal_duwp_moments(prec):
    import torch
    # a tube with walls and absorption (wave stress present), a shock between
    # reservoirs, then a 7-cell box: each call after the first is on fewer cells
    cases = [I.sod_paper(1e-4), I.mach3_small(), I.box(7, 0.8, 2.0, 150, 3.0, u=0.3)]
    g = duwp.Sim(cases, seed=3, precision=prec)
    g.step(5)
    _say("noalloc moments", prec)
    for what in WHATS:
        for k in range(len(cases)):
            nc = cases[k].ncells
            out = torch.full((nc * 5 + 3,), float("nan"), dtype=torch.float64, device="cuda")
            g.moments_noalloc(out.data_ptr(), out.numel(), k, what)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert np.all(np.isnan(got[nc * 5:]))           # nothing written past the case
            got = got[:nc * 5].reshape(nc, 5)
            ref = g.moments(k, what)
            scale = np.maximum(np.abs(ref), 1e-300)
            err = float((np.abs(got - ref) / scale).max())
            assert err <= 1e-12, (prec, what, k, err)
            if what == duwp.M_STRESS_HEAT and k == 0:
                assert np.abs(ref[:, 0] - ref[:, 2]).max() > 0     # a wave part is present
    g.close()


def test_noalloc_rejects_cases_beyond_its_staging_array():
    import torch
    c = I.box(duwp_max_cells() + 1, 1.0, 1.0, 2, 0.5)
    g = duwp.Sim(c, seed=1)
    out = torch.zeros(c.ncells * 5, dtype=torch.float64, device="cuda")
    with pytest.raises(duwp.DuwpError) as e:
        g.moments_noalloc(out.data_ptr(), out.numel(), 0, duwp.M_STRESS_HEAT)
    assert e.value.status == -1
    g.moments_noalloc(out.data_ptr(), out.numel(), 0, duwp.M_PRIM)   # no staging needed
    torch.cuda.synchronize()
    g.close()


def duwp_max_cells():
    return 65536
