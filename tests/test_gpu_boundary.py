"""The C ABI's conventions on the GPU: device memory from the caller's allocator,
checkpoints that carry the running time average, restores that change particle
counts inside a batch, a context reset after a reported error, and tile shapes
and thresholds that change no integer result."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_12071_amd import duwp
from paper_2305_12071_amd import inputs as I

from _parity import compare_diag, compare_states

pytestmark = pytest.mark.gpu

KEYS = ("x", "u", "v", "w", "off", "psi_w", "cr_max", "psi_p")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)
    duwp.lib()


def _same(a, b, keys=KEYS, label=""):
    for key in keys:
        assert np.array_equal(a[key], b[key]), (label, key)


def test_device_memory_comes_from_the_torch_allocator():
    """Every device buffer of a context comes from torch's caching allocator (the
    binding's default) and goes back to it at close; the results do not depend
    on the provider."""
    import torch
    cases = [I.mach3_small(), I.sod_paper(1e-4)]
    _say("torch allocator")
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    a = duwp.Sim(cases, seed=3, allocator="torch")
    held = torch.cuda.memory_allocated() - base
    assert held > 16 * 2 * 60000 and a.allocator.live > 40, (held, a.allocator.live)
    b = duwp.Sim(cases, seed=3, allocator="hip")
    assert torch.cuda.memory_allocated() - base == held      # hipMalloc is not torch's
    a.step(5)
    b.step(5)
    for k in range(2):
        _same(a.get_state(k), b.get_state(k), label=k)
    a.close()
    b.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    assert a.allocator.live == 0


@pytest.mark.parametrize("prec", [duwp.FP64, duwp.MIXED])
def test_checkpoint_inside_the_averaging_window_resumes_bitwise(prec):
    """A checkpoint taken in the middle of a time average carries the running sums
    and their count: the resumed context ends with the same average, bit for bit."""
    cases = [I.mach3_small(), I.sod_paper(1e-4)]
    _say("mid-average resume", prec)
    a = duwp.Sim(cases, seed=8, precision=prec)
    a.step(6)
    a.reset_average()
    a.step(5)
    saved = [a.get_state(k) for k in range(2)]
    assert saved[0]["avg_count"] == 5
    b = duwp.Sim(cases, seed=8, precision=prec)
    for k in range(2):
        b.set_state(saved[k], k)
    assert b.avg_count() == 5
    a.step(7)
    b.step(7)
    assert a.avg_count() == b.avg_count() == 12
    for k in range(2):
        ga, gb = a.get_state(k), b.get_state(k)
        _same(ga, gb, KEYS + ("avg_sum",), label=k)
        assert np.array_equal(a.moments(k, duwp.M_AVG_PRIM), b.moments(k, duwp.M_AVG_PRIM))
    a.close()
    b.close()


def test_restore_after_a_reported_error_resumes_like_the_oracle():
    """A step that reports DUWP_ERANGE leaves the context usable: restoring a valid
    state clears the error word, and the next steps match the oracle's."""
    c = I.box(60, 1.0, 1.0, 50, 1e-6)
    o = O.Oracle(c, seed=1, case_id=0)
    o.step(1)
    good = o.get_state()
    bad = dict(good)
    bad["u"] = np.array(good["u"], copy=True)
    bad["u"][int(good["off"][5])] = 25.0 * c.dx / c.dt
    g = duwp.Sim(c, seed=1, precision=duwp.FP64)
    g.set_state(bad)
    _say("error then restore")
    with pytest.raises(duwp.DuwpError) as e:
        g.step(1)
    assert e.value.status == -6
    with pytest.raises(duwp.DuwpError):
        g.sync()                    # the error stays until a restore
    g.set_state(good)
    g.sync()
    for k in range(3):
        g.step(1)
        o.step(1)
        compare_diag(g.diag(), o.diag(), f"after error:{k}")
    compare_states(g.get_state(), o.get_state(), rtol=1e-11, label="after error", psi_t=o.cells()["psi_t"])
    g.close()


def test_restore_reports_a_non_finite_loaded_total():
    c = I.sod_paper(1e-4)
    g = duwp.Sim(c, seed=3)
    g.step(2)
    good = g.get_state()
    st = dict(good)
    st["psi_w"] = good["psi_w"].copy()
    st["psi_w"][4, 4] = np.inf
    with pytest.raises(duwp.DuwpError) as e:
        g.set_state(st)
    assert e.value.status == -5
    g.set_state(good)               # a finite state resets the context
    g.step(1)
    g.close()


@pytest.mark.parametrize("prec", [duwp.FP64, duwp.MIXED])
def test_batched_restores_that_change_counts(prec):
    """Four cases in one context; the two middle ones are restored from states of
    another run (other particle counts), so the records of the cases after them move
    on the device.  One step later each restored case matches its oracle (FP64), and
    the untouched cases match a context that was never restored, bit for bit."""
    names = ["mach3", "sod_kn1e-4", "box", "sod_kn1e-2"]
    cases = [I.mach3_small(), I.sod_paper(1e-4), I.box(7, 0.8, 2.0, 150, 0.5, u=0.3), I.sod_paper(1e-2)]
    _say("batched count-changing restore", prec)
    g = duwp.Sim(cases, seed=5, precision=prec)
    ref = duwp.Sim(cases, seed=5, precision=prec)
    g.step(5)
    ref.step(5)
    other = {}
    for k in (1, 2):
        o = O.Oracle(cases[k], seed=77, case_id=k)
        o.step(5)
        other[k] = o.get_state()
    # the box's count does not depend on the seed: three particles of its cell 3 go
    st = other[2]
    b = int(st["off"][4])
    other[2] = dict(st, off=np.concatenate([st["off"][:4], st["off"][4:] - 3]),
                    **{a: np.delete(st[a], [b - 1, b - 2, b - 3]) for a in ("x", "u", "v", "w")})
    for k in (1, 2):
        assert len(other[k]["x"]) != g.n_particles(k)
    for k in (1, 2):
        g.set_state(other[k], k)
        _same(g.get_state(k), dict(other[k], psi_p=g.get_state(k)["psi_p"]),
              ("off",) + (("x", "u", "v", "w", "psi_w", "cr_max") if prec == duwp.FP64 else ("psi_w", "cr_max")),
              label=f"roundtrip {k}")
    g.step(1)
    ref.step(1)
    for k in (0, 3):
        _same(g.get_state(k), ref.get_state(k), label=names[k])
    if prec == duwp.FP64:
        for k in (1, 2):
            o = O.Oracle(cases[k], seed=5, case_id=k)
            o.set_state(other[k])
            o.step(1)
            compare_diag(g.diag(k), o.diag(), names[k])
            compare_states(g.get_state(k), o.get_state(), label=names[k], psi_t=o.cells()["psi_t"])
    g.close()
    ref.close()


TUNINGS = [
    dict(scatter_items=2),
    dict(big_min_particles=64, big_min_candidates=64),
    dict(big_min_particles=64, big_min_candidates=64, big_block=1024, big_blocks_per_cu=1),
    dict(big_min_particles=64, big_min_candidates=64, big_block=512, big_blocks_per_cu=1),
    dict(collide_by_cell_max=1, count_dests=4),
    dict(collide_by_cell_max=1, count_dests=64, scatter_items=2),
    dict(collide_by_cell_max=1, collide_blocks_per_cu=128),
    dict(big_min_particles=2147483647, big_min_candidates=2147483647),
    dict(big_min_particles=64, big_min_candidates=64, big_block=256, big_blocks_per_cu=6),
]


@pytest.mark.parametrize("tune", TUNINGS, ids=[",".join(f"{k}={v}" for k, v in t.items()) for t in TUNINGS])
def test_tuned_configurations_match_the_oracle_bitwise(tune):
    """Each tile shape and threshold the autotuner chooses from, on a batch whose
    large cells reach the block-per-cell collide under the low thresholds: integer
    results equal the oracle's, floating results within the parity tolerance, and
    every field equals the default configuration's bit for bit (to rounding where
    the scatter's chunks, which order the particle moment sums, change)."""
    cases = [I.mach3_small(), I.sod_paper(1e-2), I.sod_paper(1e-4), I.box(12, 1.0, 1.0, 300, 30.0)]
    _say("tuning", tune)
    g = duwp.Sim(cases, seed=9, precision=duwp.FP64, tune=tune)
    d = duwp.Sim(cases, seed=9, precision=duwp.FP64)
    ors = [O.Oracle(c, seed=9, case_id=k) for k, c in enumerate(cases)]
    for s in range(4):
        g.step(1)
        d.step(1)
        for k, o in enumerate(ors):
            o.step(1)
            compare_diag(g.diag(k), o.diag(), f"{k}:{s}")
    for k, o in enumerate(ors):
        gs, ds = g.get_state(k), d.get_state(k)
        compare_states(gs, o.get_state(), rtol=1e-11, label=str(k), psi_t=o.cells()["psi_t"])
        if "scatter_items" in tune:
            # the scatter's chunks set the order of the particle moment sums
            compare_states(gs, ds, rtol=1e-11, label=f"default {k}", psi_t=o.cells()["psi_t"])
        else:
            _same(gs, ds, label=f"default {k}")
    g.close()
    d.close()


@pytest.mark.parametrize("tune", TUNINGS[1:4], ids=["b512x2", "b1024x1", "b512x1"])
def test_tuned_big_cell_collide_mixed_equals_default(tune):
    """The FP32 block-per-cell collide at each block shape gives the default's result bit
    for bit (sequential candidate semantics whatever the chunk)."""
    cases = [I.sod_paper(1e-2), I.box(12, 1.0, 1.0, 300, 30.0)]
    g = duwp.Sim(cases, seed=2, precision=duwp.MIXED, tune=tune)
    d = duwp.Sim(cases, seed=2, precision=duwp.MIXED, tune=dict(big_min_particles=64, big_min_candidates=64))
    g.step(4)
    d.step(4)
    for k in range(2):
        _same(g.get_state(k), d.get_state(k), label=k)
    assert g.diag(0)["n_coll"].sum() > 1000
    g.close()
    d.close()


def test_closing_graph_contexts_returns_their_memory():
    """A context closed right after graph replays (no synchronization by the caller)
    returns every device buffer: free memory after three such contexts is what it
    was before the first."""
    import torch
    c = I.mach8_shock(1000, 1e7)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for k in range(3):
        g = duwp.Sim(c, seed=1, precision=duwp.MIXED, use_graph=True, allocator="hip")
        g.step(3)
        g.close()
    torch.cuda.synchronize()
    lost = free0 - torch.cuda.mem_get_info()[0]
    assert lost < 64 << 20, lost        # each context holds about 0.7 GB
