"""The HIP library loads on a host without a GPU and exports every entry point
that include/duwp.h declares.  No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_2305_12071_amd import duwp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "duwp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(duwp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_step_api():
    names = _declared()
    for n in ("duwp_init", "duwp_step", "duwp_moments", "duwp_get_state", "duwp_set_state",
              "duwp_destroy", "duwp_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(duwp.LIB):
        pytest.fail("libduwp.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(duwp.LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_without_device():
    lib = duwp.lib()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert lib.duwp_strerror(s)


def test_case_struct_layout_matches_header():
    # field order/size of the ctypes mirror against the C declaration
    src = open(os.path.join(ROOT, "include", "duwp.h")).read()
    body = src[src.index("typedef struct {\n    int32_t kind;"):src.index("} duwp_case;")]
    names = re.findall(r"\b([a-zA-Z_]+)\s*[,;]", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    assert names == [f for f, _ in duwp._Case._fields_]
    assert ctypes.sizeof(duwp._Case) == 4 * 2 + 8 * 18 + 4 * 8 + 8


def test_state_struct_layout_matches_header():
    src = open(os.path.join(ROOT, "include", "duwp.h")).read()
    body = src[src.index("typedef struct {\n    int64_t n_particles;"):src.index("} duwp_state;")]
    names = re.findall(r"\b([a-zA-Z_]+)\s*[,;]", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    assert names == [f for f, _ in duwp._State._fields_]
    assert duwp._State.psi_p.offset == 8 + 4 + 4 + 8 * 7
    assert duwp._State.avg_count.offset == 8 + 4 + 4 + 8 * 9
    assert ctypes.sizeof(duwp._State) == 8 + 4 + 4 + 8 * 10


def test_opts_and_tune_struct_layout_matches_header():
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "duwp.h")).read(), flags=re.S)
    body = src[src.index("typedef struct {\n    int32_t scatter_items;"):src.index("} duwp_tune;")]
    names = re.findall(r"\b([a-zA-Z_]+)\s*;", body)
    assert names == [f for f, _ in duwp._Tune._fields_]
    body = src[src.index("typedef struct {\n    uint64_t seed;"):src.index("} duwp_opts;")]
    names = re.findall(r"\b([a-zA-Z_]+)\s*;|\(\*([a-z_]+)\)", body)
    names = [a or b for a, b in names]
    assert names == [f for f, _ in duwp._Opts._fields_]
    assert duwp._Opts.alloc.offset == 40 and duwp._Opts.tune.offset == 64
    assert ctypes.sizeof(duwp._Opts) == 64 + 8 * 4


def _init_status(cases, precision=duwp.FP64, block_cells=0, tune=None, alloc_only=False):
    arr = (duwp._Case * len(cases))(*[c if isinstance(c, duwp._Case) else duwp.make_case(c) for c in cases])
    o = duwp._Opts()
    o.seed = 1
    o.precision = precision
    o.use_graph = 0
    o.stream = None
    o.headroom = 0.0
    o.block_cells = block_cells
    for k, v in (tune or {}).items():
        setattr(o.tune, k, v)
    if alloc_only:            # an allocator without its free
        o.alloc = duwp.ALLOC_FN(lambda n, c: None)
    ptr = ctypes.c_void_p()
    s = duwp.lib().duwp_init(ctypes.byref(ptr), arr, len(cases), ctypes.byref(o))
    assert not ptr.value
    return s


def test_init_rejects_bad_descriptors_before_any_device_call():
    # every argument is checked before the first device call, so these run
    # on a host without a GPU and leave nothing behind
    from dataclasses import replace
    from paper_2305_12071_amd import inputs as I
    EINVAL = -1
    good = I.box(4, 1.0, 1.0, 10, 0.5)
    for bad in (dict(ncells=0), dict(dt=0.0), dict(m_particle=-1.0), dict(x_hi=good.x_lo),
                dict(x_split=2.0), dict(rho_L=0.0), dict(T_R=-1.0), dict(lambda_ref=0.0),
                dict(bc_lo=2), dict(classify_law=2), dict(eps_law=4), dict(dsmc_full_dt=2),
                dict(absorb_stream=2)):
        assert _init_status([replace(good, **bad)]) == EINVAL, bad
    reserved = duwp.make_case(good)
    reserved.reserved_case = 1
    assert _init_status([reserved]) == EINVAL
    assert _init_status([good, replace(good, rho_R=-1.0)]) == EINVAL     # a bad second case
    assert _init_status([good], precision=7) == EINVAL
    for bc in (100, 1024, 96):
        assert _init_status([good], block_cells=bc) == EINVAL, bc
    for t in (dict(scatter_items=3), dict(big_block=128), dict(big_block=2048), dict(big_blocks_per_cu=9),
              dict(big_min_particles=10), dict(big_min_candidates=-1), dict(collide_by_cell_max=-5),
              dict(count_dests=6), dict(count_dests=512), dict(collide_blocks_per_cu=-1),
              dict(collide_blocks_per_cu=257)):
        assert _init_status([good], tune=t) == EINVAL, t
    assert _init_status([good], alloc_only=True) == EINVAL
