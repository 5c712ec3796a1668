"""The autotuner's shape families and cache lookup (no GPU: a cache written here)."""
import json

from paper_2305_12071_amd import autotune as A
from paper_2305_12071_amd import duwp
from paper_2305_12071_amd import inputs as I


def test_families_separate_the_benchmark_workloads():
    keys = {A.key_of(A.family(c, p, arch="gfx950"))
            for c, p in (([I.mach8_shock()], duwp.MIXED), ([I.mach8_shock()], duwp.FP64),
                         ([I.mach10_large()], duwp.MIXED), (I.batched_cases(256), duwp.MIXED),
                         ([I.mach3_small()], duwp.FP64), (I.sod_kn_sweep(), duwp.FP64))}
    assert len(keys) == 6
    f = A.family([I.mach10_large()], duwp.MIXED, arch="gfx950")
    assert f["wave"] == 1 and A.family([I.mach8_shock()], duwp.MIXED, arch="gfx950")["wave"] == 0
    # a Mach-8 shock at a tenth of the particles is another family (particles per cell)
    assert A.key_of(A.family([I.mach8_shock(4000, 5e6)], duwp.MIXED, "gfx950")) != \
        A.key_of(A.family([I.mach8_shock()], duwp.MIXED, "gfx950"))


def test_lookup_exact_then_nearest_family(tmp_path):
    path = str(tmp_path / "cache.json")
    fam8 = A.family([I.mach8_shock()], duwp.MIXED, arch="gfx950")
    famb = A.family(I.batched_cases(256), duwp.MIXED, arch="gfx950")
    cache = {A.key_of(fam8): {"family": fam8, "block_cells": 256, "tune": {"scatter_items": 2}},
             A.key_of(famb): {"family": famb, "block_cells": 64, "tune": {"count_dests": 64}}}
    with open(path, "w") as f:
        json.dump(cache, f)
    bc, t, k = A.lookup([I.mach8_shock()], duwp.MIXED, path, arch="gfx950")
    assert (bc, t, k) == (256, {"scatter_items": 2}, A.key_of(fam8))
    # the same shock at 4e7 particles: same family (1e4 particles per cell rounds alike)
    assert A.lookup([I.mach8_shock(4000, 4e7)], duwp.MIXED, path, arch="gfx950")[2] == A.key_of(fam8)
    # 200 batched cases: nearest family is the 256-case batch
    bc, t, k = A.lookup(I.batched_cases(200), duwp.MIXED, path, arch="gfx950")
    assert (bc, k) == (64, A.key_of(famb))
    # another precision, architecture or wave regime has no entry
    assert A.lookup([I.mach8_shock()], duwp.FP64, path, arch="gfx950") is None
    assert A.lookup([I.mach8_shock()], duwp.MIXED, path, arch="gfx942") is None
    assert A.lookup([I.mach10_large()], duwp.MIXED, path, arch="gfx950") is None


def test_candidates_apply_to_the_right_fields():
    cfg = {"block_cells": 256, "tune": {}}
    c = A._apply(cfg, "big", (1024, 1))
    assert c["tune"] == {"big_block": 1024, "big_blocks_per_cu": 1} and cfg["tune"] == {}
    c = A._apply(c, "big_min", 1024)
    assert c["tune"]["big_min_particles"] == c["tune"]["big_min_candidates"] == 1024
    assert set(c["tune"]) <= set(duwp.TUNE_FIELDS)
    assert A._candidates("big", duwp.FP64, 4000, False) == []
    assert all(1 <= pc <= 8 for _, pc in A._candidates("big", duwp.MIXED, 4000, True))
    assert A._candidates("count_dests", duwp.MIXED, 4000, False) == []
    assert A._candidates("big_min", duwp.MIXED, 4000, False) == [2147483647]
    assert A._candidates("big_min", duwp.MIXED, 4000, True)[-1] == 2147483647
    assert A._candidates("collide_blocks_per_cu", duwp.MIXED, 257183, False) == [32, 64, 128]
    assert A._candidates("collide_blocks_per_cu", duwp.MIXED, 100, False) == []
