"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer.

A small C driver (tests/oracle_asan_driver.c) calls every oracle entry point for
one case of each family the tests use: a shock between reservoirs (P = 0), Sod
tubes between walls with absorption and resampling (P > 0), both classification
laws, streamed absorption, the second-order flux, every eps law, the full-dt
DSMC duration, and a box at P near 1.  Any heap error, leak or undefined
behaviour ends the driver with a report and a non-zero status.
"""
import os
import shutil
import subprocess

import pytest

from oracle import oracle as O
from paper_2305_12071_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _cases():
    out = [I.mach3_small(), I.sod_paper(1e-5), I.sod_paper(3e-4)]
    c = I.sod_paper(1e-4)
    c.classify_law, c.eps_law = I.CLASSIFY_EXP, I.EPS_FULL
    out.append(c)
    c = I.sod_paper(1e-5)
    c.flux_order, c.eps_law, c.dsmc_full_dt = 2, I.EPS12, 1
    out.append(c)
    for law in (I.CLASSIFY_RATIONAL, I.CLASSIFY_EXP):
        b = I.box(12, 1.0, 1.0, 60, 3.0)
        b.absorb_stream, b.classify_law = 1, law
        out.append(b)
    b = I.box(6, 1.0, 1.0, 80, 30.0)      # P near 0.97
    b.eps_law = I.EPS0
    out.append(b)
    s = I.argon_shock(2.0, 40, 40.0, 4e3, name="shock_M2_abs")
    s.dt *= 1e3                           # cells of many mean free paths: absorbing reservoirs
    s.absorb_stream = 1
    out.append(s)
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_is_clean_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_asan")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall",
                    "-I", os.path.join(ROOT, "oracle"), "-o", exe,
                    os.path.join(HERE, "oracle_asan_driver.c"), O.SRC, "-lm"], check=True)
    fields = [n for n, _ in O._Case._fields_]
    lines = ["4"] + [" ".join(repr(getattr(c, f)) for f in fields) for c in _cases()]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.count("case ") == len(_cases()), r.stdout
