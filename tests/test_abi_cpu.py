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
