"""The C-ABI library loads and exports every symbol declared in include/ntu.h
(host-side checks only: nothing here launches GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ntu.h")
LIB = os.path.join(ROOT, "paper_2107_06635_amd", "libntu.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ntu_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2107_06635_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("ntu_reduce_qr", "ntu_env_contract", "ntu_metric_fix", "ntu_bond_fit", "ntu_trotter_step",
              "ntu_gate_split", "ntu_recombine", "ntu_ctx_create", "ntu_ctx_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2107_06635_amd import ntu
    for n in declared_functions():
        assert n in ntu.EXPORTED or n in ("ntu_fit_opts_default", "ntu_step_opts_default")


def test_host_only_defaults(lib):
    from paper_2107_06635_amd import ntu
    o = ntu.FitOpts()
    lib.ntu_fit_opts_default.argtypes = [ctypes.POINTER(ntu.FitOpts)]
    lib.ntu_fit_opts_default(ctypes.byref(o))
    assert o.n_iter == 20 and o.n_tol == 8
    assert abs(o.tol[0] - 1e-15) < 1e-30 and abs(o.tol[7] - 1e-8) < 1e-20
    lib.ntu_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.ntu_version()
    # invalid arguments are rejected on the host before any launch
    lib.ntu_reduce_qr.restype = ctypes.c_int
    assert lib.ntu_reduce_qr(None, 1, 2, None, 0, None, 0, None, None) == -1
