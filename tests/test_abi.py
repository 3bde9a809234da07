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
    assert lib.ntu_reduce_qr(None, 1, None, None, 0, None, None) == -1
    lib.ntu_trotter_step.restype = ctypes.c_int
    assert lib.ntu_trotter_step(None, 1, None, None, None, None, None) == -1


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structures have the C layout of ntu_tensor,
    ntu_fit_opts, ntu_step_opts and ntu_evolve_opts (offsets printed by a program compiled
    against the header with the host C compiler)."""
    import shutil
    import subprocess
    from paper_2107_06635_amd import ntu
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    fields = {"ntu_tensor": (ntu.Tensor, ["data", "dtype", "ndim", "shape", "stride"]),
              "ntu_fit_opts": (ntu.FitOpts, ["n_iter", "early_stop", "conv_tol", "kappa", "n_tol", "tol", "tie"]),
              "ntu_step_opts": (ntu.StepOpts, ["n_bonds", "order", "precision", "fix_mode", "fit", "scheme",
                                               "graph"]),
              "ntu_evolve_opts": (ntu.EvolveOpts, ["n_steps", "measure_every", "ctm_iters", "ctm_continue",
                                                   "energy_tol"])}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "ntu.h"', "int main(void) {"]
    for st, (_, names) in fields.items():
        src.append(f'  printf("{st} size %zu\\n", sizeof({st}));')
        for f in names:
            src.append(f'  printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    src.append("  return 0;\n}")
    (tmp_path / "layout.c").write_text("\n".join(src))
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(tmp_path / "layout.c"), "-o",
                    str(tmp_path / "layout")], check=True)
    out = subprocess.run([str(tmp_path / "layout")], check=True, capture_output=True, text=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for st, (cls, names) in fields.items():
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for f in names:
            assert got[(st, f)] == getattr(cls, f).offset, (st, f)
