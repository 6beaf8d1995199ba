"""The C-ABI library loads and exports every entry point declared in
include/seird.h (CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "seird.h")
LIB = os.path.join(ROOT, "paper_2208_01839_amd", "libseird.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(seird_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("seird_problem_create", "seird_residual", "seird_jacobian",
                     "seird_spmv", "seird_precond_create", "seird_precond_setup",
                     "seird_precond_apply", "seird_gmres", "seird_step"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libseird.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.seird_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.seird_version()


def test_binding_exposes_the_same_names():
    import paper_2208_01839_amd as pk
    for n in declared_functions():
        assert n in pk._SIGS, n
