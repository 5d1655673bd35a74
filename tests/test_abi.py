"""The C-ABI library loads and exports every entry point declared in include/fe.h (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2604_22087_amd", "libfe.so")


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(fe_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fe_residual", "fe_tangent_csr", "fe_apply_matfree", "fe_vjp", "fe_pcg", "fe_newton",
                     "fe_csr_indices", "fe_apply_csr"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfe.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfe.so not built")
def test_binding_signatures_cover_header():
    from paper_2604_22087_amd import fe
    bound = {s[0] for s in fe.SIGNATURES}
    assert set(declared_functions()) == bound
    lib = fe.load_library()
    assert lib.fe_status_string(5) == b"CG breakdown (p.Ap <= 0)"
