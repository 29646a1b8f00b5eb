"""The C-ABI library loads and exports every symbol include/efem.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "efem.h")
LIB = os.path.join(ROOT, "paper_2602_12365_amd", "libefem.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(efem_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["efem_create", "efem_destroy", "efem_set_material", "efem_set_dirichlet",
                     "efem_energy", "efem_residual", "efem_linearize", "efem_hvp",
                     "efem_jacobi_diag", "efem_grad_material", "efem_residual_vjp_material",
                     "efem_grad_coords", "efem_newton_solve", "efem_last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libefem.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libefem.so not built")
def test_binding_declares_every_symbol():
    from paper_2602_12365_amd import _lib
    assert set(declared_functions()) <= set(_lib.SIGNATURES)
    _lib.load()


def test_product_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2602_12365_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "efem_oracle" not in text and "liboracle" not in text, f


def test_oracle_does_not_import_product():
    for dirpath, _, files in os.walk(os.path.join(ROOT, "oracle")):
        for f in files:
            if f.endswith((".py", ".c", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"(import|from)\s+paper_2602_12365_amd", text), f
                assert "libefem" not in text, f
