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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libefem.so not built")
def test_solve_options_layout_matches_the_header():
    """efem_solve_opts_default (host only) fills the ctypes mirror of
    efem_solve_opts: every field lands where the binding expects it."""
    from paper_2602_12365_amd import _lib
    lib = _lib.load()
    o = _lib.SolveOpts()
    lib.efem_solve_opts_default(ctypes.byref(o))
    assert (o.n_steps, o.hvp_prec, o.precond, o.max_newton, o.max_cg, o.check_every) == (5, 0, 0, 50, 20000, 8)
    assert (o.rtol, o.atol_floor, o.eta_max, o.eta_min) == (1e-8, 1e-14, 0.5, 1e-10)
    assert (o.ew_gamma, o.ew_alpha, o.eta_fixed, o.predictor_rtol, o.armijo_c) == (0.9, 2.0, 0.0, 1e-4, 1e-4)
    assert (o.max_halvings, o.verbose, o.learned_iters) == (30, 0, 8)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libefem.so not built")
def test_null_context_is_rejected_without_a_device():
    from paper_2602_12365_amd import _lib
    lib = _lib.load()
    assert lib.efem_set_load(None, None) == _lib.EFEM_ERR_INVALID
    assert lib.efem_set_dirichlet(None, None) == _lib.EFEM_ERR_INVALID


@pytest.mark.skipif(not os.path.exists(LIB), reason="libefem.so not built")
def test_create_rejects_bad_meshes_without_a_device():
    """Mesh validation runs on the host before any device call: an
    out-of-range connectivity entry, and a node that no element uses (the
    element passes would leave its output entries unwritten)."""
    import ctypes
    import numpy as np
    from paper_2602_12365_amd import _lib, inputs as I
    lib = _lib.load()
    m = I.tet_mesh(1)
    h = ctypes.c_void_p()

    def create(X, conn):
        X = np.ascontiguousarray(X, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        return lib.efem_create(ctypes.byref(h), I.TET4, X.shape[0], conn.shape[0],
                               X.ctypes.data_as(ctypes.c_void_p), conn.ctypes.data_as(ctypes.c_void_p),
                               None, None)
    bad = np.array(m.conn, copy=True)
    bad[0, 0] = m.n_nodes
    assert create(m.X, bad) == _lib.EFEM_ERR_INVALID
    X_extra = np.vstack([m.X, [[2.0, 2.0, 2.0]]])
    assert create(X_extra, m.conn) == _lib.EFEM_ERR_INVALID
    assert b"no element" in lib.efem_last_error()


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """No CPU fallback: without libefem.so the binding raises ImportError."""
    from paper_2602_12365_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libefem.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()
