"""ctypes declarations of the C-ABI in ``include/efem.h`` (argument marshalling only).

Loading fails loudly when ``libefem.so`` has not been built: there is no CPU
fallback on the product path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libefem.so")

EFEM_OK = 0
EFEM_NOT_CONVERGED = 1
EFEM_ERR_INVALID = -1
EFEM_ERR_HIP = -2
EFEM_ERR_OOM = -3
EFEM_ERR_INVERTED = -4
EFEM_ERR_STATE = -5

EFEM_TET4, EFEM_HEX8, EFEM_TRI3 = 0, 1, 2
EFEM_F64, EFEM_F32 = 0, 1
EFEM_MODEL_NEO_HOOKE, EFEM_MODEL_LINEAR, EFEM_MODEL_TRANSPORT = 0, 1, 2
EFEM_SCATTER_HALO, EFEM_SCATTER_COLOR, EFEM_SCATTER_ATOMIC = 0, 1, 2

EFEM_MLP_IN, EFEM_MLP_HID, EFEM_MLP_OUT = 12, 64, 3
EFEM_MLP_PARAMS, EFEM_MLP_AUX = 5187, 12

c_void_p = ctypes.c_void_p
c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double


class Options(ctypes.Structure):
    _fields_ = [("block_elems", c_int32), ("block_nodes", c_int32), ("scatter", c_int32),
                ("threads", c_int32), ("no_pairs", c_int32), ("no_chunks", c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_blocks", c_int32), ("n_colours", c_int32), ("max_block_nodes", c_int32),
                ("max_block_elems", c_int32), ("n_shared_nodes", c_int64),
                ("n_block_nodes", c_int64), ("n_items", c_int64), ("n_chunks", c_int32),
                ("max_chunk_slots", c_int32), ("n_chunk_slots", c_int64),
                ("n_chunk_shared_nodes", c_int64)]


class SparseInfo(ctypes.Structure):
    _fields_ = [("n_rows", c_int64), ("nnz", c_int64), ("n_colours", c_int32), ("max_row", c_int32),
                ("setup_seconds", c_double), ("n_blocks", c_int64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("n_steps", c_int32), ("hvp_prec", c_int32), ("precond", c_int32),
                ("max_newton", c_int32), ("max_cg", c_int32), ("check_every", c_int32),
                ("rtol", c_double), ("atol_floor", c_double), ("eta_max", c_double),
                ("eta_min", c_double), ("ew_gamma", c_double), ("ew_alpha", c_double),
                ("eta_fixed", c_double), ("predictor_rtol", c_double), ("armijo_c", c_double),
                ("max_halvings", c_int32), ("verbose", c_int32), ("learned_iters", c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("converged", c_int32), ("steps_done", c_int32), ("newton_iters", c_int32),
                ("cg_iters", c_int32), ("precond_fallbacks", c_int32),
                ("line_search_halvings", c_int32), ("final_residual", c_double),
                ("final_energy", c_double), ("seconds", c_double),
                ("newton_per_step", c_int32 * 64), ("cg_per_step", c_int32 * 64)]


# name -> (restype, argtypes); every symbol declared in include/efem.h
SIGNATURES = {
    "efem_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, c_int64, c_int64, c_void_p,
                              c_void_p, ctypes.POINTER(Options), c_void_p]),
    "efem_destroy": (None, [c_void_p]),
    "efem_set_stream": (c_int32, [c_void_p, c_void_p]),
    "efem_set_material": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_set_model": (c_int32, [c_void_p, c_int32]),
    "efem_set_dirichlet": (c_int32, [c_void_p, c_void_p]),
    "efem_set_load": (c_int32, [c_void_p, c_void_p]),
    "efem_set_coords": (c_int32, [c_void_p, c_void_p]),
    "efem_energy": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_energy_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_residual": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_linearize": (c_int32, [c_void_p, c_void_p, c_int32]),
    "efem_hvp": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_hvp_acc": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_hvp_zeroed": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_jacobi_diag": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_jacobi_offdiag": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_grad_material": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "efem_residual_vjp_material": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "efem_grad_coords": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_get_info": (c_int32, [c_void_p, ctypes.POINTER(Info)]),
    "efem_status": (c_int32, [c_void_p, ctypes.POINTER(c_int32)]),
    "efem_solve_opts_default": (None, [ctypes.POINTER(SolveOpts)]),
    "efem_newton_solve": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveOpts),
                                    ctypes.POINTER(SolveStats)]),
    "efem_set_mlp": (c_int32, [c_void_p, c_void_p]),
    "efem_precond_apply": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "efem_precond_rows": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                                    c_void_p]),
    "efem_mlp_forward": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p]),
    "efem_mlp_forward_layers": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "efem_mlp_loss_grad": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p]),
    "efem_mlp_adam": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_float,
                                c_int32]),
    "efem_mlp_energy_rows": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p,
                                       c_void_p, c_void_p]),
    "efem_cg_snapshots": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_int32, c_void_p,
                                    c_void_p, ctypes.POINTER(c_int32)]),
    "efem_sparse_setup": (c_int32, [c_void_p, c_void_p]),
    "efem_sparse_pattern": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "efem_sparse_assemble": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_sparse_block_pattern": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "efem_sparse_spmv": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "efem_linear_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32,
                                    c_int32, c_int32, ctypes.POINTER(c_int32),
                                    ctypes.POINTER(c_int32)]),
    "efem_gmres_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32,
                                   c_int32, c_int32, ctypes.POINTER(c_int32),
                                   ctypes.POINTER(c_double)]),
    "efem_set_velocity": (c_int32, [c_void_p, ctypes.POINTER(c_double)]),
    "efem_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load ``libefem.so`` (built by ``python -m paper_2602_12365_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2602_12365_amd.build` (hipcc, gfx950)")
    import torch  # noqa: F401  -- share torch's HIP runtime (same SONAME) in this process
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class EfemError(RuntimeError):
    def __init__(self, rc, where):
        msg = load().efem_last_error().decode(errors="replace")
        super().__init__(f"{where} failed (rc={rc}): {msg}")
        self.rc = rc


def check(rc, where):
    if rc < 0:
        raise EfemError(rc, where)
    return rc
