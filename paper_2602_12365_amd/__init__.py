"""MI355X-native hot path of the energy-based FEM method of arXiv 2602.12365:
global energy, residual and matrix-free tangent actions of a mesh, their
adjoints, and a matrix-free Newton-Krylov solve, behind the C-ABI of
``include/efem.h`` (``libefem.so``, hand-written HIP for gfx950).

Importing the package is cheap; the library is loaded on first use of the
operator API and fails loudly if it has not been built.
"""
__all__ = ["Operator", "EnergyFn", "ResidualFn", "energy", "residual", "inputs"]


import importlib


def __getattr__(name):
    if name in ("Operator", "EnergyFn", "ResidualFn", "energy", "residual"):
        return getattr(importlib.import_module(__name__ + ".operator"), name)
    if name == "inputs":
        return importlib.import_module(__name__ + ".inputs")
    raise AttributeError(name)
