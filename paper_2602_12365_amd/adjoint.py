"""Derivatives through the equilibrium solve (the adjoint method).

The paper differentiates a quantity of interest through a Newton solve with
forward-mode AD (Sec. 6.2).  Here the same derivative comes from one linear
solve with the tangent at equilibrium, assembled from the library's calls:

Objective: the total reaction on a set T of prescribed DOFs (for example the
z components of the loaded face), J(m) = sum_{i in T} r_i(u*(m), m), where
u*(m) solves the reduced equilibrium r_F(u*, m) = 0 with the prescribed values
held, and m = (mu_e, lam_e) is the per-element material.  Differentiating the
constraint, K_FF du_F = -(dr_F/dm) dm with du_T = 0, so

    dJ/dm = (1_T - lambda) . dr/dm,   K_FF lambda_F = (K 1_T)_F,  lambda_T = 0.

K 1_T is one tangent action without the Dirichlet mask, lambda one masked
Krylov solve (efem_linear_solve), and the product with dr/dm one residual
vector-Jacobian product (efem_residual_vjp_material, which ignores the mask).
This is a caller-side composition of three library calls: torch allocates the
nodal vectors, forms 1_T and the difference 1_T - lambda, and sums the
selected reaction entries; every element loop and Krylov iteration runs in
the library.
"""
from __future__ import annotations

import torch

from .operator import Operator


def unmasked(op: Operator):
    """Temporarily remove the operator's Dirichlet mask (the mask in force on
    entry, if any, is restored on exit)."""
    return op.unmasked()


def reaction(op: Operator, u: torch.Tensor, sel: torch.Tensor) -> float:
    """J = sum of the residual (the reaction) over the DOFs selected by sel
    (bool or uint8 [3 n_nodes])."""
    with unmasked(op):
        r = op.residual(u)
    return float((r.reshape(-1) * sel.reshape(-1).to(r.dtype)).sum())


def reaction_gradient(op: Operator, u: torch.Tensor, sel: torch.Tensor, rtol: float = 1e-12):
    """(dJ/dmu_e, dJ/dlam_e) at the equilibrium u of the operator's Dirichlet
    problem, plus the number of CG iterations of the adjoint solve."""
    ones_t = sel.reshape(op.n_nodes, 3).to(torch.float64).contiguous()
    with unmasked(op):
        op.linearize(u, "f64")
        k1 = op.hvp(ones_t)
    lam, iters, _ = op.linear_solve(u, k1, rtol=rtol, hvp_prec="f64")
    w = (ones_t - lam).contiguous()
    dmu, dlam = op.residual_vjp_material(u, w)
    return dmu, dlam, iters
