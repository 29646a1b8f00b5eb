"""Training of the learned CG preconditioner on the method's own solves.

Pairs: for each material field and each load step k of the compression load
case, the residual at the start of step k (prescribed DOFs moved to step k,
free DOFs at the step k-1 equilibrium) and its exact Newton correction
delta = K^-1 (-r) (FP64 Jacobi-PCG to 1e-10), both from the library's own
kernels (efem_residual, efem_jacobi_diag, efem_linear_solve); the state then
advances with efem_newton_solve.  Training minimises the mean over pairs of
|M(-r) - delta|^2 / |delta|^2 with the library's MLP forward/backward kernels
and Adam (efem_mlp_loss_grad, efem_mlp_adam).  Torch only allocates, slices
and casts buffers.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib as L
from . import inputs as I
from .operator import Operator


def init_params(seed: int = 7, device="cuda") -> torch.Tensor:
    """Scaled-normal hidden layers; a zero output layer, so the untrained
    preconditioner is exactly Jacobi."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((L.EFEM_MLP_HID, L.EFEM_MLP_IN)) / np.sqrt(L.EFEM_MLP_IN)
    w2 = rng.standard_normal((L.EFEM_MLP_HID, L.EFEM_MLP_HID)) / np.sqrt(L.EFEM_MLP_HID)
    parts = [w1.ravel(), np.zeros(L.EFEM_MLP_HID), w2.ravel(), np.zeros(L.EFEM_MLP_HID),
             np.zeros(L.EFEM_MLP_OUT * L.EFEM_MLP_HID), np.zeros(L.EFEM_MLP_OUT)]
    theta = np.concatenate(parts)
    assert theta.size == L.EFEM_MLP_PARAMS
    return torch.tensor(theta, dtype=torch.float32, device=device)


def compression_case(elem, n, mu_seed, sigma=0.5, dz=-0.2):
    mesh = I.make_mesh(elem, n)
    mu = I.lognormal_field(mesh.n_elems, sigma, mu_seed)
    mask, ubc = I.clamp_top_bottom(mesh.X, dz)
    return mesh, mu, 1.5 * mu, mask, ubc


def generate_rows(n=32, seeds=range(1000, 1020), n_steps=10, elem=I.HEX8, device="cuda", log=None):
    """Training rows (X, aux) of len(seeds) * n_steps pairs, plus the operator
    that owns the MLP state used for training."""
    n_total = len(seeds) * n_steps
    Xs, auxs = [], []
    op_keep = None
    for seed in seeds:
        mesh, mu, lam, mask, ubc = compression_case(elem, n, seed)
        op = Operator(elem, mesh.X, mesh.conn, device=device)
        op.set_material(torch.as_tensor(mu, device=device), torch.as_tensor(lam, device=device))
        m = torch.as_tensor(mask, device=device)
        op.set_dirichlet(m)
        op.set_mlp(init_params(device=device))      # builds the node graph for the rows
        fixed = m.reshape(-1, 3).bool()
        ubc_t = torch.as_tensor(ubc, device=device)
        u = torch.zeros((mesh.n_nodes, 3), dtype=torch.float64, device=device)
        for k in range(1, n_steps + 1):
            u_start = torch.where(fixed, (k / n_steps) * ubc_t, u)
            r = op.residual(u_start)
            diag = op.jacobi_diag(u_start)
            delta, _, _ = op.linear_solve(u_start, r, rtol=1e-10, hvp_prec="f64", precond=0)
            X, aux = op.precond_rows((-r).float().contiguous(), diag, (-delta).float().contiguous(),
                                     n_total)
            Xs.append(X)
            auxs.append(aux)
            rc, st = op.newton_solve(u, ((k / n_steps) * ubc_t).contiguous(), n_steps=1)
            if rc != 0:
                raise RuntimeError(f"training solve did not converge (seed {seed}, step {k}): {st}")
        if log:
            log(f"pairs from mu seed {seed} done")
        if op_keep is None:
            op_keep = op
        else:
            op.close()
    return torch.cat(Xs), torch.cat(auxs), op_keep


def train(op: Operator, X, aux, epochs=400, lr=3e-3, seed=7, log=None):
    """Full-batch Adam on all rows; returns (params, loss history)."""
    theta = init_params(seed, device=op.device)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    loss = torch.empty((), dtype=torch.float64, device=op.device)
    hist = []
    t0 = time.time()
    for ep in range(1, epochs + 1):
        op.mlp_loss_grad(X, aux, theta, grad, loss)
        op.mlp_adam(theta, m, v, grad, lr, ep)
        if ep == 1 or ep % 50 == 0 or ep == epochs:
            hist.append((ep, float(loss)))
            if log:
                log(f"epoch {ep} loss {hist[-1][1]:.5f} ({time.time() - t0:.1f}s)")
    op.mlp_loss_grad(X, aux, theta, grad, loss)
    hist.append((epochs + 1, float(loss)))
    return theta, hist
