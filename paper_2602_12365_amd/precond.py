"""Training of the learned CG preconditioner on the method's own solves.

Two objectives, both evaluated by the library's kernels (torch only
allocates, slices and casts buffers):

* Energy norm (`generate_samples` + `train_energy`, the one the solver
  benchmarks use): samples are the residuals r that FP32 Jacobi-PCG actually
  meets (`efem_cg_snapshots`) on the first system of each load step of the
  compression case, linearized at the previous step's equilibrium (where the
  tangent is positive definite).  The loss is the K-norm error of one
  preconditioned step, sum_s w_s (z.Kz - 2 r.z), z = M(r), w_s = 1/(S r.D^-1 r),
  which needs no solves: `efem_mlp_energy_rows` forms z, K z and per-row
  pseudo-targets that turn `efem_mlp_loss_grad` into its gradient.
* Target fit (`generate_rows` + `train`, the configured 200-pair variant):
  the residual at each step's first Newton iterate (after the tangent
  predictor) with its exact Newton correction delta = K^-1(-r) as the target,
  mean |M(-r) - delta|^2/|delta|^2.  Kept as the first version: a 1-ring
  network cannot represent the global correction, and what it learns turns
  against the residuals that CG produces (r.z < 0 within a few iterations).
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
            # the first Newton iterate of the step: the prescribed increment dc
            # lifted into the free DOFs by the solver's tangent predictor,
            # K_ff d_f = -(K dc)_f at the previous equilibrium (K positive
            # definite there; the raw lift alone compresses the top layer of a
            # 32^3 mesh by 64%, where the tangent is indefinite)
            dc = torch.where(fixed, (k / n_steps) * ubc_t - u, torch.zeros_like(u))
            with op.unmasked():
                op.linearize(u, "f64")
                kdc = op.hvp(dc)
            d, _, _ = op.linear_solve(u, (-kdc).contiguous(), rtol=1e-4, hvp_prec="f64", precond=0)
            u_start = u + dc + d
            r = op.residual(u_start)
            diag = op.jacobi_diag(u_start)
            delta, _, _ = op.linear_solve(u_start, r, rtol=1e-10, hvp_prec="f64", precond=0)
            if not bool(torch.isfinite(delta).all()):
                raise RuntimeError(f"training pair without a finite correction (seed {seed}, step {k})")
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


# ------------------------------------------------------------ energy norm

class SampleSet:
    """Energy-norm samples of one or more operators: per state (operator,
    linearization point, residual snapshots), and the rows of all of them."""

    def __init__(self):
        self.states = []      # (op, u, R [k, n, 3] float32, first row, rows per sample)
        self.X = None
        self.aux = None
        self._X, self._aux = [], []
        self.n_rows = 0

    @property
    def n_samples(self):
        return sum(st[2].shape[0] for st in self.states)

    def add(self, op, u, diag, R):
        n = op.n_nodes
        first = self.n_rows
        for j in range(R.shape[0]):
            X, aux = op.precond_rows(R[j].contiguous(), diag, R[j].contiguous(), 1.0)
            self._X.append(X)
            self._aux.append(aux)
        self.n_rows += R.shape[0] * n
        self.states.append((op, u, R, first, n))

    def finish(self):
        self.X = torch.cat(self._X).contiguous()
        self.aux = torch.cat(self._aux).contiguous()
        self._X, self._aux = [], []
        return self


def generate_samples(n=32, seeds=range(1000, 1020), n_steps=10, snaps=(0, 5, 20, 60, 150),
                     elem=I.HEX8, device="cuda", log=None):
    """Residual snapshots of FP32 Jacobi-PCG on the first system of each load
    step, the tangent predictor K(u_k)_ff d_f = -(K(u_k) dc)_f with dc the
    increment of the prescribed values and u_k the equilibrium of step k
    (u_0 = 0), for k = 0..n_steps-1 and each material field; the state
    advances with efem_newton_solve.  Snapshots CG did not reach, or that are
    zero or not finite, are dropped."""
    S = SampleSet()
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
        for k in range(n_steps):
            if k > 0:
                rc, st = op.newton_solve(u, ((k / n_steps) * ubc_t).contiguous(), n_steps=1)
                if rc != 0:
                    raise RuntimeError(f"training solve did not converge (seed {seed}, step {k}): {st}")
            uk = u.clone()
            dc = torch.where(fixed, ubc_t / n_steps, torch.zeros_like(ubc_t)).contiguous()
            op.set_dirichlet(None)                  # K dc on the unmasked increment
            op.linearize(uk, "f64")
            kdc = op.hvp(dc)
            op.set_dirichlet(m)
            R, taken = op.cg_snapshots(uk, kdc, snaps, sign=-1.0)
            R = R[:taken]
            flat = R.reshape(R.shape[0], -1)
            keep = torch.isfinite(flat).all(dim=1) & (flat.abs().amax(dim=1) > 0)
            if bool(keep.any()):
                S.add(op, uk, op.jacobi_diag(uk), R[keep].contiguous())
        if log:
            log(f"samples from mu seed {seed} done")
    return S.finish()


def train_energy(S: SampleSet, epochs=300, lr=1e-3, seed=7, log=None):
    """Full-batch Adam on the energy-norm objective; returns (params, history
    of (epoch, objective)), the objective of the untrained (Jacobi) network
    first."""
    dev = S.X.device
    op_keep = S.states[0][0]
    theta = init_params(seed, device=dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    energy = torch.zeros((), dtype=torch.float64, device=dev)
    n_max = max(st[4] for st in S.states)
    z = torch.empty((n_max, 3), dtype=torch.float32, device=dev)
    kz = torch.empty_like(z)
    ns = float(S.n_samples)
    hist = []
    t0 = time.time()

    def objective_pass():
        energy.zero_()
        op_keep.set_mlp(theta)
        out = op_keep.mlp_forward(S.X)
        for op, u, R, first, n in S.states:
            op.linearize(u, "f32")
            for j in range(R.shape[0]):
                a, b = first + j * n, first + (j + 1) * n
                op.mlp_energy_rows(R[j], out[a:b], ns, S.aux[a:b], z[:n], kz[:n], energy)

    for ep in range(1, epochs + 1):
        objective_pass()
        if ep == 1 or ep % 50 == 0:
            hist.append((ep - 1, float(energy)))
            if log:
                log(f"epoch {ep - 1} energy objective {hist[-1][1]:.5f} ({time.time() - t0:.1f}s)")
        op_keep.mlp_loss_grad(S.X, S.aux, theta, grad, loss)
        op_keep.mlp_adam(theta, m, v, grad, lr, ep)
    objective_pass()
    hist.append((epochs, float(energy)))
    return theta, hist
