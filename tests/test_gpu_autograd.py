"""Hand-written adjoints through torch.autograd.Function (EnergyFn, ResidualFn):
gradients with respect to u, the per-element material fields and the nodal
coordinates, against the oracle and against central finite differences."""
import numpy as np
import pytest
import torch

from oracle import fem as F
from paper_2602_12365_amd import inputs as I

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype=dtype)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("elem", [I.TET4, I.HEX8])
def test_energy_fn_backward_matches_oracle(elem):
    from paper_2602_12365_amd import Operator, energy
    m = I.make_mesh(elem, 5)
    mu_h = I.lognormal_field(m.n_elems, 0.3, 4)
    lam_h = 1.5 * np.ones(m.n_elems)
    u_h = I.gaussian_field(m.n_nodes, 0.015, 0)
    op = Operator(elem, m.X, m.conn)
    u = dev(u_h).requires_grad_()
    mu = dev(mu_h).requires_grad_()
    lam = dev(lam_h).requires_grad_()
    X = op.X.clone().requires_grad_()
    psi = energy(op, u, mu, lam, X)
    (2.0 * psi).backward()
    orc = F.FEM(elem, m.X, m.conn, mu_h, lam_h)
    assert abs(psi.item() - orc.energy(u_h)) <= 1e-12 * orc.energy(u_h)
    gm, gl = orc.grad_material(u_h)
    assert rel(u.grad.cpu().numpy(), 2 * orc.residual(u_h)) <= 1e-10
    assert rel(mu.grad.cpu().numpy(), 2 * gm) <= 1e-10
    assert rel(lam.grad.cpu().numpy(), 2 * gl) <= 1e-10
    assert rel(X.grad.cpu().numpy(), 2 * orc.grad_coords(u_h)) <= 1e-10


@pytest.mark.parametrize("elem", [I.TET4, I.HEX8])
def test_residual_fn_backward_matches_oracle(elem):
    from paper_2602_12365_amd import Operator, residual
    m = I.make_mesh(elem, 4)
    mu_h = I.lognormal_field(m.n_elems, 0.3, 4)
    lam_h = 1.5 * mu_h
    u_h = I.gaussian_field(m.n_nodes, 0.015, 0)
    w_h = I.unit_direction(m.n_nodes, 9)
    op = Operator(elem, m.X, m.conn)
    u = dev(u_h).requires_grad_()
    mu = dev(mu_h).requires_grad_()
    lam = dev(lam_h).requires_grad_()
    r = residual(op, u, mu, lam)
    r.backward(dev(w_h))
    orc = F.FEM(elem, m.X, m.conn, mu_h, lam_h)
    vm, vl = orc.residual_vjp_material(u_h, w_h)
    assert rel(r.detach().cpu().numpy(), orc.residual(u_h)) <= 1e-10
    assert rel(u.grad.cpu().numpy(), orc.hvp(u_h, w_h)) <= 1e-10
    assert rel(mu.grad.cpu().numpy(), vm) <= 1e-10
    assert rel(lam.grad.cpu().numpy(), vl) <= 1e-10


# Nodal sums meet in LDS through FP64 atomics whose order between waves varies
# from call to call (the C-ABI documents last-bit variation), so a backward
# pass repeated on the same input agrees to rounding, not bitwise.
NONDET = 1e-12


def test_gradcheck_material_small():
    """torch.autograd.gradcheck (central differences) of EnergyFn and ResidualFn."""
    from paper_2602_12365_amd import Operator, EnergyFn, ResidualFn
    m = I.tet_mesh(2)
    op = Operator(I.TET4, m.X, m.conn)
    u = dev(I.gaussian_field(m.n_nodes, 0.02, 0)).requires_grad_()
    mu = dev(I.lognormal_field(m.n_elems, 0.3, 4)).requires_grad_()
    lam = dev(1.5 * np.ones(m.n_elems)).requires_grad_()
    X = op.X.clone().requires_grad_()
    assert torch.autograd.gradcheck(lambda a, b, c: EnergyFn.apply(a, b, c, X, op), (u, mu, lam),
                                    eps=1e-6, atol=1e-9, rtol=1e-6, nondet_tol=NONDET)
    assert torch.autograd.gradcheck(lambda a, b, c: ResidualFn.apply(a, b, c, op), (u, mu, lam),
                                    eps=1e-6, atol=1e-9, rtol=1e-6, nondet_tol=NONDET)


def test_gradcheck_with_dirichlet_mask():
    """gradcheck of EnergyFn and ResidualFn with a Dirichlet mask in force: the
    energy depends on every DOF (its u-gradient is the full residual), the
    masked residual's VJP is K P w and (P w).dr/dm."""
    from paper_2602_12365_amd import Operator, EnergyFn, ResidualFn
    m = I.tet_mesh(2)
    op = Operator(I.TET4, m.X, m.conn)
    mask, _ = I.clamp_top_bottom(m.X, 0.05)
    op.set_dirichlet(dev(mask, torch.uint8))
    u = dev(I.gaussian_field(m.n_nodes, 0.02, 0)).requires_grad_()
    mu = dev(I.lognormal_field(m.n_elems, 0.3, 4)).requires_grad_()
    lam = dev(1.5 * np.ones(m.n_elems)).requires_grad_()
    X = op.X.clone().requires_grad_()
    assert torch.autograd.gradcheck(lambda a, b, c: EnergyFn.apply(a, b, c, X, op), (u, mu, lam),
                                    eps=1e-6, atol=1e-9, rtol=1e-6, nondet_tol=NONDET)
    assert torch.autograd.gradcheck(lambda a, b, c: ResidualFn.apply(a, b, c, op), (u, mu, lam),
                                    eps=1e-6, atol=1e-9, rtol=1e-6, nondet_tol=NONDET)
    assert op.mask is not None   # the backward passes put the mask back


def test_residual_fn_masked_backward_matches_oracle():
    """With a mask, r.backward(w) gives K(u) P w and (P w).dr/dm (P zeroes the
    prescribed components), against the oracle's unmasked tangent action and
    material VJP on P w."""
    from paper_2602_12365_amd import Operator, residual
    m = I.hex_mesh(3)
    mu_h = I.lognormal_field(m.n_elems, 0.3, 4)
    lam_h = 1.5 * mu_h
    u_h = I.gaussian_field(m.n_nodes, 0.015, 0)
    w_h = I.unit_direction(m.n_nodes, 9)
    mask, _ = I.clamp_top_bottom(m.X, 0.05)
    op = Operator(I.HEX8, m.X, m.conn)
    op.set_dirichlet(dev(mask, torch.uint8))
    u = dev(u_h).requires_grad_()
    mu = dev(mu_h).requires_grad_()
    lam = dev(lam_h).requires_grad_()
    r = residual(op, u, mu, lam)
    r.backward(dev(w_h))
    pw = np.where(mask.reshape(-1, 3) != 0, 0.0, w_h.reshape(-1, 3))
    orc = F.FEM(I.HEX8, m.X, m.conn, mu_h, lam_h)
    r_ref = np.where(mask.reshape(-1, 3) != 0, 0.0, orc.residual(u_h).reshape(-1, 3))
    vm, vl = orc.residual_vjp_material(u_h, pw)
    assert rel(r.detach().cpu().numpy().reshape(-1, 3), r_ref) <= 1e-10
    assert rel(u.grad.cpu().numpy(), orc.hvp(u_h, pw)) <= 1e-10
    assert rel(mu.grad.cpu().numpy(), vm) <= 1e-10
    assert rel(lam.grad.cpu().numpy(), vl) <= 1e-10


def test_energy_fn_uses_given_coordinates():
    """EnergyFn evaluated at coordinates other than the operator's: the value
    and every gradient are those of the given X (the operator is moved there)."""
    from paper_2602_12365_amd import Operator, energy
    m = I.tet_mesh(3)
    mu_h = I.lognormal_field(m.n_elems, 0.3, 4)
    lam_h = 1.5 * np.ones(m.n_elems)
    u_h = I.gaussian_field(m.n_nodes, 0.015, 0)
    X2_h = m.X + I.gaussian_field(m.n_nodes, 0.01, 11)
    op = Operator(I.TET4, m.X, m.conn)
    u = dev(u_h).requires_grad_()
    X2 = dev(X2_h).requires_grad_()
    psi = energy(op, u, dev(mu_h), dev(lam_h), X2)
    psi.backward()
    orc = F.FEM(I.TET4, X2_h, m.conn, mu_h, lam_h)
    assert abs(psi.item() - orc.energy(u_h)) <= 1e-12 * abs(orc.energy(u_h))
    assert rel(u.grad.cpu().numpy(), orc.residual(u_h)) <= 1e-10
    assert rel(X2.grad.cpu().numpy(), orc.grad_coords(u_h)) <= 1e-10


def test_unmasked_restores_only_the_mask_in_force():
    """A mask removed with set_dirichlet(None) stays removed after an unmasked
    section (the reaction helpers use one)."""
    from paper_2602_12365_amd import Operator
    from paper_2602_12365_amd.adjoint import reaction
    m = I.tet_mesh(2)
    op = Operator(I.TET4, m.X, m.conn)
    mask, _ = I.clamp_top_bottom(m.X, 0.05)
    op.set_dirichlet(dev(mask, torch.uint8))
    op.set_dirichlet(None)
    u = dev(I.gaussian_field(m.n_nodes, 0.02, 0))
    sel = dev(mask, torch.uint8)
    reaction(op, u, sel)
    assert op.mask is None
    r = op.residual(u).cpu().numpy().reshape(-1)
    orc = F.FEM(I.TET4, m.X, m.conn, np.ones(m.n_elems), 1.5 * np.ones(m.n_elems))
    assert rel(r, orc.residual(u.cpu().numpy()).reshape(-1)) <= 1e-10   # no mask applied


def solve_equilibrium(op, m, mu, dz, n_steps, u0=None, **kw):
    mask, ubc = I.clamp_top_bottom(m.X, dz)
    op.set_material(dev(mu), dev(1.5 * np.ones(m.n_elems)))
    op.set_dirichlet(dev(mask, torch.uint8))
    u = torch.zeros((m.n_nodes, 3), dtype=torch.float64, device="cuda") if u0 is None else u0.clone()
    rc, st = op.newton_solve(u, dev(ubc), n_steps=n_steps, **kw)
    assert rc == 0, st
    return u


def test_cfg4_gradient_after_equilibrium_64cube():
    """64^3 Kuhn tets, mu ~ lognormal(0, 0.3) (seed 4), lam = 1.5, 5% top stretch.
    At equilibrium the free residual vanishes and the Dirichlet data do not
    depend on (mu, X), so dPsi(u*(theta), theta)/dtheta is the partial
    derivative the adjoint kernels return.  Checked by central differences with
    a re-solve (h = 1e-6) on 20 random mu entries and 20 random coordinates."""
    from paper_2602_12365_amd import Operator, energy
    n = 64
    m = I.tet_mesh(n)
    mu_h = I.lognormal_field(m.n_elems, 0.3, 4)
    op = Operator(I.TET4, m.X, m.conn)
    print("\n[cfg4] equilibrium solve 64^3", flush=True)
    ustar = solve_equilibrium(op, m, mu_h, 0.05, 5)
    mu = dev(mu_h).requires_grad_()
    lam = dev(1.5 * np.ones(m.n_elems))
    X = op.X.clone().requires_grad_()
    psi = energy(op, ustar, mu, lam, X)
    psi.backward()
    gmu, gX = mu.grad.cpu().numpy(), X.grad.cpu().numpy()
    psi0 = psi.item()
    rng = np.random.default_rng(5)
    h = 1e-6
    # One element's share of Psi is ~1e-6 of it, so with h = 1e-6 the energy
    # difference is ~1e-12 Psi and the FP64 rounding of Psi (a few eps |Psi|)
    # bounds the difference quotient's accuracy: |err| <= 8 eps |Psi| / h.
    # A second check with h = 1e-3 (error O(h^2), tiny here) pins it tightly.
    noise = 8 * np.finfo(np.float64).eps * abs(psi0) / h
    # material entries: re-solve from u* at mu +- h e_k
    for k in rng.choice(m.n_elems, 20, replace=False):
        fds = []
        for hh in (h, 1e-3):
            vals = []
            for s in (+1, -1):
                mu_p = mu_h.copy()
                mu_p[k] += s * hh
                u = solve_equilibrium(op, m, mu_p, 0.05, 1, u0=ustar)
                op.set_material(dev(mu_p), lam)
                vals.append(op.energy(u).item())
            fds.append((vals[0] - vals[1]) / (2 * hh))
        assert abs(fds[0] - gmu[k]) <= noise + 1e-6 * abs(gmu[k]), (k, fds[0], gmu[k])
        assert abs(fds[1] - gmu[k]) <= 1e-6 * abs(gmu[k]), (k, fds[1], gmu[k])
    op.set_material(dev(mu_h), lam)
    # coordinates of interior nodes: re-solve at X +- h e
    interior = np.nonzero(np.all((m.X > 0) & (m.X < 1), axis=1))[0]
    for idx in rng.choice(interior.size * 3, 20, replace=False):
        a, c = interior[idx // 3], idx % 3
        vals = []
        for s in (+1, -1):
            Xp = m.X.copy()
            Xp[a, c] += s * h
            op.set_coords(dev(Xp))
            u = solve_equilibrium(op, m, mu_h, 0.05, 1, u0=ustar)
            vals.append(op.energy(u).item())
        op.set_coords(dev(m.X))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gX[a, c]) <= 1e-5 * np.abs(gX).max(), (a, c, fd, gX[a, c])


def test_cfg4_oracle_gradient_8cube():
    """The same pipeline on an 8^3 copy: gradients equal the oracle's at the
    GPU equilibrium, and the oracle's own Newton solution gives the same
    gradients to solver tolerance."""
    from paper_2602_12365_amd import Operator, energy
    m = I.tet_mesh(8)
    mu_h = I.lognormal_field(m.n_elems, 0.3, 4)
    op = Operator(I.TET4, m.X, m.conn)
    ustar = solve_equilibrium(op, m, mu_h, 0.05, 5)
    mu = dev(mu_h).requires_grad_()
    X = op.X.clone().requires_grad_()
    energy(op, ustar, mu, dev(1.5 * np.ones(m.n_elems)), X).backward()
    orc = F.FEM(I.TET4, m.X, m.conn, mu_h, 1.5 * np.ones(m.n_elems))
    us = ustar.cpu().numpy()
    assert rel(mu.grad.cpu().numpy(), orc.grad_material(us)[0]) <= 1e-10
    assert rel(X.grad.cpu().numpy(), orc.grad_coords(us)) <= 1e-10
    mask, ubc = I.clamp_top_bottom(m.X, 0.05)
    u_ref, _ = F.newton_solve(orc, mask, ubc, F.SolveOptions(n_steps=5))
    assert rel(mu.grad.cpu().numpy(), orc.grad_material(u_ref)[0]) <= 1e-6
