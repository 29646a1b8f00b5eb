"""Full-size parity with per-element material fields (Eqs. 1-3 and their
material and coordinate derivatives), every output entry against the oracle.

* 64^3 Kuhn mesh (1,572,864 Tet4): shear modulus lognormal(0, 0.3) seed 4 and
  lam = 1.5 (the adjoint configuration); energy, residual, FP64 and FP32
  tangent actions, Jacobi diagonal, dPsi/dmu, dPsi/dlam, dPsi/dX and the
  material VJP of the residual.
* 128^3 trilinear hexahedra (2,097,152 Hex8, 2x2x2 Gauss): mu lognormal(0,
  0.5) seed 3 and lam = 1.5 mu (the compression configuration); energy,
  residual, FP64 and FP32 tangent actions and the Jacobi diagonal.

Tolerances as in the small-mesh parity suite: energy 1e-12 relative, FP64
nodal and per-element outputs 1e-10 of the largest entry, the FP32 tangent
action 5e-5.
"""
import numpy as np
import pytest
import torch

from oracle import fem as F
from paper_2602_12365_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL_E, TOL64, TOL32 = 1e-12, 1e-10, 5e-5


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def tet64():
    from paper_2602_12365_amd import Operator
    n = 64
    print(f"\n[full-size] tet n={n}, mu lognormal(0, 0.3) seed 4, lam 1.5", flush=True)
    m = I.tet_mesh(n)
    mu = I.lognormal_field(m.n_elems, 0.3, 4)
    lam = 1.5 * np.ones(m.n_elems)
    op = Operator(I.TET4, m.X, m.conn)
    op.set_material(dev(mu), dev(lam))
    u = I.gaussian_field(m.n_nodes, I.cube_amplitude(n), 0)
    yield m, op, F.FEM(I.TET4, m.X, m.conn, mu, lam), u
    op.close()


@pytest.fixture(scope="module")
def hex128():
    from paper_2602_12365_amd import Operator
    n = 128
    print(f"\n[full-size] hex n={n}, mu lognormal(0, 0.5) seed 3, lam 1.5 mu", flush=True)
    m = I.hex_mesh(n)
    mu = I.lognormal_field(m.n_elems, 0.5, 3)
    lam = 1.5 * mu
    op = Operator(I.HEX8, m.X, m.conn)
    op.set_material(dev(mu), dev(lam))
    u = I.gaussian_field(m.n_nodes, I.cube_amplitude(n), 0)
    yield m, op, F.FEM(I.HEX8, m.X, m.conn, mu, lam), u
    op.close()


def test_tet64_energy_residual(tet64):
    m, op, orc, u = tet64
    e = host(op.energy(dev(u)))
    ref = orc.energy(u)
    assert abs(e - ref) <= TOL_E * abs(ref)
    assert rel(host(op.residual(dev(u))), orc.residual(u)) <= TOL64


def test_tet64_tangent_actions(tet64):
    m, op, orc, u = tet64
    v = I.unit_direction(m.n_nodes, 100)
    ref = orc.hvp(u, v)
    op.linearize(dev(u), "f64")
    assert rel(host(op.hvp(dev(v))), ref) <= TOL64
    op.linearize(dev(u), "f32")
    assert rel(host(op.hvp(dev(v, torch.float32))), ref) <= TOL32
    assert rel(host(op.jacobi_diag(dev(u))), orc.jacobi_diag(u)) <= TOL64


def test_tet64_adjoints(tet64):
    m, op, orc, u = tet64
    gm, gl = op.grad_material(dev(u))
    rm, rl = orc.grad_material(u)
    assert rel(host(gm), rm) <= TOL64
    assert rel(host(gl), rl) <= TOL64
    assert rel(host(op.grad_coords(dev(u))), orc.grad_coords(u)) <= TOL64
    w = I.unit_direction(m.n_nodes, 2)
    vm, vl = op.residual_vjp_material(dev(u), dev(w))
    rvm, rvl = orc.residual_vjp_material(u, w)
    assert rel(host(vm), rvm) <= TOL64
    assert rel(host(vl), rvl) <= TOL64


def test_hex128_energy_residual(hex128):
    m, op, orc, u = hex128
    e = host(op.energy(dev(u)))
    ref = orc.energy(u)
    assert abs(e - ref) <= TOL_E * abs(ref)
    assert rel(host(op.residual(dev(u))), orc.residual(u)) <= TOL64


def test_hex128_tangent_actions_and_diagonal(hex128):
    m, op, orc, u = hex128
    v = I.unit_direction(m.n_nodes, 100)
    ref = orc.hvp(u, v)
    op.linearize(dev(u), "f64")
    assert rel(host(op.hvp(dev(v))), ref) <= TOL64
    op.linearize(dev(u), "f32")
    assert rel(host(op.hvp(dev(v, torch.float32))), ref) <= TOL32
    assert rel(host(op.jacobi_diag(dev(u))), orc.jacobi_diag(u)) <= TOL64
