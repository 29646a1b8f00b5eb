"""GPU Newton solves with an external load (the total potential energy of
Sec. 6.1, Psi_h(u) - s f.u) against the oracle's solve, the homogeneous
patch-test solution and Kirsch's plate-with-hole solution."""
import numpy as np
import pytest
import torch

from oracle import fem as F
from paper_2602_12365_amd import inputs as I
from tests import loads as LD
from tests.test_oracle_load import LAM, MU, T, exact_homogeneous

pytestmark = pytest.mark.gpu

R, W, SIGMA = 0.05, 0.5, 0.01


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype=dtype)


def make_op(m, model, mu, lam, mask, f):
    from paper_2602_12365_amd import Operator
    op = Operator(m.elem, m.X, m.conn, model=model)
    op.set_material(dev(mu), dev(lam))
    op.set_dirichlet(dev(mask, torch.uint8))
    if f is not None:
        op.set_load(dev(f))
    return op


def total_free_residual(orc, u, mask, f):
    return np.linalg.norm(F.masked(mask, orc.residual(u) - f))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("model", ["neo_hookean", "linear"])
@pytest.mark.parametrize("elem", [I.TRI3, I.TET4, I.HEX8])
def test_loaded_patch_solve_matches_oracle_and_closed_form(elem, model, prec):
    """Uniform dead traction on x = 1 of a jittered, shuffled mesh with
    symmetry conditions: the GPU solve against the oracle's solve (same load
    steps) and against the exact homogeneous deformation."""
    print(f"\n[load] patch elem={elem} model={model} prec={prec}", flush=True)
    n = 12 if elem == I.TRI3 else 5
    m = I.scrambled_mesh(I.make_mesh(elem, n), 21, jitter=0.25)
    mu, lam = np.full(m.n_elems, MU), np.full(m.n_elems, LAM)
    mask = I.symmetry_mask(m.X, planar=(elem == I.TRI3))
    f = LD.face_load(m, 0, 1.0, [T, 0.0, 0.0])
    op = make_op(m, model, mu, lam, mask, f)
    u = torch.zeros((m.n_nodes, 3), dtype=torch.float64, device="cuda")
    rc, st = op.newton_solve(u, dev(np.zeros_like(m.X)), n_steps=2, hvp_prec=prec, rtol=1e-10)
    assert rc == 0 and st["converged"] == 1, st
    orc = F.FEM(elem, m.X, m.conn, mu, lam, model)
    u_ref, st_ref = F.newton_solve(orc, mask, np.zeros_like(m.X),
                                   F.SolveOptions(n_steps=2, rtol=1e-10), f_ext=f)
    ug = u.cpu().numpy()
    ue = exact_homogeneous(m, model, elem == I.TRI3)
    assert np.max(np.abs(ug - u_ref)) <= 1e-8 * np.max(np.abs(ue))
    assert np.max(np.abs(ug - ue)) <= 1e-8 * np.max(np.abs(ue))
    assert total_free_residual(orc, ug, mask, f) <= 1e-9 * np.linalg.norm(F.masked(mask, f))
    # the reported energy is the total potential energy at the final load
    e_tot = orc.energy(ug) - np.sum(f * ug)
    assert st["final_energy"] == pytest.approx(e_tot, rel=1e-10, abs=1e-15)
    assert st["final_energy"] == pytest.approx(st_ref.energy_history[-1][-1], rel=1e-8)


def kirsch_case(n_t):
    n_r = 3 * n_t
    m = I.plate_with_hole_mesh(n_r, n_t, R, W)
    mu, lam = np.full(m.n_elems, MU), np.full(m.n_elems, LAM)
    mask = I.symmetry_mask(m.X, planar=True)
    f = LD.kirsch_outer_load(m, n_r, R, W, SIGMA)
    return m, mu, lam, mask, f


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_kirsch_plate_matches_oracle(prec):
    """The plate with a hole (n_t = 16, 1,617 nodes) under Kirsch's
    tractions: GPU against the oracle, node by node."""
    print(f"\n[load] kirsch parity prec={prec}", flush=True)
    m, mu, lam, mask, f = kirsch_case(16)
    op = make_op(m, "linear", mu, lam, mask, f)
    u = torch.zeros((m.n_nodes, 3), dtype=torch.float64, device="cuda")
    rc, st = op.newton_solve(u, dev(np.zeros_like(m.X)), n_steps=1, hvp_prec=prec, rtol=1e-10)
    assert rc == 0 and st["converged"] == 1, st
    orc = F.FEM(I.TRI3, m.X, m.conn, mu, lam, "linear")
    u_ref, _ = F.newton_solve(orc, mask, np.zeros_like(m.X), F.SolveOptions(n_steps=1, rtol=1e-10),
                              f_ext=f)
    ug = u.cpu().numpy()
    assert np.max(np.abs(ug - u_ref)) <= 1e-8 * np.max(np.abs(u_ref))
    assert np.all(ug[:, 2] == 0.0)


def test_kirsch_plate_converges_on_the_gpu():
    """Refinements n_t = 32, 64, 128 (up to 98,945 nodes): the element
    stresses approach Kirsch's at first order, and the hoop stress at the
    top of the hole approaches 3 sigma."""
    errs, peaks = [], []
    for n_t in (32, 64, 128):
        print(f"\n[load] kirsch n_t={n_t}", flush=True)
        m, mu, lam, mask, f = kirsch_case(n_t)
        op = make_op(m, "linear", mu, lam, mask, f)
        u = torch.zeros((m.n_nodes, 3), dtype=torch.float64, device="cuda")
        rc, st = op.newton_solve(u, dev(np.zeros_like(m.X)), n_steps=1, rtol=1e-10)
        assert rc == 0 and st["converged"] == 1, st
        err, (sxx, _, _), cen = LD.kirsch_error(m, u.cpu().numpy(), MU, LAM, R, SIGMA)
        errs.append(err)
        k = np.argmax(sxx)
        kxx = LD.kirsch_stress(cen[k, 0], cen[k, 1], R, SIGMA)[0]
        peaks.append((sxx[k], kxx, cen[k]))
        print(f"[load] kirsch n_t={n_t}: {m.n_nodes} nodes, {st['cg_iters']} CG, {st['seconds']:.3f} s, "
              f"stress L2 error {err:.3e}, peak sxx/sigma {sxx[k] / SIGMA:.4f} "
              f"(Kirsch at the centroid {kxx / SIGMA:.4f})", flush=True)
    assert errs[0] / errs[1] > 1.7 and errs[1] / errs[2] > 1.7, errs
    assert errs[2] < 1e-3, errs
    s_fe, s_k, c = peaks[-1]
    assert np.hypot(*c) < 1.1 * R and c[1] > 0.95 * np.hypot(*c)   # at the top of the hole
    assert abs(s_fe - s_k) <= 0.02 * s_k and s_fe > 2.8 * SIGMA, peaks


def test_removing_the_load():
    m = I.make_mesh(I.TET4, 3)
    mu, lam = np.full(m.n_elems, MU), np.full(m.n_elems, LAM)
    mask = I.symmetry_mask(m.X, planar=False)
    op = make_op(m, "neo_hookean", mu, lam, mask, LD.face_load(m, 0, 1.0, [T, 0, 0]))
    op.set_load(None)
    u = torch.zeros((m.n_nodes, 3), dtype=torch.float64, device="cuda")
    rc, st = op.newton_solve(u, dev(np.zeros_like(m.X)), n_steps=1)
    assert rc == 0
    assert torch.count_nonzero(u).item() == 0
