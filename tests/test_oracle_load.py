"""Pins of the oracle's loaded Newton solve: the total potential energy of
Sec. 6.1, Psi_h(u) - s f.u with the traction's nodal forces f.

* Patch tests: a uniform dead traction on the face x = 1 of a jittered mesh,
  symmetry conditions on the coordinate planes.  The exact solution is a
  homogeneous deformation, which every element type reproduces exactly, so
  the solve must return it to solver precision: small-strain principal
  strains from Young's modulus and Poisson's ratio, and neo-Hookean
  stretches from the principal-stretch form of the energy.
* Along the load steps of the linear model, u_k = s_k u* and the total
  energy at the end of step k is -s_k^2 f.u*/2.
* At equilibrium of the linear model, Psi_h(u*) = f.u*/2 (Clapeyron).
* The plate with a hole of Sec. 6.1 under Kirsch's tractions converges to
  Kirsch's stresses at first order in the mesh size.
"""
import numpy as np
import pytest

from oracle import fem as F
from paper_2602_12365_amd import inputs as I
from tests import loads as LD

MU, LAM, T = 1.0, 1.5, 0.05


def patch_case(elem, model, n, seed=11):
    m = I.scrambled_mesh(I.make_mesh(elem, n), seed, jitter=0.25)
    mu = np.full(m.n_elems, MU)
    lam = np.full(m.n_elems, LAM)
    orc = F.FEM(elem, m.X, m.conn, mu, lam, model)
    mask = I.symmetry_mask(m.X, planar=(elem == I.TRI3))
    f = LD.face_load(m, 0, 1.0, [T, 0.0, 0.0])
    return m, orc, mask, f


def exact_homogeneous(m, model, planar):
    if model == "linear":
        e = np.array(LD.uniaxial_linear(MU, LAM, T, planar))
    else:
        e = np.array(LD.uniaxial_neo_hooke(MU, LAM, T, planar)) - 1.0
    return m.X * e[None, :]


@pytest.mark.parametrize("model", ["neo_hookean", "linear"])
@pytest.mark.parametrize("elem", [I.TRI3, I.TET4, I.HEX8])
def test_patch_test_uniaxial_dead_load(elem, model):
    m, orc, mask, f = patch_case(elem, model, 4 if elem == I.TRI3 else 3)
    u, st = F.newton_solve(orc, mask, np.zeros_like(m.X), F.SolveOptions(n_steps=2, rtol=1e-12),
                           f_ext=f)
    assert st.converged
    ue = exact_homogeneous(m, model, elem == I.TRI3)
    assert np.max(np.abs(u - ue)) <= 1e-10 * np.max(np.abs(ue))


def test_load_steps_scale_the_linear_solution():
    m, orc, mask, f = patch_case(I.TET4, "linear", 3)
    n = 4
    u, st = F.newton_solve(orc, mask, np.zeros_like(m.X), F.SolveOptions(n_steps=n, rtol=1e-12),
                           f_ext=f)
    fu = np.sum(f * u)
    for k in range(1, n + 1):
        e_end = st.energy_history[k - 1][-1]
        assert e_end == pytest.approx(-0.5 * (k / n) ** 2 * fu, rel=1e-9)


def test_clapeyron_on_the_plate():
    R, W = 0.05, 0.5
    m = I.plate_with_hole_mesh(12, 4, R, W)
    mu = np.full(m.n_elems, MU)
    orc = F.FEM(I.TRI3, m.X, m.conn, mu, LAM * mu / MU, "linear")
    f = LD.kirsch_outer_load(m, 12, R, W, 0.01)
    mask = I.symmetry_mask(m.X, planar=True)
    u, st = F.newton_solve(orc, mask, np.zeros_like(m.X), F.SolveOptions(n_steps=1, rtol=1e-12),
                           f_ext=f)
    assert st.converged
    assert orc.energy(u) == pytest.approx(0.5 * np.sum(f * u), rel=1e-9)


def kirsch_solve(n_t, R=0.05, W=0.5, sigma=0.01):
    n_r = 3 * n_t
    m = I.plate_with_hole_mesh(n_r, n_t, R, W)
    mu = np.full(m.n_elems, MU)
    lam = np.full(m.n_elems, LAM)
    orc = F.FEM(I.TRI3, m.X, m.conn, mu, lam, "linear")
    f = LD.kirsch_outer_load(m, n_r, R, W, sigma)
    mask = I.symmetry_mask(m.X, planar=True)
    u, st = F.newton_solve(orc, mask, np.zeros_like(m.X), F.SolveOptions(n_steps=1, rtol=1e-10),
                           f_ext=f)
    assert st.converged
    return m, u


def test_kirsch_plate_converges_to_the_closed_form():
    errs = []
    for n_t in (4, 8, 16):
        m, u = kirsch_solve(n_t)
        err, _, _ = LD.kirsch_error(m, u, MU, LAM, 0.05, 0.01)
        errs.append(err)
    # first order in h for constant-strain triangles
    assert errs[0] / errs[1] > 1.6 and errs[1] / errs[2] > 1.6, errs
    assert errs[2] < 0.01, errs
