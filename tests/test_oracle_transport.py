"""Pins of the oracle's non-variational transport operator (virtual work,
Sec. 3.1, Eqs. 4-6; the weak form of the advection-diffusion example of Sec. 6.5 for three species).

Every closed form is checked through both oracle paths, the residual r(c) and
the assembled element matrices K c, so that a mistake in either is caught:
- constants are in the kernel when there is no reaction;
- for an affine field, sum_a r_a = int (b . grad c + k c) with b = omega x x;
- the diffusion part passes the patch test and c.Kc = D |g|^2 V;
- the advection part is skew-symmetric on interior nodes (exact Gauss rule
  on affine hexes; b is divergence-free);
- the reaction part's rows sum to int N_a.
"""
import numpy as np
import pytest

from oracle import transport as T
from paper_2602_12365_amd import inputs as I

ELEMS = [I.TET4, I.HEX8]
OMEGA = np.array([0.3, -0.5, 1.1])


def make(elem, n, D=1.0, k=0.0, omega=OMEGA, sigma=0.0):
    m = I.make_mesh(elem, n)
    Dv = D * (np.ones(m.n_elems) if sigma == 0 else I.lognormal_field(m.n_elems, sigma, 8))
    return m, T.Transport(elem, m.X, m.conn, Dv, k * np.ones(m.n_elems), omega)


def both(t, c):
    """r(c) by the residual path and by the assembled matrix."""
    return t.residual(c), (t.tangent_matrix() @ np.asarray(c).reshape(-1)).reshape(-1, 3)


@pytest.mark.parametrize("elem", ELEMS)
def test_paths_agree(elem):
    m, t = make(elem, 3, k=0.7, sigma=0.4)
    c = I.gaussian_field(m.n_nodes, 1.0, 3)
    r1, r2 = both(t, c)
    assert np.abs(r1 - r2).max() <= 1e-14 * np.abs(r1).max()


@pytest.mark.parametrize("elem", ELEMS)
def test_constants_in_kernel_without_reaction(elem):
    m, t = make(elem, 3, k=0.0, sigma=0.4)
    c = np.tile([1.5, -2.0, 0.25], (m.n_nodes, 1))
    for r in both(t, c):
        assert np.abs(r).max() <= 1e-14


@pytest.mark.parametrize("elem", ELEMS)
def test_affine_field_total(elem):
    """sum_a r_{a,s} = int b . g_s + k c_s over the unit cube (both integrands
    are linear in x, which either rule integrates exactly)."""
    k = 0.6
    m, t = make(elem, 3, D=1.3, k=k)
    G = np.array([[0.4, -1.0, 0.3], [2.0, 0.1, -0.7], [-0.2, 0.5, 1.5]])   # row s: grad c_s
    c0 = np.array([0.1, -0.3, 0.8])
    c = m.X @ G.T + c0
    xbar = np.array([0.5, 0.5, 0.5])
    ref = G @ np.cross(OMEGA, xbar) + k * (G @ xbar + c0)
    for r in both(t, c):
        assert np.abs(r.sum(axis=0) - ref).max() <= 1e-13


@pytest.mark.parametrize("elem", ELEMS)
def test_diffusion_patch_test_and_energy(elem):
    """omega = 0, k = 0: an affine field leaves no force on interior nodes,
    and c.Kc = D sum_s |g_s|^2 V."""
    D = 1.7
    m, t = make(elem, 3, D=D, omega=np.zeros(3))
    G = np.array([[0.4, -1.0, 0.3], [2.0, 0.1, -0.7], [-0.2, 0.5, 1.5]])
    c = m.X @ G.T
    inner = np.all((m.X > 1e-12) & (m.X < 1 - 1e-12), axis=1)
    for r in both(t, c):
        assert np.abs(r[inner]).max() <= 1e-14 * np.abs(r).max()
        assert abs(np.sum(c * r) - D * np.sum(G * G)) <= 1e-13 * D * np.sum(G * G)


def test_advection_skew_on_interior_nodes():
    """D = k = 0 on affine hexes (Gauss exact): K + K^T = boundary flux term,
    zero wherever an interior node is involved."""
    m, t = make(I.HEX8, 3, D=0.0)
    K = t.tangent_matrix().toarray()
    S = K + K.T
    inner = np.repeat(np.all((m.X > 1e-12) & (m.X < 1 - 1e-12), axis=1), 3)
    assert np.abs(S[inner]).max() <= 1e-15 * np.abs(K).max()
    assert np.abs(K - K.T).max() > 1e-3 * np.abs(K).max()   # genuinely non-symmetric


@pytest.mark.parametrize("elem", ELEMS)
def test_reaction_rows_sum_to_shape_integrals(elem):
    """D = 0, omega = 0, k = 1: K 1 = int N_a.  A hex node gets h^3/8 from
    each hex around it, a tet node (volume h^3/6) h^3/24 from each tet."""
    n = 3
    m, t = make(elem, n, D=0.0, k=1.0, omega=np.zeros(3))
    h = 1.0 / n
    count = np.bincount(m.conn.reshape(-1), minlength=m.n_nodes)
    ref = (h ** 3) * count / (8.0 if elem == I.HEX8 else 24.0)
    for r in both(t, np.ones((m.n_nodes, 3))):
        assert np.abs(r - ref[:, None]).max() <= 1e-15


def test_direct_solve_meets_the_equations():
    m, t = make(I.TET4, 4, D=0.8, k=2.0, sigma=0.3)
    mask = np.zeros((m.n_nodes, 3), dtype=np.uint8)
    mask[m.X[:, 0] < 1e-12] = 1
    b = I.gaussian_field(m.n_nodes, 1.0, 9)
    x = t.solve_reduced(mask, b)
    r = t.residual(x)
    free = mask == 0
    assert np.abs(r[free] - b[free]).max() <= 1e-12 * np.abs(b).max()
    assert np.all(x[mask == 1] == 0)
