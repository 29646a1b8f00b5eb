"""Pins of the oracle's assembled tangent matrix K(u) (the matrix form of
Eq. 3), which checks the colouring-based sparse assembly.  Each pin is fixed
by something other than the assembly itself: the oracle's matrix-free tangent
action, symmetry of a second derivative, the textbook small-strain stiffness
B^T D B at u = 0, rigid-body modes, and finite differences of the residual."""
import numpy as np
import pytest

from oracle import fem as F
from paper_2602_12365_amd import inputs as I
from tests import pins


def case(elem, n, amp=0.02, seed=0):
    m = I.make_mesh(elem, n)
    mu = I.lognormal_field(m.n_elems, 0.3, 1)
    orc = F.FEM(elem, m.X, m.conn, mu, 1.5 * mu)
    u = I.gaussian_field(m.n_nodes, amp / n, seed)
    return m, orc, u


@pytest.mark.parametrize("elem", [I.TET4, I.HEX8])
def test_tangent_matrix_times_v_is_the_tangent_action(elem):
    m, orc, u = case(elem, 3)
    K = orc.tangent_matrix(u)
    v = I.unit_direction(m.n_nodes, 4)
    y = orc.hvp(u, v).reshape(-1)
    assert np.abs(K @ v.reshape(-1) - y).max() <= 1e-13 * np.abs(y).max()


@pytest.mark.parametrize("elem", [I.TET4, I.HEX8])
def test_tangent_matrix_symmetric_and_pattern_is_the_node_ring(elem):
    m, orc, u = case(elem, 3)
    K = orc.tangent_matrix(u)
    d = (K - K.T).tocoo()
    assert np.abs(d.data).max() <= 1e-14 * np.abs(K.data).max()
    # every nonzero couples two nodes of one element, in full 3x3 blocks
    adj = set()
    for ce in m.conn:
        for a in ce:
            for b in ce:
                adj.add((int(a), int(b)))
    Kc = K.tocoo()
    assert all((r // 3, c // 3) in adj for r, c in zip(Kc.row, Kc.col))
    assert K.nnz == 9 * len(adj)


@pytest.mark.parametrize("elem", [I.TET4, I.HEX8])
def test_tangent_matrix_at_zero_is_the_textbook_stiffness(elem):
    m, orc, _ = case(elem, 2)
    K = orc.tangent_matrix(np.zeros((m.n_nodes, 3))).toarray()
    Klin = pins.linear_stiffness(elem, m.X, m.conn, orc.mu, orc.lam)
    assert np.abs(K - Klin).max() <= 1e-12 * np.abs(Klin).max()


@pytest.mark.parametrize("elem", [I.TET4, I.HEX8])
def test_tangent_matrix_rigid_modes_and_residual_fd(elem):
    m, orc, u = case(elem, 3)
    K = orc.tangent_matrix(u)
    n = m.n_nodes
    for c in range(3):                      # translations: K t = 0 at any u
        t = np.zeros((n, 3))
        t[:, c] = 1.0
        assert np.abs(K @ t.reshape(-1)).max() <= 1e-12 * np.abs(K.data).max()
    K0 = orc.tangent_matrix(np.zeros((n, 3)))
    W = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 0]], dtype=float)
    rot = (m.X - 0.5) @ W.T                  # infinitesimal rotation about z
    assert np.abs(K0 @ rot.reshape(-1)).max() <= 1e-12 * np.abs(K0.data).max()
    h = 1e-6
    rng = np.random.default_rng(5)
    for j in rng.choice(3 * n, 4, replace=False):
        e = np.zeros(3 * n)
        e[j] = h
        fd = (orc.residual(u + e.reshape(n, 3)) - orc.residual(u - e.reshape(n, 3))).reshape(-1) / (2 * h)
        col = K[:, j].toarray().ravel()
        assert np.abs(col - fd).max() <= 1e-7 * np.abs(col).max()


@pytest.mark.parametrize("elem", [I.TET4, I.HEX8])
@pytest.mark.parametrize("model", ["neo_hookean", "linear"])
def test_jacobi_blocks_by_central_differences(elem, model):
    """Every node's 3x3 diagonal block of K (jacobi_diag and jacobi_offdiag),
    against central differences of the residual at that node with respect to
    that node's own displacement: no assembled matrix involved."""
    m = I.make_mesh(elem, 2)
    mu = I.lognormal_field(m.n_elems, 0.3, 1)
    orc = F.FEM(elem, m.X, m.conn, mu, 1.5 * mu, model)
    u = I.gaussian_field(m.n_nodes, 0.01, 0)
    d, off = orc.jacobi_diag(u), orc.jacobi_offdiag(u)
    h = 1e-6
    for a in range(m.n_nodes):
        B = np.empty((3, 3))
        for j in range(3):
            up, um = u.copy(), u.copy()
            up[a, j] += h
            um[a, j] -= h
            B[:, j] = (orc.residual(up)[a] - orc.residual(um)[a]) / (2 * h)
        scale = np.abs(B).max()
        assert np.abs(np.diag(B) - d[a]).max() <= 1e-7 * scale
        assert np.abs(np.array([B[0, 1], B[0, 2], B[1, 2]]) - off[a]).max() <= 1e-7 * scale
        assert np.abs(B - B.T).max() <= 1e-7 * scale
