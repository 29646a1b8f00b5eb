"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one oracle operator to something other than the oracle itself:
closed forms, invariants, a textbook routine, or brute-force finite
differences, chosen so that a dropped term, a wrong sign or index, or a
transposed operand in any operator fails at least one of them.
"""
import numpy as np
import pytest

from oracle import fem as F
from paper_2602_12365_amd import inputs as I
from tests import pins

ELEMS = [I.TET4, I.HEX8]
ALL_ELEMS = [I.TET4, I.HEX8, I.TRI3]   # for pins that hold in any kinematics


MODELS = ["neo_hookean", "linear"]


def make(elem, n, mu_sigma=0.0, seed=3, lam_ratio=None, model="neo_hookean"):
    m = I.make_mesh(elem, n)
    mu = np.ones(m.n_elems) if mu_sigma == 0 else I.lognormal_field(m.n_elems, mu_sigma, seed)
    lam = 1.5 * np.ones(m.n_elems) if lam_ratio is None else lam_ratio * mu
    return m, F.FEM(elem, m.X, m.conn, mu, lam, model)


def affine(X, F0):
    return X @ (F0 - np.eye(3)).T


F0_CASES = [
    np.array([[1.10, 0.05, -0.02], [0.03, 0.95, 0.04], [-0.01, 0.02, 1.05]]),
    np.array([[0.80, 0.30, 0.00], [0.00, 1.20, 0.10], [0.10, 0.00, 0.90]]),
]


# ------------------------------------------------------------------- mesh

@pytest.mark.parametrize("elem", ELEMS)
def test_mesh_volume_and_orientation(elem):
    m, f = make(elem, 4)
    vol, rc = f.volumes()
    assert rc == 0 and np.all(vol > 0)
    assert abs(vol.sum() - 1.0) < 1e-13
    # independent volume: textbook gradients' weights
    v2 = sum(w for ce in m.conn for _, w in pins.element_points(elem, m.X[ce]))
    assert abs(v2 - 1.0) < 1e-13


def test_tet_split_conforming():
    m = I.tet_mesh(3)
    faces = {}
    for ce in m.conn:
        for f in [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]:
            key = tuple(sorted(int(ce[i]) for i in f))
            faces[key] = faces.get(key, 0) + 1
    assert max(faces.values()) == 2
    bnd = [k for k, c in faces.items() if c == 1]
    # every boundary face lies on the cube surface; 6 faces x 3^2 squares x 2 triangles
    assert len(bnd) == 6 * 9 * 2
    for k in bnd:
        P = m.X[list(k)]
        assert any(np.all(np.abs(P[:, ax] - P[0, ax]) < 1e-14) and P[0, ax] in (0.0, 1.0)
                   for ax in range(3))


def test_config_sizes():
    # the sizes the configurations are quoted on
    m = I.tet_mesh(8)
    assert (m.n_elems, m.n_nodes, m.n_dofs) == (3072, 729, 2187)
    m = I.tet_mesh(64)
    assert (m.n_elems, m.n_nodes) == (1572864, 274625)
    m = I.hex_mesh(32)
    assert (m.n_elems, m.n_nodes) == (32768, 35937)


# ----------------------------------------------------------------- energy

@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("ci", range(len(F0_CASES)))
def test_energy_affine_principal_stretches(elem, ci):
    """Affine u = (F0 - I) X: F = F0 everywhere, so Psi = psi(F0) * |unit cube|."""
    F0 = F0_CASES[ci]
    m, f = make(elem, 3)
    psi = f.energy(affine(m.X, F0))
    ref = pins.psi_principal(F0, 1.0, 1.5)
    assert abs(psi - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("elem", ELEMS)
def test_energy_heterogeneous_affine(elem):
    """Per-element material: Psi = sum_e V_e psi_e(F0)."""
    F0 = F0_CASES[0]
    m, f = make(elem, 3, mu_sigma=0.5, lam_ratio=1.5)
    vol, _ = f.volumes()
    ref = sum(v * pins.psi_principal(F0, a, b) for v, a, b in zip(vol, f.mu, f.lam))
    assert abs(f.energy(affine(m.X, F0)) - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("elem", ELEMS)
def test_rigid_rotation_zero_energy_and_residual(elem):
    R = I.random_rotation(11)
    m, f = make(elem, 3)
    u = affine(m.X, R)
    assert abs(f.energy(u)) < 1e-14
    assert np.abs(f.residual(u)).max() < 1e-14


def test_small_strain_limit_matches_linear_elastic_density():
    """psi(I + eps G) / eps^2 -> the linear-elastic density of Sec. 6.1."""
    g = np.random.default_rng(5).standard_normal((3, 3))
    m, f = make(I.TET4, 1)
    for eps in (1e-3, 1e-4):
        psi = f.energy(affine(m.X, np.eye(3) + eps * g))
        lin = pins.psi_linear(g, 1.0, 1.5)
        assert abs(psi / eps**2 - lin) <= 30 * eps * abs(lin)


def test_inverted_element_gives_inf():
    m, f = make(I.TET4, 2)
    u = np.zeros_like(m.X)
    u[m.conn[0, 3]] = -3.0 * (m.X[m.conn[0, 3]] - m.X[m.conn[0, 0]])
    assert f.energy(u, allow_inverted=True) == np.inf
    with pytest.raises(F.OracleError):
        f.residual(u)


# --------------------------------------------------------------- residual

@pytest.mark.parametrize("elem", ALL_ELEMS)
@pytest.mark.parametrize("model", MODELS)
def test_residual_fd_of_energy(elem, model):
    m, f = make(elem, 3, mu_sigma=0.3, model=model)
    u = I.gaussian_field(m.n_nodes, 0.02, 0)
    r = f.residual(u)
    for s in range(3):
        w = I.unit_direction(m.n_nodes, 20 + s)
        h = 1e-6
        fd = (f.energy(u + h * w) - f.energy(u - h * w)) / (2 * h)
        assert abs(r.ravel() @ w.ravel() - fd) <= 1e-7 * np.linalg.norm(r)


@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("ci", range(len(F0_CASES)))
def test_patch_test(elem, ci):
    """Affine u: zero interior residual; boundary residual = consistent nodal
    loads of the traction P(F0) n with P from finite differences of the
    principal-stretch energy; total force zero."""
    F0 = F0_CASES[ci]
    m, f = make(elem, 3)
    r = f.residual(affine(m.X, F0))
    P = pins.piola_fd(F0, 1.0, 1.5)
    ref = pins.consistent_traction_loads(m.X, pins.boundary_faces(elem, m.conn), P)
    scale = np.abs(ref).max()
    assert np.abs(r - ref).max() <= 1e-8 * scale   # FD stress accuracy
    interior = np.all((m.X > 1e-12) & (m.X < 1 - 1e-12), axis=1)
    assert interior.any()
    assert np.abs(r[interior]).max() <= 1e-14 * scale * 10
    assert np.abs(r.sum(axis=0)).max() <= 1e-14 * scale * 10


@pytest.mark.parametrize("elem", ELEMS)
def test_residual_objectivity(elem):
    """Rotating the deformed configuration rotates the residual: r(R phi) = R r(phi)."""
    m, f = make(elem, 3)
    u = I.gaussian_field(m.n_nodes, 0.03, 2)
    R = I.random_rotation(4)
    uR = (m.X + u) @ R.T - m.X
    assert np.abs(f.residual(uR) - f.residual(u) @ R.T).max() <= 1e-13 * np.abs(f.residual(u)).max()
    assert abs(f.energy(uR) - f.energy(u)) <= 1e-13 * abs(f.energy(u))


# ----------------------------------------------------------------- tangent

@pytest.mark.parametrize("elem", ALL_ELEMS)
@pytest.mark.parametrize("model", MODELS)
def test_hvp_fd_of_residual(elem, model):
    m, f = make(elem, 3, mu_sigma=0.3, model=model)
    u = I.gaussian_field(m.n_nodes, 0.02, 0)
    v = I.unit_direction(m.n_nodes, 1)
    h = 1e-6
    fd = (f.residual(u + h * v) - f.residual(u - h * v)) / (2 * h)
    Kv = f.hvp(u, v)
    assert np.linalg.norm(Kv - fd) <= 1e-8 * np.linalg.norm(Kv)


@pytest.mark.parametrize("elem", ALL_ELEMS)
@pytest.mark.parametrize("model", MODELS)
def test_hvp_symmetry(elem, model):
    m, f = make(elem, 3, mu_sigma=0.3, model=model)
    u = I.gaussian_field(m.n_nodes, 0.03, 0)
    v = I.unit_direction(m.n_nodes, 1)
    w = I.unit_direction(m.n_nodes, 2)
    a, b = w.ravel() @ f.hvp(u, v).ravel(), v.ravel() @ f.hvp(u, w).ravel()
    assert abs(a - b) <= 1e-13 * np.linalg.norm(f.hvp(u, v))


def dense_K(f, u):
    n = 3 * f.n_nodes
    K = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        K[:, j] = f.hvp(u, e).ravel()
    return K


@pytest.mark.parametrize("elem", ELEMS)
def test_reference_stiffness_equals_textbook_linear_elasticity(elem):
    """At u = 0 the tangent is the isotropic Hooke tensor: K(0) = sum B^T D B."""
    m, f = make(elem, 2, mu_sigma=0.4, lam_ratio=1.5)
    K = dense_K(f, np.zeros_like(m.X))
    Klin = pins.linear_stiffness(elem, m.X, m.conn, f.mu, f.lam)
    assert np.abs(K - Klin).max() <= 1e-13 * np.abs(Klin).max()


@pytest.mark.parametrize("elem", ELEMS)
def test_tangent_under_rigid_rotation(elem):
    """K(u_R) v = R K(0) R^T v blockwise for u_R = (R - I) X."""
    m, f = make(elem, 2)
    R = I.random_rotation(9)
    v = I.unit_direction(m.n_nodes, 3)
    lhs = f.hvp(affine(m.X, R), v)
    rhs = f.hvp(np.zeros_like(m.X), v @ R) @ R.T
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


@pytest.mark.parametrize("elem", ALL_ELEMS)
@pytest.mark.parametrize("model", MODELS)
def test_jacobi_diag_equals_diag_of_K(elem, model):
    m, f = make(elem, 2, mu_sigma=0.3, model=model)
    u = I.gaussian_field(m.n_nodes, 0.02, 7)
    d = f.jacobi_diag(u).ravel()
    assert np.abs(d - np.diag(dense_K(f, u))).max() <= 1e-13 * np.abs(d).max()


# ----------------------------------------------------------- adjoints

@pytest.mark.parametrize("elem", ALL_ELEMS)
@pytest.mark.parametrize("model", MODELS)
def test_grad_material_fd_and_homogeneity(elem, model):
    m, f = make(elem, 3, mu_sigma=0.3, lam_ratio=1.5, model=model)
    u = I.gaussian_field(m.n_nodes, 0.03, 0)
    gm, gl = f.grad_material(u)
    psi = f.energy(u)
    # Psi is linear in (mu, lam): Euler identity
    assert abs(gm @ f.mu + gl @ f.lam - psi) <= 1e-13 * abs(psi)
    rng = np.random.default_rng(1)
    for e in rng.choice(m.n_elems, 5, replace=False):
        for arr, g in ((f.mu, gm), (f.lam, gl)):
            old = arr[e]
            arr[e] = old + 1e-3
            ep = f.energy(u)
            arr[e] = old - 1e-3
            em = f.energy(u)
            arr[e] = old
            assert abs((ep - em) / 2e-3 - g[e]) <= 1e-9 * max(abs(g[e]), 1e-3 * abs(psi) / m.n_elems)


def test_grad_material_affine_closed_form():
    """Affine F0: dPsi/dmu_e = V_e psi|_{mu=1,lam=0}(F0), dPsi/dlam_e = V_e psi|_{mu=0,lam=1}(F0)."""
    F0 = F0_CASES[1]
    for elem in ELEMS:
        m, f = make(elem, 2)
        gm, gl = f.grad_material(affine(m.X, F0))
        vol, _ = f.volumes()
        assert np.abs(gm - vol * pins.psi_principal(F0, 1.0, 0.0)).max() <= 1e-14
        assert np.abs(gl - vol * pins.psi_principal(F0, 0.0, 1.0)).max() <= 1e-14


@pytest.mark.parametrize("elem", ALL_ELEMS)
@pytest.mark.parametrize("model", MODELS)
def test_residual_vjp_material(elem, model):
    m, f = make(elem, 3, mu_sigma=0.3, lam_ratio=1.5, model=model)
    u = I.gaussian_field(m.n_nodes, 0.03, 0)
    w = I.unit_direction(m.n_nodes, 5)
    gm, gl = f.residual_vjp_material(u, w)
    wr = w.ravel() @ f.residual(u).ravel()
    assert abs(gm @ f.mu + gl @ f.lam - wr) <= 1e-12 * np.abs(f.residual(u)).max()
    for e in np.random.default_rng(2).choice(m.n_elems, 5, replace=False):
        for arr, g in ((f.mu, gm), (f.lam, gl)):
            old = arr[e]
            arr[e] = old + 1e-3
            rp = w.ravel() @ f.residual(u).ravel()
            arr[e] = old - 1e-3
            rm = w.ravel() @ f.residual(u).ravel()
            arr[e] = old
            assert abs((rp - rm) / 2e-3 - g[e]) <= 1e-10


@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("model", MODELS)
def test_grad_coords_fd_and_invariants(elem, model):
    m, f = make(elem, 3, mu_sigma=0.3, lam_ratio=1.5, model=model)
    u = I.gaussian_field(m.n_nodes, 0.03, 0)
    g = f.grad_coords(u)
    r = f.residual(u)
    psi = f.energy(u)
    scale = np.abs(g).max()
    # translation invariance
    assert np.abs(g.sum(axis=0)).max() <= 1e-13 * scale * m.n_nodes
    # joint rotation of (X, u) leaves Psi unchanged
    mom = np.cross(m.X, g).sum(axis=0) + np.cross(u, r).sum(axis=0)
    assert np.abs(mom).max() <= 1e-13 * scale * m.n_nodes
    # joint scaling: Psi(sX, su) = s^3 Psi
    assert abs(np.sum(m.X * g) + np.sum(u * r) - 3 * psi) <= 1e-12 * abs(psi)
    # finite differences at fixed nodal u
    h = 1e-6
    for s in range(3):
        w = I.unit_direction(m.n_nodes, 40 + s)
        fp = F.FEM(elem, m.X + h * w, m.conn, f.mu, f.lam, model).energy(u)
        fm = F.FEM(elem, m.X - h * w, m.conn, f.mu, f.lam, model).energy(u)
        assert abs((fp - fm) / (2 * h) - np.sum(g * w)) <= 1e-7 * np.linalg.norm(g)


# ------------------------------------------------ small-strain linear model

@pytest.mark.parametrize("elem", ELEMS)
def test_linear_model_is_the_textbook_stiffness_at_any_state(elem):
    """Linear model: K is the Hooke-tensor B^T D B stiffness whatever u is,
    Psi(u) = u.K u / 2 and r(u) = K u exactly (a quadratic energy)."""
    m, f = make(elem, 2, mu_sigma=0.4, lam_ratio=1.5, model="linear")
    Klin = pins.linear_stiffness(elem, m.X, m.conn, f.mu, f.lam)
    u = I.gaussian_field(m.n_nodes, 0.3, 4)   # large: no smallness is assumed
    K = dense_K(f, u)
    assert np.abs(K - Klin).max() <= 1e-13 * np.abs(Klin).max()
    Ku = Klin @ u.ravel()
    assert np.abs(f.residual(u).ravel() - Ku).max() <= 1e-13 * np.abs(Ku).max()
    psi = 0.5 * u.ravel() @ Ku
    assert abs(f.energy(u) - psi) <= 1e-13 * abs(psi)


@pytest.mark.parametrize("elem", ELEMS)
def test_linear_model_equals_neo_hookean_tangent_at_zero(elem):
    """The small-strain limit: both models share the reference tangent."""
    _, fl = make(elem, 2, mu_sigma=0.3, lam_ratio=1.5, model="linear")
    m, fn = make(elem, 2, mu_sigma=0.3, lam_ratio=1.5)
    u = I.gaussian_field(m.n_nodes, 0.05, 6)
    K0 = dense_K(fn, np.zeros_like(m.X))
    assert np.abs(dense_K(fl, u) - K0).max() <= 1e-13 * np.abs(K0).max()


@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("ci", range(len(F0_CASES)))
def test_linear_model_patch_test(elem, ci):
    """Affine u = (G - I) X: Psi = V psi_lin(G - I), and the residual vanishes
    at every node not on the boundary."""
    G = F0_CASES[ci] - np.eye(3)
    m, f = make(elem, 3, model="linear")
    u = affine(m.X, np.eye(3) + G)
    vol = np.sum(f.volumes()[0])
    ref = vol * pins.psi_linear(G, 1.0, 1.5)
    assert abs(f.energy(u) - ref) <= 1e-13 * abs(ref)
    inner = np.all((m.X > 1e-12) & (m.X < 1 - 1e-12), axis=1)
    r = f.residual(u)
    assert np.abs(r[inner]).max() <= 1e-13 * np.abs(r).max()


@pytest.mark.parametrize("elem", ELEMS)
def test_linear_model_infinitesimal_rotation_is_strain_free(elem):
    """A skew displacement gradient has eps = 0: no energy, no force."""
    W = np.array([[0.0, 0.3, -0.2], [-0.3, 0.0, 0.1], [0.2, -0.1, 0.0]])
    m, f = make(elem, 3, mu_sigma=0.3, model="linear")
    u = m.X @ W.T + np.array([0.1, -0.2, 0.3])
    assert abs(f.energy(u)) <= 1e-15
    assert np.abs(f.residual(u)).max() <= 1e-14


def test_linear_model_grad_material_closed_form():
    """Affine strain: dPsi/dmu_e = V_e eps:eps, dPsi/dlam_e = V_e (tr eps)^2 / 2."""
    G = F0_CASES[0] - np.eye(3)
    eps = 0.5 * (G + G.T)
    for elem in ELEMS:
        m, f = make(elem, 2, model="linear")
        gm, gl = f.grad_material(affine(m.X, np.eye(3) + G))
        vol, _ = f.volumes()
        assert np.abs(gm - vol * np.sum(eps * eps)).max() <= 1e-15
        assert np.abs(gl - vol * 0.5 * np.trace(eps) ** 2).max() <= 1e-15


# ------------------------------------------------- Tri3 (plane strain)

def plane(F2):
    F = np.eye(3)
    F[:2, :2] = F2
    return F


def planar_affine(X, F2):
    u = X @ (plane(F2) - np.eye(3)).T
    u[:, 2] = 0.0
    return u


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("ci", range(2))
def test_tri3_plane_strain_patch_test(model, ci):
    """In-plane affine u with u_z = 0: Psi = area psi(F) with F = diag(F_2D, 1)
    (numpy SVD principal stretches, or the linear density), no force on
    interior nodes, and no out-of-plane force anywhere."""
    F2 = [np.array([[1.10, 0.05], [0.03, 0.95]]), np.array([[0.80, 0.30], [0.10, 1.20]])][ci]
    m, f = make(I.TRI3, 4, model=model)
    u = planar_affine(m.X, F2)
    F = plane(F2)
    ref = pins.psi_principal(F, 1.0, 1.5) if model == "neo_hookean" else pins.psi_linear(F - np.eye(3), 1.0, 1.5)
    assert abs(f.energy(u) - ref) <= 1e-13 * abs(ref)
    r = f.residual(u)
    inner = np.all((m.X[:, :2] > 1e-12) & (m.X[:, :2] < 1 - 1e-12), axis=1)
    assert np.abs(r[inner]).max() <= 1e-13 * np.abs(r).max()
    assert np.abs(r[:, 2]).max() <= 1e-15


def test_tri3_reference_stiffness_is_textbook_plane_strain():
    """K(0) on in-plane DOFs = sum B^T D B area with the plane-strain Hooke
    matrix; in-plane and out-of-plane DOFs do not couple."""
    m, f = make(I.TRI3, 3, mu_sigma=0.4, lam_ratio=1.5)
    K = dense_K(f, np.zeros_like(m.X))
    n = m.n_nodes
    Kt = np.zeros((2 * n, 2 * n))
    for e, ce in enumerate(m.conn):
        Xe = m.X[ce][:, :2]
        M = np.hstack([np.ones((3, 1)), Xe])
        G = np.linalg.inv(M)[1:, :].T            # [3, 2] gradients
        area = 0.5 * np.linalg.det(M)
        B = np.zeros((3, 6))
        for a in range(3):
            B[0, 2 * a], B[1, 2 * a + 1] = G[a]
            B[2, 2 * a], B[2, 2 * a + 1] = G[a, 1], G[a, 0]
        mu, lam = f.mu[e], f.lam[e]
        D = np.array([[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, mu]])
        dofs = (2 * ce[:, None] + np.arange(2)[None, :]).ravel()
        Kt[np.ix_(dofs, dofs)] += area * B.T @ D @ B
    ip = (3 * np.arange(n)[:, None] + np.arange(2)[None, :]).ravel()
    assert np.abs(K[np.ix_(ip, ip)] - Kt).max() <= 1e-13 * np.abs(Kt).max()
    assert np.abs(K[np.ix_(ip, 3 * np.arange(n) + 2)]).max() == 0.0


def test_tri3_in_plane_rotation_is_stress_free():
    th = 0.7
    R2 = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    m, f = make(I.TRI3, 4, mu_sigma=0.3)
    u = planar_affine(m.X, R2)
    assert abs(f.energy(u)) < 1e-14
    assert np.abs(f.residual(u)).max() < 1e-14
