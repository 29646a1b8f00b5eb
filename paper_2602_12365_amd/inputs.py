"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module holds no arithmetic of the method (no shape functions, no
quadrature, no material law).  It only builds structured unit-cube meshes and
draws seeded random fields, with numpy's PCG64 generator, in the layouts the
C-ABI expects:

* node coordinates ``X``: float64 ``[n_nodes, 3]`` (node-major, the flat DOF
  vector of Sec. 4 is ``u.reshape(-1)`` with ``dof = 3*node + comp``);
* connectivity ``conn``: int32 ``[n_elems, n_en]``;
* per-element material fields ``mu``, ``lam``: float64 ``[n_elems]``;
* Dirichlet masks: uint8 ``[n_nodes*3]``, 1 = prescribed.

The paper's own meshes are not available; structured cubes stand in for its 3D
tetrahedral "elasticity" scaling meshes (Sec. 5.1) and for the hexahedral
meshes of the configurations measured here.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

TET4 = 0
HEX8 = 1
TRI3 = 2
N_EN = {TET4: 4, HEX8: 8, TRI3: 3}


@dataclass
class Mesh:
    elem: int            # TET4 or HEX8
    n: int               # hexes per cube edge
    X: np.ndarray        # float64 [n_nodes, 3]
    conn: np.ndarray     # int32 [n_elems, n_en]

    @property
    def n_nodes(self) -> int:
        return self.X.shape[0]

    @property
    def n_elems(self) -> int:
        return self.conn.shape[0]

    @property
    def n_dofs(self) -> int:
        """Unknowns: 3 per node, 2 (in-plane) for the planar Tri3 mesh."""
        return (2 if self.elem == TRI3 else 3) * self.X.shape[0]


def grid_nodes(n: int) -> np.ndarray:
    """Nodes of the unit cube with n hexes per edge; id = i + (n+1)(j + (n+1)k)."""
    t = np.arange(n + 1, dtype=np.float64) / n
    k, j, i = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).copy()


def _hex_corner_ids(n: int) -> np.ndarray:
    """[n^3] ids of the (0,0,0) corner of each hex, hexes ordered k, j, i (i fastest)."""
    m = n + 1
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return (i + m * (j + m * k)).ravel().astype(np.int64)


def hex_mesh(n: int) -> Mesh:
    """Q1 hexahedra, local node order: the four z=0 corners counter-clockwise
    from the origin, then the same four at z=1 (the usual VTK order)."""
    m = n + 1
    p = _hex_corner_ids(n)
    off = [0, 1, 1 + m, m, m * m, 1 + m * m, 1 + m + m * m, m + m * m]
    conn = np.stack([p + o for o in off], axis=1).astype(np.int32)
    return Mesh(HEX8, n, grid_nodes(n), conn)


def tet_mesh(n: int) -> Mesh:
    """Each hex split into six tetrahedra along its main diagonal (Kuhn split).

    For the axis permutation (a, b, c) the tetrahedron is
    [p, p+e_a, p+e_a+e_b, p+(1,1,1)]; its edge matrix has the determinant of
    the permutation, so for odd permutations the last two local nodes are
    swapped to keep every tetrahedron positively oriented.  All hexes use the
    same diagonal, so the split is conforming.
    """
    m = n + 1
    stride = np.array([1, m, m * m], dtype=np.int64)
    p = _hex_corner_ids(n)
    tets = []
    for perm in itertools.permutations(range(3)):
        a, b, _ = perm
        # parity of the permutation: number of inversions
        inv = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        n1 = p + stride[a]
        n2 = n1 + stride[b]
        n3 = p + stride.sum()
        if inv % 2 == 0:
            tets.append(np.stack([p, n1, n2, n3], axis=1))
        else:
            tets.append(np.stack([p, n1, n3, n2], axis=1))
    # six tets per hex, consecutive
    conn = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return Mesh(TET4, n, grid_nodes(n), conn)


def tri_mesh(n: int) -> Mesh:
    """Unit square in the z = 0 plane, n x n cells, each cut into two
    counter-clockwise triangles along alternating diagonals (a criss-cross
    free of a preferred direction); node id = i + (n+1) j."""
    t = np.linspace(0.0, 1.0, n + 1)
    x, y = np.meshgrid(t, t, indexing="xy")
    X = np.stack([x.ravel(), y.ravel(), np.zeros((n + 1) ** 2)], axis=1)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    a = (i + (n + 1) * j).ravel()
    b, c, d = a + 1, a + 1 + (n + 1), a + (n + 1)
    even = ((i + j) % 2 == 0).ravel()
    t1 = np.where(even[:, None], np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t2 = np.where(even[:, None], np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    tris = np.stack([t1, t2], axis=1).reshape(-1, 3)   # cell by cell, two triangles each
    return Mesh(TRI3, n, X, tris.astype(np.int32))


def plate_with_hole_mesh(n_r: int, n_t: int, radius: float = 0.05,
                         half_width: float = 0.5) -> Mesh:
    """Quarter of a square plate (side 2 half_width) with a centred circular
    hole of ``radius``, in the z = 0 plane: the first-quadrant region between
    the circle and the square max(x, y) = half_width, for the plate-with-hole
    example of Sec. 6.1 (hole radius 0.05 there; the plate size is not
    stated, a unit plate is taken).

    Node (i, j), id = i + (n_r + 1) j, lies on the straight ray from the hole
    point at angle (pi/2) j / (2 n_t) to the point at arc length fraction
    j / (2 n_t) of the outer path (W, 0) -> (W, W) -> (0, W), W = half_width;
    both meet the diagonal at j = n_t.  Along a ray, i = 0..n_r is spaced
    geometrically with cell ratio (W / radius)^(1/n_r), which makes the x and
    y axis rays exactly logarithmic in r.  Every quad is cut into two
    counter-clockwise triangles along alternating diagonals.  Boundaries: j = 0
    is the x axis, j = 2 n_t the y axis, i = 0 the hole, i = n_r the outer
    edges x = W (j <= n_t) and y = W (j >= n_t)."""
    m_t = 2 * n_t
    g = (half_width / radius) ** (1.0 / n_r)
    xi = (g ** np.arange(n_r + 1) - 1.0) / (g ** n_r - 1.0)
    j = np.arange(m_t + 1)
    th = 0.5 * np.pi * j / m_t
    inner = radius * np.stack([np.cos(th), np.sin(th)], axis=1)
    s = 2.0 * half_width * j / m_t
    outer = np.where((s <= half_width)[:, None],
                     np.stack([np.full_like(s, half_width), s], axis=1),
                     np.stack([2.0 * half_width - s, np.full_like(s, half_width)], axis=1))
    outer[-1, 0] = 0.0
    outer[0, 1] = 0.0
    P = (1.0 - xi[None, :, None]) * inner[:, None, :] + xi[None, :, None] * outer[:, None, :]
    X = np.concatenate([P.reshape(-1, 2), np.zeros(((n_r + 1) * (m_t + 1), 1))], axis=1)
    jj, ii = np.meshgrid(np.arange(m_t), np.arange(n_r), indexing="ij")
    a = (ii + (n_r + 1) * jj).ravel()
    b, c, d = a + 1, a + 1 + (n_r + 1), a + (n_r + 1)
    even = ((ii + jj) % 2 == 0).ravel()
    t1 = np.where(even[:, None], np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t2 = np.where(even[:, None], np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    tris = np.stack([t1, t2], axis=1).reshape(-1, 3)
    return Mesh(TRI3, n_t, X, tris.astype(np.int32))


def symmetry_mask(X: np.ndarray, planar: bool) -> np.ndarray:
    """Symmetry conditions on the coordinate planes: u_x = 0 where x = 0,
    u_y = 0 where y = 0, and u_z = 0 where z = 0 (3D) or everywhere (plane
    strain, ``planar``).  uint8 [3 n_nodes]; every prescribed value is 0."""
    mask = np.zeros((X.shape[0], 3), dtype=np.uint8)
    mask[np.abs(X[:, 0]) < 1e-12, 0] = 1
    mask[np.abs(X[:, 1]) < 1e-12, 1] = 1
    if planar:
        mask[:, 2] = 1
    else:
        mask[np.abs(X[:, 2]) < 1e-12, 2] = 1
    return mask.reshape(-1)


def planar_mask(X: np.ndarray) -> np.ndarray:
    """uint8 [n_nodes, 3] holding the out-of-plane component of every node
    (plane strain on a Tri3 mesh)."""
    m = np.zeros((X.shape[0], 3), dtype=np.uint8)
    m[:, 2] = 1
    return m


def clamp_planar(X: np.ndarray, top_dy: float):
    """Plane-strain load case on the unit square: every out-of-plane
    component held at 0, the bottom edge y = 0 clamped, the top edge y = 1
    gripped and moved by top_dy in y.  Returns (mask uint8 [3 n], u_bc [n, 3])."""
    mask = planar_mask(X)
    ubc = np.zeros_like(X)
    bottom = np.abs(X[:, 1]) < 1e-12
    top = np.abs(X[:, 1] - 1.0) < 1e-12
    mask[bottom] = 1
    mask[top] = 1
    ubc[top, 1] = top_dy
    return mask.reshape(-1), ubc


def make_mesh(elem: int, n: int) -> Mesh:
    if elem == TRI3:
        return tri_mesh(n)
    return tet_mesh(n) if elem == TET4 else hex_mesh(n)


# the twelve even permutations of four local nodes (orientation-preserving)
_EVEN4 = np.array([p for p in itertools.permutations(range(4))
                   if sum(1 for x in range(4) for y in range(x + 1, 4) if p[x] > p[y]) % 2 == 0],
                  dtype=np.int64)


def scrambled_mesh(mesh: Mesh, seed: int, jitter: float = 0.1) -> Mesh:
    """The same cube with shuffled node ids and element order, interior nodes
    moved by up to ``jitter`` grid spacings per coordinate, and (tetrahedra)
    each element's local nodes rotated by a random even permutation, so no
    regular structure of the generator survives."""
    g = rng(seed)
    nn, ne = mesh.n_nodes, mesh.n_elems
    X = mesh.X.copy()
    interior = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    X[interior] += (jitter / mesh.n) * g.uniform(-1.0, 1.0, size=(int(interior.sum()), 3))
    new_id = g.permutation(nn)
    Xs = np.empty_like(X)
    Xs[new_id] = X
    conn = new_id[mesh.conn.astype(np.int64)]
    conn = conn[g.permutation(ne)]
    if mesh.elem == TET4:
        conn = np.take_along_axis(conn, _EVEN4[g.integers(0, len(_EVEN4), size=ne)], axis=1)
    return Mesh(mesh.elem, mesh.n, Xs, conn.astype(np.int32))


# ----------------------------------------------------------------- fields

def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def gaussian_field(n_nodes: int, amplitude: float, seed: int) -> np.ndarray:
    """u = amplitude * N(0,1) per DOF, float64 [n_nodes, 3]."""
    return amplitude * rng(seed).standard_normal((n_nodes, 3))


def unit_direction(n_nodes: int, seed: int) -> np.ndarray:
    """v = g / ||g||_2 with g ~ N(0,1) per DOF over all DOFs, float64 [n_nodes, 3]."""
    g = rng(seed).standard_normal((n_nodes, 3))
    return g / np.linalg.norm(g)


def lognormal_field(n_elems: int, sigma: float, seed: int) -> np.ndarray:
    """mu_e = exp(sigma * Z_e), Z_e ~ N(0,1) i.i.d. per element."""
    return np.exp(sigma * rng(seed).standard_normal(n_elems))


def constant_field(n_elems: int, value: float) -> np.ndarray:
    return np.full(n_elems, float(value))


def random_rotation(seed: int) -> np.ndarray:
    """A random proper rotation (QR of a Gaussian matrix with sign fix)."""
    q, r = np.linalg.qr(rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# ------------------------------------------------------------- boundaries

def face_nodes(X: np.ndarray, axis: int, value: float, tol: float = 1e-12) -> np.ndarray:
    return np.nonzero(np.abs(X[:, axis] - value) < tol)[0]


def clamp_top_bottom(X: np.ndarray, top_dz: float, top_all_components: bool = True):
    """Bottom face z=0 fully clamped; top face z=1 displaced by top_dz in z.

    With ``top_all_components`` the top face is gripped (u_x = u_y = 0 there as
    well); otherwise only u_z is prescribed on the top face.
    Returns (mask uint8 [3*n_nodes], u_bc float64 [n_nodes, 3]) where u_bc holds
    the prescribed values of the final load step (zero on free DOFs).
    """
    n_nodes = X.shape[0]
    mask = np.zeros((n_nodes, 3), dtype=np.uint8)
    u_bc = np.zeros((n_nodes, 3))
    bot = face_nodes(X, 2, 0.0)
    top = face_nodes(X, 2, 1.0)
    mask[bot, :] = 1
    if top_all_components:
        mask[top, :] = 1
    else:
        mask[top, 2] = 1
    u_bc[top, 2] = top_dz
    return mask.reshape(-1), u_bc


# -------------------------------------------------------- named workloads

@dataclass
class OperatorCase:
    mesh: Mesh
    mu: np.ndarray
    lam: np.ndarray
    u: np.ndarray
    v: np.ndarray


def operator_case(elem: int, n: int, u_amp: float, u_seed: int = 0, v_seed: int = 1,
                  mu_sigma: float = 0.0, mu_seed: int = 3, lam_ratio: float | None = None,
                  lam_const: float = 1.5) -> OperatorCase:
    """Mesh + material + a state u + a unit direction v.

    mu is 1 when mu_sigma == 0, else lognormal(0, mu_sigma); lam is lam_ratio*mu
    when lam_ratio is given, else the constant lam_const.
    """
    mesh = make_mesh(elem, n)
    if mu_sigma == 0.0:
        mu = constant_field(mesh.n_elems, 1.0)
    else:
        mu = lognormal_field(mesh.n_elems, mu_sigma, mu_seed)
    lam = lam_ratio * mu if lam_ratio is not None else constant_field(mesh.n_elems, lam_const)
    u = gaussian_field(mesh.n_nodes, u_amp, u_seed)
    v = unit_direction(mesh.n_nodes, v_seed)
    return OperatorCase(mesh, mu, lam, u, v)


def cube_amplitude(n: int, base: float = 0.01, base_n: int = 8) -> float:
    """Displacement amplitude that keeps the nodal-gradient scale of an n=8
    cube with amplitude ``base`` (0.01*8/n): at the literal 0.01 a 64^3 Kuhn
    mesh inverts about a third of its tetrahedra."""
    return base * base_n / n
