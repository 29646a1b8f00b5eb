"""Independent references that pin the FP64 oracle.

None of these re-types the oracle's formulas: the energy is evaluated from the
principal stretches (numpy SVD), the stress by finite differences of that
energy, the small-strain limit from the linear-elastic density of the paper's
first example (Sec. 6.1 listing), and the stiffness at the reference state by
the textbook B^T D B assembly in Voigt notation with its own shape functions.
"""
from __future__ import annotations

import itertools

import numpy as np


# ----------------------------------------------------------------- material

def psi_principal(F, mu, lam):
    """Compressible neo-Hookean energy from principal stretches s_i = svd(F):
    mu/2 (sum s_i^2 - 3) - mu ln(s1 s2 s3) + lam/2 (ln(s1 s2 s3))^2 (det F > 0)."""
    s = np.linalg.svd(np.asarray(F, dtype=np.float64), compute_uv=False)
    lnJ = np.log(s).sum()
    return 0.5 * mu * (np.sum(s * s) - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ


def piola_fd(F, mu, lam, h=1e-6):
    """First Piola-Kirchhoff stress by central differences of psi_principal."""
    F = np.asarray(F, dtype=np.float64)
    P = np.zeros((3, 3))
    for i, J in itertools.product(range(3), range(3)):
        Fp, Fm = F.copy(), F.copy()
        Fp[i, J] += h
        Fm[i, J] -= h
        P[i, J] = (psi_principal(Fp, mu, lam) - psi_principal(Fm, mu, lam)) / (2 * h)
    return P


def psi_linear(G, mu, lam):
    """Linear-elastic density of the paper's first example (3D):
    eps = sym(G), sig = 2 mu eps + lam tr(eps) I, psi = 1/2 sig : eps."""
    eps = 0.5 * (G + G.T)
    sig = 2 * mu * eps + lam * np.trace(eps) * np.eye(3)
    return 0.5 * np.sum(sig * eps)


# ------------------------------------------------------------ shape functions

def tet_gradients(Xe):
    """Textbook volume coordinates: rows of inv([[1, x, y, z]_a]) give the
    constant gradients of the four linear shape functions; volume = det/6."""
    M = np.hstack([np.ones((4, 1)), Xe])
    C = np.linalg.inv(M)          # N_a(x) = C[0,a] + C[1:,a] . x
    vol = np.linalg.det(M) / 6.0
    return [(C[1:, :].T, vol)]    # one point: ([4,3] gradients, weight*detJ)


_HEX_SIGNS = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                       [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)


def hex_gradients(Xe):
    """Trilinear isoparametric hexahedron, 2x2x2 Gauss-Legendre rule."""
    pts = []
    g = 1.0 / np.sqrt(3.0)
    for z, y, x in itertools.product((-g, g), repeat=3):
        p = np.array([x, y, z])
        # dN/dxi for N_a = prod_k (1 + s_ak p_k)/2
        f = 0.5 * (1.0 + _HEX_SIGNS * p)              # [8,3] factors
        dN = np.empty((8, 3))
        for k in range(3):
            others = [m for m in range(3) if m != k]
            dN[:, k] = 0.5 * _HEX_SIGNS[:, k] * f[:, others[0]] * f[:, others[1]]
        Jm = Xe.T @ dN                                  # dx_i/dxi_J
        gN = dN @ np.linalg.inv(Jm)                     # [8,3]
        pts.append((gN, np.linalg.det(Jm)))
    return pts


def element_points(elem, Xe):
    return tet_gradients(Xe) if elem == 0 else hex_gradients(Xe)


# ------------------------------------------------------- textbook stiffness

def voigt_D(mu, lam):
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[:3, :3] += 2 * mu * np.eye(3)
    D[3:, 3:] = mu * np.eye(3)
    return D


def voigt_B(gN):
    """Strain-displacement matrix, Voigt order (xx, yy, zz, yz, xz, xy),
    engineering shear strains."""
    n = gN.shape[0]
    B = np.zeros((6, 3 * n))
    for a in range(n):
        gx, gy, gz = gN[a]
        c = 3 * a
        B[0, c] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c + 1], B[3, c + 2] = gz, gy
        B[4, c], B[4, c + 2] = gz, gx
        B[5, c], B[5, c + 1] = gy, gx
    return B


def linear_stiffness(elem, X, conn, mu, lam):
    """Dense textbook K = sum_e sum_q B^T D B w detJ (small meshes only)."""
    n = 3 * X.shape[0]
    K = np.zeros((n, n))
    for e, ce in enumerate(conn):
        D = voigt_D(mu[e], lam[e])
        dofs = (3 * ce[:, None] + np.arange(3)[None, :]).ravel()
        for gN, wdet in element_points(elem, X[ce]):
            B = voigt_B(gN)
            K[np.ix_(dofs, dofs)] += wdet * (B.T @ D @ B)
    return K


# --------------------------------------------------------------- boundary

def boundary_faces(elem, conn):
    """Faces that belong to exactly one element, as node tuples."""
    if elem == 0:
        local = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
    else:
        local = [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]
    count = {}
    for ce in conn:
        for f in local:
            nodes = tuple(int(ce[i]) for i in f)
            key = tuple(sorted(nodes))
            count.setdefault(key, []).append(nodes)
    return [v[0] for v in count.values() if len(v) == 1]


def consistent_traction_loads(X, faces, P):
    """Nodal loads of the constant nominal traction P n on the boundary: each
    flat face of area A and outward normal n gives A/k (P n) to its k nodes
    (linear triangles and bilinear parallelograms)."""
    f = np.zeros_like(X)
    centre = X.mean(axis=0)
    for nodes in faces:
        pts = X[list(nodes)]
        if len(nodes) == 3:
            an = 0.5 * np.cross(pts[1] - pts[0], pts[2] - pts[0])
        else:
            an = np.cross(pts[1] - pts[0], pts[3] - pts[0])   # parallelogram
        if an @ (pts.mean(axis=0) - centre) < 0:
            an = -an
        for a in nodes:
            f[a] += (P @ an) / len(nodes)
    return f
