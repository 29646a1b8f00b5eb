"""Boundary loads and closed-form fields for the loaded-solve tests.

The total potential energy of the paper's plate example (Sec. 6.1) subtracts
the work of a boundary traction t.  With the linear (bilinear on hex faces)
boundary interpolation u = sum_a N_a u_a, that work is exactly f.u with
f_a = integral of t N_a over the loaded boundary.  Here f is computed from the
facet geometry alone:

* a uniform traction on a flat facet puts t |facet| / n_corners on each
  corner (edges, triangles, and the undistorted square faces of the hex
  grids, whose boundary nodes are never jittered);
* a varying traction (Kirsch's field on the plate's outer edges) is
  integrated along each straight edge with 5-point Gauss-Legendre, exact to
  degree 9 in the edge coordinate.

It also holds Kirsch's solution for an infinite plate with a circular hole
under remote uniaxial tension, which the plate example compares against, and
the element stress of the small-strain model on Tri3 meshes for that
comparison.
"""
from __future__ import annotations

import numpy as np

from paper_2602_12365_amd import inputs as I

# local facets of each element type (corner lists)
_FACETS = {
    I.TRI3: [(0, 1), (1, 2), (2, 0)],
    I.TET4: [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)],
    I.HEX8: [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)],
}


def _measure(P):
    """Length, area or (planar quad, corners in cyclic order) area of a facet."""
    if len(P) == 2:
        return np.linalg.norm(P[1] - P[0])
    if len(P) == 3:
        return 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    return 0.5 * np.linalg.norm(np.cross(P[2] - P[0], P[3] - P[1]))


def face_load(mesh, axis, value, traction, tol=1e-12):
    """Nodal forces [n_nodes, 3] of a uniform dead traction (3-vector) on the
    boundary facets lying in the plane X[:, axis] = value."""
    on = np.abs(mesh.X[:, axis] - value) < tol
    t = np.asarray(traction, dtype=np.float64)
    f = np.zeros((mesh.n_nodes, 3))
    for fc in _FACETS[mesh.elem]:
        ids = mesh.conn[:, list(fc)]
        for e in np.nonzero(np.all(on[ids], axis=1))[0]:
            share = _measure(mesh.X[ids[e]]) / len(fc)
            f[ids[e]] += share * t
    return f


# ----------------------------------------------------------------- Kirsch

def kirsch_stress(x, y, radius, sigma):
    """Cartesian in-plane stress (sxx, syy, sxy) of Kirsch's solution: an
    infinite plate with a traction-free circular hole of ``radius`` centred at
    the origin, under remote uniaxial tension ``sigma`` along x.  In polar
    components (rho = radius / r):
      s_rr = sigma/2 (1 - rho^2) + sigma/2 (1 - 4 rho^2 + 3 rho^4) cos 2th
      s_tt = sigma/2 (1 + rho^2) - sigma/2 (1 + 3 rho^4) cos 2th
      s_rt = -sigma/2 (1 + 2 rho^2 - 3 rho^4) sin 2th
    (independent of the elastic constants, in plane strain as in plane stress)."""
    r = np.hypot(x, y)
    th = np.arctan2(y, x)
    q = (radius / r) ** 2
    c2, s2 = np.cos(2 * th), np.sin(2 * th)
    srr = 0.5 * sigma * (1 - q) + 0.5 * sigma * (1 - 4 * q + 3 * q * q) * c2
    stt = 0.5 * sigma * (1 + q) - 0.5 * sigma * (1 + 3 * q * q) * c2
    srt = -0.5 * sigma * (1 + 2 * q - 3 * q * q) * s2
    c, s = np.cos(th), np.sin(th)
    sxx = srr * c * c + stt * s * s - 2 * srt * s * c
    syy = srr * s * s + stt * c * c + 2 * srt * s * c
    sxy = (srr - stt) * s * c + srt * (c * c - s * s)
    return sxx, syy, sxy


_GL5_X = np.array([-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831,
                   0.9061798459386640])
_GL5_W = np.array([0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                   0.4786286704993665, 0.2369268850561891])


def kirsch_outer_load(mesh, n_r, radius, half_width, sigma):
    """Nodal forces [n_nodes, 3] of Kirsch's traction on the outer edges
    x = W (normal +x) and y = W (normal +y) of ``plate_with_hole_mesh(n_r, n_t)``."""
    X = mesh.X
    n_t = mesh.n
    outer = np.array([n_r + (n_r + 1) * j for j in range(2 * n_t + 1)])
    f = np.zeros((mesh.n_nodes, 3))
    for a, b in zip(outer[:-1], outer[1:]):
        pa, pb = X[a, :2], X[b, :2]
        L = np.linalg.norm(pb - pa)
        mid = 0.5 * (pa + pb)
        on_right = abs(pa[0] - half_width) < 1e-12 and abs(pb[0] - half_width) < 1e-12
        for xg, wg in zip(_GL5_X, _GL5_W):
            p = mid + 0.5 * xg * (pb - pa)
            sxx, syy, sxy = kirsch_stress(p[0], p[1], radius, sigma)
            t = np.array([sxx, sxy]) if on_right else np.array([sxy, syy])
            Na, Nb = 0.5 * (1 - xg), 0.5 * (1 + xg)
            f[a, :2] += 0.5 * L * wg * Na * t
            f[b, :2] += 0.5 * L * wg * Nb * t
    return f


def tri_stress_linear(X, conn, u, mu, lam):
    """Per-element in-plane stress (sxx, syy, sxy) of the small-strain model
    sigma = 2 mu eps + lam tr(eps) I on a plane-strain Tri3 mesh (constant
    strain per triangle, from the nodal values by the triangle's own geometry).
    Returns (sxx, syy, sxy, area), each [n_elems]."""
    P = X[conn][:, :, :2]
    U = np.asarray(u).reshape(-1, 3)[conn][:, :, :2]
    x1, y1 = P[:, 1, 0] - P[:, 0, 0], P[:, 1, 1] - P[:, 0, 1]
    x2, y2 = P[:, 2, 0] - P[:, 0, 0], P[:, 2, 1] - P[:, 0, 1]
    det = x1 * y2 - x2 * y1
    # gradients of the barycentric coordinates of nodes 1 and 2; node 0 closes the sum
    g1 = np.stack([y2, -x2], 1) / det[:, None]
    g2 = np.stack([-y1, x1], 1) / det[:, None]
    g0 = -g1 - g2
    H = (U[:, 0, :, None] * g0[:, None, :] + U[:, 1, :, None] * g1[:, None, :]
         + U[:, 2, :, None] * g2[:, None, :])
    exx, eyy, exy = H[:, 0, 0], H[:, 1, 1], 0.5 * (H[:, 0, 1] + H[:, 1, 0])
    tr = exx + eyy
    return 2 * mu * exx + lam * tr, 2 * mu * eyy + lam * tr, 2 * mu * exy, 0.5 * det


def kirsch_error(mesh, u, mu, lam, radius, sigma):
    """Area-weighted relative L2 difference of the element stresses from
    Kirsch's stresses at the element centroids, and the centroids."""
    sxx, syy, sxy, area = tri_stress_linear(mesh.X, mesh.conn, u, mu, lam)
    cen = mesh.X[mesh.conn][:, :, :2].mean(axis=1)
    kxx, kyy, kxy = kirsch_stress(cen[:, 0], cen[:, 1], radius, sigma)
    num = np.sum(area * ((sxx - kxx) ** 2 + (syy - kyy) ** 2 + 2 * (sxy - kxy) ** 2))
    den = np.sum(area * (kxx ** 2 + kyy ** 2 + 2 * kxy ** 2))
    return np.sqrt(num / den), (sxx, syy, sxy), cen


# ------------------------------------------------- homogeneous uniaxial state

def uniaxial_linear(mu, lam, t, planar):
    """Principal strains (e_xx, e_yy, e_zz) of the small-strain model under
    uniaxial stress t along x: free lateral faces in 3D, e_zz = 0 in plane
    strain.  From E = mu (3 lam + 2 mu) / (lam + mu) and
    nu = lam / (2 (lam + mu))."""
    E = mu * (3 * lam + 2 * mu) / (lam + mu)
    nu = lam / (2 * (lam + mu))
    if planar:
        return t * (1 - nu * nu) / E, -t * nu * (1 + nu) / E, 0.0
    return t / E, -nu * t / E, -nu * t / E


def uniaxial_neo_hooke(mu, lam, t, planar):
    """Principal stretches (a, b, c) of the homogeneous state with nominal
    stress t along x and zero lateral nominal stress (c = 1 in plane strain,
    c = b in 3D), for the neo-Hookean energy in principal stretches
    W = mu/2 (a^2 + b^2 + c^2 - 3) - mu ln(abc) + lam/2 ln(abc)^2, whose
    principal nominal stresses are dW/da = mu (a - 1/a) + lam ln(abc) / a, etc."""
    from scipy.optimize import fsolve

    def eqs(z):
        a, b = z
        c = 1.0 if planar else b
        lnJ = np.log(a * b * c)
        return [mu * (a - 1 / a) + lam * lnJ / a - t, mu * (b - 1 / b) + lam * lnJ / b]

    a, b = fsolve(eqs, [1.0, 1.0], xtol=1e-12)
    return a, b, 1.0 if planar else b
