"""FP64 oracle of the non-variational transport problem (virtual work, Sec. 3.1,
Eqs. 4-6; the example of Sec. 6.5).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The advection-diffusion example's weak form (steady, or one implicit time
step with k = 1/dt), for three species carried in the three nodal components:

    r_{a,s}(c) = sum_e sum_q w detJ [ D_e grad c_s . grad N_a
                                      + (b(x_q) . grad c_s + k_e c_s(x_q)) N_a ]

with b(x) = omega x x.  r is linear in c, so the tangent K = dr/dc is constant,
K v = r(v), and the advection term makes it non-symmetric.  The reduced
system of a Dirichlet problem is solved directly (scipy sparse LU), so the
GPU's Krylov solve is checked against an exact solve, not another iteration.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import fem as _fem

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_ready = False


def _lib():
    global _ready
    L = _fem.lib()
    if not _ready:
        i64, c_int = ctypes.c_int64, ctypes.c_int
        head = [c_int, i64, i64, _dp, _ip, _dp, _dp, _dp]
        L.orc_transport_residual.argtypes = head + [_dp, _dp]
        L.orc_transport_residual.restype = c_int
        L.orc_transport_tangents.argtypes = head + [_dp]
        L.orc_transport_tangents.restype = c_int
        _ready = True
    return L


def _d(a):
    return a.ctypes.data_as(_dp)


@dataclass
class Transport:
    """Mesh, per-element diffusivity D and reaction k, rotation vector omega."""
    elem: int
    X: np.ndarray
    conn: np.ndarray
    D: np.ndarray
    k: np.ndarray
    omega: np.ndarray

    def __post_init__(self):
        self.X = np.ascontiguousarray(self.X, dtype=np.float64)
        self.conn = np.ascontiguousarray(self.conn, dtype=np.int32)
        self.D = np.ascontiguousarray(self.D, dtype=np.float64)
        self.k = np.ascontiguousarray(self.k, dtype=np.float64)
        self.omega = np.ascontiguousarray(self.omega, dtype=np.float64).reshape(3)

    @property
    def n_nodes(self):
        return self.X.shape[0]

    def _head(self):
        return (self.elem, self.n_nodes, self.conn.shape[0], _d(self.X), self.conn.ctypes.data_as(_ip),
                _d(self.D), _d(self.k), _d(self.omega))

    def residual(self, c):
        """r(c) [n_nodes, 3]; also the tangent action K c (r is linear)."""
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(-1, 3)
        r = np.empty_like(c)
        _fem._check(_lib().orc_transport_residual(*self._head(), _d(c), _d(r)), "transport_residual")
        return r

    hvp = residual

    def element_tangents(self):
        m = 3 * self.conn.shape[1]
        Ke = np.empty((self.conn.shape[0], m, m))
        _fem._check(_lib().orc_transport_tangents(*self._head(), _d(Ke)), "transport_tangents")
        return Ke

    def tangent_matrix(self):
        """K as scipy CSR [3 n_nodes]^2 (element matrices summed over the connectivity)."""
        import scipy.sparse as sp
        Ke = self.element_tangents()
        ne = self.conn.shape[0]
        dofs = (3 * self.conn[:, :, None] + np.arange(3)[None, None, :]).reshape(ne, -1)
        m = dofs.shape[1]
        rows = np.repeat(dofs, m, axis=1).reshape(-1)
        cols = np.tile(dofs, (1, m)).reshape(-1)
        n = 3 * self.n_nodes
        return sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()

    def diag(self):
        return self.tangent_matrix().diagonal().reshape(-1, 3)

    def solve_reduced(self, mask, b):
        """x with K_ff x_f = b_f and x = 0 on prescribed DOFs (mask uint8/bool
        [n_nodes, 3], 1 = prescribed), by a direct sparse solve."""
        import scipy.sparse.linalg as spla
        free = ~np.asarray(mask, dtype=bool).reshape(-1)
        K = self.tangent_matrix()
        Kff = K[free][:, free].tocsc()
        x = np.zeros(3 * self.n_nodes)
        x[free] = spla.spsolve(Kff, np.asarray(b, dtype=np.float64).reshape(-1)[free])
        return x.reshape(-1, 3)
