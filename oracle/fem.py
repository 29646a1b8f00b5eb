"""FP64 oracle operators, Dirichlet condensation and the Newton-CG iteration.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Layouts follow the flat DOF vector of Sec. 4 (``u_flat.reshape(-1, 3)``):
nodal arrays are float64 ``[n_nodes, 3]``, connectivity int32
``[n_elems, n_en]``, per-element fields float64 ``[n_elems]``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

TET4, HEX8, TRI3 = 0, 1, 2
# material models: compressible neo-Hookean (Sec. 6.1) and small-strain
# linear elasticity (the density of the paper's first example)
NEO_HOOKE, LINEAR = 0, 1
MODELS = {"neo_hookean": NEO_HOOKE, "linear": LINEAR}
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        # EFEM_ORACLE_LIB lets the mutation test load a deliberately broken copy
        path = os.environ.get("EFEM_ORACLE_LIB") or _build.build()
        _lib = ctypes.CDLL(path)
        i64, c_int = ctypes.c_int64, ctypes.c_int
        common = [c_int, c_int, i64, i64, _dp, _ip]
        for name, extra in [
            ("orc_energy", [_dp, _dp, _dp, _dp, _dp]),
            ("orc_residual", [_dp, _dp, _dp, _dp]),
            ("orc_hvp", [_dp, _dp, _dp, _dp, _dp]),
            ("orc_element_tangents", [_dp, _dp, _dp, _dp]),
            ("orc_jacobi_diag", [_dp, _dp, _dp, _dp]),
            ("orc_grad_material", [_dp, _dp, _dp]),
            ("orc_residual_vjp_material", [_dp, _dp, _dp, _dp]),
            ("orc_grad_coords", [_dp, _dp, _dp, _dp]),
            ("orc_volumes", [_dp]),
        ]:
            f = getattr(_lib, name)
            f.argtypes = common + extra
            f.restype = c_int
        _lib.orc_num_threads.restype = c_int
    return _lib


def num_threads() -> int:
    return lib().orc_num_threads()


def _d(a):
    return a.ctypes.data_as(_dp)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc == -4:
        raise OracleError(f"{what}: an element has det J <= 0 or det F <= 0")
    if rc != 0:
        raise OracleError(f"{what}: bad arguments (rc={rc})")


@dataclass
class FEM:
    """Mesh + per-element material: the geometric context of Sec. 4 (Operator).
    `model` is "neo_hookean" (default) or "linear"."""
    elem: int
    X: np.ndarray
    conn: np.ndarray
    mu: np.ndarray
    lam: np.ndarray
    model: str = "neo_hookean"

    def __post_init__(self):
        if self.model not in MODELS:
            raise ValueError(f"unknown material model {self.model!r}")
        self.X = np.ascontiguousarray(self.X, dtype=np.float64)
        self.conn = np.ascontiguousarray(self.conn, dtype=np.int32)
        self.mu = np.ascontiguousarray(self.mu, dtype=np.float64)
        self.lam = np.ascontiguousarray(self.lam, dtype=np.float64)

    @property
    def n_nodes(self):
        return self.X.shape[0]

    @property
    def n_elems(self):
        return self.conn.shape[0]

    def _head(self):
        return (self.elem, MODELS[self.model], self.n_nodes, self.n_elems, _d(self.X),
                self.conn.ctypes.data_as(_ip))

    @staticmethod
    def _vec(a):
        return np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 3)

    # --- Eq. (2): discrete energy
    def element_energies(self, u):
        u = self._vec(u)
        pe = np.empty(self.n_elems)
        tot = ctypes.c_double()
        rc = lib().orc_energy(*self._head(), _d(self.mu), _d(self.lam), _d(u), _d(pe),
                              ctypes.byref(tot))
        return pe, tot.value, rc

    def energy(self, u, allow_inverted=False):
        """Psi_h(u) of Eq. (2); +inf when an element is inverted (det F <= 0)."""
        _, tot, rc = self.element_energies(u)
        if rc == -4 and allow_inverted:
            return np.inf
        _check(rc, "energy")
        return tot

    # --- Eq. (1): r = grad Psi
    def residual(self, u):
        u = self._vec(u)
        r = np.empty_like(u)
        _check(lib().orc_residual(*self._head(), _d(self.mu), _d(self.lam), _d(u), _d(r)),
               "residual")
        return r

    # --- Eq. (3): K(u) v
    def hvp(self, u, v):
        u, v = self._vec(u), self._vec(v)
        y = np.empty_like(u)
        _check(lib().orc_hvp(*self._head(), _d(self.mu), _d(self.lam), _d(u), _d(v), _d(y)),
               "hvp")
        return y

    def element_tangents(self, u):
        """K_e [n_elems, 3 n_en, 3 n_en], the matrix form of Eq. (3) per element."""
        u = self._vec(u)
        m = 3 * self.conn.shape[1]
        Ke = np.empty((self.n_elems, m, m))
        _check(lib().orc_element_tangents(*self._head(), _d(self.mu), _d(self.lam), _d(u), _d(Ke)),
               "element_tangents")
        return Ke

    def tangent_matrix(self, u):
        """The global tangent K(u) as a scipy CSR matrix [3 n_nodes]^2: the sum of
        the element tangents over the connectivity (duplicates added)."""
        import scipy.sparse as sp
        Ke = self.element_tangents(u)
        dofs = (3 * self.conn[:, :, None] + np.arange(3)[None, None, :]).reshape(self.n_elems, -1)
        m = dofs.shape[1]
        rows = np.repeat(dofs, m, axis=1).reshape(-1)
        cols = np.tile(dofs, (1, m)).reshape(-1)
        n = 3 * self.X.shape[0]
        return sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()

    def jacobi_diag(self, u):
        """diag K(u), the Jacobi preconditioner of the Newton-CG solve."""
        u = self._vec(u)
        d = np.empty_like(u)
        _check(lib().orc_jacobi_diag(*self._head(), _d(self.mu), _d(self.lam), _d(u), _d(d)),
               "jacobi_diag")
        return d

    def jacobi_offdiag(self, u):
        """(K01, K02, K12) of every node's 3x3 diagonal block of K(u), [n_nodes, 3]:
        read off the assembled tangent (with jacobi_diag, the blocks of the
        block-Jacobi preconditioner)."""
        K = self.tangent_matrix(u).tocsr()
        i = 3 * np.arange(self.X.shape[0])
        return np.stack([np.asarray(K[i, i + 1]).ravel(), np.asarray(K[i, i + 2]).ravel(),
                         np.asarray(K[i + 1, i + 2]).ravel()], axis=1)

    def grad_material(self, u):
        """(dPsi/dmu_e, dPsi/dlam_e) at fixed u."""
        u = self._vec(u)
        gm, gl = np.empty(self.n_elems), np.empty(self.n_elems)
        _check(lib().orc_grad_material(*self._head(), _d(u), _d(gm), _d(gl)), "grad_material")
        return gm, gl

    def residual_vjp_material(self, u, w):
        """(w . dr/dmu_e, w . dr/dlam_e) at fixed u."""
        u, w = self._vec(u), self._vec(w)
        gm, gl = np.empty(self.n_elems), np.empty(self.n_elems)
        _check(lib().orc_residual_vjp_material(*self._head(), _d(u), _d(w), _d(gm), _d(gl)),
               "residual_vjp_material")
        return gm, gl

    def grad_coords(self, u):
        """dPsi/dX at fixed nodal displacement u, [n_nodes, 3]."""
        u = self._vec(u)
        g = np.empty_like(u)
        _check(lib().orc_grad_coords(*self._head(), _d(self.mu), _d(self.lam), _d(u), _d(g)),
               "grad_coords")
        return g

    def volumes(self):
        v = np.empty(self.n_elems)
        rc = lib().orc_volumes(*self._head(), _d(v))
        return v, rc


# ------------------------------------------------------------------ Dirichlet

def masked(mask, a):
    """Zero the prescribed DOFs (mask == 1) of a nodal array: the residual and the
    tangent action of the reduced functional over the free DOFs (Sec. 6.1)."""
    a = np.array(a, dtype=np.float64).reshape(-1)
    a[mask.reshape(-1) != 0] = 0.0
    return a.reshape(-1, 3)


# -------------------------------------------------------------- Newton-CG

@dataclass
class SolveOptions:
    n_steps: int = 5
    rtol: float = 1e-8              # ||r_free|| <= rtol * ||r_free at step start||
    atol_floor: float = 1e-14       # absolute floor, times max(1, rho0)
    eta_max: float = 0.5            # Eisenstat-Walker choice 2 parameters
    eta_min: float = 1e-10
    ew_gamma: float = 0.9
    ew_alpha: float = 2.0
    eta_fixed: float | None = None  # fixed forcing term (exact-solve cross-check)
    max_newton: int = 50
    max_cg: int = 20000
    predictor_rtol: float = 1e-4    # tangent predictor solve at each load step
    armijo_c: float = 1e-4
    max_halvings: int = 30


@dataclass
class SolveStats:
    newton_iters: list = field(default_factory=list)   # per load step
    cg_iters: list = field(default_factory=list)       # per load step (incl. predictor)
    residual_history: list = field(default_factory=list)
    energy_history: list = field(default_factory=list)
    converged: bool = True


def pcg(apply_K, b, dinv, rtol, max_iter):
    """Jacobi-preconditioned CG for K x = b from x0 = 0, stopped when
    ||b - K x|| <= rtol ||b||; on p^T K p <= 0 stop (steepest-descent step
    D^-1 b if that happens at the first iteration).  Returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0
    z = dinv * r
    p = z.copy()
    rz = r @ z
    for it in range(1, max_iter + 1):
        q = apply_K(p)
        pq = p @ q
        if not pq > 0.0:
            if it == 1:
                return dinv * b, it
            return x, it
        a = rz / pq
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= rtol * bn:
            return x, it
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iter


def newton_solve(fem: FEM, mask, u_bc_final, opts: SolveOptions, u0=None, f_ext=None):
    """Matrix-free Newton-Krylov on the reduced functional (Sec. 6.1, Sec. 6.3.1).

    The paper names the method but gives none of its parts; the reading used:
      * load steps k = 1..n, prescribed DOFs set to (k/n) of their final values;
      * each step starts from a tangent predictor: the prescribed increment is
        lifted into the free DOFs by solving K_ff d_f = -(K d_c)_f;
      * Newton: Jacobi-PCG on K_ff d = -r_f, forcing term by Eisenstat-Walker
        choice 2 with safeguards, then Armijo backtracking on the FP64 energy
        (steps that invert an element have energy +inf and are rejected; the
        sufficient-decrease test allows 64 eps |Psi| for the energy's rounding,
        below which a decrease cannot be resolved);
      * stop when ||r_f|| <= rtol ||r_f(step start)||.

    With external nodal forces f_ext (the work of a boundary traction,
    Sec. 6.1) the functional is the total potential energy Psi_h(u) - s f.u,
    s = k/n at step k: the residual gains -s f, the predictor's right-hand side
    +(s_k - s_(k-1)) f, and the line search compares total energies.
    """
    mask = np.asarray(mask).reshape(-1)
    free = (mask == 0).astype(np.float64)
    cons = 1.0 - free
    u = np.zeros(3 * fem.n_nodes) if u0 is None else np.array(u0, dtype=np.float64).reshape(-1)
    ubc = np.asarray(u_bc_final, dtype=np.float64).reshape(-1)
    st = SolveStats()
    f = np.zeros_like(u) if f_ext is None else np.asarray(f_ext, dtype=np.float64).reshape(-1)
    s = 0.0

    def K_ff(uu, p):
        return free * fem.hvp(uu, free * p).reshape(-1)

    def res_f(uu):
        return free * (fem.residual(uu).reshape(-1) - s * f)

    def total_energy(uu, allow_inverted=False):
        return fem.energy(uu, allow_inverted=allow_inverted) - s * (f @ uu)

    for k in range(1, opts.n_steps + 1):
        s_prev, s = s, k / opts.n_steps
        target = (k / opts.n_steps) * ubc
        # tangent predictor: prescribed increment dc, free part from K_ff d_f = -(K dc)_f
        dc = cons * (target - u)
        d_inv = 1.0 / np.where(cons > 0, 1.0, fem.jacobi_diag(u).reshape(-1))
        rhs = free * ((s - s_prev) * f - fem.hvp(u, dc).reshape(-1))
        df, it_pred = pcg(lambda p: K_ff(u, p), rhs, d_inv * free + cons, opts.predictor_rtol,
                          opts.max_cg)
        u_try = u + dc + free * df
        if not np.isfinite(total_energy(u_try, allow_inverted=True)):
            u_try = u + dc          # predictor inverted an element: plain lift
        u = u_try
        cg_total = it_pred
        r = res_f(u)
        rho0 = np.linalg.norm(r)
        tol = max(opts.rtol * rho0, opts.atol_floor * max(1.0, rho0))
        hist = [rho0]
        ehist = [total_energy(u)]
        eta_prev, rn_prev = opts.eta_max, None
        nit = 0
        while np.linalg.norm(r) > tol:
            if nit >= opts.max_newton:
                st.converged = False
                break
            rn = np.linalg.norm(r)
            # forcing term
            if opts.eta_fixed is not None:
                eta = opts.eta_fixed
            elif rn_prev is None:
                eta = opts.eta_max
            else:
                eta = opts.ew_gamma * (rn / rn_prev) ** opts.ew_alpha
                safe = opts.ew_gamma * eta_prev ** opts.ew_alpha
                if safe > 0.1:
                    eta = max(eta, safe)
                eta = min(eta, opts.eta_max)
                eta = max(eta, 0.5 * tol / rn)
            eta = max(eta, opts.eta_min) if opts.eta_fixed is None else eta
            dg = fem.jacobi_diag(u).reshape(-1)
            dinv = free / np.where(free > 0, dg, 1.0) + cons
            d, it = pcg(lambda p: K_ff(u, p), -r, dinv, eta, opts.max_cg)
            d = free * d
            cg_total += it
            # Armijo backtracking on the FP64 energy
            e0 = ehist[-1]
            slope = r @ d
            alpha = 1.0
            for _ in range(opts.max_halvings + 1):
                e1 = total_energy(u + alpha * d, allow_inverted=True)
                # sufficient decrease up to the rounding of the energy sum (64 eps |Psi|)
                noise = 64.0 * np.finfo(np.float64).eps * abs(e0)
                if np.isfinite(e1) and e1 <= e0 + opts.armijo_c * alpha * slope + noise:
                    break
                alpha *= 0.5
            else:
                st.converged = False
                break
            u = u + alpha * d
            rn_prev, eta_prev = rn, eta
            r = res_f(u)
            hist.append(np.linalg.norm(r))
            ehist.append(e1)
            nit += 1
        st.newton_iters.append(nit)
        st.cg_iters.append(cg_total)
        st.residual_history.append(hist)
        st.energy_history.append(ehist)
        if not st.converged:
            break
    return u.reshape(-1, 3), st
