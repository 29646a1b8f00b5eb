"""torch-facing wrapper of the C-ABI: an ``Operator`` built from a mesh (Sec. 4,
``Operator(mesh, element, batchsize)``) and the ``torch.autograd.Function``s
whose backward passes are the hand-written adjoint kernels.

PyTorch only supplies device memory and streams: every operator runs in the
HIP kernels of ``libefem.so``; this module checks shapes, dtypes and devices
and passes raw pointers.
"""
from __future__ import annotations

import contextlib
import ctypes

import numpy as np
import torch

from . import _lib as L

_ELEM = {"tet4": L.EFEM_TET4, "hex8": L.EFEM_HEX8, "tri3": L.EFEM_TRI3,
         L.EFEM_TET4: L.EFEM_TET4, L.EFEM_HEX8: L.EFEM_HEX8, L.EFEM_TRI3: L.EFEM_TRI3}
_NEN = {L.EFEM_TET4: 4, L.EFEM_HEX8: 8, L.EFEM_TRI3: 3}
_PREC = {"f64": L.EFEM_F64, "f32": L.EFEM_F32, torch.float64: L.EFEM_F64, torch.float32: L.EFEM_F32}
_MODEL = {"neo_hookean": L.EFEM_MODEL_NEO_HOOKE, "linear": L.EFEM_MODEL_LINEAR,
          "transport": L.EFEM_MODEL_TRANSPORT}
_SCATTER = {"halo": L.EFEM_SCATTER_HALO, "color": L.EFEM_SCATTER_COLOR, "atomic": L.EFEM_SCATTER_ATOMIC}


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Operator:
    """Energy, residual, tangent action and adjoints of one mesh on one GPU.

    Mesh arrays (``X`` float64 [n_nodes, 3], ``conn`` int32 [n_elems, n_en])
    are host arrays; every state tensor is a contiguous CUDA tensor, float64
    unless stated, of shape [n_nodes, 3] (or the flat [3*n_nodes]).
    Calls run on torch's current stream.
    """

    def __init__(self, elem, X, conn, *, block_elems=0, block_nodes=0, scatter="halo",
                 threads=0, pairs=True, chunks=True, model="neo_hookean", device=None):
        self._lib = L.load()
        X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
        conn = np.ascontiguousarray(np.asarray(conn, dtype=np.int32))
        if X.ndim != 2 or X.shape[1] != 3:
            raise ValueError("X must be [n_nodes, 3]")
        self.elem = _ELEM[elem]
        self.nen = _NEN[self.elem]
        if conn.ndim != 2 or conn.shape[1] != self.nen:
            raise ValueError(f"conn must be [n_elems, {self.nen}]")
        self.n_nodes, self.n_elems = X.shape[0], conn.shape[0]
        dev = torch.device(device) if device is not None else torch.device("cuda")
        if dev.type != "cuda":
            raise ValueError("the operator runs on a GPU device")
        self.device = torch.device("cuda", dev.index if dev.index is not None else torch.cuda.current_device())
        self.X_host = X
        self.pairs = bool(pairs)
        self.chunks = bool(chunks)
        opts = L.Options(block_elems, block_nodes, _SCATTER[scatter], threads, 0 if pairs else 1,
                         0 if chunks else 1)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._stream = torch.cuda.current_stream().cuda_stream
            L.check(self._lib.efem_create(ctypes.byref(h), self.elem, self.n_nodes, self.n_elems,
                                          X.ctypes.data_as(ctypes.c_void_p),
                                          conn.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts),
                                          ctypes.c_void_p(self._stream)), "efem_create")
        self._h = h
        self._lin = None
        self.X = torch.from_numpy(X).to(self.device)
        self.model = "neo_hookean"
        if model != "neo_hookean":
            self.set_model(model)

    # ------------------------------------------------------------- plumbing
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.efem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            L.check(self._lib.efem_set_stream(self._h, ctypes.c_void_p(s)), "efem_set_stream")
            self._stream = s

    def _nodal(self, t, dtype=torch.float64, name="array"):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != dtype:
            raise TypeError(f"{name} must be a {dtype} tensor on {self.device}")
        if t.numel() != 3 * self.n_nodes or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {3 * self.n_nodes} entries")
        return t

    def _elemwise(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if t.numel() != self.n_elems or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {self.n_elems} entries")
        return t

    def _new_nodal(self, dtype=torch.float64):
        return torch.empty((self.n_nodes, 3), dtype=dtype, device=self.device)

    # ---------------------------------------------------------------- setup
    def set_material(self, mu, lam):
        self._sync_stream()
        L.check(self._lib.efem_set_material(self._h, _ptr(self._elemwise(mu, "mu")),
                                            _ptr(self._elemwise(lam, "lam"))), "efem_set_material")

    def set_model(self, model):
        """Strain energy density: "neo_hookean" (default) or "linear" (small
        strain); or "transport", the non-variational advection-diffusion
        operator of three species (mu = diffusivity, lam = reaction rate,
        velocity omega x x from set_velocity), which has no energy."""
        if model not in _MODEL:
            raise ValueError(f"unknown material model {model!r}")
        L.check(self._lib.efem_set_model(self._h, _MODEL[model]), "efem_set_model")
        self.model = model
        self._lin = None

    def set_velocity(self, omega):
        """Rotation vector of the transport model's velocity b(x) = omega x x."""
        om = (ctypes.c_double * 3)(*[float(v) for v in omega])
        L.check(self._lib.efem_set_velocity(self._h, om), "efem_set_velocity")

    def set_coords(self, X):
        """Replace the reference coordinates (float64 [n_nodes, 3] device tensor),
        keeping connectivity and blocks."""
        self._sync_stream()
        X = self._nodal(X, name="X")
        L.check(self._lib.efem_set_coords(self._h, _ptr(X)), "efem_set_coords")
        self.X = X.clone()
        self._lin = None

    def set_dirichlet(self, mask):
        """mask: uint8 tensor [3*n_nodes] (1 = prescribed) or None."""
        self._sync_stream()
        if mask is None:
            L.check(self._lib.efem_set_dirichlet(self._h, None), "efem_set_dirichlet")
            self._mask = None
            return
        self._mask = self._nodal(mask, torch.uint8, "mask")
        L.check(self._lib.efem_set_dirichlet(self._h, _ptr(self._mask)), "efem_set_dirichlet")

    @property
    def mask(self):
        """The Dirichlet mask in force (uint8 [3*n_nodes]), or None."""
        return getattr(self, "_mask", None)

    @contextlib.contextmanager
    def unmasked(self):
        """Temporarily remove the Dirichlet mask; the mask in force on entry
        (if any) is put back on exit."""
        mask = self.mask
        if mask is None:
            yield self
            return
        self.set_dirichlet(None)
        try:
            yield self
        finally:
            self.set_dirichlet(mask)

    def set_load(self, f):
        """External nodal forces of the final load step (float64 [n_nodes, 3] or
        [3*n_nodes]) for ``newton_solve``, or None to remove them."""
        self._sync_stream()
        if f is None:
            L.check(self._lib.efem_set_load(self._h, None), "efem_set_load")
            return
        self._load = self._nodal(f, torch.float64, "load")
        L.check(self._lib.efem_set_load(self._h, _ptr(self._load)), "efem_set_load")

    def info(self):
        i = L.Info()
        L.check(self._lib.efem_get_info(self._h, ctypes.byref(i)), "efem_get_info")
        return {k: getattr(i, k) for k, _ in L.Info._fields_}

    def status(self):
        self._sync_stream()
        f = ctypes.c_int32()
        L.check(self._lib.efem_status(self._h, ctypes.byref(f)), "efem_status")
        return f.value

    # ------------------------------------------------------------ operators
    def energy(self, u, out=None):
        """Psi_h(u), Eq. (2), as a 0-d float64 device tensor."""
        self._sync_stream()
        out = torch.empty((), dtype=torch.float64, device=self.device) if out is None else out
        L.check(self._lib.efem_energy(self._h, _ptr(self._nodal(u, name="u")), _ptr(out)),
                "efem_energy")
        return out

    def residual(self, u, out=None):
        """r = grad Psi_h(u), Eq. (1)."""
        self._sync_stream()
        out = self._new_nodal() if out is None else self._nodal(out, name="out")
        L.check(self._lib.efem_residual(self._h, _ptr(self._nodal(u, name="u")), _ptr(out)),
                "efem_residual")
        return out

    def linearize(self, u, prec="f64"):
        self._sync_stream()
        p = _PREC[prec]
        L.check(self._lib.efem_linearize(self._h, _ptr(self._nodal(u, name="u")), p),
                "efem_linearize")
        self._lin = torch.float64 if p == L.EFEM_F64 else torch.float32

    def hvp(self, v, out=None):
        """y = K(u) v, Eq. (3), at the last linearization point."""
        self._sync_stream()
        if self._lin is None:
            raise RuntimeError("call linearize(u) first")
        out = self._new_nodal(self._lin) if out is None else self._nodal(out, self._lin, "out")
        L.check(self._lib.efem_hvp(self._h, _ptr(self._nodal(v, self._lin, "v")), _ptr(out)),
                "efem_hvp")
        return out

    def hvp_acc(self, v, out):
        """out += K(u) v in one kernel launch."""
        self._sync_stream()
        if self._lin is None:
            raise RuntimeError("call linearize(u) first")
        L.check(self._lib.efem_hvp_acc(self._h, _ptr(self._nodal(v, self._lin, "v")),
                                       _ptr(self._nodal(out, self._lin, "out"))), "efem_hvp_acc")
        return out

    def hvp_zeroed(self, v, out):
        """out = K(u) v in one kernel launch; ``out`` must hold zeros on entry."""
        self._sync_stream()
        if self._lin is None:
            raise RuntimeError("call linearize(u) first")
        L.check(self._lib.efem_hvp_zeroed(self._h, _ptr(self._nodal(v, self._lin, "v")),
                                          _ptr(self._nodal(out, self._lin, "out"))), "efem_hvp_zeroed")
        return out

    def jacobi_diag(self, u, out=None):
        self._sync_stream()
        out = self._new_nodal() if out is None else self._nodal(out, name="out")
        L.check(self._lib.efem_jacobi_diag(self._h, _ptr(self._nodal(u, name="u")), _ptr(out)),
                "efem_jacobi_diag")
        return out

    def jacobi_offdiag(self, u, out=None):
        """(K01, K02, K12) of every node's 3x3 diagonal block of K(u), float64
        [n_nodes, 3], the mask not applied (the block-Jacobi preconditioner's
        blocks with jacobi_diag)."""
        self._sync_stream()
        out = self._new_nodal() if out is None else self._nodal(out, name="out")
        L.check(self._lib.efem_jacobi_offdiag(self._h, _ptr(self._nodal(u, name="u")), _ptr(out)),
                "efem_jacobi_offdiag")
        return out

    def grad_material(self, u):
        self._sync_stream()
        dmu = torch.empty(self.n_elems, dtype=torch.float64, device=self.device)
        dlam = torch.empty_like(dmu)
        L.check(self._lib.efem_grad_material(self._h, _ptr(self._nodal(u, name="u")), _ptr(dmu),
                                             _ptr(dlam)), "efem_grad_material")
        return dmu, dlam

    def residual_vjp_material(self, u, w):
        self._sync_stream()
        dmu = torch.empty(self.n_elems, dtype=torch.float64, device=self.device)
        dlam = torch.empty_like(dmu)
        L.check(self._lib.efem_residual_vjp_material(self._h, _ptr(self._nodal(u, name="u")),
                                                     _ptr(self._nodal(w, name="w")), _ptr(dmu),
                                                     _ptr(dlam)), "efem_residual_vjp_material")
        return dmu, dlam

    def grad_coords(self, u, out=None):
        self._sync_stream()
        out = self._new_nodal() if out is None else self._nodal(out, name="out")
        L.check(self._lib.efem_grad_coords(self._h, _ptr(self._nodal(u, name="u")), _ptr(out)),
                "efem_grad_coords")
        return out


    # -------------------------------------------------------------- solver
    def newton_solve(self, u, u_bc, **opts):
        """Matrix-free Newton-Krylov solve (Sec. 6.3.1) of the reduced
        functional; needs set_dirichlet.  ``u`` (float64 [n_nodes, 3]) is
        updated in place.  Keyword options are the fields of efem_solve_opts
        (``hvp_prec`` accepts "f64"/"f32").  Returns (return code, stats dict)."""
        self._sync_stream()
        o = L.SolveOpts()
        self._lib.efem_solve_opts_default(ctypes.byref(o))
        for k, v in opts.items():
            if k == "hvp_prec":
                v = _PREC[v]
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        st = L.SolveStats()
        rc = L.check(self._lib.efem_newton_solve(self._h, _ptr(self._nodal(u, name="u")),
                                                 _ptr(self._nodal(u_bc, name="u_bc")),
                                                 ctypes.byref(o), ctypes.byref(st)),
                     "efem_newton_solve")
        k = st.steps_done
        stats = {f: getattr(st, f) for f, _ in L.SolveStats._fields_
                 if f not in ("newton_per_step", "cg_per_step")}
        stats["newton_per_step"] = list(st.newton_per_step[:min(k, 64)])
        stats["cg_per_step"] = list(st.cg_per_step[:min(k, 64)])
        return rc, stats


    # ------------------------------------------------------ sparse tangent
    def sparse_setup(self):
        """Pattern and distance-2 colouring of K (Alg. 2); returns the info dict."""
        self._sync_stream()
        i = L.SparseInfo()
        L.check(self._lib.efem_sparse_setup(self._h, ctypes.byref(i)), "efem_sparse_setup")
        self._sparse = {k: getattr(i, k) for k, _ in L.SparseInfo._fields_}
        return dict(self._sparse)

    def sparse_pattern(self):
        """(row_ptr int64 [n_rows+1], col int32 [nnz], dof_colour int32 [n_rows])."""
        info = self._sparse if getattr(self, "_sparse", None) else self.sparse_setup()
        rp = torch.empty(info["n_rows"] + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(info["nnz"], dtype=torch.int32, device=self.device)
        dc = torch.empty(info["n_rows"], dtype=torch.int32, device=self.device)
        L.check(self._lib.efem_sparse_pattern(self._h, _ptr(rp), _ptr(col), _ptr(dc)), "efem_sparse_pattern")
        return rp, col, dc

    def sparse_block_pattern(self):
        """(block_ptr int64 [n_nodes+1], block_col int32 [n_blocks]): the
        pattern by 3x3 blocks, the layout the SpMV reads."""
        info = self._sparse if getattr(self, "_sparse", None) else self.sparse_setup()
        bp = torch.empty(info["n_rows"] // 3 + 1, dtype=torch.int64, device=self.device)
        bc = torch.empty(info["n_blocks"], dtype=torch.int32, device=self.device)
        L.check(self._lib.efem_sparse_block_pattern(self._h, _ptr(bp), _ptr(bc)), "efem_sparse_block_pattern")
        return bp, bc

    def sparse_assemble(self, u, values=None):
        """K(u) values (float64 [nnz], pattern order) from n_colours tangent actions."""
        info = self._sparse if getattr(self, "_sparse", None) else self.sparse_setup()
        if values is None:
            values = torch.empty(info["nnz"], dtype=torch.float64, device=self.device)
        L.check(self._lib.efem_sparse_assemble(self._h, _ptr(self._nodal(u, name="u")), _ptr(values)),
                "efem_sparse_assemble")
        self._lin = torch.float64
        return values

    def sparse_spmv(self, values, x, out=None):
        """y = K x with assembled values, by 3x3 blocks."""
        self._sync_stream()
        out = self._new_nodal() if out is None else self._nodal(out, name="out")
        L.check(self._lib.efem_sparse_spmv(self._h, _ptr(values), _ptr(self._nodal(x, name="x")), _ptr(out)),
                "efem_sparse_spmv")
        return out

    def linear_solve(self, u, b, rtol=1e-8, hvp_prec="f64", precond=0, max_iter=100000):
        """Solve K(u)_ff x = b by preconditioned CG (precond 0 Jacobi, 1 the
        learned preconditioner with flexible CG, 2 3x3 block Jacobi); returns
        (x, iterations, fell_back)."""
        self._sync_stream()
        x = self._new_nodal()
        it, fb = ctypes.c_int32(), ctypes.c_int32()
        L.check(self._lib.efem_linear_solve(self._h, _ptr(self._nodal(u, name="u")),
                                            _ptr(self._nodal(b, name="b")), _ptr(x), float(rtol),
                                            _PREC[hvp_prec], int(precond), int(max_iter),
                                            ctypes.byref(it), ctypes.byref(fb)), "efem_linear_solve")
        return x, it.value, bool(fb.value)

    def gmres_solve(self, u, b, rtol=1e-8, hvp_prec="f64", restart=30, max_iter=100000):
        """Solve K(u)_ff x = b by restarted GMRES with right Jacobi
        preconditioning; returns (x, iterations, relative residual, converged)."""
        self._sync_stream()
        x = self._new_nodal()
        it, rr = ctypes.c_int32(), ctypes.c_double()
        rc = L.check(self._lib.efem_gmres_solve(self._h, _ptr(self._nodal(u, name="u")),
                                                _ptr(self._nodal(b, name="b")), _ptr(x), float(rtol),
                                                _PREC[hvp_prec], int(restart), int(max_iter),
                                                ctypes.byref(it), ctypes.byref(rr)), "efem_gmres_solve")
        return x, it.value, rr.value, rc == L.EFEM_OK

    # ------------------------------------------------- learned preconditioner
    def set_mlp(self, params):
        """params: float32 device tensor [EFEM_MLP_PARAMS], or None to remove."""
        self._sync_stream()
        if params is None:
            L.check(self._lib.efem_set_mlp(self._h, None), "efem_set_mlp")
            return
        if params.dtype != torch.float32 or params.numel() != L.EFEM_MLP_PARAMS or params.device != self.device:
            raise TypeError("params must be a float32 device tensor of EFEM_MLP_PARAMS entries")
        L.check(self._lib.efem_set_mlp(self._h, _ptr(params.contiguous())), "efem_set_mlp")

    def precond_apply(self, r, diag):
        self._sync_stream()
        z = self._new_nodal(torch.float32)
        L.check(self._lib.efem_precond_apply(self._h, _ptr(self._nodal(r, torch.float32, "r")),
                                             _ptr(self._nodal(diag, name="diag")), _ptr(z)),
                "efem_precond_apply")
        return z

    def precond_rows(self, b, diag, t, n_total, X=None, aux=None):
        """Training rows of one (b, t) pair: X uint16 [n_nodes, 16] (bfloat16 bits),
        aux float32 [n_nodes, EFEM_MLP_AUX]."""
        self._sync_stream()
        if X is None:
            X = torch.empty((self.n_nodes, 16), dtype=torch.int16, device=self.device)
        if aux is None:
            aux = torch.empty((self.n_nodes, L.EFEM_MLP_AUX), dtype=torch.float32, device=self.device)
        assert X.numel() == 16 * self.n_nodes and aux.numel() == L.EFEM_MLP_AUX * self.n_nodes
        L.check(self._lib.efem_precond_rows(self._h, _ptr(self._nodal(b, torch.float32, "b")),
                                            _ptr(self._nodal(diag, name="diag")),
                                            _ptr(self._nodal(t, torch.float32, "t")), float(n_total),
                                            _ptr(X), _ptr(aux)), "efem_precond_rows")
        return X, aux

    def mlp_forward(self, X):
        self._sync_stream()
        rows = X.shape[0]
        out = torch.empty((rows, 3), dtype=torch.float32, device=self.device)
        L.check(self._lib.efem_mlp_forward(self._h, rows, _ptr(X.contiguous()), _ptr(out)),
                "efem_mlp_forward")
        return out

    def mlp_forward_layers(self, X):
        """(h1, h2, out): both hidden layers' bf16 activations as int16 bit
        patterns [rows, 64] and the output [rows, 3]."""
        self._sync_stream()
        rows = X.shape[0]
        h1 = torch.empty((rows, L.EFEM_MLP_HID), dtype=torch.int16, device=self.device)
        h2 = torch.empty_like(h1)
        out = torch.empty((rows, 3), dtype=torch.float32, device=self.device)
        L.check(self._lib.efem_mlp_forward_layers(self._h, rows, _ptr(X.contiguous()), _ptr(h1), _ptr(h2),
                                                  _ptr(out)), "efem_mlp_forward_layers")
        return h1, h2, out

    def mlp_loss_grad(self, X, aux, params, grad=None, loss=None):
        self._sync_stream()
        grad = torch.empty(L.EFEM_MLP_PARAMS, dtype=torch.float32, device=self.device) if grad is None else grad
        loss = torch.empty((), dtype=torch.float64, device=self.device) if loss is None else loss
        L.check(self._lib.efem_mlp_loss_grad(self._h, X.shape[0], _ptr(X), _ptr(aux), _ptr(params),
                                             _ptr(grad), _ptr(loss)), "efem_mlp_loss_grad")
        return grad, loss

    def mlp_energy_rows(self, r, out, n_samples, aux, z, kz, energy):
        """One sample of the energy-norm objective at the current FP32
        linearization: fills z, kz, the rows' weights and pseudo-targets in aux,
        and adds the sample's energy term into the device scalar ``energy``."""
        self._sync_stream()
        L.check(self._lib.efem_mlp_energy_rows(self._h, _ptr(self._nodal(r, torch.float32, "r")),
                                               _ptr(out), float(n_samples), _ptr(aux),
                                               _ptr(self._nodal(z, torch.float32, "z")),
                                               _ptr(self._nodal(kz, torch.float32, "kz")), _ptr(energy)),
                "efem_mlp_energy_rows")

    def cg_snapshots(self, u, b, iters, sign=1.0, R=None):
        """Residuals of FP32 Jacobi-PCG on K(u)_ff x = sign b after each of
        ``iters`` iterations: (R float32 [len(iters), n_nodes, 3], number reached)."""
        self._sync_stream()
        its = (ctypes.c_int32 * len(iters))(*[int(i) for i in iters])
        if R is None:
            R = torch.empty((len(iters), self.n_nodes, 3), dtype=torch.float32, device=self.device)
        taken = ctypes.c_int32()
        L.check(self._lib.efem_cg_snapshots(self._h, _ptr(self._nodal(u, name="u")),
                                            _ptr(self._nodal(b, name="b")), float(sign), len(iters),
                                            its, _ptr(R), ctypes.byref(taken)), "efem_cg_snapshots")
        return R, taken.value

    def mlp_adam(self, params, m, v, grad, lr, t):
        self._sync_stream()
        L.check(self._lib.efem_mlp_adam(self._h, _ptr(params), _ptr(m), _ptr(v), _ptr(grad),
                                        float(lr), int(t)), "efem_mlp_adam")


# --------------------------------------------------------------- autograd

class EnergyFn(torch.autograd.Function):
    """Psi(u; mu, lam, X) with the hand-written adjoints as its backward:
    dPsi/du = r (residual kernel, without the Dirichlet mask: Psi depends on
    every DOF), dPsi/dmu, dPsi/dlam (material kernel), dPsi/dX at fixed nodal u
    (coordinate kernel).  When ``X`` is not the operator's current coordinate
    tensor, the operator is moved to ``X`` (set_coords) first."""

    @staticmethod
    def forward(ctx, u, mu, lam, X, op: Operator):
        _use_coords(op, X)
        op.set_material(mu.contiguous(), lam.contiguous())
        ctx.op = op
        ctx.save_for_backward(u, mu, lam, X)
        return op.energy(u.contiguous()).clone()

    @staticmethod
    def backward(ctx, g):
        u, mu, lam, X = ctx.saved_tensors
        op = ctx.op
        _use_coords(op, X)
        op.set_material(mu.contiguous(), lam.contiguous())
        uc = u.contiguous()
        du = dmu = dlam = dX = None
        if ctx.needs_input_grad[0]:
            with op.unmasked():
                du = (g * op.residual(uc)).reshape(u.shape)
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            gm, gl = op.grad_material(uc)
            dmu, dlam = g * gm, g * gl
        if ctx.needs_input_grad[3]:
            dX = (g * op.grad_coords(uc)).reshape(X.shape)
        return du, dmu, dlam, dX, None


def _use_coords(op: Operator, X):
    """Point the operator at the coordinates X (float64 [n_nodes, 3] device
    tensor) unless it already uses them."""
    if X is op.X:
        return
    Xc = X.detach().reshape(op.n_nodes, 3).contiguous()
    if not torch.equal(Xc, op.X):
        op.set_coords(Xc)


class ResidualFn(torch.autograd.Function):
    """r(u; mu, lam) with backward(w) = (K(u) w, w.dr/dmu, w.dr/dlam): the
    forward-over-adjoint tangent kernel and the residual's material VJP.

    With a Dirichlet mask the forward is the reduced residual P r(u) (rows of
    prescribed DOFs zero, Sec. 6.1's condensation), so its exact VJP is
    K(u) P w and (P w).dr/dm: the cotangent's prescribed components are
    dropped, and the tangent action runs without the mask so that the rows of
    prescribed DOFs keep their coupling to the free ones."""

    @staticmethod
    def forward(ctx, u, mu, lam, op: Operator):
        op.set_material(mu.contiguous(), lam.contiguous())
        ctx.op = op
        mask = op.mask
        ctx.save_for_backward(u, mu, lam, mask if mask is not None else torch.empty(0))
        ctx.masked = mask is not None
        return op.residual(u.contiguous()).reshape(u.shape)

    @staticmethod
    def backward(ctx, w):
        u, mu, lam, mask = ctx.saved_tensors
        op = ctx.op
        op.set_material(mu.contiguous(), lam.contiguous())
        uc = u.contiguous()
        wc = w.reshape(-1, 3).contiguous()
        if ctx.masked:
            # P w: the reduced residual does not depend on its prescribed rows
            wc = wc.masked_fill(mask.reshape(-1, 3).bool(), 0.0)
        du = dmu = dlam = None
        with op.unmasked():
            if ctx.needs_input_grad[0]:
                op.linearize(uc, "f64")
                du = op.hvp(wc).reshape(u.shape)
            if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
                dmu, dlam = op.residual_vjp_material(uc, wc)
        return du, dmu, dlam, None


def energy(op, u, mu, lam, X=None):
    return EnergyFn.apply(u, mu, lam, op.X if X is None else X, op)


def residual(op, u, mu, lam):
    return ResidualFn.apply(u, mu, lam, op)
