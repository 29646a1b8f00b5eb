"""Pins of the oracle's Newton-CG iteration (the matrix-free Newton-Krylov
solve of Sec. 6.3.1, with the readings listed in the oracle's docstring)."""
import numpy as np

from oracle import fem as F
from paper_2602_12365_amd import inputs as I


def setup(n, dz, elem=I.TET4, mu_sigma=0.0):
    m = I.make_mesh(elem, n)
    mu = np.ones(m.n_elems) if mu_sigma == 0 else I.lognormal_field(m.n_elems, mu_sigma, 3)
    lam = 1.5 * np.ones(m.n_elems) if mu_sigma == 0 else 1.5 * mu
    f = F.FEM(elem, m.X, m.conn, mu, lam)
    mask, ubc = I.clamp_top_bottom(m.X, dz)
    return m, f, mask, ubc


def dense_lu_newton(f, mask, ubc, n_steps, tol=1e-12):
    """Textbook full Newton with dense LU (numpy.linalg.solve) on the free DOFs."""
    mask = mask.reshape(-1)
    free = np.nonzero(mask == 0)[0]
    n = 3 * f.n_nodes
    u = np.zeros(n)
    for k in range(1, n_steps + 1):
        u[mask != 0] = (k / n_steps) * ubc.reshape(-1)[mask != 0]
        for _ in range(50):
            r = f.residual(u).ravel()[free]
            if np.linalg.norm(r) < tol:
                break
            K = np.empty((len(free), len(free)))
            for j, dof in enumerate(free):
                e = np.zeros(n)
                e[dof] = 1.0
                K[:, j] = f.hvp(u, e).ravel()[free]
            u[free] -= np.linalg.solve(K, r)
    return u.reshape(-1, 3)


def test_newton_matches_dense_lu_newton():
    m, f, mask, ubc = setup(3, 0.1)
    opts = F.SolveOptions(n_steps=2, rtol=1e-12, eta_fixed=1e-12)
    u, st = F.newton_solve(f, mask, ubc, opts)
    assert st.converged
    ref = dense_lu_newton(f, mask, ubc, 2)
    assert np.linalg.norm(u - ref) <= 1e-9 * np.linalg.norm(ref)


def test_newton_quadratic_convergence_with_exact_solves():
    m, f, mask, ubc = setup(4, 0.15)
    opts = F.SolveOptions(n_steps=1, rtol=1e-13, eta_fixed=1e-13)
    _, st = F.newton_solve(f, mask, ubc, opts)
    h = st.residual_history[0]
    # once in the basin, ||r_{k+1}|| <= C ||r_k||^2 with a moderate C
    ratios = [h[i + 1] / h[i] ** 2 for i in range(len(h) - 1) if h[i] < 1e-2 and h[i + 1] > 1e-13]
    assert len(ratios) >= 1
    assert max(ratios) < 1e3


def test_cfg1_newton_cg_converges_monotone():
    """8^3 Kuhn mesh, bottom clamped, top +0.1 z in 5 steps, Jacobi PCG, 1e-8."""
    m, f, mask, ubc = setup(8, 0.1)
    u, st = F.newton_solve(f, mask, ubc, F.SolveOptions(n_steps=5))
    assert st.converged
    free = mask.reshape(-1) == 0
    for hist, eh in zip(st.residual_history, st.energy_history):
        assert hist[-1] <= 1e-8 * hist[0] + 1e-14 * max(1, hist[0])
        assert all(b <= a + 64 * 2.2205e-16 * abs(a) for a, b in zip(eh, eh[1:]))   # Armijo descent
    r = f.residual(u).ravel()[free]
    assert np.linalg.norm(r) <= 1e-8 * st.residual_history[-1][0] * 1.0001
    # prescribed DOFs hold their final values
    assert np.array_equal(u.ravel()[~free], ubc.ravel()[~free])
    # reaction: total z-force on the top face equals minus that on the bottom face
    rr = f.residual(u)
    top = I.face_nodes(m.X, 2, 1.0)
    bot = I.face_nodes(m.X, 2, 0.0)
    assert abs(rr[top, 2].sum() + rr[bot, 2].sum()) <= 1e-7 * abs(rr[top, 2].sum())


def test_compression_needs_predictor_and_converges():
    """Hex mesh under 20% compression in 10 steps: the tangent predictor keeps
    the top element layer from inverting."""
    m, f, mask, ubc = setup(4, -0.2, elem=I.HEX8, mu_sigma=0.5)
    u, st = F.newton_solve(f, mask, ubc, F.SolveOptions(n_steps=10))
    assert st.converged
    assert np.isfinite(f.energy(u))


def test_predictor_solves_each_linear_load_step():
    """With the linear-elastic density the tangent is constant, so a load
    step's tangent predictor (K_ff d_f = -(K dc)_f, CG to predictor_rtol)
    lands on that step's solution: the step starts from the predictor solve's
    own CG residual, at most predictor_rtol times its right-hand side.  From
    a solved previous step that right-hand side is the residual the plain lift
    u + dc would leave, the same for every step (equal increments, constant
    K).  Without the predictor the step would start at the plain lift's
    residual; with the sign of its right-hand side flipped, at about twice
    that."""
    m = I.make_mesh(I.TET4, 4)
    mu = I.lognormal_field(m.n_elems, 0.3, 3)
    f = F.FEM(I.TET4, m.X, m.conn, mu, 1.5 * mu, "linear")
    mask, ubc = I.clamp_top_bottom(m.X, 0.1)
    opts = F.SolveOptions(n_steps=3)
    _, st = F.newton_solve(f, mask, ubc, opts)
    assert st.converged
    free = mask.reshape(-1) == 0
    lift = np.zeros(3 * m.n_nodes)
    lift[~free] = ubc.reshape(-1)[~free] / opts.n_steps       # step 1's plain lift from u = 0
    r_lift = np.linalg.norm(f.residual(lift.reshape(-1, 3)).ravel()[free])
    assert r_lift > 0.0
    for hist in st.residual_history:
        assert hist[0] <= opts.predictor_rtol * r_lift * 1.001 + 1e-12


def test_eisenstat_walker_forcing_gives_superlinear_steps():
    """Choice 2 of Eisenstat and Walker sets the forcing term from the square
    of the last residual ratio, so the CG tolerance tightens as Newton
    converges and the iteration turns superlinear (the exact-solve limit is
    pinned quadratic above).  On the cfg1 case every load step converges
    within 8 iterations, and in each step some iteration cuts the residual by
    at least 100x.  A forcing term held at eta_max = 0.5 converges linearly,
    by about half per iteration, and would need some 27 iterations per step."""
    m, f, mask, ubc = setup(8, 0.1)
    _, st = F.newton_solve(f, mask, ubc, F.SolveOptions(n_steps=5))
    assert st.converged
    for nit, hist in zip(st.newton_iters, st.residual_history):
        assert nit <= 8
        assert min(b / a for a, b in zip(hist, hist[1:])) <= 1e-2
