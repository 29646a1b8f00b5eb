"""GPU parity: every operator of the C-ABI against the FP64 oracle, element by
element, on the same seeded inputs.

Tolerances (relative to the largest magnitude of the oracle's output):
energy 1e-12, residual / tangent action / diagonal / adjoints in FP64 1e-10;
the FP32 tangent action 5e-5 (derived from FP32 rounding of the element
geometry: float32 coordinates carry ~6e-8 relative error, amplified by the
inverse element Jacobian and a few hundred operations).
"""
import numpy as np
import pytest
import torch

from oracle import fem as F
from paper_2602_12365_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL_E, TOL64, TOL32 = 1e-12, 1e-10, 5e-5

CASES = [
    ("tet_1", I.TET4, 1, {}),
    ("tet_3_small_blocks", I.TET4, 3, dict(block_elems=37, block_nodes=40)),
    ("tet_8", I.TET4, 8, {}),
    ("tet_8_color", I.TET4, 8, dict(scatter="color")),
    ("tet_8_atomic", I.TET4, 8, dict(scatter="atomic")),
    ("tet_3_small_blocks_atomic", I.TET4, 3, dict(block_elems=37, block_nodes=40, scatter="atomic")),
    ("tet_5_color_small", I.TET4, 5, dict(block_elems=100, block_nodes=64, scatter="color",
                                           threads=64)),
    ("tet_9_ragged", I.TET4, 9, dict(block_elems=301, block_nodes=97, threads=128)),
    ("tet_6_no_pairs", I.TET4, 6, dict(pairs=False)),
    ("tet_7_odd_blocks", I.TET4, 7, dict(block_elems=63, block_nodes=50)),
    ("tet_6_scrambled", I.TET4, 6, dict(scramble=11)),
    ("tet_5_scrambled_color", I.TET4, 5, dict(scramble=12, scatter="color", block_elems=200)),
    ("hex_1", I.HEX8, 1, {}),
    ("hex_3_small_blocks", I.HEX8, 3, dict(block_elems=5, block_nodes=27)),
    ("hex_6", I.HEX8, 6, {}),
    ("hex_6_color", I.HEX8, 6, dict(scatter="color")),
    ("hex_6_atomic", I.HEX8, 6, dict(scatter="atomic")),
    ("hex_7_ragged", I.HEX8, 7, dict(block_elems=45, block_nodes=100, threads=64)),
    ("hex_5_scrambled", I.HEX8, 5, dict(scramble=13)),
    ("tet_6_linear", I.TET4, 6, dict(model="linear")),
    ("tet_5_linear_small_blocks", I.TET4, 5, dict(model="linear", block_elems=37, block_nodes=40)),
    ("tet_5_linear_color", I.TET4, 5, dict(model="linear", scatter="color")),
    ("hex_5_linear", I.HEX8, 5, dict(model="linear")),
    ("hex_4_linear_atomic", I.HEX8, 4, dict(model="linear", scatter="atomic", block_elems=9)),
    ("tri_12", I.TRI3, 12, {}),
    ("tri_9_small_blocks", I.TRI3, 9, dict(block_elems=50, block_nodes=40, threads=64)),
    ("tri_10_color", I.TRI3, 10, dict(scatter="color")),
    ("tri_10_linear_atomic", I.TRI3, 10, dict(model="linear", scatter="atomic")),
    # the largest blocks: 768 distinct nodes (78 KB of LDS per workgroup)
    ("tet_10_max_blocks", I.TET4, 10, dict(block_elems=100000, block_nodes=768)),
    ("hex_10_max_blocks", I.HEX8, 10, dict(block_elems=100000, block_nodes=768, scatter="color")),
    ("tri_40_max_blocks", I.TRI3, 40, dict(block_elems=100000, block_nodes=768)),
]


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


class Case:
    def __init__(self, elem, n, opts, mu_sigma=0.3):
        from paper_2602_12365_amd import Operator
        opts = dict(opts)
        scramble = opts.pop("scramble", None)
        model = opts.get("model", "neo_hookean")
        self.mesh = I.make_mesh(elem, n)
        if scramble is not None:
            self.mesh = I.scrambled_mesh(self.mesh, scramble)
        m = self.mesh
        self.mu = I.lognormal_field(m.n_elems, mu_sigma, 3)
        self.lam = 1.5 * self.mu
        self.u = I.gaussian_field(m.n_nodes, min(I.cube_amplitude(n), 0.05), 0)
        self.v = I.unit_direction(m.n_nodes, 1)
        self.w = I.unit_direction(m.n_nodes, 2)
        self.orc = F.FEM(elem, m.X, m.conn, self.mu, self.lam, model)
        self.op = Operator(elem, m.X, m.conn, **opts)
        self.op.set_material(dev(self.mu), dev(self.lam))


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    _, elem, n, opts = request.param
    print(f"\n[parity case] {request.param[0]} elem={elem} n={n} opts={opts}", flush=True)
    return Case(elem, n, opts)


def test_energy(case):
    psi = host(case.op.energy(dev(case.u)))
    ref = case.orc.energy(case.u)
    assert abs(psi - ref) <= TOL_E * abs(ref)


def test_residual(case):
    r = host(case.op.residual(dev(case.u)))
    assert rel(r, case.orc.residual(case.u)) <= TOL64


def test_hvp_f64(case):
    case.op.linearize(dev(case.u), "f64")
    y = host(case.op.hvp(dev(case.v)))
    assert rel(y, case.orc.hvp(case.u, case.v)) <= TOL64


def test_hvp_f32(case):
    case.op.linearize(dev(case.u), "f32")
    y = host(case.op.hvp(dev(case.v, torch.float32)))
    assert rel(y, case.orc.hvp(case.u, case.v)) <= TOL32


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hvp_single_launch_forms(case, prec):
    """efem_hvp_acc: y += K v on an arbitrary y; efem_hvp_zeroed: y = K v on a zero y
    (with and without a Dirichlet mask)."""
    dt = torch.float64 if prec == "f64" else torch.float32
    tol = TOL64 if prec == "f64" else TOL32
    ref = case.orc.hvp(case.u, case.v)
    case.op.linearize(dev(case.u), prec)
    y0 = I.unit_direction(case.mesh.n_nodes, 77)
    y = dev(y0, dt)
    got = host(case.op.hvp_acc(dev(case.v, dt), y))
    assert rel(got - y0, ref) <= tol
    z = torch.zeros((case.mesh.n_nodes, 3), dtype=dt, device="cuda")
    assert rel(host(case.op.hvp_zeroed(dev(case.v, dt), z)), ref) <= tol
    mask, _ = I.clamp_top_bottom(case.mesh.X, 0.1)
    case.op.set_dirichlet(dev(mask, torch.uint8))
    try:
        mref = F.masked(mask, case.orc.hvp(case.u, F.masked(mask, case.v)))
        z = torch.zeros((case.mesh.n_nodes, 3), dtype=dt, device="cuda")
        assert rel(host(case.op.hvp_zeroed(dev(case.v, dt), z)), mref) <= tol
        y = dev(y0, dt)
        got = host(case.op.hvp_acc(dev(case.v, dt), y))
        assert rel(got - F.masked(mask, y0), mref) <= tol
    finally:
        case.op.set_dirichlet(None)


def test_jacobi_diag(case):
    d = host(case.op.jacobi_diag(dev(case.u)))
    assert rel(d, case.orc.jacobi_diag(case.u)) <= TOL64


def test_jacobi_offdiag(case):
    """Off-diagonal entries of the nodes' 3x3 diagonal blocks of K (the
    block-Jacobi preconditioner) against the oracle's assembled tangent."""
    o = host(case.op.jacobi_offdiag(dev(case.u)))
    ref = case.orc.jacobi_offdiag(case.u)
    scale = np.abs(case.orc.jacobi_diag(case.u)).max()
    assert np.abs(o - ref).max() <= TOL64 * scale


def test_grad_material(case):
    gm, gl = case.op.grad_material(dev(case.u))
    rm, rl = case.orc.grad_material(case.u)
    assert rel(host(gm), rm) <= TOL64
    assert rel(host(gl), rl) <= TOL64


def test_residual_vjp_material(case):
    gm, gl = case.op.residual_vjp_material(dev(case.u), dev(case.w))
    rm, rl = case.orc.residual_vjp_material(case.u, case.w)
    assert rel(host(gm), rm) <= TOL64
    assert rel(host(gl), rl) <= TOL64


def test_grad_coords(case):
    g = host(case.op.grad_coords(dev(case.u)))
    assert rel(g, case.orc.grad_coords(case.u)) <= TOL64


def test_dirichlet_reduced_functional(case):
    m = case.mesh
    if m.elem == I.TRI3:
        mask, _ = I.clamp_planar(m.X, 0.1)
    else:
        mask, _ = I.clamp_top_bottom(m.X, 0.1)
    op = case.op
    op.set_dirichlet(dev(mask, torch.uint8))
    try:
        fixed = mask.reshape(-1, 3) != 0
        r = host(op.residual(dev(case.u)))
        assert rel(r, F.masked(mask, case.orc.residual(case.u))) <= TOL64
        op.linearize(dev(case.u), "f64")
        y = host(op.hvp(dev(case.v)))
        ref = F.masked(mask, case.orc.hvp(case.u, F.masked(mask, case.v)))
        assert rel(y, ref) <= TOL64
        d = host(op.jacobi_diag(dev(case.u)))
        dref = case.orc.jacobi_diag(case.u)
        dref[fixed] = 1.0
        assert rel(d, dref) <= TOL64
        assert np.all(r[fixed] == 0.0) and np.all(y[fixed] == 0.0)
    finally:
        op.set_dirichlet(None)


def test_repeat_calls(case):
    """The energy is bitwise deterministic (no atomics: block partials summed in
    block order); nodal sums use atomics and agree to rounding."""
    u = dev(case.u)
    e1, e2 = host(case.op.energy(u)), host(case.op.energy(u))
    assert e1 == e2
    case.op.linearize(u, "f64")
    y1 = host(case.op.hvp(dev(case.v)))
    y2 = host(case.op.hvp(dev(case.v)))
    assert rel(y1, y2) <= 1e-14


@pytest.mark.parametrize("stretch", [(2.5, 0.6, 1.3), (0.5, 0.7, 0.9)], ids=["J1.95", "J0.315"])
def test_large_strain(case, stretch):
    """Affine stretches plus small noise: det F far from 1 on both sides (the
    logarithm's exponent split)."""
    m = case.mesh
    u = (m.X - 0.5) * (np.asarray(stretch) - 1.0)
    u = u + I.gaussian_field(m.n_nodes, 1e-3 / m.n, 5)
    psi = host(case.op.energy(dev(u)))
    ref = case.orc.energy(u)
    assert abs(psi - ref) <= TOL_E * abs(ref)
    assert rel(host(case.op.residual(dev(u))), case.orc.residual(u)) <= TOL64
    case.op.linearize(dev(u), "f64")
    assert rel(host(case.op.hvp(dev(case.v))), case.orc.hvp(u, case.v)) <= TOL64
    assert rel(host(case.op.jacobi_diag(dev(u))), case.orc.jacobi_diag(u)) <= TOL64


def test_work_items(case):
    """Face-sharing tetrahedra are paired into work items (a maximal matching
    inside each block); one element per item without pairing or for hexahedra."""
    info = case.op.info()
    ne = case.mesh.n_elems
    assert info["n_items"] <= ne
    if case.mesh.elem in (I.HEX8, I.TRI3) or not case.op.pairs:
        assert info["n_items"] == ne
    else:
        # every element is in exactly one item and most are paired
        assert info["n_items"] >= ne // 2
        assert info["n_items"] <= 0.6 * ne + 2 * info["n_blocks"]


def test_inverted_element_flags_and_inf():
    from paper_2602_12365_amd import Operator
    m = I.tet_mesh(2)
    op = Operator(I.TET4, m.X, m.conn)
    u = np.zeros_like(m.X)
    a, b = m.conn[0, 3], m.conn[0, 0]
    u[a] = -3.0 * (m.X[a] - m.X[b])
    assert op.status() == 0
    psi = host(op.energy(dev(u)))
    assert psi == np.inf
    assert op.status() & 1
    assert op.status() == 0          # cleared by the read


def test_residual_rejects_aliased_output():
    from paper_2602_12365_amd import Operator
    from paper_2602_12365_amd import _lib as L
    m = I.tet_mesh(2)
    op = Operator(I.TET4, m.X, m.conn)
    u = dev(np.zeros_like(m.X))
    with pytest.raises(L.EfemError):
        op.residual(u, out=u)
    op.close()


def test_error_codes():
    from paper_2602_12365_amd import Operator
    from paper_2602_12365_amd import _lib as L
    m = I.tet_mesh(2)
    op = Operator(I.TET4, m.X, m.conn)
    with pytest.raises(RuntimeError):
        op.hvp(dev(np.zeros_like(m.X)))       # not linearized
    lib = L.load()
    assert lib.efem_hvp(op._h, None, None) == L.EFEM_ERR_INVALID
    # sizes and options the library refuses before touching the GPU
    with pytest.raises(L.EfemError):
        Operator(I.TET4, m.X, m.conn[:0])                       # no elements
    with pytest.raises(L.EfemError):
        Operator(I.TET4, m.X, m.conn, block_nodes=769)          # beyond the LDS cap
    with pytest.raises(L.EfemError):
        Operator(I.TET4, m.X, m.conn, threads=96)               # not a multiple of 64
    bad = m.conn.copy()
    bad[0, 0] = m.n_nodes                                       # node id out of range
    with pytest.raises(L.EfemError):
        Operator(I.TET4, m.X, bad)
    flipped = m.conn.copy()
    flipped[0, [1, 2]] = flipped[0, [2, 1]]                     # inverted reference element
    with pytest.raises(L.EfemError):
        Operator(I.TET4, m.X, flipped)


def test_full_size_64cube_tets():
    """64^3 Kuhn mesh (1,572,864 tets, 823,875 DOF) in the launch configuration
    the benchmark times, every output entry against the oracle."""
    from paper_2602_12365_amd import Operator
    n = 64
    m = I.tet_mesh(n)
    print(f"\n[parity case] full-size tet n={n}", flush=True)
    u = I.gaussian_field(m.n_nodes, I.cube_amplitude(n), 0)
    v = I.unit_direction(m.n_nodes, 100)
    mu, lam = np.ones(m.n_elems), 1.5 * np.ones(m.n_elems)
    orc = F.FEM(I.TET4, m.X, m.conn, mu, lam)
    for scatter in ("halo", "atomic", "color"):
        op = Operator(I.TET4, m.X, m.conn, scatter=scatter)
        assert abs(host(op.energy(dev(u))) - orc.energy(u)) <= TOL_E * orc.energy(u)
        assert rel(host(op.residual(dev(u))), orc.residual(u)) <= TOL64
        ref = orc.hvp(u, v)
        op.linearize(dev(u), "f64")
        assert rel(host(op.hvp(dev(v))), ref) <= TOL64
        op.linearize(dev(u), "f32")
        assert rel(host(op.hvp(dev(v, torch.float32))), ref) <= TOL32
        op.close()


def test_full_size_64cube_tets_linear_model():
    """The same 64^3 mesh under the small-strain linear model: every output
    entry of energy, residual and both tangent actions against the oracle."""
    from paper_2602_12365_amd import Operator
    n = 64
    m = I.tet_mesh(n)
    print(f"\n[parity case] full-size tet n={n} linear model", flush=True)
    u = I.gaussian_field(m.n_nodes, I.cube_amplitude(n), 0)
    v = I.unit_direction(m.n_nodes, 100)
    mu, lam = np.ones(m.n_elems), 1.5 * np.ones(m.n_elems)
    orc = F.FEM(I.TET4, m.X, m.conn, mu, lam, "linear")
    op = Operator(I.TET4, m.X, m.conn, model="linear")
    assert abs(host(op.energy(dev(u))) - orc.energy(u)) <= TOL_E * orc.energy(u)
    assert rel(host(op.residual(dev(u))), orc.residual(u)) <= TOL64
    ref = orc.hvp(u, v)
    op.linearize(dev(u), "f64")
    assert rel(host(op.hvp(dev(v))), ref) <= TOL64
    op.linearize(dev(u), "f32")
    assert rel(host(op.hvp(dev(v, torch.float32))), ref) <= TOL32
    op.close()


def test_model_switch_and_bad_model():
    """efem_set_model switches every operator; an unknown model is rejected."""
    from paper_2602_12365_amd import Operator
    m = I.tet_mesh(3)
    u = I.gaussian_field(m.n_nodes, 0.02, 0)
    mu, lam = np.ones(m.n_elems), 1.5 * np.ones(m.n_elems)
    op = Operator(I.TET4, m.X, m.conn)
    for model in ("linear", "neo_hookean", "linear"):
        op.set_model(model)
        orc = F.FEM(I.TET4, m.X, m.conn, mu, lam, model)
        assert abs(host(op.energy(dev(u))) - orc.energy(u)) <= TOL_E * orc.energy(u)
    with pytest.raises(ValueError):
        op.set_model("hyperelastic")
    from paper_2602_12365_amd import _lib as L
    assert op._lib.efem_set_model(op._h, 7) == L.EFEM_ERR_INVALID
    op.close()


def test_zero_state(case):
    """u = 0: the energy is exactly zero (psi(I) = 0 term by term), the residual
    vanishes to rounding, and the tangent action is the small-strain
    stiffness action (the oracle's tangent at u = 0)."""
    m = case.mesh
    z = np.zeros((m.n_nodes, 3))
    assert host(case.op.energy(dev(z))) == 0.0
    r = host(case.op.residual(dev(z)))
    scale = np.abs(case.orc.residual(case.u)).max()
    assert np.abs(r).max() <= 1e-13 * scale
    case.op.linearize(dev(z), "f64")
    assert rel(host(case.op.hvp(dev(case.v))), case.orc.hvp(z, case.v)) <= TOL64
