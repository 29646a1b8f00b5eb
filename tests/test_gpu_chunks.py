"""GPU parity of the chunk pass: the FP64 Tet4 tangent action with each
chunk's node records resident in LDS while its blocks stream through as steps
(Eq. 3, the matrix-free tangent action; Alg. 1's batches are the steps).

Every case has more blocks than chunks, so chunks run several steps: records
of step t+1 load while step t computes, staging words of step t+2 arrive
through LDS, Dirichlet bits are applied after the loads land.  The output is
compared with the oracle element by element (relative 1e-10 of the largest
entry) and with the block pass of the same mesh (which differs only in the
order of the FP64 sums, so 1e-13).
"""
import numpy as np
import pytest
import torch

from oracle import fem as F
from paper_2602_12365_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64 = 1e-10

# (id, hexes per edge, Operator options, scramble seed)
CASES = [
    ("tet_16_b16", 16, dict(block_elems=16), None),        # ~6 steps of 8 items
    ("tet_12_b24_ragged", 12, dict(block_elems=24), None),  # 1 or 2 steps per chunk
    ("tet_20_b100", 20, dict(block_elems=100), None),
    ("tet_24_b64_scrambled", 24, dict(block_elems=64), 21),
    ("tet_32_b192", 32, dict(block_elems=192), None),      # 4 steps of 96 items
]


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


class ChunkCase:
    def __init__(self, n, opts, scramble):
        from paper_2602_12365_amd import Operator
        m = I.tet_mesh(n)
        if scramble is not None:
            m = I.scrambled_mesh(m, scramble)
        self.mesh = m
        self.mu = I.lognormal_field(m.n_elems, 0.3, 4)
        self.lam = 1.5 * self.mu
        self.u = I.gaussian_field(m.n_nodes, I.cube_amplitude(n), 0)
        self.v = I.unit_direction(m.n_nodes, 1)
        self.op = Operator(I.TET4, m.X, m.conn, **opts)
        self.blk = Operator(I.TET4, m.X, m.conn, chunks=False, **opts)


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def cc(request):
    name, n, opts, scramble = request.param
    print(f"\n[chunk case] {name} n={n} opts={opts} scramble={scramble}", flush=True)
    c = ChunkCase(n, opts, scramble)
    yield c
    c.op.close()
    c.blk.close()


def test_chunks_have_several_steps(cc):
    info = cc.op.info()
    assert info["n_chunks"] > 0
    assert info["n_blocks"] > info["n_chunks"]
    assert 0 < info["max_chunk_slots"] <= 1472
    assert info["n_chunk_slots"] >= cc.mesh.n_nodes
    assert cc.blk.info()["n_chunks"] == 0


@pytest.mark.parametrize("material", ["uniform", "per_element"])
@pytest.mark.parametrize("masked", [False, True], ids=["free", "dirichlet"])
def test_chunk_hvp_forms(cc, material, masked):
    """y = K v, y += K v and y = K v into zeros, each against the oracle and the block pass."""
    m = cc.mesh
    if material == "uniform":
        mu, lam = np.ones(m.n_elems), 1.5 * np.ones(m.n_elems)
    else:
        mu, lam = cc.mu, cc.lam
    orc = F.FEM(I.TET4, m.X, m.conn, mu, lam)
    mask = I.clamp_top_bottom(m.X, 0.1)[0] if masked else None
    for op in (cc.op, cc.blk):
        op.set_material(dev(mu), dev(lam))
        op.set_dirichlet(dev(mask, torch.uint8) if masked else None)
        op.linearize(dev(cc.u), "f64")
    try:
        vin = F.masked(mask, cc.v) if masked else cc.v
        ref = orc.hvp(cc.u, vin)
        if masked:
            ref = F.masked(mask, ref)
        y0 = I.unit_direction(m.n_nodes, 77)
        y0m = F.masked(mask, y0) if masked else y0
        outs = {}
        for name, op in (("chunk", cc.op), ("block", cc.blk)):
            y = host(op.hvp(dev(cc.v)))
            acc = host(op.hvp_acc(dev(cc.v), dev(y0))) - y0m
            z = host(op.hvp_zeroed(dev(cc.v), torch.zeros((m.n_nodes, 3), dtype=torch.float64,
                                                          device="cuda")))
            outs[name] = (y, acc, z)
        for y, acc, z in outs.values():
            assert rel(y, ref) <= TOL64
            assert rel(acc, ref) <= TOL64
            assert rel(z, ref) <= TOL64
        for a, b in zip(outs["chunk"], outs["block"]):
            assert rel(a, b) <= 1e-13
        if masked:
            fixed = mask.reshape(-1, 3) != 0
            assert np.all(outs["chunk"][0][fixed] == 0.0)
    finally:
        for op in (cc.op, cc.blk):
            op.set_dirichlet(None)
            op.set_material(dev(cc.mu), dev(cc.lam))


def test_chunk_repeat_and_mask_toggle(cc):
    """Setting and clearing a mask rebuilds the staging words: the unmasked
    action after a masked one is the unmasked action again."""
    m = cc.mesh
    cc.op.linearize(dev(cc.u), "f64")
    y1 = host(cc.op.hvp(dev(cc.v)))
    mask = I.clamp_top_bottom(m.X, 0.1)[0]
    cc.op.set_dirichlet(dev(mask, torch.uint8))
    ym = host(cc.op.hvp(dev(cc.v)))
    cc.op.set_dirichlet(None)
    y2 = host(cc.op.hvp(dev(cc.v)))
    assert rel(y1, y2) <= 1e-14
    assert not np.allclose(ym, y1)


def test_chunk_full_size_64cube_per_element_material():
    """64^3 Kuhn mesh in the benchmark's launch configuration (256 chunks of 4
    steps of 768 pairs) with the lognormal(0, 0.3) shear modulus field of the
    adjoint case and the clamped-top Dirichlet mask: every entry of the FP64
    tangent action (and of the block pass's residual, Eq. 1) against the oracle."""
    from paper_2602_12365_amd import Operator
    n = 64
    m = I.tet_mesh(n)
    print(f"\n[chunk case] full-size tet n={n}, per-element mu, mask", flush=True)
    u = I.gaussian_field(m.n_nodes, I.cube_amplitude(n), 0)
    v = I.unit_direction(m.n_nodes, 100)
    mu = I.lognormal_field(m.n_elems, 0.3, 4)
    lam = 1.5 * np.ones(m.n_elems)
    orc = F.FEM(I.TET4, m.X, m.conn, mu, lam)
    op = Operator(I.TET4, m.X, m.conn)
    info = op.info()
    assert info["n_chunks"] > 0 and info["n_blocks"] > info["n_chunks"]
    op.set_material(dev(mu), dev(lam))
    op.linearize(dev(u), "f64")
    assert rel(host(op.hvp(dev(v))), orc.hvp(u, v)) <= TOL64
    assert rel(host(op.residual(dev(u))), orc.residual(u)) <= TOL64
    mask, _ = I.clamp_top_bottom(m.X, 0.05)
    op.set_dirichlet(dev(mask, torch.uint8))
    ref = F.masked(mask, orc.hvp(u, F.masked(mask, v)))
    assert rel(host(op.hvp(dev(v))), ref) <= TOL64
    assert rel(host(op.residual(dev(u))), F.masked(mask, orc.residual(u))) <= TOL64
    op.close()
