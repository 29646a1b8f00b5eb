"""efem_energy_noalloc: the energy with its per-block partials in the library's
static device array, for callers that cannot allocate.  It runs the kernels of
efem_energy in the same order, so the two agree bitwise; two calls in a row,
the second on a smaller mesh, show that the array's previous contents never
leak into a result.  The energy itself is checked against the oracle (Eq. 2,
relative 1e-12)."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import fem as F
from paper_2602_12365_amd import inputs as I

pytestmark = pytest.mark.gpu


def _energy_pair(op, u):
    """(efem_energy, efem_energy_noalloc) of u through the C-ABI."""
    lib = op._lib
    ud = torch.as_tensor(np.ascontiguousarray(u)).to("cuda")
    a = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    b = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    assert lib.efem_energy(op._h, ctypes.c_void_p(ud.data_ptr()), ctypes.c_void_p(a.data_ptr())) == 0
    rc = lib.efem_energy_noalloc(op._h, ctypes.c_void_p(ud.data_ptr()), ctypes.c_void_p(b.data_ptr()))
    assert rc == 0, lib.efem_last_error()
    torch.cuda.synchronize()
    return float(a.cpu()[0]), float(b.cpu()[0])


@pytest.mark.parametrize("elem,n_big,n_small,opts", [
    (I.TET4, 12, 3, dict(block_elems=64)),
    (I.HEX8, 10, 2, dict(block_elems=16)),
])
def test_noalloc_energy_matches_energy_on_two_calls(elem, n_big, n_small, opts):
    from paper_2602_12365_amd import Operator
    for n in (n_big, n_small):          # the second call on fewer blocks
        print(f"\n[no-alloc] elem={elem} n={n} opts={opts}", flush=True)
        m = I.make_mesh(elem, n)
        mu = I.lognormal_field(m.n_elems, 0.3, 3)
        op = Operator(elem, m.X, m.conn, **opts)
        op.set_material(torch.as_tensor(mu).cuda(), torch.as_tensor(1.5 * mu).cuda())
        u = I.gaussian_field(m.n_nodes, 0.01, n)
        e, e_na = _energy_pair(op, u)
        assert e_na == e                     # bitwise: same kernels, same order
        ref = F.FEM(elem, m.X, m.conn, mu, 1.5 * mu).energy(u)
        assert abs(e_na - ref) <= 1e-12 * abs(ref)
        op.close()


def test_noalloc_energy_rejects_too_many_blocks():
    """More element blocks than the static array holds partials: a clear
    error before any launch."""
    from paper_2602_12365_amd import Operator
    from paper_2602_12365_amd import _lib as L
    m = I.tet_mesh(23)                      # 73,002 tets, one block each
    op = Operator(I.TET4, m.X, m.conn, block_elems=1)
    assert op.info()["n_blocks"] > 65536
    u = torch.zeros((m.n_nodes, 3), dtype=torch.float64, device="cuda")
    psi = torch.zeros(1, dtype=torch.float64, device="cuda")
    rc = op._lib.efem_energy_noalloc(op._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(psi.data_ptr()))
    assert rc == L.EFEM_ERR_INVALID
    assert b"65536" in L.load().efem_last_error()
    op.close()
