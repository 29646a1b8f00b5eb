"""Host check of the item deal that orders each block's items over the LDS
bank groups (csrc/api.cpp, spread_items_*): a C++ driver that includes the
library source, built with hipcc and run on the CPU (no device call)."""
import os
import subprocess

import numpy as np
import pytest

from paper_2602_12365_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2602_12365_amd")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    lib = os.path.join(PKG, "libefem.so")
    if not os.path.exists(lib):
        pytest.skip("libefem.so is not built")
    out = tmp_path_factory.mktemp("deal") / "item_deal_check"
    subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(PKG, "csrc"), os.path.join(ROOT, "tests", "item_deal_check.cpp"),
                    "-o", str(out), "-L", PKG, "-lefem", f"-Wl,-rpath,{PKG}"],
                   check=True, capture_output=True, timeout=600)
    return str(out)


# the 16^3 Tet4 mesh builds 8 chunks of 2 blocks (every block of at most 768
# items); the 10^3 one has larger blocks and takes the block pass's deal
@pytest.mark.parametrize("elem, n, chunks", [(I.TET4, 16, True), (I.TET4, 10, False), (I.HEX8, 10, False),
                                             (I.HEX8, 3, False)],
                         ids=["tet_16_chunks", "tet_10_blocks", "hex_10", "hex_3"])
def test_item_deal_keeps_items_and_spreads_banks(driver, tmp_path, elem, n, chunks):
    m = I.make_mesh(elem, n)
    path = tmp_path / "mesh.bin"
    with open(path, "wb") as f:
        np.array([m.n_nodes, m.n_elems, elem], dtype=np.int64).tofile(f)
        np.ascontiguousarray(m.X, dtype=np.float64).tofile(f)
        np.ascontiguousarray(m.conn, dtype=np.int32).tofile(f)
    res = subprocess.run([driver, str(path)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok"), res.stdout
    assert (int(res.stdout.split()[4]) > 0) == chunks, res.stdout
    print(res.stdout.strip())
