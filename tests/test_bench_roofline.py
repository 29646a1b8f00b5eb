"""The benchmark's roofline arithmetic for the FP64 Tet4 tangent action
(Eq. 3), checked against the figures of its committed rocprofv3 counter
summary, and that summary checked against the kernel sources it was taken
on (a stale summary would make the benchmark report its traffic as null)."""
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COUNTERS = os.path.join(ROOT, "profiles", "hvp_tet4_f64_64cube_counters.md")

# the 64^3 Kuhn mesh: 65^3 nodes, six tetrahedra per cube, every tetrahedron
# in one face pair
N64_NODES, N64_ELEMS = 65 ** 3, 6 * 64 ** 3


def _summary():
    with open(COUNTERS) as f:
        return f.read()


def test_alg_figures_by_hand():
    # one single tetrahedron: 16 bytes of connectivity, four 24-byte nodal
    # arrays over 4 nodes, and the single-tetrahedron operation count
    assert bench.tet4_hvp_alg(1, 4, 1) == (16 + 4 * 4 * 24, bench.FLOPS_PER_TET_HVP)
    # a face pair: two tetrahedra, 5 nodes, one item
    assert bench.tet4_hvp_alg(2, 5, 1) == (32 + 4 * 5 * 24, bench.FLOPS_PER_PAIR_HVP)
    # a pair and a single
    assert bench.tet4_hvp_alg(3, 6, 2)[1] == bench.FLOPS_PER_PAIR_HVP + bench.FLOPS_PER_TET_HVP
    assert bench.FLOPS_PER_PAIR_HVP < 2 * bench.FLOPS_PER_TET_HVP


def test_alg_bytes_match_the_counter_summary_64cube():
    text = _summary()
    assert f"{N64_ELEMS:,} Tet4 as {N64_ELEMS // 2:,} face pairs, {N64_NODES:,} nodes" in text
    byts, flops = bench.tet4_hvp_alg(N64_ELEMS, N64_NODES, N64_ELEMS // 2)
    row = next(l for l in text.splitlines() if l.startswith("| FP64 tangent action, chunk pass") and "| hot |" in l)
    assert int(row.rstrip(" |").split("|")[-1].strip().replace(",", "")) == byts
    assert f"{byts:,} algorithmic bytes" in text
    assert flops == (N64_ELEMS // 2) * bench.FLOPS_PER_PAIR_HVP
    # the byte time (6.4 us at 8 TB/s) exceeds the operation time (5.8 us at
    # 78.6 TFLOP/s): the action is rated against HBM
    assert bench.roofline_bound(byts, flops) == "hbm"
    assert bench.roofline_bound(byts, 10 * flops) == "alu"


def test_counter_summary_matches_the_kernel_sources():
    text = _summary()
    m = re.search(r"kernel_source_hash: `([0-9a-f]+)`", text)
    assert m, "the counter summary records no kernel hash"
    assert m.group(1) == bench.kernel_source_hash(), "counters taken on other kernel sources"
    t = re.search(r"traffic_bytes_per_launch: `(\d+)`", text)
    assert bench.measured_traffic() == int(t.group(1))
