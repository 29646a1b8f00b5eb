// Host check of the item deal (csrc/api.cpp): after spread_items_*, every
// block's items are a permutation of the Morton-order items, pairs stay on
// the pair positions, each item's nodes are those of its elements, each
// chunk item's block position (iperm) holds the same item, and the lanes of
// a 16-lane group share fewer bank pairs than in Morton order.
// Usage: item_deal_check <mesh file> ; prints "ok ..." or "FAIL ...".
#include "../paper_2602_12365_amd/csrc/api.cpp"

#include <set>

using namespace efem;

static int fails = 0;
#define CHECK(c, msg)                                    \
    do {                                                 \
        if (!(c)) {                                      \
            if (fails++ < 10) printf("FAIL %s\n", msg);  \
        }                                                \
    } while (0)

// the sorted global node ids of block item k (through the block's node list)
static std::vector<int32_t> item_nodes(const HostBlocks &hb, int elem, int b, int k)
{
    const int i0 = hb.istart[(size_t)b];
    const uint32_t *bn = hb.bnode.data() + hb.nstart[(size_t)b];
    std::vector<int32_t> v;
    auto g = [&](uint32_t local) { v.push_back((int32_t)(bn[local] & kGidMask)); };
    if (elem == EFEM_TET4) {
        const uint32_t w0 = hb.items[2 * (size_t)(i0 + k)], w1 = hb.items[2 * (size_t)(i0 + k) + 1];
        g(w0 & 1023u), g((w0 >> 10) & 1023u), g((w0 >> 20) & 1023u), g(w1 & 1023u), g((w1 >> 10) & 1023u);
    } else {
        for (int j = 0; j < 4; ++j) {
            const uint32_t w = hb.items[4 * (size_t)(i0 + k) + j];
            g(w & 0xffffu), g(w >> 16);
        }
    }
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    return v;
}

// the sorted node ids of the elements of block item k (from hb.order)
static std::vector<int32_t> elem_nodes(const HostBlocks &hb, const int32_t *conn, int nen, int b, int k)
{
    const int e0 = hb.estart[(size_t)b], ni = hb.istart[(size_t)b + 1] - hb.istart[(size_t)b];
    const int np = (hb.estart[(size_t)b + 1] - e0) - ni;
    std::vector<int32_t> v;
    const int first = e0 + k + std::min(k, np), cnt = k < np ? 2 : 1;
    for (int s = 0; s < cnt; ++s)
        for (int a = 0; a < nen; ++a) v.push_back(conn[(int64_t)hb.order[(size_t)(first + s)] * nen + a]);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    return v;
}

// mean over (block, column, node position, 16-lane group) of the most lanes on
// one bank pair (slot mod 16), for the block pass's lane mapping
static double block_metric(const HostBlocks &hb, int elem)
{
    const int npos = elem == EFEM_TET4 ? 5 : 8, wpi = elem == EFEM_TET4 ? 2 : 4;
    double s = 0;
    long n = 0;
    for (int b = 0; b + 1 < (int)hb.istart.size(); ++b) {
        const int i0 = hb.istart[(size_t)b], ni = hb.istart[(size_t)b + 1] - i0, S = (ni + 63) / 64;
        for (int j = 0; j < S; ++j)
            for (int a = 0; a < npos; ++a)
                for (int q = 0; q < 4; ++q) {
                    int c[16] = {}, mx = 0;
                    for (int L = 16 * q; L < 16 * q + 16; ++L) {
                        const int k = L * S + j;
                        if (k >= ni) break;
                        const uint32_t *w = hb.items.data() + (size_t)wpi * (i0 + k);
                        int l;
                        if (elem == EFEM_TET4) {
                            const int sh[5] = {0, 10, 20, 0, 10};
                            l = (int)((w[a < 3 ? 0 : 1] >> sh[a]) & 1023u);
                        } else {
                            l = (int)(a % 2 ? w[a / 2] >> 16 : w[a / 2] & 0xffffu);
                        }
                        mx = std::max(mx, ++c[l & 15]);
                    }
                    if (mx) s += mx, ++n;
                }
    }
    return s / n;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[3];
    if (fread(hdr, 8, 3, f) != 3) return 2;
    const int elem = (int)hdr[2], nen = elem == EFEM_TET4 ? 4 : 8;
    std::vector<double> X(3 * (size_t)hdr[0]);
    std::vector<int32_t> conn((size_t)nen * hdr[1]);
    if (fread(X.data(), 8, X.size(), f) != X.size() || fread(conn.data(), 4, conn.size(), f) != conn.size()) return 2;
    fclose(f);
    HostBlocks hb;
    const int be = elem == EFEM_TET4 ? 1536 : 512, bn = elem == EFEM_TET4 ? 600 : 768;
    build_blocks(elem, hdr[0], hdr[1], X.data(), conn.data(), be, bn, false, elem == EFEM_TET4, hb);
    const HostBlocks ref = hb;
    HostChunks hc;
    const bool chunks = elem == EFEM_TET4 && build_chunks(hb, hdr[0], 8, hc);
    const std::vector<uint32_t> citems0 = hc.items;
    const double m0 = block_metric(hb, elem);
    if (chunks) spread_items_chunks(hb, hc);
    else spread_items_blocks(hb, elem);
    const double m1 = block_metric(hb, elem);
    const int nb = (int)hb.istart.size() - 1;
    for (int b = 0; b < nb; ++b) {
        const int ni = hb.istart[(size_t)b + 1] - hb.istart[(size_t)b];
        const int np = (hb.estart[(size_t)b + 1] - hb.estart[(size_t)b]) - ni;
        std::multiset<std::vector<int32_t>> before, after;
        for (int k = 0; k < ni; ++k) {
            const auto nodes = item_nodes(hb, elem, b, k);
            CHECK(nodes == elem_nodes(hb, conn.data(), nen, b, k), "an item's nodes differ from its elements'");
            after.insert(nodes);
            before.insert(item_nodes(ref, elem, b, k));
            // a pair's position holds a pair (its two elements have 5 nodes)
            if (elem == EFEM_TET4) CHECK((k < np) == (nodes.size() == 5), "pair flag and position disagree");
        }
        CHECK(before == after, "the deal is not a permutation of the block's items");
        if (chunks) {
            // chunk item k and block item iperm[k] have the same nodes
            const int i0 = hb.istart[(size_t)b], c = (int)(std::upper_bound(hc.bstart.begin(), hc.bstart.end(), b)
                                                            - hc.bstart.begin()) - 1;
            const int s0 = hc.sstart[(size_t)c];
            std::multiset<std::vector<int32_t>> cset;
            for (int k = 0; k < ni; ++k) {
                const uint32_t w0 = hc.items[2 * (size_t)(i0 + k)], w1 = hc.items[2 * (size_t)(i0 + k) + 1];
                const uint32_t l[5] = {w0 & 2047u, (w0 >> 11) & 2047u, w1 & 2047u, (w0 >> 22) | ((w1 >> 22) << 10),
                                       (w1 >> 11) & 2047u};
                std::vector<int32_t> v;
                for (uint32_t x : l) v.push_back((int32_t)(hc.cnode[(size_t)(s0 + x)] & kGidMask));
                std::sort(v.begin(), v.end());
                v.erase(std::unique(v.begin(), v.end()), v.end());
                CHECK(hc.iperm[(size_t)(i0 + k)] < ni, "iperm out of range");
                CHECK(v == item_nodes(hb, elem, b, hc.iperm[(size_t)(i0 + k)]), "iperm does not match the block item");
                CHECK((k < np) == (hc.iperm[(size_t)(i0 + k)] < np), "iperm moves a pair off the pair positions");
                cset.insert(v);
            }
            CHECK(cset == after, "the chunk items are not the block's items");
        }
    }
    CHECK(m1 < m0, "the deal did not spread the block pass's bank pairs");
    if (fails) return 1;
    printf("ok blocks %d chunks %d bank-pair metric %.3f -> %.3f\n", nb, chunks ? (int)hc.bstart.size() - 1 : 0, m0, m1);
    return 0;
}
