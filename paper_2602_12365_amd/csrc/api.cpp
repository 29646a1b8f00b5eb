// C-ABI entry points: context creation (mesh blocking on the host), material
// and Dirichlet setup, and the asynchronous operator calls.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "efem_internal.h"

namespace efem {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

int hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? EFEM_ERR_OOM : EFEM_ERR_HIP;
}

#define HIP_TRY(call)                                    \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <class T>
static int dalloc(Ctx &c, T **p, size_t count)
{
    void *q = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    c.owned.push_back(q);
    *p = static_cast<T *>(q);
    return EFEM_OK;
}

template <class T>
static int upload(Ctx &c, T **p, const std::vector<T> &v)
{
    int rc = dalloc(c, p, v.size());
    if (rc) return rc;
    if (!v.empty()) HIP_TRY(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return EFEM_OK;
}

// ------------------------------------------------------------ host geometry

static double det3(const double m[9])
{
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6])
         + m[2] * (m[3] * m[7] - m[4] * m[6]);
}

// det J of the reference map at every quadrature point must be positive.
static int nodes_per_elem(int elem) { return elem == EFEM_TET4 ? 4 : (elem == EFEM_TRI3 ? 3 : 8); }

static bool reference_jacobians_positive(int elem, int nen, int64_t ne, const double *X,
                                         const int32_t *conn)
{
    static const int S[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
    const double g = 1.0 / std::sqrt(3.0);
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t *ce = conn + e * nen;
        if (elem == EFEM_TRI3) {
            // det [e1 e2 z] = (e1 x e2)_z: counter-clockwise seen from +z
            const double *a = X + 3 * (int64_t)ce[0], *b = X + 3 * (int64_t)ce[1], *c = X + 3 * (int64_t)ce[2];
            const double cz = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
            if (!(cz > 0.0)) return false;
        } else if (elem == EFEM_TET4) {
            double E[9];
            for (int i = 0; i < 3; ++i)
                for (int c = 0; c < 3; ++c) E[i * 3 + c] = X[3 * ce[c + 1] + i] - X[3 * ce[0] + i];
            if (!(det3(E) > 0.0)) return false;
        } else {
            for (int q = 0; q < 8; ++q) {
                const double p[3] = {(q & 1) ? g : -g, (q & 2) ? g : -g, (q & 4) ? g : -g};
                double J[9] = {0};
                for (int a = 0; a < 8; ++a) {
                    const double f[3] = {1 + S[a][0] * p[0], 1 + S[a][1] * p[1], 1 + S[a][2] * p[2]};
                    const double dn[3] = {0.125 * S[a][0] * f[1] * f[2], 0.125 * S[a][1] * f[0] * f[2],
                                          0.125 * S[a][2] * f[0] * f[1]};
                    for (int i = 0; i < 3; ++i)
                        for (int Jj = 0; Jj < 3; ++Jj) J[i * 3 + Jj] += X[3 * ce[a] + i] * dn[Jj];
                }
                if (!(det3(J) > 0.0)) return false;
            }
        }
    }
    return true;
}

static uint64_t spread3(uint64_t v)   // 21 bits -> every third bit
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

// ---------------------------------------------------------------- blocking

struct HostBlocks {
    std::vector<int32_t> order;      // internal -> caller element id
    std::vector<int32_t> estart, istart, nstart;
    std::vector<uint32_t> bnode;
    std::vector<uint32_t> items;     // packed local connectivity, kItemWords[elem] words per item
    std::vector<int32_t> shared_nodes;
    std::vector<std::vector<int32_t>> colours;
    int max_nodes = 0, max_elems = 0;
};

static double orient(const double *X, int32_t a, int32_t b, int32_t c, int32_t d)
{
    double E[9];
    for (int i = 0; i < 3; ++i) {
        E[i * 3 + 0] = X[3 * (int64_t)b + i] - X[3 * (int64_t)a + i];
        E[i * 3 + 1] = X[3 * (int64_t)c + i] - X[3 * (int64_t)a + i];
        E[i * 3 + 2] = X[3 * (int64_t)d + i] - X[3 * (int64_t)a + i];
    }
    return det3(E);
}

// Pair the tetrahedra el[0..n) of one block that share a face: a greedy
// maximal matching in the block's (Morton) order.  On return el holds the
// pairs first (partners adjacent), then the unpaired elements, and pw the
// node tuples (a, b, c, d1, d2) of the pairs with (a, b, c, d1) and
// (a, c, b, d2) both positively oriented.  Returns the number of pairs.
static int pair_tets(const double *X, const int32_t *conn, std::vector<int32_t> &el,
                     std::vector<std::array<int32_t, 5>> &pw)
{
    const int n = (int)el.size();
    struct Face {
        int32_t v[3];
        int32_t k;
        bool operator<(const Face &o) const
        {
            if (v[0] != o.v[0]) return v[0] < o.v[0];
            if (v[1] != o.v[1]) return v[1] < o.v[1];
            if (v[2] != o.v[2]) return v[2] < o.v[2];
            return k < o.k;
        }
        bool same(const Face &o) const { return v[0] == o.v[0] && v[1] == o.v[1] && v[2] == o.v[2]; }
    };
    std::vector<Face> faces;
    faces.reserve((size_t)n * 4);
    for (int k = 0; k < n; ++k) {
        const int32_t *ce = conn + 4 * (int64_t)el[(size_t)k];
        for (int skip = 0; skip < 4; ++skip) {
            Face f{};
            int t = 0;
            for (int a = 0; a < 4; ++a)
                if (a != skip) f.v[t++] = ce[a];
            std::sort(f.v, f.v + 3);
            f.k = k;
            faces.push_back(f);
        }
    }
    std::sort(faces.begin(), faces.end());
    // up to 4 face neighbours per element, in increasing block order
    std::vector<std::array<int32_t, 4>> nb((size_t)n);
    std::vector<int> cnt((size_t)n, 0);
    for (size_t i = 0; i + 1 < faces.size(); ++i)
        if (faces[i].same(faces[i + 1]) && (i + 2 >= faces.size() || !faces[i + 1].same(faces[i + 2]))
            && (i == 0 || !faces[i - 1].same(faces[i]))) {
            const int p = faces[i].k, q = faces[i + 1].k;
            if (p == q) continue;
            if (cnt[(size_t)p] < 4) nb[(size_t)p][(size_t)cnt[(size_t)p]++] = q;
            if (cnt[(size_t)q] < 4) nb[(size_t)q][(size_t)cnt[(size_t)q]++] = p;
        }
    for (int k = 0; k < n; ++k) std::sort(nb[(size_t)k].begin(), nb[(size_t)k].begin() + cnt[(size_t)k]);
    std::vector<int32_t> mate((size_t)n, -1);
    std::vector<int32_t> paired, single;
    pw.clear();
    for (int k = 0; k < n; ++k) {
        if (mate[(size_t)k] >= 0) continue;
        for (int t = 0; t < cnt[(size_t)k]; ++t) {
            const int j = nb[(size_t)k][(size_t)t];
            if (mate[(size_t)j] >= 0) continue;
            const int32_t *ck = conn + 4 * (int64_t)el[(size_t)k];
            const int32_t *cj = conn + 4 * (int64_t)el[(size_t)j];
            int32_t fa[3], d1 = -1, d2 = -1;
            int nf = 0;
            for (int a = 0; a < 4; ++a) {
                const bool in = ck[a] == cj[0] || ck[a] == cj[1] || ck[a] == cj[2] || ck[a] == cj[3];
                if (in && nf < 3) fa[nf++] = ck[a];
                else d1 = ck[a];
            }
            for (int a = 0; a < 4; ++a)
                if (cj[a] != fa[0] && cj[a] != fa[1] && cj[a] != fa[2]) d2 = cj[a];
            if (nf != 3 || d1 < 0 || d2 < 0) continue;
            if (!(orient(X, fa[0], fa[1], fa[2], d1) > 0.0)) std::swap(fa[1], fa[2]);
            if (!(orient(X, fa[0], fa[1], fa[2], d1) > 0.0) || !(orient(X, fa[0], fa[2], fa[1], d2) > 0.0))
                continue;
            mate[(size_t)k] = j;
            mate[(size_t)j] = k;
            paired.push_back(el[(size_t)k]);
            paired.push_back(el[(size_t)j]);
            pw.push_back({fa[0], fa[1], fa[2], d1, d2});
            break;
        }
        if (mate[(size_t)k] < 0) single.push_back(el[(size_t)k]);
    }
    const int np = (int)pw.size();
    el = paired;
    el.insert(el.end(), single.begin(), single.end());
    return np;
}

static void build_blocks(int elem, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                         int be, int bn, bool colour, bool pairs, HostBlocks &hb)
{
    const int nen = nodes_per_elem(elem);
    // Morton order of element centroids
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < nn; ++i)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], X[3 * i + k]);
            hi[k] = std::max(hi[k], X[3 * i + k]);
        }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    std::vector<std::pair<uint64_t, int32_t>> keys((size_t)ne);
    for (int64_t e = 0; e < ne; ++e) {
        double c[3] = {0, 0, 0};
        for (int a = 0; a < nen; ++a)
            for (int k = 0; k < 3; ++k) c[k] += X[3 * (int64_t)conn[e * nen + a] + k];
        uint64_t key = 0;
        for (int k = 0; k < 3; ++k) {
            double t = (c[k] / nen - lo[k]) / ext;
            uint64_t q = (uint64_t)std::min(std::max(t, 0.0) * 2097151.0, 2097151.0);
            key |= spread3(q) << k;
        }
        keys[(size_t)e] = {key, (int32_t)e};
    }
    std::sort(keys.begin(), keys.end());
    hb.order.resize((size_t)ne);
    for (int64_t e = 0; e < ne; ++e) hb.order[(size_t)e] = keys[(size_t)e].second;

    // greedy cut: at most `be` elements and `bn` distinct nodes per block
    std::vector<int32_t> mark((size_t)nn, -1);
    std::vector<int32_t> cut{0};
    int cur_e = 0, cur_n = 0, blk = 0;
    for (int64_t k = 0; k < ne; ++k) {
        const int32_t *ce = conn + (int64_t)hb.order[(size_t)k] * nen;
        int fresh = 0;
        for (int a = 0; a < nen; ++a) {
            bool dup = false;
            for (int b = 0; b < a; ++b) dup |= ce[b] == ce[a];
            if (!dup && mark[ce[a]] != blk) ++fresh;
        }
        if (cur_e > 0 && (cur_e + 1 > be || cur_n + fresh > bn)) {
            cut.push_back((int32_t)k);
            ++blk;
            cur_e = 0;
            cur_n = 0;
            fresh = 0;
            for (int a = 0; a < nen; ++a) {
                bool dup = false;
                for (int b = 0; b < a; ++b) dup |= ce[b] == ce[a];
                if (!dup) ++fresh;
            }
        }
        for (int a = 0; a < nen; ++a) mark[ce[a]] = blk;
        cur_e += 1;
        cur_n += fresh;
    }
    cut.push_back((int32_t)ne);
    const int nb = (int)cut.size() - 1;
    hb.estart = cut;

    // per-block sorted node lists, tetrahedron pairs and packed local connectivity
    hb.nstart.assign(1, 0);
    hb.istart.assign(1, 0);
    std::vector<int32_t> nodes, el;
    std::vector<std::array<int32_t, 5>> pw;
    std::vector<int32_t> nblocks((size_t)nn, 0);
    std::vector<int32_t> local((size_t)nn, -1);
    for (int b = 0; b < nb; ++b) {
        nodes.clear();
        for (int k = cut[b]; k < cut[b + 1]; ++k)
            for (int a = 0; a < nen; ++a) nodes.push_back(conn[(int64_t)hb.order[k] * nen + a]);
        std::sort(nodes.begin(), nodes.end());
        nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
        for (size_t i = 0; i < nodes.size(); ++i) {
            local[nodes[i]] = (int32_t)i;
            hb.bnode.push_back((uint32_t)nodes[i]);
            nblocks[nodes[i]] += 1;
        }
        el.assign(hb.order.begin() + cut[b], hb.order.begin() + cut[b + 1]);
        if (elem == EFEM_TET4) {
            const int np = pairs ? pair_tets(X, conn, el, pw) : 0;
            std::copy(el.begin(), el.end(), hb.order.begin() + cut[b]);
            // item words: a | b << 10 | c << 20, then d1 | d2 << 10 (local ids < 1024)
            for (int p = 0; p < np; ++p) {
                const auto &t = pw[(size_t)p];
                hb.items.push_back((uint32_t)local[t[0]] | (uint32_t)local[t[1]] << 10
                                   | (uint32_t)local[t[2]] << 20);
                hb.items.push_back((uint32_t)local[t[3]] | (uint32_t)local[t[4]] << 10);
            }
            for (size_t k = 2 * (size_t)np; k < el.size(); ++k) {
                const int32_t *ce = conn + 4 * (int64_t)el[k];
                hb.items.push_back((uint32_t)local[ce[0]] | (uint32_t)local[ce[1]] << 10
                                   | (uint32_t)local[ce[2]] << 20);
                hb.items.push_back((uint32_t)local[ce[3]] | (uint32_t)local[ce[3]] << 10);
            }
            hb.istart.push_back(hb.istart.back() + (int32_t)el.size() - np);
        } else if (elem == EFEM_TRI3) {
            // item word: a | b << 10 | c << 20 (local ids < 1024)
            for (int32_t e : el) {
                const int32_t *ce = conn + 3 * (int64_t)e;
                hb.items.push_back((uint32_t)local[ce[0]] | (uint32_t)local[ce[1]] << 10
                                   | (uint32_t)local[ce[2]] << 20);
            }
            hb.istart.push_back(hb.istart.back() + (int32_t)el.size());
        } else {
            for (int32_t e : el) {
                const int32_t *ce = conn + 8 * (int64_t)e;
                for (int a = 0; a < 8; a += 2)
                    hb.items.push_back((uint32_t)local[ce[a]] | (uint32_t)local[ce[a + 1]] << 16);
            }
            hb.istart.push_back(hb.istart.back() + (int32_t)el.size());
        }
        hb.nstart.push_back((int32_t)hb.bnode.size());
        hb.max_nodes = std::max(hb.max_nodes, (int)nodes.size());
        hb.max_elems = std::max(hb.max_elems, cut[b + 1] - cut[b]);
    }
    for (size_t i = 0; i < hb.bnode.size(); ++i)
        if (nblocks[hb.bnode[i]] > 1) hb.bnode[i] |= kShared;
    for (int64_t g = 0; g < nn; ++g)
        if (nblocks[(size_t)g] > 1) hb.shared_nodes.push_back((int32_t)g);

    if (!colour) return;
    // node -> blocks CSR over shared nodes
    std::vector<int32_t> ptr((size_t)nn + 1, 0);
    for (size_t i = 0; i < hb.bnode.size(); ++i)
        if (hb.bnode[i] & kShared) ptr[(hb.bnode[i] & kGidMask) + 1] += 1;
    for (int64_t g = 0; g < nn; ++g) ptr[(size_t)g + 1] += ptr[(size_t)g];
    std::vector<int32_t> adj(ptr[(size_t)nn]);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int b = 0; b < nb; ++b)
        for (int i = hb.nstart[b]; i < hb.nstart[b + 1]; ++i)
            if (hb.bnode[i] & kShared) adj[fill[hb.bnode[i] & kGidMask]++] = b;
    // greedy colouring of the block graph (blocks sharing a node conflict)
    std::vector<int32_t> col((size_t)nb, -1);
    std::vector<int32_t> seen;
    int ncol = 0;
    for (int b = 0; b < nb; ++b) {
        seen.assign((size_t)ncol + 1, 0);
        for (int i = hb.nstart[b]; i < hb.nstart[b + 1]; ++i) {
            if (!(hb.bnode[i] & kShared)) continue;
            const uint32_t g = hb.bnode[i] & kGidMask;
            for (int j = ptr[g]; j < ptr[g + 1]; ++j)
                if (col[adj[j]] >= 0) seen[col[adj[j]]] = 1;
        }
        int c = 0;
        while (c < ncol && seen[c]) ++c;
        col[b] = c;
        ncol = std::max(ncol, c + 1);
    }
    hb.colours.assign((size_t)ncol, {});
    for (int b = 0; b < nb; ++b) hb.colours[col[b]].push_back(b);
    // the lowest-coloured block touching a shared node writes it first
    for (int b = 0; b < nb; ++b)
        for (int i = hb.nstart[b]; i < hb.nstart[b + 1]; ++i) {
            if (!(hb.bnode[i] & kShared)) continue;
            const uint32_t g = hb.bnode[i] & kGidMask;
            bool first = true;
            for (int j = ptr[g]; j < ptr[g + 1]; ++j) first &= col[adj[j]] >= col[b];
            if (first) hb.bnode[i] |= kFirst;
        }
}

// Chunks of consecutive blocks for the LDS-resident pass of the FP64 Tet4
// tangent action.
struct HostChunks {
    std::vector<int32_t> bstart, sstart;
    std::vector<uint32_t> bnew, cnode, items;
    std::vector<uint16_t> iperm;   // per chunk item: its position in the block pass's order
    std::vector<int32_t> shared_nodes;   // nodes in more than one chunk, increasing id
    // a chunk's slots in the order their sums become final (by the last of
    // its blocks that touches them): fin_slot[s0 + j] is a global slot
    // index, and the slots final after block b are [fin_start[b], fin_start[b + 1])
    std::vector<int32_t> fin_slot, fin_start;
    int max_slots = 0;
};

// n chunks of consecutive blocks (block counts differing by at most one); each
// chunk numbers its nodes in order of first use.  False if a chunk needs more
// than kChunkCap slots.
static bool try_chunks(const HostBlocks &hb, int64_t nn, int n, HostChunks &hc)
{
    const int nb = (int)hb.estart.size() - 1;
    hc = HostChunks{};
    hc.bstart.resize((size_t)n + 1);
    for (int i = 0; i <= n; ++i) hc.bstart[(size_t)i] = (int32_t)((int64_t)nb * i / n);
    hc.sstart.assign(1, 0);
    hc.bnew.assign((size_t)nb, 0u);
    for (int c = 0; c < n; ++c)
        if (hc.bstart[(size_t)c + 1] - hc.bstart[(size_t)c] > kChunkSteps) return false;
    std::vector<int32_t> slot_of((size_t)nn, -1), nchunks((size_t)nn, 0);
    std::vector<int32_t> touched, last_blk;
    hc.fin_start.assign((size_t)nb + 1, 0);
    for (int c = 0; c < n; ++c) {
        touched.clear();
        last_blk.clear();
        int ns = 0;
        bool fits = true;
        for (int b = hc.bstart[(size_t)c]; b < hc.bstart[(size_t)c + 1] && fits; ++b) {
            const int lo = ns;
            for (int i = hb.nstart[(size_t)b]; i < hb.nstart[(size_t)b + 1]; ++i) {
                const uint32_t g = hb.bnode[(size_t)i] & kGidMask;
                if (slot_of[g] < 0) {
                    slot_of[g] = ns++;
                    touched.push_back((int32_t)g);
                    hc.cnode.push_back(g);
                    last_blk.push_back(b);
                } else {
                    last_blk[(size_t)slot_of[g]] = b;
                }
            }
            // a block's new slots must span at most one 64-slot group per wave
            const int groups = ns > lo ? ((ns - 1) >> 6) - (lo >> 6) + 1 : 0;
            if (ns > kChunkCap || groups > kChunkThreads / 64) {
                fits = false;
                break;
            }
            hc.bnew[(size_t)b] = (uint32_t)lo | (uint32_t)ns << 16;
            const uint32_t *bn = hb.bnode.data() + hb.nstart[(size_t)b];
            auto sl = [&](uint32_t local) { return (uint32_t)slot_of[bn[local] & kGidMask]; };
            for (int it = hb.istart[(size_t)b]; it < hb.istart[(size_t)b + 1]; ++it) {
                const uint32_t w0 = hb.items[2 * (size_t)it], w1 = hb.items[2 * (size_t)it + 1];
                const uint32_t a = sl(w0 & 1023u), bb = sl((w0 >> 10) & 1023u), cc = sl((w0 >> 20) & 1023u);
                const uint32_t d1 = sl(w1 & 1023u), d2 = sl((w1 >> 10) & 1023u);
                hc.items.push_back(a | bb << 11 | (d1 & 1023u) << 22);
                hc.items.push_back(cc | d2 << 11 | (d1 >> 10) << 22);
            }
        }
        for (int32_t g : touched) {
            nchunks[(size_t)g] += 1;
            slot_of[(size_t)g] = -1;
        }
        if (!fits) return false;
        // the chunk's slots by the block after which they are final (a
        // counting sort, slot order kept within a block)
        const int s0 = hc.sstart.back(), cb0 = hc.bstart[(size_t)c], cb1 = hc.bstart[(size_t)c + 1];
        std::vector<int32_t> cnt((size_t)(cb1 - cb0) + 1, 0);
        for (int l = 0; l < ns; ++l) cnt[(size_t)(last_blk[(size_t)l] - cb0) + 1] += 1;
        for (int k = 0; k < cb1 - cb0; ++k) cnt[(size_t)k + 1] += cnt[(size_t)k];
        for (int k = 0; k < cb1 - cb0; ++k) hc.fin_start[(size_t)(cb0 + k)] = s0 + cnt[(size_t)k];
        hc.fin_slot.resize((size_t)s0 + ns);
        for (int l = 0; l < ns; ++l)
            hc.fin_slot[(size_t)(s0 + cnt[(size_t)(last_blk[(size_t)l] - cb0)]++)] = s0 + l;
        hc.sstart.push_back((int32_t)hc.cnode.size());
        hc.max_slots = std::max(hc.max_slots, ns);
    }
    hc.fin_start[(size_t)nb] = (int32_t)hc.cnode.size();
    for (uint32_t &e : hc.cnode)
        if (nchunks[e & kGidMask] > 1) e |= kShared;
    for (int64_t g = 0; g < nn; ++g)
        if (nchunks[(size_t)g] > 1) hc.shared_nodes.push_back((int32_t)g);
    return true;
}

// Chunk count: a multiple of the CU count (one resident chunk per CU, all of
// them in one round when it fits), the smallest whose chunks fit the LDS; one
// block per chunk always fits.  False if the pass does not apply: blocks with
// more items than the workgroup's threads.
static bool build_chunks(const HostBlocks &hb, int64_t nn, int n_cu, HostChunks &hc)
{
    const int nb = (int)hb.estart.size() - 1;
    for (int b = 0; b < nb; ++b)
        if (hb.istart[(size_t)b + 1] - hb.istart[(size_t)b] > kChunkThreads) return false;
    for (int k = 1;; ++k) {
        const int n = (int)std::min<int64_t>(nb, (int64_t)k * std::max(n_cu, 1));
        if (try_chunks(hb, nn, n, hc)) return true;
        if (n == nb) return false;
    }
}

// Item order within each block, for the LDS.  The 64 lanes of a wave issue
// each node-record read and each FP64 LDS atomic of their items together, at
// the slots of one node position.  The LDS serves an FP64 atomic 16 lanes at a
// time, the lanes of such a group one after another where their slots l fall
// on one bank pair, (3 l + i) mod 16 for component i (one-to-one with
// l mod 16), and a 16-byte record read 8 lanes at a time, by bank quad l mod 8
// (measured: lanes paired on bank pairs within each 16-lane group cost as much
// as random slots, lanes paired across groups nothing).  In Morton order a
// group's slots are effectively random.  The items of a block are dealt to the
// lane groups greedily instead: an item goes to the group, among those with
// positions left, where its slots' residues mod 16 have been taken least
// often, counting also the residues mod 8 in the 8-lane half it lands in.
// Tetrahedron pairs are dealt over the pair positions and single tetrahedra
// over theirs (an item's position decides its pair flag); the element order
// and the item words move with the items.  Slots do not depend on the order
// of the items within a block.

// One block's items [lo, hi): slots(k, r) gives the NPOS slots of item k,
// group_of(k) the lane group (of 16) of position k among ng groups.  On
// return assign[k] is the item placed at position k.
template <int NPOS, class Slots, class Group>
static void deal_items(int lo, int hi, int ng, Group group_of, Slots slots, std::vector<int32_t> &assign)
{
    constexpr int G = 16, M = 16, M2 = 8;
    if (hi <= lo) return;
    // residue counts with the group index innermost, so that one item's cost
    // over all groups is a few contiguous sweeps
    std::vector<int32_t> cnt((size_t)NPOS * M * ng, 0), cnt2((size_t)2 * NPOS * M2 * ng, 0);
    std::vector<int32_t> cap((size_t)ng, 0), fill((size_t)ng, 0), c0((size_t)ng), c1((size_t)ng), c2((size_t)ng);
    std::vector<std::vector<int32_t>> dealt((size_t)ng);
    for (int k = lo; k < hi; ++k) cap[(size_t)group_of(k)] += 1;
    for (int k = lo; k < hi; ++k) {
        int r[NPOS];
        slots(k, r);
        std::fill(c0.begin(), c0.end(), 0);
        std::fill(c1.begin(), c1.end(), 0);
        std::fill(c2.begin(), c2.end(), 0);
        for (int a = 0; a < NPOS; ++a) {
            const int32_t *p = &cnt[((size_t)a * M + (r[a] & (M - 1))) * ng];
            const int32_t *q0 = &cnt2[(((size_t)0 * NPOS + a) * M2 + (r[a] & (M2 - 1))) * ng];
            const int32_t *q1 = &cnt2[(((size_t)1 * NPOS + a) * M2 + (r[a] & (M2 - 1))) * ng];
            for (int g = 0; g < ng; ++g) {
                c0[(size_t)g] += p[g];
                c1[(size_t)g] += q0[g];
                c2[(size_t)g] += q1[g];
            }
        }
        int best = -1, best_cost = 0;
        for (int g = 0; g < ng; ++g) {
            if (cap[(size_t)g] == 0) continue;
            const int cost = c0[(size_t)g] + (fill[(size_t)g] >= G / 2 ? c2[(size_t)g] : c1[(size_t)g]);
            if (best < 0 || cost < best_cost || (cost == best_cost && cap[(size_t)g] > cap[(size_t)best])) {
                best = g;
                best_cost = cost;
            }
        }
        const int half = fill[(size_t)best] >= G / 2 ? 1 : 0;
        for (int a = 0; a < NPOS; ++a) {
            cnt[((size_t)a * M + (r[a] & (M - 1))) * ng + best] += 1;
            cnt2[(((size_t)half * NPOS + a) * M2 + (r[a] & (M2 - 1))) * ng + best] += 1;
        }
        cap[(size_t)best] -= 1;
        fill[(size_t)best] += 1;
        dealt[(size_t)best].push_back(k);
    }
    // the positions of a group, in lane order, take its items in the order dealt
    std::vector<int32_t> next((size_t)ng, 0);
    for (int k = lo; k < hi; ++k) {
        const int g = group_of(k);
        assign[(size_t)k] = dealt[(size_t)g][(size_t)next[(size_t)g]++];
    }
}

// Block b's items to the order assign: the block pass's item words (wpi per
// item) and the elements.
static void permute_items(HostBlocks &hb, int b, int wpi, const std::vector<int32_t> &assign)
{
    const int i0 = hb.istart[(size_t)b], ni = hb.istart[(size_t)b + 1] - i0;
    const int e0 = hb.estart[(size_t)b], np = (hb.estart[(size_t)b + 1] - e0) - ni;
    const std::vector<uint32_t> bw(hb.items.begin() + (size_t)wpi * i0, hb.items.begin() + (size_t)wpi * (i0 + ni));
    const std::vector<int32_t> el(hb.order.begin() + e0, hb.order.begin() + hb.estart[(size_t)b + 1]);
    for (int k = 0; k < ni; ++k) {
        const int src = assign[(size_t)k];
        for (int j = 0; j < wpi; ++j) hb.items[(size_t)wpi * (i0 + k) + j] = bw[(size_t)wpi * src + j];
        if (k < np) {
            hb.order[(size_t)(e0 + 2 * k)] = el[2 * (size_t)src];
            hb.order[(size_t)(e0 + 2 * k + 1)] = el[2 * (size_t)src + 1];
        } else {
            hb.order[(size_t)(e0 + np + k)] = el[(size_t)(np + src)];
        }
    }
}

// For the chunk pass (Tet4 pairs): item k runs on lane k / W of wave k % W
// (W = kChunkThreads / 64), with the chunk's slots.  The block pass over the
// same blocks (the FP32 action, the residual, the energy) keys its groups on
// the block's node ids, so each pass gets its own deal: the block order (and
// with it the element order) is dealt for the block pass, the chunk items for
// the chunk pass, and iperm gives each chunk item's block position, where the
// per-element materials are found.
static void spread_items_chunks(HostBlocks &hb, HostChunks &hc)
{
    constexpr int W = kChunkThreads / 64, NG = W * 4;
    const int nb = (int)hb.estart.size() - 1;
    std::vector<int32_t> ac, ab, inv;
    std::vector<uint32_t> cw;
    hc.iperm.assign(hc.items.size() / 2, 0);
    auto group_c = [](int k) { return (k % W) * 4 + (k / W) / 16; };
    for (int b = 0; b < nb; ++b) {
        const int i0 = hb.istart[(size_t)b], ni = hb.istart[(size_t)b + 1] - i0;
        const int np = (hb.estart[(size_t)b + 1] - hb.estart[(size_t)b]) - ni;
        auto cslots = [&](int k, int r[5]) {
            const uint32_t w0 = hc.items[2 * (size_t)(i0 + k)], w1 = hc.items[2 * (size_t)(i0 + k) + 1];
            r[0] = (int)(w0 & 2047u);
            r[1] = (int)((w0 >> 11) & 2047u);
            r[2] = (int)(w1 & 2047u);
            r[3] = (int)((w0 >> 22) | ((w1 >> 22) << 10));
            r[4] = (int)((w1 >> 11) & 2047u);
        };
        const uint32_t *w = hb.items.data() + 2 * (size_t)i0;
        auto bslots = [&](int k, int r[5]) {
            const uint32_t w0 = w[2 * (size_t)k], w1 = w[2 * (size_t)k + 1];
            r[0] = (int)(w0 & 1023u);
            r[1] = (int)((w0 >> 10) & 1023u);
            r[2] = (int)((w0 >> 20) & 1023u);
            r[3] = (int)(w1 & 1023u);
            r[4] = (int)((w1 >> 10) & 1023u);
        };
        const int S = (ni + 63) / 64;
        auto group_b = [S](int k) { return (k % S) * 4 + (k / S) / 16; };
        ac.assign((size_t)ni, 0);
        ab.assign((size_t)ni, 0);
        deal_items<5>(0, np, NG, group_c, cslots, ac);
        deal_items<5>(np, ni, NG, group_c, cslots, ac);
        deal_items<5>(0, np, 4 * S, group_b, bslots, ab);
        deal_items<5>(np, ni, 4 * S, group_b, bslots, ab);
        // chunk items in their order, each with its block position
        inv.assign((size_t)ni, 0);
        for (int k = 0; k < ni; ++k) inv[(size_t)ab[(size_t)k]] = k;
        cw.assign(hc.items.begin() + 2 * (size_t)i0, hc.items.begin() + 2 * (size_t)(i0 + ni));
        for (int k = 0; k < ni; ++k) {
            const int src = ac[(size_t)k];
            hc.items[2 * (size_t)(i0 + k)] = cw[2 * (size_t)src];
            hc.items[2 * (size_t)(i0 + k) + 1] = cw[2 * (size_t)src + 1];
            hc.iperm[(size_t)(i0 + k)] = (uint16_t)inv[(size_t)src];
        }
        permute_items(hb, b, 2, ab);
    }
}

// For the block pass: item k runs on lane k / S in column k % S, S = ceil(ni
// / 64), the 64 lanes of one column together; the slots are the block's node
// ids.
static void spread_items_blocks(HostBlocks &hb, int elem)
{
    const int nb = (int)hb.estart.size() - 1;
    const int wpi = elem == EFEM_TET4 ? 2 : (elem == EFEM_TRI3 ? 1 : 4);
    std::vector<int32_t> assign;
    for (int b = 0; b < nb; ++b) {
        const int i0 = hb.istart[(size_t)b], ni = hb.istart[(size_t)b + 1] - i0;
        const int np = (hb.estart[(size_t)b + 1] - hb.estart[(size_t)b]) - ni;
        const int S = (ni + 63) / 64;
        auto group_of = [S](int k) { return (k % S) * 4 + (k / S) / 16; };
        const uint32_t *w = hb.items.data() + (size_t)wpi * i0;
        assign.assign((size_t)ni, 0);
        if (elem == EFEM_TET4) {
            auto slots = [&](int k, int r[5]) {
                const uint32_t w0 = w[2 * (size_t)k], w1 = w[2 * (size_t)k + 1];
                r[0] = (int)(w0 & 1023u);
                r[1] = (int)((w0 >> 10) & 1023u);
                r[2] = (int)((w0 >> 20) & 1023u);
                r[3] = (int)(w1 & 1023u);
                r[4] = (int)((w1 >> 10) & 1023u);
            };
            deal_items<5>(0, np, 4 * S, group_of, slots, assign);
            deal_items<5>(np, ni, 4 * S, group_of, slots, assign);
        } else if (elem == EFEM_TRI3) {
            auto slots = [&](int k, int r[3]) {
                r[0] = (int)(w[k] & 1023u);
                r[1] = (int)((w[k] >> 10) & 1023u);
                r[2] = (int)((w[k] >> 20) & 1023u);
            };
            deal_items<3>(0, ni, 4 * S, group_of, slots, assign);
        } else {
            auto slots = [&](int k, int r[8]) {
                for (int j = 0; j < 4; ++j) {
                    r[2 * j] = (int)(w[4 * (size_t)k + j] & 0xffffu);
                    r[2 * j + 1] = (int)(w[4 * (size_t)k + j] >> 16);
                }
            };
            deal_items<8>(0, ni, 4 * S, group_of, slots, assign);
        }
        permute_items(hb, b, wpi, assign);
    }
}

// Halo layout of the shared nodes (HaloSegs): each node's entries take
// consecutive slots in entry order (block or chunk order), nodes grouped by
// entry count.  hslot[i] is the slot of entry i (-1 for unshared entries);
// order lists the shared nodes in gather order; gptr the slot ranges of the
// nodes with more than kSegMax entries.
static void halo_layout(const std::vector<uint32_t> &entries, const std::vector<int32_t> &shared, int64_t nn,
                        HaloSegs &seg, std::vector<int32_t> &order, std::vector<int32_t> &gptr,
                        std::vector<int32_t> &hslot)
{
    const int32_t ns = (int32_t)shared.size();
    std::vector<int32_t> cnt((size_t)nn, 0);
    for (uint32_t ent : entries)
        if (ent & kShared) cnt[ent & kGidMask] += 1;
    auto group = [](int c) { return c <= kSegMax ? c : kSegMax + 1; };
    // shared-node order: by group, then by node id
    order.clear();
    for (int gidx = 2; gidx <= kSegMax + 1; ++gidx) {
        seg.start[gidx] = (int32_t)order.size();
        for (int32_t g : shared)
            if (group(cnt[(size_t)g]) == gidx) order.push_back(g);
    }
    seg.start[0] = seg.start[1] = 0;
    seg.n = ns;
    // first slot of each shared node
    std::vector<int32_t> first((size_t)nn, -1);
    int32_t slot = 0;
    for (int c = 2; c <= kSegMax; ++c) {
        seg.base[c] = slot;
        for (int32_t i = seg.start[c]; i < (c < kSegMax ? seg.start[c + 1] : seg.start[kSegMax + 1]); ++i) {
            first[(size_t)order[(size_t)i]] = slot;
            slot += c;
        }
    }
    seg.base[0] = seg.base[1] = 0;
    gptr.assign(1, slot);
    for (int32_t i = seg.start[kSegMax + 1]; i < ns; ++i) {
        const int32_t g = order[(size_t)i];
        first[(size_t)g] = slot;
        slot += cnt[(size_t)g];
        gptr.push_back(slot);
    }
    hslot.assign(entries.size(), -1);
    for (size_t i = 0; i < entries.size(); ++i)
        if (entries[i] & kShared) hslot[i] = first[entries[i] & kGidMask]++;
}

}  // namespace efem

using namespace efem;

struct efem_ctx : Ctx {};

// ------------------------------------------------------------------- C-ABI

extern "C" {

const char *efem_last_error(void) { return g_error.c_str(); }

void efem_destroy(efem_ctx *ctx)
{
    if (!ctx) return;
    DeviceGuard dg(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    mlp_release(*ctx);
    sparse_release(*ctx);
    for (void *p : ctx->owned) (void)hipFree(p);
    delete ctx;
}

int efem_create(efem_ctx **out, int32_t elem, int64_t n_nodes, int64_t n_elems,
                const double *coords, const int32_t *conn, const efem_options *opts, void *stream)
{
    if (!out || !coords || !conn) {
        set_error("efem_create: null pointer");
        return EFEM_ERR_INVALID;
    }
    *out = nullptr;
    if (elem != EFEM_TET4 && elem != EFEM_HEX8 && elem != EFEM_TRI3) {
        set_error("efem_create: unknown element type");
        return EFEM_ERR_INVALID;
    }
    if (n_nodes < 1 || n_elems < 1 || n_nodes > (int64_t)kGidMask || n_elems > INT32_MAX / 8) {
        set_error("efem_create: bad mesh sizes");
        return EFEM_ERR_INVALID;
    }
    const int nen = nodes_per_elem(elem);
    std::vector<uint8_t> used((size_t)n_nodes, 0);
    for (int64_t k = 0; k < n_elems * nen; ++k) {
        if (conn[k] < 0 || conn[k] >= n_nodes) {
            set_error("efem_create: connectivity entry out of range");
            return EFEM_ERR_INVALID;
        }
        used[(size_t)conn[k]] = 1;
    }
    // every output entry is written by the element passes, so a node outside
    // every element (whose rows of K are zero) would be left unwritten
    for (int64_t g = 0; g < n_nodes; ++g)
        if (!used[(size_t)g]) {
            set_error("efem_create: node in no element (remove unreferenced nodes)");
            return EFEM_ERR_INVALID;
        }
    if (!reference_jacobians_positive(elem, nen, n_elems, coords, conn)) {
        set_error("efem_create: reference element with det J <= 0");
        return EFEM_ERR_INVERTED;
    }
    // defaults measured on the 64^3 workloads: 1536 tets (768 pairs) within 600
    // nodes, or 512 hexes within 768 nodes, per block; triangles (1024^2 cells):
    // 768 within 600 nodes
    int be = elem == EFEM_TET4 ? 1536 : (elem == EFEM_TRI3 ? 768 : 512);
    int bn = elem == EFEM_HEX8 ? 768 : 600;
    int scatter = EFEM_SCATTER_HALO;
    int threads = 256;
    if (opts) {
        if (opts->block_elems > 0) be = opts->block_elems;
        if (opts->block_nodes > 0) bn = opts->block_nodes;
        scatter = opts->scatter;
        if (scatter != EFEM_SCATTER_HALO && scatter != EFEM_SCATTER_COLOR && scatter != EFEM_SCATTER_ATOMIC) {
            set_error("efem_create: unknown scatter mode");
            return EFEM_ERR_INVALID;
        }
        if (opts->threads > 0) threads = opts->threads;
    }
    // 768 nodes x (80-byte record + 24-byte FP64 sums + 4-byte node word) =
    // 81 KB of LDS, within a workgroup's 160 KB
    if (bn < nen || bn > 768 || be < 1 || threads < 64 || threads > 256 || threads % 64) {
        set_error("efem_create: block_nodes must be in [n_en, 768], threads a multiple of 64 in [64, 256]");
        return EFEM_ERR_INVALID;
    }

    auto *ctx = new (std::nothrow) efem_ctx();
    if (!ctx) return EFEM_ERR_OOM;
    ctx->elem = elem;
    ctx->nen = nen;
    ctx->nq = elem == EFEM_HEX8 ? 8 : 1;
    ctx->n_nodes = n_nodes;
    ctx->n_elems = n_elems;
    ctx->stream = (hipStream_t)stream;
    ctx->scatter = scatter == EFEM_SCATTER_COLOR ? Scatter::Color
                   : scatter == EFEM_SCATTER_ATOMIC ? Scatter::Atomic
                                                    : Scatter::Halo;
    ctx->threads = threads;
    (void)hipGetDevice(&ctx->device);
    {
        // the no-allocation energy's device array, addressed once per device
        const hipError_t e = noalloc_setup(ctx->device);
        if (e != hipSuccess) {
            const int rc0 = hip_fail(e, "efem_create: hipGetSymbolAddress of the static partials");
            delete ctx;
            return rc0;
        }
    }

    ctx->conn_host.assign(conn, conn + n_elems * nen);
    HostBlocks hb;
    build_blocks(elem, n_nodes, n_elems, coords, conn, be, bn, scatter == EFEM_SCATTER_COLOR,
                 !(opts && opts->no_pairs), hb);
    ctx->max_block_nodes = hb.max_nodes;
    ctx->max_block_elems = hb.max_elems;

    auto fail = [&](int rc) {
        efem_destroy(ctx);
        return rc;
    };
    // chunks for the LDS-resident FP64 tangent action (Tet4 pairs, halo
    // scatter), built before the uploads: the item order follows them
    int lds_max = 0, n_cu = 0;
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device);
    HostChunks hc;
    const bool use_chunks = elem == EFEM_TET4 && ctx->scatter == Scatter::Halo && !(opts && opts->no_chunks)
                            && n_nodes <= (int64_t)kStageGid && lds_max >= kChunkLds
                            && build_chunks(hb, n_nodes, n_cu, hc);
    if (use_chunks) spread_items_chunks(hb, hc);
    else spread_items_blocks(hb, elem);
    int rc;
    BlockMesh &m = ctx->m;
    m.n_blocks = (int32_t)hb.estart.size() - 1;
    std::vector<double> Xh(coords, coords + 3 * n_nodes);
    std::vector<float> Xfh(Xh.begin(), Xh.end());
    int32_t *p_es, *p_is, *p_ns, *p_eo;
    uint32_t *p_bn, *p_it;
    double *p_X;
    float *p_Xf;
    if ((rc = upload(*ctx, &p_es, hb.estart)) || (rc = upload(*ctx, &p_is, hb.istart))
        || (rc = upload(*ctx, &p_ns, hb.nstart)) || (rc = upload(*ctx, &p_bn, hb.bnode))
        || (rc = upload(*ctx, &p_it, hb.items)) || (rc = upload(*ctx, &p_eo, hb.order))
        || (rc = upload(*ctx, &p_X, Xh)) || (rc = upload(*ctx, &p_Xf, Xfh)))
        return fail(rc);
    ctx->n_items = hb.istart.back();
    m.estart = p_es;
    m.istart = p_is;
    m.nstart = p_ns;
    m.bnode = p_bn;
    m.items = p_it;
    m.eorig = p_eo;
    m.X = p_X;
    m.Xf = p_Xf;
    ctx->n_shared = (int64_t)hb.shared_nodes.size();
    m.halo = nullptr;
    m.hslot = nullptr;
    if (ctx->scatter == Scatter::Halo && ctx->n_shared > 0) {
        // each shared node's block-node entries, in block order
        std::vector<int32_t> order, gptr, hslot;
        halo_layout(hb.bnode, hb.shared_nodes, n_nodes, ctx->halo.seg, order, gptr, hslot);
        double *p_h;
        int32_t *p_hs;
        if ((rc = upload(*ctx, &ctx->halo.gptr, gptr)) || (rc = upload(*ctx, &p_hs, hslot))
            || (rc = upload(*ctx, &ctx->halo.node, order)) || (rc = dalloc(*ctx, &p_h, 3 * (size_t)gptr.back())))
            return fail(rc);
        m.halo = p_h;
        m.hslot = p_hs;
    }

    if (use_chunks) {
        ChunkMesh &ch = ctx->ch;
        ch.n_chunks = (int32_t)hc.bstart.size() - 1;
        ctx->max_chunk_slots = hc.max_slots;
        ctx->n_chunk_slots = (int64_t)hc.cnode.size();
        ctx->n_ch_shared = (int64_t)hc.shared_nodes.size();
        int32_t *p_bs, *p_ss, *p_hs = nullptr, *p_hd;
        uint32_t *p_bw, *p_cn, *p_it;
        uint16_t *p_ip;
        std::vector<int32_t> hdr((size_t)ch.n_chunks * 8, 0);
        for (int c = 0; c < ch.n_chunks; ++c) {
            const int b0 = hc.bstart[(size_t)c], b1 = hc.bstart[(size_t)c + 1];
            int32_t *h = &hdr[(size_t)c * 8];
            h[0] = b0;
            h[1] = b1 - b0;
            h[2] = hc.sstart[(size_t)c];
            h[3] = hc.sstart[(size_t)c + 1] - hc.sstart[(size_t)c];
            h[4] = hb.istart[(size_t)b0];
            h[5] = hb.istart[(size_t)b0 + 1] - hb.istart[(size_t)b0];
            h[6] = b1 - b0 > 1 ? (int32_t)hc.bnew[(size_t)b0 + 1] : 0;
        }
        if ((rc = upload(*ctx, &p_bs, hc.bstart)) || (rc = upload(*ctx, &p_ss, hc.sstart))
            || (rc = upload(*ctx, &p_bw, hc.bnew)) || (rc = upload(*ctx, &p_cn, hc.cnode))
            || (rc = upload(*ctx, &p_it, hc.items)) || (rc = upload(*ctx, &p_hd, hdr))
            || (rc = upload(*ctx, &p_ip, hc.iperm)))
            return fail(rc);
        ch.hdr = reinterpret_cast<const int4 *>(p_hd);
        ch.bstart = p_bs;
        ch.sstart = p_ss;
        ch.bnew = p_bw;
        ch.cnode = p_cn;
        ch.items = p_it;
        ch.iperm = p_ip;
        ch.halo = nullptr;
        if (ctx->n_ch_shared > 0) {
            std::vector<int32_t> order, gptr, hslot;
            halo_layout(hc.cnode, hc.shared_nodes, n_nodes, ctx->ch_halo.seg, order, gptr, hslot);
            double *p_h;
            if ((rc = upload(*ctx, &ctx->ch_halo.gptr, gptr)) || (rc = upload(*ctx, &p_hs, hslot))
                || (rc = upload(*ctx, &ctx->ch_halo.node, order)) || (rc = dalloc(*ctx, &p_h, 3 * (size_t)gptr.back())))
                return fail(rc);
            ch.halo = p_h;
        } else {
            std::vector<int32_t> none(hc.cnode.size(), -1);
            if ((rc = upload(*ctx, &p_hs, none))) return fail(rc);
        }
        ch.hslot = p_hs;
        std::vector<uint16_t> fin_rel(hc.fin_slot.size());
        for (int c = 0; c < ch.n_chunks; ++c)
            for (int32_t j = hc.sstart[(size_t)c]; j < hc.sstart[(size_t)c + 1]; ++j)
                fin_rel[(size_t)j] = (uint16_t)(hc.fin_slot[(size_t)j] - hc.sstart[(size_t)c]);
        int32_t *p_fs, *p_fg;
        uint16_t *p_fr;
        if ((rc = dalloc(*ctx, &ch.cword, hc.cnode.size()))
            || (rc = dalloc(*ctx, &ch.cword0, (size_t)ch.n_chunks * kChunkThreads))
            || (rc = upload(*ctx, &p_fs, hc.fin_start)) || (rc = upload(*ctx, &p_fr, fin_rel))
            || (rc = upload(*ctx, &p_fg, hc.fin_slot)) || (rc = dalloc(*ctx, &ch.fin_dst, hc.cnode.size())))
            return fail(rc);
        ch.fin_start = p_fs;
        ch.fin_slot = p_fr;
        ch.fin_gslot = p_fg;
    }

    // default material mu = 1, lam = 1.5
    std::vector<double> ones((size_t)n_elems, 1.0), lam15((size_t)n_elems, 1.5);
    if ((rc = upload(*ctx, &ctx->mu, ones)) || (rc = upload(*ctx, &ctx->lam, lam15))) return fail(rc);
    m.mu = nullptr;   // uniform until efem_set_material gives a varying field
    m.lam = nullptr;
    m.mu0 = 1.0;
    m.lam0 = 1.5;
    if ((rc = dalloc(*ctx, &ctx->flags, 2)) || (rc = dalloc(*ctx, &ctx->partials, m.n_blocks))
        || (rc = dalloc(*ctx, &ctx->counter, 1)))
        return fail(rc);
    if (hipMemset(ctx->flags, 0, sizeof(int32_t)) != hipSuccess
        || hipMemset(ctx->counter, 0, sizeof(uint32_t)) != hipSuccess)
        return fail(hip_fail(hipGetLastError(), "hipMemset"));
    m.flags = ctx->flags;
    m.nmask = nullptr;
    if (ctx->ch.n_chunks > 0) {
        const hipError_t e = launch_chunk_words(*ctx);
        if (e != hipSuccess) return fail(hip_fail(e, "chunk staging words"));
    }

    if (scatter == EFEM_SCATTER_COLOR) {
        for (auto &lst : hb.colours) {
            int32_t *p;
            if ((rc = upload(*ctx, &p, lst))) return fail(rc);
            ctx->passes.push_back({p, (int32_t)lst.size()});
        }
    } else {
        ctx->passes.push_back({nullptr, m.n_blocks});
    }
    *out = ctx;
    return EFEM_OK;
}

int efem_set_stream(efem_ctx *ctx, void *stream)
{
    if (!ctx) return EFEM_ERR_INVALID;
    ctx->stream = (hipStream_t)stream;
    return EFEM_OK;
}

int efem_set_model(efem_ctx *ctx, int32_t model)
{
    if (!ctx) {
        set_error("efem_set_model: null context");
        return EFEM_ERR_INVALID;
    }
    if (model != EFEM_MODEL_NEO_HOOKE && model != EFEM_MODEL_LINEAR && model != EFEM_MODEL_TRANSPORT) {
        set_error("efem_set_model: unknown material model");
        return EFEM_ERR_INVALID;
    }
    ctx->model = model;
    return EFEM_OK;
}

int efem_set_velocity(efem_ctx *ctx, const double *omega)
{
    if (!ctx || !omega) {
        set_error("efem_set_velocity: null pointer");
        return EFEM_ERR_INVALID;
    }
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(omega[i])) {
            set_error("efem_set_velocity: omega must be finite");
            return EFEM_ERR_INVALID;
        }
    for (int i = 0; i < 3; ++i) ctx->omega[i] = omega[i];
    return EFEM_OK;
}

int efem_set_material(efem_ctx *ctx, const double *mu, const double *lam)
{
    if (!ctx || !mu || !lam) {
        set_error("efem_set_material: null pointer");
        return EFEM_ERR_INVALID;
    }
    DeviceGuard dg(ctx->device);
    // a uniform field is passed to the kernels as two scalars (no per-element loads)
    int32_t *flag = ctx->flags + 1;
    const int32_t one = 1;
    HIP_TRY(hipMemcpyAsync(flag, &one, sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(launch_uniform_check(mu, lam, ctx->n_elems, flag, ctx->stream));
    int32_t uni = 0;
    double v0[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&uni, flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(&v0[0], mu, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(&v0[1], lam, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (uni) {
        ctx->m.mu = ctx->m.lam = nullptr;
        ctx->m.mu0 = v0[0];
        ctx->m.lam0 = v0[1];
        return EFEM_OK;
    }
    HIP_TRY(launch_permute_elems(*ctx, mu, ctx->mu));
    HIP_TRY(launch_permute_elems(*ctx, lam, ctx->lam));
    ctx->m.mu = ctx->mu;
    ctx->m.lam = ctx->lam;
    return EFEM_OK;
}

int efem_set_coords(efem_ctx *ctx, const double *coords)
{
    if (!ctx || !coords) {
        set_error("efem_set_coords: null pointer");
        return EFEM_ERR_INVALID;
    }
    DeviceGuard dg(ctx->device);
    const size_t n = 3 * (size_t)ctx->n_nodes;
    HIP_TRY(hipMemcpyAsync(const_cast<double *>(ctx->m.X), coords, n * sizeof(double),
                           hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(launch_cast_f32(ctx->m.X, const_cast<float *>(ctx->m.Xf), (int64_t)n, ctx->stream));
    ctx->lin_prec = -1;   // a linearization point refers to the old coordinates
    return EFEM_OK;
}

int efem_set_dirichlet(efem_ctx *ctx, const uint8_t *mask)
{
    if (!ctx) return EFEM_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!mask) {
        ctx->m.nmask = nullptr;
    } else {
        if (!ctx->nmask) {
            int rc = dalloc(*ctx, &ctx->nmask, (size_t)ctx->n_nodes);
            if (rc) return rc;
        }
        HIP_TRY(launch_build_nmask(*ctx, mask, ctx->nmask));
        ctx->m.nmask = ctx->nmask;
    }
    // the chunk pass reads each slot's Dirichlet bits with its node id
    if (ctx->ch.n_chunks > 0) HIP_TRY(launch_chunk_words(*ctx));
    return EFEM_OK;
}

int efem_set_load(efem_ctx *ctx, const double *f)
{
    if (!ctx) return EFEM_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!f) {
        ctx->have_load = false;
        return EFEM_OK;
    }
    if (!ctx->fext) {
        int rc = dalloc(*ctx, &ctx->fext, (size_t)(3 * ctx->n_nodes));
        if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(ctx->fext, f, 3 * ctx->n_nodes * sizeof(double),
                           hipMemcpyDeviceToDevice, ctx->stream));
    ctx->have_load = true;
    return EFEM_OK;
}

#define CHECK_ARGS(cond, name)                         \
    do {                                               \
        if (!ctx || !(cond)) {                         \
            set_error(name ": null pointer");          \
            return EFEM_ERR_INVALID;                   \
        }                                              \
    } while (0)

// The transport model is non-variational: it has a residual and a tangent
// but no energy, so the energy and its parameter / coordinate derivatives
// are refused.
#define NEEDS_ENERGY(name)                                                              \
    do {                                                                                \
        if (ctx->model == EFEM_MODEL_TRANSPORT) {                                       \
            set_error(name ": the transport model has no energy (non-variational)");    \
            return EFEM_ERR_STATE;                                                      \
        }                                                                               \
    } while (0)

int efem_energy(efem_ctx *ctx, const double *u, double *psi)
{
    CHECK_ARGS(u && psi, "efem_energy");
    NEEDS_ENERGY("efem_energy");
    DeviceGuard dg(ctx->device);
    HIP_TRY(launch_energy(*ctx, u, psi));
    return EFEM_OK;
}

int efem_energy_noalloc(efem_ctx *ctx, const double *u, double *psi)
{
    CHECK_ARGS(u && psi, "efem_energy_noalloc");
    NEEDS_ENERGY("efem_energy_noalloc");
    if (ctx->m.n_blocks > kNoAllocBlocks) {
        set_error("efem_energy_noalloc: " + std::to_string(ctx->m.n_blocks) + " element blocks exceed the " +
                  std::to_string(kNoAllocBlocks) + " partials of the static array");
        return EFEM_ERR_INVALID;
    }
    DeviceGuard dg(ctx->device);
    HIP_TRY(launch_energy_noalloc(*ctx, u, psi));
    return EFEM_OK;
}

int efem_residual(efem_ctx *ctx, const double *u, double *r)
{
    CHECK_ARGS(u && r, "efem_residual");
    if (u == r) {
        set_error("efem_residual: r aliases u");
        return EFEM_ERR_INVALID;
    }
    DeviceGuard dg(ctx->device);
    HIP_TRY(launch_residual(*ctx, u, r));
    return EFEM_OK;
}

int efem_linearize(efem_ctx *ctx, const double *u, int32_t prec)
{
    CHECK_ARGS(u, "efem_linearize");
    if (prec != EFEM_F64 && prec != EFEM_F32) {
        set_error("efem_linearize: unknown precision");
        return EFEM_ERR_INVALID;
    }
    DeviceGuard dg(ctx->device);
    const size_t n = 3 * (size_t)ctx->n_nodes;
    int rc;
    if (prec == EFEM_F64) {
        if (!ctx->xlin && (rc = dalloc(*ctx, &ctx->xlin, 2 * n))) return rc;
        HIP_TRY(launch_lin_record(*ctx, u, ctx->xlin));
    } else {
        if (!ctx->ulin && (rc = dalloc(*ctx, &ctx->ulin, n))) return rc;
        HIP_TRY(launch_cast_f32(u, ctx->ulin, (int64_t)n, ctx->stream));
    }
    ctx->lin_prec = prec;
    return EFEM_OK;
}

static int hvp_impl(efem_ctx *ctx, const void *v, void *y, WriteMode mode, const char *name)
{
    if (!ctx || !v || !y) {
        set_error(std::string(name) + ": null pointer");
        return EFEM_ERR_INVALID;
    }
    if (v == y) {
        set_error(std::string(name) + ": y aliases v");
        return EFEM_ERR_INVALID;
    }
    if (ctx->lin_prec < 0) {
        set_error(std::string(name) + ": call efem_linearize first");
        return EFEM_ERR_STATE;
    }
    DeviceGuard dg(ctx->device);
    if (ctx->lin_prec == EFEM_F64)
        HIP_TRY(launch_hvp_f64(*ctx, ctx->xlin, (const double *)v, (double *)y, nullptr, mode));
    else
        HIP_TRY(launch_hvp_f32(*ctx, ctx->ulin, (const float *)v, (float *)y, nullptr, mode));
    return EFEM_OK;
}

int efem_hvp(efem_ctx *ctx, const void *v, void *y)
{
    return hvp_impl(ctx, v, y, WriteMode::Overwrite, "efem_hvp");
}

int efem_hvp_acc(efem_ctx *ctx, const void *v, void *y)
{
    return hvp_impl(ctx, v, y, WriteMode::Accumulate, "efem_hvp_acc");
}

int efem_hvp_zeroed(efem_ctx *ctx, const void *v, void *y)
{
    return hvp_impl(ctx, v, y, WriteMode::Zeroed, "efem_hvp_zeroed");
}

int efem_jacobi_diag(efem_ctx *ctx, const double *u, double *d)
{
    CHECK_ARGS(u && d, "efem_jacobi_diag");
    DeviceGuard dg(ctx->device);
    HIP_TRY(launch_diag(*ctx, u, d));
    return EFEM_OK;
}

int efem_jacobi_offdiag(efem_ctx *ctx, const double *u, double *o)
{
    CHECK_ARGS(u && o, "efem_jacobi_offdiag");
    if (ctx->model == EFEM_MODEL_TRANSPORT) {
        set_error("efem_jacobi_offdiag: neo-Hookean and linear models only");
        return EFEM_ERR_STATE;
    }
    DeviceGuard dg(ctx->device);
    HIP_TRY(launch_offdiag(*ctx, u, o));
    return EFEM_OK;
}

int efem_grad_material(efem_ctx *ctx, const double *u, double *dmu, double *dlam)
{
    CHECK_ARGS(u && dmu && dlam, "efem_grad_material");
    NEEDS_ENERGY("efem_grad_material");
    DeviceGuard dg(ctx->device);
    HIP_TRY(launch_grad_material(*ctx, u, dmu, dlam));
    return EFEM_OK;
}

int efem_residual_vjp_material(efem_ctx *ctx, const double *u, const double *w, double *dmu,
                               double *dlam)
{
    CHECK_ARGS(u && w && dmu && dlam, "efem_residual_vjp_material");
    NEEDS_ENERGY("efem_residual_vjp_material");
    DeviceGuard dg(ctx->device);
    HIP_TRY(launch_vjp_material(*ctx, u, w, dmu, dlam));
    return EFEM_OK;
}

int efem_grad_coords(efem_ctx *ctx, const double *u, double *dX)
{
    CHECK_ARGS(u && dX, "efem_grad_coords");
    NEEDS_ENERGY("efem_grad_coords");
    DeviceGuard dg(ctx->device);
    HIP_TRY(launch_grad_coords(*ctx, u, dX));
    return EFEM_OK;
}

int efem_status(efem_ctx *ctx, int32_t *flags)
{
    CHECK_ARGS(flags, "efem_status");
    DeviceGuard dg(ctx->device);
    HIP_TRY(hipMemcpyAsync(flags, ctx->flags, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->flags, 0, sizeof(int32_t), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return EFEM_OK;
}

int efem_get_info(efem_ctx *ctx, efem_info *info)
{
    CHECK_ARGS(info, "efem_get_info");
    info->n_blocks = ctx->m.n_blocks;
    info->n_colours = ctx->scatter == Scatter::Color ? (int32_t)ctx->passes.size() : 0;
    info->max_block_nodes = ctx->max_block_nodes;
    info->max_block_elems = ctx->max_block_elems;
    info->n_shared_nodes = ctx->n_shared;
    info->n_items = ctx->n_items;
    info->n_block_nodes = 0;
    // total block-node entries = nstart[n_blocks]
    int32_t tot = 0;
    HIP_TRY(hipMemcpy(&tot, ctx->m.nstart + ctx->m.n_blocks, sizeof(int32_t), hipMemcpyDeviceToHost));
    info->n_block_nodes = tot;
    info->n_chunks = ctx->ch.n_chunks;
    info->max_chunk_slots = ctx->max_chunk_slots;
    info->n_chunk_slots = ctx->n_chunk_slots;
    info->n_chunk_shared_nodes = ctx->n_ch_shared;

    return EFEM_OK;
}

}  // extern "C"
