// Internal declarations shared by the C-ABI host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "efem.h"

namespace efem {

// bnode entries: global node id in the low 30 bits, flags above.
constexpr uint32_t kGidMask = 0x3fffffffu;
constexpr uint32_t kShared = 0x80000000u;   // node touched by more than one block
constexpr uint32_t kFirst = 0x40000000u;    // colour scatter: this block writes first

// Device view of the blocked mesh, passed by value to every element kernel.
// A block's elements are its work items' elements: tetrahedron pairs first
// (partners adjacent in the internal order), then single elements, so item k of
// a block with np pairs covers internal elements e0 + k + min(k, np) (+1 for the
// second tetrahedron of a pair).
struct BlockMesh {
    int32_t n_blocks;
    int32_t pad;
    const int32_t *estart;    // [n_blocks+1] internal element ranges
    const int32_t *istart;    // [n_blocks+1] work item ranges (np = elements - items)
    const int32_t *nstart;    // [n_blocks+1] ranges into bnode
    const uint32_t *bnode;    // block-local node -> global id | flags
    const uint32_t *items;    // packed block-local node ids: Tet4 2 words per item
                              // (a | b<<10 | c<<20, d1 | d2<<10), Hex8 4 words (2 x 16 bit)
    const int32_t *eorig;     // [n_elems] internal -> caller element id
    const double *X;          // [n_nodes*3]
    const float *Xf;          // [n_nodes*3]
    const double *mu, *lam;   // [n_elems] internal order, or null: uniform (mu0, lam0)
    double mu0, lam0;
    const uint8_t *nmask;     // [n_nodes] bit c = component c prescribed, or null
    int32_t *flags;           // bit 0: det F <= 0 met
    // halo scatter: block-node entry i of a shared node stores its block sum
    // at halo[3 * hslot[i] + c]; the entries of one node are consecutive
    double *halo;             // [3 * number of shared entries]
    const int32_t *hslot;     // [n_block_nodes]
};

// Chunks: runs of consecutive blocks whose distinct nodes all stay resident in
// one workgroup's LDS while the blocks stream through it (the FP64 Tet4
// tangent action).  Node slots are numbered in order of first use; block b of
// a chunk brings the new slots [lo, hi) with bnew[b] = lo | hi << 16.  A node
// touched by more than one chunk is shared: its chunk sum goes to a halo entry
// (hslot), and the nodes' entries are consecutive and in chunk order.
constexpr int kChunkCap = 1472;      // node slots per chunk (23 groups of 64)
constexpr int kChunkThreads = 768;   // 12 waves per workgroup: 3 per SIMD
// LDS of a chunk: five 16-byte record pieces and three FP64 sums per slot, and
// one 64-slot group of staging words per wave, and the chunk's block table
constexpr int kPieceBytes = kChunkCap * 16;
constexpr int kChunkSteps = 32;      // blocks per chunk at most
constexpr int kChunkLds = 5 * kPieceBytes + kChunkCap * 24 + kChunkThreads * 4 + (4 * kChunkSteps + 3) * 4;
// staging word of a chunk slot: global id | Dirichlet bits << 28
constexpr uint32_t kStageGid = 0x0fffffffu;
struct ChunkMesh {
    int32_t n_chunks;
    int32_t pad;
    const int32_t *bstart;    // [n_chunks+1] block ranges
    const int32_t *sstart;    // [n_chunks+1] slot ranges into cnode / hslot
    const uint32_t *bnew;     // [n_blocks] chunk-relative new-slot range of each block
    const uint32_t *cnode;    // slot -> global id | kShared
    uint32_t *cword;          // slot -> staging word (global id | Dirichlet bits << 28)
    uint32_t *cword0;         // [n_chunks * kChunkThreads] the first block's staging words,
                              // indexed by chunk and thread (no load of sstart in front)
    const int4 *hdr;          // [2 * n_chunks] per chunk: {b0, nsteps, s0, ns},
                              // {istart[b0], items of block b0, bnew[b0 + 1] (0 if none), 0}
    const uint32_t *items;    // chunk-slot connectivity, 2 words per item, 11-bit ids:
                              // a | b<<11 | (d1 & 1023)<<22,  c | d2<<11 | (d1 >> 10)<<22
    const uint16_t *iperm;    // [items] each item's position in the block pass's order
                              // (where the element arrays find it)
    const int32_t *hslot;     // [slots] halo entry of a shared slot, else -1
    double *halo;             // [3 * entries]
    // write-out in the order the slots' sums become final: the slots final
    // after block b are entries [fin_start[b], fin_start[b + 1]) (a chunk's
    // entries lie in its slot range); fin_slot is the chunk-relative slot,
    // fin_dst where its sum goes: kShared | halo entry, or global id |
    // Dirichlet bits << 28 (rebuilt with the staging words); fin_gslot the
    // global slot, for that rebuild
    const int32_t *fin_start;   // [n_blocks + 1]
    const uint16_t *fin_slot;   // [slots]
    const int32_t *fin_gslot;   // [slots]
    uint32_t *fin_dst;          // [slots]
};

// Halo entries of the shared nodes, grouped by how many blocks (or chunks)
// share a node: the nodes with c entries, c = 2 .. kSegMax, form segment c, in
// which node p's entries are the c consecutive slots base[c] + c p + k.  So a
// gather thread finds its slots from its own index, with no load in front.
// Nodes with more entries come last and use a slot-range array (gptr).
constexpr int kSegMax = 16;
struct HaloSegs {
    int32_t start[kSegMax + 2];   // start[c]: first shared-node index of segment c
                                  // (c = 2 .. kSegMax); start[kSegMax + 1] = the others
    int32_t base[kSegMax + 1];    // base[c]: first slot of segment c
    int32_t n;                    // shared nodes
};
struct HaloMap {
    HaloSegs seg{};
    int32_t *gptr = nullptr;      // [others + 1] slot ranges of the nodes past the segments
    int32_t *node = nullptr;      // [n] global node id of shared node i
};

// How block sums reach nodes shared between blocks:
//   Halo:   plain stores into a per-entry buffer, then a gather kernel sums each
//           shared node's entries in block order (no device atomics);
//   Color:  one pass per block colour, read-modify-write;
//   Atomic: device-scope atomic adds.
enum class Scatter { Halo = 0, Color = 1, Atomic = 2 };

// One launch over a set of blocks: all blocks (list == null) or one colour.
struct Pass {
    const int32_t *list;
    int32_t count;
};

struct Ctx;

// ---- kernel launchers (kernels_*.hip) -------------------------------------
// All return hipError_t of the launch.  T = double or float.
hipError_t launch_energy(const Ctx &c, const double *u, double *psi);
// The energy with its per-block partials in a file-scope device array of
// kNoAllocBlocks doubles (no allocation).  noalloc_setup(device) takes the
// array's device address once per device, with that device current; the
// launch returns hipErrorNotInitialized if it has not run for c.device.
constexpr int kNoAllocBlocks = 1 << 16;
hipError_t noalloc_setup(int device);
hipError_t launch_energy_noalloc(const Ctx &c, const double *u, double *psi);
hipError_t launch_residual(const Ctx &c, const double *u, double *r);
// How a nodal output is written:
//   Overwrite:  y = K v (halo scatter: block pass, then the gather of shared
//               nodes; atomic scatter: a fill pre-pass clears y, prescribed
//               components to their value, before the block pass adds into
//               shared nodes);
//   Accumulate: y += K v (plain read-modify-write on block-private nodes);
//   Zeroed:     y = K v for a y that holds zeros on entry (no fill pre-pass).
enum class WriteMode { Overwrite = 0, Accumulate = 1, Zeroed = 2 };
hipError_t launch_hvp_f64(const Ctx &c, const double *xlin, const double *v, double *y,
                          const int32_t *skip, WriteMode mode);
hipError_t launch_hvp_f32(const Ctx &c, const float *ulin, const float *v, float *y,
                          const int32_t *skip, WriteMode mode);
hipError_t launch_diag(const Ctx &c, const double *u, double *d);
// (K01, K02, K12) of every node's 3x3 diagonal block of K(u), unmasked
hipError_t launch_offdiag(const Ctx &c, const double *u, double *o);
hipError_t launch_grad_material(const Ctx &c, const double *u, double *dmu, double *dlam);
hipError_t launch_vjp_material(const Ctx &c, const double *u, const double *w, double *dmu,
                               double *dlam);
hipError_t launch_grad_coords(const Ctx &c, const double *u, double *g);

// small utility kernels (kernels_util.hip)
hipError_t launch_permute_elems(const Ctx &c, const double *src, double *dst);
hipError_t launch_build_nmask(const Ctx &c, const uint8_t *dofmask, uint8_t *nmask);
// xrec[6 i + c] = X[3 i + c], xrec[6 i + 3 + c] = X[3 i + c] + u[3 i + c]
hipError_t launch_lin_record(const Ctx &c, const double *u, double *xrec);
hipError_t launch_cast_f32(const double *src, float *dst, int64_t n, hipStream_t s);
// staging words of the chunk slots from cnode and the node mask (null = none)
hipError_t launch_chunk_words(const Ctx &c);
// flag = 1 if a[i] == a[0] and b[i] == b[0] for all i (flag must hold 1 on entry)
hipError_t launch_uniform_check(const double *a, const double *b, int64_t n, int32_t *flag,
                                hipStream_t s);

// ---- context ---------------------------------------------------------------
struct Ctx {
    int elem = 0, nen = 4, nq = 1;
    int32_t model = EFEM_MODEL_NEO_HOOKE;
    double omega[3] = {0.0, 0.0, 0.0};   // transport model: velocity b(x) = omega x x
    int64_t n_nodes = 0, n_elems = 0, n_items = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    Scatter scatter = Scatter::Halo;
    int threads = 256;
    int max_block_nodes = 0;        // max nodes over blocks (LDS sizing)
    int max_block_elems = 0;
    // chunk pass of the FP64 Tet4 tangent action (n_chunks = 0: block pass only)
    ChunkMesh ch{};
    HaloMap ch_halo;                  // gather of the chunk pass's shared nodes
    int64_t n_ch_shared = 0;          // nodes in more than one chunk
    int64_t n_chunk_slots = 0;        // sum over chunks of distinct nodes
    int max_chunk_slots = 0;

    // device buffers owned by the context
    BlockMesh m{};
    std::vector<void *> owned;      // every hipMalloc of the context
    int64_t n_shared = 0;               // nodes touched by several blocks
    // halo scatter: shared node i = halo.node[i] sums its halo entries (its
    // blocks in block order)
    HaloMap halo;
    std::vector<Pass> passes;           // colour lists (Color) or one pass (Atomic)
    double *partials = nullptr;         // [n_blocks] per-block energy partials
    uint32_t *counter = nullptr;        // last-block-done ticket
    double *mu = nullptr, *lam = nullptr;
    uint8_t *nmask = nullptr;
    int32_t *flags = nullptr;
    // external nodal forces of the final load step (efem_set_load)
    double *fext = nullptr;
    bool have_load = false;

    // linearization point
    int lin_prec = -1;
    double *xlin = nullptr;   // [n_nodes][6] = (X, X + u) per node (FP64 tangent)
    float *ulin = nullptr;    // u in FP32 (FP32 tangent)

    // learned preconditioner state (precond.cpp) and the host connectivity it
    // builds the node 1-ring from
    void *mlp = nullptr;
    // sparse tangent by colouring (sparse.cpp), built on first use
    void *sparse = nullptr;
    std::vector<int32_t> conn_host;
};

// learned preconditioner resources of a context (precond.cpp)
void mlp_release(Ctx &c);
// sparse-tangent resources of a context (sparse.cpp)
void sparse_release(Ctx &c);

// error helpers (api.cpp)
void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);

}  // namespace efem
