// Small streaming kernels: material permutation, Dirichlet node masks,
// linearization caches.
#include "efem_internal.h"

namespace efem {

__global__ void k_permute_elems(const int32_t *__restrict__ eorig, int64_t n,
                                const double *__restrict__ src, double *__restrict__ dst)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) dst[e] = src[eorig[e]];
}

__global__ void k_build_nmask(const uint8_t *__restrict__ dofmask, int64_t n_nodes,
                              uint8_t *__restrict__ nmask)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    nmask[i] = (uint8_t)((dofmask[3 * i] != 0) | ((dofmask[3 * i + 1] != 0) << 1)
                         | ((dofmask[3 * i + 2] != 0) << 2));
}

// the linearization record of each node: (X, X + u), 48 contiguous bytes
__global__ void k_lin_record(const double *__restrict__ X, const double *__restrict__ u, int64_t n,
                             double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // DOF
    if (i < n) {
        const int64_t node = i / 3, c = i - 3 * node;
        const double x = X[i];
        out[6 * node + c] = x;
        out[6 * node + 3 + c] = x + u[i];
    }
}

__global__ void k_cast_f32(const double *__restrict__ src, int64_t n, float *__restrict__ dst)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

__global__ void k_uniform_check(const double *__restrict__ a, const double *__restrict__ b,
                                int64_t n, int32_t *flag)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n && (a[i] != a[0] || b[i] != b[0])) atomicAnd(flag, 0);
}

static unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_uniform_check(const double *a, const double *b, int64_t n, int32_t *flag,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_uniform_check, dim3(grid_for(n)), dim3(256), 0, s, a, b, n, flag);
    return hipGetLastError();
}

hipError_t launch_permute_elems(const Ctx &c, const double *src, double *dst)
{
    hipLaunchKernelGGL(k_permute_elems, dim3(grid_for(c.n_elems)), dim3(256), 0, c.stream,
                       c.m.eorig, c.n_elems, src, dst);
    return hipGetLastError();
}

hipError_t launch_build_nmask(const Ctx &c, const uint8_t *dofmask, uint8_t *nmask)
{
    hipLaunchKernelGGL(k_build_nmask, dim3(grid_for(c.n_nodes)), dim3(256), 0, c.stream, dofmask,
                       c.n_nodes, nmask);
    return hipGetLastError();
}

hipError_t launch_lin_record(const Ctx &c, const double *u, double *xrec)
{
    hipLaunchKernelGGL(k_lin_record, dim3(grid_for(3 * c.n_nodes)), dim3(256), 0, c.stream, c.m.X, u,
                       3 * c.n_nodes, xrec);
    return hipGetLastError();
}

// staging word of each chunk slot: its node id and the node's Dirichlet bits
__global__ void k_chunk_words(int64_t n, const uint32_t *__restrict__ cnode, const uint8_t *__restrict__ nmask,
                              uint32_t *__restrict__ cword)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        const uint32_t g = cnode[i] & kStageGid;
        cword[i] = g | (nmask ? (uint32_t)(nmask[g] & 7u) << 28 : 0u);
    }
}

// the same words for the first block of every chunk, by (chunk, thread):
// thread t of chunk c stages slot t of the chunk if t is below the block's
// new-slot end, else its word is all ones (node ids stay below 2^28)
__global__ void k_chunk_words0(ChunkMesh ch, const uint8_t *__restrict__ nmask)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)ch.n_chunks * kChunkThreads) return;
    const int c = (int)(i / kChunkThreads), t = (int)(i % kChunkThreads);
    const int hi = (int)(ch.bnew[ch.bstart[c]] >> 16);
    uint32_t w = 0xffffffffu;   // no slot for this thread
    if (t < hi) {
        const uint32_t g = ch.cnode[ch.sstart[c] + t] & kStageGid;
        w = g | (nmask ? (uint32_t)(nmask[g] & 7u) << 28 : 0u);
    }
    ch.cword0[i] = w;
}

// where slot sums go in the write-out order: kShared | halo entry for a node
// other chunks share, else global id | Dirichlet bits << 28
__global__ void k_chunk_fin_dst(int64_t n, ChunkMesh ch, const uint8_t *__restrict__ nmask)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t gs = ch.fin_gslot[j];
    const int32_t hs = ch.hslot[gs];
    const uint32_t g = ch.cnode[gs] & kStageGid;
    ch.fin_dst[j] = hs >= 0 ? (kShared | (uint32_t)hs) : (g | (nmask ? (uint32_t)(nmask[g] & 7u) << 28 : 0u));
}

hipError_t launch_chunk_words(const Ctx &c)
{
    hipLaunchKernelGGL(k_chunk_fin_dst, dim3(grid_for(c.n_chunk_slots)), dim3(256), 0, c.stream, c.n_chunk_slots,
                       c.ch, c.m.nmask);
    hipLaunchKernelGGL(k_chunk_words, dim3(grid_for(c.n_chunk_slots)), dim3(256), 0, c.stream, c.n_chunk_slots,
                       c.ch.cnode, c.m.nmask, c.ch.cword);
    hipLaunchKernelGGL(k_chunk_words0, dim3(grid_for((int64_t)c.ch.n_chunks * kChunkThreads)), dim3(256), 0,
                       c.stream, c.ch, c.m.nmask);
    return hipGetLastError();
}

hipError_t launch_cast_f32(const double *src, float *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cast_f32, dim3(grid_for(n)), dim3(256), 0, s, src, n, dst);
    return hipGetLastError();
}

}  // namespace efem
