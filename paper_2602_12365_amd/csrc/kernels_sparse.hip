// Kernels of the colouring-based sparse tangent: indicator vectors of a
// colour, extraction of a colour's entries from K times that vector, and the
// sparse matrix-vector product by 3x3 blocks.
#include "efem_sparse.h"

namespace efem {

__global__ void __launch_bounds__(256) k_seed(int64_t n, const int32_t *__restrict__ dof_colour,
                                              int32_t colour, double *__restrict__ seed)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < n) seed[j] = dof_colour[j] == colour ? 1.0 : 0.0;
}

// values[ent[t]] = y[ent_row[t]]: with a distance-2 colouring, row i meets at
// most one column of the colour, so (K s)_i is exactly that entry
__global__ void __launch_bounds__(256) k_extract(int64_t count, const int64_t *__restrict__ ent,
                                                 const int32_t *__restrict__ ent_row,
                                                 const double *__restrict__ y, double *__restrict__ values)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < count) values[ent[t]] = y[ent_row[t]];
}

// y = K x by 3x3 blocks.  The values keep the CSR order: node row i's
// three component rows follow each other, 3 len_i values each (len_i blocks),
// block t's row a at 3t of component row a.  A group of kLanesPerNode lanes
// takes one node row; lane t takes blocks t, t + kLanesPerNode, ...: one
// column index and one x triple per block, the block's three rows from the
// three component-row streams (consecutive lanes on consecutive 24-byte
// triples of each).  A butterfly over the group sums the three outputs.
constexpr int kLanesPerNode = 16;
__global__ void __launch_bounds__(256) k_block_spmv(int64_t n_nodes, const int64_t *__restrict__ bptr,
                                                    const int32_t *__restrict__ bcol,
                                                    const double *__restrict__ val,
                                                    const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kLanesPerNode;
    const int sub = threadIdx.x % kLanesPerNode;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (i < n_nodes) {
        const int64_t b = bptr[i], len = bptr[i + 1] - b;
        const double *r0 = val + 9 * b, *r1 = r0 + 3 * len, *r2 = r1 + 3 * len;
        for (int64_t t = sub; t < len; t += kLanesPerNode) {
            const int64_t c = 3 * (int64_t)bcol[b + t];
            const double x0 = x[c], x1 = x[c + 1], x2 = x[c + 2];
            s0 += r0[3 * t] * x0 + r0[3 * t + 1] * x1 + r0[3 * t + 2] * x2;
            s1 += r1[3 * t] * x0 + r1[3 * t + 1] * x1 + r1[3 * t + 2] * x2;
            s2 += r2[3 * t] * x0 + r2[3 * t + 1] * x1 + r2[3 * t + 2] * x2;
        }
    }
#pragma unroll
    for (int off = kLanesPerNode / 2; off > 0; off >>= 1) {
        s0 += __shfl_xor(s0, off, kLanesPerNode);
        s1 += __shfl_xor(s1, off, kLanesPerNode);
        s2 += __shfl_xor(s2, off, kLanesPerNode);
    }
    if (i < n_nodes && sub < 3) y[3 * i + sub] = sub == 0 ? s0 : (sub == 1 ? s1 : s2);
}

static unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_seed(hipStream_t s, int64_t n, const int32_t *dof_colour, int32_t colour, double *seed)
{
    hipLaunchKernelGGL(k_seed, dim3(g256(n)), dim3(256), 0, s, n, dof_colour, colour, seed);
    return hipGetLastError();
}

hipError_t launch_extract(hipStream_t s, int64_t count, const int64_t *ent, const int32_t *ent_row,
                          const double *y, double *values)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_extract, dim3(g256(count)), dim3(256), 0, s, count, ent, ent_row, y, values);
    return hipGetLastError();
}

hipError_t launch_block_spmv(hipStream_t s, int64_t n_nodes, const int64_t *bptr, const int32_t *bcol,
                             const double *val, const double *x, double *y)
{
    if (n_nodes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_spmv, dim3(g256(n_nodes * kLanesPerNode)), dim3(256), 0, s, n_nodes, bptr, bcol,
                       val, x, y);
    return hipGetLastError();
}

}  // namespace efem
