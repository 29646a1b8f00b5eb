// Kernels of the colouring-based sparse tangent: indicator vectors of a
// colour, extraction of a colour's entries from K times that vector, and a
// CSR sparse matrix-vector product.
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

// y = K x.  The pattern is built per node: a row's nonzeros come in triples,
// the three components of one neighbour node in consecutive columns.  So a
// lane takes whole triples (one column index, three contiguous values and
// three contiguous x entries), kLanesPerRow lanes stride over the row's
// triples (coalesced), and a butterfly sums over them.
#ifndef EFEM_SPMV_LANES
#define EFEM_SPMV_LANES 16
#endif
constexpr int kLanesPerRow = EFEM_SPMV_LANES;
__global__ void __launch_bounds__(256) k_spmv(int64_t n_rows, const int64_t *__restrict__ row_ptr,
                                              const int32_t *__restrict__ col,
                                              const double *__restrict__ val,
                                              const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t row = tid / kLanesPerRow;
    const int sub = threadIdx.x % kLanesPerRow;
    double s = 0.0;
    if (row < n_rows) {
        const int64_t b = row_ptr[row], e = row_ptr[row + 1];
        for (int64_t k = b + 3 * sub; k < e; k += 3 * kLanesPerRow) {
            const int64_t c = col[k];
            s += val[k] * x[c] + val[k + 1] * x[c + 1] + val[k + 2] * x[c + 2];
        }
    }
#pragma unroll
    for (int off = kLanesPerRow / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kLanesPerRow);
    if (row < n_rows && sub == 0) y[row] = s;
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

hipError_t launch_spmv(hipStream_t s, int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                       const double *val, const double *x, double *y)
{
    hipLaunchKernelGGL(k_spmv, dim3(g256(n_rows * kLanesPerRow)), dim3(256), 0, s, n_rows, row_ptr, col,
                       val, x, y);
    return hipGetLastError();
}

}  // namespace efem
