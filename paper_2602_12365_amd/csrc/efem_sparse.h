// Sparse tangent by colouring (the paper's Alg. 2): declarations shared by
// sparse.cpp and kernels_sparse.hip.
#pragma once

#include <vector>

#include "efem_internal.h"

namespace efem {

// Per-context state: the CSR pattern of K (node 1-ring in 3x3 blocks), a
// distance-2 colouring of the DOFs, and the entries grouped by the colour of
// their column, so that the product of K with a colour's indicator vector
// gives every entry of that colour at once.
struct SparseState {
    int64_t n_rows = 0, nnz = 0;
    int32_t n_colours = 0, max_row = 0;
    double setup_seconds = 0.0;
    int64_t *row_ptr = nullptr;     // device [n_rows+1]
    int32_t *col = nullptr;         // device [nnz]
    // the same pattern by 3x3 blocks: node row i holds the blocks (i, j) of
    // the nodes j of its 1-ring, bcol[bptr[i] .. bptr[i+1]) (sorted); the
    // values of node row i start at 9 bptr[i]
    int64_t n_blocks = 0;
    int64_t *bptr = nullptr;        // device [n_nodes+1]
    int32_t *bcol = nullptr;        // device [n_blocks]
    int32_t *dof_colour = nullptr;  // device [n_rows]
    std::vector<int64_t> cstart;    // host [n_colours+1]: ranges into ent / ent_row
    int64_t *ent = nullptr;         // device [nnz]: entry index, grouped by column colour
    int32_t *ent_row = nullptr;     // device [nnz]: row of that entry
    double *seed = nullptr, *y = nullptr;   // device [n_rows] scratch
    std::vector<void *> owned;
};

hipError_t launch_seed(hipStream_t s, int64_t n, const int32_t *dof_colour, int32_t colour, double *seed);
hipError_t launch_extract(hipStream_t s, int64_t count, const int64_t *ent, const int32_t *ent_row,
                          const double *y, double *values);
hipError_t launch_block_spmv(hipStream_t s, int64_t n_nodes, const int64_t *bptr, const int32_t *bcol,
                             const double *val, const double *x, double *y);

}  // namespace efem
