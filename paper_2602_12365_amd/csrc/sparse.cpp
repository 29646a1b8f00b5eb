// Sparse tangent by colouring (the paper's Alg. 2): the tangent K(u) is
// recovered from a few tangent actions.  Two DOFs may share a colour when no
// row of K has both as nonzero columns, i.e. when their nodes are more than
// two element-adjacency steps apart (a distance-2 colouring of the node
// graph) and they are not components of one node; the product of K with the
// indicator vector of a colour then holds, in each row, the single entry of
// that colour.  The pattern is the node 1-ring in 3x3 blocks.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>

#include "efem_sparse.h"

namespace efem {

namespace {

#define TRY(call)                                              \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(e_, #call);      \
    } while (0)

template <class T>
int alloc_into(SparseState &S, T **p, size_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    S.owned.push_back(q);
    *p = static_cast<T *>(q);
    return EFEM_OK;
}

template <class T>
int upload_into(SparseState &S, T **p, const std::vector<T> &v)
{
    int rc = alloc_into(S, p, v.size());
    if (rc) return rc;
    if (!v.empty()) TRY(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return EFEM_OK;
}

void free_state(SparseState *S)
{
    for (void *p : S->owned) (void)hipFree(p);
    delete S;
}

// node -> nodes sharing an element with it (itself included), sorted
void node_ring(const Ctx &c, std::vector<int64_t> &ptr, std::vector<int32_t> &idx)
{
    const int64_t nn = c.n_nodes, ne = c.n_elems;
    const int nen = c.nen;
    std::vector<int64_t> eptr((size_t)nn + 1, 0);
    for (int64_t k = 0; k < ne * nen; ++k) eptr[(size_t)c.conn_host[(size_t)k] + 1] += 1;
    for (int64_t i = 0; i < nn; ++i) eptr[(size_t)i + 1] += eptr[(size_t)i];
    std::vector<int32_t> elist((size_t)eptr[(size_t)nn]);
    std::vector<int64_t> fill(eptr.begin(), eptr.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < nen; ++a)
            elist[(size_t)fill[(size_t)c.conn_host[(size_t)(e * nen + a)]]++] = (int32_t)e;
    ptr.assign(1, 0);
    idx.clear();
    std::vector<int32_t> cand;
    for (int64_t i = 0; i < nn; ++i) {
        cand.clear();
        for (int64_t k = eptr[(size_t)i]; k < eptr[(size_t)i + 1]; ++k) {
            const int64_t e = elist[(size_t)k];
            for (int a = 0; a < nen; ++a) cand.push_back(c.conn_host[(size_t)(e * nen + a)]);
        }
        if (cand.empty()) cand.push_back((int32_t)i);
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        idx.insert(idx.end(), cand.begin(), cand.end());
        ptr.push_back((int64_t)idx.size());
    }
}

int build(Ctx &c, SparseState &S)
{
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<int64_t> rp;
    std::vector<int32_t> ri;
    node_ring(c, rp, ri);
    const int64_t nn = c.n_nodes;
    // greedy distance-2 colouring of the nodes, in node order
    std::vector<int32_t> ncol((size_t)nn, -1), stamp;
    int32_t n_node_colours = 0;
    for (int64_t i = 0; i < nn; ++i) {
        if ((int64_t)stamp.size() < n_node_colours + 1) stamp.resize((size_t)n_node_colours + 1, -1);
        for (int64_t a = rp[(size_t)i]; a < rp[(size_t)i + 1]; ++a) {
            const int32_t k = ri[(size_t)a];
            for (int64_t b = rp[(size_t)k]; b < rp[(size_t)k + 1]; ++b) {
                const int32_t j = ri[(size_t)b];
                if (j != i && ncol[(size_t)j] >= 0) stamp[(size_t)ncol[(size_t)j]] = (int32_t)i;
            }
        }
        int32_t col = 0;
        while (col < n_node_colours && stamp[(size_t)col] == (int32_t)i) ++col;
        ncol[(size_t)i] = col;
        n_node_colours = std::max(n_node_colours, col + 1);
    }
    // CSR over DOFs: row 3i+a has columns 3j+b for j in ring(i), b = 0..2
    const int64_t n_rows = 3 * nn;
    std::vector<int64_t> row_ptr((size_t)n_rows + 1, 0);
    int32_t max_row = 0;
    for (int64_t i = 0; i < nn; ++i) {
        const int64_t len = 3 * (rp[(size_t)i + 1] - rp[(size_t)i]);
        max_row = std::max<int32_t>(max_row, (int32_t)len);
        for (int a = 0; a < 3; ++a) row_ptr[(size_t)(3 * i + a) + 1] = row_ptr[(size_t)(3 * i + a)] + len;
    }
    const int64_t nnz = row_ptr[(size_t)n_rows];
    if (nnz > INT32_MAX) {
        set_error("efem_sparse_setup: more than 2^31 nonzeros");
        return EFEM_ERR_INVALID;
    }
    std::vector<int32_t> col((size_t)nnz), dcol((size_t)n_rows);
    for (int64_t i = 0; i < nn; ++i)
        for (int a = 0; a < 3; ++a) {
            int64_t k = row_ptr[(size_t)(3 * i + a)];
            for (int64_t t = rp[(size_t)i]; t < rp[(size_t)i + 1]; ++t)
                for (int b = 0; b < 3; ++b) col[(size_t)k++] = 3 * ri[(size_t)t] + b;
            dcol[(size_t)(3 * i + a)] = 3 * ncol[(size_t)i] + a;
        }
    // entries grouped by the colour of their column (counting sort)
    const int32_t n_colours = 3 * n_node_colours;
    std::vector<int64_t> cstart((size_t)n_colours + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) cstart[(size_t)dcol[(size_t)col[(size_t)k]] + 1] += 1;
    for (int32_t q = 0; q < n_colours; ++q) cstart[(size_t)q + 1] += cstart[(size_t)q];
    std::vector<int64_t> ent((size_t)nnz), pos(cstart.begin(), cstart.end() - 1);
    std::vector<int32_t> ent_row((size_t)nnz);
    for (int64_t r = 0; r < n_rows; ++r)
        for (int64_t k = row_ptr[(size_t)r]; k < row_ptr[(size_t)r + 1]; ++k) {
            const int64_t p = pos[(size_t)dcol[(size_t)col[(size_t)k]]]++;
            ent[(size_t)p] = k;
            ent_row[(size_t)p] = (int32_t)r;
        }
    int rc;
    if ((rc = upload_into(S, &S.row_ptr, row_ptr)) || (rc = upload_into(S, &S.col, col))
        || (rc = upload_into(S, &S.dof_colour, dcol)) || (rc = upload_into(S, &S.ent, ent))
        || (rc = upload_into(S, &S.ent_row, ent_row)) || (rc = alloc_into(S, &S.seed, (size_t)n_rows))
        || (rc = alloc_into(S, &S.y, (size_t)n_rows)) || (rc = upload_into(S, &S.bptr, rp))
        || (rc = upload_into(S, &S.bcol, ri)))
        return rc;
    S.n_blocks = (int64_t)ri.size();
    S.n_rows = n_rows;
    S.nnz = nnz;
    S.n_colours = n_colours;
    S.max_row = max_row;
    S.cstart = std::move(cstart);
    S.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return EFEM_OK;
}

}  // namespace

void sparse_release(Ctx &c)
{
    if (c.sparse) free_state(static_cast<SparseState *>(c.sparse));
    c.sparse = nullptr;
}

}  // namespace efem

using namespace efem;

struct efem_ctx : Ctx {};

extern "C" {

int efem_sparse_setup(efem_ctx *ctx, efem_sparse_info *info)
{
    if (!ctx || !info) {
        set_error("efem_sparse_setup: null pointer");
        return EFEM_ERR_INVALID;
    }
    if (!ctx->sparse) {
        auto *S = new (std::nothrow) SparseState();
        if (!S) return EFEM_ERR_OOM;
        int dev_prev = -1;
        (void)hipGetDevice(&dev_prev);
        if (dev_prev != ctx->device) (void)hipSetDevice(ctx->device);
        const int rc = build(*ctx, *S);
        if (dev_prev >= 0 && dev_prev != ctx->device) (void)hipSetDevice(dev_prev);
        if (rc) {
            free_state(S);
            return rc;
        }
        ctx->sparse = S;
    }
    const SparseState &S = *static_cast<SparseState *>(ctx->sparse);
    info->n_rows = S.n_rows;
    info->nnz = S.nnz;
    info->n_colours = S.n_colours;
    info->max_row = S.max_row;
    info->setup_seconds = S.setup_seconds;
    info->n_blocks = S.n_blocks;
    return EFEM_OK;
}

int efem_sparse_pattern(efem_ctx *ctx, int64_t *row_ptr, int32_t *col, int32_t *dof_colour)
{
    if (!ctx || !row_ptr || !col || !dof_colour) {
        set_error("efem_sparse_pattern: null pointer");
        return EFEM_ERR_INVALID;
    }
    if (!ctx->sparse) {
        set_error("efem_sparse_pattern: call efem_sparse_setup first");
        return EFEM_ERR_STATE;
    }
    const SparseState &S = *static_cast<SparseState *>(ctx->sparse);
    TRY(hipMemcpyAsync(row_ptr, S.row_ptr, (S.n_rows + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                       ctx->stream));
    TRY(hipMemcpyAsync(col, S.col, S.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
    TRY(hipMemcpyAsync(dof_colour, S.dof_colour, S.n_rows * sizeof(int32_t), hipMemcpyDeviceToDevice,
                       ctx->stream));
    return EFEM_OK;
}

int efem_sparse_assemble(efem_ctx *ctx, const double *u, double *values)
{
    if (!ctx || !u || !values) {
        set_error("efem_sparse_assemble: null pointer");
        return EFEM_ERR_INVALID;
    }
    if (!ctx->sparse) {
        set_error("efem_sparse_assemble: call efem_sparse_setup first");
        return EFEM_ERR_STATE;
    }
    const int rc = efem_linearize(ctx, u, EFEM_F64);
    if (rc) return rc;
    const SparseState &S = *static_cast<SparseState *>(ctx->sparse);
    for (int32_t q = 0; q < S.n_colours; ++q) {
        const int64_t b = S.cstart[(size_t)q], cnt = S.cstart[(size_t)q + 1] - b;
        if (cnt == 0) continue;
        TRY(launch_seed(ctx->stream, S.n_rows, S.dof_colour, q, S.seed));
        TRY(launch_hvp_f64(*ctx, ctx->xlin, S.seed, S.y, nullptr, WriteMode::Overwrite));
        TRY(launch_extract(ctx->stream, cnt, S.ent + b, S.ent_row + b, S.y, values));
    }
    return EFEM_OK;
}

int efem_sparse_spmv(efem_ctx *ctx, const double *values, const double *x, double *y)
{
    if (!ctx || !values || !x || !y) {
        set_error("efem_sparse_spmv: null pointer");
        return EFEM_ERR_INVALID;
    }
    if (!ctx->sparse) {
        set_error("efem_sparse_spmv: call efem_sparse_setup first");
        return EFEM_ERR_STATE;
    }
    const SparseState &S = *static_cast<SparseState *>(ctx->sparse);
    TRY(launch_block_spmv(ctx->stream, S.n_rows / 3, S.bptr, S.bcol, values, x, y));
    return EFEM_OK;
}

int efem_sparse_block_pattern(efem_ctx *ctx, int64_t *block_ptr, int32_t *block_col)
{
    if (!ctx || !block_ptr || !block_col) {
        set_error("efem_sparse_block_pattern: null pointer");
        return EFEM_ERR_INVALID;
    }
    if (!ctx->sparse) {
        set_error("efem_sparse_block_pattern: call efem_sparse_setup first");
        return EFEM_ERR_STATE;
    }
    const SparseState &S = *static_cast<SparseState *>(ctx->sparse);
    TRY(hipMemcpyAsync(block_ptr, S.bptr, (S.n_rows / 3 + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                       ctx->stream));
    TRY(hipMemcpyAsync(block_col, S.bcol, std::max<int64_t>(S.n_blocks, 0) * sizeof(int32_t),
                       hipMemcpyDeviceToDevice, ctx->stream));
    return EFEM_OK;
}

}  // extern "C"
