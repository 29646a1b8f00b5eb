// Learned CG preconditioner: per-context state, the node 1-ring graph, and
// the C-ABI of the preconditioner and of its training.
#include <algorithm>
#include <cstring>
#include <vector>

#include "efem_mlp.h"

namespace efem {

#define TRY(call)                                              \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(e_, #call);      \
    } while (0)

void mlp_release(Ctx &c)
{
    auto *M = static_cast<MlpState *>(c.mlp);
    if (!M) return;
    for (void *p : M->owned) (void)hipFree(p);
    delete M;
    c.mlp = nullptr;
}

template <class T>
static int malloc_into(MlpState &M, T **p, size_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    M.owned.push_back(q);
    *p = static_cast<T *>(q);
    return EFEM_OK;
}

// Node 1-ring (nodes sharing an element, excluding the node), sorted per node.
static void build_ring(const Ctx &c, std::vector<int64_t> &ptr, std::vector<int32_t> &idx)
{
    const int64_t nn = c.n_nodes, ne = c.n_elems;
    const int nen = c.nen;
    std::vector<int64_t> eptr((size_t)nn + 1, 0);
    for (int64_t k = 0; k < ne * nen; ++k) eptr[(size_t)c.conn_host[(size_t)k] + 1] += 1;
    for (int64_t i = 0; i < nn; ++i) eptr[(size_t)i + 1] += eptr[(size_t)i];
    std::vector<int32_t> elist((size_t)eptr[(size_t)nn]);
    std::vector<int64_t> fill(eptr.begin(), eptr.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < nen; ++a) elist[(size_t)fill[(size_t)c.conn_host[(size_t)(e * nen + a)]]++] = (int32_t)e;
    ptr.assign((size_t)nn + 1, 0);
    idx.clear();
    std::vector<int32_t> cand;
    for (int64_t i = 0; i < nn; ++i) {
        cand.clear();
        for (int64_t p = eptr[(size_t)i]; p < eptr[(size_t)i + 1]; ++p) {
            const int32_t e = elist[(size_t)p];
            for (int a = 0; a < nen; ++a) {
                const int32_t j = c.conn_host[(size_t)(e * nen + a)];
                if (j != i) cand.push_back(j);
            }
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        idx.insert(idx.end(), cand.begin(), cand.end());
        ptr[(size_t)i + 1] = (int64_t)idx.size();
    }
}

// Create the state (graph + buffers) on first use.
MlpState *mlp_state(Ctx &c, int *rc)
{
    *rc = EFEM_OK;
    if (c.mlp) return static_cast<MlpState *>(c.mlp);
    auto *M = new (std::nothrow) MlpState();
    if (!M) {
        *rc = EFEM_ERR_OOM;
        return nullptr;
    }
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
    build_ring(c, ptr, idx);
    const int64_t nn = c.n_nodes;
    int r;
    if ((r = malloc_into(*M, &M->ptr, ptr.size())) || (r = malloc_into(*M, &M->idx, idx.size()))
        || (r = malloc_into(*M, &M->W, kP)) || (r = malloc_into(*M, &M->X, (size_t)nn * kInPad))
        || (r = malloc_into(*M, &M->scale, (size_t)nn)) || (r = malloc_into(*M, &M->g4, (size_t)nn + 1))
        || (r = malloc_into(*M, &M->dinv, 3 * (size_t)nn))
        || (r = malloc_into(*M, &M->z, 3 * (size_t)nn)) || (r = malloc_into(*M, &M->zold, 3 * (size_t)nn))
        || (r = malloc_into(*M, &M->prz, 2048)) || (r = malloc_into(*M, &M->gpart, (size_t)kGradBlocks * kP))
        || (r = malloc_into(*M, &M->lpart, kGradBlocks)) || (r = malloc_into(*M, &M->tt, 1))
        || (r = malloc_into(*M, &M->epart, 2 * kEnergyBlocks))) {
        for (void *p : M->owned) (void)hipFree(p);
        delete M;
        *rc = r;
        return nullptr;
    }
    // the 1-ring again, column-major and padded to the largest degree, so that
    // the per-iteration feature gather reads its indices coalesced
    int32_t max_deg = 0;
    for (int64_t i = 0; i < nn; ++i) max_deg = std::max<int32_t>(max_deg, (int32_t)(ptr[(size_t)i + 1] - ptr[(size_t)i]));
    std::vector<int32_t> ell((size_t)max_deg * (size_t)nn, (int32_t)nn);
    for (int64_t i = 0; i < nn; ++i)
        for (int64_t p = ptr[(size_t)i]; p < ptr[(size_t)i + 1]; ++p)
            ell[(size_t)(p - ptr[(size_t)i]) * (size_t)nn + (size_t)i] = idx[(size_t)p];
    M->max_deg = max_deg;
    if ((r = malloc_into(*M, &M->ell, ell.size()))
        || hipMemcpy(M->ell, ell.data(), ell.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess
        || hipMemset(M->g4 + nn, 0, sizeof(float4)) != hipSuccess) {
        for (void *p : M->owned) (void)hipFree(p);
        delete M;
        *rc = r ? r : hip_fail(hipGetLastError(), "hipMemcpy");
        return nullptr;
    }
    if (hipMemcpy(M->ptr, ptr.data(), ptr.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess
        || (!idx.empty()
            && hipMemcpy(M->idx, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)) {
        for (void *p : M->owned) (void)hipFree(p);
        delete M;
        *rc = hip_fail(hipGetLastError(), "hipMemcpy");
        return nullptr;
    }
    c.mlp = M;
    return M;
}

// Features of r (static part from diag) and z = M(r); partials of r.z in M.prz.
hipError_t mlp_precondition(Ctx &c, MlpState &M, const float *r, float *z)
{
    hipError_t e = mlp_features_dyn(c.stream, M, c.n_nodes, r, M.dinv, M.X, M.scale, M.g4);
    if (e != hipSuccess) return e;
    return mlp_apply(c.stream, M.W, c.n_nodes, M.X, r, M.dinv, M.scale, z, M.prz);
}

// Jacobi inverse (float, 0 on prescribed DOFs) and the static features for diag.
hipError_t mlp_prepare(Ctx &c, MlpState &M, const double *diag)
{
    hipError_t e = mlp_dinv_f32(c.stream, 3 * c.n_nodes, diag, c.m.nmask, M.dinv);
    if (e != hipSuccess) return e;
    return mlp_features_static(c.stream, M, c.n_nodes, diag, c.m.nmask, M.X);
}

}  // namespace efem

using namespace efem;

struct efem_ctx : Ctx {};

extern "C" {

int efem_set_mlp(efem_ctx *ctx, const float *params)
{
    if (!ctx) return EFEM_ERR_INVALID;
    int rc;
    MlpState *M = mlp_state(*ctx, &rc);
    if (!M) return rc;
    if (!params) {
        M->have_weights = false;
        return EFEM_OK;
    }
    TRY(mlp_to_bf16(ctx->stream, params, M->W));
    M->have_weights = true;
    return EFEM_OK;
}

int efem_precond_apply(efem_ctx *ctx, const float *r, const double *diag, float *z)
{
    if (!ctx || !r || !diag || !z) {
        set_error("efem_precond_apply: null pointer");
        return EFEM_ERR_INVALID;
    }
    auto *M = static_cast<MlpState *>(ctx->mlp);
    if (!M || !M->have_weights) {
        set_error("efem_precond_apply: call efem_set_mlp first");
        return EFEM_ERR_STATE;
    }
    TRY(mlp_prepare(*ctx, *M, diag));
    TRY(mlp_precondition(*ctx, *M, r, z));
    return EFEM_OK;
}

int efem_precond_rows(efem_ctx *ctx, const float *b, const double *diag, const float *t,
                      double n_total, uint16_t *X, float *aux)
{
    if (!ctx || !b || !diag || !t || !X || !aux || !(n_total > 0)) {
        set_error("efem_precond_rows: bad argument");
        return EFEM_ERR_INVALID;
    }
    auto *M = static_cast<MlpState *>(ctx->mlp);
    if (!M) {
        set_error("efem_precond_rows: call efem_set_mlp first (builds the node graph)");
        return EFEM_ERR_STATE;
    }
    TRY(mlp_dinv_f32(ctx->stream, 3 * ctx->n_nodes, diag, ctx->m.nmask, M->dinv));
    TRY(mlp_features_static(ctx->stream, *M, ctx->n_nodes, diag, ctx->m.nmask, X));
    TRY(mlp_features_dyn(ctx->stream, *M, ctx->n_nodes, b, M->dinv, X, M->scale, M->g4));
    TRY(mlp_rows_aux(ctx->stream, ctx->n_nodes, b, M->dinv, t, M->scale, M->tt, n_total, aux));
    return EFEM_OK;
}

int efem_mlp_forward(efem_ctx *ctx, int64_t rows, const uint16_t *X, float *out)
{
    if (!ctx || !X || !out || rows < 0) return EFEM_ERR_INVALID;
    auto *M = static_cast<MlpState *>(ctx->mlp);
    if (!M || !M->have_weights) {
        set_error("efem_mlp_forward: call efem_set_mlp first");
        return EFEM_ERR_STATE;
    }
    if (rows == 0) return EFEM_OK;
    TRY(mlp_forward(ctx->stream, M->W, rows, X, out));
    return EFEM_OK;
}

int efem_mlp_forward_layers(efem_ctx *ctx, int64_t rows, const uint16_t *X, uint16_t *h1, uint16_t *h2,
                            float *out)
{
    if (!ctx || !X || !h1 || !h2 || !out || rows < 0) return EFEM_ERR_INVALID;
    auto *M = static_cast<MlpState *>(ctx->mlp);
    if (!M || !M->have_weights) {
        set_error("efem_mlp_forward_layers: call efem_set_mlp first");
        return EFEM_ERR_STATE;
    }
    if (rows == 0) return EFEM_OK;
    TRY(mlp_forward(ctx->stream, M->W, rows, X, out, h1, h2));
    return EFEM_OK;
}

int efem_mlp_loss_grad(efem_ctx *ctx, int64_t rows, const uint16_t *X, const float *aux,
                       const float *params, float *grad, double *loss)
{
    if (!ctx || !X || !aux || !params || !grad || !loss || rows < 0) return EFEM_ERR_INVALID;
    int rc;
    MlpState *M = mlp_state(*ctx, &rc);
    if (!M) return rc;
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(kGradBlocks, (rows + 15) / 16));
    TRY(mlp_loss_grad(ctx->stream, rows, X, aux, params, M->gpart, M->lpart, G, grad, loss));
    return EFEM_OK;
}

int efem_mlp_energy_rows(efem_ctx *ctx, const float *r, const float *out, double n_samples,
                         float *aux, float *z, float *kz, double *energy)
{
    if (!ctx || !r || !out || !aux || !z || !kz || !energy || !(n_samples > 0)) {
        set_error("efem_mlp_energy_rows: bad argument");
        return EFEM_ERR_INVALID;
    }
    if (ctx->lin_prec != EFEM_F32 || !ctx->ulin) {
        set_error("efem_mlp_energy_rows: linearize with EFEM_F32 first");
        return EFEM_ERR_STATE;
    }
    int rc;
    MlpState *M = mlp_state(*ctx, &rc);
    if (!M) return rc;
    const int64_t n = ctx->n_nodes;
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, kEnergyBlocks));
    TRY(mlp_energy_z(ctx->stream, n, r, out, aux, z, M->epart, G));
    TRY(launch_hvp_f32(*ctx, ctx->ulin, z, kz, nullptr, WriteMode::Overwrite));
    TRY(mlp_energy_target(ctx->stream, n, r, out, z, kz, aux, M->epart, n_samples,
                          M->epart + kEnergyBlocks, G, energy));
    return EFEM_OK;
}

int efem_mlp_adam(efem_ctx *ctx, float *params, float *m, float *v, const float *g, float lr,
                  int32_t t)
{
    if (!ctx || !params || !m || !v || !g || t < 1) return EFEM_ERR_INVALID;
    TRY(mlp_adam(ctx->stream, params, m, v, g, lr, 0.9f, 0.999f, 1e-8f, t));
    return EFEM_OK;
}

}  // extern "C"
