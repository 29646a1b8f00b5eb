// Learned-preconditioner declarations shared by kernels_mlp.hip and precond.cpp.
#pragma once

#include <algorithm>

#include "efem_internal.h"

namespace efem {

constexpr int kIn = EFEM_MLP_IN, kInPad = 16, kHid = EFEM_MLP_HID, kOut = EFEM_MLP_OUT;
constexpr int kAux = 12;   // training row: g(3), t(3), m(3), s, w, pad
// flat parameter layout: W1 [64][12], b1 [64], W2 [64][64], b2 [64], W3 [3][64], b3 [3]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHid * kIn;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kOut * kHid;
constexpr int kP = kOffB3 + kOut;
static_assert(kP == EFEM_MLP_PARAMS, "parameter count");

// Per-context state of the learned preconditioner.
struct MlpState {
    int64_t *ptr = nullptr;      // [n_nodes+1] node 1-ring CSR
    int32_t *idx = nullptr;
    int32_t *ell = nullptr;      // [max_deg][n_nodes] the same 1-ring, column-major,
    int32_t max_deg = 0;         //   padded with n_nodes (a zero record of g4)
    uint16_t *W = nullptr;       // bf16 parameters [kP]
    bool have_weights = false;
    uint16_t *X = nullptr;       // [n_nodes][16] bf16 features
    float *scale = nullptr;      // [n_nodes]
    float4 *g4 = nullptr;        // [n_nodes + 1] (D^-1 r, |D^-1 r|^2) of the features; last = 0
    float *dinv = nullptr;       // [3 n_nodes]
    float *z = nullptr;          // [3 n_nodes] scratch of the apply
    float *zold = nullptr;       // [3 n_nodes] flexible CG
    double *prz = nullptr;       // [2048] partials
    float *gpart = nullptr;      // [kGradBlocks][kP]
    double *lpart = nullptr;     // [kGradBlocks]
    double *epart = nullptr;     // [2 kEnergyBlocks] energy-row partials
    double *tt = nullptr;        // scalar
    std::vector<void *> owned;
};
constexpr int kGradBlocks = 1024;
constexpr int kEnergyBlocks = 512;

hipError_t mlp_features_static(hipStream_t s, const MlpState &M, int64_t n, const double *diag,
                               const uint8_t *nmask, uint16_t *X);
hipError_t mlp_features_dyn(hipStream_t s, const MlpState &M, int64_t n, const float *r,
                            const float *dinv, uint16_t *X, float *scale, float4 *g4);
// H1, H2 (both or neither): the hidden layers' bf16 activations [n][64]
hipError_t mlp_forward(hipStream_t s, const uint16_t *W, int64_t n, const uint16_t *X, float *out,
                       uint16_t *H1 = nullptr, uint16_t *H2 = nullptr);
int mlp_apply_grid(int64_t n);
hipError_t mlp_apply(hipStream_t s, const uint16_t *W, int64_t n, const uint16_t *X, const float *r,
                     const float *dinv, const float *scale, float *z, double *prz);
hipError_t mlp_rows_aux(hipStream_t s, int64_t n, const float *b, const float *dinv, const float *t,
                        const float *scale, double *tt, double n_total, float *aux);
hipError_t mlp_loss_grad(hipStream_t s, int64_t rows, const uint16_t *X, const float *aux,
                         const float *params, float *gpart, double *lpart, int G, float *grad,
                         double *loss);
// energy-norm training rows of one sample: z = m (g + s out) and partials of
// r.g (G blocks), then, with K z in kz, the pseudo-targets, the weights and
// energy += w (z.Kz - 2 r.z); `part` holds 2 G doubles
hipError_t mlp_energy_z(hipStream_t s, int64_t n, const float *r, const float *out, const float *aux,
                        float *z, double *part, int G);
hipError_t mlp_energy_target(hipStream_t s, int64_t n, const float *r, const float *out, const float *z,
                             const float *kz, float *aux, const double *rgpart, double n_samples,
                             double *part, int G, double *energy);
hipError_t mlp_adam(hipStream_t s, float *p, float *m, float *v, const float *g, float lr, float b1,
                    float b2, float eps, int t);
hipError_t mlp_to_bf16(hipStream_t s, const float *p, uint16_t *out);
hipError_t mlp_dinv_f32(hipStream_t s, int64_t n, const double *diag, const uint8_t *nmask,
                        float *dinv);

}  // namespace efem
