// Streaming kernels of the restarted GMRES solve (kernels_gmres.hip) used by
// the host driver (gmres.cpp).  Basis vectors are float64, stored one after
// another with stride n.
#pragma once

#include "efem_internal.h"

namespace efem {

constexpr int kGmresRedBlocks = 512;   // workgroups of the multi-dot
constexpr int kGmresMaxRestart = 100;

// h[j] = V_j . w for j < k (partials in `part` [k][kGmresRedBlocks], then a
// fixed-order sum per j: deterministic)
hipError_t gm_mdot(hipStream_t s, int64_t n, const double *V, int k, const double *w, double *part,
                   double *h);
// w -= sum_{j<k} h[j] V_j   (h on the device)
hipError_t gm_subtract(hipStream_t s, int64_t n, const double *V, int k, const double *h, double *w);
// out = alpha * w
hipError_t gm_scale(hipStream_t s, int64_t n, double alpha, const double *w, double *out);
// out = a * b (elementwise)
hipError_t gm_mul(hipStream_t s, int64_t n, const double *a, const double *b, double *out);
// out = b - Kx on free DOFs, 0 on prescribed ones
hipError_t gm_residual(hipStream_t s, int64_t n, const double *b, const double *kx, const uint8_t *nmask,
                       double *out);
// x += dinv * sum_{j<k} y[j] V_j   (y on the device)
hipError_t gm_update_x(hipStream_t s, int64_t n, const double *V, int k, const double *y, const double *dinv,
                       double *x);
// conversions for the FP32 tangent action
hipError_t gm_to_f32(hipStream_t s, int64_t n, const double *a, float *out);
hipError_t gm_to_f64(hipStream_t s, int64_t n, const float *a, double *out);
// dinv = 1/diag on free DOFs, 0 on prescribed ones
hipError_t gm_dinv(hipStream_t s, int64_t n, const double *diag, const uint8_t *nmask, double *dinv);

}  // namespace efem
