// Declarations of the Krylov-solve kernels (kernels_cg.hip) used by the host
// Newton driver (newton.cpp).
#pragma once

#include <algorithm>

#include "efem_internal.h"

namespace efem {

constexpr int kMaxRedBlocks = 1024;   // grid cap of the streaming reductions

// Device-resident scalars of one CG solve.
struct CgScalars {
    double rz, rr, bb, tol2, pq, alpha, beta, pad;
    int32_t done, breakdown, iter, pad2;
};

// Reduction scratch: 2 doubles per block and a last-block ticket.
struct CgWorkspace {
    double *partials = nullptr;   // [2 * kMaxRedBlocks]
    uint32_t *counter = nullptr;  // must be 0 between kernels
};

template <class T>
struct CgLaunch {
    int64_t n;          // vector length (3 * n_nodes)
    hipStream_t s;
    CgWorkspace ws;

    hipError_t init(const double *b, double sign, const T *dinv, const uint8_t *nmask, T *x, T *r,
                    T *p, T *q, CgScalars *sc, double eta2) const;
    hipError_t pq(const T *p, const T *q, CgScalars *sc) const;
    hipError_t update(T *x, T *r, const T *p, T *q, const T *dinv, CgScalars *sc) const;
    hipError_t dir(T *p, const T *r, const T *dinv, const CgScalars *sc) const;
    hipError_t dinv_from_diag(const double *diag, const uint8_t *nmask, T *dinv) const;
    hipError_t axpy_state(const double *u, double alpha, const T *d, double *out) const;
    hipError_t scaled(const T *dinv, const double *b, double sign, T *x) const;
    hipError_t dot_state(const double *a, const T *b, double *out) const;
    hipError_t apply_predictor(const double *u_old, const double *dc, const T *df,
                               const uint8_t *nmask, bool use_df, double *u) const;
};

hipError_t launch_bc_increment(hipStream_t s, int64_t n, const double *u, const double *u_bc,
                               double frac, const uint8_t *nmask, double *dc, double *u_old);
hipError_t launch_dot64(hipStream_t s, const CgWorkspace &ws, int64_t n, const double *a,
                        const double *b, double *out);

}  // namespace efem
