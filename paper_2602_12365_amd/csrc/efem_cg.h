// Declarations of the Krylov-solve kernels (kernels_cg.hip) used by the host
// Newton solver (newton.cpp).
#pragma once

#include <algorithm>

#include "efem_internal.h"

namespace efem {

constexpr int kMaxRedBlocks = 1024;   // grid cap of the streaming reductions

// Device-resident scalars of one CG solve.  Every workgroup of a kernel reads
// the scalars the previous iteration left while workgroup 0 publishes the
// new ones, so whatever is both read and replaced within one kernel (rz, the
// best residual and the stall count) is kept in two slots indexed by the
// iteration parity.
struct CgScalars {
    double rz[2], rr, bb, tol2, pq, alpha, beta, best[2];
    int32_t done, breakdown, iter, fallback, stall[2];
};

// Reduction scratch: four arrays of per-workgroup partials.
struct CgWorkspace {
    double *partials = nullptr;   // [4 * kMaxRedBlocks]
};

int red_grid(int64_t n);

template <class T>
struct CgLaunch {
    int64_t n;          // vector length (3 * n_nodes)
    hipStream_t s;
    CgWorkspace ws;
    // the update kernel clears q for the next tangent action (only the
    // atomic scatter's single-launch form needs q = 0 on entry)
    bool clear_q = true;
    // 3x3 block Jacobi: [n_nodes][6] inverse blocks in bfloat16
    // (k_block_inv); when set, init / update / dir / scaled apply them and
    // ignore dinv
    const uint16_t *binv = nullptr;

    hipError_t init(const double *b, double sign, const T *dinv, const uint8_t *nmask, T *x, T *r,
                    T *p, T *q, CgScalars *sc, double eta2) const;
    hipError_t pq(const T *p, const T *q, CgScalars *sc) const;
    hipError_t update(T *x, T *r, const T *p, T *q, const T *dinv, CgScalars *sc, int j) const;
    hipError_t dir(T *p, const T *r, const T *dinv, CgScalars *sc, int j) const;
    hipError_t dinv_from_diag(const double *diag, const uint8_t *nmask, T *dinv) const;
    hipError_t axpy_state(const double *u, double alpha, const T *d, double *out) const;
    hipError_t scaled(const T *dinv, const double *b, double sign, T *x) const;
    hipError_t widen(const T *a, double *out) const;   // out = (double) a
    hipError_t add_to(T *x, const T *d) const;          // x += d
    hipError_t dot_state(const double *a, const T *b, double *out) const;
    hipError_t apply_predictor(const double *u_old, const double *dc, const T *df,
                               const uint8_t *nmask, bool use_df, double *u) const;
};

// Flexible CG with a nonlinear preconditioner z = M(r) (Notay's flexible CG:
// Polak-Ribiere beta = r.(z_new - z_old) / rz_old).  The apply kernel writes
// partials of r.z into `prz` (count `nz`).
template <class T>
struct FcgLaunch {
    int64_t n;
    hipStream_t s;
    CgWorkspace ws;
    bool clear_q = true;   // as in CgLaunch
    // after M(r) -> z: rz = r.z; p = z; breakdown / fallback if rz <= 0
    hipError_t start(const T *z, T *p, CgScalars *sc, const double *prz, int nz) const;
    // alpha = rz/pq; x += alpha p; r -= alpha q; q = 0 (clear_q); partials of r.r and r.z_old
    hipError_t update(T *x, T *r, const T *p, T *q, const T *zold, CgScalars *sc, int j) const;
    // convergence / stagnation test; beta = (r.z_new - r.z_old)/rz; p = z + beta p
    hipError_t dir(T *p, const T *z, CgScalars *sc, const double *prz, int nz, int j,
                   int stall_limit) const;
};

// binv [n_nodes][6] from the diagonal d [3 n_nodes] and the off-diagonals o
// [n_nodes][3] of the nodes' 3x3 blocks of K (prescribed components removed)
hipError_t launch_block_inv(hipStream_t s, int64_t n_nodes, const double *d, const double *o,
                            const uint8_t *nmask, uint16_t *binv);
hipError_t launch_bc_increment(hipStream_t s, int64_t n, const double *u, const double *u_bc,
                               double frac, const uint8_t *nmask, double *dc, double *u_old);
hipError_t launch_dot64(hipStream_t s, const CgWorkspace &ws, int64_t n, const double *a,
                        const double *b, double *out);
// y -= scale f on the DOFs the node mask leaves free (all of them for a null mask)
hipError_t launch_sub_load(hipStream_t s, int64_t n, double *y, const double *f, double scale,
                           const uint8_t *nmask);

}  // namespace efem
