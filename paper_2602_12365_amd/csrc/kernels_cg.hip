// Streaming kernels of the Krylov solve.  CG scalars live on the device so a
// batch of iterations runs without host round trips.  Reductions are split
// across kernel boundaries instead of device-wide fences: a kernel writes one
// partial per workgroup with plain stores, and every workgroup of the next
// kernel sums those partials in the same fixed order, so all of them derive
// identical scalars (alpha, beta, convergence) and the result is
// deterministic.  Workgroup 0 publishes the scalars the host reads.  Once
// `done` is set, every later kernel of the batch returns at once.  Vectors are
// float64 (plain solve) or float32 (mixed precision); every reduction
// accumulates in float64.
#include "efem_cg.h"

namespace efem {

constexpr int kThreads = 256;

__device__ __forceinline__ bool dof_fixed(const uint8_t *nmask, int64_t i)
{
    return nmask && ((nmask[i / 3] >> (i % 3)) & 1);
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < (n); i += (int64_t)gridDim.x * kThreads)

// Workgroup tree sum of one value per thread; every thread gets the total.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

// Sum of the `count` partials of the previous kernel (same order in every workgroup).
__device__ __forceinline__ double sum_partials(const double *part, int count, double *red)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += kThreads) s += part[i];
    return block_sum(s, red);
}

// r = sign * b (prescribed -> 0), z = dinv r, p = z, x = 0, q = 0; partials of r.r, r.z
template <class T>
__global__ void __launch_bounds__(kThreads) k_cg_init(int64_t n, const double *__restrict__ b,
                                                      double sign, const T *__restrict__ dinv,
                                                      const uint8_t *__restrict__ nmask,
                                                      T *__restrict__ x, T *__restrict__ r,
                                                      T *__restrict__ p, T *__restrict__ q,
                                                      double *__restrict__ prr, double *__restrict__ prz)
{
    __shared__ double red[kThreads];
    double rz = 0.0, rr = 0.0;
    GRID_STRIDE(i, n)
    {
        const T ri = dof_fixed(nmask, i) ? T(0) : T(sign * b[i]);
        const T zi = dinv[i] * ri;
        r[i] = ri;
        p[i] = zi;
        x[i] = T(0);
        q[i] = T(0);
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    const double srr = block_sum(rr, red);
    const double srz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        prr[blockIdx.x] = srr;
        prz[blockIdx.x] = srz;
    }
}

__global__ void __launch_bounds__(kThreads) k_cg_init_fin(const double *__restrict__ prr,
                                                          const double *__restrict__ prz, int count,
                                                          CgScalars *sc, double eta2)
{
    __shared__ double red[kThreads];
    const double rr = sum_partials(prr, count, red);
    const double rz = sum_partials(prz, count, red);
    if (threadIdx.x == 0) {
        sc->rz[0] = rz;
        sc->rz[1] = 0.0;
        sc->rr = rr;
        sc->bb = rr;
        sc->tol2 = eta2 * rr;
        sc->done = (rr == 0.0) ? 1 : 0;
        sc->breakdown = 0;
        sc->fallback = 0;
        sc->stall[0] = sc->stall[1] = 0;
        sc->best[0] = sc->best[1] = rr;
        sc->iter = 0;
        sc->alpha = sc->beta = sc->pq = 0.0;
    }
}

// partials of p.q
template <class T>
__global__ void __launch_bounds__(kThreads) k_cg_pq(int64_t n, const T *__restrict__ p,
                                                    const T *__restrict__ q, const CgScalars *sc,
                                                    double *__restrict__ ppq)
{
    __shared__ double red[kThreads];
    if (sc->done) return;
    double pq = 0.0;
    GRID_STRIDE(i, n) pq += (double)p[i] * (double)q[i];
    const double s = block_sum(pq, red);
    if (threadIdx.x == 0) ppq[blockIdx.x] = s;
}

// alpha = rz / pq (breakdown if pq <= 0 or not finite); x += alpha p,
// r -= alpha q, q = 0 if CLEAR (for a next tangent action that adds into q);
// partials of r.r and r.(dinv r).  `j` is the iteration index and `par` its
// parity (which rz slot is current).
template <class T, bool CLEAR>
__global__ void __launch_bounds__(kThreads) k_cg_update(int64_t n, T *__restrict__ x,
                                                        T *__restrict__ r, const T *__restrict__ p,
                                                        T *__restrict__ q, const T *__restrict__ dinv,
                                                        CgScalars *sc, const double *__restrict__ ppq,
                                                        int count, double *__restrict__ prr,
                                                        double *__restrict__ prz, int par, int j)
{
    __shared__ double red[kThreads];
    if (sc->done) return;
    const double pq = sum_partials(ppq, count, red);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->pq = pq;
            sc->breakdown = 1;
            sc->done = 1;
        }
        return;
    }
    const double alpha = sc->rz[par] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = alpha;
        sc->iter = j + 1;
    }
    const T a = (T)alpha;
    double rr = 0.0, rz = 0.0;
    GRID_STRIDE(i, n)
    {
        x[i] += a * p[i];
        const T ri = r[i] - a * q[i];
        r[i] = ri;
        if (CLEAR) q[i] = T(0);
        const T zi = dinv[i] * ri;
        rr += (double)ri * (double)ri;
        rz += (double)ri * (double)zi;
    }
    const double srr = block_sum(rr, red);
    const double srz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        prr[blockIdx.x] = srr;
        prz[blockIdx.x] = srz;
    }
}

// convergence test rr <= tol2; beta = rz_new / rz; p = dinv r + beta p
template <class T>
__global__ void __launch_bounds__(kThreads) k_cg_dir(int64_t n, T *__restrict__ p,
                                                     const T *__restrict__ r,
                                                     const T *__restrict__ dinv, CgScalars *sc,
                                                     const double *__restrict__ prr,
                                                     const double *__restrict__ prz, int count,
                                                     int par)
{
    __shared__ double red[kThreads];
    if (sc->done) return;
    const double rr = sum_partials(prr, count, red);
    const double rz = sum_partials(prz, count, red);
    if (rr <= sc->tol2 || !isfinite(rr)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rr = rr;
            sc->done = 1;
        }
        return;
    }
    const double beta = rz / sc->rz[par];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rz[par ^ 1] = rz;
        sc->rr = rr;
        sc->beta = beta;
    }
    const T bt = (T)beta;
    GRID_STRIDE(i, n) p[i] = dinv[i] * r[i] + bt * p[i];
}

// ------------------------------------------------ 3x3 block Jacobi

// bfloat16 storage of the inverse blocks (round to nearest even): the
// preconditioner only has to stay symmetric positive definite, which a
// relative perturbation of 2^-9 keeps, and the CG update and direction
// kernels read the blocks every iteration (12 bytes per node instead of 24)
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// binv [n_nodes][6] = (B00, B11, B22, B01, B02, B12), the inverse of each
// node's 3x3 diagonal block of K_ff: diagonal d [3 n_nodes], off-diagonals
// o [n_nodes][3] = (K01, K02, K12).  Prescribed components leave the block
// (their rows and columns of the inverse are 0).  A block that is not
// positive definite (leading minors) falls back to its diagonal inverse.
__global__ void k_block_inv(int64_t nn, const double *__restrict__ d, const double *__restrict__ o,
                            const uint8_t *__restrict__ nmask, uint16_t *__restrict__ binv)
{
    GRID_STRIDE(i, nn)
    {
        const uint8_t m = nmask ? nmask[i] : 0;
        const bool f0 = m & 1, f1 = (m >> 1) & 1, f2 = (m >> 2) & 1;
        const double a00 = f0 ? 1.0 : d[3 * i], a11 = f1 ? 1.0 : d[3 * i + 1], a22 = f2 ? 1.0 : d[3 * i + 2];
        const double a01 = (f0 || f1) ? 0.0 : o[3 * i], a02 = (f0 || f2) ? 0.0 : o[3 * i + 1];
        const double a12 = (f1 || f2) ? 0.0 : o[3 * i + 2];
        const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
        const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
        const double det = a00 * c00 + a01 * c01 + a02 * c02;
        double b[6];
        if (a00 > 0.0 && c22 > 0.0 && det > 0.0 && isfinite(det)) {
            const double r = 1.0 / det;
            b[0] = c00 * r, b[1] = c11 * r, b[2] = c22 * r, b[3] = c01 * r, b[4] = c02 * r, b[5] = c12 * r;
        } else {
            b[0] = a00 > 0.0 ? 1.0 / a00 : 0.0;
            b[1] = a11 > 0.0 ? 1.0 / a11 : 0.0;
            b[2] = a22 > 0.0 ? 1.0 / a22 : 0.0;
            b[3] = b[4] = b[5] = 0.0;
        }
        if (f0) b[0] = b[3] = b[4] = 0.0;
        if (f1) b[1] = b[3] = b[5] = 0.0;
        if (f2) b[2] = b[4] = b[5] = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) binv[6 * i + k] = to_bf16((float)b[k]);
    }
}

// z = B r for node i's block
template <class T>
__device__ __forceinline__ void block_apply(const uint16_t *__restrict__ binv, int64_t i, T r0, T r1, T r2, T &z0,
                                            T &z1, T &z2)
{
    const T b00 = T(from_bf16(binv[6 * i])), b11 = T(from_bf16(binv[6 * i + 1])), b22 = T(from_bf16(binv[6 * i + 2]));
    const T b01 = T(from_bf16(binv[6 * i + 3])), b02 = T(from_bf16(binv[6 * i + 4]));
    const T b12 = T(from_bf16(binv[6 * i + 5]));
    z0 = b00 * r0 + b01 * r1 + b02 * r2;
    z1 = b01 * r0 + b11 * r1 + b12 * r2;
    z2 = b02 * r0 + b12 * r1 + b22 * r2;
}

// The PCG kernels with the block preconditioner, one node (three DOFs) per
// thread; their reductions and scalar logic are those of the DOF-wise ones.
template <class T>
__global__ void __launch_bounds__(kThreads) k_cgb_init(int64_t nn, const double *__restrict__ b, double sign,
                                                       const uint16_t *__restrict__ binv,
                                                       const uint8_t *__restrict__ nmask, T *__restrict__ x,
                                                       T *__restrict__ r, T *__restrict__ p, T *__restrict__ q,
                                                       double *__restrict__ prr, double *__restrict__ prz)
{
    __shared__ double red[kThreads];
    double rz = 0.0, rr = 0.0;
    GRID_STRIDE(i, nn)
    {
        T rv[3], z[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) rv[c] = dof_fixed(nmask, 3 * i + c) ? T(0) : T(sign * b[3 * i + c]);
        block_apply(binv, i, rv[0], rv[1], rv[2], z[0], z[1], z[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            r[3 * i + c] = rv[c];
            p[3 * i + c] = z[c];
            x[3 * i + c] = T(0);
            q[3 * i + c] = T(0);
            rz += (double)rv[c] * (double)z[c];
            rr += (double)rv[c] * (double)rv[c];
        }
    }
    const double srr = block_sum(rr, red);
    const double srz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        prr[blockIdx.x] = srr;
        prz[blockIdx.x] = srz;
    }
}

template <class T, bool CLEAR>
__global__ void __launch_bounds__(kThreads) k_cgb_update(int64_t nn, T *__restrict__ x, T *__restrict__ r,
                                                         const T *__restrict__ p, T *__restrict__ q,
                                                         const uint16_t *__restrict__ binv, CgScalars *sc,
                                                         const double *__restrict__ ppq, int count,
                                                         double *__restrict__ prr, double *__restrict__ prz,
                                                         int par, int j)
{
    __shared__ double red[kThreads];
    if (sc->done) return;
    const double pq = sum_partials(ppq, count, red);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->pq = pq;
            sc->breakdown = 1;
            sc->done = 1;
        }
        return;
    }
    const double alpha = sc->rz[par] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = alpha;
        sc->iter = j + 1;
    }
    const T a = (T)alpha;
    double rr = 0.0, rz = 0.0;
    GRID_STRIDE(i, nn)
    {
        T rv[3], z[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t k = 3 * i + c;
            x[k] += a * p[k];
            rv[c] = r[k] - a * q[k];
            r[k] = rv[c];
            if (CLEAR) q[k] = T(0);
        }
        block_apply(binv, i, rv[0], rv[1], rv[2], z[0], z[1], z[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            rr += (double)rv[c] * (double)rv[c];
            rz += (double)rv[c] * (double)z[c];
        }
    }
    const double srr = block_sum(rr, red);
    const double srz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        prr[blockIdx.x] = srr;
        prz[blockIdx.x] = srz;
    }
}

template <class T>
__global__ void __launch_bounds__(kThreads) k_cgb_dir(int64_t nn, T *__restrict__ p, const T *__restrict__ r,
                                                      const uint16_t *__restrict__ binv, CgScalars *sc,
                                                      const double *__restrict__ prr,
                                                      const double *__restrict__ prz, int count, int par)
{
    __shared__ double red[kThreads];
    if (sc->done) return;
    const double rr = sum_partials(prr, count, red);
    const double rz = sum_partials(prz, count, red);
    if (rr <= sc->tol2 || !isfinite(rr)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rr = rr;
            sc->done = 1;
        }
        return;
    }
    const double beta = rz / sc->rz[par];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rz[par ^ 1] = rz;
        sc->rr = rr;
        sc->beta = beta;
    }
    const T bt = (T)beta;
    GRID_STRIDE(i, nn)
    {
        T z[3];
        block_apply(binv, i, r[3 * i], r[3 * i + 1], r[3 * i + 2], z[0], z[1], z[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) p[3 * i + c] = z[c] + bt * p[3 * i + c];
    }
}

template <class T>
__global__ void k_cgb_scaled(int64_t nn, const uint16_t *__restrict__ binv, const double *__restrict__ b,
                             double sign, T *__restrict__ x)
{
    GRID_STRIDE(i, nn)
    {
        T z[3];
        block_apply(binv, i, T(sign * b[3 * i]), T(sign * b[3 * i + 1]), T(sign * b[3 * i + 2]), z[0], z[1], z[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) x[3 * i + c] = z[c];
    }
}

// partials of a.b
template <class TA, class TB>
__global__ void __launch_bounds__(kThreads) k_dot(int64_t n, const TA *__restrict__ a,
                                                  const TB *__restrict__ b, double *__restrict__ part)
{
    __shared__ double red[kThreads];
    double s = 0.0;
    GRID_STRIDE(i, n) s += (double)a[i] * (double)b[i];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kThreads) k_dot_fin(const double *__restrict__ part, int count,
                                                      double *__restrict__ out)
{
    __shared__ double red[kThreads];
    const double s = sum_partials(part, count, red);
    if (threadIdx.x == 0) *out = s;
}

// dinv = 1/diag on free DOFs, 0 on prescribed ones
template <class T>
__global__ void k_dinv(int64_t n, const double *__restrict__ diag, const uint8_t *__restrict__ nmask,
                       T *__restrict__ dinv)
{
    GRID_STRIDE(i, n) dinv[i] = dof_fixed(nmask, i) ? T(0) : T(1.0 / diag[i]);
}

// out = u + alpha d   (float64 state, d of the solve precision)
template <class T>
__global__ void k_axpy_state(int64_t n, const double *__restrict__ u, double alpha,
                             const T *__restrict__ d, double *__restrict__ out)
{
    GRID_STRIDE(i, n) out[i] = u[i] + alpha * (double)d[i];
}

// out = (double) a
template <class T>
__global__ void k_widen(int64_t n, const T *__restrict__ a, double *__restrict__ out)
{
    GRID_STRIDE(i, n) out[i] = (double)a[i];
}

// x += d
template <class T>
__global__ void k_add_to(int64_t n, T *__restrict__ x, const T *__restrict__ d)
{
    GRID_STRIDE(i, n) x[i] += d[i];
}

// x = dinv * sign * b (steepest-descent fallback step)
template <class T>
__global__ void k_scaled(int64_t n, const T *__restrict__ dinv, const double *__restrict__ b,
                         double sign, T *__restrict__ x)
{
    GRID_STRIDE(i, n) x[i] = dinv[i] * T(sign * b[i]);
}

// Load step: dc = frac*u_bc - u on prescribed DOFs (0 elsewhere), u_old = u.
__global__ void k_bc_increment(int64_t n, const double *__restrict__ u,
                               const double *__restrict__ u_bc, double frac,
                               const uint8_t *__restrict__ nmask, double *__restrict__ dc,
                               double *__restrict__ u_old)
{
    GRID_STRIDE(i, n)
    {
        const double ui = u[i];
        dc[i] = dof_fixed(nmask, i) ? frac * u_bc[i] - ui : 0.0;
        u_old[i] = ui;
    }
}

// u = u_old + dc + free(df)
template <class T>
__global__ void k_apply_predictor(int64_t n, const double *__restrict__ u_old,
                                  const double *__restrict__ dc, const T *__restrict__ df,
                                  const uint8_t *__restrict__ nmask, int use_df,
                                  double *__restrict__ u)
{
    GRID_STRIDE(i, n)
    {
        const double f = (use_df && !dof_fixed(nmask, i)) ? (double)df[i] : 0.0;
        u[i] = u_old[i] + dc[i] + f;
    }
}

// ------------------------------------------------------------------ launchers

int red_grid(int64_t n)
{
    int64_t g = (n + kThreads - 1) / kThreads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, kMaxRedBlocks));
}

template <class T>
hipError_t CgLaunch<T>::init(const double *b, double sign, const T *dinv, const uint8_t *nmask,
                             T *x, T *r, T *p, T *q, CgScalars *sc, double eta2) const
{
    const int g = binv ? red_grid(n / 3) : red_grid(n);
    if (binv)
        hipLaunchKernelGGL(k_cgb_init<T>, dim3(g), dim3(kThreads), 0, s, n / 3, b, sign, binv, nmask, x, r, p, q,
                           ws.partials + kMaxRedBlocks, ws.partials + 2 * kMaxRedBlocks);
    else
        hipLaunchKernelGGL(k_cg_init<T>, dim3(g), dim3(kThreads), 0, s, n, b, sign, dinv, nmask, x, r,
                           p, q, ws.partials + kMaxRedBlocks, ws.partials + 2 * kMaxRedBlocks);
    hipLaunchKernelGGL(k_cg_init_fin, dim3(1), dim3(kThreads), 0, s, ws.partials + kMaxRedBlocks,
                       ws.partials + 2 * kMaxRedBlocks, g, sc, eta2);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::pq(const T *p, const T *q, CgScalars *sc) const
{
    hipLaunchKernelGGL(k_cg_pq<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, p, q, sc, ws.partials);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::update(T *x, T *r, const T *p, T *q, const T *dinv, CgScalars *sc, int j) const
{
    const int gpq = red_grid(n);   // partials of k_cg_pq
    if (binv) {
        const int g = red_grid(n / 3);
        auto kern = clear_q ? k_cgb_update<T, true> : k_cgb_update<T, false>;
        hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, s, n / 3, x, r, p, q, binv, sc, ws.partials, gpq,
                           ws.partials + kMaxRedBlocks, ws.partials + 2 * kMaxRedBlocks, j & 1, j);
        return hipGetLastError();
    }
    auto kern = clear_q ? k_cg_update<T, true> : k_cg_update<T, false>;
    hipLaunchKernelGGL(kern, dim3(gpq), dim3(kThreads), 0, s, n, x, r, p, q, dinv, sc, ws.partials, gpq,
                       ws.partials + kMaxRedBlocks, ws.partials + 2 * kMaxRedBlocks, j & 1, j);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::dir(T *p, const T *r, const T *dinv, CgScalars *sc, int j) const
{
    if (binv) {
        const int g = red_grid(n / 3);
        hipLaunchKernelGGL(k_cgb_dir<T>, dim3(g), dim3(kThreads), 0, s, n / 3, p, r, binv, sc,
                           ws.partials + kMaxRedBlocks, ws.partials + 2 * kMaxRedBlocks, g, j & 1);
        return hipGetLastError();
    }
    const int g = red_grid(n);
    hipLaunchKernelGGL(k_cg_dir<T>, dim3(g), dim3(kThreads), 0, s, n, p, r, dinv, sc,
                       ws.partials + kMaxRedBlocks, ws.partials + 2 * kMaxRedBlocks, g, j & 1);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::dinv_from_diag(const double *diag, const uint8_t *nmask, T *dinv) const
{
    hipLaunchKernelGGL(k_dinv<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, diag, nmask, dinv);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::axpy_state(const double *u, double alpha, const T *d, double *out) const
{
    hipLaunchKernelGGL(k_axpy_state<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, u, alpha, d, out);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::widen(const T *a, double *out) const
{
    hipLaunchKernelGGL(k_widen<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, a, out);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::add_to(T *x, const T *d) const
{
    hipLaunchKernelGGL(k_add_to<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, x, d);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::scaled(const T *dinv, const double *b, double sign, T *x) const
{
    if (binv) {
        hipLaunchKernelGGL(k_cgb_scaled<T>, dim3(red_grid(n / 3)), dim3(kThreads), 0, s, n / 3, binv, b, sign, x);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scaled<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, dinv, b, sign, x);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::dot_state(const double *a, const T *b, double *out) const
{
    const int g = red_grid(n);
    hipLaunchKernelGGL((k_dot<double, T>), dim3(g), dim3(kThreads), 0, s, n, a, b,
                       ws.partials + 3 * kMaxRedBlocks);
    hipLaunchKernelGGL(k_dot_fin, dim3(1), dim3(kThreads), 0, s, ws.partials + 3 * kMaxRedBlocks, g,
                       out);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::apply_predictor(const double *u_old, const double *dc, const T *df,
                                        const uint8_t *nmask, bool use_df, double *u) const
{
    hipLaunchKernelGGL(k_apply_predictor<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, u_old, dc,
                       df, nmask, use_df ? 1 : 0, u);
    return hipGetLastError();
}

hipError_t launch_bc_increment(hipStream_t s, int64_t n, const double *u, const double *u_bc,
                               double frac, const uint8_t *nmask, double *dc, double *u_old)
{
    hipLaunchKernelGGL(k_bc_increment, dim3(red_grid(n)), dim3(kThreads), 0, s, n, u, u_bc, frac,
                       nmask, dc, u_old);
    return hipGetLastError();
}

// y -= s f on the free DOFs (prescribed entries of y are left as they are)
__global__ void k_sub_load(int64_t n, double *__restrict__ y, const double *__restrict__ f,
                           double s, const uint8_t *__restrict__ nmask)
{
    GRID_STRIDE(i, n)
    {
        if (!dof_fixed(nmask, i)) y[i] -= s * f[i];
    }
}

hipError_t launch_sub_load(hipStream_t s, int64_t n, double *y, const double *f, double scale,
                           const uint8_t *nmask)
{
    hipLaunchKernelGGL(k_sub_load, dim3(red_grid(n)), dim3(kThreads), 0, s, n, y, f, scale, nmask);
    return hipGetLastError();
}

hipError_t launch_dot64(hipStream_t s, const CgWorkspace &ws, int64_t n, const double *a,
                        const double *b, double *out)
{
    const int g = red_grid(n);
    hipLaunchKernelGGL((k_dot<double, double>), dim3(g), dim3(kThreads), 0, s, n, a, b,
                       ws.partials + 3 * kMaxRedBlocks);
    hipLaunchKernelGGL(k_dot_fin, dim3(1), dim3(kThreads), 0, s, ws.partials + 3 * kMaxRedBlocks, g,
                       out);
    return hipGetLastError();
}

// ------------------------------------------------------------- flexible CG

// rz = r.z from the apply's partials; p = z.  A non-positive rz means the
// preconditioner is not usable here: request the Jacobi fallback.
template <class T>
__global__ void __launch_bounds__(kThreads) k_fcg_start(int64_t n, const T *__restrict__ z,
                                                        T *__restrict__ p, CgScalars *sc,
                                                        const double *__restrict__ prz, int nz)
{
    __shared__ double red[kThreads];
    if (sc->done) return;
    const double rz = sum_partials(prz, nz, red);
    if (!(rz > 0.0) || !isfinite(rz)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->fallback = 1;
            sc->done = 1;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rz[0] = rz;
        sc->best[0] = sc->rr;
        sc->stall[0] = 0;
        sc->fallback = 0;
    }
    GRID_STRIDE(i, n) p[i] = z[i];
}

// alpha = rz/pq; x += alpha p; r -= alpha q; q = 0 if CLEAR; partials of r.r and r.z_old
template <class T, bool CLEAR>
__global__ void __launch_bounds__(kThreads) k_fcg_update(int64_t n, T *__restrict__ x,
                                                         T *__restrict__ r, const T *__restrict__ p,
                                                         T *__restrict__ q, const T *__restrict__ zold,
                                                         CgScalars *sc, const double *__restrict__ ppq,
                                                         int count, double *__restrict__ prr,
                                                         double *__restrict__ prz, int par, int j)
{
    __shared__ double red[kThreads];
    if (sc->done) return;
    const double pq = sum_partials(ppq, count, red);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->pq = pq;
            sc->breakdown = 1;
            sc->fallback = 1;
            sc->done = 1;
        }
        return;
    }
    const double alpha = sc->rz[par] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = alpha;
        sc->iter = j + 1;
    }
    const T a = (T)alpha;
    double rr = 0.0, rzo = 0.0;
    GRID_STRIDE(i, n)
    {
        x[i] += a * p[i];
        const T ri = r[i] - a * q[i];
        r[i] = ri;
        if (CLEAR) q[i] = T(0);
        rr += (double)ri * (double)ri;
        rzo += (double)ri * (double)zold[i];
    }
    const double s0 = block_sum(rr, red);
    const double s1 = block_sum(rzo, red);
    if (threadIdx.x == 0) {
        prr[blockIdx.x] = s0;
        prz[blockIdx.x] = s1;
    }
}

// Convergence (rr <= tol2), stagnation (no new best rr for stall_limit
// iterations) and positivity (r.z_new > 0) tests; beta = (r.z_new - r.z_old) / rz;
// p = z_new + beta p.
template <class T>
__global__ void __launch_bounds__(kThreads) k_fcg_dir(int64_t n, T *__restrict__ p,
                                                      const T *__restrict__ z, CgScalars *sc,
                                                      const double *__restrict__ prr,
                                                      const double *__restrict__ przo, int count,
                                                      const double *__restrict__ przn, int nz,
                                                      int par, int stall_limit)
{
    __shared__ double red[kThreads];
    if (sc->done) return;
    const double rr = sum_partials(prr, count, red);
    const double rzo = sum_partials(przo, count, red);
    const double rzn = sum_partials(przn, nz, red);
    const bool first = blockIdx.x == 0 && threadIdx.x == 0;
    if (rr <= sc->tol2 || !isfinite(rr)) {
        if (first) {
            sc->rr = rr;
            sc->done = 1;
        }
        return;
    }
    const double best = sc->best[par];
    const int stall = rr < best ? 0 : sc->stall[par] + 1;
    if (!(rzn > 0.0) || !isfinite(rzn) || stall >= stall_limit) {
        if (first) {
            sc->rr = rr;
            sc->fallback = 1;
            sc->done = 1;
        }
        return;
    }
    const double beta = (rzn - rzo) / sc->rz[par];
    if (first) {
        sc->rz[par ^ 1] = rzn;
        sc->rr = rr;
        sc->beta = beta;
        sc->stall[par ^ 1] = stall;
        sc->best[par ^ 1] = rr < best ? rr : best;
    }
    const T bt = (T)beta;
    GRID_STRIDE(i, n) p[i] = z[i] + bt * p[i];
}

template <class T>
hipError_t FcgLaunch<T>::start(const T *z, T *p, CgScalars *sc, const double *prz, int nz) const
{
    hipLaunchKernelGGL(k_fcg_start<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, z, p, sc, prz, nz);
    return hipGetLastError();
}

template <class T>
hipError_t FcgLaunch<T>::update(T *x, T *r, const T *p, T *q, const T *zold, CgScalars *sc, int j) const
{
    const int g = red_grid(n);
    auto kern = clear_q ? k_fcg_update<T, true> : k_fcg_update<T, false>;
    hipLaunchKernelGGL(kern, dim3(g), dim3(kThreads), 0, s, n, x, r, p, q, zold, sc, ws.partials, g,
                       ws.partials + kMaxRedBlocks, ws.partials + 2 * kMaxRedBlocks, j & 1, j);
    return hipGetLastError();
}

template <class T>
hipError_t FcgLaunch<T>::dir(T *p, const T *z, CgScalars *sc, const double *prz, int nz, int j,
                             int stall_limit) const
{
    const int g = red_grid(n);
    hipLaunchKernelGGL(k_fcg_dir<T>, dim3(g), dim3(kThreads), 0, s, n, p, z, sc,
                       ws.partials + kMaxRedBlocks, ws.partials + 2 * kMaxRedBlocks, g, prz, nz,
                       j & 1, stall_limit);
    return hipGetLastError();
}

hipError_t launch_block_inv(hipStream_t s, int64_t n_nodes, const double *d, const double *o,
                            const uint8_t *nmask, uint16_t *binv)
{
    hipLaunchKernelGGL(k_block_inv, dim3(red_grid(n_nodes)), dim3(kThreads), 0, s, n_nodes, d, o, nmask, binv);
    return hipGetLastError();
}

template struct CgLaunch<double>;
template struct CgLaunch<float>;
template struct FcgLaunch<float>;

}  // namespace efem
