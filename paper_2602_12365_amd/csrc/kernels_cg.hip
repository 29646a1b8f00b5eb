// Streaming kernels of the Krylov solve.  CG scalars live on the device: each
// reduction ends with the last workgroup (ticket counter) summing the block
// partials in block order -- deterministic -- and deriving the next scalars
// (alpha, beta, convergence), so that a batch of iterations runs without host
// round trips; once `done` is set every later kernel of the batch returns at
// once.  Vectors are float64 (plain solve) or float32 (mixed precision);
// every reduction accumulates in float64.
#include "efem_cg.h"

namespace efem {

constexpr int kThreads = 256;

__device__ __forceinline__ bool dof_fixed(const uint8_t *nmask, int64_t i)
{
    return nmask && ((nmask[i / 3] >> (i % 3)) & 1);
}

// Sum two per-thread values over the grid.  Returns true in thread 0 of the
// last block, with the totals in s0, s1.
__device__ bool grid_sum2(double a, double b, double *partials, uint32_t *counter, double &s0,
                          double &s1)
{
    __shared__ double ra[kThreads], rb[kThreads];
    __shared__ bool last;
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rb[threadIdx.x] += rb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = ra[0];
        partials[2 * blockIdx.x + 1] = rb[0];
        __threadfence();
        last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double x = 0.0, y = 0.0;
    for (unsigned i = threadIdx.x; i < gridDim.x; i += kThreads) {
        x += __hip_atomic_load(&partials[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        y += __hip_atomic_load(&partials[2 * i + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ra[threadIdx.x] = x;
    rb[threadIdx.x] = y;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rb[threadIdx.x] += rb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return false;
    s0 = ra[0];
    s1 = rb[0];
    *counter = 0u;
    return true;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < (n); i += (int64_t)gridDim.x * kThreads)

// r = sign * b (prescribed -> 0), z = dinv r, p = z, x = 0, q = 0; rz, rr.
template <class T>
__global__ void __launch_bounds__(kThreads) k_cg_init(int64_t n, const double *__restrict__ b,
                                                      double sign, const T *__restrict__ dinv,
                                                      const uint8_t *__restrict__ nmask,
                                                      T *__restrict__ x, T *__restrict__ r,
                                                      T *__restrict__ p, T *__restrict__ q,
                                                      CgScalars *sc, double eta2, double *partials,
                                                      uint32_t *counter)
{
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
    double s0, s1;
    if (grid_sum2(rz, rr, partials, counter, s0, s1)) {
        sc->rz = s0;
        sc->rr = s1;
        sc->bb = s1;
        sc->tol2 = eta2 * s1;
        sc->done = (s1 == 0.0) ? 1 : 0;
        sc->breakdown = 0;
        sc->iter = 0;
        sc->alpha = sc->beta = sc->pq = 0.0;
    }
}

// pq = p . q; alpha = rz / pq, or breakdown if pq <= 0 / not finite.
template <class T>
__global__ void __launch_bounds__(kThreads) k_cg_pq(int64_t n, const T *__restrict__ p,
                                                    const T *__restrict__ q, CgScalars *sc,
                                                    double *partials, uint32_t *counter)
{
    if (sc->done) return;
    double pq = 0.0;
    GRID_STRIDE(i, n) pq += (double)p[i] * (double)q[i];
    double s0, s1;
    if (grid_sum2(pq, 0.0, partials, counter, s0, s1)) {
        sc->pq = s0;
        if (!(s0 > 0.0) || !isfinite(s0)) {
            sc->breakdown = 1;
            sc->done = 1;
        } else {
            sc->alpha = sc->rz / s0;
        }
    }
}

// x += alpha p, r -= alpha q, q = 0; rr = r.r, rz_new = r.(dinv r);
// convergence when rr <= tol2; beta = rz_new / rz.
template <class T>
__global__ void __launch_bounds__(kThreads) k_cg_update(int64_t n, T *__restrict__ x,
                                                        T *__restrict__ r, const T *__restrict__ p,
                                                        T *__restrict__ q, const T *__restrict__ dinv,
                                                        CgScalars *sc, double *partials,
                                                        uint32_t *counter)
{
    if (sc->done) return;
    const T a = (T)sc->alpha;
    double rr = 0.0, rz = 0.0;
    GRID_STRIDE(i, n)
    {
        x[i] += a * p[i];
        const T ri = r[i] - a * q[i];
        r[i] = ri;
        q[i] = T(0);
        const T zi = dinv[i] * ri;
        rr += (double)ri * (double)ri;
        rz += (double)ri * (double)zi;
    }
    double s0, s1;
    if (grid_sum2(rr, rz, partials, counter, s0, s1)) {
        sc->rr = s0;
        sc->iter += 1;
        sc->beta = s1 / sc->rz;
        sc->rz = s1;
        if (s0 <= sc->tol2 || !isfinite(s0)) sc->done = 1;
    }
}

// p = dinv r + beta p
template <class T>
__global__ void __launch_bounds__(kThreads) k_cg_dir(int64_t n, T *__restrict__ p,
                                                     const T *__restrict__ r,
                                                     const T *__restrict__ dinv, const CgScalars *sc)
{
    if (sc->done) return;
    const T bt = (T)sc->beta;
    GRID_STRIDE(i, n) p[i] = dinv[i] * r[i] + bt * p[i];
}

// out = a . b (float64), masked entries count normally (callers pass masked vectors)
template <class TA, class TB>
__global__ void __launch_bounds__(kThreads) k_dot(int64_t n, const TA *__restrict__ a,
                                                  const TB *__restrict__ b, double *out,
                                                  double *partials, uint32_t *counter)
{
    double s = 0.0;
    GRID_STRIDE(i, n) s += (double)a[i] * (double)b[i];
    double s0, s1;
    if (grid_sum2(s, 0.0, partials, counter, s0, s1)) *out = s0;
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

static unsigned red_grid(int64_t n)
{
    int64_t g = (n + kThreads - 1) / kThreads;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, kMaxRedBlocks));
}

template <class T>
hipError_t CgLaunch<T>::init(const double *b, double sign, const T *dinv, const uint8_t *nmask,
                             T *x, T *r, T *p, T *q, CgScalars *sc, double eta2) const
{
    hipLaunchKernelGGL(k_cg_init<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, b, sign, dinv,
                       nmask, x, r, p, q, sc, eta2, ws.partials, ws.counter);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::pq(const T *p, const T *q, CgScalars *sc) const
{
    hipLaunchKernelGGL(k_cg_pq<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, p, q, sc, ws.partials,
                       ws.counter);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::update(T *x, T *r, const T *p, T *q, const T *dinv, CgScalars *sc) const
{
    hipLaunchKernelGGL(k_cg_update<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, x, r, p, q, dinv,
                       sc, ws.partials, ws.counter);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::dir(T *p, const T *r, const T *dinv, const CgScalars *sc) const
{
    hipLaunchKernelGGL(k_cg_dir<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, p, r, dinv, sc);
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
hipError_t CgLaunch<T>::scaled(const T *dinv, const double *b, double sign, T *x) const
{
    hipLaunchKernelGGL(k_scaled<T>, dim3(red_grid(n)), dim3(kThreads), 0, s, n, dinv, b, sign, x);
    return hipGetLastError();
}

template <class T>
hipError_t CgLaunch<T>::dot_state(const double *a, const T *b, double *out) const
{
    hipLaunchKernelGGL((k_dot<double, T>), dim3(red_grid(n)), dim3(kThreads), 0, s, n, a, b, out,
                       ws.partials, ws.counter);
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

hipError_t launch_dot64(hipStream_t s, const CgWorkspace &ws, int64_t n, const double *a,
                        const double *b, double *out)
{
    hipLaunchKernelGGL((k_dot<double, double>), dim3(red_grid(n)), dim3(kThreads), 0, s, n, a, b,
                       out, ws.partials, ws.counter);
    return hipGetLastError();
}

template struct CgLaunch<double>;
template struct CgLaunch<float>;

}  // namespace efem
