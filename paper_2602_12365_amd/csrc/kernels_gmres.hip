// Streaming kernels of the restarted GMRES solve: the multi-dot and the
// multi-axpy of classical Gram-Schmidt, and a few elementwise helpers.  All
// are bandwidth-bound passes over float64 vectors of length 3 n_nodes.
#include "efem_gmres.h"

namespace efem {

namespace {

constexpr int kT = 256;

#define GSTRIDE(i, n) \
    for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < (n); i += (int64_t)gridDim.x * kT)

unsigned grid_for(int64_t n)
{
    const int64_t g = (n + kT - 1) / kT;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 2048));
}

__device__ __forceinline__ bool fixed_dof(const uint8_t *nmask, int64_t i)
{
    return nmask && ((nmask[i / 3] >> (i % 3)) & 1);
}

// Each workgroup covers a grid-stride share of the entries.  A thread keeps
// the products with up to kChunk basis vectors in registers, so w is read
// once per chunk, then every sum is reduced across the wave with shuffles and
// across the four waves in LDS; partial j of workgroup g goes to part[j * G + g].
constexpr int kChunk = 16;

__global__ void __launch_bounds__(kT) k_mdot(int64_t n, const double *__restrict__ V, int k,
                                             const double *__restrict__ w, double *__restrict__ part)
{
    __shared__ double red[kT / 64][kChunk];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j0 = 0; j0 < k; j0 += kChunk) {
        const int kc = min(kChunk, k - j0);
        double acc[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j) acc[j] = 0.0;
        GSTRIDE(i, n) {
            const double wi = w[i];
#pragma unroll
            for (int j = 0; j < kChunk; ++j)
                if (j < kc) acc[j] += V[(int64_t)(j0 + j) * n + i] * wi;
        }
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            double v = acc[j];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) red[wave][j] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x < kc) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < kT / 64; ++q) t += red[q][threadIdx.x];
            part[(int64_t)(j0 + threadIdx.x) * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// one workgroup per j: fixed-order sum of the G partials
__global__ void __launch_bounds__(kT) k_mdot_fin(const double *__restrict__ part, int G, double *__restrict__ h)
{
    __shared__ double red[kT];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += kT) s += part[(int64_t)j * G + g];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int q = kT / 2; q > 0; q >>= 1) {
        if ((int)threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[j] = red[0];
}

__global__ void __launch_bounds__(kT) k_subtract(int64_t n, const double *__restrict__ V, int k,
                                                 const double *__restrict__ h, double *__restrict__ w)
{
    __shared__ double hs[kGmresMaxRestart + 1];
    for (int j = threadIdx.x; j < k; j += kT) hs[j] = h[j];
    __syncthreads();
    GSTRIDE(i, n) {
        double t = w[i];
        int j = 0;
        for (; j + 4 <= k; j += 4)
            t -= (hs[j] * V[(int64_t)j * n + i] + hs[j + 1] * V[(int64_t)(j + 1) * n + i])
               + (hs[j + 2] * V[(int64_t)(j + 2) * n + i] + hs[j + 3] * V[(int64_t)(j + 3) * n + i]);
        for (; j < k; ++j) t -= hs[j] * V[(int64_t)j * n + i];
        w[i] = t;
    }
}

__global__ void __launch_bounds__(kT) k_scale(int64_t n, double alpha, const double *__restrict__ w,
                                              double *__restrict__ out)
{
    GSTRIDE(i, n) out[i] = alpha * w[i];
}

__global__ void __launch_bounds__(kT) k_mul(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                                            double *__restrict__ out)
{
    GSTRIDE(i, n) out[i] = a[i] * b[i];
}

__global__ void __launch_bounds__(kT) k_residual(int64_t n, const double *__restrict__ b,
                                                 const double *__restrict__ kx, const uint8_t *__restrict__ nmask,
                                                 double *__restrict__ out)
{
    GSTRIDE(i, n) out[i] = fixed_dof(nmask, i) ? 0.0 : b[i] - kx[i];
}

__global__ void __launch_bounds__(kT) k_update_x(int64_t n, const double *__restrict__ V, int k,
                                                 const double *__restrict__ y, const double *__restrict__ dinv,
                                                 double *__restrict__ x)
{
    GSTRIDE(i, n) {
        double t = 0.0;
        for (int j = 0; j < k; ++j) t += y[j] * V[(int64_t)j * n + i];
        x[i] += dinv[i] * t;
    }
}

__global__ void __launch_bounds__(kT) k_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ out)
{
    GSTRIDE(i, n) out[i] = (float)a[i];
}

__global__ void __launch_bounds__(kT) k_to_f64(int64_t n, const float *__restrict__ a, double *__restrict__ out)
{
    GSTRIDE(i, n) out[i] = (double)a[i];
}

__global__ void __launch_bounds__(kT) k_gm_dinv(int64_t n, const double *__restrict__ diag,
                                                const uint8_t *__restrict__ nmask, double *__restrict__ dinv)
{
    GSTRIDE(i, n) dinv[i] = fixed_dof(nmask, i) ? 0.0 : 1.0 / diag[i];
}

}  // namespace

hipError_t gm_mdot(hipStream_t s, int64_t n, const double *V, int k, const double *w, double *part, double *h)
{
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mdot, dim3(kGmresRedBlocks), dim3(kT), 0, s, n, V, k, w, part);
    hipLaunchKernelGGL(k_mdot_fin, dim3(k), dim3(kT), 0, s, part, kGmresRedBlocks, h);
    return hipGetLastError();
}

hipError_t gm_subtract(hipStream_t s, int64_t n, const double *V, int k, const double *h, double *w)
{
    hipLaunchKernelGGL(k_subtract, dim3(grid_for(n)), dim3(kT), 0, s, n, V, k, h, w);
    return hipGetLastError();
}

hipError_t gm_scale(hipStream_t s, int64_t n, double alpha, const double *w, double *out)
{
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kT), 0, s, n, alpha, w, out);
    return hipGetLastError();
}

hipError_t gm_mul(hipStream_t s, int64_t n, const double *a, const double *b, double *out)
{
    hipLaunchKernelGGL(k_mul, dim3(grid_for(n)), dim3(kT), 0, s, n, a, b, out);
    return hipGetLastError();
}

hipError_t gm_residual(hipStream_t s, int64_t n, const double *b, const double *kx, const uint8_t *nmask,
                       double *out)
{
    hipLaunchKernelGGL(k_residual, dim3(grid_for(n)), dim3(kT), 0, s, n, b, kx, nmask, out);
    return hipGetLastError();
}

hipError_t gm_update_x(hipStream_t s, int64_t n, const double *V, int k, const double *y, const double *dinv,
                       double *x)
{
    hipLaunchKernelGGL(k_update_x, dim3(grid_for(n)), dim3(kT), 0, s, n, V, k, y, dinv, x);
    return hipGetLastError();
}

hipError_t gm_to_f32(hipStream_t s, int64_t n, const double *a, float *out)
{
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(kT), 0, s, n, a, out);
    return hipGetLastError();
}

hipError_t gm_to_f64(hipStream_t s, int64_t n, const float *a, double *out)
{
    hipLaunchKernelGGL(k_to_f64, dim3(grid_for(n)), dim3(kT), 0, s, n, a, out);
    return hipGetLastError();
}

hipError_t gm_dinv(hipStream_t s, int64_t n, const double *diag, const uint8_t *nmask, double *dinv)
{
    hipLaunchKernelGGL(k_gm_dinv, dim3(grid_for(n)), dim3(kT), 0, s, n, diag, nmask, dinv);
    return hipGetLastError();
}

}  // namespace efem
