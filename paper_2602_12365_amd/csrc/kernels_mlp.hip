// Learned CG preconditioner kernels: node features over the 1-ring, the
// per-node MLP 12 -> 64 -> 64 -> 3 (softplus) on bf16 matrix cores, and its
// training (forward + backward on the vector units, Adam).
//
// Preconditioner (per node i, N(i) = nodes sharing an element with i):
//   g_i = D_i^-1 r_i (0 on prescribed DOFs), s_i = 1-ring RMS of g,
//   z_i = g_i + s_i * MLP(f_i), prescribed DOFs -> 0, with the 12 features
//   f = [g_i/s_i, mean_N(i) g/s_i, log(D_i / mean_{N(i)+i} D), prescribed
//   fraction of i, of N(i), |N(i)|/26].
// Weights and every layer input are rounded to bfloat16; accumulation is FP32.
#include "efem_mlp.h"

namespace efem {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (one hardware conversion on gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float bfr(float f) { return bf2f(f2bf(f)); }

// softplus(x) = max(x, 0) + ln(1 + t), t = e^-|x| in (0, 1], with the
// hardware base-2 exponential and logarithm (the exponent is <= 0 and the
// logarithm's argument lies in [1, 2], so neither needs range reduction).
// For x < 0 softplus is ln(1 + t) alone, so that term needs relative
// accuracy, which the logarithm of the rounded u = 1 + t lacks for small t
// (off by up to 2^-24 / t relative: several bfloat16 ulps once x < -12).
// The rounding error e = (1 + t) - u = t - (u - 1) is exact (u - 1 is exact
// for u in [1, 2], and t and u - 1 differ by at most an ulp of u), and
// ln(1 + t) = ln u + ln(1 + e/u) = ln u + e to within 2^-24 relative
// (|e| <= 2^-24, u >= 1); where 1 + t rounds to 1 this gives t itself.
__device__ __forceinline__ float softplus(float x)
{
    const float t = __builtin_amdgcn_exp2f(-fabsf(x) * 1.4426950408889634f);
    const float u = 1.f + t;
    const float e = t - (u - 1.f);
    return fmaxf(x, 0.f) + fmaf(0.6931471805599453f, __builtin_amdgcn_logf(u), e);
}
__device__ __forceinline__ float sigmoidf_(float x) { return 1.f / (1.f + __expf(-x)); }

// ------------------------------------------------------------------ features

// Static features (depend on the Jacobi diagonal and the mask only): slots 6..15.
__global__ void k_feat_static(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                              const double *__restrict__ diag, const uint8_t *__restrict__ nmask,
                              uint16_t *__restrict__ X)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t p0 = ptr[i], p1 = ptr[i + 1];
    const int deg = (int)(p1 - p0);
    double sd[3] = {diag[3 * i], diag[3 * i + 1], diag[3 * i + 2]};
    float sm = 0.f;
    for (int64_t p = p0; p < p1; ++p) {
        const int64_t j = idx[p];
        sd[0] += diag[3 * j];
        sd[1] += diag[3 * j + 1];
        sd[2] += diag[3 * j + 2];
        if (nmask) sm += (float)__popc(nmask[j]);
    }
    uint16_t *x = X + i * kInPad;
#pragma unroll
    for (int c = 0; c < 3; ++c) x[6 + c] = f2bf((float)log(diag[3 * i + c] / (sd[c] / (deg + 1))));
    const float mi = nmask ? (float)__popc(nmask[i]) : 0.f;
    x[9] = f2bf(mi / 3.f);
    x[10] = f2bf(sm / (3.f * (float)max(deg, 1)));
    x[11] = f2bf((float)deg / 26.f);
    x[12] = x[13] = x[14] = x[15] = 0;
}

// g = D^-1 r per node with |g|^2, one 16-byte record each, so that the
// 1-ring gather of the features reads one vector per neighbour.
__global__ void k_g4(int64_t n, const float *__restrict__ r, const float *__restrict__ dinv,
                     float4 *__restrict__ g4)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float a = r[3 * i] * dinv[3 * i], b = r[3 * i + 1] * dinv[3 * i + 1], c = r[3 * i + 2] * dinv[3 * i + 2];
    g4[i] = make_float4(a, b, c, a * a + b * b + c * c);
}

// Dynamic features (slots 0..5) and the scale s from g4 = (D^-1 r, |D^-1 r|^2)
// (dinv = 0 on prescribed DOFs).  The 1-ring comes column-major (ell[k][i],
// padded with the zero record g4[n]), so every neighbour slot is one
// coalesced index load; slots are taken two at a time.
__global__ void k_feat_dyn(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ ell,
                           int max_deg, const float4 *__restrict__ g4, uint16_t *__restrict__ X,
                           float *__restrict__ s_out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int deg = (int)(ptr[i + 1] - ptr[i]);
    const float4 gi = g4[i];
    const float g0 = gi.x, g1 = gi.y, g2 = gi.z;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, q = gi.w;
    int k = 0;
    for (; k + 2 <= max_deg; k += 2) {
        const float4 a = g4[ell[(int64_t)k * n + i]], b = g4[ell[(int64_t)(k + 1) * n + i]];
        s0 += a.x + b.x;
        s1 += a.y + b.y;
        s2 += a.z + b.z;
        q += a.w + b.w;
    }
    if (k < max_deg) {
        const float4 a = g4[ell[(int64_t)k * n + i]];
        s0 += a.x;
        s1 += a.y;
        s2 += a.z;
        q += a.w;
    }
    const float s = sqrtf(q / (3.f * (float)(deg + 1)));
    uint16_t *x = X + i * kInPad;
    if (s > 0.f) {
        const float rs = 1.f / s, rd = rs / (float)max(deg, 1);
        x[0] = f2bf(g0 * rs), x[1] = f2bf(g1 * rs), x[2] = f2bf(g2 * rs);
        x[3] = f2bf(s0 * rd), x[4] = f2bf(s1 * rd), x[5] = f2bf(s2 * rd);
    } else {
        x[0] = x[1] = x[2] = x[3] = x[4] = x[5] = 0;
    }
    s_out[i] = s;
}

// ------------------------------------------------------------- MLP forward

// One wave evaluates 16 nodes per step on 16x16x16 bf16 matrix cores, nodes on
// the N dimension: D[h][node] = sum_k W[h][k] H[k][node].  The accumulator
// layout (lane = node + 16*(h/4), element h%4) is the B-operand layout of the
// next layer, so activations never leave registers.  Lane l holds
//   A[m][k]: m = l%16, k = 4(l/16)+v;  B[k][n]: n = l%16, k = 4(l/16)+v;
//   D[m][n]: n = l%16, m = 4(l/16)+v.
struct MlpRegs {
    s4 A1[4], A2[4][4], A3[4];
    float B1[4][4], B2[4][4], B3[4];
};

__device__ __forceinline__ void load_weights(const uint16_t *__restrict__ W, MlpRegs &R)
{
    const int lane = threadIdx.x & 63, col = lane & 15, quad = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = 4 * quad + v;
            R.A1[t][v] = k < kIn ? (short)W[kOffW1 + (16 * t + col) * kIn + k] : (short)0;
            R.A3[t][v] = col < kOut ? (short)W[kOffW3 + col * kHid + 16 * t + k] : (short)0;
            R.B1[t][v] = bf2f(W[kOffB1 + 16 * t + k]);
            R.B2[t][v] = bf2f(W[kOffB2 + 16 * t + k]);
        }
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                R.A2[t2][t][v] = (short)W[kOffW2 + (16 * t2 + col) * kHid + 16 * t + 4 * quad + v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) R.B3[v] = (4 * quad + v < kOut) ? bf2f(W[kOffB3 + 4 * quad + v]) : 0.f;
}

// The bf16 activations of one hidden layer for this lane's node: hidden
// units 16 t + 4 quad + (0..3) of tile t, one 8-byte store per tile
// (H [n][64], only where node < n).
__device__ __forceinline__ void store_layer(uint16_t *__restrict__ H, const s4 h[4], int64_t node, int64_t n)
{
    if (node >= n) return;
    const int quad = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) *reinterpret_cast<s4 *>(H + node * kHid + 16 * t + 4 * quad) = h[t];
}

// out[v] for v < 3 is valid in lanes 0..15 (node = lane).  LAYERS: the two
// hidden layers' bf16 activations also go to H1 and H2 ([n][64]) for this
// lane's node.
template <bool LAYERS = false>
__device__ __forceinline__ f4 mlp16(const MlpRegs &R, s4 xb, uint16_t *H1 = nullptr, uint16_t *H2 = nullptr,
                                    int64_t node = 0, int64_t n = 0)
{
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    s4 hb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.A1[t], xb, zero, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) hb[t][v] = (short)f2bf(softplus(d[v] + R.B1[t][v]));
    }
    if constexpr (LAYERS) store_layer(H1, hb, node, n);
    s4 h2[4];
#pragma unroll
    for (int t2 = 0; t2 < 4; ++t2) {
        f4 d = zero;
#pragma unroll
        for (int t = 0; t < 4; ++t) d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.A2[t2][t], hb[t], d, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) h2[t2][v] = (short)f2bf(softplus(d[v] + R.B2[t2][v]));
    }
    if constexpr (LAYERS) store_layer(H2, h2, node, n);
    f4 o = zero;
#pragma unroll
    for (int t = 0; t < 4; ++t) o = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.A3[t], h2[t], o, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) o[v] += R.B3[v];
    return o;
}

__device__ __forceinline__ s4 load_x(const uint16_t *__restrict__ X, int64_t node, int64_t n)
{
    const int quad = (threadIdx.x & 63) >> 4;
    if (node >= n) return s4{0, 0, 0, 0};
    return *reinterpret_cast<const s4 *>(X + node * kInPad + 4 * quad);
}

// out [n, 3] = MLP(X); LAYERS: the hidden activations to H1, H2 as well
template <bool LAYERS>
__global__ void __launch_bounds__(256) k_mlp_forward(int64_t n, const uint16_t *__restrict__ X,
                                                     const uint16_t *__restrict__ W,
                                                     float *__restrict__ out, uint16_t *__restrict__ H1,
                                                     uint16_t *__restrict__ H2)
{
    MlpRegs R;
    load_weights(W, R);
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // the next group's features are loaded while this group is evaluated
    s4 xn = load_x(X, wave * 16 + (lane & 15), n);
    for (int64_t g0 = wave * 16; g0 < n; g0 += nw * 16) {
        const int64_t node = g0 + (lane & 15);
        const s4 xb = xn;
        xn = load_x(X, node + nw * 16, n);
        const f4 o = mlp16<LAYERS>(R, xb, H1, H2, node, n);
        if (lane < 16 && node < n) {
            out[3 * node] = o[0];
            out[3 * node + 1] = o[1];
            out[3 * node + 2] = o[2];
        }
    }
}

// z = g + s * MLP(X) with g = dinv r; z = 0 where dinv = 0 or s = 0;
// per-workgroup partials of r.z
__global__ void __launch_bounds__(256) k_mlp_apply(int64_t n, const uint16_t *__restrict__ X,
                                                   const uint16_t *__restrict__ W,
                                                   const float *__restrict__ r,
                                                   const float *__restrict__ dinv,
                                                   const float *__restrict__ s,
                                                   float *__restrict__ z, double *__restrict__ prz)
{
    __shared__ double red[256];
    MlpRegs R;
    load_weights(W, R);
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    double rz = 0.0;
    // the next group's features are loaded while this group is evaluated
    s4 xn = load_x(X, wave * 16 + (lane & 15), n);
    for (int64_t g0 = wave * 16; g0 < n; g0 += nw * 16) {
        const int64_t node = g0 + (lane & 15);
        const s4 xb = xn;
        xn = load_x(X, node + nw * 16, n);
        const f4 o = mlp16(R, xb);
        if (lane < 16 && node < n) {
            // z = g + gamma c with g = D^-1 r, c = s MLP; gamma < 1 only where
            // r_i.z_i would fall below half of r_i.g_i, so r.z >= r.D^-1 r / 2
            const float si = s[node];
            float ri[3], gi[3], ci[3], a = 0.f, b = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float di = dinv[3 * node + c];
                ri[c] = r[3 * node + c];
                gi[c] = ri[c] * di;
                ci[c] = (di == 0.f || si == 0.f) ? 0.f : si * o[c];
                a += ri[c] * gi[c];
                b += ri[c] * ci[c];
            }
            const float gam = (a + b < 0.5f * a) ? (-0.5f * a) / b : 1.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float zi = gi[c] + gam * ci[c];
                z[3 * node + c] = zi;
                rz += (double)ri[c] * (double)zi;
            }
        }
    }
    red[threadIdx.x] = rz;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) prz[blockIdx.x] = red[0];
}

// ------------------------------------------------- energy-norm training rows

// Block sum of one double per thread (256 threads); thread 0 gets the total.
__device__ __forceinline__ double block_sum256(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// z = m (g + s out) for one sample's rows aux = [g(3), t(3), m(3), s, w, 0];
// partials of r . g (the Jacobi share, which normalises the sample).
__global__ void __launch_bounds__(256) k_energy_z(int64_t n, const float *__restrict__ r,
                                                  const float *__restrict__ out,
                                                  const float *__restrict__ aux, float *__restrict__ z,
                                                  double *__restrict__ part)
{
    __shared__ double red[256];
    double rg = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float *a = aux + i * kAux;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            z[3 * i + c] = a[6 + c] * (a[c] + a[9] * out[3 * i + c]);
            rg += (double)r[3 * i + c] * (double)a[c];
        }
    }
    const double t = block_sum256(rg, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// With w = 1 / (n_samples r.g): aux w = w, aux t = (g + s out) - (K z - r), so
// that the target-fit loss gradient of the rows equals the gradient of
// w (z.Kz - 2 r.z); partials of that energy term.
__global__ void __launch_bounds__(256) k_energy_target(int64_t n, const float *__restrict__ r,
                                                       const float *__restrict__ out,
                                                       const float *__restrict__ z,
                                                       const float *__restrict__ kz, float *__restrict__ aux,
                                                       const double *__restrict__ rgpart, int G,
                                                       double n_samples, double *__restrict__ part)
{
    __shared__ double red[256];
    double rg = 0.0;
    for (int k = threadIdx.x; k < G; k += blockDim.x) rg += rgpart[k];
    rg = block_sum256(rg, red);
    const double w = rg > 0.0 ? 1.0 / (n_samples * rg) : 0.0;
    double e = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float *a = aux + i * kAux;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float ri = r[3 * i + c], zi = z[3 * i + c], ki = kz[3 * i + c];
            a[3 + c] = (a[c] + a[9] * out[3 * i + c]) - (ki - ri);
            e += (double)zi * (double)ki - 2.0 * (double)ri * (double)zi;
        }
        a[10] = (float)w;
    }
    const double t = block_sum256(e, red);
    if (threadIdx.x == 0) part[blockIdx.x] = w * t;
}

__global__ void __launch_bounds__(256) k_energy_acc(const double *__restrict__ part, int G,
                                                    double *__restrict__ energy)
{
    __shared__ double red[256];
    double e = 0.0;
    for (int k = threadIdx.x; k < G; k += blockDim.x) e += part[k];
    e = block_sum256(e, red);
    if (threadIdx.x == 0) *energy += e;
}

// ------------------------------------------------------------------ training

// Training rows of one sample: X (features of b), aux = [g(3), t(3), m(3), s, w, 0]
// with m = 1 on free DOFs, w = 1 / (|t|^2 n_total).  tt = |t|^2 (device scalar).
__global__ void k_rows_aux(int64_t n, const float *__restrict__ b, const float *__restrict__ dinv,
                           const float *__restrict__ t, const float *__restrict__ s,
                           const double *__restrict__ tt, double n_total, float *__restrict__ aux)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float *a = aux + i * kAux;
    const float w = (float)(1.0 / (tt[0] * n_total));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float d = dinv[3 * i + c];
        a[c] = b[3 * i + c] * d;
        a[3 + c] = t[3 * i + c];
        a[6 + c] = d == 0.f ? 0.f : 1.f;
    }
    a[9] = s[i];
    a[10] = w;
    a[11] = 0.f;
}

// Forward + backward on the vector units for rows of (X, aux); each workgroup
// loops over chunks of 16 rows and accumulates its share of the parameter
// gradient in registers, then writes one partial row [kP] and a loss partial.
// Matches the matrix-core forward: bf16 weights and layer inputs, FP32 sums;
// the roundings are treated as identity in the backward pass.
constexpr int kRowsPerChunk = 16;
constexpr int kGradPerThread = (kP + 255) / 256;

__global__ void __launch_bounds__(256) k_mlp_grad(int64_t rows, const uint16_t *__restrict__ X,
                                                  const float *__restrict__ aux,
                                                  const float *__restrict__ params,
                                                  float *__restrict__ gpart, double *__restrict__ lpart)
{
    __shared__ float Wl[kP];
    __shared__ float X0[kRowsPerChunk][kIn];
    __shared__ float A1[kRowsPerChunk][kHid], H1[kRowsPerChunk][kHid];
    __shared__ float A2[kRowsPerChunk][kHid], H2[kRowsPerChunk][kHid];
    __shared__ float DZ[kRowsPerChunk][kHid];
    __shared__ float DO[kRowsPerChunk][4];
    __shared__ double red[256];
    const int tid = threadIdx.x;
    for (int k = tid; k < kP; k += 256) Wl[k] = bfr(params[k]);
    float gacc[kGradPerThread];
#pragma unroll
    for (int q = 0; q < kGradPerThread; ++q) gacc[q] = 0.f;
    double loss = 0.0;
    const int rr = tid / 16;     // row of the chunk handled by this thread
    const int part = tid % 16;   // 4 hidden units each: 4*part .. 4*part+3
    __syncthreads();
    for (int64_t c0 = (int64_t)blockIdx.x * kRowsPerChunk; c0 < rows;
         c0 += (int64_t)gridDim.x * kRowsPerChunk) {
        const int64_t row = c0 + rr;
        const bool valid = row < rows;
        if (part < kIn) X0[rr][part] = valid ? bf2f(X[row * kInPad + part]) : 0.f;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int h = 4 * part + u;
            float a = Wl[kOffB1 + h];
#pragma unroll
            for (int k = 0; k < kIn; ++k) a += Wl[kOffW1 + h * kIn + k] * X0[rr][k];
            A1[rr][h] = a;
            H1[rr][h] = bfr(softplus(a));
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int h = 4 * part + u;
            float a = Wl[kOffB2 + h];
            for (int k = 0; k < kHid; ++k) a += Wl[kOffW2 + h * kHid + k] * H1[rr][k];
            A2[rr][h] = a;
            H2[rr][h] = bfr(softplus(a));
        }
        __syncthreads();
        if (part < kOut) {
            float o = Wl[kOffB3 + part];
            for (int k = 0; k < kHid; ++k) o += Wl[kOffW3 + part * kHid + k] * H2[rr][k];
            float d = 0.f;
            if (valid) {
                const float *a = aux + row * kAux;
                const float z = a[6 + part] * (a[part] + a[9] * o);
                const float e = z - a[6 + part] * a[3 + part];
                loss += (double)a[10] * (double)e * (double)e;
                d = 2.f * a[10] * a[9] * a[6 + part] * e;
            }
            DO[rr][part] = d;
        }
        __syncthreads();
        // dz2 = (W3^T dout) * sigmoid(a2)
        float dz2[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int h = 4 * part + u;
            const float dh = Wl[kOffW3 + h] * DO[rr][0] + Wl[kOffW3 + kHid + h] * DO[rr][1]
                           + Wl[kOffW3 + 2 * kHid + h] * DO[rr][2];
            dz2[u] = dh * sigmoidf_(A2[rr][h]);
        }
        __syncthreads();   // A2 is reused below as the dz2 store
#pragma unroll
        for (int u = 0; u < 4; ++u) A2[rr][4 * part + u] = dz2[u];
        __syncthreads();
        // dz1 = (W2^T dz2) * sigmoid(a1)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * part + u;
            float dh = 0.f;
            for (int h = 0; h < kHid; ++h) dh += Wl[kOffW2 + h * kHid + j] * A2[rr][h];
            DZ[rr][j] = dh * sigmoidf_(A1[rr][j]);
        }
        __syncthreads();
        // parameter gradients over the chunk's rows (A2 now holds dz2)
#pragma unroll
        for (int q = 0; q < kGradPerThread; ++q) {
            const int k = tid + 256 * q;
            if (k >= kP) continue;
            float g = 0.f;
            if (k < kOffB1) {
                const int h = k / kIn, c = k % kIn;
                for (int r2 = 0; r2 < kRowsPerChunk; ++r2) g += DZ[r2][h] * X0[r2][c];
            } else if (k < kOffW2) {
                const int h = k - kOffB1;
                for (int r2 = 0; r2 < kRowsPerChunk; ++r2) g += DZ[r2][h];
            } else if (k < kOffB2) {
                const int h = (k - kOffW2) / kHid, j = (k - kOffW2) % kHid;
                for (int r2 = 0; r2 < kRowsPerChunk; ++r2) g += A2[r2][h] * H1[r2][j];
            } else if (k < kOffW3) {
                const int h = k - kOffB2;
                for (int r2 = 0; r2 < kRowsPerChunk; ++r2) g += A2[r2][h];
            } else if (k < kOffB3) {
                const int c = (k - kOffW3) / kHid, h = (k - kOffW3) % kHid;
                for (int r2 = 0; r2 < kRowsPerChunk; ++r2) g += DO[r2][c] * H2[r2][h];
            } else {
                const int c = k - kOffB3;
                for (int r2 = 0; r2 < kRowsPerChunk; ++r2) g += DO[r2][c];
            }
            gacc[q] += g;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kGradPerThread; ++q) {
        const int k = tid + 256 * q;
        if (k < kP) gpart[(int64_t)blockIdx.x * kP + k] = gacc[q];
    }
    red[tid] = loss;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    if (tid == 0) lpart[blockIdx.x] = red[0];
}

// column sums of gpart [G][kP] (fixed order) and the loss partials
__global__ void k_grad_reduce(int G, const float *__restrict__ gpart, const double *__restrict__ lpart,
                              float *__restrict__ grad, double *__restrict__ loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kP) {
        double s = 0.0;
        for (int b = 0; b < G; ++b) s += gpart[(int64_t)b * kP + k];
        grad[k] = (float)s;
    }
    if (k == 0) {
        double s = 0.0;
        for (int b = 0; b < G; ++b) s += lpart[b];
        *loss = s;
    }
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float eps, int t)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kP) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / (1.f - powf(b1, (float)t)), vh = vk / (1.f - powf(b2, (float)t));
    p[k] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_to_bf16(const float *__restrict__ p, int n, uint16_t *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = f2bf(p[k]);
}

// |t|^2 of a float vector (one workgroup)
__global__ void k_norm2_f32(int64_t n, const float *__restrict__ t, double *__restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)t[i] * (double)t[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_dinv_f32(int64_t n, const double *__restrict__ diag, const uint8_t *__restrict__ nmask,
                           float *__restrict__ dinv)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool fixed = nmask && ((nmask[i / 3] >> (i % 3)) & 1);
    dinv[i] = fixed ? 0.f : (float)(1.0 / diag[i]);
}

// ---------------------------------------------------------------- launchers

static unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }
// The MLP kernels load the weights once per wave; a grid of about the
// resident wave count (3 waves per SIMD) spreads that over many node groups.
static unsigned mlp_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 63) / 64, 768)); }

hipError_t mlp_features_static(hipStream_t s, const MlpState &M, int64_t n, const double *diag,
                               const uint8_t *nmask, uint16_t *X)
{
    hipLaunchKernelGGL(k_feat_static, dim3(g256(n)), dim3(256), 0, s, n, M.ptr, M.idx, diag, nmask, X);
    return hipGetLastError();
}

hipError_t mlp_features_dyn(hipStream_t s, const MlpState &M, int64_t n, const float *r,
                            const float *dinv, uint16_t *X, float *scale, float4 *g4)
{
    hipLaunchKernelGGL(k_g4, dim3(g256(n)), dim3(256), 0, s, n, r, dinv, g4);
    hipLaunchKernelGGL(k_feat_dyn, dim3(g256(n)), dim3(256), 0, s, n, M.ptr, M.ell, M.max_deg, g4, X, scale);
    return hipGetLastError();
}

hipError_t mlp_forward(hipStream_t s, const uint16_t *W, int64_t n, const uint16_t *X, float *out, uint16_t *H1,
                       uint16_t *H2)
{
    if (H1 && H2)
        hipLaunchKernelGGL(k_mlp_forward<true>, dim3(mlp_grid(n)), dim3(256), 0, s, n, X, W, out, H1, H2);
    else
        hipLaunchKernelGGL(k_mlp_forward<false>, dim3(mlp_grid(n)), dim3(256), 0, s, n, X, W, out, H1, H2);
    return hipGetLastError();
}

int mlp_apply_grid(int64_t n) { return (int)mlp_grid(n); }

hipError_t mlp_apply(hipStream_t s, const uint16_t *W, int64_t n, const uint16_t *X, const float *r,
                     const float *dinv, const float *scale, float *z, double *prz)
{
    hipLaunchKernelGGL(k_mlp_apply, dim3(mlp_grid(n)), dim3(256), 0, s, n, X, W, r, dinv, scale, z, prz);
    return hipGetLastError();
}

hipError_t mlp_rows_aux(hipStream_t s, int64_t n, const float *b, const float *dinv, const float *t,
                        const float *scale, double *tt, double n_total, float *aux)
{
    hipLaunchKernelGGL(k_norm2_f32, dim3(1), dim3(256), 0, s, 3 * n, t, tt);
    hipLaunchKernelGGL(k_rows_aux, dim3(g256(n)), dim3(256), 0, s, n, b, dinv, t, scale, tt, n_total, aux);
    return hipGetLastError();
}

hipError_t mlp_loss_grad(hipStream_t s, int64_t rows, const uint16_t *X, const float *aux,
                         const float *params, float *gpart, double *lpart, int G, float *grad,
                         double *loss)
{
    hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(256), 0, s, rows, X, aux, params, gpart, lpart);
    hipLaunchKernelGGL(k_grad_reduce, dim3(g256(kP)), dim3(256), 0, s, G, gpart, lpart, grad, loss);
    return hipGetLastError();
}

hipError_t mlp_energy_z(hipStream_t s, int64_t n, const float *r, const float *out, const float *aux,
                        float *z, double *part, int G)
{
    hipLaunchKernelGGL(k_energy_z, dim3(G), dim3(256), 0, s, n, r, out, aux, z, part);
    return hipGetLastError();
}

hipError_t mlp_energy_target(hipStream_t s, int64_t n, const float *r, const float *out, const float *z,
                             const float *kz, float *aux, const double *rgpart, double n_samples,
                             double *part, int G, double *energy)
{
    hipLaunchKernelGGL(k_energy_target, dim3(G), dim3(256), 0, s, n, r, out, z, kz, aux, rgpart, G,
                       n_samples, part);
    hipLaunchKernelGGL(k_energy_acc, dim3(1), dim3(256), 0, s, part, G, energy);
    return hipGetLastError();
}

hipError_t mlp_adam(hipStream_t s, float *p, float *m, float *v, const float *g, float lr, float b1,
                    float b2, float eps, int t)
{
    hipLaunchKernelGGL(k_adam, dim3(g256(kP)), dim3(256), 0, s, p, m, v, g, lr, b1, b2, eps, t);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(hipStream_t s, const float *p, uint16_t *out)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(g256(kP)), dim3(256), 0, s, p, kP, out);
    return hipGetLastError();
}

hipError_t mlp_dinv_f32(hipStream_t s, int64_t n, const double *diag, const uint8_t *nmask, float *dinv)
{
    hipLaunchKernelGGL(k_dinv_f32, dim3(g256(n)), dim3(256), 0, s, n, diag, nmask, dinv);
    return hipGetLastError();
}

}  // namespace efem
