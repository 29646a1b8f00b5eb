// Element kernels of the energy-based FEM hot path for gfx950 (MI355X).
//
// Every operator is one pass over element blocks, one workgroup per block:
//   1. stage the block's distinct nodes (coordinates, state, direction) from
//      HBM into LDS, once per block (the gather of Alg. 1);
//   2. one thread per element: reference-space gradients, quadrature-point
//      math, element forces accumulated into LDS with LDS atomics;
//   3. write the block's nodal sums out: nodes owned by this block alone with
//      plain stores, nodes shared with other blocks with global atomics (or,
//      in the colour scatter, with a plain read-modify-write per colour).
// The energy reduces per block and a one-workgroup kernel sums the block
// partials in block order, so the energy is bitwise deterministic.  Nodal sums
// are accumulated in FP64 in LDS for both precisions.
//
// Quadrature-point math (Eq. 2 and its exact derivatives, Eqs. 1 and 3) is
// written in terms of the reference Jacobian Jx = dX/dxi, the deformed one
// Jd = dx/dxi and the direction's dJ = dv/dxi, so that no 81-entry tangent is
// ever formed.  With Ae = adj(Jx), De = det Jx, Ad = adj(Jd), Dd = det Jd,
// J = Dd/De, c1 = mu - lam ln J, S = Ae Ae^T, the element forces are
// f_a = Q dN_a/dxi with, for the tangent action,
//   Q = w [ mu/De dJ S + lam De tr(Ad dJ)/Dd^2 Ad^T + c1 De/Dd^2 (Ad dJ Ad)^T ],
// which is w det Jx dP Jx^-T with dP = mu dF + lam tr(F^-1 dF) F^-T
// + c1 F^-T dF^T F^-T, F = Jd Jx^-1, dF = dJ Jx^-1.
#include <mutex>

#include "efem_internal.h"

namespace efem {

// ------------------------------------------------------------------ helpers

// Workgroup i runs on XCD i % 8.  Give each XCD a contiguous range of
// (Morton-ordered) blocks so that blocks sharing nodes share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int n)
{
    constexpr int NX = 8;
    const int q = n / NX, r = n % NX;
    const int x = bid % NX, k = bid / NX;
    return x * q + min(x, r) + k;
}

template <class T>
__device__ __forceinline__ T adj_det(const T m[9], T a[9])
{
    a[0] = m[4] * m[8] - m[5] * m[7];
    a[1] = m[2] * m[7] - m[1] * m[8];
    a[2] = m[1] * m[5] - m[2] * m[4];
    a[3] = m[5] * m[6] - m[3] * m[8];
    a[4] = m[0] * m[8] - m[2] * m[6];
    a[5] = m[2] * m[3] - m[0] * m[5];
    a[6] = m[3] * m[7] - m[4] * m[6];
    a[7] = m[1] * m[6] - m[0] * m[7];
    a[8] = m[0] * m[4] - m[1] * m[3];
    return m[0] * a[0] + m[1] * a[3] + m[2] * a[6];
}

// adj_det with the adjugate's last row given: row 2 of adj(m) is the cross
// product of m's first two columns, which the two tetrahedra of a face pair
// share up to sign (their first two edges are the shared face's, swapped)
template <class T>
__device__ __forceinline__ T adj_det_row2(const T m[9], const T r2[3], T a[9])
{
    a[0] = m[4] * m[8] - m[5] * m[7];
    a[1] = m[2] * m[7] - m[1] * m[8];
    a[2] = m[1] * m[5] - m[2] * m[4];
    a[3] = m[5] * m[6] - m[3] * m[8];
    a[4] = m[0] * m[8] - m[2] * m[6];
    a[5] = m[2] * m[3] - m[0] * m[5];
    a[6] = r2[0];
    a[7] = r2[1];
    a[8] = r2[2];
    return m[0] * a[0] + m[1] * a[3] + m[2] * a[6];
}

// Reciprocal: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r) (each step squares the relative error), so the FP64
// result is correct to about an ulp for the normal-range determinants used
// here; FP32 uses the hardware reciprocal directly (1 ulp).
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Natural logarithms for the material law.  The device library's FP64 log
// costs about 100 instructions (general special-case handling); these cost
// about 25.  Method: the exponent split y = 2^k m with m in [1/sqrt2, sqrt2),
// then ln m = 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 3 - 2 sqrt2 = 0.1716,
// by its odd power series 2 (s + s^3/3 + ... + s^19/19); the first omitted
// term, s^21/21, is below 2.4e-17 of the sum.  m - 1 is exact (Sterbenz), and
// the quotient gets one residual correction, so the result is within a few
// ulp.  Arguments must be positive and finite (the callers flag det F <= 0
// before the value is used).
// The series coefficients 1/19, 1/17, ..., 1/3 live in constant memory: read
// with scalar loads they sit in scalar registers, where the compiler would
// otherwise keep 16 vector registers of constants across the element loops.
__constant__ double kAtanhCoef[9] = {1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0,
                                     1.0 / 9.0,  1.0 / 7.0,  1.0 / 5.0,  1.0 / 3.0};
__device__ __forceinline__ double two_atanh(double s)
{
    const double z = s * s;
    double p = kAtanhCoef[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) p = fma(p, z, kAtanhCoef[i]);
    const double s2 = s + s;
    return fma(s2 * z, p, s2);
}

// t / d to within about half an ulp: the refined reciprocal, then one
// residual step on the quotient.
__device__ __forceinline__ double quot(double t, double d)
{
    const double r = rcp(d);
    const double q = t * r;
    return fma(fma(-q, d, t), r, q);
}

constexpr double kLn2 = 0.69314718055994530942;   // rounded once to double
constexpr double kSqrtHalf = 0.70710678118654752440;

// y = 2^k m, m in [1/sqrt2, sqrt2)
__device__ __forceinline__ double split_exp(double y, int &k)
{
    double m = __builtin_amdgcn_frexp_mant(y);   // [0.5, 1)
    k = __builtin_amdgcn_frexp_exp(y);
    const bool lo = m < kSqrtHalf;
    m = lo ? m + m : m;
    k = lo ? k - 1 : k;
    return m;
}

__device__ __forceinline__ double log_(double x)
{
    int k;
    const double m = split_exp(x, k);
    return fma((double)k, kLn2, two_atanh(quot(m - 1.0, m + 1.0)));
}

// ln(1 + x) for x > -1.  When 1 + x lies in [1/sqrt2, sqrt2) the argument
// s = x / (2 + x) is formed from x itself, so the rounding of 1 + x never
// enters (this is where ln J is small and the energy cancels to second order).
__device__ __forceinline__ double log1p_(double x)
{
    int k;
    const double m = split_exp(1.0 + x, k);
    const bool near = k == 0;
    const double t = near ? x : m - 1.0;
    const double d = near ? 2.0 + x : m + 1.0;
    return fma((double)k, kLn2, two_atanh(quot(t, d)));
}

__device__ __forceinline__ float log_(float x) { return __logf(x); }

__device__ __forceinline__ void flag_inverted(int32_t *flags) { atomicOr(flags, 1); }

// ------------------------------------------------------------ element types

// Work items.  An item is what one thread computes: a pair of tetrahedra that
// share a face, or one hexahedron.  NEN nodes per item, NQ quadrature points
// per item, NSUB elements per item (sub(q) is the element of point q).
//
// Interface of an item type E:
//   Field<T>, prep(f, F)      what the gradients are formed from, given the
//                             NEN nodal values f of one field;
//   grad(F, q, G)             G[i*3+J] = d f_i / d xi_J at point q;
//   Acc<T>, add_forces<INIT>(Q, q, A), finish(A, out)
//                             nodal forces out_a = sum_q Q_q dN_a/dxi(q)
//                             (INIT: the points arrive in ascending order and
//                             none is skipped but possibly the last, starting
//                             from an uninitialised A; otherwise A was zeroed
//                             and every point adds);
//   dN(q, a, J)               the shape-function derivatives themselves.
//
// Tet4 pair: nodes (a, b, c, d1, d2) with tet 1 = (a, b, c, d1) positively
// oriented and tet 2 = (a, c, b, d2), also positive since d2 lies on the
// other side of the shared face.  A tetrahedron without a partner is stored as
// (n0, n1, n2, n3, n3) and its second point skipped.
// Each tetrahedron: N0 = 1 - xi - eta - zeta, N_k = xi_k; one point, w = 1/6.
struct Tet4Pair {
    static constexpr int NEN = 5, NQ = 2, NSUB = 2;
    using Lean = Tet4Pair;   // the form with the fewest live registers
    // completes the gradient of a coordinate field (planar elements only)
    template <class T> __device__ static __forceinline__ void geom(T *) {}
    template <class T> __device__ static constexpr T weight() { return T(1.0 / 6.0); }
    __device__ static constexpr int sub(int q) { return q; }
    // the second point of an unpaired tetrahedron is skipped
    __device__ static constexpr bool skip(int q, bool pair) { return q > 0 && !pair; }
    // pair node of local tet node k (k = 0..3) of tet q
    __device__ static constexpr int node(int q, int k)
    {
        return q == 0 ? k : (k == 1 ? 2 : (k == 2 ? 1 : (k == 3 ? 4 : 0)));
    }
    template <class T> struct Field {
        T f[NEN][3];
    };
    template <class T>
    __device__ static __forceinline__ void prep(const T f[NEN][3], Field<T> &F)
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) F.f[a][i] = f[a][i];
    }
    template <class T>
    __device__ static __forceinline__ void grad(const Field<T> &F, int q, T G[9])
    {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int J = 0; J < 3; ++J) G[i * 3 + J] = F.f[node(q, J + 1)][i] - F.f[0][i];
    }
    template <class T> struct Acc {
        T f[NEN][3];
    };
    template <class T> __device__ static __forceinline__ void zero(Acc<T> &A)
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a) A.f[a][0] = A.f[a][1] = A.f[a][2] = T(0);
    }
    // Node forms accumulate straight into the caller's nodal array.  INIT:
    // points arrive in ascending order from an uninitialised accumulator (the
    // first point assigns); otherwise every point adds.
    template <bool INIT, class T>
    __device__ static __forceinline__ void add_forces_to(const T Q[9], int q, T out[NEN][3])
    {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T s = -(Q[i * 3 + 0] + Q[i * 3 + 1] + Q[i * 3 + 2]);
            if (INIT && q == 0) {   // point 0 of tet 1 touches nodes 0..3 only
                out[node(q, 1)][i] = Q[i * 3 + 0];
                out[node(q, 2)][i] = Q[i * 3 + 1];
                out[node(q, 3)][i] = Q[i * 3 + 2];
                out[0][i] = s;
                out[4][i] = T(0);
            } else {
                out[node(q, 1)][i] += Q[i * 3 + 0];
                out[node(q, 2)][i] += Q[i * 3 + 1];
                out[node(q, 3)][i] += Q[i * 3 + 2];
                out[0][i] += s;
            }
        }
    }
    template <bool INIT, class T>
    __device__ static __forceinline__ void add_forces(const T Q[9], int q, Acc<T> &A)
    {
        add_forces_to<INIT>(Q, q, A.f);
    }
    template <class T>
    __device__ static __forceinline__ void finish(const Acc<T> &A, T out[NEN][3])
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) out[a][i] = A.f[a][i];
    }
    // The pair's forces on nodes 1..4, points in order 0, 1 (1 possibly
    // skipped); node 0 is left to close0.  Each tetrahedron's nodal forces sum
    // to zero (its shape functions sum to one), so node 0 carries minus the
    // sum of the others, which saves each point its own node-0 sum.
    template <class T>
    __device__ static __forceinline__ void add_forces_open(const T Q[9], int q, T out[NEN][3])
    {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (q == 0) {
                out[1][i] = Q[i * 3 + 0];
                out[2][i] = Q[i * 3 + 1];
                out[3][i] = Q[i * 3 + 2];
                out[4][i] = T(0);
            } else {   // tet 2 = (a, c, b, d2); only it touches node 4
                out[2][i] += Q[i * 3 + 0];
                out[1][i] += Q[i * 3 + 1];
                out[4][i] = Q[i * 3 + 2];
            }
        }
    }
    template <class T> __device__ static __forceinline__ void close0(T out[NEN][3])
    {
#pragma unroll
        for (int i = 0; i < 3; ++i) out[0][i] = -((out[1][i] + out[2][i]) + (out[3][i] + out[4][i]));
    }
    // d N_a / d xi_J of pair node a at point q (0 for the node outside tet q)
    template <class T> __device__ static __forceinline__ T dN(int q, int a, int J)
    {
        if (a == 0) return T(-1);
        return node(q, J + 1) == a ? T(1) : T(0);
    }
    // N_a at point q, the centroid of tet q: 1/4 on its four nodes
    template <class T> __device__ static __forceinline__ T N(int q, int a)
    {
        return (q == 0 ? a != 4 : a != 3) ? T(0.25) : T(0);
    }
};

// Tri3: linear triangle in the x-y plane, one centroid point, weight 1/2 (the
// reference area), unit thickness.  The third reference direction is the
// thickness: no field varies along it, so grad() leaves column 2 zero and
// geom() puts the unit z column into the gradient of a coordinate field, which
// makes Jx = [Jx_2D 0; 0 1] and, with u_z held, F = [F_2D 0; 0 1] (plane strain).
struct Tri3 {
    static constexpr int NEN = 3, NQ = 1, NSUB = 1;
    using Lean = Tri3;
    template <class T> __device__ static constexpr T weight() { return T(0.5); }
    __device__ static constexpr int sub(int) { return 0; }
    __device__ static constexpr bool skip(int, bool) { return false; }
    template <class T> __device__ static __forceinline__ void geom(T *G) { G[8] += T(1); }
    template <class T> struct Field {
        T f[NEN][3];
    };
    template <class T>
    __device__ static __forceinline__ void prep(const T f[NEN][3], Field<T> &F)
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) F.f[a][i] = f[a][i];
    }
    template <class T>
    __device__ static __forceinline__ void grad(const Field<T> &F, int, T G[9])
    {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            G[i * 3 + 0] = F.f[1][i] - F.f[0][i];
            G[i * 3 + 1] = F.f[2][i] - F.f[0][i];
            G[i * 3 + 2] = T(0);
        }
    }
    template <class T> struct Acc {
        T f[NEN][3];
    };
    template <class T> __device__ static __forceinline__ void zero(Acc<T> &A)
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a) A.f[a][0] = A.f[a][1] = A.f[a][2] = T(0);
    }
    template <bool INIT, class T>
    __device__ static __forceinline__ void add_forces_to(const T Q[9], int, T out[NEN][3])
    {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T s = -(Q[i * 3 + 0] + Q[i * 3 + 1]);
            if (INIT) {
                out[1][i] = Q[i * 3 + 0];
                out[2][i] = Q[i * 3 + 1];
                out[0][i] = s;
            } else {
                out[1][i] += Q[i * 3 + 0];
                out[2][i] += Q[i * 3 + 1];
                out[0][i] += s;
            }
        }
    }
    template <bool INIT, class T>
    __device__ static __forceinline__ void add_forces(const T Q[9], int q, Acc<T> &A)
    {
        add_forces_to<INIT>(Q, q, A.f);
    }
    template <class T>
    __device__ static __forceinline__ void finish(const Acc<T> &A, T out[NEN][3])
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) out[a][i] = A.f[a][i];
    }
    template <class T> __device__ static __forceinline__ T dN(int, int a, int J)
    {
        if (J == 2) return T(0);
        if (a == 0) return T(-1);
        return a == J + 1 ? T(1) : T(0);
    }
    template <class T> __device__ static __forceinline__ T N(int, int) { return T(1.0 / 3.0); }
};

// Hex8 in node form: the same element with gradients and forces as sums over
// the 8 nodes (8 terms per entry).  It keeps 24 values per field live instead
// of 36, which is what the three-field FP64 tangent action needs to stay out
// of scratch memory.
__device__ constexpr int kHexSgn[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                          {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
struct Hex8Nodes {
    static constexpr int NEN = 8;
    template <class T> __device__ static __forceinline__ void geom(T *) {}
    template <class T> __device__ static __forceinline__ T dN(int q, int a, int J)
    {
        const T g = T(0.57735026918962576451);
        const T p0 = (q & 1) ? g : -g, p1 = (q & 2) ? g : -g, p2 = (q & 4) ? g : -g;
        const T f0 = T(1) + T(kHexSgn[a][0]) * p0;
        const T f1 = T(1) + T(kHexSgn[a][1]) * p1;
        const T f2 = T(1) + T(kHexSgn[a][2]) * p2;
        const T s = T(0.125) * T(kHexSgn[a][J]);
        return J == 0 ? s * f1 * f2 : (J == 1 ? s * f0 * f2 : s * f0 * f1);
    }
    // N_a at Gauss point q
    template <class T> __device__ static __forceinline__ T N(int q, int a)
    {
        const T g = T(0.57735026918962576451);
        const T p0 = (q & 1) ? g : -g, p1 = (q & 2) ? g : -g, p2 = (q & 4) ? g : -g;
        return T(0.125) * (T(1) + T(kHexSgn[a][0]) * p0) * (T(1) + T(kHexSgn[a][1]) * p1)
             * (T(1) + T(kHexSgn[a][2]) * p2);
    }
    template <class T> struct Field {
        T f[NEN][3];
    };
    template <class T>
    __device__ static __forceinline__ void prep(const T f[NEN][3], Field<T> &F)
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) F.f[a][i] = f[a][i];
    }
    template <class T>
    __device__ static __forceinline__ void grad(const Field<T> &F, int q, T G[9])
    {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int J = 0; J < 3; ++J) {
                T t = T(0);
#pragma unroll
                for (int a = 0; a < NEN; ++a) t += F.f[a][i] * dN<T>(q, a, J);
                G[i * 3 + J] = t;
            }
    }
    template <class T> struct Acc {
        T f[NEN][3];
    };
    template <class T> __device__ static __forceinline__ void zero(Acc<T> &A)
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a) A.f[a][0] = A.f[a][1] = A.f[a][2] = T(0);
    }
    template <bool INIT, class T>
    __device__ static __forceinline__ void add_forces_to(const T Q[9], int q, T out[NEN][3])
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (INIT && q == 0) out[a][i] = T(0);
                out[a][i] += Q[i * 3 + 0] * dN<T>(q, a, 0) + Q[i * 3 + 1] * dN<T>(q, a, 1)
                           + Q[i * 3 + 2] * dN<T>(q, a, 2);
            }
    }
    template <bool INIT, class T>
    __device__ static __forceinline__ void add_forces(const T Q[9], int q, Acc<T> &A)
    {
        add_forces_to<INIT>(Q, q, A.f);
    }
    template <class T>
    __device__ static __forceinline__ void finish(const Acc<T> &A, T out[NEN][3])
    {
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) out[a][i] = A.f[a][i];
    }
};

// Hex8: trilinear on [-1,1]^3, nodes (0,0,0),(1,0,0),(1,1,0),(0,1,0) then z=1;
// 2x2x2 Gauss points at +-1/sqrt(3), point q = qx + 2 qy + 4 qz, w = 1.
//
// The derivative of a trilinear field along one reference direction depends
// only on the differences along the four element edges of that direction,
// interpolated bilinearly in the other two coordinates:
//   d f / d xi_J (q) = sum_e w_J(e, q) (f[e+] - f[e-]),
//   w_J(e, q) = (1 + s1_e p1_q)(1 + s2_e p2_q) / 8,
// with (s1_e, s2_e) the signs of edge e in the two other directions and p_q
// the point's coordinates.  So the gradient is formed from 12 edge
// differences per field (36 subtractions per element, shared by the 8
// points) and 4 terms per entry instead of 8; the nodal forces take the
// transposed route through 12 edge accumulators.
__device__ constexpr int kHexS[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                        {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
// edges (e-, e+) of each direction J, ordered by the signs of the other two
// directions (the lower-numbered one varies fastest)
__device__ constexpr int kHexEdge[3][4][2] = {{{0, 1}, {3, 2}, {4, 5}, {7, 6}},
                                              {{0, 3}, {1, 2}, {4, 7}, {5, 6}},
                                              {{0, 4}, {1, 5}, {3, 7}, {2, 6}}};
struct Hex8 {
    static constexpr int NEN = 8, NQ = 8, NSUB = 1;
    using Lean = Hex8Nodes;   // the form with the fewest live registers
    template <class T> __device__ static __forceinline__ void geom(T *) {}
    template <class T> __device__ static constexpr T weight() { return T(1); }
    __device__ static constexpr int sub(int) { return 0; }
    __device__ static constexpr bool skip(int, bool) { return false; }
    static constexpr double kG = 0.57735026918962576451;   // 1/sqrt(3)
    // the two directions other than J
    __device__ static constexpr int oth1(int J) { return J == 0 ? 1 : 0; }
    __device__ static constexpr int oth2(int J) { return J == 2 ? 1 : 2; }
    // which of the 4 columns of direction J point q uses: its coordinate
    // signs in the two other directions
    __device__ static constexpr int col(int J, int q)
    {
        return ((q >> oth1(J)) & 1) + 2 * ((q >> oth2(J)) & 1);
    }
    // (1 + s p g) for edge sign s and point coordinate sign p, and its eighth
    __device__ static constexpr double lw(int s_pos, int p_pos)
    {
        return 1.0 + ((s_pos == p_pos) ? kG : -kG);
    }
    __device__ static constexpr double lw8(int s_pos, int p_pos) { return 0.125 * lw(s_pos, p_pos); }
    // index of the edge of direction J that node a ends
    __device__ static constexpr int edge_of(int J, int a)
    {
        return (kHexS[a][oth1(J)] > 0 ? 1 : 0) + (kHexS[a][oth2(J)] > 0 ? 2 : 0);
    }
    // The 12 distinct gradient columns of a field: c[J][k] = d f / d xi_J at
    // the points whose other two coordinates have signs k (4 combinations),
    // from the 4 edge differences of direction J by one interpolation along
    // each of the two other directions.
    template <class T> struct Field {
        T c[3][4][3];   // [direction][column][component]
    };
    template <class T>
    __device__ static __forceinline__ void prep(const T f[NEN][3], Field<T> &F)
    {
#pragma unroll
        for (int J = 0; J < 3; ++J)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T d[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) d[e] = f[kHexEdge[J][e][1]][i] - f[kHexEdge[J][e][0]][i];
                // along the first other direction: A[p1][lev], lev = edge sign in the second
                T A[2][2];
#pragma unroll
                for (int p1 = 0; p1 < 2; ++p1)
#pragma unroll
                    for (int lev = 0; lev < 2; ++lev)
                        A[p1][lev] = fma(T(lw(1, p1)), d[1 + 2 * lev], T(lw(0, p1)) * d[2 * lev]);
#pragma unroll
                for (int p1 = 0; p1 < 2; ++p1)
#pragma unroll
                    for (int p2 = 0; p2 < 2; ++p2)
                        F.c[J][p1 + 2 * p2][i] = fma(T(lw8(1, p2)), A[p1][1], T(lw8(0, p2)) * A[p1][0]);
            }
    }
    template <class T>
    __device__ static __forceinline__ void grad(const Field<T> &F, int q, T G[9])
    {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int J = 0; J < 3; ++J) G[i * 3 + J] = F.c[J][col(J, q)][i];
    }
    // forces: the transposed route, columns -> edges -> nodes
    template <class T> struct Acc {
        T c[3][4][3];
    };
    template <class T> __device__ static __forceinline__ void zero(Acc<T> &A)
    {
#pragma unroll
        for (int J = 0; J < 3; ++J)
#pragma unroll
            for (int k = 0; k < 4; ++k) A.c[J][k][0] = A.c[J][k][1] = A.c[J][k][2] = T(0);
    }
    // INIT: points arrive in ascending order from an uninitialised accumulator,
    // so a column is assigned at its first point (coordinate J negative)
    template <bool INIT, class T>
    __device__ static __forceinline__ void add_forces(const T Q[9], int q, Acc<T> &A)
    {
#pragma unroll
        for (int J = 0; J < 3; ++J)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T &a = A.c[J][col(J, q)][i];
                if (INIT && !((q >> J) & 1)) a = Q[i * 3 + J];
                else a += Q[i * 3 + J];
            }
    }
    template <class T>
    __device__ static __forceinline__ void finish(const Acc<T> &A, T out[NEN][3])
    {
        T E[3][4][3];   // edge forces: +E to the edge's + end, -E to its - end
#pragma unroll
        for (int J = 0; J < 3; ++J)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T B[2][2];   // [p1][lev]
#pragma unroll
                for (int p1 = 0; p1 < 2; ++p1)
#pragma unroll
                    for (int lev = 0; lev < 2; ++lev)
                        B[p1][lev] = fma(T(lw8(lev, 1)), A.c[J][p1 + 2][i], T(lw8(lev, 0)) * A.c[J][p1][i]);
#pragma unroll
                for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
                    for (int lev = 0; lev < 2; ++lev)
                        E[J][s1 + 2 * lev][i] = fma(T(lw(s1, 1)), B[1][lev], T(lw(s1, 0)) * B[0][lev]);
            }
        // every node ends exactly one edge of each direction: its + end where
        // its sign in that direction is +, else its - end
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int e0 = edge_of(0, a), e1 = edge_of(1, a), e2 = edge_of(2, a);
                const T t0 = kHexS[a][0] > 0 ? E[0][e0][i] : -E[0][e0][i];
                const T t1 = kHexS[a][1] > 0 ? t0 + E[1][e1][i] : t0 - E[1][e1][i];
                out[a][i] = kHexS[a][2] > 0 ? t1 + E[2][e2][i] : t1 - E[2][e2][i];
            }
    }
    template <class T> __device__ static __forceinline__ T dN(int q, int a, int J)
    {
        const T g = T(kG);
        const T p0 = (q & 1) ? g : -g, p1 = (q & 2) ? g : -g, p2 = (q & 4) ? g : -g;
        const T f0 = T(1) + T(kHexS[a][0]) * p0;
        const T f1 = T(1) + T(kHexS[a][1]) * p1;
        const T f2 = T(1) + T(kHexS[a][2]) * p2;
        const T s = T(0.125) * T(kHexS[a][J]);
        return J == 0 ? s * f1 * f2 : (J == 1 ? s * f0 * f2 : s * f0 * f1);
    }
};

// ------------------------------------------------------ quadrature-point math

// Tangent action at one point: Q = w det Jx dP Jx^-T.  Returns false if det Jd <= 0.
// The two tetrahedra of a face pair share what depends only on the face: the
// adjugates' last rows (cross products of the first two Jacobian columns,
// which the second tetrahedron has swapped), S22 = |last row of Ae|^2, and
// W20, W21 (the last row of Ad against the face's two edges of v).
// ROW2 = 1: those go out to r2x = {Ae row 2, S22}, r2d = {Ad row 2, W20,
// W21}; ROW2 = 2: they are taken from there, signs and columns swapped.
// FOLD: the scalars a, b, c enter the matrix products (S scaled by a, W
// replaced by c W + b I; 12 fewer operations, but each entry of Q becomes
// one six-term chain).  The Hex8 kernels, at 1 or 2 waves per SIMD, keep
// the separate terms: there the longer chains cost more than they save.
template <class T, int ROW2 = 0, bool FOLD = true>
__device__ __forceinline__ bool qp_hvp(T w, const T Jx[9], const T Jd[9], const T dJ[9], T mu,
                                       T lam, T Q[9], T *r2x = nullptr, T *r2d = nullptr)
{
    T Ae[9], Ad[9];
    T De, Dd;
    if constexpr (ROW2 == 2) {
        const T nx[3] = {-r2x[0], -r2x[1], -r2x[2]}, nd[3] = {-r2d[0], -r2d[1], -r2d[2]};
        De = adj_det_row2(Jx, nx, Ae);
        Dd = adj_det_row2(Jd, nd, Ad);
    } else {
        De = adj_det(Jx, Ae);
        Dd = adj_det(Jd, Ad);
        if constexpr (ROW2 == 1) {
#pragma unroll
            for (int i = 0; i < 3; ++i) r2x[i] = Ae[6 + i], r2d[i] = Ad[6 + i];
        }
    }
    const T rDe = rcp(De), rDd = rcp(Dd);
    const T a = w * mu * rDe;
    const T s2 = w * De * rDd * rDd;
    const T lnJ = log_(Dd * rDe);
    const T c1 = mu - lam * lnJ;
    // S = Ae Ae^T (symmetric), times a when FOLD
    T S22;
    if constexpr (ROW2 == 2) S22 = r2x[3];
    else S22 = Ae[6] * Ae[6] + Ae[7] * Ae[7] + Ae[8] * Ae[8];
    if constexpr (ROW2 == 1) r2x[3] = S22;
    const T sa = FOLD ? a : T(1);
    const T S00 = sa * (Ae[0] * Ae[0] + Ae[1] * Ae[1] + Ae[2] * Ae[2]);
    const T S01 = sa * (Ae[0] * Ae[3] + Ae[1] * Ae[4] + Ae[2] * Ae[5]);
    const T S02 = sa * (Ae[0] * Ae[6] + Ae[1] * Ae[7] + Ae[2] * Ae[8]);
    const T S11 = sa * (Ae[3] * Ae[3] + Ae[4] * Ae[4] + Ae[5] * Ae[5]);
    const T S12 = sa * (Ae[3] * Ae[6] + Ae[4] * Ae[7] + Ae[5] * Ae[8]);
    S22 = sa * S22;
    const T S[9] = {S00, S01, S02, S01, S11, S12, S02, S12, S22};
    // W = Ad dJ
    T W[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (ROW2 == 2 && i == 2 && j < 2) continue;
            W[i * 3 + j] = Ad[i * 3 + 0] * dJ[0 * 3 + j] + Ad[i * 3 + 1] * dJ[1 * 3 + j]
                         + Ad[i * 3 + 2] * dJ[2 * 3 + j];
        }
    if constexpr (ROW2 == 2) {
        W[6] = -r2d[4];
        W[7] = -r2d[3];
    }
    if constexpr (ROW2 == 1) {
        r2d[3] = W[6];
        r2d[4] = W[7];
    }
    const T tr = W[0] + W[4] + W[8];
    const T b = lam * tr * s2;
    const T c = c1 * s2;
    if constexpr (FOLD) {
        // V = c W + b I: the two Ad^T terms of dP become one product
        T V[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? fma(c, W[k], b) : c * W[k];
        // Q[i][J] = (dJ S)[i][J] + (V Ad)[J][i]
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int J = 0; J < 3; ++J)
                Q[i * 3 + J] = dJ[i * 3 + 0] * S[0 * 3 + J] + dJ[i * 3 + 1] * S[1 * 3 + J]
                             + dJ[i * 3 + 2] * S[2 * 3 + J] + V[J * 3 + 0] * Ad[0 * 3 + i]
                             + V[J * 3 + 1] * Ad[1 * 3 + i] + V[J * 3 + 2] * Ad[2 * 3 + i];
    } else {
        // Q[i][J] = a (dJ S)[i][J] + b Ad[J][i] + c (W Ad)[J][i]
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T d0 = dJ[i * 3 + 0], d1 = dJ[i * 3 + 1], d2 = dJ[i * 3 + 2];
            const T dS[3] = {d0 * S[0] + d1 * S[3] + d2 * S[6], d0 * S[1] + d1 * S[4] + d2 * S[7],
                             d0 * S[2] + d1 * S[5] + d2 * S[8]};
#pragma unroll
            for (int J = 0; J < 3; ++J) {
                const T Mji = W[J * 3 + 0] * Ad[0 * 3 + i] + W[J * 3 + 1] * Ad[1 * 3 + i]
                            + W[J * 3 + 2] * Ad[2 * 3 + i];
                Q[i * 3 + J] = a * dS[J] + b * Ad[J * 3 + i] + c * Mji;
            }
        }
    }
    return Dd > T(0);
}

// Residual at one point: Q = w det Jx P Jx^-T = w [mu/De Jd S + (lam lnJ - mu) De/Dd Ad^T].
template <class T>
__device__ __forceinline__ bool qp_residual(T w, const T Jx[9], const T Jd[9], T mu, T lam, T Q[9])
{
    T Ae[9], Ad[9];
    const T De = adj_det(Jx, Ae);
    const T Dd = adj_det(Jd, Ad);
    T S[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            S[i * 3 + j] = Ae[i * 3 + 0] * Ae[j * 3 + 0] + Ae[i * 3 + 1] * Ae[j * 3 + 1]
                         + Ae[i * 3 + 2] * Ae[j * 3 + 2];
    const T rDe = rcp(De), rDd = rcp(Dd);
    const T lnJ = log_(Dd * rDe);
    const T a = w * mu * rDe;
    const T c = w * (lam * lnJ - mu) * De * rDd;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int J = 0; J < 3; ++J)
            Q[i * 3 + J] = a * (Jd[i * 3 + 0] * S[0 * 3 + J] + Jd[i * 3 + 1] * S[1 * 3 + J]
                                + Jd[i * 3 + 2] * S[2 * 3 + J])
                         + c * Ad[J * 3 + i];
    return Dd > T(0);
}

// ---- small-strain linear elasticity (the second material model)
//   psi = mu eps:eps + lam/2 (tr eps)^2,  sigma = mu (H + H^T) + lam tr(H) I,
// with H = Hxi Jx^-1 = Hxi Ae / De the gradient of a nodal field.

// H of a nodal field; returns det Jx, and Ae (Jx^-1 = Ae / De).
template <class T>
__device__ __forceinline__ T lin_grad(const T Jx[9], const T Hxi[9], T Ae[9], T H[9])
{
    const T De = adj_det(Jx, Ae);
    const T r = rcp(De);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int L = 0; L < 3; ++L)
            H[i * 3 + L] = (Hxi[i * 3 + 0] * Ae[0 * 3 + L] + Hxi[i * 3 + 1] * Ae[1 * 3 + L]
                            + Hxi[i * 3 + 2] * Ae[2 * 3 + L]) * r;
    return De;
}

template <class T>
__device__ __forceinline__ void lin_stress(const T H[9], T mu, T lam, T S[9])
{
    const T t = lam * (H[0] + H[4] + H[8]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int L = 0; L < 3; ++L) S[i * 3 + L] = mu * (H[i * 3 + L] + H[L * 3 + i]) + (i == L ? t : T(0));
}

// eps:eps and tr eps of H
template <class T>
__device__ __forceinline__ void lin_invariants(const T H[9], T &ee, T &tr)
{
    tr = H[0] + H[4] + H[8];
    ee = H[0] * H[0] + H[4] * H[4] + H[8] * H[8];
    const T a = T(0.5) * (H[1] + H[3]), b = T(0.5) * (H[2] + H[6]), c = T(0.5) * (H[5] + H[7]);
    ee += T(2) * (a * a + b * b + c * c);
}

// Nodal forces of the linear model at one point: Q = w det Jx sigma Jx^-T =
// w sigma Ae^T.  Linear in Hxi, so the residual (Hxi of u) and the tangent
// action (Hxi of v) are the same map.
template <class T>
__device__ __forceinline__ void qp_linear(T w, const T Jx[9], const T Hxi[9], T mu, T lam, T Q[9])
{
    T Ae[9], H[9], S[9];
    lin_grad(Jx, Hxi, Ae, H);
    lin_stress(H, mu, lam, S);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int J = 0; J < 3; ++J)
            Q[i * 3 + J] = w * (S[i * 3 + 0] * Ae[J * 3 + 0] + S[i * 3 + 1] * Ae[J * 3 + 1]
                                + S[i * 3 + 2] * Ae[J * 3 + 2]);
}

// Kinematics of the displacement gradient H = Hxi Jx^-1 without cancellation:
// I1 - 3 = 2 tr H + H:H, J - 1 = tr H + ((tr H)^2 - tr H^2)/2 + det H.
struct Kin {
    double H[9], wDe, I1m3, Jm1;
};

__device__ __forceinline__ void kinematics(double w, const double Jx[9], const double Hxi[9], Kin &k)
{
    double Ae[9];
    const double De = adj_det(Jx, Ae);
    const double rDe = 1.0 / De;
    k.wDe = w * De;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int L = 0; L < 3; ++L)
            k.H[i * 3 + L] = (Hxi[i * 3 + 0] * Ae[0 * 3 + L] + Hxi[i * 3 + 1] * Ae[1 * 3 + L]
                              + Hxi[i * 3 + 2] * Ae[2 * 3 + L]) * rDe;
    const double *H = k.H;
    const double trH = H[0] + H[4] + H[8];
    double HH = 0, trH2 = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            HH += H[i * 3 + j] * H[i * 3 + j];
            trH2 += H[i * 3 + j] * H[j * 3 + i];
        }
    double tmp[9];
    const double detH = adj_det(H, tmp);
    k.I1m3 = 2.0 * trH + HH;
    k.Jm1 = trH + 0.5 * (trH * trH - trH2) + detH;
}

// ------------------------------------------------------------- LDS staging

// Node record of the FP64 tangent action: X, x = X + u, v (80 B, 16-B aligned).
struct alignas(16) NodeH64 {
    double X[3], x[3], v[3], pad;
};
// FP32 tangent action: X, u, v.
struct alignas(16) NodeH32 {
    float X[3], u[3], v[3], pad[3];
};
// X and u (energy, residual, diagonal, adjoints).
struct alignas(16) NodeXU {
    double X[3], u[3];
};
// X, u and a second nodal field w (residual VJP).
struct alignas(16) NodeXUW {
    double X[3], u[3], w[3], pad;
};

template <class T>
__device__ __forceinline__ void load3(const T *__restrict__ p, int64_t g, T out[3])
{
    out[0] = p[3 * g + 0];
    out[1] = p[3 * g + 1];
    out[2] = p[3 * g + 2];
}

__device__ __forceinline__ bool comp_fixed(const uint8_t *nmask, int64_t g, int c)
{
    return nmask && ((nmask[g] >> c) & 1);
}

// Write the block's nodal sums acc[l*3+c] out; prescribed components get
// `fixed_val`.  Under the halo scatter a node shared with other blocks is not
// written here: its sum goes to its halo slot (hslot[l]), and k_halo_gather
// adds each node's slots up afterwards.
template <bool ACC, class T>
__device__ __forceinline__ void write_out(const BlockMesh &m, const uint32_t *bnode, int nn,
                                          const double *acc, T *__restrict__ y, Scatter mode,
                                          bool use_mask, T fixed_val, T *__restrict__ halo,
                                          const int32_t *__restrict__ hslot)
{
    for (int l = threadIdx.x; l < nn; l += blockDim.x) {
        const uint32_t ent = bnode[l];
        const int64_t g = ent & kGidMask;
        if ((ent & kShared) && mode == Scatter::Halo) {
            T *h = halo + 3 * (int64_t)hslot[l];
            h[0] = T(acc[l * 3 + 0]);
            h[1] = T(acc[l * 3 + 1]);
            h[2] = T(acc[l * 3 + 2]);
            continue;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const bool fixed = use_mask && comp_fixed(m.nmask, g, c);
            T val = T(acc[l * 3 + c]);
            T *dst = &y[3 * g + c];
            if (ACC) {
                // y += K v: plain read-modify-write where no other block writes
                if (fixed) *dst = fixed_val;
                else if (!(ent & kShared) || mode == Scatter::Color) *dst += val;
                else unsafeAtomicAdd(dst, val);
            } else if (!(ent & kShared)) {
                *dst = fixed ? fixed_val : val;
            } else if (mode == Scatter::Atomic) {
                if (!fixed) unsafeAtomicAdd(dst, val);
                // prescribed entries were set by the pre-pass
            } else {
                if (ent & kFirst) *dst = fixed ? fixed_val : val;
                else if (!fixed) *dst += val;
            }
        }
    }
}

// --------------------------------------------------------------- operations

// Every op provides: Node (LDS record), stage(), element<Elem>(), and whether
// it accumulates nodal vectors.

template <class T> struct HvpOp;

template <> struct HvpOp<double> {
    using Node = NodeH64;
    const double *xrec;   // [n_nodes][6]: X, x = X + u
    const double *v;
    double *y;
    __device__ void stage(const BlockMesh &m, Node &n, int64_t g) const
    {
        const double *p = xrec + 6 * g;
        n.X[0] = p[0], n.X[1] = p[1], n.X[2] = p[2];
        n.x[0] = p[3], n.x[1] = p[4], n.x[2] = p[5];
        load3(v, g, n.v);
        if (m.nmask) {
            const uint8_t b = m.nmask[g];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if ((b >> c) & 1) n.v[c] = 0.0;
        }
    }
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const double *mu,
                                            const double *lam, bool pair, double f[E::NEN][3]) const
    {
        double Xe[E::NEN][3], xe[E::NEN][3], ve[E::NEN][3];
#pragma unroll
        for (int a = 0; a < E::NEN; ++a) {
            const Node &n = sn[lc[a]];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                Xe[a][i] = n.X[i];
                xe[a][i] = n.x[i];
                ve[a][i] = n.v[i];
            }
        }
        return compute<E>(Xe, xe, ve, mu, lam, pair, f);
    }
    // the element's forces from its nodal X, x and v
    template <class E>
    __device__ static __forceinline__ bool compute(const double Xe[E::NEN][3], const double xe[E::NEN][3],
                                                   const double ve[E::NEN][3], const double *mu,
                                                   const double *lam, bool pair, double f[E::NEN][3])
    {
        if constexpr (std::is_same<E, Hex8>::value) {
            // Hex8 in the column form (gradients from edge differences,
            // forces back through the columns): half the operations of the
            // node form; at one wave per SIMD the accumulation registers
            // hold it
            typename E::template Field<double> FX, Fx, Fv;
            E::prep(Xe, FX);
            E::prep(xe, Fx);
            E::prep(ve, Fv);
            typename E::template Acc<double> A;
            bool ok = true;
#pragma unroll
            for (int q = 0; q < E::NQ; ++q) {
                double Jx[9], Jd[9], dJ[9], Q[9];
                E::grad(FX, q, Jx);
                E::grad(Fx, q, Jd);
                E::grad(Fv, q, dJ);
                ok &= qp_hvp<double, 0, false>(E::template weight<double>(), Jx, Jd, dJ, mu[0], lam[0], Q);
                E::template add_forces<true>(Q, q, A);
            }
            E::finish(A, f);
            return ok;
        }
        // three fields: the register-lean form (node sums for Hex8)
        using G = typename E::Lean;
        typename G::template Field<double> FX, Fx, Fv;
        G::prep(Xe, FX);
        G::prep(xe, Fx);
        G::prep(ve, Fv);
        bool ok = true;
        if constexpr (std::is_same<E, Tet4Pair>::value) {
            // a face pair: the second tetrahedron reuses the shared face's
            // cross products from the first
            double Jx[9], Jd[9], dJ[9], Q[9], r2x[4], r2d[5];
            G::grad(FX, 0, Jx);
            G::grad(Fx, 0, Jd);
            G::grad(Fv, 0, dJ);
            ok &= qp_hvp<double, 1>(E::template weight<double>(), Jx, Jd, dJ, mu[0], lam[0], Q, r2x, r2d);
            E::add_forces_open(Q, 0, f);
            if (pair) {
                G::grad(FX, 1, Jx);
                G::grad(Fx, 1, Jd);
                G::grad(Fv, 1, dJ);
                ok &= qp_hvp<double, 2>(E::template weight<double>(), Jx, Jd, dJ, mu[1], lam[1], Q, r2x, r2d);
                E::add_forces_open(Q, 1, f);
            }
            E::close0(f);
            return ok;
        }
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            double Jx[9], Jd[9], dJ[9], Q[9];
            G::grad(FX, q, Jx);
            G::geom(Jx);
            G::grad(Fx, q, Jd);
            G::geom(Jd);
            G::grad(Fv, q, dJ);
            ok &= qp_hvp(E::template weight<double>(), Jx, Jd, dJ, mu[E::sub(q)], lam[E::sub(q)], Q);
            G::template add_forces_to<true>(Q, q, f);
        }
        return ok;
    }
};

template <> struct HvpOp<float> {
    using Node = NodeH32;
    const float *Xf, *ulin, *v;
    float *y;
    __device__ void stage(const BlockMesh &m, Node &n, int64_t g) const
    {
        load3(Xf, g, n.X);
        load3(ulin, g, n.u);
        load3(v, g, n.v);
        if (m.nmask) {
            const uint8_t b = m.nmask[g];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if ((b >> c) & 1) n.v[c] = 0.0f;
        }
    }
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const float *mu,
                                            const float *lam, bool pair, float f[E::NEN][3]) const
    {
        float Xe[E::NEN][3], ue[E::NEN][3], ve[E::NEN][3];
#pragma unroll
        for (int a = 0; a < E::NEN; ++a) {
            const Node &n = sn[lc[a]];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                Xe[a][i] = n.X[i];
                ue[a][i] = n.u[i];
                ve[a][i] = n.v[i];
            }
        }
        typename E::template Field<float> FX, Fu, Fv;
        E::prep(Xe, FX);
        E::prep(ue, Fu);
        E::prep(ve, Fv);
        typename E::template Acc<float> A;
        bool ok = true;
        // face pairs: the second tetrahedron reuses the face's shared terms
        float r2x[4], r2d[5];
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            float Jx[9], Jd[9], dJ[9], Q[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fu, q, Jd);
#pragma unroll
            for (int k = 0; k < 9; ++k) Jd[k] += Jx[k];
            E::grad(Fv, q, dJ);
            if constexpr (std::is_same<E, Tet4Pair>::value) {
                if (q == 0)
                    ok &= qp_hvp<float, 1>(E::template weight<float>(), Jx, Jd, dJ, mu[0], lam[0], Q, r2x, r2d);
                else
                    ok &= qp_hvp<float, 2>(E::template weight<float>(), Jx, Jd, dJ, mu[1], lam[1], Q, r2x, r2d);
            } else {
                ok &= qp_hvp<float, 0, !std::is_same<E, Hex8>::value>(E::template weight<float>(), Jx, Jd, dJ,
                                                                      mu[E::sub(q)], lam[E::sub(q)], Q);
            }
            if constexpr (std::is_same<E, Tet4Pair>::value) E::add_forces_open(Q, q, A.f);
            else E::template add_forces<true>(Q, q, A);
        }
        if constexpr (std::is_same<E, Tet4Pair>::value) E::close0(A.f);
        E::finish(A, f);
        return ok;
    }
};

// X and u of an item's nodes from LDS, in the item type's gradient form
template <class E>
__device__ __forceinline__ void gather_xu(const NodeXU *sn, const uint16_t *lc,
                                          typename E::template Field<double> &FX,
                                          typename E::template Field<double> &Fu)
{
    double Xe[E::NEN][3], ue[E::NEN][3];
#pragma unroll
    for (int a = 0; a < E::NEN; ++a) {
        const NodeXU &n = sn[lc[a]];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Xe[a][i] = n.X[i];
            ue[a][i] = n.u[i];
        }
    }
    E::prep(Xe, FX);
    E::prep(ue, Fu);
}

struct XUStage {
    const double *X, *u;
    __device__ void stage(const BlockMesh &, NodeXU &n, int64_t g) const
    {
        load3(X, g, n.X);
        load3(u, g, n.u);
    }
};
// stages X, u and w (residual VJP)
struct XUWStage {
    const double *X, *u, *w;
    __device__ __forceinline__ void stage(const BlockMesh &, NodeXUW &n, int64_t g) const
    {
        load3(X, g, n.X);
        load3(u, g, n.u);
        load3(w, g, n.w);
    }
};

struct ResidualOp : XUStage {
    using Node = NodeXU;
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const double *mu,
                                            const double *lam, bool pair, double f[E::NEN][3]) const
    {
        typename E::template Field<double> FX, Fu;
        gather_xu<E>(sn, lc, FX, Fu);
        typename E::template Acc<double> A;
        bool ok = true;
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            double Jx[9], Jd[9], Q[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fu, q, Jd);
#pragma unroll
            for (int k = 0; k < 9; ++k) Jd[k] += Jx[k];
            ok &= qp_residual(E::template weight<double>(), Jx, Jd, mu[E::sub(q)], lam[E::sub(q)], Q);
            E::template add_forces<true>(Q, q, A);
        }
        E::finish(A, f);
        return ok;
    }
};

// diag K: w [ mu/De n^T S n + (lam + c1) De/Dd^2 ((Ad^T n)_i)^2 ], n = dN_a/dxi
struct DiagOp : XUStage {
    using Node = NodeXU;
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const double *mu,
                                            const double *lam, bool pair, double f[E::NEN][3]) const
    {
        typename E::template Field<double> FX, Fu;
        gather_xu<E>(sn, lc, FX, Fu);
#pragma unroll
        for (int a = 0; a < E::NEN; ++a) f[a][0] = f[a][1] = f[a][2] = 0.0;
        bool ok = true;
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            const double mq = mu[E::sub(q)], lq = lam[E::sub(q)];
            double Jx[9], Jd[9], Ae[9], Ad[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fu, q, Jd);
#pragma unroll
            for (int k = 0; k < 9; ++k) Jd[k] += Jx[k];
            const double De = adj_det(Jx, Ae);
            const double Dd = adj_det(Jd, Ad);
            ok &= Dd > 0.0;
            const double w = E::template weight<double>();
            const double lnJ = log_(Dd / De);
            const double a = w * mq / De;
            const double b = w * (lq + mq - lq * lnJ) * De / (Dd * Dd);
#pragma unroll
            for (int n = 0; n < E::NEN; ++n) {
                const double g0 = E::template dN<double>(q, n, 0);
                const double g1 = E::template dN<double>(q, n, 1);
                const double g2 = E::template dN<double>(q, n, 2);
                // Ae^T n, |.|^2 = n^T S n
                const double t0 = Ae[0] * g0 + Ae[3] * g1 + Ae[6] * g2;
                const double t1 = Ae[1] * g0 + Ae[4] * g1 + Ae[7] * g2;
                const double t2 = Ae[2] * g0 + Ae[5] * g1 + Ae[8] * g2;
                const double nSn = t0 * t0 + t1 * t1 + t2 * t2;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double k = Ad[0 * 3 + i] * g0 + Ad[1 * 3 + i] * g1 + Ad[2 * 3 + i] * g2;
                    f[n][i] += a * nSn + b * k * k;
                }
            }
        }
        return ok;
    }
};

// Off-diagonal entries of the 3x3 diagonal blocks of K(u): node n's block
// is the sum over its elements' points of a (n.S n) I + b k k^T with k =
// Ad^T grad_xi N_n (DiagOp keeps the diagonal of it), so its off-diagonal
// entries are b k_i k_j; out [n][3] = (K01, K02, K12).  The linear model's
// block is (w / De) (mu (t.t) I + (mu + lam) t t^T), t = Ae^T grad_xi N_n.
template <bool LIN>
struct OffDiagOp : XUStage {
    using Node = NodeXU;
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const double *mu,
                                            const double *lam, bool pair, double f[E::NEN][3]) const
    {
        typename E::template Field<double> FX, Fu;
        gather_xu<E>(sn, lc, FX, Fu);
#pragma unroll
        for (int a = 0; a < E::NEN; ++a) f[a][0] = f[a][1] = f[a][2] = 0.0;
        bool ok = true;
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            const double mq = mu[E::sub(q)], lq = lam[E::sub(q)];
            double Jx[9], A[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            double b;
            if (LIN) {
                const double De = adj_det(Jx, A);
                b = E::template weight<double>() * (mq + lq) / De;
            } else {
                double Jd[9], Ae[9];
                E::grad(Fu, q, Jd);
#pragma unroll
                for (int k = 0; k < 9; ++k) Jd[k] += Jx[k];
                const double De = adj_det(Jx, Ae);
                const double Dd = adj_det(Jd, A);
                ok &= Dd > 0.0;
                const double lnJ = log_(Dd / De);
                b = E::template weight<double>() * (lq + mq - lq * lnJ) * De / (Dd * Dd);
            }
#pragma unroll
            for (int n = 0; n < E::NEN; ++n) {
                const double g0 = E::template dN<double>(q, n, 0);
                const double g1 = E::template dN<double>(q, n, 1);
                const double g2 = E::template dN<double>(q, n, 2);
                double k[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) k[i] = A[0 * 3 + i] * g0 + A[1 * 3 + i] * g1 + A[2 * 3 + i] * g2;
                f[n][0] += b * k[0] * k[1];
                f[n][1] += b * k[0] * k[2];
                f[n][2] += b * k[1] * k[2];
            }
        }
        return ok;
    }
};

// dPsi/dX at fixed nodal u: Q = w det Jx (psi I - H^T P) Jx^-T
struct GradCoordsOp : XUStage {
    using Node = NodeXU;
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const double *mu,
                                            const double *lam, bool pair, double f[E::NEN][3]) const
    {
        typename E::template Field<double> FX, Fu;
        gather_xu<E>(sn, lc, FX, Fu);
        typename E::template Acc<double> A;
        E::zero(A);   // a point may be skipped (inverted), so no point initialises
        bool ok = true;
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            const double mu_ = mu[E::sub(q)], lam_ = lam[E::sub(q)];
            double Jx[9], Hxi[9], Ae[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fu, q, Hxi);
            Kin k;
            kinematics(E::template weight<double>(), Jx, Hxi, k);
            if (!(1.0 + k.Jm1 > 0.0)) {
                ok = false;
                continue;
            }
            const double lnJ = log1p_(k.Jm1);
            const double psi = 0.5 * mu_ * k.I1m3 - mu_ * lnJ + 0.5 * lam_ * lnJ * lnJ;
            double F[9], Fa[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) F[i] = k.H[i] + ((i % 4) == 0 ? 1.0 : 0.0);
            const double detF = adj_det(F, Fa);   // F^-1 = Fa / detF
            const double rdF = 1.0 / detF;
            double P[9], Sg[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int J = 0; J < 3; ++J) {
                    const double FiT = Fa[J * 3 + i] * rdF;   // F^-T_iJ
                    P[i * 3 + J] = mu_ * (F[i * 3 + J] - FiT) + lam_ * lnJ * FiT;
                }
#pragma unroll
            for (int mm = 0; mm < 3; ++mm)
#pragma unroll
                for (int L = 0; L < 3; ++L)
                    Sg[mm * 3 + L] = (mm == L ? psi : 0.0) - (k.H[0 * 3 + mm] * P[0 * 3 + L]
                                     + k.H[1 * 3 + mm] * P[1 * 3 + L] + k.H[2 * 3 + mm] * P[2 * 3 + L]);
            // Q = w det Jx Sg Jx^-T = w Sg Ae^T
            adj_det(Jx, Ae);
            const double w = E::template weight<double>();
            double Q[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int J = 0; J < 3; ++J)
                    Q[i * 3 + J] = w * (Sg[i * 3 + 0] * Ae[J * 3 + 0] + Sg[i * 3 + 1] * Ae[J * 3 + 1]
                                        + Sg[i * 3 + 2] * Ae[J * 3 + 2]);
            E::template add_forces<false>(Q, q, A);
        }
        E::finish(A, f);
        return ok;
    }
};

// ---- operations of the linear model

// X and a direction v: the linear model's tangent does not depend on u.
template <class T> struct alignas(16) NodeXV {
    T X[3], v[3];
};

template <class T> struct LinHvpOp {
    using Node = NodeXV<T>;
    const T *X, *v;
    __device__ void stage(const BlockMesh &m, Node &n, int64_t g) const
    {
        load3(X, g, n.X);
        load3(v, g, n.v);
        if (m.nmask) {
            const uint8_t b = m.nmask[g];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if ((b >> c) & 1) n.v[c] = T(0);
        }
    }
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const T *mu, const T *lam,
                                            bool pair, T f[E::NEN][3]) const
    {
        T Xe[E::NEN][3], ve[E::NEN][3];
#pragma unroll
        for (int a = 0; a < E::NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                Xe[a][i] = sn[lc[a]].X[i];
                ve[a][i] = sn[lc[a]].v[i];
            }
        typename E::template Field<T> FX, Fv;
        E::prep(Xe, FX);
        E::prep(ve, Fv);
        typename E::template Acc<T> A;
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            T Jx[9], dJ[9], Q[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fv, q, dJ);
            qp_linear(E::template weight<T>(), Jx, dJ, mu[E::sub(q)], lam[E::sub(q)], Q);
            E::template add_forces<true>(Q, q, A);
        }
        E::finish(A, f);
        return true;
    }
};

struct LinResidualOp : XUStage {
    using Node = NodeXU;
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const double *mu,
                                            const double *lam, bool pair, double f[E::NEN][3]) const
    {
        typename E::template Field<double> FX, Fu;
        gather_xu<E>(sn, lc, FX, Fu);
        typename E::template Acc<double> A;
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            double Jx[9], Hxi[9], Q[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fu, q, Hxi);
            qp_linear(E::template weight<double>(), Jx, Hxi, mu[E::sub(q)], lam[E::sub(q)], Q);
            E::template add_forces<true>(Q, q, A);
        }
        E::finish(A, f);
        return true;
    }
};

// diag K of the linear model: w det Jx [mu |grad N_a|^2 + (mu + lam) (grad N_a)_i^2]
// = w / De [mu |Ae^T n|^2 + (mu + lam) ((Ae^T n)_i)^2],  n = dN_a/dxi
struct LinDiagOp : XUStage {
    using Node = NodeXU;
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const double *mu,
                                            const double *lam, bool pair, double f[E::NEN][3]) const
    {
        typename E::template Field<double> FX, Fu;
        gather_xu<E>(sn, lc, FX, Fu);
#pragma unroll
        for (int a = 0; a < E::NEN; ++a) f[a][0] = f[a][1] = f[a][2] = 0.0;
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            const double mq = mu[E::sub(q)], lq = lam[E::sub(q)];
            double Jx[9], Ae[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            const double De = adj_det(Jx, Ae);
            const double c = E::template weight<double>() / De;
#pragma unroll
            for (int n = 0; n < E::NEN; ++n) {
                const double g0 = E::template dN<double>(q, n, 0);
                const double g1 = E::template dN<double>(q, n, 1);
                const double g2 = E::template dN<double>(q, n, 2);
                const double t[3] = {Ae[0] * g0 + Ae[3] * g1 + Ae[6] * g2,
                                     Ae[1] * g0 + Ae[4] * g1 + Ae[7] * g2,
                                     Ae[2] * g0 + Ae[5] * g1 + Ae[8] * g2};
                const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
#pragma unroll
                for (int i = 0; i < 3; ++i) f[n][i] += c * (mq * tt + (mq + lq) * t[i] * t[i]);
            }
        }
        return true;
    }
};

// dPsi/dX of the linear model at fixed nodal u: Q = w det Jx (psi I - H^T sigma) Jx^-T
struct LinGradCoordsOp : XUStage {
    using Node = NodeXU;
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const double *mu,
                                            const double *lam, bool pair, double f[E::NEN][3]) const
    {
        typename E::template Field<double> FX, Fu;
        gather_xu<E>(sn, lc, FX, Fu);
        typename E::template Acc<double> A;
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            const double mq = mu[E::sub(q)], lq = lam[E::sub(q)];
            double Jx[9], Hxi[9], Ae[9], H[9], S[9], Sg[9], Q[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fu, q, Hxi);
            lin_grad(Jx, Hxi, Ae, H);
            lin_stress(H, mq, lq, S);
            double ee, tr;
            lin_invariants(H, ee, tr);
            const double psi = mq * ee + 0.5 * lq * tr * tr;
#pragma unroll
            for (int mm = 0; mm < 3; ++mm)
#pragma unroll
                for (int L = 0; L < 3; ++L)
                    Sg[mm * 3 + L] = (mm == L ? psi : 0.0) - (H[0 * 3 + mm] * S[0 * 3 + L]
                                     + H[1 * 3 + mm] * S[1 * 3 + L] + H[2 * 3 + mm] * S[2 * 3 + L]);
            const double w = E::template weight<double>();
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int J = 0; J < 3; ++J)
                    Q[i * 3 + J] = w * (Sg[i * 3 + 0] * Ae[J * 3 + 0] + Sg[i * 3 + 1] * Ae[J * 3 + 1]
                                        + Sg[i * 3 + 2] * Ae[J * 3 + 2]);
            E::template add_forces<true>(Q, q, A);
        }
        E::finish(A, f);
        return true;
    }
};

// ---- non-variational transport (virtual work): three species in the three
// nodal components, per species s and node a
//   r_{a,s} = sum_q w det J [ D grad c_s . grad N_a + (b(x_q) . grad c_s + k c_s) N_a ]
// with b(x) = omega x x, D = mu_e, k = lam_e.  Linear in c: the residual of c
// and the tangent action on v are the same map; the advection term makes the
// tangent non-symmetric.  Gradients and forces in the node form (E::Lean),
// which also interpolates values.

template <class T> struct TransportOp {
    using Node = NodeXV<T>;
    const T *X, *c;
    T om0, om1, om2;
    int mask_input;   // tangent action: prescribed components of v read as 0
    __device__ void stage(const BlockMesh &m, Node &n, int64_t g) const
    {
        load3(X, g, n.X);
        load3(c, g, n.v);
        if (mask_input && m.nmask) {
            const uint8_t b = m.nmask[g];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if ((b >> i) & 1) n.v[i] = T(0);
        }
    }
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const T *mu, const T *lam,
                                            bool pair, T f[E::NEN][3]) const
    {
        using G = typename E::Lean;
        T Xe[E::NEN][3], ce[E::NEN][3];
#pragma unroll
        for (int a = 0; a < E::NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                Xe[a][i] = sn[lc[a]].X[i];
                ce[a][i] = sn[lc[a]].v[i];
                f[a][i] = T(0);
            }
        typename G::template Field<T> FX, Fc;
        G::prep(Xe, FX);
        G::prep(ce, Fc);
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            T Jx[9], Cxi[9], Ae[9], Gc[9], Q[9];
            G::grad(FX, q, Jx);
            G::geom(Jx);
            G::grad(Fc, q, Cxi);
            const T De = lin_grad(Jx, Cxi, Ae, Gc);   // Gc[s][L] = d c_s / d x_L
            T xq[3] = {T(0), T(0), T(0)}, cq[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int a = 0; a < E::NEN; ++a) {
                const T Na = G::template N<T>(q, a);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    xq[i] += Na * Xe[a][i];
                    cq[i] += Na * ce[a][i];
                }
            }
            const T b0 = om1 * xq[2] - om2 * xq[1], b1 = om2 * xq[0] - om0 * xq[2], b2 = om0 * xq[1] - om1 * xq[0];
            const T w = E::template weight<T>(), D = mu[E::sub(q)], k = lam[E::sub(q)];
            // diffusion: w det Jx D grad c Jx^-T = w D Gc Ae^T
#pragma unroll
            for (int sp = 0; sp < 3; ++sp)
#pragma unroll
                for (int J = 0; J < 3; ++J)
                    Q[sp * 3 + J] = w * D * (Gc[sp * 3 + 0] * Ae[J * 3 + 0] + Gc[sp * 3 + 1] * Ae[J * 3 + 1]
                                             + Gc[sp * 3 + 2] * Ae[J * 3 + 2]);
            G::template add_forces_to<false>(Q, q, f);
            const T wDe = w * De;
            T g[3];
#pragma unroll
            for (int sp = 0; sp < 3; ++sp)
                g[sp] = wDe * (b0 * Gc[sp * 3 + 0] + b1 * Gc[sp * 3 + 1] + b2 * Gc[sp * 3 + 2] + k * cq[sp]);
#pragma unroll
            for (int a = 0; a < E::NEN; ++a) {
                const T Na = G::template N<T>(q, a);
#pragma unroll
                for (int sp = 0; sp < 3; ++sp) f[a][sp] += Na * g[sp];
            }
        }
        return true;
    }
};

// diag K of the transport operator (the same for the three species):
// w det J [D |grad N_a|^2 + (b . grad N_a) N_a + k N_a^2], grad N_a = Ae^T n / De
struct TransportDiagOp : XUStage {
    using Node = NodeXU;
    double om0, om1, om2;
    template <class E>
    __device__ __forceinline__ bool element(const Node *sn, const uint16_t *lc, const double *mu,
                                            const double *lam, bool pair, double f[E::NEN][3]) const
    {
        using G = typename E::Lean;
        double Xe[E::NEN][3];
#pragma unroll
        for (int a = 0; a < E::NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                Xe[a][i] = sn[lc[a]].X[i];
                f[a][i] = 0.0;
            }
        typename G::template Field<double> FX;
        G::prep(Xe, FX);
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            double Jx[9], Ae[9];
            G::grad(FX, q, Jx);
            G::geom(Jx);
            const double De = adj_det(Jx, Ae);
            double xq[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int a = 0; a < E::NEN; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i) xq[i] += G::template N<double>(q, a) * Xe[a][i];
            const double b0 = om1 * xq[2] - om2 * xq[1], b1 = om2 * xq[0] - om0 * xq[2],
                         b2 = om0 * xq[1] - om1 * xq[0];
            const double w = E::template weight<double>(), D = mu[E::sub(q)], k = lam[E::sub(q)];
#pragma unroll
            for (int n = 0; n < E::NEN; ++n) {
                const double g0 = G::template dN<double>(q, n, 0);
                const double g1 = G::template dN<double>(q, n, 1);
                const double g2 = G::template dN<double>(q, n, 2);
                const double t0 = Ae[0] * g0 + Ae[3] * g1 + Ae[6] * g2;
                const double t1 = Ae[1] * g0 + Ae[4] * g1 + Ae[7] * g2;
                const double t2 = Ae[2] * g0 + Ae[5] * g1 + Ae[8] * g2;
                const double Nn = G::template N<double>(q, n);
                const double d = w * (D * (t0 * t0 + t1 * t1 + t2 * t2) / De + (b0 * t0 + b1 * t1 + b2 * t2) * Nn
                                      + De * k * Nn * Nn);
                f[n][0] += d;
                f[n][1] += d;
                f[n][2] += d;
            }
        }
        return true;
    }
};

// ------------------------------------------------------------ per-item inputs

// Work items of one block.  Pairs come first; item k covers the internal
// elements e0 + k + min(k, np) (+ s for sub-element s of a pair).
struct ItemRange {
    int i0, ni, e0, np;
    __device__ __forceinline__ int elem(int k, int s) const { return e0 + k + min(k, np) + s; }
};

__device__ __forceinline__ ItemRange item_range(const BlockMesh &m, int b)
{
    ItemRange r;
    r.i0 = m.istart[b];
    r.ni = m.istart[b + 1] - r.i0;
    r.e0 = m.estart[b];
    r.np = (m.estart[b + 1] - r.e0) - r.ni;
    return r;
}

// Packed local connectivity of one item in one vector load, plus its
// materials.  Loaded one item ahead of its use so that the global-load latency
// overlaps the previous item's arithmetic.
template <class E> struct ItemWord;
template <> struct ItemWord<Tet4Pair> { uint2 w; };
template <> struct ItemWord<Hex8> { uint4 w; };
template <> struct ItemWord<Tri3> { uint32_t w; };

template <class E> struct IData {
    ItemWord<E> lc;
    double mu[E::NSUB], lam[E::NSUB];
};

template <class E>
__device__ __forceinline__ IData<E> fetch_item(const BlockMesh &m, const ItemRange &r, int k)
{
    IData<E> d;
    const int64_t i = r.i0 + k;
    if constexpr (E::NEN == 5) d.lc.w = *reinterpret_cast<const uint2 *>(m.items + 2 * i);
    else if constexpr (E::NEN == 3) d.lc.w = m.items[i];
    else d.lc.w = *reinterpret_cast<const uint4 *>(m.items + 4 * i);
#pragma unroll
    for (int s = 0; s < E::NSUB; ++s) {
        if (m.mu) {
            // an unpaired tetrahedron has no second element: repeat the first
            const int e = r.elem(k, (s > 0 && k >= r.np) ? 0 : s);
            d.mu[s] = m.mu[e];
            d.lam[s] = m.lam[e];
        } else {
            d.mu[s] = m.mu0;
            d.lam[s] = m.lam0;
        }
    }
    return d;
}

// the packed local connectivity of item k alone (one vector load)
template <class E>
__device__ __forceinline__ ItemWord<E> fetch_lc(const BlockMesh &m, const ItemRange &r, int k)
{
    ItemWord<E> w;
    const int64_t i = r.i0 + k;
    if constexpr (E::NEN == 5) w.w = *reinterpret_cast<const uint2 *>(m.items + 2 * i);
    else if constexpr (E::NEN == 3) w.w = m.items[i];
    else w.w = *reinterpret_cast<const uint4 *>(m.items + 4 * i);
    return w;
}

// materials of item k: the two kernel-argument scalars when uniform, else
// per element (an unpaired tetrahedron repeats its first element)
template <class E, class T>
__device__ __forceinline__ void item_materials(const BlockMesh &m, const ItemRange &r, int k, T mu[E::NSUB],
                                               T lam[E::NSUB])
{
#pragma unroll
    for (int s = 0; s < E::NSUB; ++s) {
        if (m.mu) {
            const int e = r.elem(k, (s > 0 && k >= r.np) ? 0 : s);
            mu[s] = T(m.mu[e]);
            lam[s] = T(m.lam[e]);
        } else {
            mu[s] = T(m.mu0);
            lam[s] = T(m.lam0);
        }
    }
}

template <class E>
__device__ __forceinline__ void unpack_lc(const ItemWord<E> &l, uint16_t lc[E::NEN])
{
    if constexpr (E::NEN == 5) {
        lc[0] = l.w.x & 1023u, lc[1] = (l.w.x >> 10) & 1023u, lc[2] = (l.w.x >> 20) & 1023u;
        lc[3] = l.w.y & 1023u, lc[4] = (l.w.y >> 10) & 1023u;
    } else if constexpr (E::NEN == 3) {
        lc[0] = l.w & 1023u, lc[1] = (l.w >> 10) & 1023u, lc[2] = (l.w >> 20) & 1023u;
    } else {
        lc[0] = l.w.x & 0xffff, lc[1] = l.w.x >> 16, lc[2] = l.w.y & 0xffff, lc[3] = l.w.y >> 16;
        lc[4] = l.w.z & 0xffff, lc[5] = l.w.z >> 16, lc[6] = l.w.w & 0xffff, lc[7] = l.w.w >> 16;
    }
}

template <class E, class T>
__device__ __forceinline__ void materials(const IData<E> &d, T mu[E::NSUB], T lam[E::NSUB])
{
#pragma unroll
    for (int s = 0; s < E::NSUB; ++s) {
        mu[s] = T(d.mu[s]);
        lam[s] = T(d.lam[s]);
    }
}

// Stage a block's node records into LDS.  A thread issues all its global
// loads (block-node words, then node data) before its LDS stores, so the phase
// costs two memory latencies however many nodes the thread stages; extra(l,
// word) runs beside each record's store.
template <class Node, class St, class Extra>
__device__ __forceinline__ void stage_nodes(const BlockMesh &m, const St &st, Node *sn,
                                            const uint32_t *bnode, int nn, Extra extra)
{
    constexpr int kU = 3;
    const int nt = blockDim.x;
    for (int l0 = threadIdx.x; l0 < nn; l0 += kU * nt) {
        uint32_t ent[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) ent[u] = l0 + u * nt < nn ? bnode[l0 + u * nt] : 0u;
        Node tmp[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (l0 + u * nt < nn) st.stage(m, tmp[u], ent[u] & kGidMask);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int l = l0 + u * nt;
            if (l < nn) {
                sn[l] = tmp[u];
                extra(l, ent[u]);
            }
        }
    }
}

// ---------------------------------------------------------- block pass kernel

// Waves per SIMD the register allocator must leave room for.  The FP64 Tet4
// pair pass needs 170 VGPRs unconstrained (2 waves per SIMD); held to 168 for
// 3 waves it spills one register and runs about 3% faster.  The other item
// kernels keep the compiler's choice.
#ifndef EFEM_TET64_MIN_WAVES
#define EFEM_TET64_MIN_WAVES 3
#endif
template <class E, class Op> struct MinWaves {
    static constexpr int value = 1;
};
template <> struct MinWaves<Tet4Pair, HvpOp<double>> {
    static constexpr int value = EFEM_TET64_MIN_WAVES;
};


template <class E, class Op, class T, bool ACC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MinWaves<E, Op>::value, 8)))
k_accumulate(BlockMesh m, Op op, T *__restrict__ y,
                                                    const int32_t *__restrict__ list, int count,
                                                    Scatter mode, int use_mask, T fixed_val,
                                                    const int32_t *__restrict__ skip)
{
    using Node = typename Op::Node;
    extern __shared__ __align__(16) unsigned char smem[];
    if (skip && *skip) return;
    const int lb = xcd_remap(blockIdx.x, count);
    const int b = list ? list[lb] : lb;
    const int n0 = m.nstart[b], nn = m.nstart[b + 1] - n0;
    const ItemRange r = item_range(m, b);
    Node *sn = reinterpret_cast<Node *>(smem);
    // nodal sums are accumulated in FP64 in LDS for both precisions
    double *acc = reinterpret_cast<double *>(smem + sizeof(Node) * nn);
    const uint32_t *bnode = m.bnode + n0;
    const int nt = blockDim.x;
    // The 64 lanes of a wave take items S apart in the block's Morton order
    // (lane * S + j), so that the lanes of one LDS atomic rarely hit the same
    // node; wave w takes columns j = w, w + W, ...
    const int W = nt >> 6, lane = threadIdx.x & 63;
    const int S = (r.ni + 63) >> 6;
    int j = threadIdx.x >> 6;
    auto item_of = [&](int jj) { return lane * S + jj; };
    // the next item's connectivity is in flight while this one computes; its
    // materials are read at use (two scalars when uniform), which keeps four
    // doubles per item out of the registers
    ItemWord<E> nxt{};
    if (j < S && item_of(j) < r.ni) nxt = fetch_lc<E>(m, r, item_of(j));   // in flight during staging
    // the block-node words stay in LDS for write_out
    uint32_t *sbn = reinterpret_cast<uint32_t *>(acc + 3 * nn);
    stage_nodes(m, op, sn, bnode, nn, [&](int l, uint32_t ent) {
        sbn[l] = ent;
        acc[3 * l + 0] = 0.0;
        acc[3 * l + 1] = 0.0;
        acc[3 * l + 2] = 0.0;
    });
    __syncthreads();
    bool bad = false;
    for (; j < S; j += W) {
        const int k = item_of(j);
        if (k >= r.ni) break;
        const ItemWord<E> cur = nxt;
        if (j + W < S && item_of(j + W) < r.ni) nxt = fetch_lc<E>(m, r, item_of(j + W));
        uint16_t lc[E::NEN];
        unpack_lc<E>(cur, lc);
        T mu[E::NSUB], lam[E::NSUB];
        item_materials<E>(m, r, k, mu, lam);
        T f[E::NEN][3];   // written in full by element()
        bad |= !op.template element<E>(sn, lc, mu, lam, k < r.np, f);
#pragma unroll
        for (int a = 0; a < E::NEN; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) atomicAdd(&acc[3 * lc[a] + i], (double)f[a][i]);
    }
    if (bad) flag_inverted(m.flags);
    __syncthreads();
    write_out<ACC>(m, sbn, nn, acc, y, mode, use_mask != 0, fixed_val,
                   reinterpret_cast<T *>(m.halo), m.hslot ? m.hslot + n0 : nullptr);
}

// Second half of the halo scatter: shared node i = node[i] sums its halo
// slots (its blocks or chunks in order; in FP64, so the result does not depend
// on the schedule), then y = sum (ACC: y += sum); prescribed components get
// fixed_val.  The slots of a node in segment c of the layout follow from the
// thread's index, so the slot loads, the node id and the node's Dirichlet bits
// are all one memory latency away (nodes past the segments read their range
// first).  MASK: a Dirichlet mask is in force (a template flag, so that the
// mask's load is not behind a branch whose merge would wait for it).
// s += the N slots at p, in order (all loads before the first add)
template <int N, class T>
__device__ __forceinline__ void halo_sum(const T *__restrict__ p, double s[3])
{
    T h[N][3];
#pragma unroll
    for (int k = 0; k < N; ++k) h[k][0] = p[3 * k], h[k][1] = p[3 * k + 1], h[k][2] = p[3 * k + 2];
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += (double)h[k][c];
}

// Shared node i of the halo layout: its slots summed in order, written to y.
template <class T, bool ACC, bool MASK>
__device__ __forceinline__ void gather_node(const HaloSegs &seg, const int32_t *__restrict__ gptr,
                                            const int32_t *__restrict__ node, const T *__restrict__ halo,
                                            T *__restrict__ y, const uint8_t *__restrict__ nmask, T fixed_val,
                                            int i)
{
    int64_t k0, cnt;
    if (i < seg.start[kSegMax + 1]) {
        // the segment by selects over constant indices (a dynamic index would
        // put the kernel-argument arrays behind a memory load)
        int c = 2, st = seg.start[2], bs = seg.base[2];
#pragma unroll
        for (int cc = 3; cc <= kSegMax; ++cc) {
            int sc = seg.start[cc], bc = seg.base[cc];
            asm volatile("" : "+s"(sc), "+s"(bc));   // values in scalar registers, not re-read by index
            const bool in = i >= sc;
            c = in ? cc : c;
            st = in ? sc : st;
            bs = in ? bc : bs;
        }
        cnt = c;
        k0 = bs + (int64_t)c * (i - st);
    } else {
        const int j = i - seg.start[kSegMax + 1];
        k0 = gptr[j];
        cnt = gptr[j + 1] - k0;
    }
    const int64_t g = node[i];
    const uint8_t b = MASK ? nmask[g] : 0;
    // exactly cnt slot loads, issued back to back (cnt is the same for the
    // lanes of a wave but at segment boundaries)
    double s[3] = {0.0, 0.0, 0.0};
    switch (cnt) {
        case 2: halo_sum<2>(halo + 3 * k0, s); break;
        case 3: halo_sum<3>(halo + 3 * k0, s); break;
        case 4: halo_sum<4>(halo + 3 * k0, s); break;
        case 5: halo_sum<5>(halo + 3 * k0, s); break;
        case 6: halo_sum<6>(halo + 3 * k0, s); break;
        case 7: halo_sum<7>(halo + 3 * k0, s); break;
        case 8: halo_sum<8>(halo + 3 * k0, s); break;
        default:
            for (int64_t k = 0; k < cnt; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) s[c] += (double)halo[3 * (k0 + k) + c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T *dst = &y[3 * g + c];
        if ((b >> c) & 1) *dst = fixed_val;
        else *dst = ACC ? *dst + T(s[c]) : T(s[c]);
    }
}

template <class T, bool ACC, bool MASK>
__global__ void __launch_bounds__(256) k_halo_gather(HaloSegs seg, const int32_t *__restrict__ gptr,
                                                     const int32_t *__restrict__ node,
                                                     const T *__restrict__ halo, T *__restrict__ y,
                                                     const uint8_t *__restrict__ nmask, T fixed_val,
                                                     const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < seg.n) gather_node<T, ACC, MASK>(seg, gptr, node, halo, y, nmask, fixed_val, i);
}

// y = 0, prescribed components = fixed_val, before an atomic pass adds into
// the nodes that several blocks share (the block-private ones it overwrites).
// A contiguous fill of the whole vector: cheaper than an indexed one over the
// shared nodes alone.
template <class T>
__global__ void __launch_bounds__(256) k_fill_nodal(int64_t n_nodes, T *__restrict__ y,
                                                    const uint8_t *__restrict__ nmask, T fixed_val)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;   // node
    if (i >= n_nodes) return;
    const uint8_t b = nmask ? nmask[i] : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) y[3 * i + c] = ((b >> c) & 1) ? fixed_val : T(0);
}

// ----------------------------------------------------------- chunk pass

// The FP64 Tet4 tangent action over chunks (one workgroup per chunk, the
// whole LDS of a CU).  Every node record of a chunk stays resident while its
// blocks stream through as steps: while the items of step t compute, the
// records that step t+1 brings are already on their way from HBM with
// global-to-LDS loads, which take no registers, so the 3 waves per SIMD of the
// item arithmetic keep their occupancy.  One barrier per step makes the
// records of step t+1 visible.  The chunk's nodal sums stay in LDS until the
// last step; shared nodes then go to their halo entries as in the block pass.
//
// LDS: five 16-byte record pieces per node slot, each piece in an array of its
// own, so that one wave's 64-lane load fills 64 consecutive slots:
//   P0 = (X0, X1), P1 = (X2, x0), P2 = (x1, x2)  from the 48-byte record (X, x)
//   P3 = (v0, v1), P4 = (v1, v2)                 two overlapping reads of v
// then the FP64 sums, 3 per slot (kChunkLds bytes in all).
// Global-to-LDS loads, written as instructions: lane i's 16 (or 4) bytes land
// at LDS byte address lds + 16 i (4 i); lds must be the same in every lane.
// The compiler does not see these loads, so it neither waits for them before
// unrelated LDS reads (it would otherwise assume they may alias) nor counts
// them; every use of their data follows an explicit wait_vm_loads() and a
// barrier.  They write no registers.  m0 is set inside the statement (one
// wait state before the load uses it).
__device__ __forceinline__ uint32_t lds_addr(const void *p) { return (uint32_t)(uintptr_t)p; }
__device__ __forceinline__ void load_to_lds16(const void *src, uint32_t lds)
{
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(lds) : "m0");
}
__device__ __forceinline__ void load_to_lds4(const void *src, uint32_t lds)
{
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off" ::"v"(src), "s"(lds) : "m0");
}

// The slot a lane stages for a block's new-slot range lo | hi << 16: wave w
// takes slot group (lo >> 6) + w (the host keeps a block's new slots within
// one group per wave); -1 if the lane has none.
__device__ __forceinline__ int chunk_stage_slot(uint32_t lohi, int wave, int lane)
{
    const int lo = (int)(lohi & 0xffffu), hi = (int)(lohi >> 16);
    const int l = ((lo >> 6) + wave) * 64 + lane;
    return (l >= lo && l < hi) ? l : -1;
}

// Record-piece loads of slot l from its staging word (node id and Dirichlet
// bits); the wave's 64 slots form one group of the piece arrays.
__device__ __forceinline__ void chunk_stage_records(unsigned char *smem, const double *__restrict__ xrec,
                                                    const double *__restrict__ v, int l, uint32_t word)
{
    if (l < 0) return;
    const int64_t g = word & kStageGid;
    const double *pr = xrec + 6 * g;
    const double *pv = v + 3 * g;
    const uint32_t dst = __builtin_amdgcn_readfirstlane(lds_addr(smem) + (uint32_t)(l >> 6) * 1024u);
    load_to_lds16(pr, dst);
    load_to_lds16(pr + 2, dst + kPieceBytes);
    load_to_lds16(pr + 4, dst + 2 * kPieceBytes);
    load_to_lds16(pv, dst + 3 * kPieceBytes);
    load_to_lds16(pv + 1, dst + 4 * kPieceBytes);
}

// After slot l's loads have landed: prescribed direction components read as 0
// (only while a mask is in force: a caller may clear m.nmask for one launch to
// take the action on the unmasked input, the staging words keep their bits).
__device__ __forceinline__ void chunk_stage_mask(const BlockMesh &m, unsigned char *smem, int l, uint32_t word)
{
    const uint32_t bits = word >> 28;
    if (!m.nmask || l < 0 || !bits) return;
    double *p3 = reinterpret_cast<double *>(smem + 3 * kPieceBytes + 16 * l);
    double *p4 = reinterpret_cast<double *>(smem + 4 * kPieceBytes + 16 * l);
    if (bits & 1u) p3[0] = 0.0;
    if (bits & 2u) p3[1] = 0.0, p4[0] = 0.0;
    if (bits & 4u) p4[1] = 0.0;
}

// Write-out of one chunk slot whose sum is final: to its halo entry (dst =
// kShared | entry) or to y (dst = global id | Dirichlet bits << 28; ACC:
// y += sum), prescribed components fixed_val while a mask is in force.
template <bool ACC>
__device__ __forceinline__ void chunk_fin_store(const double *acc, int slot, uint32_t dst, double *__restrict__ y,
                                                double *__restrict__ halo, bool masked, double fixed_val)
{
    const double s0 = acc[3 * slot], s1 = acc[3 * slot + 1], s2 = acc[3 * slot + 2];
    if (dst & kShared) {
        double *h = halo + 3 * (int64_t)(dst & ~kShared);
        h[0] = s0, h[1] = s1, h[2] = s2;
        return;
    }
    const int64_t g = dst & kStageGid;
    const uint32_t bits = masked ? (dst >> 28) & 7u : 0u;
    const double sv[3] = {s0, s1, s2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double *d = &y[3 * g + c];
        if ((bits >> c) & 1u) *d = fixed_val;
        else *d = ACC ? *d + sv[c] : sv[c];
    }
}

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima).  The builtin,
// not inline asm, so that the compiler's own wait insertion knows every
// vector-memory load has completed here.
__device__ __forceinline__ void wait_vm_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// UNI: a uniform material (the two kernel-argument scalars); otherwise per element.
template <bool ACC, bool UNI>
__global__ void __launch_bounds__(kChunkThreads)
k_chunk_hvp64(BlockMesh m, ChunkMesh ch, const double *__restrict__ xrec, const double *__restrict__ v,
              double *__restrict__ y, int use_mask, double fixed_val, const int32_t *__restrict__ skip)
{
    __shared__ __align__(16) unsigned char smem[kChunkLds];
    if (skip && *skip) return;
    constexpr int W = kChunkThreads / 64;
    const int c = xcd_remap(blockIdx.x, ch.n_chunks);
    // Step 0 first: thread t stages slot t from a word indexed by chunk and
    // thread, read beside the chunk's header (scalar loads), so the record
    // loads wait for one memory latency only.  Everything else the first step
    // needs arrives while they are in flight, through LDS or in registers: a
    // vector load waited for here would also wait for the records.
    const uint32_t word0 = ch.cword0[(int64_t)c * kChunkThreads + threadIdx.x];
    const int4 h0 = ch.hdr[2 * c], h1 = ch.hdr[2 * c + 1];
    const int l0 = word0 != 0xffffffffu ? (int)threadIdx.x : -1;
    chunk_stage_records(smem, xrec, v, l0, word0);

    const int b0 = h0.x, nsteps = h0.y, s0 = h0.z, ns = h0.w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *acc = reinterpret_cast<double *>(smem + 5 * kPieceBytes);
    // this wave's staging words: those of the step after next arrive with
    // global-to-LDS loads, so issuing a step's record loads waits for LDS only
    uint32_t *words = reinterpret_cast<uint32_t *>(smem + 5 * kPieceBytes + kChunkCap * 24) + 64 * wave;
    const uint32_t wdst = __builtin_amdgcn_readfirstlane(lds_addr(words));
    // the chunk's block table in LDS: no global load is waited for inside a
    // step, where the wait would also wait for the records in flight
    int32_t *t_istart = reinterpret_cast<int32_t *>(smem + 5 * kPieceBytes + kChunkCap * 24 + kChunkThreads * 4);
    int32_t *t_estart = t_istart + kChunkSteps + 1;
    uint32_t *t_bnew = reinterpret_cast<uint32_t *>(t_estart + kChunkSteps + 1);
    int32_t *t_fin = reinterpret_cast<int32_t *>(t_bnew + kChunkSteps);
    const uint32_t *cword = ch.cword + s0;
    // the items of a step: lane L of wave w takes item L * W + w, so the
    // lanes of one LDS atomic are W items apart in Morton order
    const int k = lane * W + wave;
    uint2 itw = make_uint2(0u, 0u);
    // per-element materials: the item's position in the block pass's order,
    // which the element arrays follow (the chunk pass orders items its own way)
    int kb = 0;
    if (k < h1.y) {
        itw = *reinterpret_cast<const uint2 *>(ch.items + 2 * (int64_t)(h1.x + k));
        if (!UNI) kb = ch.iperm[h1.x + k];
    }
    if (nsteps > 1) {
        const int l1 = chunk_stage_slot((uint32_t)h1.z, wave, lane);
        if (l1 >= 0) load_to_lds4(cword + l1, wdst);
    }
    // the block table (nsteps + 1 <= 64 entries) by wave 0 with LDS loads
    if (wave == 0 && lane <= nsteps) {
        load_to_lds4(m.istart + b0 + lane, __builtin_amdgcn_readfirstlane(lds_addr(t_istart)));
        load_to_lds4(m.estart + b0 + lane, __builtin_amdgcn_readfirstlane(lds_addr(t_estart)));
        load_to_lds4(ch.fin_start + b0 + lane, __builtin_amdgcn_readfirstlane(lds_addr(t_fin)));
    }
    if (wave == 0 && lane < nsteps) load_to_lds4(ch.bnew + b0 + lane, __builtin_amdgcn_readfirstlane(lds_addr(t_bnew)));
    for (int i = threadIdx.x; i < 3 * ns; i += kChunkThreads) acc[i] = 0.0;
    wait_vm_loads();
    chunk_stage_mask(m, smem, l0, word0);
    __syncthreads();

    bool bad = false;
    const bool masked = use_mask != 0 && m.nmask;
    // Progressive write-out: a slot's sum is final at the barrier after the
    // last block that touches it.  Its store goes out at the start of the
    // next step, under that step's arithmetic, instead of in one burst after
    // the last step.  The destinations are loaded a step ahead, and the
    // stores are issued at a step's start: every store counts in vmcnt, so a
    // store issued late in a step would hold up the step's closing wait.
    int fj = -1, fslot = 0;   // this thread's pending slot (final after the previous block)
    uint32_t fdst = 0u;
    for (int t = 0; t < nsteps; ++t) {
        if (fj >= 0) {
            chunk_fin_store<ACC>(acc, fslot, fdst, y, ch.halo, masked, fixed_val);
            // more final slots than threads (not met at the default sizes)
            for (int j = fj + kChunkThreads; j < t_fin[t]; j += kChunkThreads)
                chunk_fin_store<ACC>(acc, ch.fin_slot[j], ch.fin_dst[j], y, ch.halo, masked, fixed_val);
        }
        // records of step t+1 on their way, then the words of step t+2
        uint32_t word1 = 0u;
        if (t + 1 < nsteps) {
            const int l1 = chunk_stage_slot(t_bnew[t + 1], wave, lane);
            if (l1 >= 0) word1 = words[lane];
            chunk_stage_records(smem, xrec, v, l1, word1);
            if (t + 2 < nsteps) {
                const int l2 = chunk_stage_slot(t_bnew[t + 2], wave, lane);
                if (l2 >= 0) load_to_lds4(cword + l2, wdst);
            }
        }
        // the slots final after this step, stored at the next step's start
        fj = -1;
        if (t + 1 < nsteps) {
            const int j = t_fin[t] + (int)threadIdx.x;
            if (j < t_fin[t + 1]) {
                fj = j;
                fslot = ch.fin_slot[j];
                fdst = ch.fin_dst[j];
            }
        }
        const uint2 cur = itw;
        const int kbc = kb;
        const int i0 = t_istart[t], ni = t_istart[t + 1] - i0;
        if (t + 1 < nsteps && k < t_istart[t + 2] - t_istart[t + 1]) {
            itw = *reinterpret_cast<const uint2 *>(ch.items + 2 * (int64_t)(t_istart[t + 1] + k));
            if (!UNI) kb = ch.iperm[t_istart[t + 1] + k];
        }

        if (k < ni) {
            ItemRange r;
            r.i0 = i0;
            r.ni = ni;
            r.e0 = t_estart[t];
            r.np = (t_estart[t + 1] - r.e0) - ni;
            int lc[5];
            lc[0] = (int)(cur.x & 2047u);
            lc[1] = (int)((cur.x >> 11) & 2047u);
            lc[2] = (int)(cur.y & 2047u);
            lc[3] = (int)((cur.x >> 22) | ((cur.y >> 22) << 10));
            lc[4] = (int)((cur.y >> 11) & 2047u);
            double Xe[5][3], xe[5][3], ve[5][3];
            const double2 *P = reinterpret_cast<const double2 *>(smem);
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                const int s = lc[a];
                const double2 p0 = P[s], p1 = P[kChunkCap + s], p2 = P[2 * kChunkCap + s];
                const double2 p3 = P[3 * kChunkCap + s];
                const double v2 = reinterpret_cast<const double *>(P + 4 * kChunkCap + s)[1];
                Xe[a][0] = p0.x, Xe[a][1] = p0.y, Xe[a][2] = p1.x;
                xe[a][0] = p1.y, xe[a][1] = p2.x, xe[a][2] = p2.y;
                ve[a][0] = p3.x, ve[a][1] = p3.y, ve[a][2] = v2;
            }
            double mu[2], lam[2];
            if (UNI) {
                mu[0] = mu[1] = m.mu0;
                lam[0] = lam[1] = m.lam0;
            } else {
                item_materials<Tet4Pair>(m, r, kbc, mu, lam);
            }
            double f[5][3];
            bad |= !HvpOp<double>::compute<Tet4Pair>(Xe, xe, ve, mu, lam, k < r.np, f);
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i) atomicAdd(&acc[3 * lc[a] + i], f[a][i]);
        }
        wait_vm_loads();
        if (t + 1 < nsteps) chunk_stage_mask(m, smem, chunk_stage_slot(t_bnew[t + 1], wave, lane), word1);
        __syncthreads();
    }
    if (bad) flag_inverted(m.flags);
    // the slots final after the last step
    for (int j = t_fin[nsteps - 1] + (int)threadIdx.x; j < t_fin[nsteps]; j += kChunkThreads)
        chunk_fin_store<ACC>(acc, ch.fin_slot[j], ch.fin_dst[j], y, ch.halo, masked, fixed_val);
}

// ------------------------------------------------------------------- energy

template <class E, bool LIN>
__global__ void __launch_bounds__(256) k_energy(BlockMesh m, const double *__restrict__ X,
                                                const double *__restrict__ u,
                                                double *__restrict__ partials)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[256];
    const int count = m.n_blocks;
    const int b = xcd_remap(blockIdx.x, count);
    const int n0 = m.nstart[b], nn = m.nstart[b + 1] - n0;
    const ItemRange r = item_range(m, b);
    NodeXU *sn = reinterpret_cast<NodeXU *>(smem);
    XUStage st{X, u};
    const int nt = blockDim.x;
    int k = threadIdx.x;
    IData<E> nxt{};
    if (k < r.ni) nxt = fetch_item<E>(m, r, k);
    stage_nodes(m, st, sn, m.bnode + n0, nn, [](int, uint32_t) {});
    __syncthreads();
    double acc = 0.0;
    bool bad = false;
    for (; k < r.ni; k += nt) {
        const IData<E> cur = nxt;
        if (k + nt < r.ni) nxt = fetch_item<E>(m, r, k + nt);
        uint16_t lc[E::NEN];
        unpack_lc<E>(cur.lc, lc);
        typename E::template Field<double> FX, Fu;
        gather_xu<E>(sn, lc, FX, Fu);
        const bool pair = k < r.np;
        double pe = 0.0;
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            const double mu = cur.mu[E::sub(q)], lam = cur.lam[E::sub(q)];
            double Jx[9], Hxi[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fu, q, Hxi);
            if (LIN) {
                double Ae[9], H[9], ee, tr;
                const double De = lin_grad(Jx, Hxi, Ae, H);
                lin_invariants(H, ee, tr);
                pe += E::template weight<double>() * De * (mu * ee + 0.5 * lam * tr * tr);
                continue;
            }
            Kin kk;
            kinematics(E::template weight<double>(), Jx, Hxi, kk);
            if (!(1.0 + kk.Jm1 > 0.0)) {
                bad = true;
                continue;
            }
            const double lnJ = log1p_(kk.Jm1);
            pe += kk.wDe * (0.5 * mu * kk.I1m3 - mu * lnJ + 0.5 * lam * lnJ * lnJ);
        }
        acc += pe;
    }
    if (bad) {
        flag_inverted(m.flags);
        acc = INFINITY;
    }
    // deterministic tree over the workgroup
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[b] = red[0];
}

// One workgroup: Neumaier sums of the block partials over a fixed strided
// assignment, then a fixed tree.  A separate launch, so the partials of the
// previous kernel are visible without device-wide fences.
__global__ void __launch_bounds__(256) k_sum_partials(const double *__restrict__ partials, int count,
                                                      double *__restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        const double x = partials[i];
        const double t = s + x;
        if (isfinite(t)) c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    red[threadIdx.x] = isfinite(s) ? s + c : s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ---------------------------------------------------- per-element adjoint kernels

// dPsi/dmu_e, dPsi/dlam_e at fixed u.
template <class E, bool LIN>
__global__ void __launch_bounds__(256) k_grad_material(BlockMesh m, const double *__restrict__ X,
                                                       const double *__restrict__ u,
                                                       double *__restrict__ dmu,
                                                       double *__restrict__ dlam)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = xcd_remap(blockIdx.x, m.n_blocks);
    const int n0 = m.nstart[b], nn = m.nstart[b + 1] - n0;
    const ItemRange r = item_range(m, b);
    NodeXU *sn = reinterpret_cast<NodeXU *>(smem);
    XUStage st{X, u};
    stage_nodes(m, st, sn, m.bnode + n0, nn, [](int, uint32_t) {});
    __syncthreads();
    bool bad = false;
    for (int k = threadIdx.x; k < r.ni; k += blockDim.x) {
        const IData<E> d = fetch_item<E>(m, r, k);
        uint16_t lc[E::NEN];
        unpack_lc<E>(d.lc, lc);
        typename E::template Field<double> FX, Fu;
        gather_xu<E>(sn, lc, FX, Fu);
        const bool pair = k < r.np;
        double gm[E::NSUB] = {}, gl[E::NSUB] = {};
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            double Jx[9], Hxi[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fu, q, Hxi);
            if (LIN) {
                double Ae[9], H[9], ee, tr;
                const double wDe = E::template weight<double>() * lin_grad(Jx, Hxi, Ae, H);
                lin_invariants(H, ee, tr);
                gm[E::sub(q)] += wDe * ee;
                gl[E::sub(q)] += wDe * 0.5 * tr * tr;
                continue;
            }
            Kin kk;
            kinematics(E::template weight<double>(), Jx, Hxi, kk);
            if (!(1.0 + kk.Jm1 > 0.0)) {
                bad = true;
                continue;
            }
            const double lnJ = log1p_(kk.Jm1);
            gm[E::sub(q)] += kk.wDe * (0.5 * kk.I1m3 - lnJ);
            gl[E::sub(q)] += kk.wDe * 0.5 * lnJ * lnJ;
        }
#pragma unroll
        for (int s = 0; s < E::NSUB; ++s) {
            if (s > 0 && !pair) break;
            const int eo = m.eorig[r.elem(k, s)];
            dmu[eo] = gm[s];
            dlam[eo] = gl[s];
        }
    }
    if (bad) flag_inverted(m.flags);
}

// w . dr/dmu_e = sum_q w detJ (F - F^-T) : grad w,  w . dr/dlam_e = sum_q w detJ lnJ F^-T : grad w
// linear model: w . dr/dmu_e = sum_q w detJ 2 eps(u) : grad w,  w . dr/dlam_e = sum_q w detJ tr eps(u) div w
template <class E, bool LIN>
__global__ void __launch_bounds__(256) k_vjp_material(BlockMesh m, const double *__restrict__ X,
                                                      const double *__restrict__ u,
                                                      const double *__restrict__ wv,
                                                      double *__restrict__ dmu,
                                                      double *__restrict__ dlam)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = xcd_remap(blockIdx.x, m.n_blocks);
    const int n0 = m.nstart[b], nn = m.nstart[b + 1] - n0;
    const ItemRange r = item_range(m, b);
    NodeXUW *sn = reinterpret_cast<NodeXUW *>(smem);
    XUWStage st{X, u, wv};
    stage_nodes(m, st, sn, m.bnode + n0, nn, [](int, uint32_t) {});
    __syncthreads();
    bool bad = false;
    for (int k = threadIdx.x; k < r.ni; k += blockDim.x) {
        const IData<E> d = fetch_item<E>(m, r, k);
        uint16_t lc[E::NEN];
        unpack_lc<E>(d.lc, lc);
        typename E::template Field<double> FX, Fu, Fw;
        {
            double Xe[E::NEN][3], ue[E::NEN][3], we[E::NEN][3];
#pragma unroll
            for (int a = 0; a < E::NEN; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    Xe[a][i] = sn[lc[a]].X[i];
                    ue[a][i] = sn[lc[a]].u[i];
                    we[a][i] = sn[lc[a]].w[i];
                }
            E::prep(Xe, FX);
            E::prep(ue, Fu);
            E::prep(we, Fw);
        }
        const bool pair = k < r.np;
        double gm[E::NSUB] = {}, gl[E::NSUB] = {};
#pragma unroll
        for (int q = 0; q < E::NQ; ++q) {
            if (E::skip(q, pair)) continue;
            double Jx[9], Hxi[9], Wxi[9], Ae[9];
            E::grad(FX, q, Jx);
            E::geom(Jx);
            E::grad(Fu, q, Hxi);
            E::grad(Fw, q, Wxi);
            if (LIN) {
                double H[9], Gw[9];
                const double wDe = E::template weight<double>() * lin_grad(Jx, Hxi, Ae, H);
                lin_grad(Jx, Wxi, Ae, Gw);
                double sm = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int J = 0; J < 3; ++J) sm += (H[i * 3 + J] + H[J * 3 + i]) * Gw[i * 3 + J];
                gm[E::sub(q)] += wDe * sm;
                gl[E::sub(q)] += wDe * (H[0] + H[4] + H[8]) * (Gw[0] + Gw[4] + Gw[8]);
                continue;
            }
            Kin kk;
            kinematics(E::template weight<double>(), Jx, Hxi, kk);
            if (!(1.0 + kk.Jm1 > 0.0)) {
                bad = true;
                continue;
            }
            const double lnJ = log1p_(kk.Jm1);
            const double De = adj_det(Jx, Ae);
            double F[9], Fa[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) F[i] = kk.H[i] + ((i % 4) == 0 ? 1.0 : 0.0);
            const double rdF = 1.0 / adj_det(F, Fa);
            double sm = 0.0, sl = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int J = 0; J < 3; ++J) {
                    const double gw = (Wxi[i * 3 + 0] * Ae[0 * 3 + J] + Wxi[i * 3 + 1] * Ae[1 * 3 + J]
                                       + Wxi[i * 3 + 2] * Ae[2 * 3 + J]) / De;
                    const double FiT = Fa[J * 3 + i] * rdF;
                    sm += (F[i * 3 + J] - FiT) * gw;
                    sl += lnJ * FiT * gw;
                }
            gm[E::sub(q)] += kk.wDe * sm;
            gl[E::sub(q)] += kk.wDe * sl;
        }
#pragma unroll
        for (int s = 0; s < E::NSUB; ++s) {
            if (s > 0 && !pair) break;
            const int eo = m.eorig[r.elem(k, s)];
            dmu[eo] = gm[s];
            dlam[eo] = gl[s];
        }
    }
    if (bad) flag_inverted(m.flags);
}

// ---------------------------------------------------------------- launchers

template <class Op>
static size_t lds_bytes(const Ctx &c, size_t acc_elem)
{
    // node records, FP64 accumulators and the block-node words
    return (sizeof(typename Op::Node) + 3 * acc_elem + sizeof(uint32_t)) * (size_t)c.max_block_nodes;
}

template <class T>
static void launch_gather(const Ctx &c, bool acc, const HaloMap &hm, const T *halo, T *y, const uint8_t *mask,
                          T fixed_val, const int32_t *skip)
{
    const unsigned gb = (unsigned)((hm.seg.n + 255) / 256);
    auto kern = acc ? (mask ? k_halo_gather<T, true, true> : k_halo_gather<T, true, false>)
                    : (mask ? k_halo_gather<T, false, true> : k_halo_gather<T, false, false>);
    hipLaunchKernelGGL(kern, dim3(gb), dim3(256), 0, c.stream, hm.seg, hm.gptr, hm.node, halo, y, mask, fixed_val,
                       skip);
}

// The chunk pass of the FP64 Tet4 tangent action, then the gather of the
// nodes that several chunks share.
static hipError_t run_chunks(const Ctx &c, const HvpOp<double> &op, double *y, bool use_mask,
                             const int32_t *skip, WriteMode mode)
{
    const bool acc = mode == WriteMode::Accumulate, uni = c.m.mu == nullptr;
    const uint8_t *gmask = use_mask ? c.m.nmask : nullptr;
    auto kern = acc ? (uni ? k_chunk_hvp64<true, true> : k_chunk_hvp64<true, false>)
                    : (uni ? k_chunk_hvp64<false, true> : k_chunk_hvp64<false, false>);
    hipLaunchKernelGGL(kern, dim3(c.ch.n_chunks), dim3(kChunkThreads), 0, c.stream, c.m, c.ch, op.xrec, op.v, y,
                       use_mask ? 1 : 0, 0.0, skip);
    if (c.n_ch_shared > 0)
        launch_gather<double>(c, acc, c.ch_halo, c.ch.halo, y, gmask, 0.0, skip);
    return hipGetLastError();
}

template <class E, class Op, class T>
static hipError_t run_accumulate(const Ctx &c, const Op &op, T *y, bool use_mask, T fixed_val,
                                 const int32_t *skip, WriteMode mode)
{
    if constexpr (std::is_same<E, Tet4Pair>::value && std::is_same<Op, HvpOp<double>>::value)
        if (c.ch.n_chunks > 0 && c.scatter == Scatter::Halo) return run_chunks(c, op, y, use_mask, skip, mode);
    const size_t lds = lds_bytes<Op>(c, sizeof(double));
    const bool halo = c.scatter == Scatter::Halo && c.n_shared > 0;
    const uint8_t *gmask = use_mask ? c.m.nmask : nullptr;
    if (mode == WriteMode::Accumulate) {
        for (const Pass &p : c.passes) {
            if (p.count == 0) continue;
            hipLaunchKernelGGL((k_accumulate<E, Op, T, true>), dim3(p.count), dim3(c.threads), lds,
                               c.stream, c.m, op, y, p.list, p.count, c.scatter, use_mask ? 1 : 0,
                               fixed_val, skip);
        }
        if (halo)
            launch_gather<T>(c, true, c.halo, reinterpret_cast<const T *>(c.m.halo), y, gmask, fixed_val, skip);
        return hipGetLastError();
    }
    if (mode == WriteMode::Overwrite && c.scatter == Scatter::Atomic && c.n_shared > 0) {
        const int64_t n = c.n_nodes;
        hipLaunchKernelGGL((k_fill_nodal<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           c.stream, n, y, use_mask ? c.m.nmask : nullptr, fixed_val);
    }
    for (const Pass &p : c.passes) {
        if (p.count == 0) continue;
        hipLaunchKernelGGL((k_accumulate<E, Op, T, false>), dim3(p.count), dim3(c.threads), lds, c.stream,
                           c.m, op, y, p.list, p.count, c.scatter, use_mask ? 1 : 0, fixed_val,
                           skip);
    }
    if (halo)
        launch_gather<T>(c, false, c.halo, reinterpret_cast<const T *>(c.m.halo), y, gmask, fixed_val, skip);
    return hipGetLastError();
}

template <class Op, class T>
static hipError_t dispatch(const Ctx &c, const Op &op, T *y, bool use_mask, T fixed_val,
                           const int32_t *skip = nullptr, WriteMode mode = WriteMode::Overwrite)
{
    if (c.elem == EFEM_TRI3) return run_accumulate<Tri3>(c, op, y, use_mask, fixed_val, skip, mode);
    return c.elem == EFEM_TET4 ? run_accumulate<Tet4Pair>(c, op, y, use_mask, fixed_val, skip, mode)
                               : run_accumulate<Hex8>(c, op, y, use_mask, fixed_val, skip, mode);
}

hipError_t launch_residual(const Ctx &c, const double *u, double *r)
{
    if (c.model == EFEM_MODEL_TRANSPORT) {
        TransportOp<double> op{c.m.X, u, c.omega[0], c.omega[1], c.omega[2], 0};
        return dispatch(c, op, r, true, 0.0);
    }
    if (c.model == EFEM_MODEL_LINEAR) {
        LinResidualOp op;
        op.X = c.m.X;
        op.u = u;
        return dispatch(c, op, r, true, 0.0);
    }
    ResidualOp op;
    op.X = c.m.X;
    op.u = u;
    return dispatch(c, op, r, true, 0.0);
}

hipError_t launch_diag(const Ctx &c, const double *u, double *d)
{
    if (c.model == EFEM_MODEL_TRANSPORT) {
        TransportDiagOp op;
        op.X = c.m.X;
        op.u = u;
        op.om0 = c.omega[0];
        op.om1 = c.omega[1];
        op.om2 = c.omega[2];
        return dispatch(c, op, d, true, 1.0);
    }
    if (c.model == EFEM_MODEL_LINEAR) {
        LinDiagOp op;
        op.X = c.m.X;
        op.u = u;
        return dispatch(c, op, d, true, 1.0);
    }
    DiagOp op;
    op.X = c.m.X;
    op.u = u;
    return dispatch(c, op, d, true, 1.0);
}

hipError_t launch_offdiag(const Ctx &c, const double *u, double *o)
{
    if (c.model == EFEM_MODEL_LINEAR) {
        OffDiagOp<true> op;
        op.X = c.m.X;
        op.u = u;
        return dispatch(c, op, o, false, 0.0);
    }
    OffDiagOp<false> op;
    op.X = c.m.X;
    op.u = u;
    return dispatch(c, op, o, false, 0.0);
}

hipError_t launch_grad_coords(const Ctx &c, const double *u, double *g)
{
    if (c.model == EFEM_MODEL_LINEAR) {
        LinGradCoordsOp op;
        op.X = c.m.X;
        op.u = u;
        return dispatch(c, op, g, false, 0.0);
    }
    GradCoordsOp op;
    op.X = c.m.X;
    op.u = u;
    return dispatch(c, op, g, false, 0.0);
}

hipError_t launch_hvp_f64(const Ctx &c, const double *xlin, const double *v, double *y,
                          const int32_t *skip, WriteMode mode)
{
    if (c.model == EFEM_MODEL_TRANSPORT) {
        TransportOp<double> op{c.m.X, v, c.omega[0], c.omega[1], c.omega[2], 1};
        return dispatch(c, op, y, true, 0.0, skip, mode);
    }
    if (c.model == EFEM_MODEL_LINEAR) {
        LinHvpOp<double> op{c.m.X, v};
        return dispatch(c, op, y, true, 0.0, skip, mode);
    }
    HvpOp<double> op{xlin, v, y};
    return dispatch(c, op, y, true, 0.0, skip, mode);
}

hipError_t launch_hvp_f32(const Ctx &c, const float *ulin, const float *v, float *y,
                          const int32_t *skip, WriteMode mode)
{
    if (c.model == EFEM_MODEL_TRANSPORT) {
        TransportOp<float> op{c.m.Xf, v, float(c.omega[0]), float(c.omega[1]), float(c.omega[2]), 1};
        return dispatch(c, op, y, true, 0.0f, skip, mode);
    }
    if (c.model == EFEM_MODEL_LINEAR) {
        LinHvpOp<float> op{c.m.Xf, v};
        return dispatch(c, op, y, true, 0.0f, skip, mode);
    }
    HvpOp<float> op{c.m.Xf, ulin, v, y};
    return dispatch(c, op, y, true, 0.0f, skip, mode);
}

template <class E, bool LIN>
static void energy_pass(const Ctx &c, const double *u, size_t lds, double *partials)
{
    hipLaunchKernelGGL((k_energy<E, LIN>), dim3(c.m.n_blocks), dim3(256), lds, c.stream, c.m, c.m.X, u,
                       partials);
}

// The energy's two launches with the per-block partials in `partials`.
static hipError_t energy_into(const Ctx &c, const double *u, double *psi, double *partials)
{
    const size_t lds = sizeof(NodeXU) * (size_t)c.max_block_nodes;
    const bool lin = c.model == EFEM_MODEL_LINEAR;
    if (c.elem == EFEM_TET4)
        lin ? energy_pass<Tet4Pair, true>(c, u, lds, partials) : energy_pass<Tet4Pair, false>(c, u, lds, partials);
    else if (c.elem == EFEM_TRI3)
        lin ? energy_pass<Tri3, true>(c, u, lds, partials) : energy_pass<Tri3, false>(c, u, lds, partials);
    else lin ? energy_pass<Hex8, true>(c, u, lds, partials) : energy_pass<Hex8, false>(c, u, lds, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, c.stream, partials, c.m.n_blocks, psi);
    return hipGetLastError();
}

hipError_t launch_energy(const Ctx &c, const double *u, double *psi)
{
    return energy_into(c, u, psi, c.partials);
}

// ---------------------------------------------- energy without allocation

// The per-block energy partials of efem_energy_noalloc live in this array, one
// copy per GPU for the life of the process.  In host code `scratch` names a
// host-side stand-in, never the device memory: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is ever handed to a kernel.
static __device__ __align__(256) double scratch[kNoAllocBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the caller made `device` current
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double *>(p);
    return hipSuccess;
}

hipError_t launch_energy_noalloc(const Ctx &c, const double *u, double *psi)
{
    double *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mutex);
        if (c.device >= 0 && c.device < kMaxDevices) p = g_scratch_ptr[c.device];
    }
    if (!p) return hipErrorNotInitialized;
    // every partial is written by its block before k_sum_partials reads it,
    // so the array needs no clearing between calls
    return energy_into(c, u, psi, p);
}

template <class E, bool LIN>
static void grad_material_pass(const Ctx &c, const double *u, double *dmu, double *dlam, size_t lds)
{
    hipLaunchKernelGGL((k_grad_material<E, LIN>), dim3(c.m.n_blocks), dim3(c.threads), lds, c.stream, c.m,
                       c.m.X, u, dmu, dlam);
}

hipError_t launch_grad_material(const Ctx &c, const double *u, double *dmu, double *dlam)
{
    const size_t lds = sizeof(NodeXU) * (size_t)c.max_block_nodes;
    const bool lin = c.model == EFEM_MODEL_LINEAR;
    if (c.elem == EFEM_TET4)
        lin ? grad_material_pass<Tet4Pair, true>(c, u, dmu, dlam, lds)
            : grad_material_pass<Tet4Pair, false>(c, u, dmu, dlam, lds);
    else if (c.elem == EFEM_TRI3)
        lin ? grad_material_pass<Tri3, true>(c, u, dmu, dlam, lds) : grad_material_pass<Tri3, false>(c, u, dmu, dlam, lds);
    else
        lin ? grad_material_pass<Hex8, true>(c, u, dmu, dlam, lds)
            : grad_material_pass<Hex8, false>(c, u, dmu, dlam, lds);
    return hipGetLastError();
}

template <class E, bool LIN>
static void vjp_material_pass(const Ctx &c, const double *u, const double *w, double *dmu, double *dlam,
                              size_t lds)
{
    hipLaunchKernelGGL((k_vjp_material<E, LIN>), dim3(c.m.n_blocks), dim3(c.threads), lds, c.stream, c.m,
                       c.m.X, u, w, dmu, dlam);
}

hipError_t launch_vjp_material(const Ctx &c, const double *u, const double *w, double *dmu,
                               double *dlam)
{
    const size_t lds = sizeof(NodeXUW) * (size_t)c.max_block_nodes;
    const bool lin = c.model == EFEM_MODEL_LINEAR;
    if (c.elem == EFEM_TET4)
        lin ? vjp_material_pass<Tet4Pair, true>(c, u, w, dmu, dlam, lds)
            : vjp_material_pass<Tet4Pair, false>(c, u, w, dmu, dlam, lds);
    else if (c.elem == EFEM_TRI3)
        lin ? vjp_material_pass<Tri3, true>(c, u, w, dmu, dlam, lds)
            : vjp_material_pass<Tri3, false>(c, u, w, dmu, dlam, lds);
    else
        lin ? vjp_material_pass<Hex8, true>(c, u, w, dmu, dlam, lds)
            : vjp_material_pass<Hex8, false>(c, u, w, dmu, dlam, lds);
    return hipGetLastError();
}

}  // namespace efem
