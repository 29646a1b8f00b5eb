// Restarted GMRES with right Jacobi preconditioning, the Krylov solver for a
// non-symmetric tangent (the non-variational transport model: the virtual-work form of Sec. 3.1,
// where CG does not apply), usable with every model.  Solves
//     K(u)_ff x_f = b_f,   x = 0 on prescribed DOFs,
// from x = 0.  The Arnoldi basis is float64 on the device; orthogonalisation
// is classical Gram-Schmidt applied twice (one multi-dot and one multi-axpy
// kernel per pass, the projections kept on the device), so each iteration
// needs one small host read (both projections and w.w).  The Hessenberg matrix, its Givens rotations
// and the small triangular solve live on the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "efem_gmres.h"

namespace efem {

namespace {

struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

int dev_alloc(DevBuf &b, size_t bytes)
{
    hipError_t e = hipMalloc(&b.p, std::max<size_t>(bytes, 8));
    if (e != hipSuccess) {
        b.p = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    return EFEM_OK;
}

#define GTRY(call)                                             \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(e_, #call);      \
    } while (0)

struct Gmres {
    Ctx &c;
    int prec, m;
    int64_t n;
    hipStream_t s;
    DevBuf V, w, z, dinv, diag, part, hdev, z32, w32;

    Gmres(Ctx &ctx, int prec_, int m_) : c(ctx), prec(prec_), m(m_), n(3 * ctx.n_nodes), s(ctx.stream) {}

    int setup()
    {
        int rc;
        const size_t nb = (size_t)n * sizeof(double);
        if ((rc = dev_alloc(V, nb * (size_t)(m + 1))) || (rc = dev_alloc(w, nb)) || (rc = dev_alloc(z, nb))
            || (rc = dev_alloc(dinv, nb)) || (rc = dev_alloc(diag, nb))
            || (rc = dev_alloc(part, sizeof(double) * kGmresRedBlocks * (size_t)(m + 2)))
            || (rc = dev_alloc(hdev, sizeof(double) * (size_t)(2 * m + 3))))
            return rc;
        if (prec == EFEM_F32 && ((rc = dev_alloc(z32, (size_t)n * sizeof(float))) || (rc = dev_alloc(w32, (size_t)n * sizeof(float)))))
            return rc;
        return EFEM_OK;
    }
    double *Vj(int j) const { return V.as<double>() + (int64_t)j * n; }

    // out = K in (masked: prescribed inputs read as 0, prescribed outputs 0)
    int apply(const double *in, double *out)
    {
        if (prec == EFEM_F64) {
            GTRY(launch_hvp_f64(c, c.xlin, in, out, nullptr, WriteMode::Overwrite));
        } else {
            GTRY(gm_to_f32(s, n, in, z32.as<float>()));
            GTRY(launch_hvp_f32(c, c.ulin, z32.as<float>(), w32.as<float>(), nullptr, WriteMode::Overwrite));
            GTRY(gm_to_f64(s, n, w32.as<float>(), out));
        }
        return EFEM_OK;
    }
    int norm(const double *vec, double &out)
    {
        double h = 0.0;
        GTRY(gm_mdot(s, n, vec, 1, vec, part.as<double>(), hdev.as<double>()));
        GTRY(hipMemcpyAsync(&h, hdev.p, sizeof(double), hipMemcpyDeviceToHost, s));
        GTRY(hipStreamSynchronize(s));
        out = std::sqrt(std::max(h, 0.0));
        return EFEM_OK;
    }

    int run(const double *b, double *x, double rtol, int max_iter, int *iters, double *relres)
    {
        int rc;
        const uint8_t *mask = c.m.nmask;
        GTRY(launch_diag(c, x, diag.as<double>()));   // x holds u here: the diagonal at u
        GTRY(gm_dinv(s, n, diag.as<double>(), mask, dinv.as<double>()));
        GTRY(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), s));
        std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), h(m + 1), h2(m + 2), y(m);
        auto Hx = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
        double bnorm = -1.0, tol = 0.0;
        int total = 0;
        bool converged = false;
        for (;;) {
            // r = b - K x on free DOFs, into V_0
            if (total == 0) {
                GTRY(hipMemsetAsync(w.p, 0, (size_t)n * sizeof(double), s));
            } else if ((rc = apply(x, w.as<double>()))) {
                return rc;
            }
            GTRY(gm_residual(s, n, b, w.as<double>(), mask, Vj(0)));
            double beta;
            if ((rc = norm(Vj(0), beta))) return rc;
            if (bnorm < 0) {
                bnorm = beta;
                tol = rtol * bnorm;
            }
            if (beta <= tol || bnorm == 0.0) {
                converged = true;
                break;
            }
            if (total >= max_iter) break;
            GTRY(gm_scale(s, n, 1.0 / beta, Vj(0), Vj(0)));
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int jend = 0;
            for (int j = 0; j < m; ++j) {
                // the new vector is built in place, in basis slot j + 1
                double *wj = Vj(j + 1);
                double *h1d = hdev.as<double>(), *h2d = hdev.as<double>() + (m + 1);
                GTRY(gm_mul(s, n, dinv.as<double>(), Vj(j), z.as<double>()));
                if ((rc = apply(z.as<double>(), wj))) return rc;
                // classical Gram-Schmidt twice; the projections stay on the
                // device for the subtractions, and the second multi-dot also
                // takes w.w (slot j + 1 is w itself), so one read-back per
                // iteration serves the Hessenberg column and the new norm
                GTRY(gm_mdot(s, n, V.as<double>(), j + 1, wj, part.as<double>(), h1d));
                GTRY(gm_subtract(s, n, V.as<double>(), j + 1, h1d, wj));
                GTRY(gm_mdot(s, n, V.as<double>(), j + 2, wj, part.as<double>(), h2d));
                GTRY(gm_subtract(s, n, V.as<double>(), j + 1, h2d, wj));
                GTRY(hipMemcpyAsync(h.data(), h1d, sizeof(double) * (size_t)(j + 1), hipMemcpyDeviceToHost, s));
                GTRY(hipMemcpyAsync(h2.data(), h2d, sizeof(double) * (size_t)(j + 2), hipMemcpyDeviceToHost, s));
                GTRY(hipStreamSynchronize(s));
                // |w - V h2|^2 = w.w - |h2|^2 for orthonormal V; after the first
                // pass h2 is small against w, and where it is not (near a
                // breakdown) the norm is taken directly
                double hh = 0.0;
                for (int i = 0; i <= j; ++i) hh += h2[i] * h2[i];
                const double ww = h2[j + 1];
                double hn;
                if (ww - hh > 1e-8 * ww) {
                    hn = std::sqrt(ww - hh);
                } else if ((rc = norm(wj, hn))) {
                    return rc;
                }
                for (int i = 0; i <= j; ++i) Hx(i, j) = h[i] + h2[i];
                Hx(j + 1, j) = hn;
                // previous rotations, then a new one that zeroes H(j+1, j)
                for (int i = 0; i < j; ++i) {
                    const double t = cs[i] * Hx(i, j) + sn[i] * Hx(i + 1, j);
                    Hx(i + 1, j) = -sn[i] * Hx(i, j) + cs[i] * Hx(i + 1, j);
                    Hx(i, j) = t;
                }
                const double d = std::hypot(Hx(j, j), Hx(j + 1, j));
                cs[j] = d > 0 ? Hx(j, j) / d : 1.0;
                sn[j] = d > 0 ? Hx(j + 1, j) / d : 0.0;
                Hx(j, j) = d;
                Hx(j + 1, j) = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                ++total;
                jend = j + 1;
                const double res = std::fabs(g[j + 1]);
                const bool breakdown = !(hn > 1e-300 * beta);
                if (!breakdown) GTRY(gm_scale(s, n, 1.0 / hn, wj, wj));
                if (res <= tol || breakdown || total >= max_iter) break;
            }
            // y = H^-1 g (upper triangular), x += dinv V y
            for (int i = jend - 1; i >= 0; --i) {
                double t = g[i];
                for (int k = i + 1; k < jend; ++k) t -= Hx(i, k) * y[k];
                y[i] = Hx(i, i) != 0.0 ? t / Hx(i, i) : 0.0;
            }
            GTRY(hipMemcpyAsync(hdev.p, y.data(), sizeof(double) * (size_t)jend, hipMemcpyHostToDevice, s));
            GTRY(gm_update_x(s, n, V.as<double>(), jend, hdev.as<double>(), dinv.as<double>(), x));
            GTRY(hipStreamSynchronize(s));   // hdev is reused by the next cycle
        }
        // the true residual of the returned x
        if ((rc = apply(x, w.as<double>()))) return rc;
        GTRY(gm_residual(s, n, b, w.as<double>(), mask, z.as<double>()));
        double rn;
        if ((rc = norm(z.as<double>(), rn))) return rc;
        *iters = total;
        *relres = bnorm > 0 ? rn / bnorm : 0.0;
        return converged ? EFEM_OK : EFEM_NOT_CONVERGED;
    }
};

}  // namespace

}  // namespace efem

using namespace efem;

struct efem_ctx : Ctx {};

extern "C" int efem_gmres_solve(efem_ctx *ctx, const double *u, const double *b, double *x, double rtol,
                                int32_t hvp_prec, int32_t restart, int32_t max_iter, int32_t *iters,
                                double *relres)
{
    if (!ctx || !u || !b || !x || !iters || !relres || !(rtol > 0) || max_iter < 1 || restart < 1
        || restart > kGmresMaxRestart || (hvp_prec != EFEM_F64 && hvp_prec != EFEM_F32) || b == x || u == x) {
        set_error("efem_gmres_solve: bad argument");
        return EFEM_ERR_INVALID;
    }
    int dev_prev = -1;
    (void)hipGetDevice(&dev_prev);
    if (dev_prev != ctx->device) (void)hipSetDevice(ctx->device);
    int rc = efem_linearize(ctx, u, hvp_prec);
    if (rc == EFEM_OK) {
        Gmres solver(*ctx, hvp_prec, restart);
        rc = solver.setup();
        if (rc == EFEM_OK) {
            // the diagonal at u: stage it through x, which the solve overwrites anyway
            hipError_t e = hipMemcpyAsync(x, u, 3 * (size_t)ctx->n_nodes * sizeof(double),
                                          hipMemcpyDeviceToDevice, ctx->stream);
            rc = e == hipSuccess ? solver.run(b, x, rtol, max_iter, iters, relres) : hip_fail(e, "hipMemcpyAsync");
        }
    }
    if (dev_prev >= 0 && dev_prev != ctx->device) (void)hipSetDevice(dev_prev);
    return rc;
}
