// Matrix-free Newton-Krylov solver: a host loop over the element kernels
// (energy, residual, Jacobi diagonal, tangent action) and the streaming CG
// kernels.  The paper names the method (Sec. 6.3.1) but none of its parts; the
// reading implemented here:
//   * load steps k = 1..n: prescribed DOFs ramp to k/n of their final values;
//   * each step starts with a tangent predictor: the prescribed increment dc
//     is lifted into the free DOFs by solving K_ff d_f = -(K dc)_f;
//   * Newton iterations: Jacobi-PCG on K_ff d = -r_f with an Eisenstat-Walker
//     (choice 2) forcing term, then Armijo backtracking on the FP64 energy
//     (a step that inverts an element has energy +inf and is rejected), with a
//     slack of 64 eps |Psi| for the rounding of the energy sum;
//   * stop when ||r_f|| <= rtol ||r_f at the start of the step||.
// With hvp_prec = EFEM_F32 the CG vectors and tangent actions are float32;
// the residual, energy, line search and state stay float64.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <type_traits>

#include "efem_cg.h"
#include "efem_mlp.h"

namespace efem {

hipError_t mlp_precondition(Ctx &c, MlpState &M, const float *r, float *z);
hipError_t mlp_prepare(Ctx &c, MlpState &M, const double *diag);

// flexible-CG iterations without a new smallest residual before falling back
constexpr int kStallLimit = 30;

namespace {

#define TRY(call)                                              \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(e_, #call);      \
    } while (0)

template <class T>
struct Solver {
    Ctx &c;
    efem_solve_opts o;
    int64_t n;
    std::vector<void *> bufs;
    double *r = nullptr, *dc = nullptr, *u_old = nullptr, *u_trial = nullptr, *diag = nullptr,
           *kdc = nullptr, *dscal = nullptr;
    T *x = nullptr, *rv = nullptr, *p = nullptr, *q = nullptr, *dinv = nullptr;
    double *off = nullptr;   // precond = 2: off-diagonals of the nodes' 3x3 blocks
    uint16_t *binv = nullptr;   // and their inverses [n_nodes][6], bfloat16
    double load_s = 0.0;   // load factor of the current step
    CgScalars *sc = nullptr;
    CgWorkspace ws;
    CgScalars *h_sc = nullptr;
    double *h_scal = nullptr;
    CgLaunch<T> L{};

    Solver(Ctx &c_, const efem_solve_opts &o_) : c(c_), o(o_), n(3 * c_.n_nodes) {}

    ~Solver()
    {
        for (void *b : bufs) (void)hipFree(b);
        if (h_sc) (void)hipHostFree(h_sc);
        if (h_scal) (void)hipHostFree(h_scal);
    }

    template <class U>
    int alloc(U **ptr, size_t count)
    {
        void *q_ = nullptr;
        hipError_t e = hipMalloc(&q_, std::max<size_t>(count, 1) * sizeof(U));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        bufs.push_back(q_);
        *ptr = static_cast<U *>(q_);
        return EFEM_OK;
    }

    int setup()
    {
        int rc;
        if ((rc = alloc(&r, n)) || (rc = alloc(&dc, n)) || (rc = alloc(&u_old, n))
            || (rc = alloc(&u_trial, n)) || (rc = alloc(&diag, n)) || (rc = alloc(&kdc, n))
            || (rc = alloc(&dscal, 4)) || (rc = alloc(&x, n)) || (rc = alloc(&rv, n))
            || (rc = alloc(&p, n)) || (rc = alloc(&q, n)) || (rc = alloc(&dinv, n))
            || (rc = alloc(&sc, 1)) || (rc = alloc(&ws.partials, 4 * kMaxRedBlocks)))
            return rc;
        if (o.precond == 2 && ((rc = alloc(&off, n)) || (rc = alloc(&binv, 2 * n)))) return rc;   // 6 per node
        if (!c.xlin) {
            void *q_ = nullptr;
            TRY(hipMalloc(&q_, 2 * n * sizeof(double)));   // (X, X + u) per node
            c.owned.push_back(q_);
            c.xlin = static_cast<double *>(q_);
        }
        if (!c.ulin) {
            void *q_ = nullptr;
            TRY(hipMalloc(&q_, n * sizeof(float)));
            c.owned.push_back(q_);
            c.ulin = static_cast<float *>(q_);
        }
        TRY(hipHostMalloc((void **)&h_sc, sizeof(CgScalars), hipHostMallocDefault));
        TRY(hipHostMalloc((void **)&h_scal, 4 * sizeof(double), hipHostMallocDefault));
        L = CgLaunch<T>{n, c.stream, ws};
        L.clear_q = c.scatter == Scatter::Atomic;
        return EFEM_OK;
    }

    int read_scalar(const double *dptr, double &out)
    {
        TRY(hipMemcpyAsync(h_scal, dptr, sizeof(double), hipMemcpyDeviceToHost, c.stream));
        TRY(hipStreamSynchronize(c.stream));
        out = h_scal[0];
        return EFEM_OK;
    }

    // total potential energy Psi_h(u) - s f.u at load factor s (f = 0 without a load)
    int energy(const double *u, double &e)
    {
        TRY(launch_energy(c, u, dscal));
        if (!c.have_load) return read_scalar(dscal, e);
        TRY(launch_dot64(c.stream, ws, n, c.fext, u, dscal + 3));
        TRY(hipMemcpyAsync(h_scal, dscal, 4 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        TRY(hipStreamSynchronize(c.stream));
        e = h_scal[0] - load_s * h_scal[3];
        return EFEM_OK;
    }

    // its gradient over the free DOFs: r = (grad Psi_h(u) - s f)_free
    hipError_t residual(const double *u)
    {
        hipError_t e = launch_residual(c, u, r);
        if (e != hipSuccess || !c.have_load) return e;
        return launch_sub_load(c.stream, n, r, c.fext, load_s, c.m.nmask);
    }

    int norm(const double *v, double &out)
    {
        TRY(launch_dot64(c.stream, ws, n, v, v, dscal + 1));
        int rc = read_scalar(dscal + 1, out);
        out = std::sqrt(out);
        return rc;
    }

    int linearize(const double *u)
    {
        if (std::is_same<T, double>::value) TRY(launch_lin_record(c, u, c.xlin));
        else TRY(launch_cast_f32(u, c.ulin, n, c.stream));
        c.lin_prec = std::is_same<T, double>::value ? EFEM_F64 : EFEM_F32;
        return EFEM_OK;
    }

    // The single-launch form: under the halo and colour scatters it writes
    // every entry of q; under the atomic scatter it adds into a q that the
    // CG init/update kernels have cleared (clear_q)
    hipError_t hvp_acc(const T *v, T *y, const int32_t *skip)
    {
        if constexpr (std::is_same<T, double>::value)
            return launch_hvp_f64(c, c.xlin, v, y, skip, WriteMode::Zeroed);
        else
            return launch_hvp_f32(c, c.ulin, v, y, skip, WriteMode::Zeroed);
    }

    // Jacobi-PCG for K_ff x = sign * b from x = 0; dinv must be set.
    int pcg(const double *b, double sign, double eta, int max_it, int &iters)
    {
        TRY(L.init(b, sign, dinv, c.m.nmask, x, rv, p, q, sc, eta * eta));
        const int every = std::max(1, o.check_every);
        int j = 0;
        for (;;) {
            for (int k = 0; k < every; ++k, ++j) {
                TRY(hvp_acc(p, q, &sc->done));
                TRY(L.pq(p, q, sc));
                TRY(L.update(x, rv, p, q, dinv, sc, j));
                TRY(L.dir(p, rv, dinv, sc, j));
            }
            TRY(hipMemcpyAsync(h_sc, sc, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
            TRY(hipStreamSynchronize(c.stream));
            if (h_sc->done || h_sc->iter >= max_it) break;
        }
        iters = h_sc->iter + (h_sc->breakdown ? 1 : 0);
        if (h_sc->breakdown && h_sc->iter == 0) TRY(L.scaled(dinv, b, sign, x));
        return EFEM_OK;
    }

    // Flexible CG with the learned preconditioner for K_ff x = sign * b from
    // x = 0.  On breakdown, non-positive r.z or stagnation it falls back to
    // Jacobi PCG, and after learned_iters iterations (if set) it hands over to
    // it.  Jacobi PCG continues from the flexible-CG iterate when that is
    // finite (K d = r for its residual r, to the original tolerance, then
    // x += d), else starts again from x = 0.
    int fcg(const double *b, double sign, double eta, int max_it, int &iters, int &fallbacks)
    {
        MlpState &M = *static_cast<MlpState *>(c.mlp);
        FcgLaunch<float> F{n, c.stream, ws};
        F.clear_q = c.scatter == Scatter::Atomic;
        const int nz = mlp_apply_grid(c.n_nodes);
        TRY(L.init(b, sign, dinv, c.m.nmask, x, rv, p, q, sc, eta * eta));
        TRY(mlp_precondition(c, M, rv, M.z));
        TRY(F.start(M.z, p, sc, M.prz, nz));
        const int every = std::max(1, o.check_every);
        int j = 0;
        for (;;) {
            for (int k = 0; k < every; ++k, ++j) {
                TRY(hvp_acc(p, q, &sc->done));
                TRY(L.pq(p, q, sc));
                TRY(F.update(x, rv, p, q, M.z, sc, j));
                TRY(mlp_precondition(c, M, rv, M.z));
                TRY(F.dir(p, M.z, sc, M.prz, nz, j, kStallLimit));
            }
            TRY(hipMemcpyAsync(h_sc, sc, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
            TRY(hipStreamSynchronize(c.stream));
            if (h_sc->done || h_sc->iter >= max_it) break;
            if (o.learned_iters > 0 && h_sc->iter >= o.learned_iters) break;
        }
        iters = h_sc->iter;
        const bool capped = !h_sc->done && iters < max_it;
        if (h_sc->fallback || capped) {
            if (h_sc->fallback) fallbacks += 1;
            int it2 = 0, rc;
            // the flexible-CG residual as the new right-hand side (diag is
            // free here: the features are built and dinv is set)
            const double bnorm = std::sqrt(h_sc->bb);
            double rnorm = 0.0;
            TRY(L.widen(rv, diag));
            if ((rc = norm(diag, rnorm))) return rc;
            if (std::isfinite(rnorm) && rnorm > 0.0 && bnorm > 0.0 && iters > 0) {
                TRY(hipMemcpyAsync(M.zold, x, n * sizeof(T), hipMemcpyDeviceToDevice, c.stream));
                rc = pcg(diag, 1.0, eta * bnorm / rnorm, std::max(1, max_it - iters), it2);
                if (rc) return rc;
                TRY(L.add_to(x, reinterpret_cast<const T *>(M.zold)));
            } else {
                rc = pcg(b, sign, eta, max_it, it2);
                if (rc) return rc;
            }
            iters += it2;
        }
        return EFEM_OK;
    }

    // the Jacobi diagonal at u (and with precond = 2 the inverses of the
    // nodes' 3x3 diagonal blocks, which PCG then applies instead)
    int set_dinv(const double *u)
    {
        TRY(launch_diag(c, u, diag));
        TRY(L.dinv_from_diag(diag, c.m.nmask, dinv));
        L.binv = nullptr;
        if (o.precond == 2) {
            TRY(launch_offdiag(c, u, off));
            TRY(launch_block_inv(c.stream, c.n_nodes, diag, off, c.m.nmask, binv));
            L.binv = binv;
        }
        return EFEM_OK;
    }

    // K(u)_ff x = sign * b
    int linear_solve(const double *u, const double *b, double eta, int max_it, int &iters,
                     int &fallbacks, double sign = -1.0)
    {
        int rc;
        if ((rc = set_dinv(u)) || (rc = linearize(u))) return rc;
        if constexpr (std::is_same<T, float>::value) {
            auto *M = static_cast<MlpState *>(c.mlp);
            if (o.precond == 1 && M && M->have_weights) {
                TRY(mlp_prepare(c, *M, diag));
                return fcg(b, sign, eta, max_it, iters, fallbacks);
            }
        }
        return pcg(b, sign, eta, max_it, iters);
    }

    // Jacobi-PCG on K(u)_ff x = sign b from x = 0, keeping the CG residual after
    // its[k] iterations in R + k n (ascending its); returns how many were
    // reached before CG stopped (later ones repeat the last residual).
    int snapshots(const double *u, const double *b, double sign, int nsnap, const int32_t *its,
                  T *R, int32_t *taken)
    {
        int rc = setup();
        if (rc) return rc;
        if ((rc = set_dinv(u)) || (rc = linearize(u))) return rc;
        TRY(L.init(b, sign, dinv, c.m.nmask, x, rv, p, q, sc, 0.0));
        int k = 0;
        for (int j = 0;; ++j) {
            while (k < nsnap && its[k] == j) {
                TRY(hipMemcpyAsync(R + (int64_t)k * n, rv, n * sizeof(T), hipMemcpyDeviceToDevice,
                                   c.stream));
                ++k;
            }
            if (k == nsnap) break;
            TRY(hvp_acc(p, q, &sc->done));
            TRY(L.pq(p, q, sc));
            TRY(L.update(x, rv, p, q, dinv, sc, j));
            TRY(L.dir(p, rv, dinv, sc, j));
        }
        TRY(hipMemcpyAsync(h_sc, sc, sizeof(CgScalars), hipMemcpyDeviceToHost, c.stream));
        TRY(hipStreamSynchronize(c.stream));
        int got = 0;
        for (int i = 0; i < nsnap; ++i)
            if (!h_sc->done || its[i] <= h_sc->iter) ++got;
        *taken = got;
        return EFEM_OK;
    }

    // K(u)_ff xout = b, FP64 result
    int solve_into(const double *u, const double *b, double rtol, int max_it, double *xout,
                   int32_t *iters, int32_t *fb)
    {
        int rc = setup();
        if (rc) return rc;
        int it = 0, f = 0;
        if ((rc = linear_solve(u, b, rtol, max_it, it, f, +1.0))) return rc;
        TRY(hipMemsetAsync(xout, 0, n * sizeof(double), c.stream));
        TRY(L.axpy_state(xout, 1.0, x, xout));
        TRY(hipStreamSynchronize(c.stream));
        if (iters) *iters = it;
        if (fb) *fb = f;
        return EFEM_OK;
    }

    int run(double *u, const double *u_bc, efem_solve_stats *st)
    {
        int rc = setup();
        if (rc) return rc;
        const auto t0 = std::chrono::steady_clock::now();
        const bool f32 = std::is_same<T, float>::value;
        const double eta_min = f32 ? std::max(o.eta_min, 1e-5) : o.eta_min;
        st->converged = 1;
        for (int k = 1; k <= o.n_steps; ++k) {
            const double frac = (double)k / o.n_steps, dload = frac - load_s;
            load_s = frac;
            int cg_step = 0, nit = 0, fb = 0;
            // tangent predictor: K_ff d_f = (dload f - K dc)_f, with K dc taken on the
            // unmasked input
            TRY(launch_bc_increment(c.stream, n, u, u_bc, frac, c.m.nmask, dc, u_old));
            TRY(launch_lin_record(c, u, c.xlin));
            const uint8_t *mask = c.m.nmask;
            c.m.nmask = nullptr;
            hipError_t he = launch_hvp_f64(c, c.xlin, dc, kdc, nullptr, WriteMode::Overwrite);
            c.m.nmask = mask;
            TRY(he);
            if (c.have_load) TRY(launch_sub_load(c.stream, n, kdc, c.fext, dload, nullptr));
            int it = 0;
            if ((rc = linear_solve(u, kdc, o.predictor_rtol, o.max_cg, it, fb))) return rc;
            cg_step += it;
            TRY(L.apply_predictor(u_old, dc, x, c.m.nmask, true, u));
            double e0;
            if ((rc = energy(u, e0))) return rc;
            if (!std::isfinite(e0)) {
                TRY(L.apply_predictor(u_old, dc, x, c.m.nmask, false, u));
                if ((rc = energy(u, e0))) return rc;
                if (!std::isfinite(e0)) {
                    set_error("efem_newton_solve: the load increment inverts an element");
                    return EFEM_ERR_INVERTED;
                }
            }
            double rho;
            TRY(residual(u));
            if ((rc = norm(r, rho))) return rc;
            const double rho0 = rho;
            const double tol = std::max(o.rtol * rho0, o.atol_floor * std::max(1.0, rho0));
            double eta_prev = o.eta_max, rho_prev = -1.0;
            while (rho > tol) {
                if (nit >= o.max_newton) {
                    st->converged = 0;
                    break;
                }
                double eta;
                if (o.eta_fixed > 0) eta = o.eta_fixed;
                else if (rho_prev < 0) eta = o.eta_max;
                else {
                    eta = o.ew_gamma * std::pow(rho / rho_prev, o.ew_alpha);
                    const double safe = o.ew_gamma * std::pow(eta_prev, o.ew_alpha);
                    if (safe > 0.1) eta = std::max(eta, safe);
                    eta = std::min(eta, o.eta_max);
                    eta = std::max(eta, 0.5 * tol / rho);
                }
                if (o.eta_fixed <= 0) eta = std::max(eta, eta_min);
                if ((rc = linear_solve(u, r, eta, o.max_cg, it, fb))) return rc;
                cg_step += it;
                double slope;
                TRY(L.dot_state(r, x, dscal + 2));
                if ((rc = read_scalar(dscal + 2, slope))) return rc;
                double alpha = 1.0, e1 = INFINITY;
                int h = 0;
                for (; h <= o.max_halvings; ++h) {
                    TRY(L.axpy_state(u, alpha, x, u_trial));
                    if ((rc = energy(u_trial, e1))) return rc;
                    // sufficient decrease, up to the rounding of the FP64 energy sum: near the
                    // solution the decrease falls below eps |Psi| and cannot be resolved
                    const double noise = 64.0 * 2.220446049250313e-16 * std::fabs(e0);
                    if (std::isfinite(e1) && e1 <= e0 + o.armijo_c * alpha * slope + noise) break;
                    alpha *= 0.5;
                }
                if (h > o.max_halvings) {
                    st->converged = 0;
                    break;
                }
                st->line_search_halvings += h;
                TRY(hipMemcpyAsync(u, u_trial, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
                e0 = e1;
                rho_prev = rho;
                eta_prev = eta;
                TRY(residual(u));
                if ((rc = norm(r, rho))) return rc;
                ++nit;
                if (o.verbose)
                    std::fprintf(stderr, "[newton] step %d it %d |r| %.3e (rel %.3e) eta %.2e cg %d alpha %g\n",
                                 k, nit, rho, rho / rho0, eta, it, alpha);
            }
            st->steps_done = k;
            st->newton_iters += nit;
            st->cg_iters += cg_step;
            st->precond_fallbacks += fb;
            if (k - 1 < 64) {
                st->newton_per_step[k - 1] = nit;
                st->cg_per_step[k - 1] = cg_step;
            }
            st->final_residual = rho;
            st->final_energy = e0;
            if (!st->converged) break;
        }
        TRY(hipMemsetAsync(c.flags, 0, sizeof(int32_t), c.stream));
        TRY(hipStreamSynchronize(c.stream));
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return st->converged ? EFEM_OK : EFEM_NOT_CONVERGED;
    }
};

}  // namespace
}  // namespace efem

using namespace efem;

struct efem_ctx : Ctx {};

extern "C" {

void efem_solve_opts_default(efem_solve_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_steps = 5;
    o->hvp_prec = EFEM_F64;
    o->precond = 0;
    o->max_newton = 50;
    o->max_cg = 20000;
    o->check_every = 8;
    o->rtol = 1e-8;
    o->atol_floor = 1e-14;
    o->eta_max = 0.5;
    o->eta_min = 1e-10;
    o->ew_gamma = 0.9;
    o->ew_alpha = 2.0;
    o->eta_fixed = 0.0;
    o->predictor_rtol = 1e-4;
    o->armijo_c = 1e-4;
    o->max_halvings = 30;
    o->verbose = 0;
    o->learned_iters = 8;
}

int efem_newton_solve(efem_ctx *ctx, double *u_inout, const double *u_bc, const efem_solve_opts *opts,
                      efem_solve_stats *stats)
{
    if (!ctx || !u_inout || !u_bc || !opts || !stats) {
        set_error("efem_newton_solve: null pointer");
        return EFEM_ERR_INVALID;
    }
    if (!ctx->m.nmask) {
        set_error("efem_newton_solve: set a Dirichlet mask first (efem_set_dirichlet)");
        return EFEM_ERR_STATE;
    }
    if (ctx->model == EFEM_MODEL_TRANSPORT) {
        set_error("efem_newton_solve: the transport model has no energy; use efem_gmres_solve");
        return EFEM_ERR_STATE;
    }
    if (opts->n_steps < 1 || opts->max_cg < 1 || opts->max_newton < 0 || opts->rtol <= 0
        || (opts->hvp_prec != EFEM_F64 && opts->hvp_prec != EFEM_F32) || opts->precond < 0 || opts->precond > 2) {
        set_error("efem_newton_solve: bad options");
        return EFEM_ERR_INVALID;
    }
    if (opts->precond == 1 && (!ctx->mlp || !static_cast<MlpState *>(ctx->mlp)->have_weights
                               || opts->hvp_prec != EFEM_F32)) {
        set_error("efem_newton_solve: the learned preconditioner needs efem_set_mlp and EFEM_F32");
        return EFEM_ERR_STATE;
    }
    std::memset(stats, 0, sizeof(*stats));
    int dev_prev = -1;
    (void)hipGetDevice(&dev_prev);
    if (dev_prev != ctx->device) (void)hipSetDevice(ctx->device);
    int rc;
    if (opts->hvp_prec == EFEM_F64) {
        Solver<double> s(*ctx, *opts);
        rc = s.run(u_inout, u_bc, stats);
    } else {
        Solver<float> s(*ctx, *opts);
        rc = s.run(u_inout, u_bc, stats);
    }
    if (dev_prev >= 0 && dev_prev != ctx->device) (void)hipSetDevice(dev_prev);
    return rc;
}

}  // extern "C"

extern "C" int efem_linear_solve(efem_ctx *ctx, const double *u, const double *b, double *x,
                                 double rtol, int32_t hvp_prec, int32_t precond, int32_t max_iter,
                                 int32_t *iters, int32_t *fallback)
{
    if (!ctx || !u || !b || !x || !(rtol > 0) || max_iter < 1
        || (hvp_prec != EFEM_F64 && hvp_prec != EFEM_F32) || precond < 0 || precond > 2) {
        set_error("efem_linear_solve: bad argument");
        return EFEM_ERR_INVALID;
    }
    if (!ctx->m.nmask) {
        set_error("efem_linear_solve: set a Dirichlet mask first (efem_set_dirichlet)");
        return EFEM_ERR_STATE;
    }
    if (ctx->model == EFEM_MODEL_TRANSPORT) {
        set_error("efem_linear_solve: CG needs a symmetric tangent; use efem_gmres_solve");
        return EFEM_ERR_STATE;
    }
    if (precond == 1) {
        auto *M = static_cast<MlpState *>(ctx->mlp);
        if (!M || !M->have_weights || hvp_prec != EFEM_F32) {
            set_error("efem_linear_solve: the learned preconditioner needs efem_set_mlp and EFEM_F32");
            return EFEM_ERR_STATE;
        }
    }
    efem_solve_opts o;
    efem_solve_opts_default(&o);
    o.precond = precond;
    o.hvp_prec = hvp_prec;
    o.learned_iters = 0;   // the learned preconditioner alone, no hand-over
    int dev_prev = -1;
    (void)hipGetDevice(&dev_prev);
    if (dev_prev != ctx->device) (void)hipSetDevice(ctx->device);
    int rc;
    if (hvp_prec == EFEM_F64) {
        Solver<double> s(*ctx, o);
        rc = s.solve_into(u, b, rtol, max_iter, x, iters, fallback);
    } else {
        Solver<float> s(*ctx, o);
        rc = s.solve_into(u, b, rtol, max_iter, x, iters, fallback);
    }
    if (dev_prev >= 0 && dev_prev != ctx->device) (void)hipSetDevice(dev_prev);
    return rc;
}

extern "C" int efem_cg_snapshots(efem_ctx *ctx, const double *u, const double *b, double sign,
                                 int32_t n_snap, const int32_t *iters, float *R, int32_t *taken)
{
    if (!ctx || !u || !b || !iters || !R || !taken || n_snap < 1 || !(sign == 1.0 || sign == -1.0)) {
        set_error("efem_cg_snapshots: bad argument");
        return EFEM_ERR_INVALID;
    }
    for (int k = 0; k < n_snap; ++k)
        if (iters[k] < 0 || iters[k] > 1000000 || (k > 0 && iters[k] < iters[k - 1])) {
            set_error("efem_cg_snapshots: iters must be ascending and in [0, 1e6]");
            return EFEM_ERR_INVALID;
        }
    if (!ctx->m.nmask) {
        set_error("efem_cg_snapshots: set a Dirichlet mask first (efem_set_dirichlet)");
        return EFEM_ERR_STATE;
    }
    if (ctx->model == EFEM_MODEL_TRANSPORT) {
        set_error("efem_cg_snapshots: CG needs a symmetric tangent");
        return EFEM_ERR_STATE;
    }
    efem_solve_opts o;
    efem_solve_opts_default(&o);
    o.hvp_prec = EFEM_F32;
    int dev_prev = -1;
    (void)hipGetDevice(&dev_prev);
    if (dev_prev != ctx->device) (void)hipSetDevice(ctx->device);
    Solver<float> s(*ctx, o);
    const int rc = s.snapshots(u, b, sign, n_snap, iters, R, taken);
    if (dev_prev >= 0 && dev_prev != ctx->device) (void)hipSetDevice(dev_prev);
    return rc;
}
