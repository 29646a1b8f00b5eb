/*
 * Plain FP64 CPU oracle of the energy-based FEM operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link or call this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code with the HIP library.
 *
 * What it computes is the plain definition of the discrete energy of Eq. (2)
 * of the paper and of its exact first and second derivatives, Eq. (1) and the
 * tangent action of Eq. (3).  The paper obtains these derivatives by automatic
 * differentiation, exact to rounding (Sec. 1); here they are written
 * out in closed form, element by element and quadrature point by quadrature
 * point, with no blocking, fusion or reordering:
 *
 *   Psi(u) = sum_e sum_q  w_q det J_e(xi_q) psi_e(F_eq)                 Eq. (2)
 *   J_e(xi) = sum_a X_a (x) dN_a/dxi,   grad N_a = J^-T dN_a/dxi
 *   F_eq    = I + sum_a u_a (x) grad N_a(xi_q)                     Alg. 1 step "Compute"
 *
 * Material (the paper names a compressible neo-Hookean law but elides its
 * formula, Sec. 6.1; the reading used here is the standard form):
 *   psi = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2,  J = det F
 *   P   = mu (F - F^-T) + lam ln J F^-T
 *   A_iJkL = dP_iJ/dF_kL = mu d_ik d_JL + lam Finv_Ji Finv_Lk
 *                          + (mu - lam ln J) Finv_Jk Finv_Li
 * The tangent action uses the explicit 81-entry A.  I_1 - 3 and ln J are
 * evaluated as 2 tr H + H:H and log1p(tr H + ((tr H)^2 - tr H^2)/2 + det H)
 * with H = F - I, which are the same quantities written without cancellation.
 *
 * Second material (model ORC_LINEAR): small-strain linear elasticity, the
 * density of the paper's linear-elastic example (Sec. 6.1), in 3D:
 *   eps = (H + H^T)/2,  psi = mu eps:eps + lam/2 (tr eps)^2
 *   P   = sigma = 2 mu eps + lam tr(eps) I
 *   A_iJkL = mu (d_ik d_JL + d_iL d_Jk) + lam d_iJ d_kL   (constant)
 * It has no det F condition; only det J <= 0 is an error.
 *
 * Every entry point takes the element type and the material model first.
 *
 * Elements: Tet4 with the one-point centroid rule (w = 1/6) and trilinear
 * Hex8 on [-1,1]^3 with the 2x2x2 Gauss rule (points +-1/sqrt 3, w = 1); the
 * paper leaves the rules unspecified (Eq. 2).  Tri3 (the 2D setup of Sec. 5):
 * linear triangles in the x-y plane with the centroid rule (w = 1/2) and unit
 * thickness, carried in the same three nodal components; with the
 * out-of-plane component held at zero this is plane strain.
 *
 * Assembly: every element writes its own contribution block in parallel
 * (OpenMP); the blocks are then summed serially in element order, so results
 * are bitwise identical for any thread count.  Energies are summed with
 * Neumaier compensation.
 *
 * Return codes: 0 ok, -1 bad argument, -4 an element with det J <= 0 or
 * det F <= 0 was met (energy is then +inf; other outputs are unspecified).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TET4 0
#define ORC_HEX8 1
#define ORC_TRI3 2

#define ORC_NEO_HOOKE 0
#define ORC_LINEAR 1

typedef struct {
    int nen;            /* nodes per element */
    int nq;             /* quadrature points */
    double w[8];        /* weights */
    double dN[8][8][3]; /* dN[q][a][J]: reference gradients at point q */
    double N[8][8];     /* N[q][a]: shape function values at point q */
    int planar;         /* 2D element in the x-y plane: unit thickness along z */
} rule_t;

static int make_rule(int type, rule_t *r)
{
    r->planar = 0;
    if (type == ORC_TRI3) {
        /* linear triangle N0 = 1 - xi - eta, N1 = xi, N2 = eta, one centroid
         * point of weight 1/2 (the reference area).  The third reference
         * direction is the thickness: no shape function varies along it and
         * qp_eval adds a unit z column to J, so J = [J_2D 0; 0 1], grad N has
         * no z part, and with u_z held at zero F = [F_2D 0; 0 1] (plane strain) */
        static const double g[3][3] = {{-1, -1, 0}, {1, 0, 0}, {0, 1, 0}};
        r->nen = 3;
        r->nq = 1;
        r->w[0] = 0.5;
        r->planar = 1;
        for (int a = 0; a < 3; ++a) {
            for (int J = 0; J < 3; ++J) r->dN[0][a][J] = g[a][J];
            r->N[0][a] = 1.0 / 3.0;
        }
        return 0;
    }
    if (type == ORC_TET4) {
        /* N0 = 1 - xi - eta - zeta, N1 = xi, N2 = eta, N3 = zeta */
        static const double g[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        r->nen = 4;
        r->nq = 1;
        r->w[0] = 1.0 / 6.0;
        for (int a = 0; a < 4; ++a) {
            for (int J = 0; J < 3; ++J) r->dN[0][a][J] = g[a][J];
            r->N[0][a] = 0.25;   /* the centroid xi = eta = zeta = 1/4 */
        }
        return 0;
    }
    if (type == ORC_HEX8) {
        /* N_a = 1/8 (1 + s_a xi)(1 + t_a eta)(1 + z_a zeta) */
        static const double c[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                       {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
        const double g = 1.0 / sqrt(3.0);
        r->nen = 8;
        r->nq = 8;
        int q = 0;
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i, ++q) {
                    double p[3] = {(2 * i - 1) * g, (2 * j - 1) * g, (2 * k - 1) * g};
                    r->w[q] = 1.0;
                    for (int a = 0; a < 8; ++a) {
                        double f0 = 1 + c[a][0] * p[0], f1 = 1 + c[a][1] * p[1], f2 = 1 + c[a][2] * p[2];
                        r->dN[q][a][0] = 0.125 * c[a][0] * f1 * f2;
                        r->dN[q][a][1] = 0.125 * f0 * c[a][1] * f2;
                        r->dN[q][a][2] = 0.125 * f0 * f1 * c[a][2];
                        r->N[q][a] = 0.125 * f0 * f1 * f2;
                    }
                }
        return 0;
    }
    return -1;
}

static double det3(const double M[3][3])
{
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
         - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
         + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

/* inverse via the adjugate; returns the determinant */
static double inv3(const double M[3][3], double Mi[3][3])
{
    double d = det3(M);
    Mi[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) / d;
    Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / d;
    Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / d;
    Mi[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) / d;
    Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / d;
    Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / d;
    Mi[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) / d;
    Mi[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / d;
    Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / d;
    return d;
}

/* Everything the operators need at one quadrature point of one element. */
typedef struct {
    double wdetJ;       /* w_q det J */
    double gN[8][3];    /* grad_X N_a */
    double F[3][3], Finv[3][3];
    double H[3][3];     /* F - I */
    double lnJ;
    double I1m3;        /* tr(F^T F) - 3 */
    double eps[3][3];   /* (H + H^T)/2 */
    double treps;
    int model;
    int ok;             /* det J > 0, and det F > 0 for the neo-Hookean model */
} qp_t;

static void qp_eval(const rule_t *r, int q, const double Xe[8][3], const double ue[8][3], int model,
                    qp_t *s)
{
    double Jm[3][3] = {{0}}, Ji[3][3];
    for (int a = 0; a < r->nen; ++a)
        for (int i = 0; i < 3; ++i)
            for (int J = 0; J < 3; ++J) Jm[i][J] += Xe[a][i] * r->dN[q][a][J];
    if (r->planar) Jm[2][2] += 1.0;   /* unit thickness */
    double detJ = inv3(Jm, Ji);
    s->ok = detJ > 0.0;
    s->wdetJ = r->w[q] * detJ;
    /* grad N_a = J^-T dN_a/dxi :  (grad N_a)_L = sum_J Ji[J][L] dN[a][J] */
    for (int a = 0; a < r->nen; ++a)
        for (int L = 0; L < 3; ++L) {
            double t = 0;
            for (int J = 0; J < 3; ++J) t += Ji[J][L] * r->dN[q][a][J];
            s->gN[a][L] = t;
        }
    for (int i = 0; i < 3; ++i)
        for (int L = 0; L < 3; ++L) {
            double t = 0;
            for (int a = 0; a < r->nen; ++a) t += ue[a][i] * s->gN[a][L];
            s->H[i][L] = t;
            s->F[i][L] = (i == L ? 1.0 : 0.0) + t;
        }
    const double (*H)[3] = (const double (*)[3])s->H;
    double trH = H[0][0] + H[1][1] + H[2][2];
    s->model = model;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s->eps[i][j] = 0.5 * (H[i][j] + H[j][i]);
    s->treps = trH;
    if (model == ORC_LINEAR) {
        s->lnJ = 0.0;
        s->I1m3 = 0.0;
        return;
    }
    double HH = 0, trH2 = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            HH += H[i][j] * H[i][j];
            trH2 += H[i][j] * H[j][i];
        }
    double Jm1 = trH + 0.5 * (trH * trH - trH2) + det3(H);   /* det(I+H) - 1 */
    s->I1m3 = 2.0 * trH + HH;
    if (!(1.0 + Jm1 > 0.0)) {
        s->ok = 0;
        s->lnJ = NAN;
        return;
    }
    s->lnJ = log1p(Jm1);
    inv3(s->F, s->Finv);
}

static double eps_dot(const qp_t *s)
{
    double t = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t += s->eps[i][j] * s->eps[i][j];
    return t;
}

/* dpsi/dmu and dpsi/dlam (psi is linear in both, for both models) */
static void psi_parts(const qp_t *s, double *dmu, double *dlam)
{
    if (s->model == ORC_LINEAR) {
        *dmu = eps_dot(s);
        *dlam = 0.5 * s->treps * s->treps;
    } else {
        *dmu = 0.5 * s->I1m3 - s->lnJ;
        *dlam = 0.5 * s->lnJ * s->lnJ;
    }
}

static double psi_of(const qp_t *s, double mu, double lam)
{
    double pm, pl;
    psi_parts(s, &pm, &pl);
    return mu * pm + lam * pl;
}

/* dP/dmu and dP/dlam (P is linear in both):
 *   neo-Hookean: F - F^-T and ln J F^-T;   linear: 2 eps and tr(eps) I */
static void piola_parts(const qp_t *s, double Pm[3][3], double Pl[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int J = 0; J < 3; ++J) {
            if (s->model == ORC_LINEAR) {
                Pm[i][J] = 2.0 * s->eps[i][J];
                Pl[i][J] = i == J ? s->treps : 0.0;
            } else {
                Pm[i][J] = s->F[i][J] - s->Finv[J][i];
                Pl[i][J] = s->lnJ * s->Finv[J][i];
            }
        }
}

/* first Piola-Kirchhoff stress P = mu dP/dmu + lam dP/dlam:
 * neo-Hookean mu (F - F^-T) + lam lnJ F^-T, linear sigma */
static void piola(const qp_t *s, double mu, double lam, double P[3][3])
{
    double Pm[3][3], Pl[3][3];
    piola_parts(s, Pm, Pl);
    for (int i = 0; i < 3; ++i)
        for (int J = 0; J < 3; ++J) P[i][J] = mu * Pm[i][J] + lam * Pl[i][J];
}

/* explicit tangent A_iJkL = dP_iJ / dF_kL */
static void tangent(const qp_t *s, double mu, double lam, double A[3][3][3][3])
{
    if (s->model == ORC_LINEAR) {
        for (int i = 0; i < 3; ++i)
            for (int J = 0; J < 3; ++J)
                for (int k = 0; k < 3; ++k)
                    for (int L = 0; L < 3; ++L)
                        A[i][J][k][L] = mu * ((i == k && J == L ? 1.0 : 0.0) + (i == L && J == k ? 1.0 : 0.0))
                                      + (i == J && k == L ? lam : 0.0);
        return;
    }
    const double (*Fi)[3] = (const double (*)[3])s->Finv;
    double c = mu - lam * s->lnJ;
    for (int i = 0; i < 3; ++i)
        for (int J = 0; J < 3; ++J)
            for (int k = 0; k < 3; ++k)
                for (int L = 0; L < 3; ++L)
                    A[i][J][k][L] = (i == k && J == L ? mu : 0.0) + lam * Fi[J][i] * Fi[L][k]
                                  + c * Fi[J][k] * Fi[L][i];
}

static void gather(const rule_t *r, const double *V, const int32_t *ce, double out[8][3])
{
    for (int a = 0; a < r->nen; ++a)
        for (int i = 0; i < 3; ++i) out[a][i] = V[3 * (int64_t)ce[a] + i];
}

/* serial scatter of per-element blocks [ne][nen][3] into out [nn][3], element order */
static void scatter_blocks(const rule_t *r, int64_t nn, int64_t ne, const int32_t *conn,
                           const double *blk, double *out)
{
    memset(out, 0, sizeof(double) * 3 * (size_t)nn);
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < r->nen; ++a)
            for (int i = 0; i < 3; ++i)
                out[3 * (int64_t)conn[e * r->nen + a] + i] += blk[(e * r->nen + a) * 3 + i];
}

static int check_args(int type, int model, int64_t nn, int64_t ne, const int32_t *conn, rule_t *r)
{
    if (make_rule(type, r) != 0 || nn <= 0 || ne < 0) return -1;
    if (model != ORC_NEO_HOOKE && model != ORC_LINEAR) return -1;
    for (int64_t k = 0; k < ne * r->nen; ++k)
        if (conn[k] < 0 || conn[k] >= nn) return -1;
    return 0;
}

/* ------------------------------------------------------------------ energy */

/* Per-element energies psi_e [ne] and their compensated sum (Eq. 2). */
int orc_energy(int type, int model, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
               const double *mu, const double *lam, const double *u, double *psi_e, double *total)
{
    rule_t r;
    if (check_args(type, model, nn, ne, conn, &r)) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ue[8][3];
        gather(&r, X, conn + e * r.nen, Xe);
        gather(&r, u, conn + e * r.nen, ue);
        double pe = 0;
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, ue, model, &s);
            if (!s.ok) { bad = 1; pe = INFINITY; break; }
            pe += s.wdetJ * psi_of(&s, mu[e], lam[e]);
        }
        psi_e[e] = pe;
    }
    /* Neumaier summation in element order */
    double sum = 0, comp = 0;
    for (int64_t e = 0; e < ne; ++e) {
        double t = sum + psi_e[e];
        if (fabs(sum) >= fabs(psi_e[e])) comp += (sum - t) + psi_e[e];
        else comp += (psi_e[e] - t) + sum;
        sum = t;
    }
    *total = bad ? INFINITY : sum + comp;
    return bad ? -4 : 0;
}

/* --------------------------------------------------------------- residual */

/* r_{a,i} = sum_e sum_q w detJ P_iJ grad_J N_a        (Eq. 1, r = grad Psi) */
int orc_residual(int type, int model, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                 const double *mu, const double *lam, const double *u, double *res)
{
    rule_t r;
    if (check_args(type, model, nn, ne, conn, &r)) return -1;
    double *blk = (double *)calloc((size_t)(ne * r.nen * 3 + 1), sizeof(double));
    if (!blk) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ue[8][3], P[3][3];
        gather(&r, X, conn + e * r.nen, Xe);
        gather(&r, u, conn + e * r.nen, ue);
        double *f = blk + e * r.nen * 3;
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, ue, model, &s);
            if (!s.ok) { bad = 1; break; }
            piola(&s, mu[e], lam[e], P);
            for (int a = 0; a < r.nen; ++a)
                for (int i = 0; i < 3; ++i) {
                    double t = 0;
                    for (int J = 0; J < 3; ++J) t += P[i][J] * s.gN[a][J];
                    f[a * 3 + i] += s.wdetJ * t;
                }
        }
    }
    scatter_blocks(&r, nn, ne, conn, blk, res);
    free(blk);
    return bad ? -4 : 0;
}

/* -------------------------------------------------------------------- hvp */

/* (K v)_{a,i} = sum_e sum_q w detJ A_iJkL (sum_b v_bk grad_L N_b) grad_J N_a   (Eq. 3) */
int orc_hvp(int type, int model, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
            const double *mu, const double *lam, const double *u, const double *v, double *y)
{
    rule_t r;
    if (check_args(type, model, nn, ne, conn, &r)) return -1;
    double *blk = (double *)calloc((size_t)(ne * r.nen * 3 + 1), sizeof(double));
    if (!blk) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ue[8][3], ve[8][3], A[3][3][3][3];
        gather(&r, X, conn + e * r.nen, Xe);
        gather(&r, u, conn + e * r.nen, ue);
        gather(&r, v, conn + e * r.nen, ve);
        double *f = blk + e * r.nen * 3;
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, ue, model, &s);
            if (!s.ok) { bad = 1; break; }
            tangent(&s, mu[e], lam[e], A);
            double dF[3][3], dP[3][3];
            for (int k = 0; k < 3; ++k)
                for (int L = 0; L < 3; ++L) {
                    double t = 0;
                    for (int b = 0; b < r.nen; ++b) t += ve[b][k] * s.gN[b][L];
                    dF[k][L] = t;
                }
            for (int i = 0; i < 3; ++i)
                for (int J = 0; J < 3; ++J) {
                    double t = 0;
                    for (int k = 0; k < 3; ++k)
                        for (int L = 0; L < 3; ++L) t += A[i][J][k][L] * dF[k][L];
                    dP[i][J] = t;
                }
            for (int a = 0; a < r.nen; ++a)
                for (int i = 0; i < 3; ++i) {
                    double t = 0;
                    for (int J = 0; J < 3; ++J) t += dP[i][J] * s.gN[a][J];
                    f[a * 3 + i] += s.wdetJ * t;
                }
        }
    }
    scatter_blocks(&r, nn, ne, conn, blk, y);
    free(blk);
    return bad ? -4 : 0;
}

/* ------------------------------------------------------- element tangents */

/* Element tangent matrices, the matrix form of Eq. (3):
 *   K_e[(a,i),(b,k)] = sum_q w detJ sum_{J,L} A_iJkL grad_J N_a grad_L N_b
 * written to Ke [ne][nen*3][nen*3] (row (a,i) = 3a + i).  The global tangent
 * is their sum over the connectivity; its sparsity pattern is the node 1-ring
 * in 3x3 blocks.  Used to check the colouring-based sparse assembly. */
int orc_element_tangents(int type, int model, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                         const double *mu, const double *lam, const double *u, double *Ke)
{
    rule_t r;
    if (check_args(type, model, nn, ne, conn, &r)) return -1;
    const int m = r.nen * 3;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ue[8][3], A[3][3][3][3];
        gather(&r, X, conn + e * r.nen, Xe);
        gather(&r, u, conn + e * r.nen, ue);
        double *K = Ke + e * (int64_t)m * m;
        memset(K, 0, sizeof(double) * (size_t)(m * m));
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, ue, model, &s);
            if (!s.ok) { bad = 1; break; }
            tangent(&s, mu[e], lam[e], A);
            for (int a = 0; a < r.nen; ++a)
                for (int i = 0; i < 3; ++i)
                    for (int b = 0; b < r.nen; ++b)
                        for (int k = 0; k < 3; ++k) {
                            double t = 0;
                            for (int J = 0; J < 3; ++J)
                                for (int L = 0; L < 3; ++L)
                                    t += A[i][J][k][L] * s.gN[a][J] * s.gN[b][L];
                            K[(3 * a + i) * m + 3 * b + k] += s.wdetJ * t;
                        }
        }
    }
    return bad ? -4 : 0;
}

/* ----------------------------------------------------------- jacobi diag */

/* K_{(a,i),(a,i)} = sum_e sum_q w detJ sum_JL A_iJiL grad_J N_a grad_L N_a */
int orc_jacobi_diag(int type, int model, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                    const double *mu, const double *lam, const double *u, double *d)
{
    rule_t r;
    if (check_args(type, model, nn, ne, conn, &r)) return -1;
    double *blk = (double *)calloc((size_t)(ne * r.nen * 3 + 1), sizeof(double));
    if (!blk) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ue[8][3], A[3][3][3][3];
        gather(&r, X, conn + e * r.nen, Xe);
        gather(&r, u, conn + e * r.nen, ue);
        double *f = blk + e * r.nen * 3;
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, ue, model, &s);
            if (!s.ok) { bad = 1; break; }
            tangent(&s, mu[e], lam[e], A);
            for (int a = 0; a < r.nen; ++a)
                for (int i = 0; i < 3; ++i) {
                    double t = 0;
                    for (int J = 0; J < 3; ++J)
                        for (int L = 0; L < 3; ++L) t += A[i][J][i][L] * s.gN[a][J] * s.gN[a][L];
                    f[a * 3 + i] += s.wdetJ * t;
                }
        }
    }
    scatter_blocks(&r, nn, ne, conn, blk, d);
    free(blk);
    return bad ? -4 : 0;
}

/* ------------------------------------------------------ material adjoints */

/* dPsi/dmu_e = sum_q w detJ dpsi/dmu,  dPsi/dlam_e = sum_q w detJ dpsi/dlam:
 * neo-Hookean (tr C - 3)/2 - ln J and (ln J)^2 / 2; linear eps:eps and (tr eps)^2 / 2 */
int orc_grad_material(int type, int model, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                      const double *u, double *dmu, double *dlam)
{
    rule_t r;
    if (check_args(type, model, nn, ne, conn, &r)) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ue[8][3];
        gather(&r, X, conn + e * r.nen, Xe);
        gather(&r, u, conn + e * r.nen, ue);
        double gm = 0, gl = 0;
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, ue, model, &s);
            if (!s.ok) { bad = 1; break; }
            double pm, pl;
            psi_parts(&s, &pm, &pl);
            gm += s.wdetJ * pm;
            gl += s.wdetJ * pl;
        }
        dmu[e] = gm;
        dlam[e] = gl;
    }
    return bad ? -4 : 0;
}

/* w . dr/dmu_e = sum_q w detJ dP/dmu : grad w,   w . dr/dlam_e = sum_q w detJ dP/dlam : grad w */
int orc_residual_vjp_material(int type, int model, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                              const double *u, const double *wv, double *dmu, double *dlam)
{
    rule_t r;
    if (check_args(type, model, nn, ne, conn, &r)) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ue[8][3], we[8][3];
        gather(&r, X, conn + e * r.nen, Xe);
        gather(&r, u, conn + e * r.nen, ue);
        gather(&r, wv, conn + e * r.nen, we);
        double gm = 0, gl = 0;
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, ue, model, &s);
            if (!s.ok) { bad = 1; break; }
            double Pm[3][3], Pl[3][3];
            piola_parts(&s, Pm, Pl);
            for (int i = 0; i < 3; ++i)
                for (int J = 0; J < 3; ++J) {
                    double gw = 0;
                    for (int a = 0; a < r.nen; ++a) gw += we[a][i] * s.gN[a][J];
                    gm += s.wdetJ * Pm[i][J] * gw;
                    gl += s.wdetJ * Pl[i][J] * gw;
                }
        }
        dmu[e] = gm;
        dlam[e] = gl;
    }
    return bad ? -4 : 0;
}

/* ---------------------------------------------------- coordinate adjoint */

/* dPsi/dX_a (at fixed nodal u) = sum_e sum_q w detJ (psi I - H^T P) grad N_a */
int orc_grad_coords(int type, int model, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                    const double *mu, const double *lam, const double *u, double *gX)
{
    rule_t r;
    if (check_args(type, model, nn, ne, conn, &r)) return -1;
    double *blk = (double *)calloc((size_t)(ne * r.nen * 3 + 1), sizeof(double));
    if (!blk) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ue[8][3], P[3][3], S[3][3];
        gather(&r, X, conn + e * r.nen, Xe);
        gather(&r, u, conn + e * r.nen, ue);
        double *f = blk + e * r.nen * 3;
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, ue, model, &s);
            if (!s.ok) { bad = 1; break; }
            piola(&s, mu[e], lam[e], P);
            double psi = psi_of(&s, mu[e], lam[e]);
            for (int m = 0; m < 3; ++m)
                for (int L = 0; L < 3; ++L) {
                    double t = (m == L ? psi : 0.0);
                    for (int i = 0; i < 3; ++i) t -= s.H[i][m] * P[i][L];
                    S[m][L] = t;
                }
            for (int a = 0; a < r.nen; ++a)
                for (int m = 0; m < 3; ++m) {
                    double t = 0;
                    for (int L = 0; L < 3; ++L) t += S[m][L] * s.gN[a][L];
                    f[a * 3 + m] += s.wdetJ * t;
                }
        }
    }
    scatter_blocks(&r, nn, ne, conn, blk, gX);
    free(blk);
    return bad ? -4 : 0;
}

/* ------------------------------------------- non-variational transport */

/* The virtual-work form of Sec. 3.1 (Eqs. 4-6), for the advection-diffusion example's
 * weak form (steady, or one implicit time step with k = 1/dt), applied to
 * three species carried in the three nodal components s:
 *   W(c, v) = sum_s int [ D grad c_s . grad v_s + (b . grad c_s) v_s + k c_s v_s ]
 *   r = dW/dv:  r_{a,s} = sum_e sum_q w detJ [ D grad c_s . grad N_a
 *                                              + (b(x_q) . grad c_s + k c_s(x_q)) N_a ]
 * with b(x) = omega x x (a rigid rotation: divergence-free, as in the
 * example), D = D_e and k = k_e per element.  r is linear in c, so the tangent
 * K = dr/dc is constant and K v = r(v); the advection term makes it
 * non-symmetric.  With `Ke` non-null the element matrices
 * Ke[e][(a,s)][(b,t)] = dr_{a,s}/dc_{b,t} are written instead of r. */
static int transport(int type, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                     const double *D, const double *k, const double *omega, const double *c,
                     double *res, double *Ke)
{
    rule_t r;
    if (check_args(type, ORC_NEO_HOOKE, nn, ne, conn, &r)) return -1;
    const int m = 3 * r.nen;
    double *blk = NULL;
    if (!Ke) {
        blk = (double *)calloc((size_t)(ne * r.nen * 3 + 1), sizeof(double));
        if (!blk) return -1;
    }
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ce[8][3] = {{0}}, zero[8][3] = {{0}};
        gather(&r, X, conn + e * r.nen, Xe);
        if (c) gather(&r, c, conn + e * r.nen, ce);
        double *f = Ke ? NULL : blk + e * r.nen * 3;
        double *K = Ke ? Ke + e * (int64_t)m * m : NULL;
        if (K) memset(K, 0, sizeof(double) * (size_t)(m * m));
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, zero, ORC_LINEAR, &s);   /* geometry only */
            if (!s.ok) { bad = 1; break; }
            double xq[3] = {0, 0, 0};
            for (int a = 0; a < r.nen; ++a)
                for (int i = 0; i < 3; ++i) xq[i] += r.N[q][a] * Xe[a][i];
            const double b[3] = {omega[1] * xq[2] - omega[2] * xq[1], omega[2] * xq[0] - omega[0] * xq[2],
                                 omega[0] * xq[1] - omega[1] * xq[0]};
            if (K) {
                /* dr_{a,s}/dc_{b,s} = w detJ [D gN_a.gN_b + (b.gN_b) N_a + k N_b N_a] */
                for (int a = 0; a < r.nen; ++a)
                    for (int bb = 0; bb < r.nen; ++bb) {
                        double dd = 0, adv = 0;
                        for (int L = 0; L < 3; ++L) {
                            dd += s.gN[a][L] * s.gN[bb][L];
                            adv += b[L] * s.gN[bb][L];
                        }
                        const double kab = s.wdetJ * (D[e] * dd + adv * r.N[q][a] + k[e] * r.N[q][bb] * r.N[q][a]);
                        for (int sp = 0; sp < 3; ++sp) K[(3 * a + sp) * m + 3 * bb + sp] += kab;
                    }
                continue;
            }
            for (int sp = 0; sp < 3; ++sp) {
                double gc[3] = {0, 0, 0}, cq = 0;
                for (int a = 0; a < r.nen; ++a) {
                    cq += r.N[q][a] * ce[a][sp];
                    for (int L = 0; L < 3; ++L) gc[L] += ce[a][sp] * s.gN[a][L];
                }
                const double val = b[0] * gc[0] + b[1] * gc[1] + b[2] * gc[2] + k[e] * cq;
                for (int a = 0; a < r.nen; ++a) {
                    const double diff = gc[0] * s.gN[a][0] + gc[1] * s.gN[a][1] + gc[2] * s.gN[a][2];
                    f[a * 3 + sp] += s.wdetJ * (D[e] * diff + val * r.N[q][a]);
                }
            }
        }
    }
    if (!Ke) {
        scatter_blocks(&r, nn, ne, conn, blk, res);
        free(blk);
    }
    return bad ? -4 : 0;
}

int orc_transport_residual(int type, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                           const double *D, const double *k, const double *omega, const double *c,
                           double *res)
{
    if (!c || !res) return -1;
    return transport(type, nn, ne, X, conn, D, k, omega, c, res, NULL);
}

int orc_transport_tangents(int type, int64_t nn, int64_t ne, const double *X, const int32_t *conn,
                           const double *D, const double *k, const double *omega, double *Ke)
{
    if (!Ke) return -1;
    return transport(type, nn, ne, X, conn, D, k, omega, NULL, NULL, Ke);
}

/* Element volumes sum_q w detJ, for mesh checks.  Returns -4 if any det J <= 0. */
int orc_volumes(int type, int model, int64_t nn, int64_t ne, const double *X, const int32_t *conn, double *vol)
{
    rule_t r;
    if (check_args(type, model, nn, ne, conn, &r)) return -1;
    int bad = 0;
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[8][3], ue[8][3] = {{0}};
        gather(&r, X, conn + e * r.nen, Xe);
        double v = 0;
        for (int q = 0; q < r.nq; ++q) {
            qp_t s;
            qp_eval(&r, q, Xe, ue, model, &s);
            if (!s.ok) bad = 1;
            v += s.wdetJ;
        }
        vol[e] = v;
    }
    return bad ? -4 : 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
