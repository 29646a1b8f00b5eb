/*
 * efem.h -- C-ABI of the energy-based finite-element hot path for AMD MI355X
 * (gfx950): the global potential energy of a mesh, its gradient (the nodal
 * residual) and matrix-free tangent actions (Hessian-vector products), their
 * adjoints with respect to material fields and nodal coordinates, a
 * matrix-free Newton-Krylov solve built on them, the sparse tangent matrix by
 * colouring, and a learned CG preconditioner.
 *
 * The calls follow the paper's statement of the problem (arXiv 2602.12365):
 *   - an operator object built from a mesh, an element type and a batch
 *     (block) size, Sec. 4 (the geometric context of an operator);
 *   - the discrete energy Psi_h of a flat DOF vector, Eq. (2) and Alg. 1;
 *   - the residual r = grad Psi_h, Eq. (1);
 *   - the tangent action dr = K du, Eq. (3);
 *   - Dirichlet conditions as a reduced functional over the free DOFs, Sec. 6.1;
 *   - a matrix-free Newton-Krylov solve, Sec. 6.3.1;
 *   - the sparse tangent recovered from tangent actions by colouring, Alg. 2.
 *
 * Element types: 4-node tetrahedra with the one-point centroid rule, 8-node
 * trilinear hexahedra with the 2x2x2 Gauss rule, and linear triangles with
 * the centroid rule for the 2D setup (Sec. 5).  Triangles lie in the x-y
 * plane (counter-clockwise seen from +z) with unit thickness along z and use
 * the same three nodal components: the reference Jacobian is [J_2D 0; 0 1],
 * and with the z components held by the Dirichlet mask the model is plane
 * strain.  Material (per-element mu,
 * lam): compressible neo-Hookean, psi = mu/2 (tr F^T F - 3) - mu ln J +
 * lam/2 (ln J)^2 (Sec. 6.1), or small-strain linear elasticity, psi = mu
 * eps:eps + lam/2 (tr eps)^2 with eps = sym grad u (the density of the
 * paper's first example, Sec. 6.1), chosen with efem_set_model.
 *
 * Conventions (all calls):
 *   - Layout: nodal arrays are node-major interleaved, entry 3*node + comp
 *     (the reshape(-1, 3) of the flat DOF vector, Sec. 4).  Per-element arrays
 *     are indexed by the caller's element numbering.
 *   - Ownership: mesh arrays passed to efem_create are HOST pointers and are
 *     copied.  Every other array argument is a caller-owned DEVICE pointer
 *     (hipMalloc'd or a contiguous torch CUDA tensor) on the context's device;
 *     the library never frees it and does not keep it after the call returns,
 *     except where stated (efem_set_material copies, efem_linearize copies).
 *   - Streams: operator calls are asynchronous on the context's stream (set at
 *     creation or with efem_set_stream); results are ready when that stream
 *     reaches the point of the call.  Calls documented as synchronous wait.
 *   - Errors: functions return EFEM_OK (0), a warning (> 0) or an error (< 0);
 *     efem_last_error() gives a message for the calling thread.  No C++
 *     exception crosses this boundary.
 *   - Thread safety: a context may be used by one host thread and one stream
 *     at a time.  Distinct contexts are independent.
 */
#ifndef EFEM_H
#define EFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define EFEM_OK              0
#define EFEM_NOT_CONVERGED   1   /* newton_solve stopped at an iteration cap */
#define EFEM_ERR_INVALID    -1   /* bad argument: null pointer, size, index */
#define EFEM_ERR_HIP        -2   /* a HIP runtime call failed */
#define EFEM_ERR_OOM        -3   /* device or host allocation failed */
#define EFEM_ERR_INVERTED   -4   /* an element with det J <= 0 or det F <= 0 */
#define EFEM_ERR_STATE      -5   /* call out of order (e.g. hvp before linearize) */

/* element types */
#define EFEM_TET4 0
#define EFEM_HEX8 1
#define EFEM_TRI3 2   /* planar: triangles in the x-y plane, unit thickness */

/* material models (efem_set_model) */
#define EFEM_MODEL_NEO_HOOKE 0
#define EFEM_MODEL_LINEAR    1
#define EFEM_MODEL_TRANSPORT 2   /* non-variational: virtual work, no energy */

/* arithmetic of the tangent action */
#define EFEM_F64 0
#define EFEM_F32 1

/* how element contributions are summed into nodal vectors (within a block
 * always in LDS, with LDS atomics, so results vary in the last bits) */
#define EFEM_SCATTER_HALO   0   /* default: block sums of nodes shared between
                                   blocks are stored per (block, node) and a
                                   second kernel adds each node's entries in block
                                   order; no global atomics */
#define EFEM_SCATTER_COLOR  1   /* blocks coloured so that no two blocks of one
                                   colour share a node; one pass per colour */
#define EFEM_SCATTER_ATOMIC 2   /* global atomic adds on shared nodes (after a
                                   clearing fill of the output) */

typedef struct efem_ctx efem_ctx;

typedef struct {
    int32_t block_elems;   /* max elements per workgroup block (the paper's batch
                              size N_B, Alg. 1); 0 = default for the element type */
    int32_t block_nodes;   /* max distinct nodes per block (<= 768, so that two
                              blocks fit a CU's 160 KB of LDS); 0 = default */
    int32_t scatter;       /* EFEM_SCATTER_HALO (0, default), _COLOR or _ATOMIC */
    int32_t threads;       /* threads per workgroup (64..256, multiple of 64); 0 = default */
    int32_t no_pairs;      /* EFEM_TET4: nonzero = one tetrahedron per work item; by
                              default two tetrahedra that share a face form one item
                              (5 nodes instead of 8), which results do not depend on
                              beyond rounding */
    int32_t no_chunks;     /* EFEM_TET4, halo scatter: nonzero = the FP64 tangent
                              action runs block by block.  By default runs of
                              consecutive blocks form chunks whose nodes stay
                              resident in one workgroup's LDS (the whole 160 KB of
                              a CU) while the blocks stream through, the next
                              block's nodes loading during the current block's
                              arithmetic; a chunk's nodal sums leave LDS once */
} efem_options;

/* Build an operator for a mesh (Sec. 4, Operator(mesh, element, batchsize)).
 *   elem      EFEM_TET4, EFEM_HEX8 or EFEM_TRI3
 *   coords    HOST float64 [n_nodes*3] reference coordinates X
 *   conn      HOST int32 [n_elems*n_en] connectivity (4, 8 or 3 nodes, element-major;
 *             hexahedra in the order (0,0,0),(1,0,0),(1,1,0),(0,1,0), then z=1;
 *             triangles counter-clockwise seen from +z)
 *   opts      may be NULL (defaults)
 *   stream    hipStream_t to run on, NULL = the null stream
 * Elements are reordered internally along a Morton curve and cut into blocks
 * that each fit one workgroup's LDS.  The material is set to mu = 1, lam = 1.5
 * until efem_set_material is called.  Synchronous.
 * Errors: EFEM_ERR_INVALID on a null pointer, n_nodes < 1, n_elems < 1, a
 * connectivity entry outside [0, n_nodes) or a node that no element uses
 * (outputs are written by the element passes only); EFEM_ERR_INVERTED if an
 * element of the reference mesh has det J <= 0 at a quadrature point. */
int efem_create(efem_ctx **out, int32_t elem, int64_t n_nodes, int64_t n_elems,
                const double *coords, const int32_t *conn, const efem_options *opts,
                void *stream);

/* Release every device and host resource of the context.  Synchronizes its stream. */
void efem_destroy(efem_ctx *ctx);

/* Change the stream later calls run on. */
int efem_set_stream(efem_ctx *ctx, void *stream);

/* Per-element material (DEVICE float64 [n_elems] each, caller's element order).
 * Copied into the context; mu, lam must be finite.  Synchronous: a field that
 * is the same in every element is detected and kept as two scalars. */
int efem_set_material(efem_ctx *ctx, const double *mu, const double *lam);

/* Material model of the strain energy density: EFEM_MODEL_NEO_HOOKE (the
 * default) or EFEM_MODEL_LINEAR.  Every later operator call (energy,
 * residual, tangent action, diagonal, adjoints, solves, sparse tangent) uses
 * it.  Under the linear model the tangent does not depend on u, so the state
 * given to efem_linearize is not read by efem_hvp (linearize is still required
 * first), and there is no det F condition.
 *
 * EFEM_MODEL_TRANSPORT is the non-variational case of Sec. 3.1 (Eqs. 4-6): a virtual-work
 * functional W(c, v) instead of an energy, here the advection-diffusion
 * example's weak form (Sec. 6.5) (steady, or one implicit time step with k = 1/dt) for
 * three species carried in the three nodal components:
 *   r_{a,s}(c) = sum_e sum_q w det J [ D grad c_s . grad N_a
 *                                      + (b(x_q) . grad c_s + k c_s) N_a ]
 * with D = mu_e, k = lam_e (efem_set_material) and b(x) = omega x x
 * (efem_set_velocity).  efem_residual returns r(c), efem_hvp K v (K = dr/dc
 * is constant and non-symmetric), efem_jacobi_diag diag K, and
 * efem_gmres_solve solves with it.  There is no energy: efem_energy, the
 * material and coordinate adjoints, efem_newton_solve and the CG-based
 * solves return EFEM_ERR_STATE.  Returns EFEM_ERR_INVALID for an unknown
 * model. */
int efem_set_model(efem_ctx *ctx, int32_t model);

/* Rotation vector omega (HOST float64 [3]) of the transport model's
 * velocity b(x) = omega x x (divergence-free).  Default 0. */
int efem_set_velocity(efem_ctx *ctx, const double *omega);

/* Replace the reference coordinates (DEVICE float64 [3*n_nodes]) keeping the
 * connectivity and the element blocks (e.g. for derivatives with respect to X
 * by finite differences, or shape updates).  Copied; asynchronous.  The
 * positivity of the reference Jacobians is not re-checked: an inverted
 * reference element makes later results undefined. */
int efem_set_coords(efem_ctx *ctx, const double *coords);

/* Dirichlet mask (DEVICE uint8 [3*n_nodes], 1 = prescribed DOF), or NULL to
 * clear it.  With a mask set, the residual, the tangent action and the Jacobi
 * diagonal are those of the reduced functional over the free DOFs (Sec. 6.1):
 * prescribed entries of the output are 0 and prescribed entries of the
 * direction v are ignored.  The energy is unaffected (the prescribed values
 * are part of u).  Copied into the context. */
int efem_set_dirichlet(efem_ctx *ctx, const uint8_t *mask);

/* External nodal forces f (DEVICE float64 [3*n_nodes]) of the final load step,
 * or NULL to remove them.  The total potential energy of Sec. 6.1 subtracts
 * the work of a boundary traction t; for the linear boundary interpolation
 * that work is exactly f.u with f_a the integral of t N_a over the loaded
 * boundary, which the caller computes.  Only efem_newton_solve uses f: at
 * load step k of n it minimizes Psi_h(u) - (k/n) f.u.  efem_energy,
 * efem_residual and the tangent action stay those of Psi_h.  Entries of f on
 * prescribed DOFs have no effect on the solution.  Copied; asynchronous. */
int efem_set_load(efem_ctx *ctx, const double *f);

/* Psi_h(u), Eq. (2): u DEVICE float64 [3*n_nodes]; psi DEVICE float64 [1].
 * A block-wise then compensated FP64 sum, bitwise deterministic.  If an element
 * has det F <= 0 the result is +inf and the context's inverted flag is set
 * (see efem_status). */
int efem_energy(efem_ctx *ctx, const double *u, double *psi);

/* efem_energy for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bitwise, with the per-block partials in a
 * static device array of 65536 doubles (512 KiB) that each GPU the library
 * runs on holds until the process ends.  Allocates nothing and calls no
 * allocating routine.  Returns EFEM_ERR_INVALID if the mesh has more than
 * 65536 element blocks (efem_get_info n_blocks).  All calls on one GPU share
 * its array: calls that overlap in time on one GPU (other streams, other
 * threads or contexts) race and must be ordered by the caller.  Asynchronous
 * on the context's stream, like efem_energy. */
int efem_energy_noalloc(efem_ctx *ctx, const double *u, double *psi);

/* r = grad Psi_h(u), Eq. (1): u, r DEVICE float64 [3*n_nodes].  r must not
 * be u (EFEM_ERR_INVALID): the elements read u while nodal sums are stored. */
int efem_residual(efem_ctx *ctx, const double *u, double *r);

/* Fix the linearization point u (DEVICE float64 [3*n_nodes]) of efem_hvp and
 * its arithmetic prec (EFEM_F64 or EFEM_F32).  u is copied (rounded to float32
 * for EFEM_F32), so the caller may change u afterwards. */
int efem_linearize(efem_ctx *ctx, const double *u, int32_t prec);

/* y = K(u) v, Eq. (3), at the point of the last efem_linearize: v, y DEVICE
 * [3*n_nodes] of the linearize precision (float64 or float32).  y must not
 * alias v.  EFEM_ERR_STATE if efem_linearize was never called. */
int efem_hvp(efem_ctx *ctx, const void *v, void *y);

/* y += K(u) v, Eq. (3), in a single kernel launch (efem_hvp needs a second,
 * small launch to clear the entries that several blocks add into).  Same
 * arguments and errors as efem_hvp; prescribed entries of y are set to 0. */
int efem_hvp_acc(efem_ctx *ctx, const void *v, void *y);

/* y = K(u) v in a single launch for a y that holds zeros on entry (e.g. cleared
 * by the caller's preceding vector kernel, as the library's Krylov loop does);
 * the result is undefined if y is not zero.  Same arguments as efem_hvp. */
int efem_hvp_zeroed(efem_ctx *ctx, const void *v, void *y);

/* d = diag K(u), DEVICE float64 [3*n_nodes] (the Jacobi preconditioner);
 * with a Dirichlet mask, prescribed entries are 1. */
int efem_jacobi_diag(efem_ctx *ctx, const double *u, double *d);

/* The off-diagonal entries of every node's 3x3 diagonal block of K(u) (the
 * blocks of the block-Jacobi preconditioner, whose diagonals efem_jacobi_diag
 * gives): o DEVICE float64 [n_nodes][3] = (K01, K02, K12), the mask not
 * applied.  Neo-Hookean and linear models (EFEM_ERR_STATE for transport). */
int efem_jacobi_offdiag(efem_ctx *ctx, const double *u, double *o);

/* Adjoint with respect to the material at fixed u:
 *   dmu[e] = dPsi/dmu_e, dlam[e] = dPsi/dlam_e   (DEVICE float64 [n_elems]). */
int efem_grad_material(efem_ctx *ctx, const double *u, double *dmu, double *dlam);

/* Residual vector-Jacobian product with respect to the material at fixed u:
 *   dmu[e] = w . dr/dmu_e, dlam[e] = w . dr/dlam_e   (w DEVICE [3*n_nodes];
 *   outputs DEVICE float64 [n_elems]).  The Dirichlet mask is not applied. */
int efem_residual_vjp_material(efem_ctx *ctx, const double *u, const double *w,
                               double *dmu, double *dlam);

/* Adjoint with respect to the reference coordinates at fixed nodal u:
 *   dX = dPsi/dX, DEVICE float64 [3*n_nodes].  Uses the coordinates given to
 *   efem_create. */
int efem_grad_coords(efem_ctx *ctx, const double *u, double *dX);

/* Blocking statistics of a context (host values; synchronous). */
typedef struct {
    int32_t n_blocks;         /* workgroup element blocks */
    int32_t n_colours;        /* colour passes (EFEM_SCATTER_COLOR), else 0 */
    int32_t max_block_nodes;  /* largest per-block distinct node count */
    int32_t max_block_elems;
    int64_t n_shared_nodes;   /* nodes touched by more than one block */
    int64_t n_block_nodes;    /* sum over blocks of distinct nodes (>= n_nodes) */
    int64_t n_items;          /* work items: face-sharing tetrahedron pairs count once */
    int32_t n_chunks;         /* chunks of the FP64 Tet4 tangent action, 0 = block pass */
    int32_t max_chunk_slots;  /* largest per-chunk distinct node count (<= 1472) */
    int64_t n_chunk_slots;    /* sum over chunks of distinct nodes */
    int64_t n_chunk_shared_nodes; /* nodes touched by more than one chunk */
} efem_info;

int efem_get_info(efem_ctx *ctx, efem_info *info);

/* Read and clear the context's device flags (synchronizes the stream):
 * bit 0 = an element with det F <= 0 was met since the last call. */
int efem_status(efem_ctx *ctx, int32_t *flags);

/* ------------------------------------------------------------ Newton-Krylov */

typedef struct {
    int32_t n_steps;          /* load steps; prescribed values ramp as k/n_steps */
    int32_t hvp_prec;         /* EFEM_F64 or EFEM_F32 for the CG tangent actions */
    int32_t precond;          /* 0 = Jacobi, 1 = learned (efem_set_mlp) with Jacobi fallback,
                                 2 = 3x3 block Jacobi (the inverses of the nodes' diagonal
                                 blocks of K_ff, stored in bfloat16 and rebuilt at every
                                 linearization) */
    int32_t max_newton;       /* per load step */
    int32_t max_cg;           /* per linear solve */
    int32_t check_every;      /* CG iterations between host convergence checks (>= 1) */
    double rtol;              /* ||r_free|| <= rtol * ||r_free at step start|| */
    double atol_floor;        /* absolute floor, times max(1, ||r_free at step start||) */
    double eta_max, eta_min;  /* Eisenstat-Walker choice 2 forcing bounds */
    double ew_gamma, ew_alpha;
    double eta_fixed;         /* > 0: fixed forcing term instead of Eisenstat-Walker */
    double predictor_rtol;    /* tolerance of the tangent predictor of each load step */
    double armijo_c;          /* sufficient-decrease constant of the line search */
    int32_t max_halvings;
    int32_t verbose;          /* 0 silent, 1 one line per Newton iteration on stderr */
    int32_t learned_iters;    /* precond = 1: flexible-CG iterations with the learned
                                 preconditioner, after which a Krylov solve continues
                                 with Jacobi PCG from the flexible-CG iterate (default
                                 8; 0: no limit; rounded up to a multiple of
                                 check_every) */
} efem_solve_opts;

typedef struct {
    int32_t converged;        /* 1 if every load step met its tolerance */
    int32_t steps_done;
    int32_t newton_iters;     /* total */
    int32_t cg_iters;         /* total, including predictors */
    int32_t precond_fallbacks;/* learned-preconditioner solves restarted with Jacobi */
    int32_t line_search_halvings;
    double final_residual;    /* ||r_free|| at the end (FP64) */
    double final_energy;
    double seconds;           /* host wall time of the solve */
    int32_t newton_per_step[64];
    int32_t cg_per_step[64];
} efem_solve_stats;

/* Fill opts with the defaults (n_steps 5, FP64, Jacobi, rtol 1e-8,
 * learned_iters 8, ...). */
void efem_solve_opts_default(efem_solve_opts *opts);

/* Matrix-free Newton-Krylov solve of the reduced functional (Sec. 6.1,
 * Sec. 6.3.1).  Requires efem_set_dirichlet.
 *   u_inout   DEVICE float64 [3*n_nodes]: initial free values in, solution out
 *   u_bc      DEVICE float64 [3*n_nodes]: prescribed values of the final load
 *             step (entries on free DOFs are ignored)
 * Per load step: prescribed DOFs set to k/n of u_bc and the load of
 * efem_set_load to k/n of f, a tangent predictor, then Newton iterations with
 * PCG (Jacobi or learned), Eisenstat-Walker forcing and Armijo backtracking on
 * the FP64 total energy Psi_h(u) - (k/n) f.u.  final_energy reports that
 * total and final_residual the norm of its free gradient.  Synchronous.
 * Returns EFEM_OK, EFEM_NOT_CONVERGED (stats say where) or an error. */
int efem_newton_solve(efem_ctx *ctx, double *u_inout, const double *u_bc,
                      const efem_solve_opts *opts, efem_solve_stats *stats);

/* ------------------------------------------------- learned preconditioner */

/* Learned CG preconditioner (this project's addition to the method, used by
 * efem_newton_solve with precond = 1 and hvp_prec = EFEM_F32).  Per node i,
 * with N(i) the nodes sharing an element with i and D the Jacobi diagonal:
 *   g_i = D_i^-1 r_i (0 on prescribed DOFs), s_i = RMS of g over {i} + N(i),
 *   f_i = [g_i/s_i, mean_N(i) g/s_i, log(D_i/mean_{N(i)+i} D), prescribed
 *          fraction of i, of N(i), |N(i)|/26]                     (12 inputs)
 *   z_i = g_i + gamma_i s_i MLP(f_i), prescribed DOFs 0, where gamma_i = 1
 *         unless r_i.z_i would fall below r_i.g_i / 2; then gamma_i in [0, 1)
 *         makes it exactly half (so r.z >= r.D^-1 r / 2 > 0 for any network),
 * MLP 12 -> 64 -> 64 -> 3 with softplus hidden layers (the activation of the
 * paper's neural energy terms, Sec. 6.6.1), bfloat16 weights and layer inputs,
 * FP32 accumulation on the matrix cores.  z is positively homogeneous in r;
 * Krylov solves use flexible CG with Jacobi PCG as the fallback.
 * Parameters: FP32 vector of EFEM_MLP_PARAMS values, W1 [64][12], b1 [64],
 * W2 [64][64], b2 [64], W3 [3][64], b3 [3] (row-major, output index first). */
#define EFEM_MLP_IN     12
#define EFEM_MLP_HID    64
#define EFEM_MLP_OUT    3
#define EFEM_MLP_PARAMS 5187
#define EFEM_MLP_AUX    12   /* floats per training row */

/* Set the preconditioner's parameters (DEVICE float32 [EFEM_MLP_PARAMS],
 * rounded to bfloat16 and copied), or NULL to remove the network.  The first
 * call builds the node 1-ring graph (host work, synchronous). */
int efem_set_mlp(efem_ctx *ctx, const float *params);

/* z = M(r) (DEVICE float32 [3*n_nodes] each) with diag the Jacobi diagonal
 * (DEVICE float64 [3*n_nodes], as efem_jacobi_diag returns it) and the context's
 * Dirichlet mask.  EFEM_ERR_STATE without efem_set_mlp. */
int efem_precond_apply(efem_ctx *ctx, const float *r, const double *diag, float *z);

/* Training rows of one (right-hand side b, target t) pair, b and t DEVICE float32
 * [3*n_nodes], diag as above: X DEVICE uint16 (bfloat16) [n_nodes][16] (the 12
 * features, zero padded), aux DEVICE float32 [n_nodes][EFEM_MLP_AUX] =
 * [g(3), t(3), free-DOF flags(3), s, w, 0] with w = 1 / (|t|^2 n_total), so that
 * the loss of efem_mlp_loss_grad over all rows of n_total pairs is the mean over
 * pairs of |M(b) - t|^2 / |t|^2.  Needs the graph (efem_set_mlp called once). */
int efem_precond_rows(efem_ctx *ctx, const float *b, const double *diag, const float *t,
                      double n_total, uint16_t *X, float *aux);

/* out [rows][3] = MLP(X) on the matrix cores with the context's parameters. */
int efem_mlp_forward(efem_ctx *ctx, int64_t rows, const uint16_t *X, float *out);

/* The same forward pass with both hidden layers' activations as well: h1, h2
 * DEVICE uint16 (bfloat16 bits) [rows][EFEM_MLP_HID], h_k = bf16(softplus(
 * W_k h_{k-1} + b_k)) exactly as the next layer reads it; out as above.  For
 * checking the network layer by layer. */
int efem_mlp_forward_layers(efem_ctx *ctx, int64_t rows, const uint16_t *X, uint16_t *h1, uint16_t *h2,
                            float *out);

/* Loss sum_rows w |m (g + s MLP_params(X)) - m t|^2 and its gradient with respect
 * to params (DEVICE float32 [EFEM_MLP_PARAMS]) into grad (DEVICE float32
 * [EFEM_MLP_PARAMS], overwritten) and loss (DEVICE float64 [1]); forward and
 * backward on the vector units, the bfloat16 roundings of the forward treated
 * as identity in the backward pass.  Deterministic. */
int efem_mlp_loss_grad(efem_ctx *ctx, int64_t rows, const uint16_t *X, const float *aux,
                       const float *params, float *grad, double *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on DEVICE float32 params,
 * moments m, v and gradient g (all [EFEM_MLP_PARAMS]); t = step number >= 1. */
int efem_mlp_adam(efem_ctx *ctx, float *params, float *m, float *v, const float *g, float lr,
                  int32_t t);

/* Energy-norm training of the preconditioner, one sample (the objective is the
 * K-norm error of one preconditioned step, sum over samples of
 * w (z.Kz - 2 r.z) = w (|K^-1 r - z|_K^2 - |K^-1 r|_K^2), z = m (g + s MLP),
 * which needs no solves).  At the context's current FP32 linearization
 * (efem_linearize(u, EFEM_F32)) and Dirichlet mask, for a residual r (DEVICE
 * float32 [3*n_nodes]) whose rows efem_precond_rows built into aux, and the
 * network outputs out (DEVICE float32 [n_nodes][3], efem_mlp_forward of
 * those rows):
 *   z = m (g + s out)             -> z  (DEVICE float32 [3*n_nodes])
 *   K z                           -> kz (DEVICE float32 [3*n_nodes])
 *   w = 1 / (n_samples r.g)       -> aux[:, 10]
 *   t = (g + s out) - (K z - r)   -> aux[:, 3:6]
 *   energy += w (z.Kz - 2 r.z)    (DEVICE float64 scalar, accumulated)
 * With these t and w, efem_mlp_loss_grad over the rows returns the gradient of
 * the energy objective at the current parameters (its loss value is then
 * sum w |K z - r|^2 on free DOFs).  EFEM_ERR_STATE without an FP32
 * linearization. */
int efem_mlp_energy_rows(efem_ctx *ctx, const float *r, const float *out, double n_samples,
                         float *aux, float *z, float *kz, double *energy);

/* Residuals that Jacobi-preconditioned CG meets on K(u)_ff x = sign b from
 * x = 0 (FP32 tangent actions; the training samples of the preconditioner).
 * sign = +1 or -1; iters HOST int32 [n_snap], ascending; R DEVICE float32
 * [n_snap][3*n_nodes] receives the CG residual after iters[k] iterations.
 * *taken = snapshots reached before CG stopped (exact zero residual or
 * breakdown); later ones repeat the last residual.  Requires a Dirichlet
 * mask; synchronous. */
int efem_cg_snapshots(efem_ctx *ctx, const double *u, const double *b, double sign, int32_t n_snap,
                      const int32_t *iters, float *R, int32_t *taken);

/* Solve K(u)_ff x = b (b, x DEVICE float64 [3*n_nodes]; prescribed entries of b
 * ignored and of x set to 0) by preconditioned CG from x = 0 to
 * ||b - K x|| <= rtol ||b||, with the tangent action in hvp_prec and precond 0
 * (Jacobi), 1 (learned, flexible CG for the whole solve, Jacobi fallback;
 * needs EFEM_F32) or 2 (3x3 block Jacobi).
 * Requires a Dirichlet mask.  Synchronous; *iters receives the CG iterations,
 * *fallback 1 if the learned solve fell back to Jacobi. */
int efem_linear_solve(efem_ctx *ctx, const double *u, const double *b, double *x, double rtol,
                      int32_t hvp_prec, int32_t precond, int32_t max_iter, int32_t *iters,
                      int32_t *fallback);

/* Derivative through the equilibrium solve (the derivative of a quantity of
 * interest through a Newton solve, Sec. 6.2) is a caller-side composition of
 * the calls above, with no entry point of its own.  For the total reaction
 * J = sum_{i in T} r_i(u*) on a set T of prescribed DOFs at an equilibrium
 * u* of the masked problem:
 *   1. efem_hvp without the mask on 1_T (the indicator of T): k = K 1_T;
 *   2. efem_linear_solve with the mask on b = k: lambda (lambda_T = 0);
 *   3. efem_residual_vjp_material with w = 1_T - lambda:
 *      dJ/dmu_e = w . dr/dmu_e, dJ/dlam_e = w . dr/dlam_e.
 * The caller forms 1_T and 1_T - lambda and sums the selected entries of r. */

/* Solve K(u)_ff x = b by restarted GMRES(restart) with right Jacobi
 * preconditioning, from x = 0, to ||b - K x|| <= rtol ||b|| on the free DOFs
 * (all DOFs without a Dirichlet mask).  The Krylov solver of the
 * non-symmetric transport model (Sec. 3.1), usable with every model.
 * u, b, x: DEVICE float64 [3*n_nodes] (x distinct from u and b; prescribed
 * entries of b ignored, of x set to 0).  hvp_prec: EFEM_F64 or EFEM_F32 for
 * the tangent actions (the basis is float64 either way); restart in
 * [1, 100]; max_iter caps the total iterations.  Allocates (restart + 5)
 * float64 vectors for the solve.  Synchronous; *iters receives the
 * iterations, *relres the relative residual ||b - K x|| / ||b|| of the
 * returned x, recomputed with one more tangent action.  Returns
 * EFEM_NOT_CONVERGED when max_iter is reached first. */
int efem_gmres_solve(efem_ctx *ctx, const double *u, const double *b, double *x, double rtol,
                     int32_t hvp_prec, int32_t restart, int32_t max_iter, int32_t *iters,
                     double *relres);

/* ------------------------------------------ sparse tangent by colouring
 * The paper's second technique (Alg. 2): the tangent K(u) as a sparse matrix,
 * recovered from n_colours tangent actions.  Its pattern is the node 1-ring in
 * 3x3 blocks (CSR over DOFs, columns sorted).  DOF colours come from a greedy
 * distance-2 colouring of the node graph, times 3 components, so no row has
 * two columns of one colour; K times the indicator vector of a colour holds,
 * in each row, that row's entry of the colour.  With a Dirichlet mask the
 * rows and columns of prescribed DOFs are zero (the reduced K_ff, as
 * efem_hvp applies it). */
typedef struct {
    int64_t n_rows;           /* 3 n_nodes */
    int64_t nnz;
    int32_t n_colours;
    int32_t max_row;          /* most nonzeros in a row */
    double setup_seconds;     /* host time of the pattern and the colouring */
    int64_t n_blocks;         /* 3x3 blocks, nnz / 9 (node pairs of the 1-ring) */
} efem_sparse_info;

/* Build the pattern and the colouring (host work, synchronous; the first call
 * builds, later calls only report).  EFEM_ERR_INVALID beyond 2^31 nonzeros. */
int efem_sparse_setup(efem_ctx *ctx, efem_sparse_info *info);

/* Copy the pattern out: row_ptr DEVICE int64 [n_rows+1], col DEVICE int32
 * [nnz], dof_colour DEVICE int32 [n_rows].  EFEM_ERR_STATE before setup. */
int efem_sparse_pattern(efem_ctx *ctx, int64_t *row_ptr, int32_t *col, int32_t *dof_colour);

/* values (DEVICE float64 [nnz], in pattern order) = K(u) from n_colours FP64
 * tangent actions at u (DEVICE float64 [3*n_nodes]; the context's FP64
 * linearization is set to u). */
int efem_sparse_assemble(efem_ctx *ctx, const double *u, double *values);

/* The same pattern by 3x3 blocks: block_ptr DEVICE int64 [n_nodes+1],
 * block_col DEVICE int32 [n_blocks]; node row i holds the blocks (i, j) for
 * j = block_col[block_ptr[i] .. block_ptr[i+1]) (sorted).  In the values'
 * pattern order, node row i's entries start at 9 block_ptr[i]: its three
 * component rows one after the other, 3 len values each (len = its block
 * count), row a of block t at offset 3 t of component row a.  Enqueued on the
 * context's stream.  EFEM_ERR_STATE before setup. */
int efem_sparse_block_pattern(efem_ctx *ctx, int64_t *block_ptr, int32_t *block_col);

/* y = K x with the assembled values (x, y DEVICE float64 [3*n_nodes]), by
 * 3x3 blocks: one column index per block (the block pattern above), so the
 * bytes moved are the values, n_blocks column indices, n_nodes+1 block
 * offsets, x and y.  Enqueued on the context's stream. */
int efem_sparse_spmv(efem_ctx *ctx, const double *values, const double *x, double *y);

const char *efem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EFEM_H */
