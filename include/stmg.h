/*
 * stmg.h -- C ABI of the MI355X space-time multigrid Newton-Krylov library.
 *
 * One context holds one space-time slab I_n = (t_{n-1}, t_n] of the tensor
 * product discretization: mapped Q_{r+1}/P_r^disc in space on a structured
 * (optionally vertex-perturbed) grid of [0,1]^d, discontinuous Galerkin DG(k)
 * in time with the right-sided (k+1)-point Gauss-Radau rule (Problem
 * "Local algebraic Navier-Stokes problem", eq. InAlgNS).
 *
 * Vector layout (slab vectors, length N = (k+1)(Nv1 + Np1)), following
 * eq. DefSubvec: U = (V^1, ..., V^{k+1}, P^1, ..., P^{k+1}).
 *   V^a : d blocks (component c), each over the ((r+1)n_0+1) x ((r+1)n_1+1)
 *         (x ((r+1)n_2+1)) velocity nodes, x fastest.  Nv1 = d * Nnodes.
 *   P^a : per cell (x fastest) the C(r+d,d) coefficients of the mapped
 *         orthonormal Legendre basis of total degree <= r, first index
 *         fastest.  Np1 = ncells * C(r+d,d).
 *
 * Memory: every vector argument is a DEVICE pointer owned by the caller
 * (e.g. a torch tensor); the library never frees it.  FP64 arguments are
 * double*, FP32 arguments float* (selected by a stmg_prec argument).  All
 * device memory of a context (level tables, transfer matrices, operator
 * work buffers, smoother factors, coarse-level matrices, Krylov bases, the
 * staging of the captured V-cycle, slab data) is laid out once, when the
 * context is created, in one block of exactly stmg_footprint_bytes bytes:
 * the caller's workspace (e.g. a torch tensor, so that the caller's
 * allocator is the only one) or one library allocation; nothing is
 * allocated afterwards.
 *
 * Streams: all work of a context is enqueued on the hipStream_t given at
 * creation (NULL = the default stream).  Calls that return scalars or
 * statistics synchronize that stream; the others are asynchronous.
 *
 * Errors: 0 = success; negative = error, nothing is thrown across the ABI:
 *   STMG_EINVAL (-1) invalid argument or unsupported size,
 *   STMG_ENOMEM (-2) device allocation failed,
 *   STMG_EHIP   (-3) a HIP call failed,
 *   STMG_ESTATE (-4) call order (e.g. a smoother call before a rebuild),
 *   STMG_ENONFINITE (-5) non-finite value detected.
 * A positive value STMG_NOT_CONVERGED (+1) means a solve stopped at its
 * iteration limit; results and statistics are still written.
 * stmg_last_error returns a context-owned message for the last failure.
 */
#ifndef STMG_H
#define STMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STMG_OK 0
#define STMG_EINVAL (-1)
#define STMG_ENOMEM (-2)
#define STMG_EHIP (-3)
#define STMG_ESTATE (-4)
#define STMG_ENONFINITE (-5)
#define STMG_NOT_CONVERGED 1

typedef struct stmg_ctx stmg_ctx;

typedef enum {
    STMG_F64 = 0,
    STMG_F32 = 1,
    /* batched patch factorizations only: FP32 matrices whose trailing
     * updates take BF16 / FP16 operands on MFMA with FP32 accumulation */
    STMG_F32_BF16 = 2,
    STMG_F32_F16 = 3
} stmg_prec;

/* Data of one slab (Problem LocAlgNS; Nitsche boundary forms eq. def-b-gam,
 * eq. def-a-gam-tp).  Boundary face f = 2*axis + side (side 0: x_axis = 0,
 * side 1: x_axis = 1); bit f of dirichlet_faces set = face in Gamma_D
 * (Nitsche), clear = Gamma_N (do-nothing).  vertices: HOST pointer to
 * ((n_0+1)(n_1+1)(n_2+1)) * d coordinates, x fastest, copied at creation;
 * NULL = the uniform Cartesian grid. */
typedef struct {
    int dim;                  /* 2 or 3 */
    int n_cells[3];           /* cells per direction (n_cells[2] ignored in 2D) */
    const double *vertices;   /* host, may be NULL */
    int r;                    /* pressure degree r (1..3); velocity Q_{r+1} */
    int k;                    /* time degree k (0..3) */
    double nu;                /* kinematic viscosity */
    double tau;               /* slab length tau_n */
    unsigned dirichlet_faces; /* bit mask, see above */
    double gamma1, gamma2;    /* Nitsche penalties (Sec. "Numerical experiments": 10, 10) */
} stmg_problem;

/* Solver options.  stmg_default_options fills the values used in Sec.
 * "Numerical experiments" where the paper states them and documented
 * defaults where it is silent. */
typedef struct {
    int n_q;                  /* Gauss points per direction; 0 = ceil((3r+4)/2) */
    int max_levels;           /* multigrid levels cap; 0 = coarsen to 2^d cells */
    int nu1, nu2;             /* pre/post smoothing steps (1, 1) */
    double vanka_omega;       /* relaxation omega of eq. LVS; 0 = default (1.0 weighted, 1.4/2^d plain) */
    int prec_mg;              /* stmg_prec of the multigrid preconditioner */
    /* Newton (Alg. "Inexact Newton-Krylov") */
    double newton_rtol, newton_atol;
    int newton_maxit;
    /* Eisenstat-Walker forcing */
    double ew_eta0, ew_c, ew_theta, ew_eta_min, ew_eta_max;
    /* Armijo line search (Alg. "Armijo") */
    double ls_lambda0, ls_c, ls_tau, ls_alpha_min;
    int ls_window, ls_max_backtracks;
    /* smoother rebuild triggers */
    double rb_theta_N, rb_theta_L, rb_kappa_abs, rb_stag_theta;
    int rb_stag_s;
    /* FGMRES */
    int fgmres_maxit;
    /* Vanka sweep weighting (eq. vanka0 leaves omega open): 1 = each
     * unknown's correction divided by the number of patches holding it
     * (partition of unity, omega default 1.0; the default); 0 = the plain
     * sum of the patch corrections with a scalar omega (default 1.4/2^d). */
    int vanka_weighting;
    /* Patch solves of the midpoint surrogate (eq. DefTildeHn): 1 = split the
     * time coupling by the eigen-decomposition of W^{-1} K, one spatial
     * (complex for a conjugate eigenvalue pair) factorization per distinct
     * eigen-system, the same result as the full space-time patch up to
     * rounding at (k+1)x less factor memory (the default); 0 = factor the
     * full (k+1)-node patch. */
    int vanka_time_decoupled;
    /* 1 = each FGMRES preconditioner application (the V-cycle of the
     * hierarchy, Sec. "Preconditioning of GMRES by hp-STMG") replays one
     * captured HIP graph on two library-owned N-vectors (captured again after
     * every smoother rebuild or state change; eager launches if capture is
     * refused); 0 = eager kernel launches.  Results are identical. */
    int use_graphs;
    /* p-coarsening in time (Sec. "Preconditioning of GMRES by hp-STMG"):
     * 0 = DG(k) kept on every level (default: the V-cycle contraction stays
     * about 0.3 for k = 2, 3 under h-refinement); 1 = k -> floor(k/2) together
     * with the spatial p steps, the order the paper states (contraction
     * 0.56 -> 0.84 for k = 2 and 0.69 -> 0.96 for k = 3 from h = 1/4 to
     * 1/32 on the 2D convergence problem). */
    int time_coarsening;
    /* FP32 multigrid with time-decoupled patches only (ignored otherwise):
     * the factors are still computed in FP32, but the smoothing sweeps read a
     * BF16 copy (round to nearest even; half the bytes per sweep, entries
     * relative to 2^-9), widened to FP32 for the substitutions.  0 (default)
     * or 1.  The copy adds half of the FP32 factor bytes to the footprint. */
    int vanka_factor_bf16;
    /* Diagonal Vanka (the cheaper smoothing the paper's conclusions call
     * for): in every patch system the velocity-velocity block keeps only its
     * spatial diagonal (time coupling and pressure blocks stay), and the
     * patch is solved through its pressure Schur complement.  2: the
     * velocity-velocity blocks keep their node blocks instead (all velocity
     * components of one node).  Time-decoupled patches only (ignored
     * otherwise).  0 (default), 1 or 2. */
    int vanka_diagonal;
} stmg_options;

typedef struct {
    int newton_its;
    int fgmres_its_total;
    int fgmres_its[64];       /* per Newton step */
    int rebuilds;
    int backtracks;
    double res0_M, res_M;     /* initial / final ||R||_M */
    double wall_s;
} stmg_stats;

void stmg_default_options(stmg_options *opt);

/* Device bytes a context of this problem and these options consumes: the
 * exact size of its workspace, measured by running the context's own
 * construction code without device memory (host only, no GPU needed); 0 for
 * an invalid problem or options (see stmg_create). */
size_t stmg_footprint_bytes(const stmg_problem *prob, const stmg_options *opt);

/* Create a context on the current HIP device.  workspace: DEVICE pointer to
 * ws_bytes >= stmg_footprint_bytes bytes, 256-byte aligned, owned by the
 * caller and used by the context until stmg_destroy (the library then calls
 * no device allocator for this context); NULL = the library allocates one
 * block of the footprint itself and frees it in stmg_destroy.  stream:
 * hipStream_t or NULL.  Returns STMG_EINVAL, before any device work, for
 * unsupported (dim, r, k, n_q) combinations, options outside their
 * documented ranges (prec_mg other than STMG_F64/STMG_F32, a negative count,
 * a flag other than 0/1, vanka_diagonal other than 0/1/2) or a misaligned
 * workspace, STMG_ENOMEM for a workspace smaller than the footprint; with the
 * environment variable STMG_VERBOSE set the reason is printed on stderr. */
int stmg_create(const stmg_problem *prob, const stmg_options *opt, void *workspace, size_t ws_bytes, void *stream,
                stmg_ctx **out);
/* Bytes of the workspace the context has laid out (equal to
 * stmg_footprint_bytes of its problem and options, up to the final 256-byte
 * rounding). */
size_t stmg_workspace_used(const stmg_ctx *ctx);
int stmg_destroy(stmg_ctx *ctx);
const char *stmg_last_error(const stmg_ctx *ctx);

/* New viscosity nu and slab length tau for an existing context (same mesh,
 * degrees, boundary data and options): the time matrices of every level are
 * recomputed; the state, smoother and captured V-cycle are invalidated (the
 * next stmg_set_state / stmg_smoother_rebuild / Newton solve sets them up
 * again); slab data stay.  Synchronizes the context stream. */
int stmg_set_coefficients(stmg_ctx *ctx, double nu, double tau);

/* Sizes of the slab vectors: total N, velocity part (k+1)Nv1, pressure part. */
int stmg_sizes(const stmg_ctx *ctx, long long *n_total, long long *n_velocity, long long *n_pressure);

/* Slab data of eq. InAlgNS: rhs = F_n + L_n (velocity rows) and the
 * continuity-row data (length N, FP64, device) and v_prev = the velocity
 * coefficients v_{n-1}^{k+1} (or v_0) of one time node (length Nv1, FP64,
 * device).  Both are copied; NULL means zero. */
int stmg_set_slab_data(stmg_ctx *ctx, const double *rhs, const double *v_prev);

/* Slab residual R_n(U; V_{n-1}) of eq. InAlgNS in FP64:
 *   r_v^a = sum_b K_ab M_h u_v^b + w_a s_v(u^a) - rhs_v^a - phi_a(t_{n-1}^+) M_h v_prev
 *   r_p^a = w_a s_p(u^a) - rhs_p^a
 * with s the spatial form A^tp_gamma (convection in divergence form,
 * eq. ns-form-tp, reduced Radau quadrature in time, eq. QuadNL) and w_a the
 * diagonal of M_n^tau.  u, r: device, length N; r is overwritten. */
int stmg_residual(stmg_ctx *ctx, const double *u, double *r);

/* y = J_n(U) x (eq. JacobianLocal): the exact slab Jacobian at the state
 * u_state (only its velocity part is read), applied matrix-free with sum
 * factorization (Sec. "Matrix-free operator evaluation").  prec selects
 * FP64 (double*) or FP32 (float*) for u_state, x and y.  y is overwritten. */
int stmg_jacobian_vmult(stmg_ctx *ctx, int prec, const void *u_state, const void *x, void *y);

/* Batched form: nvec vectors stored contiguously with stride N (x, y) and
 * the same state for all (applied one vector per launch on the finest
 * level: the work buffers are laid out for one). */
int stmg_jacobian_vmult_batched(stmg_ctx *ctx, int prec, const void *u_state, const void *x, void *y, int nvec);

/* y = blockdiag(M^tau (x) M_h, M^tau (x) M_h^p) x: the weight of the norm
 * ||.||_M of eq. inexact. */
int stmg_mass_vmult(stmg_ctx *ctx, int prec, const void *x, void *y);

/* ---- hp space-time multigrid (Sec. "Preconditioning of GMRES by hp
 * space-time multigrid") ----------------------------------------------------
 * Levels: 0 = the slab itself; p-coarsening first, (k, r) -> (k, max(1,
 * r//2)) by default, or (k//2 if k >= 2 else k, max(1, r//2)) with
 * opt.time_coarsening = 1, then h-coarsening of the mesh while every n_cells
 * is even and >= 4 (capped by opt.max_levels).  Level vectors use the slab
 * layout of their own (k, r, n_cells). */
int stmg_num_levels(const stmg_ctx *ctx);
int stmg_level_info(const stmg_ctx *ctx, int level, int *k, int *r, int *n_cells, long long *n_total);

/* Set the Newton state U (FP64, device, length N): the level states (finer
 * state evaluated at the coarser nodes and Radau nodes) and the FP64 LU of
 * the coarsest level Jacobian (bordered by the constant pressures of each
 * time node when every face is Dirichlet). */
int stmg_set_state(stmg_ctx *ctx, const double *u_state);
/* Copy of the state of a level (FP64 slab vector of that level). */
int stmg_level_state(stmg_ctx *ctx, int level, double *out);

/* Set the state and rebuild the inexact space-time Vanka smoother on every
 * level but the coarsest (eq. DefTildeHn, eq. DefVnAst: the spatial core at
 * the midpoint value V* = sum_a phi_a(t*) V^a, shared by all time nodes;
 * patch = all unknowns of one cell at all time nodes; local matrix = the
 * principal submatrix of the surrogate; LU with partial pivoting in the
 * multigrid precision). */
int stmg_smoother_rebuild(stmg_ctx *ctx, const double *u_state);

/* y = J_level x at the level state (FP64, or FP32 if the multigrid runs in
 * FP32). */
int stmg_level_jacobian_vmult(stmg_ctx *ctx, int level, int prec, const void *x, void *y);

/* The full space-time surrogate patch of one cell (eq. LVS with the core of
 * eq. DefTildeHn, before factorization): the principal submatrix of the
 * surrogate Jacobian on all unknowns of `cell` at all time nodes, m x m
 * row-major with m = (k+1)(d (r+2)^d + C(r+d,d)) of that level, unknowns
 * ordered velocity [a][c][local node], then pressure [a][mode].  Uses the
 * element matrices of the last stmg_smoother_rebuild (STMG_ESTATE before
 * it).  out: device array of m*m values in the multigrid precision (prec
 * must equal opt.prec_mg). */
int stmg_level_patch(stmg_ctx *ctx, int level, int cell, int prec, void *out);

/* `sweeps` additive Vanka sweeps on a level (eq. vanka0):
 *   d <- d + omega sum_K R_K^T S_K^{-1} R_K (r - J_level d).
 * r, d: device slab vectors of that level in the multigrid precision
 * (prec must equal opt.prec_mg); d is updated in place.  STMG_ESTATE if the
 * smoother has not been built. */
int stmg_vanka_smooth(stmg_ctx *ctx, int level, int prec, const void *r, void *d, int sweeps);

/* d = B r: one V-cycle from a zero initial guess (nu1 pre- and nu2
 * post-smoothing sweeps, restriction = transpose of the canonical-embedding
 * prolongation, coarsest level solved directly), in the multigrid
 * precision on the finest-level slab vectors. */
int stmg_vcycle(stmg_ctx *ctx, int prec, const void *r, void *d);

/* Grid transfers between level and level+1 (slab vectors of the two
 * levels): y_fine = P x_coarse (eq. MatGeomProl and the polynomial
 * prolongation), y_coarse = P^T x_fine. */
int stmg_prolongate(stmg_ctx *ctx, int level, int prec, const void *xc, void *yf);
int stmg_restrict(stmg_ctx *ctx, int level, int prec, const void *xf, void *yc);

/* Right-preconditioned flexible GMRES on J(u_state) x = b (FP64, zero
 * initial guess, Arnoldi in the M inner product, preconditioner = one
 * V-cycle), stopped when the M-norm residual estimate is <= rtol ||b||_M or
 * after maxit iterations (maxit <= opt.fgmres_maxit, the size of the Krylov
 * workspace; STMG_EINVAL otherwise).  its: iterations; hist: its+1 residual estimates
 * (host array, may be NULL).  Needs a built smoother.  Returns
 * STMG_NOT_CONVERGED at the iteration limit. */
int stmg_fgmres(stmg_ctx *ctx, const double *u_state, const double *b, double *x, double rtol, int maxit, int *its,
                double *hist);

/* Solve the slab problem R_n(U; V_{n-1}) = 0 (eq. InAlgNS) by the inexact
 * Newton method of Alg. "Inexact Newton-Krylov" with Alg. "Armijo":
 * Eisenstat-Walker forcing, nonmonotone Armijo backtracking, smoother
 * rebuilds on Newton/linear deterioration and FGMRES stagnation, FGMRES
 * preconditioned by one hp-STMG V-cycle.  u_inout: initial guess in,
 * solution out (device, FP64).  Stops when ||R||_M <= max(atol, rtol
 * ||R_0||_M).  stats may be NULL. */
int stmg_newton_gmres_solve(stmg_ctx *ctx, double *u_inout, stmg_stats *stats);

/* Time marching over consecutive slabs I_1, ..., I_nslabs: the slab-by-slab
 * solution of Problem LocAlgNS (Sec. "Space-time discretization"), each slab
 * by stmg_newton_gmres_solve.  The previous-slab velocity of slab n >= 1 is
 * the discrete velocity at t_{n-1}^-, i.e. the velocity block of the last
 * time node of slab n-1's solution (the right Radau rule has its last node at
 * the slab end).
 *   rhs : device, slab data of slab n at rhs + n * rhs_stride (length N, as
 *         in stmg_set_slab_data); NULL = zero data
 *   v0  : device, the initial velocity (length Nv1); NULL = zero
 *   u   : device, slab n's vector at u + n * u_stride (stride >= N); on entry
 *         slab 0's entries are its Newton initial guess, slab n >= 1 starts
 *         from slab n-1's solution; on return every slab's solution
 *   stats: host array of nslabs entries, or NULL.
 * Returns 0, STMG_NOT_CONVERGED if some slab stopped short of the tolerance
 * (marching continues from its last iterate), or a negative error code
 * (marching stops at that slab). */
int stmg_march(stmg_ctx *ctx, int nslabs, const double *rhs, long long rhs_stride, const double *v0, double *u,
               long long u_stride, stmg_stats *stats);

/* ---- batched patch factorizations (no context) ---------------------------
 * A batch of dense matrices of mixed sizes, factored by LU with partial
 * pivoting (the Vanka patch factorization of Sec. "Inexact space-time Vanka
 * smoother" as a standalone batch) in ONE persistent launch: a grid of
 * workgroups sized to stay resident takes the matrices, largest first, from a
 * device work queue; each matrix is factored by one workgroup with blocked
 * right-looking panels in LDS and the trailing updates on MFMA
 * (v_mfma_f32_16x16x4f32 in FP32, v_mfma_f64_16x16x4f64 in FP64).  The
 * workgroups per CU and the panel width of each size class come from a table
 * written by the package's tuner (paper_2602_13841_amd/tune_lu.py).  prec:
 * STMG_F64, STMG_F32, or STMG_F32_BF16 / STMG_F32_F16 (FP32 matrices and
 * factors; the L21 and U12 blocks of each trailing update A22 -= L21 U12 are
 * rounded to BF16 / FP16 for the MFMA, A22 accumulates in FP32; the solve is
 * the FP32 one).  Matrix b is m_of[b] x m_of[b], row-major, at element offset
 * a_off[b] of the device array A and is overwritten by its factors (unit
 * lower L below the diagonal, U on and above); piv + p_off[b] receives
 * m_of[b] 0-based row interchanges (row j was swapped with row piv[j],
 * applied in order j = 0, 1, ...).  m_of, a_off, p_off are HOST arrays of
 * `batch` entries; A and piv are device arrays owned by the caller; info
 * (device, may be NULL) is incremented for every exactly zero pivot.
 * stream: a hipStream_t or NULL; the call synchronizes it.  Returns 0,
 * STMG_EINVAL (bad sizes, m > 2048), STMG_ENOMEM or STMG_EHIP. */
int stmg_batched_lu(int prec, void *A, const long long *a_off, const int *m_of, int batch, int *piv,
                    const long long *p_off, int *info, void *stream);

/* Tuning form of stmg_batched_lu (used by the tuner): explicit launch
 * parameters instead of the table.  wg_per_cu in 1..4 sets the LDS budget of
 * the persistent launch (160 KiB / wg_per_cu per workgroup); nb_by_class[c]
 * in {4, 8, 16} is the panel width for matrices of size <= 128, 256, 512,
 * 1024, 2048 (c = 0..4), halved while the panel does not fit the budget.
 * wg_per_cu = 0: one launch per size class instead (no work queue), the
 * untuned reference.  threads (256 or 512): the workgroup that factors one
 * matrix (4 or 8 wavefronts).  Other arguments as in stmg_batched_lu. */
int stmg_batched_lu_config(int prec, void *A, const long long *a_off, const int *m_of, int batch, int *piv,
                           const long long *p_off, int *info, int wg_per_cu, int threads, const int *nb_by_class,
                           void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * factorization as stmg_batched_lu, with the device staging of the
 * per-matrix sizes and offsets (32 bytes per matrix) in a fixed library
 * array of STMG_NOALLOC_MAX_BATCH entries per device (2 MiB, held by every
 * device the library runs on until the process ends) instead of a per-call
 * allocation; it calls no hipMalloc or hipFree.  Returns STMG_EINVAL for
 * batch > STMG_NOALLOC_MAX_BATCH.  All calls on one device share the array
 * and every call overwrites it before use: calls that overlap on one device
 * (other host threads, other streams) race and must be serialized by the
 * caller.  The call synchronizes `stream` before it returns. */
#define STMG_NOALLOC_MAX_BATCH 65536
int stmg_batched_lu_noalloc(int prec, void *A, const long long *a_off, const int *m_of, int batch, int *piv,
                            const long long *p_off, int *info, void *stream);

/* Solve with the factors of stmg_batched_lu: right-hand side b (device) of
 * matrix b at element offset b_off[b] (HOST array), overwritten by the
 * solution.  Same metadata as the factorization. */
int stmg_batched_lu_solve(int prec, const void *LU, const long long *a_off, const int *m_of, int batch,
                          const int *piv, const long long *p_off, void *b, const long long *b_off, void *stream);

/* ---- serving (continuous batching of slab solves) ------------------------
 * A request is one slab problem with HOST data: v_prev (Nv1 doubles, may be
 * NULL = 0), rhs (N doubles or NULL), u_init (N doubles or NULL = 0) and the
 * output buffer u_out (N doubles, may be NULL).  arrival_s: arrival time in
 * seconds after the start of stmg_serve.  prob.vertices must stay valid
 * until stmg_serve returns. */
typedef struct {
    stmg_problem prob;
    double arrival_s;
    const double *v_prev;
    const double *rhs;
    const double *u_init;
    double *u_out;
} stmg_request;

typedef struct {
    double start_s, end_s;    /* admission and completion time */
    double latency_s;         /* completion - arrival */
    int rc;                   /* return code of the solve */
    size_t footprint;         /* device bytes reserved for the request */
    stmg_stats stats;
    int reused_context;       /* 1: served by a pooled context of an earlier request */
} stmg_request_result;

/* Serve n requests with `slots` concurrent solves on the current device
 * (continuous batching).  When a slot is free, the earliest arrived request
 * that fits is admitted (first fit in arrival order): it fits when an idle
 * context of the same discretization (everything but nu and tau) is pooled,
 * or when its footprint (stmg_footprint_bytes) next to the running requests
 * stays within hbm_budget bytes (0 = 85 % of the device memory free at the
 * start), idle pooled contexts being destroyed for it.  Every admitted
 * request runs on its own stream and context, so the work of overlapping
 * requests overlaps on the device; finished contexts return to the pool and
 * are reused (stmg_set_coefficients) by later requests of the same shape.
 * Request vectors are staged in per-slot device buffers sized for the largest
 * request.  wall_s: total time (may be NULL).  Returns 0, or the last
 * negative request code; STMG_ENOMEM if a single request exceeds the budget. */
int stmg_serve(const stmg_request *reqs, int n, const stmg_options *opt, int slots, size_t hbm_budget,
               stmg_request_result *res, double *wall_s);

/* Named kernel timers (hipEvent pairs on the context stream around each
 * kernel launch, e.g. "cell_jac_f64", "gather_f64", "cell_res_f64",
 * "cell_mass_f32"); off by default.  stmg_timing_get synchronizes the
 * recorded events and returns the accumulated milliseconds and the number
 * of launches of that name since the last reset. */
int stmg_timing_enable(stmg_ctx *ctx, int on);
int stmg_timing_reset(stmg_ctx *ctx);
int stmg_timing_get(stmg_ctx *ctx, const char *name, double *total_ms, long long *count);

#ifdef __cplusplus
}
#endif

#endif /* STMG_H */
