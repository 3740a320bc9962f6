/*
 * gmg.h -- C ABI of the MI355X two-grid matching-aggregation AMG solver.
 *
 * The library solves A x = b, A in R^{N x N} sparse, x, b in R^N (the paper's
 * statement of the problem, Eq. (system) and the caption of Algorithm 1) with
 * flexible GMRES(m) right-preconditioned by the two-grid operator B~ of
 * Eq. (twogrid) / Algorithm 1:
 *   - aggregates G_i from deterministic multi-pass handshake graph matching
 *     (the paper calls a graph partitioner; Section 2, "Aggregation based on
 *     graph matching"), boolean prolongation P (Eq. (interp), Eq. (aggr));
 *   - Galerkin coarse matrix A_c = P^T A P (Eq. (E:galerkin));
 *   - smoother S = L0 U0 = ILU(0)(A), one application, no post-smoothing
 *     (Section 2, the paragraph defining S and Eq. (twogrid));
 *   - inexact coarse solve with ILUT(tau) factors of A_c (Section 2, the
 *     ILU(t) paragraph; Algorithm 1 "SOLVE M~g=h").
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers (HIP device memory, e.g. torch CUDA
 *     tensors on ROCm) unless the parameter says "host".  The caller keeps
 *     ownership; the library never frees caller memory.
 *   - CSR matrices use int32 row pointers and column indices and float64
 *     values; columns strictly ascending within each row; every row stores its
 *     diagonal.  Violations return GMG_ERR_INVALID_ARG, non-finite values
 *     GMG_ERR_NONFINITE.
 *   - Multi-vector arguments (b, x, g, lambda) are (N, nrhs) row-major.
 *   - All device work is enqueued on the stream given to gmg_setup (or set with
 *     gmg_set_stream).  Entry points return after their results are complete on
 *     that stream.  A handle must not be used from two threads at once.
 *   - Every function returns a gmg_status; on an error gmg_last_error() gives a
 *     thread-local message.  A status > 0 is a warning whose outputs are valid.
 */
#ifndef GMG_H
#define GMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmg_solver* gmg_handle;

typedef enum {
  GMG_OK = 0,
  GMG_NOT_CONVERGED = 1,     /* maxit reached; the best iterate is returned (the paper's NC) */
  GMG_ERR_INVALID_ARG = -1,
  GMG_ERR_HIP = -2,          /* a HIP runtime call failed                               */
  GMG_ERR_OOM = -3,          /* device or host allocation failed (the paper's ME)       */
  GMG_ERR_ZERO_PIVOT = -4,   /* ILU(0) or ILUT met a zero pivot                         */
  GMG_ERR_BREAKDOWN = -5,    /* Givens rotation with a zero column                      */
  GMG_ERR_NONFINITE = -6,    /* NaN/Inf in an input or in a residual                    */
  GMG_ERR_NOT_SETUP = -7,
  GMG_ERR_STALLED = -8       /* a dependency wait in a triangular sweep exceeded its
                                time limit (internal error; results are invalid)        */
} gmg_status;

typedef struct {
  double cf;            /* coarsening factor N / N_c: matching passes stop once
                           N_c <= floor(N / cf) (default 4)                          */
  int max_passes;       /* matching passes at most (default 8)                       */
  int match_qbits;      /* mantissa bits of an edge weight kept in the matching key;
                           ties inside a bin are broken by a hash (default 4; 52 =
                           exact weights)                                             */
  uint64_t hash_seed;   /* seed of that hash                                         */
  double ilut_tau;      /* ILUT drop tolerance relative to the row 2-norm (1e-4)     */
  int coarse_mode;      /* 0: exact triangular sweeps with the ILUT factors;
                           1: coarse_sweeps Jacobi sweeps per factor (FP64);
                           2: e_c = M r_c with a sparse approximate inverse M of
                           A_c on A_c's pattern (no ILUT is computed);
                           3: e_c = A_c^{-1} r_c with the dense inverse, the exact
                           coarse solve of the EGMG variant of Section 3, for
                           N_c <= 8192 (no ILUT is computed; larger N_c give
                           GMG_ERR_INVALID_ARG at setup, a zero pivot of the
                           no-pivot elimination GMG_ERR_ZERO_PIVOT)              */
  int coarse_sweeps;    /* (default 3)                                               */
  int restart;          /* FGMRES restart length m (default 30, at most 2048)        */
  int maxit;            /* total FGMRES steps at most (default 600)                  */
  int precond_fp32;     /* 1: the whole preconditioner runs in FP32 on FP32 copies of
                           A and of the factors; the Krylov part stays FP64          */
  int x0_given;         /* 1: x holds the initial guess on entry, else x0 = 0         */
  int sweep_waves;      /* resident waves of the triangular sweeps (0: auto)          */
  int coarse_order;     /* numbering of the aggregates, hence of A_c and its ILUT
                           factors: 0 by smallest fine index; 1 nested dissection
                           of A_c's graph (default)                                   */
  int sweep_kernel;     /* 0 (default): fine factors with 2D- or 3D-grid structure
                           (five- or seven-point operators in natural order) use
                           the wavefront sweep, coarse factors in nested-dissection
                           order the tree solve, other factors the level sweeps
                           (single-CU ring for narrow factors, else level ranges
                           on one workgroup or the whole device); 3: as 0 but
                           with level sweeps for the coarse factors; 1: the
                           whole-device level sweep for every factor; 2: the
                           one-workgroup level sweep for every factor.  1, 2
                           and 3 give bitwise identical results; 0 differs from
                           them only in the coarse solves' summation order      */
  int sweep_wg_chunks;  /* level sweeps under sweep_kernel 0 or 3: dependency levels of at most this many
                           64-lane chunks run on one workgroup (default 8; 0: never) */
  int fine_order;       /* numbering of the ILU(0) smoother: 0 (default) A's own;
                           1 nested dissection of A's graph (the GMG-ND variant of
                           Section 3.1): S = Q^T L0 U0 Q with L0 U0 = ILU(0) of
                           Q A Q^T, applied over the dissection tree under
                           sweep_kernel 0 (level sweeps otherwise, or when a
                           separator exceeds 2048 rows); 2 colour classes of a
                           greedy colouring in natural order (red-black on 5-
                           and 7-point grids; multicolour ILU(0)), applied by
                           level sweeps with one level per colour.  Aggregates,
                           A_c and its ILUT do not depend on it.                */
} gmg_options;

typedef struct {
  int iters;            /* FGMRES steps of the last solve (summed over RHS)           */
  int restarts;
  int converged;        /* number of right-hand sides that reached tol               */
  int passes;           /* matching passes                                           */
  int rounds;           /* handshake rounds, summed over passes                      */
  int levels_L0, levels_U0, levels_Lc, levels_Uc;  /* dependency depths of the sweeps */
  int64_t n, nnz, n_coarse, nnz_coarse, nnz_lc, nnz_uc;
  double relres_true;   /* max over RHS of ||b - A x|| / ||b|| after the solve       */
  double relres_est;    /* FGMRES estimate at exit                                   */
  double setup_ms, solve_ms;
} gmg_info;

/* Fill *opts with the defaults listed above. */
void gmg_default_options(gmg_options* opts);

/* Setup phase of Algorithm 1: copies A (device CSR, n rows, nnz entries) into
 * library memory, builds the aggregates, A_c, ILU(0)(A), ILUT(A_c) and the
 * schedules of the triangular sweeps.  `stream` is a hipStream_t (NULL = the
 * default stream).  On success *h owns all library memory; free it with
 * gmg_destroy.  The caller may free A after return.  Process-wide state:
 * device blocks the library frees are cached per device for later calls (at
 * most an eighth of the device's memory, or GMG_POOL_MB megabytes), and large
 * host-device copies of the setup go through pinned host chunks of 4 MB that
 * are kept until the process ends (eight per copy in flight). */
gmg_status gmg_setup(gmg_handle* h, int64_t n, int64_t nnz, const int32_t* rowptr,
                     const int32_t* col, const double* val, const gmg_options* opts,
                     void* stream);

/* Solve phase of Algorithm 1: A x = b to ||b - A x|| / ||b|| < tol for each
 * of nrhs columns (device arrays of N*nrhs doubles, row-major) by flexible
 * GMRES preconditioned with B~.  Uses the options given to gmg_setup, except
 * x0_given/maxit/restart/precond_fp32, taken from `opts` when it is not NULL.
 * With nrhs > 1 and restart <= 32 the columns are solved in batches of up to
 * 16 that share every kernel launch (one FGMRES recurrence per column; each
 * column stops at its own tolerance); otherwise one after another.  `info`
 * (host, may be NULL) receives statistics, steps summed over the columns.
 * GMG_NOT_CONVERGED when a column is not at tol after maxit steps (its best
 * iterate is returned). */
gmg_status gmg_solve(gmg_handle h, const double* b, double* x, int nrhs, double tol,
                     const gmg_options* opts, gmg_info* info);

/* Adjoint solve A^T lambda = g, preconditioned by B~^{-T} (the exact transpose
 * of the two-grid operator of Eq. (twogrid): the transposed coarse solve
 * (transposed ILUT factors; for coarse_mode 1 the Jacobi sweeps on U~^T, then
 * on L~^T; for 2 and 3 the transposed approximate or dense inverse), the
 * residual with A^T, the transposed ILU(0) sweeps in the smoother's
 * numbering).  Not in the paper: the backward pass of a differentiable solve.
 * Same layout, batching and statuses as gmg_solve; every coarse_mode and
 * fine_order; FP64 only (precond_fp32 must be 0, else GMG_ERR_INVALID_ARG). */
gmg_status gmg_solve_adjoint(gmg_handle h, const double* g, double* lambda, int nrhs,
                             double tol, const gmg_options* opts, gmg_info* info);

/* One application q = B~^{-1} z (adjoint: q = B~^{-T} z) of the two-grid
 * preconditioner, Algorithm 1 "SOLVE B~q = z" in its one-coarse-solve form
 * (device vectors of N doubles).  precision 0: FP64; 1: FP32 internally
 * (the adjoint application is FP64 only). */
gmg_status gmg_apply_precond(gmg_handle h, const double* z, double* q, int precision,
                             int adjoint);

/* y = A x (transposed != 0: y = A^T x), device vectors of N doubles: the
 * product with the system matrix that every Arnoldi step of Algorithm 1 takes
 * (w = A z_j), with the library's copy of A. */
gmg_status gmg_spmv(gmg_handle h, int transposed, const double* x, double* y);

/* Setup statistics (sizes, passes, levels, setup time) into *info (host).
 * Not a step of the paper: inspection of the setup phase. */
gmg_status gmg_get_info(gmg_handle h, gmg_info* info);

/* Residual history of the last gmg_solve / gmg_solve_adjoint on h: the
 * FGMRES estimate |g_{j+1}| / ||b|| after every step, right-hand sides one
 * after another, restarts included (the convergence curves of Section 3,
 * Figures F:curvePres and F:curveJUMP).  Copies min(cap, count) values into
 * the host array hist and the number of steps into *count (host). */
gmg_status gmg_get_history(gmg_handle h, int cap, double* hist, int* count);

/* Cheap condition estimates of Section 3 (the lemma on diagonal entries and
 * the estimate for an incomplete factorization that follows it), computed on
 * demand on the host: *est_coarse = max_i |(A_c)_ii| / min_i |(A_c)_ii|, a
 * lower bound of cond(A_c) when A_c is SPD; *est_ilut = max_i |(L~U~)_ii| /
 * min_i |(L~U~)_ii|, the unsymmetric form of the factorization's estimate,
 * (L~U~)_ii = u_ii + sum_{j<i} l_ij u_ji.  Both are host doubles; a zero
 * denominator gives +inf.  GMG_ERR_INVALID_ARG under coarse_mode 2 or 3. */
gmg_status gmg_cond_estimate(gmg_handle h, double* est_coarse, double* est_ilut);

/* Aggregate of every fine unknown (the sets G_i of Eq. (aggr), column i of
 * the boolean P of Eq. (interp)): agg device int32[N], ids 0..N_c-1 in the
 * numbering of the coarse unknowns: nested dissection of A_c's graph under
 * coarse_order 1 (the default), by each aggregate's smallest fine index
 * under coarse_order 0. */
gmg_status gmg_get_aggregates(gmg_handle h, int32_t* agg);

/* The Galerkin coarse matrix A_c = P^T A P of Eq. (E:galerkin) as CSR, rows
 * and columns in the coarse numbering of gmg_get_aggregates, into device
 * arrays rowptr[N_c+1], col[nnz_coarse], val[nnz_coarse] (sizes from
 * gmg_get_info; structural zeros kept). */
gmg_status gmg_get_coarse(gmg_handle h, int32_t* rowptr, int32_t* col, double* val);

/* The smoother S = L0 U0 = ILU(0) (Section 2, the paragraph defining S;
 * Algorithm 1's setup) as values on the pattern of the smoother's matrix
 * (device double[nnz]): A's pattern, or under fine_order 1 or 2 that of
 * Q A Q^T (row k is row perm[k] of A, columns renumbered and ascending).
 * The strictly lower part is L0 (unit diagonal implied), the rest is U0. */
gmg_status gmg_get_ilu0(gmg_handle h, double* val);

/* The smoother's numbering: perm (device int32[N]) with position k holding
 * fine unknown perm[k]; the identity under fine_order 0, the nested
 * dissection (GMG-ND, Section 3.1) under 1, the colour classes under 2. */
gmg_status gmg_get_fine_perm(gmg_handle h, int32_t* perm);

/* The sparse approximate inverse of A_c (coarse_mode 2), a parallel inexact
 * coarse solve (Section 2 leaves parallel inexact coarse solves for large
 * coarse grids to future work): A_c's pattern, column j the least-squares
 * minimiser of ||A_c m - e_j||_2 over that column's pattern.  Device arrays
 * rowptr[N_c+1], col[nnz_coarse], val[nnz_coarse]; GMG_ERR_INVALID_ARG under
 * another coarse_mode. */
gmg_status gmg_get_spai(gmg_handle h, int32_t* rowptr, int32_t* col, double* val);

/* The dense exact inverse of A_c (coarse_mode 3; the EGMG variant's exact
 * coarse solve, Section 3) into the device array inv[N_c * N_c], row-major.
 * GMG_ERR_INVALID_ARG under another coarse_mode. */
gmg_status gmg_get_coarse_inverse(gmg_handle h, double* inv);

/* ILUT(tau) factors of A_c (Section 2, the ILU(t) paragraph; Algorithm 1's
 * setup of the inexact coarse solve): L~ strictly lower (unit diagonal
 * implied) and U~ with its diagonal first in each row; device arrays sized by
 * gmg_get_info (nothing to copy under coarse_mode 2 or 3, which compute no
 * ILUT: nnz_lc = nnz_uc = 0). */
gmg_status gmg_get_ilut(gmg_handle h, int32_t* lrowptr, int32_t* lcol, double* lval,
                        int32_t* urowptr, int32_t* ucol, double* uval);

/* Change the stream used by later calls on h (not from the paper). */
gmg_status gmg_set_stream(gmg_handle h, void* stream);

/* Per-kernel-class timing with HIP events on the handle's stream (not from
 * the paper: the measurement of this implementation).
 * gmg_profile_enable(h, 1) starts recording every class (resets the
 * counters); enable > 1 records only the classes c whose bit c + 1 is set
 * (each recorded class boundary costs the stream a few microseconds); 0 stops;
 * negative values are GMG_ERR_INVALID_ARG.
 * gmg_profile_read fills up to `cap` records (host arrays) with the class
 * name index, launch count, total milliseconds and algorithmic bytes moved,
 * and returns the number of classes in *count.  Names: gmg_profile_name. */
gmg_status gmg_profile_enable(gmg_handle h, int enable);
gmg_status gmg_profile_read(gmg_handle h, int cap, int* count, int64_t* launches,
                            double* ms, double* bytes);
const char* gmg_profile_name(int cls);

/* Release everything owned by h (NULL is ignored; not from the paper). */
void gmg_destroy(gmg_handle h);

/* Message of the last error on this thread ("" if none; not from the paper). */
const char* gmg_last_error(void);

/* ---------------------------------------------------------------------------
 * Finite-volume convection-diffusion assembly and its gradient, for the
 * differentiable solve.  Discretisation of Eq. (pde) on [0,1]^dim with
 * n cells per direction, unknown i + n j (+ n^2 k), Dirichlet faces y = 0, 1,
 * Neumann elsewhere; harmonic face transmissibilities 2 k_c k_m / ((k_c+k_m) h^2),
 * Dirichlet faces 2 k_c / h^2, first-order upwind convection with the given
 * face-averaged velocities.
 *   kappa: device double[n^dim]; vel_x, vel_y(, vel_z): device face velocities,
 *   direction d array has n+1 entries along d (x fastest memory order);
 *   rowptr/col/val: device outputs sized for the 5-/7-point pattern
 *   (gmg_fv_nnz gives nnz); pattern identical to the one the Python
 *   generator builds.
 * ------------------------------------------------------------------------- */
int64_t gmg_fv_nnz(int n, int dim);
gmg_status gmg_fv_assemble(int n, int dim, const double* kappa, const double* vel_x,
                           const double* vel_y, const double* vel_z, int32_t* rowptr,
                           int32_t* col, double* val, void* stream);

/* gmg_fv_assemble for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that forbid hipMalloc): the same arguments,
 * layout and results (bitwise identical), with no hipMalloc, hipFree or other
 * allocation.  Its only scratch, the block sums of the row-pointer scan, is a
 * static device array of GMG_FV_NOALLOC_SCRATCH_INTS ints (128 KiB) that each
 * GPU the library runs on holds until the process ends; the row counts are
 * formed in rowptr itself.  The first call on a device looks the array up
 * (make it outside graph capture).  Limit: n^dim <= GMG_FV_NOALLOC_MAX_CELLS,
 * else GMG_ERR_INVALID_ARG before any device work.  Unlike gmg_fv_assemble it
 * does not synchronise: the results are complete in the order of `stream`.
 * All calls on one GPU share its array, so calls that overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller. */
#define GMG_FV_NOALLOC_SCRATCH_INTS 32768
#define GMG_FV_NOALLOC_MAX_CELLS 33553407LL
gmg_status gmg_fv_assemble_noalloc(int n, int dim, const double* kappa, const double* vel_x,
                                   const double* vel_y, const double* vel_z, int32_t* rowptr,
                                   int32_t* col, double* val, void* stream);

/* dL/dkappa for L(x(kappa)) given the adjoint lambda = A^{-T} dL/dx and the
 * solution x, nrhs columns (device (N, nrhs) row-major each), summed over the
 * right-hand sides: dL/dkappa_c = -sum_r lambda_r^T (dA/dkappa_c) x_r, with
 * dA/dkappa_c from the discretisation of Eq. (pde) above.  Not in the paper
 * (the gradient of the differentiable solve).  grad: device double[N],
 * overwritten. */
gmg_status gmg_fv_kappa_grad(int n, int dim, const double* kappa, const double* lambda,
                             const double* x, int nrhs, double* grad, void* stream);

/* dL/dA on A's pattern: gval[p] = -sum_r lambda[i(p), r] * x[j(p), r], the
 * gradient of a loss through x = A^{-1} b restricted to the stored entries
 * (not in the paper).  Device arrays: rowptr/col of A (n rows), lambda and x
 * (N, nrhs) row-major, gval double[nnz], overwritten. */
gmg_status gmg_pattern_grad(int64_t n, const int32_t* rowptr, const int32_t* col,
                            const double* lambda, const double* x, int nrhs, double* gval,
                            void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GMG_H */
