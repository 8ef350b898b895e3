/*
 * omg.h -- C ABI of the MI355X orthonormalization-multigrid (OrthoMG) library.
 *
 * The library solves A x = b for a symmetric positive definite block-sparse
 * A (one dense bs x bs block per cell of a Cartesian grid) with the K-cycle
 * orthonormalization multigrid of the paper: residual minimisation by modified
 * Gram-Schmidt (Algorithm 1, Sec. 3.1) inside the multiplicative cycle
 * (Algorithm 2, Sec. 3.1) or the semi-asynchronous cycle (Algorithm 5, Sec. 4,
 * in a deterministic form), damped block-Jacobi smoothing (Algorithm 4,
 * Sec. 3.3), 2x2x2 agglomeration transfers with Galerkin coarse operators,
 * level-local stopping rules (Sec. 4.2) and a dense Cholesky solve on the
 * coarsest level.
 *
 * Conventions
 *   - Pointers are DEVICE pointers (hipMalloc'd, or torch CUDA tensors) unless
 *     a comment says "host".
 *   - Vectors are FP64 in cell-major DOF order: entry k of cell c is at
 *     c*bs + k. Cells are numbered i + nx*(j + ny*k), x fastest.
 *   - Basis per cell (used by omg_setup_sip and by the transfers): orthonormal
 *     total-degree-p Legendre products h^{-3/2} psi_a psi_b psi_c,
 *     psi_m(t) = sqrt(2m+1) P_m(2t-1), ordered by total degree then (a,b,c)
 *     lexicographically descending: (000),(100),(010),(001),(200),...
 *     bs = (p+1)(p+2)(p+3)/6.
 *   - Every call is ordered on the hip stream given at setup (NULL = default
 *     stream). The host blocks only to read residual norms for stopping tests.
 *   - Every function returns a status and never throws across the ABI.
 *   - One host thread per solver. Solvers are independent.
 */
#ifndef OMG_H
#define OMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OMG_OK = 0,
    OMG_EINVAL = -1,       /* bad argument, malformed matrix, NaN/Inf input */
    OMG_ENOMEM = -2,       /* device or host allocation failed */
    OMG_EHIP = -3,         /* a HIP runtime call failed */
    OMG_ENOTSPD = -4,      /* a diagonal block or the coarsest operator is not SPD */
    OMG_ENOCONV = -5,      /* max_iter reached; x holds the best iterate */
    OMG_EBREAKDOWN = -6,   /* reserved: every direction of a solve broke down */
    OMG_EUNSUPPORTED = -7  /* operation not available for this solver */
} omg_status;

/* cycle variant (the configurations of Table 1): multiplicative synchronous
 * (Algorithm 2, pre- and post-smoothing); additive task-parallel in the
 * deterministic form of Algorithm 5 (coarse correction from the residual at
 * the start of the cycle, computed on a second stream, n_s smoother+RM steps,
 * then RM of the correction); hybrid (Algorithm 2 on the finest level, the
 * Algorithm 5 form on every coarser level, the first coarse level forking);
 * additive synchronous (the Algorithm 5 order on one stream). */
enum { OMG_SYNC_MULT = 0, OMG_OVERLAP_DET = 1, OMG_HYBRID = 2, OMG_ADD_SYNC = 3 };
enum { OMG_FP64 = 0, OMG_MIXED_IR = 1, OMG_MIXED_FLEX = 2 };    /* precision */
/* smoother: damped block-Jacobi (Algorithm 4), or additive Schwarz
 * (Algorithm 3) with one subdomain per cell and an overlap of one cell (the
 * cells its matrix row couples to), local problems solved with inverses
 * formed at setup (single precision in the mixed forms), P <= 2; the same
 * omega damps its sweeps */
enum { OMG_SMOOTH_BJ = 0, OMG_SMOOTH_AS = 1 };
enum { OMG_MAX_LEVELS = 16 };

typedef struct omg_solver omg_solver; /* opaque, library-owned */

/* Cartesian grid and hierarchy: nx*ny*nz cubes of side h, polynomial degree
 * p, n_levels agglomeration levels (level l has nx>>l cells per side; every
 * coarsened side must be even). penalty_c scales the SIP penalty
 * penalty_c (p+1)(p+3)/h (omg_setup_sip only). */
typedef struct {
    int32_t nx, ny, nz, p, n_levels;
    int32_t pad;
    double h, penalty_c;
} omg_grid;

/* Block sparse matrix, HOST pointers: row_ptr[n_cells+1], col_idx[nnzb]
 * (sorted, in range, diagonal present), val[nnzb][bs][bs] row-major FP64.
 * Copied at setup; the caller may free it afterwards. */
typedef struct {
    int32_t n_cells, bs;
    int64_t nnzb;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
} omg_bsr;

typedef struct {
    int32_t variant;      /* OMG_SYNC_MULT, OMG_OVERLAP_DET, OMG_HYBRID or OMG_ADD_SYNC (above);
                             another value: OMG_EINVAL at setup */
    int32_t coarse_sync;  /* OVERLAP_DET, ADD_SYNC: 1 = levels >= 1 run the multiplicative cycle */
    int32_t s_pre;        /* block-Jacobi iterations per pre-smoother call */
    int32_t s_post;       /* block-Jacobi iterations per post-smoother call */
    int32_t n_s;          /* additive levels: smoother+RM steps per cycle (>= 1) */
    int32_t max_iter;     /* finest-level cycles before OMG_ENOCONV */
    int32_t precision;    /* OMG_FP64, OMG_MIXED_IR (FP32 inner + FP64 refinement), OMG_MIXED_FLEX */
    int32_t max_outer;    /* OMG_MIXED_IR: refinement steps */
    int32_t overlap_streams; /* OVERLAP_DET, HYBRID: 1 = coarse path of the forking level on a
                                second stream, 0 = one stream (same results bit for bit) */
    int32_t trace;        /* 1 = record the finest-level residual after every RM (extra syncs) */
    int32_t n_s_max;      /* > n_s: timing-adaptive cycle (Sec. 4.3) on the forking level of
                             OVERLAP_DET / HYBRID with two streams: the smoother side keeps
                             taking smoother+RM steps until the coarse path has finished, at
                             least n_s and at most n_s_max (counts: omg_get_step_counts);
                             results then depend on timing. <= n_s: deterministic */
    int32_t smoother;     /* OMG_SMOOTH_BJ or OMG_SMOOTH_AS (OMG_EUNSUPPORTED for P3); batched
                             solves of such solvers go column by column */
    int32_t m_max;        /* 0: directions grow within a level solve (the paper sets no limit);
                             > 0: a level holding m_max directions restarts before its next RM
                             from x0 = x, r0 = r with W = Z = {} (bounds their storage);
                             batched solves of such solvers go column by column */
    int32_t pad1;
    double omega;         /* block-Jacobi damping */
    double inner_tol;     /* OMG_MIXED_IR: relative tolerance of each inner solve */
    double breakdown;     /* RM drops a direction when ||w_out|| <= breakdown * ||w_in|| */
    double crit_rel[OMG_MAX_LEVELS]; /* level l>=1: stop when ||r|| <= crit_rel[l-1]*||r0|| (<0: off) */
    int32_t crit_max[OMG_MAX_LEVELS];/* level l>=1: stop after crit_max[l-1] iterations */
} omg_options;

typedef struct {
    int32_t status;
    int32_t iters_fine;     /* finest-level cycles (summed over refinement steps) */
    int32_t n_dirs_fine;    /* directions stored on the finest level */
    int32_t n_breakdowns;   /* directions dropped by RM, all levels */
    int32_t outer_iters;    /* OMG_MIXED_IR refinement steps */
    int32_t n_visits;       /* entries in the visit log (omg_get_visits) */
    int32_t n_trace;        /* entries in the residual trace (omg_get_trace) */
    int32_t pad;
    double rel_res_rec;     /* recursive ||r||/||b|| on the finest level */
    double rel_res_true;    /* ||b - A x||/||b|| recomputed in FP64 */
    double t_solve_ms;      /* wall time of the solve (host clock, stream synchronised) */
} omg_report;

/* Defaults: SYNC_MULT, coarse_sync = 0, s_pre = s_post = 1, n_s = 1,
 * n_s_max = 0 (deterministic cycles), omega = 0.7, max_iter = 1000, FP64
 * (max_outer = 50, inner_tol = 1e-5 for MIXED_IR), overlap_streams = 1,
 * trace = 0, block-Jacobi smoother, m_max = 0 (no restarts), level criteria
 * of Sec. 4.2 (level 1: 0.1 or 20 iterations; level 2: 0.5 or 2; deeper: 1
 * iteration), breakdown 1e-14. */
void omg_default_options(omg_options *opt);

/* Setup from an assembled fine operator (Algorithm 2's A). Builds the
 * hierarchy of the grid (2x2x2 agglomeration, P = L2 embedding of coarse
 * polynomials, R = P^T, Galerkin A_{l+1} = P^T A_l P), the block-diagonal
 * inverses of Algorithm 4 and the dense Cholesky factor of the coarsest level.
 * A->bs must equal the basis size of grid->p; A->n_cells = nx*ny*nz.
 * hip_stream: hipStream_t (NULL = default). Errors: OMG_EINVAL (shape,
 * pattern, non-finite values, option values out of range), OMG_EUNSUPPORTED
 * (an option combination this library does not run, e.g. the Schwarz
 * smoother at P3), OMG_ENOTSPD, OMG_ENOMEM, OMG_EHIP. *out is set only on
 * success; the solver owns everything it allocates (omg_destroy). */
omg_status omg_setup(const omg_bsr *A, const omg_grid *grid, const omg_options *opt, void *hip_stream,
                     omg_solver **out);

/* Setup with the operator assembled on the device from a per-cell coefficient
 * nu[n_cells] (DEVICE pointer, FP64, > 0): symmetric interior penalty DG for
 * -div(nu grad u) = f on the grid (Sec. 2), face terms weighted by the
 * harmonic mean 2 nu- nu+ / (nu- + nu+), penalty penalty_c (p+1)(p+3)/h,
 * Nitsche Dirichlet faces weighted by the cell's nu. Enables
 * omg_solve_backward's g_nu. Errors as omg_setup, plus OMG_EINVAL for a
 * non-positive or non-finite nu or h. nu is copied; the caller keeps it. */
omg_status omg_setup_sip(const omg_grid *grid, const double *nu, const omg_options *opt, void *hip_stream,
                         omg_solver **out);

/* (x, r) = MG(A, b, x0) (Algorithm 2 / 5): on entry x holds x0, on exit the
 * solution with ||b - A x|| <= tol ||b|| (recursive residual; the true
 * residual is reported). b is not written. r_out (nullable) receives the
 * final recursive residual. rep (host, nullable) is filled. OMG_ENOCONV
 * leaves the last iterate in x. b = 0 gives x = 0 at once. Errors:
 * OMG_EINVAL (non-finite b or x0, NULL pointers, tol < 0), OMG_ENOCONV,
 * OMG_ENOMEM (direction storage), OMG_EHIP (a runtime failure, or a bounded
 * wait of the persistent RM kernel that expired: the results are then not
 * trustworthy). Calls on one solver must not overlap. */
omg_status omg_solve(omg_solver *s, const double *b, double *x, double tol, double *r_out, omg_report *rep);

/* Batched solve. n_inst solvers (host array s[n_inst]), each with nrhs
 * right-hand sides: b[i], x[i] are device arrays of shape (N_i, nrhs) with
 * the RHS index fastest. Each column is the same solve as omg_solve on that
 * column alone. rep: host array of n_inst*nrhs reports (nullable). Solvers
 * whose options the lockstep engines do not run (Schwarz smoother,
 * timing-adaptive cycles, m_max restarts) are solved column by column.
 * Returns the first failure (as omg_solve), OMG_OK if every column
 * converged. */
omg_status omg_solve_batched(omg_solver *const *s, int32_t n_inst, int32_t nrhs, const double *const *b,
                             double *const *x, double tol, omg_report *rep);

/* Gradient of a scalar loss L(u) with u = A(nu)^-1 f, given u and g_u = dL/du:
 * lambda = A^-1 g_u (adjoint solve on the same hierarchy, A symmetric),
 * g_f = lambda, g_nu[K] = -lambda^T (dA/dnu_K) u (per-cell contraction).
 * g_f, g_nu nullable. g_nu needs a solver from omg_setup_sip
 * (else OMG_EUNSUPPORTED). */
omg_status omg_solve_backward(omg_solver *s, const double *u, const double *g_u, double *g_f, double *g_nu,
                              double tol, omg_report *rep);

void omg_destroy(omg_solver *s);
const char *omg_strerror(omg_status st);

/* ---- inspection (for tests and benchmarks) ------------------------------ */

/* Level sizes: cells, stored blocks per row (ELL width), directions stored. */
omg_status omg_level_info(const omg_solver *s, int32_t level, int32_t *n_cells, int32_t *ell_width,
                          int32_t *k_dirs);
/* Copy level l's operator out in BSR form (host arrays sized from
 * omg_level_info: row_ptr[n+1], col_idx[n*width], val[n*width*bs*bs]);
 * returns the number of stored blocks in *nnzb (explicit zero padding
 * blocks are dropped). */
omg_status omg_level_matrix(const omg_solver *s, int32_t level, int32_t *row_ptr, int32_t *col_idx, double *val,
                            int64_t *nnzb);
/* y = b - A_l x (b nullable: y = A_l x), FP64, cell-major device vectors. */
omg_status omg_level_spmv(omg_solver *s, int32_t level, const double *x, const double *b, double *y);
/* out = Smoother(A_l, r, 0) with `sweeps` iterations of the solver's
 * smoother: block-Jacobi (Algorithm 4) or additive Schwarz (Algorithm 3). */
omg_status omg_level_smoother(omg_solver *s, int32_t level, const double *r, int32_t sweeps, double *out);
/* rc = P_l^T r (level l -> l+1) and z = P_l zc (level l+1 -> l). */
omg_status omg_level_restrict(omg_solver *s, int32_t level, const double *r, double *rc);
omg_status omg_level_prolong(omg_solver *s, int32_t level, const double *zc, double *z);
/* x = A_c^-1 b on the coarsest level. */
omg_status omg_coarse_solve(omg_solver *s, const double *b, double *x);
/* Multi-right-hand-side forms of the level operations, as run inside
 * omg_solve_batched (matrix-core block products): X, B, Y are device arrays
 * of shape (N_l, nrhs), RHS index fastest, cell-major DOFs, 1 <= nrhs <= 32.
 * op OMG_MR_SPMV: Y = A_l X (B null) or Y = B - A_l X; OMG_MR_SMOOTHER:
 * Y = Smoother(A_l, X, 0) with `sweeps` block-Jacobi iterations
 * (Algorithm 4); OMG_MR_COARSE: Y = A_c^-1 X (coarsest level, FP64 only).
 * fp32 = 1 uses the FP32 operator copies (inputs rounded to FP32, FP32
 * arithmetic, results widened to FP64). OMG_EUNSUPPORTED for bs > 16. */
enum { OMG_MR_SPMV = 0, OMG_MR_SMOOTHER = 1, OMG_MR_COARSE = 2 };
/* Launch configurations the autotuners chose on a level, host shapes[17]:
 * [0..11] the multi-right-hand-side kernels (tuned on the first batched
 * solve), indexed [op: SpMV, first block-Jacobi iteration, fused iteration]
 * [FP64, FP32][up to 16 columns, 17..32 columns]; shape s in 0..5 is
 * (wavefronts per block, 16-column tiles per wavefront) = (4,2), (2,2),
 * (1,2), (4,1), (2,1), (1,1); -1 = not tuned. [12..16] the persistent
 * residual-minimisation kernel (tuned at setup): blocks, vector entries per
 * thread, directions per grid exchange, exchange form (0 all-to-all, 1
 * leader block), compute waves per block of the exchange-wave form (0:
 * plain form); -1 if the level does not use it. */
omg_status omg_level_tuning(const omg_solver *s, int32_t level, int32_t *shapes);
omg_status omg_level_multi(omg_solver *s, int32_t level, int32_t op, int32_t nrhs, int32_t sweeps, int32_t fp32,
                           const double *X, const double *B, double *Y);
/* One residual-minimisation step (Algorithm 1 after w = A z) with level l's
 * persistent kernel on caller data: the vectors are flat device arrays of
 * N_l entries (RM has no cell structure); W holds k orthonormal directions
 * as rows of a k x N_l array; cfg (host, nullable) = (blocks, entries per
 * thread, directions per exchange, leader exchange, compute waves) selects
 * one of the co-resident configurations of omg_level_rm_configs (NULL: the
 * tuned one).
 * Outputs: Wk (the new orthonormal direction), r_new, and host
 * coeff[k + 2] = (beta_0..beta_{k-1}, gamma, alpha). The level's own work
 * storage is overwritten. OMG_EUNSUPPORTED if the level does not use the
 * persistent kernel. */
omg_status omg_level_rm_step(omg_solver *s, int32_t level, int32_t k, const double *W, const double *w,
                             const double *z, const double *r, const int32_t *cfg, double *Wk, double *r_new,
                             double *coeff);
/* The co-resident launch configurations of level l's persistent RM kernel:
 * host out[5*cap] (blocks, entries per thread, directions per exchange,
 * leader exchange, compute waves: 0 for the plain form, 3 or 4 for the
 * exchange-wave form, where one more wave per block performs the grid
 * exchanges), their count in *n (out nullable to query the count). */
omg_status omg_level_rm_configs(const omg_solver *s, int32_t level, int32_t *out, int32_t cap, int32_t *n);
/* Stored directions of level l after the last solve (device, cell-major,
 * [k][N] each); W or Z nullable. */
omg_status omg_get_dirs(const omg_solver *s, int32_t level, double *W, double *Z);
/* Visit log of the last solve: pairs (level, iterations) in visit order
 * (host out[2*cap]); returns the count through *n. */
omg_status omg_get_visits(const omg_solver *s, int32_t *out, int32_t cap, int32_t *n);
/* Residual trace of the last solve (needs opt.trace): triples
 * (step, ||r||, type: 0 initial, 1 smoother, 2 coarse, 3 final), host. */
omg_status omg_get_trace(const omg_solver *s, double *out, int32_t cap, int32_t *n);
/* Smoother+RM steps taken in each cycle of the forking level during the
 * last solve (OVERLAP_DET: the finest level; HYBRID: level 1), in execution
 * order, into host out[cap] (caller-owned; at most cap written); count in *n
 * (out nullable to query it). n_s each unless the cycle was timing-adaptive
 * (adaptive loops, Sec. 4.3), where replaying these counts reproduces the
 * solve. OMG_EINVAL for a NULL solver or n. */
omg_status omg_get_step_counts(const omg_solver *s, int32_t *out, int32_t cap, int32_t *n);
/* Replay: make the next solve(s) use these per-visit iteration counts
 * (host pairs (level, iterations), n entries) instead of the level tests;
 * n = 0 switches replay off. */
omg_status omg_set_replay(omg_solver *s, const int32_t *visits, int32_t n);

/* ---- kernel timing (benchmarks) -------------------------------------- */
enum {
    OMG_K_SPMV = 0,      /* w = A z, block SpMV of one level (FP64) */
    OMG_K_SPMV32 = 1,    /* the same with the FP32 operator */
    OMG_K_BJ = 2,        /* fused block-Jacobi iteration x' = x + omega D^-1 (r - A x) (FP64) */
    OMG_K_BJ32 = 3,      /* the same in FP32 */
    OMG_K_MGS = 4,       /* one modified Gram-Schmidt step of residual minimisation */
    OMG_K_RESTRICT = 5,  /* r_c = P^T r */
    OMG_K_PROLONG = 6,   /* z = P z_c */
    OMG_K_COARSE = 7,    /* coarsest-level solve (dense inverse GEMV) */
    OMG_K_RMFIN = 8,     /* RM normalisation + update (two kernels) */
    OMG_K_BJFIRST = 9,   /* first block-Jacobi iteration from zero, x = omega D^-1 r */
    OMG_K_RMP = 10,      /* persistent residual minimisation (whole MGS loop + update, one launch) */
    OMG_K_COPY = 11,     /* plain copy of one level vector (reference for traffic counters) */
    OMG_K_COUNT = 12
};
/* Launch kernel `kind` of level `level` `reps` times on the solver's stream
 * between two HIP events (inputs are the level's work buffers, filled with
 * finite data); *avg_ms = mean duration per launch, *alg_bytes = the bytes
 * the operation must move per launch (operator values and column indices of
 * the stored blocks, each vector read or written once). */
omg_status omg_bench_kernel(omg_solver *s, int32_t kind, int32_t level, int32_t reps, double *avg_ms,
                            double *alg_bytes);
/* Arm a probe: during the following solves, every launch of kernel `kind` on
 * `level` (up to max_launches) is bracketed by HIP events on the stream it is
 * launched on. omg_probe_result returns the number of timed launches, their
 * mean duration and the algorithmic bytes per launch, and disarms the probe. */
omg_status omg_probe_kernel(omg_solver *s, int32_t kind, int32_t level, int32_t max_launches);
omg_status omg_probe_result(omg_solver *s, int64_t *launches, double *avg_ms, double *alg_bytes);
/* Launch counts of the last solve(s) since the previous call, per kernel kind
 * and level: host out[OMG_K_COUNT][OMG_MAX_LEVELS]; counters are reset. */
omg_status omg_get_kernel_counts(omg_solver *s, int64_t *out);

#ifdef __cplusplus
}
#endif
#endif /* OMG_H */
