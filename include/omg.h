/*
 * omg.h -- C ABI of the MI355X orthonormalization-multigrid (OrthoMG) library.
 *
 * The library solves A x = b for a symmetric positive definite block-sparse
 * A (one dense bs x bs block per pair of coupled cells) with the K-cycle
 * orthonormalization multigrid of the paper: residual minimisation by modified
 * Gram-Schmidt (Algorithm 1, Sec. 3.1) inside the multiplicative cycle
 * (Algorithm 2, Sec. 3.1) or the semi-asynchronous cycle (Algorithm 5, Sec. 4,
 * in a deterministic form), damped block-Jacobi smoothing (Algorithm 4,
 * Sec. 3.3), agglomeration transfers with Galerkin coarse operators,
 * level-local stopping rules (Sec. 4.2) and a dense Cholesky solve on the
 * coarsest level.
 *
 * Conventions
 *   - Pointers are DEVICE pointers (hipMalloc'd, or torch CUDA tensors) unless
 *     a comment says "host".
 *   - Vectors are FP64 in cell-major DOF order: entry k of cell c is at
 *     c*bs + k. On a Cartesian grid cells are numbered i + nx*(j + ny*k),
 *     x fastest.
 *   - Basis per cell (used by omg_setup_sip and by the transfers): orthonormal
 *     total-degree-p Legendre products h^{-3/2} psi_a psi_b psi_c,
 *     psi_m(t) = sqrt(2m+1) P_m(2t-1), ordered by total degree then (a,b,c)
 *     lexicographically descending: (000),(100),(010),(001),(200),...
 *     bs = (p+1)(p+2)(p+3)/6.
 *   - Every call is ordered on the hip stream given at setup (NULL = default
 *     stream). The host blocks only to read residual norms for stopping tests.
 *   - Every function returns a status and never throws across the ABI.
 *   - One host thread per solver. Solvers are independent.
 *   - Inspection and timing calls used by tests and benchmarks are declared
 *     in omg_inspect.h.
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

/* Cartesian grid: nx*ny*nz cubes of side h, polynomial degree p; n_levels
 * levels of its 2x2x2 agglomeration (level l has nx>>l cells per side; every
 * coarsened side must be even) when no hierarchy is given. penalty_c scales
 * the SIP penalty penalty_c (p+1)(p+3)/h (omg_setup_sip only). */
typedef struct {
    int32_t nx, ny, nz, p, n_levels;
    int32_t pad;
    double h, penalty_c;
} omg_grid;

/* Agglomeration hierarchy (the restriction R and prolongation P of
 * Algorithm 2, Sec. 3.1), HOST pointers, copied at setup. Level l+1's cells
 * are unions of level l's cells: parent[l][K] (0 <= parent < n_cells[l+1])
 * is the coarse cell containing cell K of level l, and slot[l][K] (0..7)
 * selects the embedding block E_slot, a bs x bs row-major block of
 * embed[8][bs][bs] that maps a coarse cell's basis coefficients to those of
 * its finer cell K. P_l has block E_{slot(K)} at (K, parent(K)), R_l = P_l^T,
 * and the coarse operators are A_{l+1} = P_l^T A_l P_l (Galerkin). Every
 * coarse cell needs at least one finer cell; it may have fewer than eight
 * (sides of odd length). n_levels = 1: the direct solve on the operator.
 * For the 2x2x2 agglomeration of a Cartesian grid, omg_grid_hierarchy and
 * omg_embedding fill these arrays. */
typedef struct {
    int32_t n_levels;
    int32_t pad;
    const int32_t *n_cells;        /* host [n_levels] */
    const int32_t *const *parent;  /* host [n_levels-1] arrays of n_cells[l] entries */
    const uint8_t *const *slot;    /* host [n_levels-1] arrays of n_cells[l] entries */
    const double *embed;           /* host [8][bs][bs] */
} omg_hierarchy;

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
    double breakdown;     /* RM drops a direction when ||w_out|| <= breakdown * ||w_in||: its slot
                             is stored as a zero vector (x, r unchanged) and still counts as a
                             stored direction (toward m_max and n_dirs_fine) */
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

/* The 2x2x2 agglomeration of the Cartesian grid g: for level < g->n_levels-1,
 * parent[K] and slot[K] (host, n_cells(level) = (nx>>level)(ny>>level)(nz>>level)
 * entries each) of every cell K = i + nx_l (j + ny_l k) of that level: parent
 * (i/2, j/2, k/2) on level+1, slot (i&1) + 2(j&1) + 4(k&1). Every coarsened
 * side must be even (else OMG_EINVAL). */
omg_status omg_grid_hierarchy(const omg_grid *g, int32_t level, int32_t *parent, uint8_t *slot);

/* The eight embedding blocks of the library's orthonormal Legendre basis of
 * degree p (0..3) on a cube and its 2x2x2 children: E[s][i][j] = L2 inner
 * product of child basis function i (child s, normalised on the child) with
 * coarse basis function j (host E[8][bs][bs]). */
omg_status omg_embedding(int32_t p, double *E);

/* Setup from an assembled fine operator A (Algorithm 2's A) and an
 * agglomeration hierarchy H (both host memory, copied; the caller may free
 * them afterwards). Builds the Galerkin coarse operators P^T A P, the
 * block-diagonal inverses of Algorithm 4 and the dense factor of the
 * coarsest level. A->bs must be 1, 4, 10 or 20 (the total-degree bases of
 * P0..P3) and H->n_cells[0] = A->n_cells. hip_stream: hipStream_t (NULL =
 * default). Errors: OMG_EINVAL (shape, pattern, non-finite values, maps out
 * of range, a coarse cell with no finer cell, option values out of range),
 * OMG_EUNSUPPORTED (a block size or option combination this library does not
 * run, e.g. the Schwarz smoother at P3), OMG_ENOTSPD, OMG_ENOMEM, OMG_EHIP.
 * *out is set only on success; the solver owns everything it allocates
 * (omg_destroy). */
omg_status omg_setup(const omg_bsr *A, const omg_hierarchy *H, const omg_options *opt, void *hip_stream,
                     omg_solver **out);

/* Setup with the operator assembled on the device from a per-cell coefficient
 * nu[n_cells] (DEVICE pointer, FP64, > 0): symmetric interior penalty DG for
 * -div(nu grad u) = f on the grid (Sec. 2), face terms weighted by the
 * harmonic mean 2 nu- nu+ / (nu- + nu+), penalty penalty_c (p+1)(p+3)/h,
 * Nitsche Dirichlet faces weighted by the cell's nu. H (nullable) is the
 * hierarchy; NULL takes the grid's 2x2x2 agglomeration with grid->n_levels
 * levels, and an H with embed = NULL takes omg_embedding(grid->p). Enables
 * omg_solve_backward's g_nu. Errors as omg_setup, plus OMG_EINVAL for a
 * non-positive or non-finite nu or h. nu is copied; the caller keeps it. */
omg_status omg_setup_sip(const omg_grid *grid, const double *nu, const omg_hierarchy *H, const omg_options *opt,
                         void *hip_stream, omg_solver **out);

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
 * lambda = A^-1 g_u (adjoint solve on the same hierarchy, A symmetric,
 * tolerance tol), g_f = lambda, g_nu[K] = -lambda^T (dA/dnu_K) u (per-cell
 * contraction). g_f, g_nu nullable (device, N and n_cells entries). g_nu
 * needs a solver from omg_setup_sip (else OMG_EUNSUPPORTED). If the adjoint
 * solve does not converge, OMG_ENOCONV is returned and g_f, g_nu are not
 * written. Errors otherwise as omg_solve. */
omg_status omg_solve_backward(omg_solver *s, const double *u, const double *g_u, double *g_f, double *g_nu,
                              double tol, omg_report *rep);

void omg_destroy(omg_solver *s);
const char *omg_strerror(omg_status st);

#ifdef __cplusplus
}
#endif
#endif /* OMG_H */
