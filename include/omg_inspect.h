/*
 * omg_inspect.h -- inspection and timing calls of the OrthoMG library, for
 * tests and benchmarks. Not needed to solve; the conventions of omg.h apply
 * (device pointers unless marked host, cell-major FP64 vectors, every call
 * ordered on the solver's stream, a status returned, nothing thrown).
 */
#ifndef OMG_INSPECT_H
#define OMG_INSPECT_H

#include "omg.h"

#ifdef __cplusplus
extern "C" {
#endif

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
/* Level operations on cell-major device vectors, with the kernels a solve
 * runs: fp32 = 0 in FP64; fp32 = 1 in the single-precision form of the mixed
 * solves (operator, inverses and embedding blocks rounded to float, inputs
 * rounded to float, float arithmetic, results widened to FP64).
 * y = b - A_l x (b nullable: y = A_l x). */
omg_status omg_level_spmv(omg_solver *s, int32_t level, int32_t fp32, const double *x, const double *b, double *y);
/* out = Smoother(A_l, r, 0) with `sweeps` iterations of the solver's
 * smoother: block-Jacobi (Algorithm 4) or additive Schwarz (Algorithm 3). */
omg_status omg_level_smoother(omg_solver *s, int32_t level, int32_t fp32, const double *r, int32_t sweeps,
                              double *out);
/* rc = P_l^T r (level l -> l+1) and z = P_l zc (level l+1 -> l). */
omg_status omg_level_restrict(omg_solver *s, int32_t level, int32_t fp32, const double *r, double *rc);
omg_status omg_level_prolong(omg_solver *s, int32_t level, int32_t fp32, const double *zc, double *z);
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
/* Launch configurations the autotuners chose on a level, host shapes[19]:
 * [0..11] the multi-right-hand-side kernels (tuned on the first batched
 * solve), indexed [op: SpMV, first block-Jacobi iteration, fused iteration]
 * [FP64, FP32][up to 16 columns, 17..32 columns]; shape s in 0..1 is the
 * number of consecutive cells a block of four wavefronts handles for all
 * columns: 16, 8; -1 = not tuned. [12..16] the persistent
 * residual-minimisation kernel (tuned at setup): blocks, vector entries per
 * thread, directions per grid exchange, exchange form (0 all-to-all, 1
 * leader block), compute waves per block of the exchange-wave form (0:
 * plain form), exchanges kept in flight by the lagged form (0: not lagged);
 * -1 if the level does not use it. [18] the number of RM configurations the
 * tuner timed on this level and dropped because a bounded wait expired (a
 * grid that was not resident at once). */
omg_status omg_level_tuning(const omg_solver *s, int32_t level, int32_t *shapes);
omg_status omg_level_multi(omg_solver *s, int32_t level, int32_t op, int32_t nrhs, int32_t sweeps, int32_t fp32,
                           const double *X, const double *B, double *Y);
/* One residual-minimisation step (Algorithm 1 after w = A z) with level l's
 * persistent kernel on caller data: the vectors are flat device arrays of
 * N_l entries (RM has no cell structure); W holds k orthonormal directions
 * as rows of a k x N_l array; cfg (host, nullable) = (blocks, entries per
 * thread, directions per exchange, leader exchange, compute waves, lag)
 * selects one of the co-resident configurations of omg_level_rm_configs
 * (NULL: the tuned one).
 * Outputs: Wk (the new orthonormal direction), r_new, and host
 * coeff[k + 2] = (beta_0..beta_{k-1}, gamma, alpha). The level's own work
 * storage is overwritten. OMG_EUNSUPPORTED if the level does not use the
 * persistent kernel. */
omg_status omg_level_rm_step(omg_solver *s, int32_t level, int32_t k, const double *W, const double *w,
                             const double *z, const double *r, const int32_t *cfg, double *Wk, double *r_new,
                             double *coeff);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step
 * of omg_level_rm_step on caller arrays without a solver. It allocates
 * nothing: all scratch (grid-exchange words, block partials, abort flag, MGS
 * coefficients, the pointer table of W's rows) is one fixed device array of
 * the library, under 512 KB, which each GPU it runs on holds until the
 * process ends. Sizes: 1 <= N <= OMG_NOALLOC_MAX_N entries, 0 <= k <=
 * OMG_NOALLOC_MAX_K stored directions; beyond them (or a NULL or non-finite
 * argument) OMG_EINVAL and nothing is launched.
 * Inputs (device): W, k orthonormal directions as rows of a k x N array; w =
 * A z; z; r. breakdown: the step drops the direction when ||w_out|| <=
 * breakdown ||w_in|| (gamma = alpha = 0, Wk = 0, r_new = r). Outputs: Wk
 * (device, N), r_new (device, N; may be r itself), host coeff[k + 2] =
 * (beta_0..beta_{k-1}, gamma, alpha). Ordered on hip_stream (NULL: default),
 * synchronised before returning; OMG_EHIP if a bounded wait of the kernel
 * expired (results then not trustworthy). Every call on one GPU uses that
 * GPU's single scratch array: calls that overlap in time on one GPU (other
 * host threads, other streams) race and must not be made. */
enum { OMG_NOALLOC_MAX_K = 256, OMG_NOALLOC_MAX_N = 5242880 };
omg_status omg_rm_step_noalloc(int64_t N, int32_t k, const double *W, const double *w, const double *z,
                               const double *r, double breakdown, void *hip_stream, double *Wk, double *r_new,
                               double *coeff);
/* The co-resident launch configurations of level l's persistent RM kernel:
 * host out[6*cap] (blocks, entries per thread, directions per exchange,
 * leader exchange, compute waves: 0 for the plain form, 3 or 4 for the
 * exchange-wave form, where one more wave per block performs the grid
 * exchanges; lag: 1 or 2 for the lagged form, which takes the dot products
 * of each block of directions against w before the previous 1 or 2 blocks'
 * updates and corrects them with stored Gram entries, so that as many
 * exchanges are in flight), their count in *n (out nullable to query the
 * count). */
/* Make level l of this solver use one of its co-resident RM configurations
 * (cfg[6] as in omg_level_rm_configs, host) instead of the tuned one, for the
 * following solves; OMG_EINVAL if cfg is not among them, OMG_EUNSUPPORTED if
 * the level does not use the persistent kernel. */
omg_status omg_level_set_rm_config(omg_solver *s, int32_t level, const int32_t *cfg);
omg_status omg_level_rm_configs(const omg_solver *s, int32_t level, int32_t *out, int32_t cap, int32_t *n);
/* Stored directions of level l after the last solve (device, cell-major,
 * [k][N] each); W or Z nullable. */
omg_status omg_get_dirs(const omg_solver *s, int32_t level, double *W, double *Z);
/* Visit log of the last solve: pairs (level, iterations) in visit order
 * (host out[2*cap]); returns the count through *n. */
omg_status omg_get_visits(const omg_solver *s, int32_t *out, int32_t cap, int32_t *n);
/* Per-visit residual log of the last solve (host out[cap] doubles, count in
 * *n; out nullable to query it): for each level visit in completion order
 * (the order of omg_get_visits) the level, its iterations `it`, ||r0|| and
 * then ||r|| after each of the `it` iterations -- the norms the level tests
 * of Sec. 4.2 compared. */
omg_status omg_get_visit_norms(const omg_solver *s, double *out, int32_t cap, int32_t *n);
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
 * (host pairs (level, iterations), n entries, copied) instead of the level
 * tests: the k-th visit of level l takes the iteration count of the k-th
 * pair of level l (visits beyond the list use the tests); n = 0 switches
 * replay off. Applies to every level, also to the coarse levels a
 * timing-adaptive cycle runs from its second host thread. */
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
#endif /* OMG_INSPECT_H */
