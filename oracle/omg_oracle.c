/*
 * omg_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for the
 * orthonormalization-multigrid (OrthoMG) solve.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library. It shares no code with the GPU
 * library: its own basis, quadrature, assembly, Galerkin product, smoother,
 * residual minimisation and dense Cholesky are written here from the paper and
 * from textbook definitions.
 *
 * What it follows:
 *   - residual minimisation: Algorithm 1 (Sec. 3.1), modified Gram-Schmidt of
 *     w = A z against the stored orthonormal W with the same coefficients
 *     applied to z, normalisation, append, alpha = w . r, x += alpha z,
 *     r -= alpha w;
 *   - multiplicative synchronous OrthoMG: Algorithm 2 (Sec. 3.1) with the
 *     level-local stopping rules of Sec. 4.2;
 *   - block-Jacobi smoother: Algorithm 4 (Sec. 3.3) with precomputed block
 *     inverses, started from zero, a fixed number of sweeps;
 *   - additive Schwarz smoother: Algorithm 3 (Sec. 3.2) with one subdomain
 *     per cell and an overlap of one cell (the cells its matrix row couples
 *     to), local problems solved with stored Cholesky factors, corrections
 *     summed, damped by omega like the block-Jacobi sweeps; in the mixed
 *     forms the local solves are single precision (the patch inverse formed
 *     in FP64 and rounded, the local residual rounded, products summed in
 *     float), as the paper does;
 *   - semi-asynchronous OrthoMG, Algorithm 5 (Sec. 4), in a deterministic form:
 *     the coarse correction is computed from a snapshot of r taken at the start
 *     of the cycle, the smoother side runs a fixed number of smoother+RM steps,
 *     then RM of the coarse correction; executed sequentially here, which is
 *     also the additive synchronous configuration of Table 1;
 *   - the hybrid configuration of Table 1: Algorithm 2 (pre- and
 *     post-smoothing, multiplicative) on the finest level and the Algorithm 5
 *     form on every coarser level;
 *   - the adaptive loops of Sec. 4.3 choose the number of smoother steps per
 *     cycle by timing; the oracle takes such counts as an input (a schedule
 *     for the cycles of the level whose coarse path runs concurrently: the
 *     finest level for variant 1, level 1 for variant 2) and otherwise runs
 *     n_s steps;
 *   - coarsest level: direct solve (dense Cholesky);
 *   - discretisation: symmetric interior penalty DG (Sec. 2) on a Cartesian
 *     grid, weighted (harmonic-mean) face coefficient, Nitsche Dirichlet
 *     boundary, orthonormal total-degree Legendre basis; element matrices by
 *     tensor Gauss-Legendre quadrature;
 *   - hierarchy: 2x2x2 agglomeration, P = L2 embedding of coarse polynomials
 *     into the children, R = P^T, A_c = P^T A P.
 *
 * A direction that breaks down in residual minimisation (its orthogonalised
 * w is at most `breakdown` times the w it started from) is dropped: its slot
 * is stored as a zero vector, which leaves x and r exactly as discarding it
 * would and counts it among the level's stored directions (the restart limit
 * m_max and the reported direction count see it).
 *
 * Every floating-point operation is FP64 except the optional FP32 emulation of
 * the mixed-precision forms, which rounds operands and results to float.
 * Dot products are plain sequential sums. Row-wise loops (SpMV, smoother,
 * transfers, vector updates) are OpenMP-parallel; each row is computed by one
 * thread in a fixed order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ENOTSPD (-4)
#define OR_ENOCONV (-5)
#define OR_EUNSUPPORTED (-7)

#define MAXLEV 16

/* ------------------------------------------------------------------------- */
/* Options and report (mirrored by the ctypes wrapper)                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int variant;       /* 0: multiplicative synchronous (Alg. 2); 1: deterministic semi-async (Alg. 5);
                          2: hybrid (Alg. 2 on the finest level, Alg. 5 below; Table 1);
                          3: additive synchronous (Table 1; the Alg. 5 order, which this
                          sequential code runs for variant 1 as well) */
    int coarse_sync;   /* variants 1, 3: 1 = levels >= 1 use Alg. 2 instead of the Alg. 5 form */
    int s_pre;         /* block-Jacobi iterations of the pre-smoother call */
    int s_post;        /* block-Jacobi iterations of the post-smoother call */
    int n_s;           /* variant 1: smoother+RM steps per cycle on the smoother side */
    int max_iter;      /* finest level: maximum cycles */
    int precision;     /* 0 FP64; 1 FP32-inner iterative refinement; 2 flexible (A64 in fine RM) */
    int gs;            /* 0 MGS; 1 MGS with one DGKS re-orthogonalisation pass */
    int alpha_mode;    /* 0: alpha = w.r (current residual); 1: literal alpha = w.r0, x = x0 + Z alpha */
    int m_max;         /* 0 unbounded; else restart the level's W,Z when they hold m_max columns */
    int max_outer;     /* precision 1: maximum refinement steps */
    int n_crit;        /* number of entries used in crit_rel/crit_max (levels 1..n_crit) */
    int smoother;      /* 0 block-Jacobi (Alg. 4); 1 additive Schwarz (Alg. 3) */
    int pad_smoother;
    double omega;      /* block-Jacobi damping */
    double inner_tol;  /* precision 1: relative tolerance of each inner solve */
    double breakdown;  /* RM discards a direction when ||w_out|| <= breakdown * ||w_in|| */
    double crit_rel[MAXLEV]; /* level l>=1: stop when ||r|| <= crit_rel[l-1] * ||r0|| (<0: off) */
    int crit_max[MAXLEV];    /* level l>=1: stop when it >= crit_max[l-1] */
} or_opts;

typedef struct {
    int status;
    int iters_fine;     /* cycles on the finest level (summed over refinement steps) */
    int n_dirs_fine;    /* directions stored on the finest level at exit */
    int n_breakdowns;   /* directions discarded by RM on any level */
    int outer_iters;    /* refinement steps (precision 1) */
    int n_visits;       /* entries in the visit log */
    int n_trace;        /* entries in the finest-level residual trace */
    int n_vnorm;        /* doubles in the per-visit residual log */
    double rel_res_rec; /* ||r|| / ||b|| of the recursive residual (fine level) */
    double rel_res_true;/* ||b - A x|| / ||b|| recomputed in FP64 */
} or_report;

/* ------------------------------------------------------------------------- */
/* 1D Legendre basis on [0,1]: psi_m(t) = sqrt(2m+1) P_m(2t-1)                */
/* ------------------------------------------------------------------------- */
static double leg(int m, double s) {
    double p0 = 1.0, p1 = s;
    if (m == 0) return p0;
    for (int n = 1; n < m; ++n) {
        double p2 = ((2.0 * n + 1.0) * s * p1 - n * p0) / (n + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}
/* P'_{n+1}(s) = (n+1) P_n(s) + s P'_n(s) */
static double dleg(int m, double s) {
    double d = 0.0;
    for (int n = 0; n < m; ++n) d = (n + 1.0) * leg(n, s) + s * d;
    return d;
}
static double psi1(int m, double t) { return sqrt(2.0 * m + 1.0) * leg(m, 2.0 * t - 1.0); }
static double dpsi1(int m, double t) { return sqrt(2.0 * m + 1.0) * 2.0 * dleg(m, 2.0 * t - 1.0); }

/* Gauss-Legendre nodes/weights on [0,1] (Newton iteration on P_q). */
static void gauss01(int q, double *x, double *w) {
    for (int i = 0; i < q; ++i) {
        double s = cos(M_PI * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double ds = leg(q, s) / dleg(q, s);
            s -= ds;
            if (fabs(ds) < 1e-16) break;
        }
        double d = dleg(q, s);
        x[i] = 0.5 * (s + 1.0);
        w[i] = 0.5 * 2.0 / ((1.0 - s * s) * d * d);
    }
}

/* Basis ordering: by total degree, then (a,b,c) lexicographically descending:
 * (000),(100),(010),(001),(200),(110),(101),(020),(011),(002),... */
static int basis_index(int p, int (*abc)[3]) {
    int n = 0;
    for (int d = 0; d <= p; ++d)
        for (int a = d; a >= 0; --a)
            for (int b = d - a; b >= 0; --b) {
                abc[n][0] = a;
                abc[n][1] = b;
                abc[n][2] = d - a - b;
                ++n;
            }
    return n;
}

int oracle_nbasis(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

/* phi_m on a cube of side h with lower corner at the origin:
 * phi(x) = h^{-3/2} prod_d psi(x_d/h); grad component d gets an extra 1/h. */
static double phi_val(const int *m, double h, const double *x) {
    return pow(h, -1.5) * psi1(m[0], x[0] / h) * psi1(m[1], x[1] / h) * psi1(m[2], x[2] / h);
}
static double phi_grad(const int *m, double h, const double *x, int d) {
    double v = pow(h, -1.5) / h;
    for (int e = 0; e < 3; ++e) v *= (e == d) ? dpsi1(m[e], x[e] / h) : psi1(m[e], x[e] / h);
    return v;
}

/* ------------------------------------------------------------------------- */
/* Element matrices for unit coefficient (SIP, weighted-average reading)      */
/* ------------------------------------------------------------------------- */
typedef struct {
    int p, bs;
    double h, sigma;
    double *S;          /* [bs*bs] volume: int grad phi_n . grad phi_m */
    double *F[3][2][2]; /* interior face normal +e_d: F[d][X][Y] test in X, trial in Y; X,Y: 0 = lower cell, 1 = upper cell */
    double *B[3][2];    /* boundary face normal direction d, side 0 = low (outward -e_d), 1 = high */
} elem_t;

static void elem_free(elem_t *E) {
    free(E->S);
    for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 2; ++a) {
            free(E->B[d][a]);
            for (int b = 0; b < 2; ++b) free(E->F[d][a][b]);
        }
}

/* Unit-coefficient bilinear form pieces (row = test m, col = trial n):
 *   volume:   int_K grad u . grad v
 *   interior: - int_F {du/dn}[v] - int_F {dv/dn}[u] + sigma int_F [u][v]
 *   boundary: - int_F (du/dn) v - int_F (dv/dn) u + sigma int_F u v
 * with [u] = u_lower - u_upper, {g} = (g_lower + g_upper)/2, n = +e_d on an
 * interior face, outward on a boundary face. */
static int elem_build(elem_t *E, int p, double h, double penalty_c) {
    int abc[64][3];
    int bs = basis_index(p, abc);
    int q = p + 2;
    double xq[16], wq[16];
    gauss01(q, xq, wq);
    memset(E, 0, sizeof(*E));
    E->p = p;
    E->bs = bs;
    E->h = h;
    E->sigma = penalty_c * (p + 1.0) * (p + 3.0) / h;
    E->S = calloc((size_t)bs * bs, sizeof(double));
    if (!E->S) return OR_ENOMEM;
    for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 2; ++a) {
            E->B[d][a] = calloc((size_t)bs * bs, sizeof(double));
            for (int b = 0; b < 2; ++b) E->F[d][a][b] = calloc((size_t)bs * bs, sizeof(double));
        }
    /* volume */
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k) {
                double x[3] = {xq[i] * h, xq[j] * h, xq[k] * h};
                double wt = wq[i] * wq[j] * wq[k] * h * h * h;
                for (int m = 0; m < bs; ++m)
                    for (int n = 0; n < bs; ++n) {
                        double g = 0.0;
                        for (int d = 0; d < 3; ++d) g += phi_grad(abc[n], h, x, d) * phi_grad(abc[m], h, x, d);
                        E->S[m * bs + n] += wt * g;
                    }
            }
    /* faces */
    for (int d = 0; d < 3; ++d) {
        int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
                double wt = wq[i] * wq[j] * h * h;
                /* point on the face in the lower cell's frame (x_d = h) and the
                 * upper cell's frame (x_d = 0) */
                double xl[3], xu[3];
                xl[t1] = xu[t1] = xq[i] * h;
                xl[t2] = xu[t2] = xq[j] * h;
                xl[d] = h;
                xu[d] = 0.0;
                for (int m = 0; m < bs; ++m)
                    for (int n = 0; n < bs; ++n) {
                        for (int X = 0; X < 2; ++X)
                            for (int Y = 0; Y < 2; ++Y) {
                                const double *xv = X ? xu : xl, *xu_ = Y ? xu : xl;
                                double v = phi_val(abc[m], h, xv), dv = phi_grad(abc[m], h, xv, d);
                                double u = phi_val(abc[n], h, xu_), du = phi_grad(abc[n], h, xu_, d);
                                double sv = X ? -1.0 : 1.0, su = Y ? -1.0 : 1.0; /* jump signs */
                                double val = -0.5 * du * (sv * v) - 0.5 * dv * (su * u) + E->sigma * (su * u) * (sv * v);
                                E->F[d][X][Y][m * bs + n] += wt * val;
                            }
                        /* boundary: low side (x_d = 0, outward -e_d), high side (x_d = h, +e_d) */
                        for (int side = 0; side < 2; ++side) {
                            const double *xb = side ? xl : xu; /* xl has x_d = h, xu has x_d = 0 */
                            double nsg = side ? 1.0 : -1.0;
                            double v = phi_val(abc[m], h, xb), dv = nsg * phi_grad(abc[m], h, xb, d);
                            double u = phi_val(abc[n], h, xb), du = nsg * phi_grad(abc[n], h, xb, d);
                            E->B[d][side][m * bs + n] += wt * (-du * v - dv * u + E->sigma * u * v);
                        }
                    }
            }
    }
    return OR_OK;
}

/* Harmonic-mean face coefficient and its derivative w.r.t. the first argument. */
static double nu_face(double a, double b) { return 2.0 * a * b / (a + b); }
static double dnu_face(double a, double b) { return 2.0 * b * b / ((a + b) * (a + b)); }

/* ------------------------------------------------------------------------- */
/* Block sparse matrix                                                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n, bs;
    int64_t nnzb;
    int *row_ptr, *col;
    double *val; /* [nnzb][bs][bs] row-major */
} bsr_t;

static void bsr_free(bsr_t *A) {
    free(A->row_ptr);
    free(A->col);
    free(A->val);
    memset(A, 0, sizeof(*A));
}

static int64_t bsr_find(const bsr_t *A, int i, int j) {
    for (int64_t q = A->row_ptr[i]; q < A->row_ptr[i + 1]; ++q)
        if (A->col[q] == j) return q;
    return -1;
}

/* 7-point stencil pattern of an nx*ny*nz grid, sorted columns. */
static int stencil_pattern(bsr_t *A, int nx, int ny, int nz, int bs) {
    int n = nx * ny * nz;
    A->n = n;
    A->bs = bs;
    A->row_ptr = malloc(sizeof(int) * (n + 1));
    if (!A->row_ptr) return OR_ENOMEM;
    int64_t cnt = 0;
    A->row_ptr[0] = 0;
    for (int c = 0; c < n; ++c) {
        int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        cnt += 1 + (i > 0) + (i < nx - 1) + (j > 0) + (j < ny - 1) + (k > 0) + (k < nz - 1);
        A->row_ptr[c + 1] = (int)cnt;
    }
    A->nnzb = cnt;
    A->col = malloc(sizeof(int) * cnt);
    A->val = calloc((size_t)cnt * bs * bs, sizeof(double));
    if (!A->col || !A->val) return OR_ENOMEM;
    for (int c = 0; c < n; ++c) {
        int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        int q = A->row_ptr[c];
        if (k > 0) A->col[q++] = c - nx * ny;
        if (j > 0) A->col[q++] = c - nx;
        if (i > 0) A->col[q++] = c - 1;
        A->col[q++] = c;
        if (i < nx - 1) A->col[q++] = c + 1;
        if (j < ny - 1) A->col[q++] = c + nx;
        if (k < nz - 1) A->col[q++] = c + nx * ny;
    }
    return OR_OK;
}

static void blk_axpy(double *dst, double s, const double *src, int bs) {
    for (int t = 0; t < bs * bs; ++t) dst[t] += s * src[t];
}

/* Assemble A(nu): sum over cells nu_K S, interior faces nu_F F, boundary faces nu_K B. */
static int assemble(bsr_t *A, const elem_t *E, int nx, int ny, int nz, const double *nu) {
    int rc = stencil_pattern(A, nx, ny, nz, E->bs);
    if (rc) return rc;
    int bs = E->bs, n = nx * ny * nz;
    int stride[3] = {1, nx, nx * ny};
    int dims[3] = {nx, ny, nz};
    for (int c = 0; c < n; ++c) {
        int ijk[3] = {c % nx, (c / nx) % ny, c / (nx * ny)};
        double *Acc = A->val + (size_t)bsr_find(A, c, c) * bs * bs;
        blk_axpy(Acc, nu[c], E->S, bs);
        for (int d = 0; d < 3; ++d) {
            /* face towards +e_d: this cell is the lower cell */
            if (ijk[d] < dims[d] - 1) {
                int u = c + stride[d];
                double nf = nu_face(nu[c], nu[u]);
                blk_axpy(Acc, nf, E->F[d][0][0], bs);
                blk_axpy(A->val + (size_t)bsr_find(A, c, u) * bs * bs, nf, E->F[d][0][1], bs);
            } else {
                blk_axpy(Acc, nu[c], E->B[d][1], bs);
            }
            /* face towards -e_d: this cell is the upper cell */
            if (ijk[d] > 0) {
                int l = c - stride[d];
                double nf = nu_face(nu[l], nu[c]);
                blk_axpy(Acc, nf, E->F[d][1][1], bs);
                blk_axpy(A->val + (size_t)bsr_find(A, c, l) * bs * bs, nf, E->F[d][1][0], bs);
            } else {
                blk_axpy(Acc, nu[c], E->B[d][0], bs);
            }
        }
    }
    return OR_OK;
}

/* y = A x (or y = b - A x when b != NULL). Row-parallel. */
static void spmv(const bsr_t *A, const double *x, const double *b, double *y) {
    int bs = A->bs;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < A->n; ++i) {
        double acc[64];
        for (int r = 0; r < bs; ++r) acc[r] = 0.0;
        for (int q = A->row_ptr[i]; q < A->row_ptr[i + 1]; ++q) {
            const double *blk = A->val + (size_t)q * bs * bs;
            const double *xj = x + (size_t)A->col[q] * bs;
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < bs; ++c) acc[r] += blk[r * bs + c] * xj[c];
        }
        for (int r = 0; r < bs; ++r) y[(size_t)i * bs + r] = b ? b[(size_t)i * bs + r] - acc[r] : acc[r];
    }
}

/* FP32 emulation: matrix entries pre-rounded to float (val32); x rounded to
 * float; products and sums in float. */
static void spmv32(const bsr_t *A, const float *val32, const double *x, const double *b, double *y) {
    int bs = A->bs;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < A->n; ++i) {
        float acc[64];
        for (int r = 0; r < bs; ++r) acc[r] = 0.0f;
        for (int q = A->row_ptr[i]; q < A->row_ptr[i + 1]; ++q) {
            const float *blk = val32 + (size_t)q * bs * bs;
            const double *xj = x + (size_t)A->col[q] * bs;
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < bs; ++c) acc[r] += blk[r * bs + c] * (float)xj[c];
        }
        for (int r = 0; r < bs; ++r) {
            size_t o = (size_t)i * bs + r;
            y[o] = b ? (double)((float)b[o] - acc[r]) : (double)acc[r];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Small dense helpers                                                        */
/* ------------------------------------------------------------------------- */
static double dot(const double *a, const double *b, size_t n) {
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}
static double nrm2(const double *a, size_t n) { return sqrt(dot(a, a, n)); }

/* Cholesky A = L L^T of an n x n row-major SPD matrix (in place, lower part).
 * Returns OR_ENOTSPD on a non-positive pivot. */
static int chol_factor(double *L, int n, int parallel) {
    for (int j = 0; j < n; ++j) {
        double *Lj = L + (size_t)j * n;
        double d = Lj[j] - dot(Lj, Lj, (size_t)j);
        if (!(d > 0.0)) return OR_ENOTSPD;
        Lj[j] = sqrt(d);
        double ljj = Lj[j];
        if (parallel) {
#pragma omp parallel for schedule(static)
            for (int i = j + 1; i < n; ++i) {
                double *Li = L + (size_t)i * n;
                Li[j] = (Li[j] - dot(Li, Lj, (size_t)j)) / ljj;
            }
        } else {
            for (int i = j + 1; i < n; ++i) {
                double *Li = L + (size_t)i * n;
                Li[j] = (Li[j] - dot(Li, Lj, (size_t)j)) / ljj;
            }
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) L[(size_t)i * n + j] = 0.0;
    return OR_OK;
}

/* Solve L L^T x = b. */
static void chol_solve(const double *L, int n, const double *b, double *x) {
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * x[k];
        x[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
        x[i] = s / L[(size_t)i * n + i];
    }
}

/* Inverse of a small SPD block via Cholesky: solve A X = I column by column. */
static int spd_inverse(const double *A, int bs, double *Ainv) {
    double L[64 * 64], e[64], x[64];
    memcpy(L, A, sizeof(double) * bs * bs);
    if (chol_factor(L, bs, 0)) return OR_ENOTSPD;
    for (int c = 0; c < bs; ++c) {
        for (int r = 0; r < bs; ++r) e[r] = (r == c) ? 1.0 : 0.0;
        chol_solve(L, bs, e, x);
        for (int r = 0; r < bs; ++r) Ainv[r * bs + c] = x[r];
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Embedding E_s: fine coefficients = E_s * coarse coefficients (L2 projection */
/* of the coarse cell's polynomials onto child s, s = sx + 2 sy + 4 sz)       */
/* ------------------------------------------------------------------------- */
static void embedding(int p, double *E /* [8][bs][bs] */) {
    int abc[64][3];
    int bs = basis_index(p, abc);
    int q = p + 2;
    double xq[16], wq[16];
    gauss01(q, xq, wq);
    double h = 1.0; /* child side; the coarse cell has side 2 and the entries do not depend on h */
    for (int s = 0; s < 8; ++s) {
        int off[3] = {s & 1, (s >> 1) & 1, (s >> 2) & 1};
        double *Es = E + (size_t)s * bs * bs;
        memset(Es, 0, sizeof(double) * bs * bs);
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j)
                for (int k = 0; k < q; ++k) {
                    double xc[3] = {xq[i] * h, xq[j] * h, xq[k] * h};    /* child frame */
                    double xp[3] = {xc[0] + off[0] * h, xc[1] + off[1] * h, xc[2] + off[2] * h}; /* coarse frame */
                    double wt = wq[i] * wq[j] * wq[k] * h * h * h;
                    for (int m = 0; m < bs; ++m)
                        for (int n = 0; n < bs; ++n)
                            Es[m * bs + n] += wt * phi_val(abc[m], h, xc) * phi_val(abc[n], 2.0 * h, xp);
                }
    }
}

/* ------------------------------------------------------------------------- */
/* Solver state                                                               */
/* ------------------------------------------------------------------------- */
typedef struct {
    int nx, ny, nz, n; /* cells */
    size_t N;          /* DOFs */
    bsr_t A;
    float *A32;        /* FP32 copy of A.val (mixed forms) */
    double *Dinv;      /* [n][bs][bs] block inverses (non-coarsest levels) */
    int as_w;          /* additive Schwarz: cells per patch (row length of A) */
    int *as_cells;     /* [n][as_w] patch of cell c: c, then its row's other columns (-1: none) */
    double *as_L;      /* [n][(as_w bs)^2] Cholesky factors of the patch matrices */
    float *as_inv32;   /* mixed forms: [n][m][m] patch inverses rounded to float, row-major */
    float *Dinv32;
    double *Lc;        /* coarsest: dense Cholesky factor */
    /* residual minimisation storage */
    int k, cap;
    double *W, *Z;     /* [cap][N] */
    /* work vectors */
    double *r, *x, *z, *w, *t, *t2, *rsnap, *zcor, *r0, *x0;
    /* transfers to the next coarser level: parent cell and child slot */
    int *parent;
    unsigned char *slot;
    /* children of each cell of this level (levels >= 1): kids[kid_ptr[I] ..
     * kid_ptr[I+1]) are the finer level's cells K with parent(K) = I, in
     * order of (slot, K) */
    int *kid_ptr, *kids;
} level_t;

typedef struct {
    int nlev, bs, p;
    or_opts opt;
    level_t lev[MAXLEV];
    double E[8 * 64 * 64];
    float E32[8 * 64 * 64];
    int has_sip;
    elem_t elem;
    double *nu;
    int mode32;        /* current inner precision: 0 FP64, 1 FP32 everywhere, 2 FP32 except fine RM */
    /* logs */
    int *visits;       /* pairs (level, iterations) */
    int n_visits, cap_visits;
    double *trace;     /* triples (step, ||r||, type) on the finest level */
    int n_trace, cap_trace, step;
    double *vnorm;     /* per visit, in completion order: level, iterations, ||r0||, then ||r||
                          after each iteration (the quantities the level tests of Sec. 4.2 read) */
    int n_vnorm, cap_vnorm;
    int n_breakdowns;
    double bnorm_fine;
    int *sched;        /* smoother steps per cycle of the forking level (NULL: n_s) */
    int sched_n, sched_pos;
} oracle_t;

static void level_free(level_t *L) {
    bsr_free(&L->A);
    free(L->A32);
    free(L->Dinv);
    free(L->Dinv32);
    free(L->Lc);
    free(L->W);
    free(L->Z);
    free(L->r); free(L->x); free(L->z); free(L->w); free(L->t); free(L->t2);
    free(L->rsnap); free(L->zcor); free(L->r0); free(L->x0);
    free(L->parent);
    free(L->slot);
    free(L->kid_ptr);
    free(L->kids);
    free(L->as_cells);
    free(L->as_L);
    free(L->as_inv32);
}

void oracle_destroy(void *h) {
    oracle_t *o = h;
    if (!o) return;
    for (int l = 0; l < o->nlev; ++l) level_free(&o->lev[l]);
    if (o->has_sip) elem_free(&o->elem);
    free(o->nu);
    free(o->visits);
    free(o->trace);
    free(o->vnorm);
    free(o->sched);
    free(o);
}

/* Smoother-step counts for the cycles of the forking level, consumed in
 * order by the following solves (n = 0 clears; cycles beyond the schedule
 * take n_s). Each count must be >= 1. */
int oracle_set_step_schedule(void *h, const int *counts, int n) {
    oracle_t *o = h;
    if (!o || n < 0 || (n > 0 && !counts)) return OR_EINVAL;
    for (int i = 0; i < n; ++i)
        if (counts[i] < 1) return OR_EINVAL;
    free(o->sched);
    o->sched = NULL;
    o->sched_n = o->sched_pos = 0;
    if (n == 0) return OR_OK;
    o->sched = malloc(sizeof(int) * n);
    if (!o->sched) return OR_ENOMEM;
    memcpy(o->sched, counts, sizeof(int) * n);
    o->sched_n = n;
    return OR_OK;
}

/* the level whose cycles have a concurrent coarse path (-1: none) */
static int fork_level(const oracle_t *o) {
    if (o->opt.variant == 1) return 0;
    if (o->opt.variant == 2) return 1;
    return -1;
}

static void log_visit(oracle_t *o, int l, int it) {
    if (o->n_visits == o->cap_visits) {
        o->cap_visits = o->cap_visits ? 2 * o->cap_visits : 256;
        o->visits = realloc(o->visits, sizeof(int) * 2 * o->cap_visits);
    }
    o->visits[2 * o->n_visits] = l;
    o->visits[2 * o->n_visits + 1] = it;
    o->n_visits++;
}

static void log_vnorm(oracle_t *o, int l, int it, double r0n, const double *rns) {
    int need = o->n_vnorm + 3 + it;
    if (need > o->cap_vnorm) {
        int cap = o->cap_vnorm ? o->cap_vnorm : 1024;
        while (cap < need) cap *= 2;
        o->vnorm = realloc(o->vnorm, sizeof(double) * cap);
        o->cap_vnorm = cap;
    }
    double *v = o->vnorm + o->n_vnorm;
    v[0] = l;
    v[1] = it;
    v[2] = r0n;
    for (int i = 0; i < it; ++i) v[3 + i] = rns[i];
    o->n_vnorm = need;
}

/* type: 0 initial, 1 smoother, 2 coarse, 3 final (the paper's residual-trace kinds) */
static void log_trace(oracle_t *o, double rn, int type) {
    if (o->n_trace == o->cap_trace) {
        o->cap_trace = o->cap_trace ? 2 * o->cap_trace : 256;
        o->trace = realloc(o->trace, sizeof(double) * 3 * o->cap_trace);
    }
    o->trace[3 * o->n_trace] = o->step;
    o->trace[3 * o->n_trace + 1] = rn;
    o->trace[3 * o->n_trace + 2] = type;
    o->n_trace++;
}

/* Galerkin product A_c = P^T A P, P having block E_{slot(K)} at (K, parent(K)). */
static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Block pattern of P^T A P: coarse cells I and J couple when a child of I
 * couples with a child of J in A. Sorted columns, zero values. */
static int coarse_pattern(const bsr_t *Af, const level_t *F, const level_t *C, int bs, bsr_t *Ac) {
    int n = C->n;
    Ac->n = n;
    Ac->bs = bs;
    Ac->row_ptr = malloc(sizeof(int) * (n + 1));
    int *tmp = malloc(sizeof(int) * ((size_t)Af->nnzb + 1));
    if (!Ac->row_ptr || !tmp) { free(tmp); return OR_ENOMEM; }
    int64_t cnt = 0;
    Ac->row_ptr[0] = 0;
    /* pass 1: count unique parents of the children's columns per coarse row */
    for (int I = 0; I < n; ++I) {
        int m = 0;
        for (int q = C->kid_ptr[I]; q < C->kid_ptr[I + 1]; ++q) {
            int K = C->kids[q];
            for (int e = Af->row_ptr[K]; e < Af->row_ptr[K + 1]; ++e) tmp[m++] = F->parent[Af->col[e]];
        }
        qsort(tmp, m, sizeof(int), cmp_int);
        int u = 0;
        for (int a = 0; a < m; ++a)
            if (a == 0 || tmp[a] != tmp[a - 1]) ++u;
        cnt += u;
        Ac->row_ptr[I + 1] = (int)cnt;
    }
    Ac->nnzb = cnt;
    Ac->col = malloc(sizeof(int) * (cnt ? cnt : 1));
    Ac->val = calloc((size_t)(cnt ? cnt : 1) * bs * bs, sizeof(double));
    if (!Ac->col || !Ac->val) { free(tmp); return OR_ENOMEM; }
    for (int I = 0; I < n; ++I) {
        int m = 0;
        for (int q = C->kid_ptr[I]; q < C->kid_ptr[I + 1]; ++q) {
            int K = C->kids[q];
            for (int e = Af->row_ptr[K]; e < Af->row_ptr[K + 1]; ++e) tmp[m++] = F->parent[Af->col[e]];
        }
        qsort(tmp, m, sizeof(int), cmp_int);
        int o_ = Ac->row_ptr[I];
        for (int a = 0; a < m; ++a)
            if (a == 0 || tmp[a] != tmp[a - 1]) Ac->col[o_++] = tmp[a];
    }
    free(tmp);
    return OR_OK;
}

static int galerkin(const bsr_t *Af, const level_t *F, const level_t *C, const double *E, int bs, bsr_t *Ac) {
    int rc = coarse_pattern(Af, F, C, bs, Ac);
    if (rc) return rc;
    double tmp[64 * 64];
    for (int K = 0; K < Af->n; ++K) {
        int I = F->parent[K];
        const double *EK = E + (size_t)F->slot[K] * bs * bs;
        for (int q = Af->row_ptr[K]; q < Af->row_ptr[K + 1]; ++q) {
            int Kp = Af->col[q];
            int J = F->parent[Kp];
            const double *EKp = E + (size_t)F->slot[Kp] * bs * bs;
            const double *a = Af->val + (size_t)q * bs * bs;
            int64_t qc = bsr_find(Ac, I, J);
            if (qc < 0) return OR_EINVAL;
            double *ac = Ac->val + (size_t)qc * bs * bs;
            /* tmp = A_{K,K'} E_{K'} */
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < bs; ++c) {
                    double s = 0.0;
                    for (int m = 0; m < bs; ++m) s += a[r * bs + m] * EKp[m * bs + c];
                    tmp[r * bs + c] = s;
                }
            /* ac += E_K^T tmp */
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < bs; ++c) {
                    double s = 0.0;
                    for (int m = 0; m < bs; ++m) s += EK[m * bs + r] * tmp[m * bs + c];
                    ac[r * bs + c] += s;
                }
        }
    }
    return OR_OK;
}

static double *dalloc(size_t n) { return calloc(n ? n : 1, sizeof(double)); }

static int level_alloc_work(level_t *L) {
    size_t N = L->N;
    L->r = dalloc(N); L->x = dalloc(N); L->z = dalloc(N); L->w = dalloc(N);
    L->t = dalloc(N); L->t2 = dalloc(N); L->rsnap = dalloc(N); L->zcor = dalloc(N);
    L->r0 = dalloc(N); L->x0 = dalloc(N);
    if (!L->r || !L->x || !L->z || !L->w || !L->t || !L->t2 || !L->rsnap || !L->zcor || !L->r0 || !L->x0)
        return OR_ENOMEM;
    return OR_OK;
}

static void default_opts(or_opts *o) {
    memset(o, 0, sizeof(*o));
    o->variant = 0;
    o->s_pre = 1;
    o->s_post = 1;
    o->n_s = 1;
    o->max_iter = 500;
    o->omega = 0.7;
    o->inner_tol = 1e-5;
    o->max_outer = 50;
    o->breakdown = 1e-14;
    o->n_crit = 2;
    o->crit_rel[0] = 0.1; o->crit_max[0] = 20;
    o->crit_rel[1] = 0.5; o->crit_max[1] = 2;
    for (int l = 2; l < MAXLEV; ++l) { o->crit_rel[l] = -1.0; o->crit_max[l] = 1; }
}

void oracle_default_opts(or_opts *o) { default_opts(o); }

static int as_setup(oracle_t *o, int l);

/* Agglomeration hierarchy: level l+1's cells are unions of level l's cells;
 * parent[l][K] is the coarse cell of fine cell K and slot[l][K] in 0..7 picks
 * the embedding block E_slot (fine x coarse) of P_l, which has block
 * E_{slot(K)} at (K, parent(K)). Maps of all levels are concatenated. */
typedef struct {
    int nlev;
    const int *n_cells;          /* [nlev] */
    const int *parent;           /* levels 0..nlev-2, n_cells[l] each */
    const unsigned char *slot;
    const double *E;             /* [8][bs][bs], NULL: the Cartesian embedding of degree p */
} hier_t;

/* The 2x2x2 agglomeration of an nx*ny*nz grid (every halved side even):
 * parent (i/2, j/2, k/2), slot (i&1) + 2(j&1) + 4(k&1). Caller frees. */
static int cartesian_maps(int nx, int ny, int nz, int nlev, int **n_cells, int **parent, unsigned char **slot) {
    *n_cells = malloc(sizeof(int) * nlev);
    size_t tot = 0;
    for (int l = 0; l < nlev; ++l) {
        int ax = nx >> l, ay = ny >> l, az = nz >> l;
        if ((ax << l) != nx || (ay << l) != ny || (az << l) != nz || ax < 1) return OR_EINVAL;
        (*n_cells)[l] = ax * ay * az;
        if (l + 1 < nlev) tot += (size_t)ax * ay * az;
    }
    *parent = malloc(sizeof(int) * (tot ? tot : 1));
    *slot = malloc(tot ? tot : 1);
    size_t off = 0;
    for (int l = 0; l + 1 < nlev; ++l) {
        int ax = nx >> l, ay = ny >> l, cx = ax / 2, cy = ay / 2;
        for (int c = 0; c < (*n_cells)[l]; ++c) {
            int i = c % ax, j = (c / ax) % ay, k = c / (ax * ay);
            (*parent)[off + c] = (i / 2) + cx * ((j / 2) + cy * (k / 2));
            (*slot)[off + c] = (unsigned char)((i & 1) + 2 * (j & 1) + 4 * (k & 1));
        }
        off += (*n_cells)[l];
    }
    return OR_OK;
}

static int setup_common(oracle_t *o, const hier_t *H, int p) {
    int bs = o->bs, nlev = H->nlev;
    if (H->E) memcpy(o->E, H->E, sizeof(double) * 8 * bs * bs);
    else embedding(p, o->E);
    for (int t = 0; t < 8 * bs * bs; ++t) o->E32[t] = (float)o->E[t];
    for (int l = 0; l < nlev; ++l) {
        level_t *L = &o->lev[l];
        if (H->n_cells[l] < 1) return OR_EINVAL;
        if (l == 0 && H->n_cells[0] != L->A.n) return OR_EINVAL;
        L->n = H->n_cells[l];
        L->N = (size_t)L->n * bs;
        int rc = level_alloc_work(L);
        if (rc) return rc;
    }
    /* parent / slot maps and, per coarse cell, its children in (slot, index) order */
    size_t off = 0;
    for (int l = 0; l + 1 < nlev; ++l) {
        level_t *L = &o->lev[l], *C = &o->lev[l + 1];
        L->parent = malloc(sizeof(int) * L->n);
        L->slot = malloc(L->n);
        C->kid_ptr = calloc((size_t)C->n + 1, sizeof(int));
        C->kids = malloc(sizeof(int) * L->n);
        if (!L->parent || !L->slot || !C->kid_ptr || !C->kids) return OR_ENOMEM;
        for (int c = 0; c < L->n; ++c) {
            int I = H->parent[off + c], sl = H->slot[off + c];
            if (I < 0 || I >= C->n || sl > 7) return OR_EINVAL;
            L->parent[c] = I;
            L->slot[c] = (unsigned char)sl;
            C->kid_ptr[I + 1]++;
        }
        for (int I = 0; I < C->n; ++I) {
            if (C->kid_ptr[I + 1] == 0) return OR_EINVAL; /* a coarse cell without children */
            C->kid_ptr[I + 1] += C->kid_ptr[I];
        }
        int *fill = malloc(sizeof(int) * C->n);
        if (!fill) return OR_ENOMEM;
        memcpy(fill, C->kid_ptr, sizeof(int) * C->n);
        for (int sl = 0; sl < 8; ++sl)
            for (int c = 0; c < L->n; ++c)
                if (L->slot[c] == sl) C->kids[fill[L->parent[c]]++] = c;
        free(fill);
        off += L->n;
    }
    /* coarse operators */
    for (int l = 0; l + 1 < nlev; ++l) {
        int rc = galerkin(&o->lev[l].A, &o->lev[l], &o->lev[l + 1], o->E, bs, &o->lev[l + 1].A);
        if (rc) return rc;
    }
    /* block inverses and FP32 copies */
    for (int l = 0; l < nlev; ++l) {
        level_t *L = &o->lev[l];
        size_t nv = (size_t)L->A.nnzb * bs * bs;
        L->A32 = malloc(sizeof(float) * (nv ? nv : 1));
        for (size_t t = 0; t < nv; ++t) L->A32[t] = (float)L->A.val[t];
        if (l + 1 < nlev) {
            L->Dinv = dalloc((size_t)L->n * bs * bs);
            L->Dinv32 = malloc(sizeof(float) * (size_t)L->n * bs * bs);
            int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
            for (int c = 0; c < L->n; ++c) {
                int64_t q = bsr_find(&L->A, c, c);
                if (q < 0 || spd_inverse(L->A.val + (size_t)q * bs * bs, bs, L->Dinv + (size_t)c * bs * bs)) bad = 1;
            }
            if (bad) return OR_ENOTSPD;
            for (size_t t = 0; t < (size_t)L->n * bs * bs; ++t) L->Dinv32[t] = (float)L->Dinv[t];
            if (o->opt.smoother == 1) {
                int rc = as_setup(o, l);
                if (rc) return rc;
            }
        } else {
            /* coarsest: densify and factor */
            size_t n = L->N;
            L->Lc = dalloc(n * n);
            if (!L->Lc) return OR_ENOMEM;
            for (int i = 0; i < L->n; ++i)
                for (int q = L->A.row_ptr[i]; q < L->A.row_ptr[i + 1]; ++q) {
                    int j = L->A.col[q];
                    for (int r = 0; r < bs; ++r)
                        for (int c = 0; c < bs; ++c)
                            L->Lc[((size_t)i * bs + r) * n + (size_t)j * bs + c] = L->A.val[(size_t)q * bs * bs + r * bs + c];
                }
            int rc = chol_factor(L->Lc, (int)n, 1);
            if (rc) return rc;
        }
    }
    return OR_OK;
}

static int validate_bsr(int n, int bs, const int *row_ptr, const int *col, int64_t nnzb) {
    if (n <= 0 || bs <= 0 || bs > 64) return OR_EINVAL;
    if (row_ptr[0] != 0 || row_ptr[n] != nnzb) return OR_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return OR_EINVAL;
        int diag = 0;
        for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
            if (col[q] < 0 || col[q] >= n) return OR_EINVAL;
            if (q > row_ptr[i] && col[q] <= col[q - 1]) return OR_EINVAL;
            if (col[q] == i) diag = 1;
        }
        if (!diag) return OR_EINVAL;
    }
    return OR_OK;
}

int oracle_setup(const int *row_ptr, const int *col, const double *val, int64_t nnzb, int nx, int ny, int nz,
                 int p, int nlev, const or_opts *opt, void **out) {
    *out = NULL;
    if (nlev < 1 || nlev > MAXLEV || p < 0 || p > 5) return OR_EINVAL;
    if (opt && (opt->variant < 0 || opt->variant > 3 || opt->smoother < 0 || opt->smoother > 1)) return OR_EINVAL;
    int bs = oracle_nbasis(p), n = nx * ny * nz;
    int rc = validate_bsr(n, bs, row_ptr, col, nnzb);
    if (rc) return rc;
    oracle_t *o = calloc(1, sizeof(oracle_t));
    if (!o) return OR_ENOMEM;
    o->nlev = nlev;
    o->bs = bs;
    o->p = p;
    if (opt) o->opt = *opt; else default_opts(&o->opt);
    bsr_t *A = &o->lev[0].A;
    A->n = n; A->bs = bs; A->nnzb = nnzb;
    A->row_ptr = malloc(sizeof(int) * (n + 1));
    A->col = malloc(sizeof(int) * (nnzb ? nnzb : 1));
    A->val = malloc(sizeof(double) * (size_t)(nnzb ? nnzb : 1) * bs * bs);
    memcpy(A->row_ptr, row_ptr, sizeof(int) * (n + 1));
    memcpy(A->col, col, sizeof(int) * nnzb);
    memcpy(A->val, val, sizeof(double) * (size_t)nnzb * bs * bs);
    for (size_t t = 0; t < (size_t)nnzb * bs * bs; ++t)
        if (!isfinite(A->val[t])) { oracle_destroy(o); return OR_EINVAL; }
    int *nc = NULL, *par = NULL;
    unsigned char *sl = NULL;
    rc = cartesian_maps(nx, ny, nz, nlev, &nc, &par, &sl);
    if (!rc) {
        hier_t H = {nlev, nc, par, sl, NULL};
        rc = setup_common(o, &H, p);
    }
    free(nc); free(par); free(sl);
    if (rc) { oracle_destroy(o); return rc; }
    *out = o;
    return OR_OK;
}

/* Setup from a caller-supplied fine BSR matrix (copied) with a caller-supplied
 * agglomeration hierarchy: n_cells[nlev], parent and slot maps of levels
 * 0..nlev-2 concatenated, embedding blocks E[8][bs][bs]. */
int oracle_setup_h(const int *row_ptr, const int *col, const double *val, int64_t nnzb, int bs, int nlev,
                   const int *n_cells, const int *parent, const unsigned char *slot, const double *E,
                   const or_opts *opt, void **out) {
    *out = NULL;
    if (nlev < 1 || nlev > MAXLEV || bs < 1 || bs > 64 || !n_cells || !E) return OR_EINVAL;
    if (nlev > 1 && (!parent || !slot)) return OR_EINVAL;
    if (opt && (opt->variant < 0 || opt->variant > 3 || opt->smoother < 0 || opt->smoother > 1)) return OR_EINVAL;
    int n = n_cells[0];
    int rc = validate_bsr(n, bs, row_ptr, col, nnzb);
    if (rc) return rc;
    oracle_t *o = calloc(1, sizeof(oracle_t));
    if (!o) return OR_ENOMEM;
    o->nlev = nlev;
    o->bs = bs;
    o->p = -1;
    if (opt) o->opt = *opt; else default_opts(&o->opt);
    bsr_t *A = &o->lev[0].A;
    A->n = n; A->bs = bs; A->nnzb = nnzb;
    A->row_ptr = malloc(sizeof(int) * (n + 1));
    A->col = malloc(sizeof(int) * (nnzb ? nnzb : 1));
    A->val = malloc(sizeof(double) * (size_t)(nnzb ? nnzb : 1) * bs * bs);
    memcpy(A->row_ptr, row_ptr, sizeof(int) * (n + 1));
    memcpy(A->col, col, sizeof(int) * nnzb);
    memcpy(A->val, val, sizeof(double) * (size_t)nnzb * bs * bs);
    for (size_t t = 0; t < (size_t)nnzb * bs * bs; ++t)
        if (!isfinite(A->val[t])) { oracle_destroy(o); return OR_EINVAL; }
    for (int t = 0; t < 8 * bs * bs; ++t)
        if (!isfinite(E[t])) { oracle_destroy(o); return OR_EINVAL; }
    hier_t H = {nlev, n_cells, parent, slot, E};
    rc = setup_common(o, &H, -1);
    if (rc) { oracle_destroy(o); return rc; }
    *out = o;
    return OR_OK;
}

int oracle_setup_sip(int nx, int ny, int nz, int p, double h, double penalty_c, const double *nu, int nlev,
                     const or_opts *opt, void **out) {
    *out = NULL;
    if (nlev < 1 || nlev > MAXLEV || p < 0 || p > 5 || !(h > 0)) return OR_EINVAL;
    if (opt && (opt->variant < 0 || opt->variant > 3 || opt->smoother < 0 || opt->smoother > 1)) return OR_EINVAL;
    int n = nx * ny * nz;
    for (int c = 0; c < n; ++c)
        if (!(nu[c] > 0.0) || !isfinite(nu[c])) return OR_EINVAL;
    oracle_t *o = calloc(1, sizeof(oracle_t));
    if (!o) return OR_ENOMEM;
    o->nlev = nlev;
    o->bs = oracle_nbasis(p);
    o->p = p;
    if (opt) o->opt = *opt; else default_opts(&o->opt);
    int rc = elem_build(&o->elem, p, h, penalty_c);
    o->has_sip = 1;
    o->nu = dalloc(n);
    memcpy(o->nu, nu, sizeof(double) * n);
    if (!rc) rc = assemble(&o->lev[0].A, &o->elem, nx, ny, nz, nu);
    o->lev[0].nx = nx; o->lev[0].ny = ny; o->lev[0].nz = nz;
    int *nc = NULL, *par = NULL;
    unsigned char *sl = NULL;
    if (!rc) rc = cartesian_maps(nx, ny, nz, nlev, &nc, &par, &sl);
    if (!rc) {
        hier_t H = {nlev, nc, par, sl, NULL};
        rc = setup_common(o, &H, p);
    }
    free(nc); free(par); free(sl);
    if (rc) { oracle_destroy(o); return rc; }
    *out = o;
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Level operations                                                           */
/* ------------------------------------------------------------------------- */
static int use32(const oracle_t *o, int l, int is_rm) {
    if (o->mode32 == 1) return 1;
    if (o->mode32 == 2) return !(l == 0 && is_rm);
    return 0;
}

static void level_spmv(const oracle_t *o, int l, const double *x, const double *b, double *y, int is_rm) {
    const level_t *L = &o->lev[l];
    if (use32(o, l, is_rm)) spmv32(&L->A, L->A32, x, b, y);
    else spmv(&L->A, x, b, y);
}

/* y = scale * Dinv * v, blockwise */
static void apply_dinv(const oracle_t *o, int l, const double *v, double scale, double *y, const double *add) {
    const level_t *L = &o->lev[l];
    int bs = o->bs, f32 = use32(o, l, 0);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < L->n; ++c) {
        const double *vc = v + (size_t)c * bs;
        for (int r = 0; r < bs; ++r) {
            size_t o_ = (size_t)c * bs + r;
            if (f32) {
                const float *D = L->Dinv32 + (size_t)c * bs * bs;
                float s = 0.0f;
                for (int k = 0; k < bs; ++k) s += D[r * bs + k] * (float)vc[k];
                float val = (float)scale * s;
                y[o_] = add ? (double)((float)add[o_] + val) : (double)val;
            } else {
                const double *D = L->Dinv + (size_t)c * bs * bs;
                double s = 0.0;
                for (int k = 0; k < bs; ++k) s += D[r * bs + k] * vc[k];
                y[o_] = add ? add[o_] + scale * s : scale * s;
            }
        }
    }
}

/* Additive Schwarz subdomains (Algorithm 3): subdomain i is cell i, its
 * overlap of one cell is every cell its matrix row couples to; the local
 * matrix A_i = R_i A P_i is the dense restriction of A to those cells, stored
 * as its Cholesky factor. */
static int as_setup(oracle_t *o, int l) {
    level_t *L = &o->lev[l];
    const bsr_t *A = &L->A;
    int bs = o->bs, w = 1;
    for (int c = 0; c < L->n; ++c) {
        int len = A->row_ptr[c + 1] - A->row_ptr[c];
        if (len > w) w = len;
    }
    int m = w * bs;
    if (m > 64 * 8) return OR_EUNSUPPORTED;
    L->as_w = w;
    L->as_cells = malloc(sizeof(int) * (size_t)L->n * w);
    L->as_L = dalloc((size_t)L->n * m * m);
    if (!L->as_cells || !L->as_L) return OR_ENOMEM;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int c = 0; c < L->n; ++c) {
        int *cells = L->as_cells + (size_t)c * w, np = 1;
        cells[0] = c;
        for (int q = A->row_ptr[c]; q < A->row_ptr[c + 1]; ++q)
            if (A->col[q] != c) cells[np++] = A->col[q];
        for (int a = np; a < w; ++a) cells[a] = -1;
        int mc = np * bs;
        double *Lf = L->as_L + (size_t)c * m * m; /* leading mc x mc block, row-major, stride mc */
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) {
                int64_t q = bsr_find(A, cells[a], cells[b]);
                for (int r = 0; r < bs; ++r)
                    for (int cc = 0; cc < bs; ++cc)
                        Lf[(size_t)(a * bs + r) * mc + b * bs + cc] =
                            q < 0 ? 0.0 : A->val[(size_t)q * bs * bs + r * bs + cc];
            }
        if (chol_factor(Lf, mc, 0)) bad = 1;
    }
    if (bad) return OR_ENOTSPD;
    if (o->opt.precision != 0) { /* single-precision local solves: inverse columns by Cholesky solves */
        L->as_inv32 = malloc(sizeof(float) * (size_t)L->n * m * m);
        if (!L->as_inv32) return OR_ENOMEM;
#pragma omp parallel for schedule(static)
        for (int c = 0; c < L->n; ++c) {
            const int *cells = L->as_cells + (size_t)c * w;
            int np = 0;
            while (np < w && cells[np] >= 0) ++np;
            int mc = np * bs;
            double e[64 * 8], x[64 * 8];
            float *I32 = L->as_inv32 + (size_t)c * m * m;
            for (int j = 0; j < mc; ++j) {
                for (int i = 0; i < mc; ++i) e[i] = (i == j) ? 1.0 : 0.0;
                chol_solve(L->as_L + (size_t)c * m * m, mc, e, x);
                for (int i = 0; i < mc; ++i) I32[(size_t)i * mc + j] = (float)x[i];
            }
        }
    }
    return OR_OK;
}

static int use32(const oracle_t *o, int l, int is_rm);

/* y = sum_i P_i A_i^-1 R_i v (one additive Schwarz correction); subdomains
 * in index order, so the sums are deterministic. Single-precision local
 * solves where the level's smoother runs in FP32. */
static void as_apply(const oracle_t *o, int l, const double *v, double *y) {
    const level_t *L = &o->lev[l];
    int bs = o->bs, w = L->as_w, m = w * bs, f32 = use32(o, l, 0);
    double rl[64 * 8], zl[64 * 8];
    float r32[64 * 8];
    memset(y, 0, sizeof(double) * L->N);
    for (int c = 0; c < L->n; ++c) {
        const int *cells = L->as_cells + (size_t)c * w;
        int np = 0;
        while (np < w && cells[np] >= 0) ++np;
        for (int a = 0; a < np; ++a)
            for (int r = 0; r < bs; ++r) rl[a * bs + r] = v[(size_t)cells[a] * bs + r];
        if (f32) {
            int mc = np * bs;
            const float *I32 = L->as_inv32 + (size_t)c * m * m;
            for (int i = 0; i < mc; ++i) r32[i] = (float)rl[i];
            for (int i = 0; i < mc; ++i) {
                float s = 0.0f;
                for (int j = 0; j < mc; ++j) s += I32[(size_t)i * mc + j] * r32[j];
                zl[i] = (double)s;
            }
        } else {
            chol_solve(L->as_L + (size_t)c * m * m, np * bs, rl, zl);
        }
        for (int a = 0; a < np; ++a)
            for (int r = 0; r < bs; ++r) y[(size_t)cells[a] * bs + r] += zl[a * bs + r];
    }
}

/* Block-Jacobi (Algorithm 4) from x0 = 0 with s iterations:
 * x = omega D^-1 r, then x <- x + omega D^-1 (r - A x). Result in out. */
static void smoother(oracle_t *o, int l, const double *r, int s, double *out) {
    level_t *L = &o->lev[l];
    double om = o->opt.omega;
    if (o->opt.smoother == 1) { /* additive Schwarz: x = omega M r, then x <- x + omega M (r - A x) */
        as_apply(o, l, r, out);
        for (size_t e = 0; e < L->N; ++e) out[e] *= om;
        for (int it = 1; it < s; ++it) {
            level_spmv(o, l, out, r, L->t2, 0);
            as_apply(o, l, L->t2, L->t);
            for (size_t e = 0; e < L->N; ++e) out[e] += om * L->t[e];
        }
        return;
    }
    apply_dinv(o, l, r, om, out, NULL);
    for (int it = 1; it < s; ++it) {
        level_spmv(o, l, out, r, L->t2, 0);     /* t2 = r - A x */
        apply_dinv(o, l, L->t2, om, out, out);  /* x = x + omega D^-1 t2 */
    }
}

static int grow_dirs(level_t *L) {
    int ncap = L->cap ? 2 * L->cap : 16;
    double *W = realloc(L->W, sizeof(double) * L->N * ncap);
    if (!W) return OR_ENOMEM;
    L->W = W;
    double *Z = realloc(L->Z, sizeof(double) * L->N * ncap);
    if (!Z) return OR_ENOMEM;
    L->Z = Z;
    L->cap = ncap;
    return OR_OK;
}

/* Residual minimisation (Algorithm 1). z is consumed (overwritten).
 * Updates L->x, L->r, appends to W, Z. Returns 1 if the direction was kept. */
static int rm(oracle_t *o, int l, double *z) {
    level_t *L = &o->lev[l];
    size_t N = L->N;
    double *w = L->w;
    if (o->opt.m_max > 0 && L->k >= o->opt.m_max) {
        /* restart: the current iterate becomes the new starting point, W = Z = {} */
        L->k = 0;
        memcpy(L->x0, L->x, sizeof(double) * N);
        memcpy(L->r0, L->r, sizeof(double) * N);
    }
    level_spmv(o, l, z, NULL, w, 1);               /* w_{l+1} = A z */
    double n_in = nrm2(w, N), n_ref = n_in;
    int passes = 1;
    for (int pass = 0; pass < passes; ++pass) {
        for (int i = 0; i < L->k; ++i) {           /* modified Gram-Schmidt */
            const double *Wi = L->W + (size_t)i * N, *Zi = L->Z + (size_t)i * N;
            double beta = dot(Wi, w, N);
#pragma omp parallel for schedule(static)
            for (size_t e = 0; e < N; ++e) {
                w[e] -= beta * Wi[e];
                z[e] -= beta * Zi[e];
            }
        }
        if (o->opt.gs == 1 && pass == 0) {
            double n_mid = nrm2(w, N);
            if (n_mid < n_ref / sqrt(2.0)) passes = 2; /* DGKS: orthogonalise once more */
            n_ref = n_mid;
        }
    }
    double n_out = nrm2(w, N);
    if (L->k == L->cap && grow_dirs(L)) return 0;
    double *Wk = L->W + (size_t)L->k * N, *Zk = L->Z + (size_t)L->k * N;
    if (!(n_out > o->opt.breakdown * n_in)) {   /* also catches n_out == 0 and NaN */
        /* breakdown: w lies in span(W) to working precision, so the direction
         * carries nothing new and is dropped. Its slot is kept as a zero
         * vector (W_k = Z_k = 0): every later coefficient against it is zero,
         * so x and r are those of discarding it, and it still counts as one
         * of the level's stored directions (toward m_max and n_dirs). */
        o->n_breakdowns++;
        memset(Wk, 0, sizeof(double) * N);
        memset(Zk, 0, sizeof(double) * N);
        L->k++;
        return 0;
    }
    double gamma = 1.0 / n_out;
#pragma omp parallel for schedule(static)
    for (size_t e = 0; e < N; ++e) {
        Wk[e] = gamma * w[e];
        Zk[e] = gamma * z[e];
    }
    L->k++;
    if (o->opt.alpha_mode == 0) {
        double alpha = dot(Wk, L->r, N);
#pragma omp parallel for schedule(static)
        for (size_t e = 0; e < N; ++e) {
            L->x[e] += alpha * Zk[e];
            L->r[e] -= alpha * Wk[e];
        }
    } else {
        /* literal form: alpha_i = w_i . r0 for all stored directions,
         * x = x0 + Z alpha, r = r0 - W alpha */
        memcpy(L->x, L->x0, sizeof(double) * N);
        memcpy(L->r, L->r0, sizeof(double) * N);
        for (int i = 0; i < L->k; ++i) {
            const double *Wi = L->W + (size_t)i * N, *Zi = L->Z + (size_t)i * N;
            double a = dot(Wi, L->r0, N);
#pragma omp parallel for schedule(static)
            for (size_t e = 0; e < N; ++e) {
                L->x[e] += a * Zi[e];
                L->r[e] -= a * Wi[e];
            }
        }
    }
    return 1;
}

/* restriction r_c = P^T r: coarse cell C sums E_s^T r_K over its children */
static void restrict_(oracle_t *o, int l, const double *r, double *rc) {
    level_t *L = &o->lev[l], *C = &o->lev[l + 1];
    int bs = o->bs, f32 = use32(o, l, 0);
    memset(rc, 0, sizeof(double) * C->N);
    /* loop over coarse cells so each output is written by one thread, children in (slot, index) order */
#pragma omp parallel for schedule(static)
    for (int I = 0; I < C->n; ++I) {
        for (int q = C->kid_ptr[I]; q < C->kid_ptr[I + 1]; ++q) {
            int K = C->kids[q], s = L->slot[K];
            for (int c = 0; c < bs; ++c) {
                if (f32) {
                    const float *E = o->E32 + (size_t)s * bs * bs;
                    float acc = 0.0f;
                    for (int m = 0; m < bs; ++m) acc += E[m * bs + c] * (float)r[(size_t)K * bs + m];
                    rc[(size_t)I * bs + c] = (double)((float)rc[(size_t)I * bs + c] + acc);
                } else {
                    const double *E = o->E + (size_t)s * bs * bs;
                    double acc = 0.0;
                    for (int m = 0; m < bs; ++m) acc += E[m * bs + c] * r[(size_t)K * bs + m];
                    rc[(size_t)I * bs + c] += acc;
                }
            }
        }
    }
}

/* prolongation z = P z_c: z_K = E_{slot(K)} z_{parent(K)} */
static void prolong(oracle_t *o, int l, const double *zc, double *z) {
    level_t *L = &o->lev[l];
    int bs = o->bs, f32 = use32(o, l, 0);
#pragma omp parallel for schedule(static)
    for (int K = 0; K < L->n; ++K) {
        int I = L->parent[K], s = L->slot[K];
        for (int r = 0; r < bs; ++r) {
            if (f32) {
                const float *E = o->E32 + (size_t)s * bs * bs;
                float acc = 0.0f;
                for (int c = 0; c < bs; ++c) acc += E[r * bs + c] * (float)zc[(size_t)I * bs + c];
                z[(size_t)K * bs + r] = acc;
            } else {
                const double *E = o->E + (size_t)s * bs * bs;
                double acc = 0.0;
                for (int c = 0; c < bs; ++c) acc += E[r * bs + c] * zc[(size_t)I * bs + c];
                z[(size_t)K * bs + r] = acc;
            }
        }
    }
}

static int mg(oracle_t *o, int l, const double *b, double *xout, double tol, int variant);

/* coarse-grid correction of level l: z = P MG_{l+1}(P^T r, 0) */
static int coarse_correction(oracle_t *o, int l, const double *r, double *z, double tol, int variant) {
    level_t *C = &o->lev[l + 1];
    double *rc = C->t, *zc = C->zcor; /* the coarse level's t/zcor are free while it is not iterating */
    restrict_(o, l, r, rc);
    int rc_ = mg(o, l + 1, rc, zc, tol, variant);
    prolong(o, l, zc, z);
    return rc_;
}

static int stop_level(const oracle_t *o, int l, double rn, double r0n, double bn, int it, double tol) {
    if (l == 0) return (rn <= tol * bn) || it >= o->opt.max_iter;
    int idx = l - 1;
    double rel = idx < MAXLEV ? o->opt.crit_rel[idx] : -1.0;
    int mx = idx < MAXLEV ? o->opt.crit_max[idx] : 1;
    if (rel >= 0.0 && rn <= rel * r0n) return 1;
    return it >= mx;
}

/* (x, r) = MG_l(b, 0): Algorithm 2 (variants 0 and 2) or the deterministic
 * Algorithm 5 (variants 1 and 3) on level l with the level-local stopping rule;
 * the coarsest level is the Cholesky solve. Variant 2 (hybrid) hands the
 * Algorithm 5 form to the coarser levels. Result in xout (N_l). */
static int mg(oracle_t *o, int l, const double *b, double *xout, double tol, int variant) {
    level_t *L = &o->lev[l];
    size_t N = L->N;
    if (l == o->nlev - 1) {
        chol_solve(L->Lc, (int)N, b, xout);
        return OR_OK;
    }
    /* W = Z = {}, x = x0 = 0, r0 = b - A x0 = b */
    L->k = 0;
    memset(L->x, 0, sizeof(double) * N);
    memcpy(L->r, b, sizeof(double) * N);
    memset(L->x0, 0, sizeof(double) * N);
    memcpy(L->r0, b, sizeof(double) * N);
    double r0n = nrm2(L->r, N), bn = r0n;
    if (l == 0) o->bnorm_fine = bn;
    if (l == 0) log_trace(o, r0n, 0);
    int it = 0, status = OR_OK;
    double rn = r0n;
    int sub_variant = variant;
    if (variant == 2) sub_variant = 1;
    else if ((variant == 1 || variant == 3) && o->opt.coarse_sync) sub_variant = 0;
    const int multiplicative = (variant == 0 || variant == 2);
    double *rns = NULL; /* ||r|| after each iteration of this visit */
    int cap_rns = 0;
    while (!stop_level(o, l, rn, r0n, bn, it, tol)) {
        if (multiplicative) {
            smoother(o, l, L->r, o->opt.s_pre, L->z);
            rm(o, l, L->z);
            if (l == 0) { o->step++; log_trace(o, nrm2(L->r, N), 1); }
            coarse_correction(o, l, L->r, L->z, tol, sub_variant);
            rm(o, l, L->z);
            if (l == 0) { o->step++; log_trace(o, nrm2(L->r, N), 2); }
            smoother(o, l, L->r, o->opt.s_post, L->z);
            rm(o, l, L->z);
            if (l == 0) { o->step++; log_trace(o, nrm2(L->r, N), 1); }
        } else {
            memcpy(L->rsnap, L->r, sizeof(double) * N);
            coarse_correction(o, l, L->rsnap, L->zcor, tol, sub_variant);
            int ns = o->opt.n_s;
            if (o->sched && l == fork_level(o) && o->sched_pos < o->sched_n) ns = o->sched[o->sched_pos++];
            for (int t = 0; t < ns; ++t) {
                smoother(o, l, L->r, o->opt.s_post, L->z);
                rm(o, l, L->z);
                if (l == 0) { o->step++; log_trace(o, nrm2(L->r, N), 1); }
            }
            rm(o, l, L->zcor);
            if (l == 0) { o->step++; log_trace(o, nrm2(L->r, N), 2); }
        }
        it++;
        rn = nrm2(L->r, N);
        if (it > cap_rns) {
            cap_rns = cap_rns ? 2 * cap_rns : 32;
            rns = realloc(rns, sizeof(double) * cap_rns);
        }
        rns[it - 1] = rn;
        if (!isfinite(rn)) { status = OR_EINVAL; break; }
    }
    if (l == 0 && status == OR_OK && rn > tol * bn) status = OR_ENOCONV;
    log_visit(o, l, it);
    log_vnorm(o, l, it, r0n, rns);
    free(rns);
    memcpy(xout, L->x, sizeof(double) * N);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Public solve                                                               */
/* ------------------------------------------------------------------------- */
int oracle_solve(void *h, const double *b, double *x, double tol, or_report *rep) {
    oracle_t *o = h;
    level_t *L = &o->lev[0];
    size_t N = L->N;
    o->n_visits = 0;
    o->n_trace = 0;
    o->n_vnorm = 0;
    o->step = 0;
    o->n_breakdowns = 0;
    o->sched_pos = 0;
    or_report R;
    memset(&R, 0, sizeof(R));
    for (size_t e = 0; e < N; ++e)
        if (!isfinite(b[e]) || !isfinite(x[e])) { R.status = OR_EINVAL; if (rep) *rep = R; return OR_EINVAL; }
    double bn = nrm2(b, N);
    if (bn == 0.0) {
        memset(x, 0, sizeof(double) * N);
        R.status = OR_OK;
        if (rep) *rep = R;
        return OR_OK;
    }
    double *rr = dalloc(N), *e = dalloc(N);
    int status = OR_OK;
    if (o->opt.precision == 1) {
        /* iterative refinement: outer FP64 residual, inner FP32 OrthoMG */
        int outer = 0;
        for (;;) {
            spmv(&L->A, x, b, rr);
            double rn = nrm2(rr, N);
            if (rn <= tol * bn) { status = OR_OK; break; }
            if (outer >= o->opt.max_outer) { status = OR_ENOCONV; break; }
            o->mode32 = 1;
            int st = mg(o, 0, rr, e, o->opt.inner_tol, o->opt.variant);
            o->mode32 = 0;
            if (o->n_visits > 0) R.iters_fine += o->visits[2 * (o->n_visits - 1) + 1];
            if (st == OR_EINVAL) { status = st; break; }
            for (size_t t = 0; t < N; ++t) x[t] += e[t];
            outer++;
        }
        R.outer_iters = outer;
        R.rel_res_rec = nrm2(rr, N) / bn;
    } else {
        /* x0 as given: solve A e = b - A x0 with e0 = 0, x = x0 + e */
        spmv(&L->A, x, b, rr);
        o->mode32 = (o->opt.precision == 2) ? 2 : 0;
        status = mg(o, 0, rr, e, tol * bn / nrm2(rr, N), o->opt.variant);
        o->mode32 = 0;
        for (size_t t = 0; t < N; ++t) x[t] += e[t];
        if (o->nlev > 1) {
            R.iters_fine = o->visits[2 * (o->n_visits - 1) + 1];
            R.rel_res_rec = nrm2(L->r, N) / bn;
            log_trace(o, nrm2(L->r, N), 3);
        }
    }
    spmv(&L->A, x, b, rr);
    R.rel_res_true = nrm2(rr, N) / bn;
    R.status = status;
    R.n_dirs_fine = L->k;
    R.n_breakdowns = o->n_breakdowns;
    R.n_visits = o->n_visits;
    R.n_trace = o->n_trace;
    R.n_vnorm = o->n_vnorm;
    free(rr);
    free(e);
    if (rep) *rep = R;
    return status;
}

/* a^T M b for one bs x bs block */
static double qform(const double *a, const double *M, const double *b, int bs) {
    double s = 0.0;
    for (int r = 0; r < bs; ++r)
        for (int c = 0; c < bs; ++c) s += a[r] * M[r * bs + c] * b[c];
    return s;
}

/* Gradient of L = 0.5 ||u - u_t||^2 with u = A(nu)^-1 f, given u and g_u = u - u_t:
 *   lambda = A^-1 g_u (adjoint solve, A symmetric), dL/df = lambda,
 *   dL/dnu_K = - lambda^T (dA/dnu_K) u. */
int oracle_grad(void *h, const double *u, const double *g_u, double *g_f, double *g_nu, double tol, or_report *rep) {
    oracle_t *o = h;
    if (!o->has_sip) return OR_EUNSUPPORTED;
    size_t N = o->lev[0].N;
    double *lam = dalloc(N);
    int st = oracle_solve(h, g_u, lam, tol, rep);
    if (st != OR_OK && st != OR_ENOCONV) { free(lam); return st; }
    if (g_f) memcpy(g_f, lam, sizeof(double) * N);
    if (g_nu) {
        const level_t *L = &o->lev[0];
        const elem_t *E = &o->elem;
        int bs = o->bs, nx = L->nx, ny = L->ny, nz = L->nz, n = L->n;
        int stride[3] = {1, nx, nx * ny}, dims[3] = {nx, ny, nz};
        const double *nu = o->nu;
        for (int c = 0; c < n; ++c) g_nu[c] = 0.0;
#define QF(M, X, Y) qform(lam + (size_t)(X) * bs, (M), u + (size_t)(Y) * bs, bs)
        for (int c = 0; c < n; ++c) {
            int ijk[3] = {c % nx, (c / nx) % ny, c / (nx * ny)};
            g_nu[c] += QF(E->S, c, c);
            for (int d = 0; d < 3; ++d) {
                if (ijk[d] == 0) g_nu[c] += QF(E->B[d][0], c, c);
                if (ijk[d] == dims[d] - 1) g_nu[c] += QF(E->B[d][1], c, c);
                if (ijk[d] < dims[d] - 1) {
                    int up = c + stride[d];
                    double face = QF(E->F[d][0][0], c, c) + QF(E->F[d][0][1], c, up) + QF(E->F[d][1][0], up, c) +
                                  QF(E->F[d][1][1], up, up);
                    g_nu[c] += dnu_face(nu[c], nu[up]) * face;
                    g_nu[up] += dnu_face(nu[up], nu[c]) * face;
                }
            }
        }
#undef QF
        for (int c = 0; c < n; ++c) g_nu[c] = -g_nu[c];
    }
    free(lam);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Accessors for tests                                                        */
/* ------------------------------------------------------------------------- */
int oracle_level_info(void *h, int l, int *n_cells, int64_t *nnzb, int *k_dirs) {
    oracle_t *o = h;
    if (l < 0 || l >= o->nlev) return OR_EINVAL;
    *n_cells = o->lev[l].n;
    *nnzb = o->lev[l].A.nnzb;
    *k_dirs = o->lev[l].k;
    return OR_OK;
}

int oracle_get_matrix(void *h, int l, int *row_ptr, int *col, double *val) {
    oracle_t *o = h;
    if (l < 0 || l >= o->nlev) return OR_EINVAL;
    const bsr_t *A = &o->lev[l].A;
    memcpy(row_ptr, A->row_ptr, sizeof(int) * (A->n + 1));
    memcpy(col, A->col, sizeof(int) * A->nnzb);
    memcpy(val, A->val, sizeof(double) * (size_t)A->nnzb * A->bs * A->bs);
    return OR_OK;
}

int oracle_get_embedding(void *h, double *E) {
    oracle_t *o = h;
    memcpy(E, o->E, sizeof(double) * 8 * o->bs * o->bs);
    return OR_OK;
}

int oracle_embedding_p(int p, double *E) {
    if (p < 0 || p > 5) return OR_EINVAL;
    embedding(p, E);
    return OR_OK;
}

/* stored directions of level l after the last solve: W, Z as [k][N] */
int oracle_get_dirs(void *h, int l, double *W, double *Z) {
    oracle_t *o = h;
    const level_t *L = &o->lev[l];
    memcpy(W, L->W, sizeof(double) * L->N * L->k);
    memcpy(Z, L->Z, sizeof(double) * L->N * L->k);
    return OR_OK;
}

int oracle_get_residual(void *h, int l, double *r) {
    oracle_t *o = h;
    memcpy(r, o->lev[l].r, sizeof(double) * o->lev[l].N);
    return OR_OK;
}

int oracle_get_visits(void *h, int *out) {
    oracle_t *o = h;
    memcpy(out, o->visits, sizeof(int) * 2 * o->n_visits);
    return o->n_visits;
}

int oracle_get_trace(void *h, double *out) {
    oracle_t *o = h;
    memcpy(out, o->trace, sizeof(double) * 3 * o->n_trace);
    return o->n_trace;
}

/* y = A_l x (or b - A_l x) on level l, FP64 */
int oracle_spmv(void *h, int l, const double *x, const double *b, double *y) {
    oracle_t *o = h;
    spmv(&o->lev[l].A, x, b, y);
    return OR_OK;
}

/* The per-visit residual log of the last solve (out sized from the report's
 * n_vnorm); returns its length. */
int oracle_get_visit_norms(void *h, double *out) {
    oracle_t *o = h;
    memcpy(out, o->vnorm, sizeof(double) * o->n_vnorm);
    return o->n_vnorm;
}

/* Single-precision forms of the level operations, as the mixed solves run
 * them (Sec. 3.2 precedent): y = A_l x (or b - A_l x) with the operator and
 * x rounded to float and float sums; r_c = P^T r and z = P z_c with the
 * embedding blocks and inputs rounded to float. */
int oracle_spmv32(void *h, int l, const double *x, const double *b, double *y) {
    oracle_t *o = h;
    if (l < 0 || l >= o->nlev) return OR_EINVAL;
    spmv32(&o->lev[l].A, o->lev[l].A32, x, b, y);
    return OR_OK;
}

int oracle_restrict32(void *h, int l, const double *r, double *rc) {
    oracle_t *o = h;
    if (l < 0 || l >= o->nlev - 1) return OR_EINVAL;
    int saved = o->mode32;
    o->mode32 = 1;
    restrict_(o, l, r, rc);
    o->mode32 = saved;
    return OR_OK;
}

int oracle_prolong32(void *h, int l, const double *zc, double *z) {
    oracle_t *o = h;
    if (l < 0 || l >= o->nlev - 1) return OR_EINVAL;
    int saved = o->mode32;
    o->mode32 = 1;
    prolong(o, l, zc, z);
    o->mode32 = saved;
    return OR_OK;
}

/* coarsest-level direct solve and single smoother call, for unit pins */
int oracle_smoother(void *h, int l, const double *r, int s, double *out) {
    oracle_t *o = h;
    if (l >= o->nlev - 1) return OR_EINVAL;
    smoother(o, l, r, s, out);
    return OR_OK;
}

/* The smoother in the single-precision form of the mixed solves (FP32
 * matrices and local solves); needs a solver set up with a mixed precision. */
int oracle_smoother32(void *h, int l, const double *r, int s, double *out) {
    oracle_t *o = h;
    /* the single-precision Schwarz inverses exist only in the mixed forms */
    if (l >= o->nlev - 1 || (o->opt.smoother == 1 && o->opt.precision == 0)) return OR_EINVAL;
    int saved = o->mode32;
    o->mode32 = 1;
    smoother(o, l, r, s, out);
    o->mode32 = saved;
    return OR_OK;
}

int oracle_restrict(void *h, int l, const double *r, double *rc) {
    oracle_t *o = h;
    if (l >= o->nlev - 1) return OR_EINVAL;
    restrict_(o, l, r, rc);
    return OR_OK;
}

int oracle_prolong(void *h, int l, const double *zc, double *z) {
    oracle_t *o = h;
    if (l >= o->nlev - 1) return OR_EINVAL;
    prolong(o, l, zc, z);
    return OR_OK;
}

int oracle_coarse_solve(void *h, const double *b, double *x) {
    oracle_t *o = h;
    const level_t *L = &o->lev[o->nlev - 1];
    chol_solve(L->Lc, (int)L->N, b, x);
    return OR_OK;
}

int oracle_get_dinv(void *h, int l, double *D) {
    oracle_t *o = h;
    if (l >= o->nlev - 1) return OR_EINVAL;
    memcpy(D, o->lev[l].Dinv, sizeof(double) * (size_t)o->lev[l].n * o->bs * o->bs);
    return OR_OK;
}

/* unit-coefficient element matrices, for pins: S, F[3][2][2], B[3][2] */
int oracle_element(int p, double h, double penalty_c, double *S, double *F, double *B) {
    elem_t E;
    int rc = elem_build(&E, p, h, penalty_c);
    if (rc) return rc;
    int bb = E.bs * E.bs;
    memcpy(S, E.S, sizeof(double) * bb);
    for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 2; ++a) {
            memcpy(B + (size_t)(d * 2 + a) * bb, E.B[d][a], sizeof(double) * bb);
            for (int b2 = 0; b2 < 2; ++b2) memcpy(F + (size_t)((d * 2 + a) * 2 + b2) * bb, E.F[d][a][b2], sizeof(double) * bb);
        }
    elem_free(&E);
    return OR_OK;
}

/* Threads of the row-parallel loops for the following calls (n >= 1). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
