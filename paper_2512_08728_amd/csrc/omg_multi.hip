// Multi-right-hand-side kernels on the matrix cores (batched solves).
//
// With many right-hand sides on one operator, the block products Y = A X,
// T = R - A X and D^-1 T become small dense products per cell,
// (bs x bs) x (bs x nrhs), and the coarsest-level solve becomes a dense
// (N x N) x (N x nrhs) product. One wavefront handles one cell for up to
// kMaxCols = 32 right-hand sides (two 16-wide tiles) with the FP64
// instruction V_MFMA_F64_16X16X4F64 (C[16x16] += A[16x4] B[4x16]; the FP32
// variant for the mixed-precision inner solve). bs <= 16 rows/columns are
// padded with zeros; the operator block is read once per cell for all
// right-hand sides, which divides the operator traffic of a sweep by nrhs.
//
// Operand layout (64 lanes): the A element of lane l is (row l%16, k l/16),
// the B element is (k l/16, column l%16); the FP64 result of lane l, register
// i is (row 4i + l/16, column l%16) and the FP32 result is (row 4(l/16) + i,
// column l%16).
//
// Each right-hand side keeps the component-major vector layout of the single
// solve (entry k of cell c at k*n + c), passed as a pointer per column, so the
// per-column residual minimisation runs on the same vectors unchanged. The
// operator blocks are read from block-contiguous copies (bs*bs values per
// stored block, row-major).
#include "omg_internal.h"

namespace omg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    using acc = d4;
    static __device__ __forceinline__ d4 mma(double a, double b, d4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int i) { return 4 * i + (l >> 4); }
};
template <> struct Mfma<float> {
    using acc = f4;
    static __device__ __forceinline__ f4 mma(float a, float b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int i) { return 4 * (l >> 4) + i; }
};

// Tile shape of a launch (chosen per level and column count by the
// autotuner below): WAVES wavefronts per block, and TPW 16-column tiles per
// wavefront (TPW = 2: one wavefront covers both tiles of a cell and loads
// each operator block once; TPW = 1: one wavefront per (cell, tile), twice
// the wavefronts for the same work).
struct WaveTask {
    int cell, tb, nt; // cell, first tile, tiles of this wavefront
};
template <int WAVES, int TPW>
__device__ __forceinline__ bool wave_task(int n, int nr, WaveTask& w) {
    const int wave = blockIdx.x * WAVES + (threadIdx.x >> 6);
    const int ntile = (nr + 15) >> 4;
    if (TPW == 2) {
        w.cell = wave;
        w.tb = 0;
        w.nt = ntile;
    } else {
        w.cell = wave / ntile;
        w.tb = wave % ntile;
        w.nt = 1;
    }
    return w.cell < n;
}

// Y[c] = A X[c], or Y[c] = B[c] - A X[c] when hasB (columns c < nr).
// Ablk: [n][width][BS][BS] (type MT).
template <int BS, typename MT, bool hasB, int WAVES, int TPW>
__global__ __launch_bounds__(64 * WAVES) void k_spmv_mr(int n, int width, const int* __restrict__ col,
                                                        const MT* __restrict__ Ablk, int nr, ColPtrs X, ColPtrs B,
                                                        ColPtrs Y) {
    using M = Mfma<MT>;
    using AT = typename M::acc;
    const int l = threadIdx.x & 63;
    WaveTask wt;
    if (!wave_task<WAVES, TPW>(n, nr, wt)) return; // whole wavefront
    const int cell = wt.cell;
    const int arow = l & 15, ak = l >> 4;
    int jc[TPW];
    const double* xp[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        jc[u] = (wt.tb + u) * 16 + (l & 15);
        xp[u] = (u < wt.nt && jc[u] < nr) ? X.p[jc[u]] : nullptr;
    }
    AT acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = AT{0, 0, 0, 0};
    for (int j = 0; j < width; ++j) {
        const int c = col[(int64_t)j * n + cell];
        const MT* ab = Ablk + ((int64_t)cell * width + j) * (BS * BS);
#pragma unroll
        for (int ks = 0; ks < (BS + 3) / 4; ++ks) {
            const int k = ks * 4 + ak;
            const bool kin = k < BS;
            const MT a = (arow < BS && kin) ? ab[arow * BS + k] : MT(0);
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                if (u < wt.nt) {
                    const MT b = (xp[u] && kin) ? (MT)xp[u][(int64_t)k * n + c] : MT(0);
                    acc[u] = M::mma(a, b, acc[u]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = M::row(l, i);
        if (row >= BS) continue;
        const int64_t o = (int64_t)row * n + cell;
#pragma unroll
        for (int u = 0; u < TPW; ++u)
            if (xp[u]) Y.p[jc[u]][o] = hasB ? (double)((MT)B.p[jc[u]][o] - acc[u][i]) : (double)acc[u][i];
    }
}

// X[c] = omega D^-1 R[c] (first block-Jacobi iteration from zero).
template <int BS, typename MT, int WAVES, int TPW>
__global__ __launch_bounds__(64 * WAVES) void k_bj_first_mr(int n, const MT* __restrict__ Dblk, MT omega, int nr,
                                                            ColPtrs R, ColPtrs X) {
    using M = Mfma<MT>;
    using AT = typename M::acc;
    const int l = threadIdx.x & 63;
    WaveTask wt;
    if (!wave_task<WAVES, TPW>(n, nr, wt)) return;
    const int cell = wt.cell;
    const int arow = l & 15, ak = l >> 4;
    int jc[TPW];
    const double* rp[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        jc[u] = (wt.tb + u) * 16 + (l & 15);
        rp[u] = (u < wt.nt && jc[u] < nr) ? R.p[jc[u]] : nullptr;
    }
    const MT* db = Dblk + (int64_t)cell * (BS * BS);
    AT acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = AT{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < (BS + 3) / 4; ++ks) {
        const int k = ks * 4 + ak;
        const bool kin = k < BS;
        const MT a = (arow < BS && kin) ? db[arow * BS + k] : MT(0);
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            if (u < wt.nt) {
                const MT b = (rp[u] && kin) ? (MT)rp[u][(int64_t)k * n + cell] : MT(0);
                acc[u] = M::mma(a, b, acc[u]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = M::row(l, i);
        if (row >= BS) continue;
        const int64_t o = (int64_t)row * n + cell;
#pragma unroll
        for (int u = 0; u < TPW; ++u)
            if (rp[u]) X.p[jc[u]][o] = (double)(omega * acc[u][i]);
    }
}

// Xout[c] = Xin[c] + omega D^-1 (R[c] - A Xin[c]). The residual block moves
// from the result layout to the B-operand layout through LDS (per wavefront).
template <int BS, typename MT, int WAVES, int TPW>
__global__ __launch_bounds__(64 * WAVES) void k_bj_sweep_mr(int n, int width, const int* __restrict__ col,
                                                            const MT* __restrict__ Ablk,
                                                            const MT* __restrict__ Dblk, MT omega, int nr,
                                                            ColPtrs R, ColPtrs Xin, ColPtrs Xout) {
    using M = Mfma<MT>;
    using AT = typename M::acc;
    __shared__ MT tt[WAVES][TPW][16][17];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    WaveTask wt;
    if (!wave_task<WAVES, TPW>(n, nr, wt)) return; // LDS is private to the wavefront: no block barrier
    const int cell = wt.cell;
    const int arow = l & 15, ak = l >> 4;
    int jc[TPW];
    const double* xp[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        jc[u] = (wt.tb + u) * 16 + (l & 15);
        xp[u] = (u < wt.nt && jc[u] < nr) ? Xin.p[jc[u]] : nullptr;
    }
    AT acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = AT{0, 0, 0, 0};
    for (int j = 0; j < width; ++j) {
        const int c = col[(int64_t)j * n + cell];
        const MT* ab = Ablk + ((int64_t)cell * width + j) * (BS * BS);
#pragma unroll
        for (int ks = 0; ks < (BS + 3) / 4; ++ks) {
            const int k = ks * 4 + ak;
            const bool kin = k < BS;
            const MT a = (arow < BS && kin) ? ab[arow * BS + k] : MT(0);
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                if (u < wt.nt) {
                    const MT b = (xp[u] && kin) ? (MT)xp[u][(int64_t)k * n + c] : MT(0);
                    acc[u] = M::mma(a, b, acc[u]);
                }
            }
        }
    }
    // t = R - A Xin into LDS as [tile][row][column]; rows >= BS are zero
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = M::row(l, i);
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            MT tv = MT(0);
            if (row < BS && xp[u]) tv = (MT)R.p[jc[u]][(int64_t)row * n + cell] - acc[u][i];
            tt[wv][u][row][l & 15] = tv;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const MT* db = Dblk + (int64_t)cell * (BS * BS);
    AT d[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) d[u] = AT{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < (BS + 3) / 4; ++ks) {
        const int k = ks * 4 + ak;
        const bool kin = k < BS;
        const MT a = (arow < BS && kin) ? db[arow * BS + k] : MT(0);
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            if (u < wt.nt) {
                const MT b = kin ? tt[wv][u][k][l & 15] : MT(0);
                d[u] = M::mma(a, b, d[u]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = M::row(l, i);
        if (row >= BS) continue;
        const int64_t o = (int64_t)row * n + cell;
#pragma unroll
        for (int u = 0; u < TPW; ++u)
            if (xp[u]) Xout.p[jc[u]][o] = (double)((MT)Xin.p[jc[u]][o] + omega * d[u][i]);
    }
}

constexpr int kWaves = kThreads / 64;

// Y[c] = Ainv X[c] for the coarsest level: Ainv [np][np] row-major (n used).
// One block per 16 rows; the four wavefronts split the k range and their
// partial products are summed in a fixed order through LDS.
__global__ __launch_bounds__(kThreads) void k_dense_mr(int n, int np, const double* __restrict__ A, int nr,
                                                       ColPtrs X, ColPtrs Y) {
    using M = Mfma<double>;
    __shared__ double red[kWaves][2][4][64];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row0 = blockIdx.x * 16;
    const int arow = row0 + (l & 15), ak = l >> 4;
    const int j0 = l & 15, j1 = 16 + (l & 15);
    const bool two = nr > 16;
    const double* x0 = j0 < nr ? X.p[j0] : nullptr;
    const double* x1 = (two && j1 < nr) ? X.p[j1] : nullptr;
    const int nk = (n + 3) / 4;                 // k steps of 4
    const int per = (nk + kWaves - 1) / kWaves; // steps per wavefront
    const int s0 = wv * per, s1 = min(nk, s0 + per);
    const double* arowp = A + (int64_t)min(arow, n - 1) * np;
    d4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    for (int st = s0; st < s1; ++st) {
        const int k = st * 4 + ak;
        const bool kin = k < n;
        const double a = (arow < n && kin) ? arowp[k] : 0.0;
        const double b0 = (x0 && kin) ? x0[k] : 0.0;
        acc0 = M::mma(a, b0, acc0);
        if (two) {
            const double b1 = (x1 && kin) ? x1[k] : 0.0;
            acc1 = M::mma(a, b1, acc1);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        red[wv][0][i][l] = acc0[i];
        red[wv][1][i][l] = acc1[i];
    }
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = row0 + M::row(l, i);
        if (row >= n) continue;
        double s0v = red[0][0][i][l], s1v = red[0][1][i][l];
        for (int w = 1; w < kWaves; ++w) {
            s0v += red[w][0][i][l];
            s1v += red[w][1][i][l];
        }
        if (j0 < nr) Y.p[j0][row] = s0v;
        if (two && j1 < nr) Y.p[j1][row] = s1v;
    }
}

// Block-contiguous copy of the column-pair ELL layout: out[i][j][r][c].
template <typename MT>
__global__ void k_to_blocks(int n, int width, int bs, int bsh, const double* __restrict__ val, MT* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n * width * bs * bs;
    if (t >= total) return;
    const int c = (int)(t % bs);
    const int r = (int)((t / bs) % bs);
    const int j = (int)((t / ((int64_t)bs * bs)) % width);
    const int i = (int)(t / ((int64_t)bs * bs * width));
    out[t] = (MT)val[((((int64_t)j * bs + r) * bsh + (c >> 1)) * n + i) * 2 + (c & 1)];
}

// Launch shapes: (wavefronts per block, tiles per wavefront).
constexpr int kShapes[][2] = {{4, 2}, {2, 2}, {1, 2}, {4, 1}, {2, 1}, {1, 1}};
constexpr int kNumShapes = 6;

static inline unsigned grid_for(int n, int nr, int waves, int tpw) {
    const int64_t w = (int64_t)n * (tpw == 2 ? 1 : (nr + 15) / 16);
    return (unsigned)((w + waves - 1) / waves);
}

#define OMG_MR_BS(bs, CALL)                            \
    switch (bs) {                                      \
    case 1: { constexpr int BSV = 1; CALL; } break;    \
    case 4: { constexpr int BSV = 4; CALL; } break;    \
    case 10: { constexpr int BSV = 10; CALL; } break;  \
    default: return hipErrorInvalidValue;              \
    }
#define OMG_MR_SHAPE(shape, CALL)                                                    \
    switch (shape) {                                                                 \
    case 0: { constexpr int WV = 4, TP = 2; CALL; } break;                           \
    case 1: { constexpr int WV = 2, TP = 2; CALL; } break;                           \
    case 2: { constexpr int WV = 1, TP = 2; CALL; } break;                           \
    case 3: { constexpr int WV = 4, TP = 1; CALL; } break;                           \
    case 4: { constexpr int WV = 2, TP = 1; CALL; } break;                           \
    case 5: { constexpr int WV = 1, TP = 1; CALL; } break;                           \
    default: return hipErrorInvalidValue;                                            \
    }

static inline bool mr_ok(const Level& L, int bs, int nr) {
    return nr >= 1 && nr <= kMaxCols && L.n > 0 && L.ablk && bs <= 16;
}

static hipError_t spmv_mr_shape(int shape, const Level& L, int bs, bool fp32, int nr, const ColPtrs& X,
                                const ColPtrs* B, const ColPtrs& Y, hipStream_t st) {
    const ColPtrs Bv = B ? *B : ColPtrs{};
    const int wv = kShapes[shape][0], tp = kShapes[shape][1];
    const dim3 g(grid_for(L.n, nr, wv, tp)), t(64 * wv);
    if (fp32) {
        if (B) {
            OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_spmv_mr<BSV, float, true, WV, TP>), g, t, 0, st,
                                                                 L.n, L.width, L.col, L.ablk32, nr, X, Bv, Y)))
        } else {
            OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_spmv_mr<BSV, float, false, WV, TP>), g, t, 0, st,
                                                                 L.n, L.width, L.col, L.ablk32, nr, X, Bv, Y)))
        }
    } else {
        if (B) {
            OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_spmv_mr<BSV, double, true, WV, TP>), g, t, 0,
                                                                 st, L.n, L.width, L.col, L.ablk, nr, X, Bv, Y)))
        } else {
            OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_spmv_mr<BSV, double, false, WV, TP>), g, t, 0,
                                                                 st, L.n, L.width, L.col, L.ablk, nr, X, Bv, Y)))
        }
    }
    return hipGetLastError();
}

static hipError_t bj_first_mr_shape(int shape, const Level& L, int bs, bool fp32, double omega, int nr,
                                    const ColPtrs& R, const ColPtrs& X, hipStream_t st) {
    const int wv = kShapes[shape][0], tp = kShapes[shape][1];
    const dim3 g(grid_for(L.n, nr, wv, tp)), t(64 * wv);
    if (fp32) {
        OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_bj_first_mr<BSV, float, WV, TP>), g, t, 0, st, L.n,
                                                             L.dblk32, (float)omega, nr, R, X)))
    } else {
        OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_bj_first_mr<BSV, double, WV, TP>), g, t, 0, st, L.n,
                                                             L.dblk, omega, nr, R, X)))
    }
    return hipGetLastError();
}

static hipError_t bj_sweep_mr_shape(int shape, const Level& L, int bs, bool fp32, double omega, int nr,
                                    const ColPtrs& R, const ColPtrs& Xin, const ColPtrs& Xout, hipStream_t st) {
    const int wv = kShapes[shape][0], tp = kShapes[shape][1];
    const dim3 g(grid_for(L.n, nr, wv, tp)), t(64 * wv);
    if (fp32) {
        OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_bj_sweep_mr<BSV, float, WV, TP>), g, t, 0, st, L.n,
                                                             L.width, L.col, L.ablk32, L.dblk32, (float)omega, nr, R,
                                                             Xin, Xout)))
    } else {
        OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_bj_sweep_mr<BSV, double, WV, TP>), g, t, 0, st, L.n,
                                                             L.width, L.col, L.ablk, L.dblk, omega, nr, R, Xin,
                                                             Xout)))
    }
    return hipGetLastError();
}

// Tuned shape of (op, precision, tile count) on a level; 0 (4 waves, both
// tiles per wavefront) until tuned.
static inline int shape_of(const Level& L, int op, bool fp32, int nr) {
    const int s = L.mr_shape[op][fp32 ? 1 : 0][nr > 16 ? 1 : 0];
    return s > 0 ? s - 1 : 0;
}

hipError_t launch_spmv_mr(const Level& L, int bs, bool fp32, int nr, const ColPtrs& X, const ColPtrs* B,
                          const ColPtrs& Y, hipStream_t st) {
    if (!mr_ok(L, bs, nr)) return hipErrorInvalidValue;
    return spmv_mr_shape(shape_of(L, 0, fp32, nr), L, bs, fp32, nr, X, B, Y, st);
}

hipError_t launch_bj_first_mr(const Level& L, int bs, bool fp32, double omega, int nr, const ColPtrs& R,
                              const ColPtrs& X, hipStream_t st) {
    if (!mr_ok(L, bs, nr) || !L.dblk) return hipErrorInvalidValue;
    return bj_first_mr_shape(shape_of(L, 1, fp32, nr), L, bs, fp32, omega, nr, R, X, st);
}

hipError_t launch_bj_sweep_mr(const Level& L, int bs, bool fp32, double omega, int nr, const ColPtrs& R,
                              const ColPtrs& Xin, const ColPtrs& Xout, hipStream_t st) {
    if (!mr_ok(L, bs, nr) || !L.dblk) return hipErrorInvalidValue;
    return bj_sweep_mr_shape(shape_of(L, 2, fp32, nr), L, bs, fp32, omega, nr, R, Xin, Xout, st);
}

// Autotuner: time every launch shape of the three multi-RHS operations on
// this level for nr columns (both precisions), `reps` launches each between
// HIP events, and keep the fastest. X, Y, T are nr work vectors of the level
// (filled here with zeros; the timed launches only read X/T and write Y).
hipError_t tune_mr(Level& L, int bs, int nr, const ColPtrs& X, const ColPtrs& Y, const ColPtrs& T, int reps,
                   hipStream_t st, double* best_us) {
    if (!mr_ok(L, bs, nr) || !L.dblk) return hipErrorInvalidValue;
    for (int i = 0; i < nr; ++i) {
        hipError_t e = launch_fill(X.p[i], 0.0, L.N, st);
        if (e == hipSuccess) e = launch_fill(T.p[i], 0.0, L.N, st);
        if (e != hipSuccess) return e;
    }
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return e;
    }
    const int ti = nr > 16 ? 1 : 0;
    for (int op = 0; op < 3 && e == hipSuccess; ++op)
        for (int f = 0; f < 2 && e == hipSuccess; ++f) {
            float best = 1e30f;
            int bsh = 0;
            for (int sh = 0; sh < kNumShapes && e == hipSuccess; ++sh) {
                auto run = [&]() -> hipError_t {
                    if (op == 0) return spmv_mr_shape(sh, L, bs, f == 1, nr, X, nullptr, Y, st);
                    if (op == 1) return bj_first_mr_shape(sh, L, bs, f == 1, 0.7, nr, X, Y, st);
                    return bj_sweep_mr_shape(sh, L, bs, f == 1, 0.7, nr, X, T, Y, st);
                };
                if ((e = run()) != hipSuccess) break; // warm-up
                if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
                for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
                if (e != hipSuccess) break;
                if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
                if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
                float ms = 0.f;
                if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
                if (ms < best) {
                    best = ms;
                    bsh = sh;
                }
            }
            L.mr_shape[op][f][ti] = bsh + 1;
            if (best_us) best_us[op * 2 + f] = 1e3 * best / reps;
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return e;
}

hipError_t launch_dense_mr(const Level& L, int nr, const ColPtrs& X, const ColPtrs& Y, hipStream_t st) {
    const int n = (int)L.N;
    if (nr < 1 || nr > kMaxCols || !L.ainv || n < 1 || L.np < n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dense_mr, dim3((unsigned)((n + 15) / 16)), dim3(kThreads), 0, st, n, L.np, L.ainv, nr, X,
                       Y);
    return hipGetLastError();
}

// Block-contiguous operator and inverse copies (FP64 and FP32) of a level.
// Levels without a stored operator (a coarsest level below the finest keeps
// only its dense inverse) get none; the inverses exist below the coarsest.
hipError_t build_blocks(Level& L, int bs, int bsh, hipStream_t st) {
    if (L.ablk || !L.val || L.width < 1) return hipSuccess;
    const int64_t na = (int64_t)L.n * L.width * bs * bs, nd = (int64_t)L.n * bs * bs;
    hipError_t e;
    if ((e = hipMalloc((void**)&L.ablk, sizeof(double) * na)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&L.ablk32, sizeof(float) * na)) != hipSuccess) return e;
    const unsigned ga = (unsigned)((na + 255) / 256), gd = (unsigned)((nd + 255) / 256);
    hipLaunchKernelGGL(k_to_blocks<double>, dim3(ga), dim3(256), 0, st, L.n, L.width, bs, bsh, L.val, L.ablk);
    hipLaunchKernelGGL(k_to_blocks<float>, dim3(ga), dim3(256), 0, st, L.n, L.width, bs, bsh, L.val, L.ablk32);
    if (L.dinv) {
        if ((e = hipMalloc((void**)&L.dblk, sizeof(double) * nd)) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&L.dblk32, sizeof(float) * nd)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_to_blocks<double>, dim3(gd), dim3(256), 0, st, L.n, 1, bs, bsh, L.dinv, L.dblk);
        hipLaunchKernelGGL(k_to_blocks<float>, dim3(gd), dim3(256), 0, st, L.n, 1, bs, bsh, L.dinv, L.dblk32);
    }
    return hipGetLastError();
}

} // namespace omg
