// Multi-right-hand-side kernels on the matrix cores (batched solves).
//
// With many right-hand sides on one operator, the block products Y = A X,
// T = R - A X and D^-1 T become small dense products per cell,
// (bs x bs) x (bs x nrhs), and the coarsest-level solve becomes a dense
// (N x N) x (N x nrhs) product. Each (cell, 16-column tile) product runs on
// the FP64 instruction V_MFMA_F64_16X16X4F64 (C[16x16] += A[16x4] B[4x16];
// the FP32 variant for the mixed-precision inner solve) for up to kMaxCols =
// 32 right-hand sides; bs <= 16 rows/columns are padded with zeros; the
// operator block is read once per cell for all right-hand sides, which
// divides the operator traffic of a sweep by nrhs.
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

// Cell tiles. A block of four wavefronts handles CT consecutive cells for
// all nr columns. Every right-hand side is its own component-major vector,
// so a lane-per-(column, component) access pattern would touch one 8-byte
// entry per cache line; instead the vector entries of a tile move between
// HBM and the block's LDS with consecutive lanes on consecutive cells of one
// (column, component) (CT * 8 contiguous bytes per row, neighbour cells of a
// structured grid are consecutive too), the matrix-core products read their
// B operand from LDS, and their results return to LDS before the same kind
// of coalesced store. Wavefront w computes cells w CT/4 .. (w+1) CT/4 - 1;
// per (cell, 16-column tile) the products are accumulated in the order of
// the block row (slot), then of the component steps of 4.
constexpr int kTileWaves = 4;

// Tile of this block. Blocks are dispatched to the eight XCDs in turn, each
// XCD with its own L2; tiles are handed out so that the blocks of one XCD
// take one contiguous range of cells, and the neighbour entries a tile reads
// were mostly read by that XCD's previous tiles (a bijection for any grid,
// whatever the dispatch order: only the cache reuse depends on it).
__device__ __forceinline__ int tile_of_block() {
    constexpr int X = 8;
    const int g = gridDim.x, b = blockIdx.x;
    const int q = g / X, r = g % X, x = b % X, i = b / X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

template <int BS, int CT>
struct TileBuf {
    static constexpr int LD = CT + 1; // row pitch (spreads the banks of one row)
    double v[kMaxCols * BS * LD];
    __device__ __forceinline__ double& at(int q, int k, int t) { return v[(q * BS + k) * LD + t]; }
};

// buf(q, k, t) = P_q[k n + src(c0 + t)] with src = the slot's neighbour
// (nbr[cell]) or the cell itself; zero past the last cell.
template <int BS, int CT>
__device__ __forceinline__ void tile_load(TileBuf<BS, CT>& buf, const ColPtrs& P, int nr, int n, int c0,
                                          const int* __restrict__ nbr) {
    const int total = nr * BS * CT;
    for (int e = threadIdx.x; e < total; e += kTileWaves * 64) {
        const int t = e % CT, k = (e / CT) % BS, q = e / (CT * BS);
        const int cell = c0 + t;
        double v = 0.0;
        if (cell < n) v = P.p[q][(int64_t)k * n + (nbr ? nbr[cell] : cell)];
        buf.at(q, k, t) = v;
    }
}

template <int BS, int CT>
__device__ __forceinline__ void tile_store(TileBuf<BS, CT>& buf, const ColPtrs& P, int nr, int n, int c0) {
    const int total = nr * BS * CT;
    for (int e = threadIdx.x; e < total; e += kTileWaves * 64) {
        const int t = e % CT, k = (e / CT) % BS, q = e / (CT * BS);
        const int cell = c0 + t;
        if (cell < n) P.p[q][(int64_t)k * n + cell] = buf.at(q, k, t);
    }
}

// acc[q][u] += sum over the block row of A(cell, slot) X(neighbour) for the
// wavefront's cells q and tiles u (X staged slot by slot through buf).
template <int BS, typename MT, int CT>
__device__ __forceinline__ void tile_ax(TileBuf<BS, CT>& buf, typename Mfma<MT>::acc (&acc)[CT / kTileWaves][2],
                                        int n, int width, const int* __restrict__ col, const MT* __restrict__ Ablk,
                                        int nr, const ColPtrs& X, int c0) {
    using M = Mfma<MT>;
    constexpr int CW = CT / kTileWaves;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int arow = l & 15, ak = l >> 4;
    const int ntile = (nr + 15) >> 4;
    for (int j = 0; j < width; ++j) {
        __syncthreads(); // the previous slot's operands have been read
        tile_load<BS, CT>(buf, X, nr, n, c0, col + (int64_t)j * n);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CW; ++q) {
            const int t = wv * CW + q, cell = c0 + t;
            if (cell >= n) continue; // uniform in the wavefront
            const MT* ab = Ablk + ((int64_t)cell * width + j) * (BS * BS);
#pragma unroll
            for (int ks = 0; ks < (BS + 3) / 4; ++ks) {
                const int k = ks * 4 + ak;
                const bool kin = k < BS;
                const MT a = (arow < BS && kin) ? ab[arow * BS + k] : MT(0);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (u < ntile) {
                        const int cq = u * 16 + (l & 15);
                        const MT b = (kin && cq < nr) ? (MT)buf.at(cq, k, t) : MT(0);
                        acc[q][u] = M::mma(a, b, acc[q][u]);
                    }
                }
            }
        }
    }
}

// The results of a wavefront's cells go to its own entries of buf (which
// only that wavefront reads), so no barrier separates its reads of the
// staged operands from these writes.
template <int BS, typename MT>
__device__ __forceinline__ void tile_put(double& slot, MT v) { slot = (double)v; }

// Y[c] = A X[c], or Y[c] = B[c] - A X[c] when hasB (columns c < nr).
// Ablk: [n][width][BS][BS] (type MT).
template <int BS, typename MT, bool hasB, int CT>
__global__ __launch_bounds__(64 * kTileWaves) void k_spmv_mr(int n, int width, const int* __restrict__ col,
                                                             const MT* __restrict__ Ablk, int nr, ColPtrs X,
                                                             ColPtrs B, ColPtrs Y) {
    using M = Mfma<MT>;
    using AT = typename M::acc;
    constexpr int CW = CT / kTileWaves;
    __shared__ TileBuf<BS, CT> buf;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c0 = tile_of_block() * CT;
    const int ntile = (nr + 15) >> 4;
    AT acc[CW][2];
#pragma unroll
    for (int q = 0; q < CW; ++q) acc[q][0] = acc[q][1] = AT{0, 0, 0, 0};
    tile_ax<BS, MT, CT>(buf, acc, n, width, col, Ablk, nr, X, c0);
#pragma unroll
    for (int q = 0; q < CW; ++q) {
        const int t = wv * CW + q;
        if (c0 + t >= n) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = M::row(l, i);
            if (row >= BS) continue;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int cq = u * 16 + (l & 15);
                if (u < ntile && cq < nr) tile_put<BS, MT>(buf.at(cq, row, t), acc[q][u][i]);
            }
        }
    }
    __syncthreads();
    // Y = A X, or B - A X with B read on the way out (same order of
    // operations: the product is exact in buf)
    const int total = nr * BS * CT;
    for (int e = threadIdx.x; e < total; e += kTileWaves * 64) {
        const int t = e % CT, k = (e / CT) % BS, q = e / (CT * BS);
        const int cell = c0 + t;
        if (cell >= n) continue;
        const int64_t o = (int64_t)k * n + cell;
        const double ax = buf.at(q, k, t);
        Y.p[q][o] = hasB ? (double)((MT)B.p[q][o] - (MT)ax) : ax;
    }
}

// X[c] = omega D^-1 R[c] (first block-Jacobi iteration from zero).
template <int BS, typename MT, int CT>
__global__ __launch_bounds__(64 * kTileWaves) void k_bj_first_mr(int n, const MT* __restrict__ Dblk, MT omega,
                                                                 int nr, ColPtrs R, ColPtrs X) {
    using M = Mfma<MT>;
    using AT = typename M::acc;
    constexpr int CW = CT / kTileWaves;
    __shared__ TileBuf<BS, CT> buf;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int arow = l & 15, ak = l >> 4;
    const int c0 = tile_of_block() * CT;
    const int ntile = (nr + 15) >> 4;
    tile_load<BS, CT>(buf, R, nr, n, c0, nullptr);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CW; ++q) {
        const int t = wv * CW + q, cell = c0 + t;
        if (cell >= n) continue;
        const MT* db = Dblk + (int64_t)cell * (BS * BS);
        AT acc[2] = {AT{0, 0, 0, 0}, AT{0, 0, 0, 0}};
#pragma unroll
        for (int ks = 0; ks < (BS + 3) / 4; ++ks) {
            const int k = ks * 4 + ak;
            const bool kin = k < BS;
            const MT a = (arow < BS && kin) ? db[arow * BS + k] : MT(0);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u < ntile) {
                    const int cq = u * 16 + (l & 15);
                    const MT b = (kin && cq < nr) ? (MT)buf.at(cq, k, t) : MT(0);
                    acc[u] = M::mma(a, b, acc[u]);
                }
            }
        }
        // the wavefront has read this cell's R entries (the products above
        // depend on them) before any lane overwrites them
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = M::row(l, i);
            if (row >= BS) continue;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int cq = u * 16 + (l & 15);
                if (u < ntile && cq < nr) tile_put<BS, MT>(buf.at(cq, row, t), omega * acc[u][i]);
            }
        }
    }
    __syncthreads();
    tile_store<BS, CT>(buf, X, nr, n, c0);
}

// Xout[c] = Xin[c] + omega D^-1 (R[c] - A Xin[c]). The residual block of a
// (cell, tile) moves from the result layout to the B-operand layout through
// a per-wavefront LDS square; Xin is read again on the way out.
template <int BS, typename MT, int CT>
__global__ __launch_bounds__(64 * kTileWaves) void k_bj_sweep_mr(int n, int width, const int* __restrict__ col,
                                                                 const MT* __restrict__ Ablk,
                                                                 const MT* __restrict__ Dblk, MT omega, int nr,
                                                                 ColPtrs R, ColPtrs Xin, ColPtrs Xout) {
    using M = Mfma<MT>;
    using AT = typename M::acc;
    constexpr int CW = CT / kTileWaves;
    __shared__ TileBuf<BS, CT> buf;
    __shared__ MT tt[kTileWaves][16][17];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int arow = l & 15, ak = l >> 4;
    const int c0 = tile_of_block() * CT;
    const int ntile = (nr + 15) >> 4;
    AT acc[CW][2];
#pragma unroll
    for (int q = 0; q < CW; ++q) acc[q][0] = acc[q][1] = AT{0, 0, 0, 0};
    tile_ax<BS, MT, CT>(buf, acc, n, width, col, Ablk, nr, Xin, c0);
    __syncthreads();
    tile_load<BS, CT>(buf, R, nr, n, c0, nullptr);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CW; ++q) {
        const int t = wv * CW + q, cell = c0 + t;
        if (cell >= n) continue;
        const MT* db = Dblk + (int64_t)cell * (BS * BS);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u >= ntile) continue;
            const int cq = u * 16 + (l & 15);
            // t = R - A Xin of this (cell, tile) into the square as [row][column]
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = M::row(l, i);
                MT tv = MT(0);
                if (row < BS && cq < nr) tv = (MT)buf.at(cq, row, t) - acc[q][u][i];
                tt[wv][row][l & 15] = tv;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            AT d = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < (BS + 3) / 4; ++ks) {
                const int k = ks * 4 + ak;
                const bool kin = k < BS;
                const MT a = (arow < BS && kin) ? db[arow * BS + k] : MT(0);
                const MT b = kin ? tt[wv][k][l & 15] : MT(0);
                d = M::mma(a, b, d);
            }
            // D^-1 t of this (cell, tile) replaces its R entries in buf
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = M::row(l, i);
                if (row < BS && cq < nr) tile_put<BS, MT>(buf.at(cq, row, t), d[i]);
            }
            // the square is rewritten for the next (cell, tile) only after
            // every lane has read it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
    }
    __syncthreads();
    const int total = nr * BS * CT;
    for (int e = threadIdx.x; e < total; e += kTileWaves * 64) {
        const int t = e % CT, k = (e / CT) % BS, q = e / (CT * BS);
        const int cell = c0 + t;
        if (cell >= n) continue;
        const int64_t o = (int64_t)k * n + cell;
        Xout.p[q][o] = (double)((MT)Xin.p[q][o] + omega * (MT)buf.at(q, k, t));
    }
}

// Y[c] = Ainv X[c] for the coarsest level: Ainv [np][np] row-major (n used),
// symmetric bit for bit (each entry pair is the same sum of the same
// products), so element (row, k) is read as (k, row) and the 16 rows of a k
// step are 128 contiguous bytes. Tiles of 64 rows x 256 k: a block of four
// wavefronts stages the tile's k range of every column in LDS (coalesced
// along each column), each wavefront forms 16 rows for all columns on the
// FP64 matrix cores in k order with the next 16 k steps of loads in flight
// (the first while the columns are staged), and the tile's products go to
// part[k tile][row][column]; k_dense_mr_sum adds the k tiles in order. At
// 5,120 rows that is 1,600 blocks, each streaming its own 128 KB of the
// inverse once.
constexpr int kDenseRows = 64, kDenseK = 256, kDenseU = 16;
__global__ __launch_bounds__(kDenseK) void k_dense_mr(int n, int np, const double* __restrict__ A, int nr, ColPtrs X,
                                                      double* __restrict__ part) {
    using M = Mfma<double>;
    __shared__ double xs[kMaxCols][kDenseK + 2];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int k0 = blockIdx.y * kDenseK, kn = min(kDenseK, n - k0);
    const bool two = nr > 16;
    const int r0 = blockIdx.x * kDenseRows + wv * 16;
    const int row = r0 + (l & 15), kk = l >> 4, c = l & 15;
    const bool rin = row < n;
    // the tile's 64 k steps of 4 in four rounds of kDenseU; entries past kn
    // are zero on both sides (exact), so every tile runs the same rounds and
    // the next round's loads are always issued before this round's products
    auto load = [&](double (&a)[kDenseU], int s0) {
#pragma unroll
        for (int u = 0; u < kDenseU; ++u) {
            const int kl = (s0 + u) * 4 + kk;
            a[u] = (rin && kl < kn) ? A[(int64_t)(k0 + kl) * np + row] : 0.0;
        }
    };
    d4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    auto mma = [&](const double (&a)[kDenseU], int s0) {
#pragma unroll
        for (int u = 0; u < kDenseU; ++u) {
            const int kl = (s0 + u) * 4 + kk;
            acc0 = M::mma(a[u], xs[c][kl], acc0);
            if (two) acc1 = M::mma(a[u], xs[16 + c][kl], acc1);
        }
    };
    double a0[kDenseU], a1[kDenseU];
    load(a0, 0); // in flight together with the column loads
    {
        // every column load is issued before the first is waited for (a
        // column past nr reads column 0 again, an entry past kn the last
        // one; both are stored as zero)
        const int kt = min((int)threadIdx.x, kn - 1);
        double xv[kMaxCols];
#pragma unroll
        for (int q = 0; q < kMaxCols; ++q) xv[q] = X.p[q < nr ? q : 0][k0 + kt];
#pragma unroll
        for (int q = 0; q < kMaxCols; ++q) xs[q][threadIdx.x] = (q < nr && (int)threadIdx.x < kn) ? xv[q] : 0.0;
    }
    __syncthreads();
    static_assert(kDenseK == 4 * 4 * kDenseU, "four rounds per tile");
    load(a1, kDenseU);
    mma(a0, 0);
    load(a0, 2 * kDenseU);
    mma(a1, kDenseU);
    load(a1, 3 * kDenseU);
    mma(a0, 2 * kDenseU);
    mma(a1, 3 * kDenseU);
    double* pb = part + (size_t)blockIdx.y * n * kMaxCols;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + M::row(l, i);
        if (r >= n) continue;
        pb[(size_t)r * kMaxCols + c] = acc0[i];
        if (two) pb[(size_t)r * kMaxCols + 16 + c] = acc1[i];
    }
}

// Y[c][row] = sum over k tiles (in order) of part[k tile][row][c].
__global__ void k_dense_mr_sum(int n, int nr, int nkt, const double* __restrict__ part, ColPtrs Y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = (int)(t % kMaxCols);
    const int64_t row = t / kMaxCols;
    if (row >= n || q >= nr) return;
    double s = 0.0;
    for (int kt = 0; kt < nkt; ++kt) s += part[((size_t)kt * n + row) * kMaxCols + q];
    Y.p[q][row] = s;
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

// Launch shapes: cells per tile (CT).
constexpr int kShapes[] = {16, 8};
constexpr int kNumShapes = 2;

static inline unsigned grid_for(int n, int ct) { return (unsigned)((n + ct - 1) / ct); }

#define OMG_MR_BS(bs, CALL)                            \
    switch (bs) {                                      \
    case 1: { constexpr int BSV = 1; CALL; } break;    \
    case 4: { constexpr int BSV = 4; CALL; } break;    \
    case 10: { constexpr int BSV = 10; CALL; } break;  \
    default: return hipErrorInvalidValue;              \
    }
#define OMG_MR_SHAPE(shape, CALL)                           \
    switch (shape) {                                        \
    case 0: { constexpr int CTV = 16; CALL; } break;        \
    case 1: { constexpr int CTV = 8; CALL; } break;         \
    default: return hipErrorInvalidValue;                   \
    }

static inline bool mr_ok(const Level& L, int bs, int nr) {
    return nr >= 1 && nr <= kMaxCols && L.n > 0 && L.ablk && bs <= 16;
}

static hipError_t spmv_mr_shape(int shape, const Level& L, int bs, bool fp32, int nr, const ColPtrs& X,
                                const ColPtrs* B, const ColPtrs& Y, hipStream_t st) {
    const ColPtrs Bv = B ? *B : ColPtrs{};
    const dim3 g(grid_for(L.n, kShapes[shape])), t(64 * kTileWaves);
    if (fp32) {
        if (B) {
            OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_spmv_mr<BSV, float, true, CTV>), g, t, 0, st,
                                                                 L.n, L.width, L.col, L.ablk32, nr, X, Bv, Y)))
        } else {
            OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_spmv_mr<BSV, float, false, CTV>), g, t, 0, st,
                                                                 L.n, L.width, L.col, L.ablk32, nr, X, Bv, Y)))
        }
    } else {
        if (B) {
            OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_spmv_mr<BSV, double, true, CTV>), g, t, 0, st,
                                                                 L.n, L.width, L.col, L.ablk, nr, X, Bv, Y)))
        } else {
            OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_spmv_mr<BSV, double, false, CTV>), g, t, 0, st,
                                                                 L.n, L.width, L.col, L.ablk, nr, X, Bv, Y)))
        }
    }
    return hipGetLastError();
}

static hipError_t bj_first_mr_shape(int shape, const Level& L, int bs, bool fp32, double omega, int nr,
                                    const ColPtrs& R, const ColPtrs& X, hipStream_t st) {
    const dim3 g(grid_for(L.n, kShapes[shape])), t(64 * kTileWaves);
    if (fp32) {
        OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_bj_first_mr<BSV, float, CTV>), g, t, 0, st, L.n,
                                                             L.dblk32, (float)omega, nr, R, X)))
    } else {
        OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_bj_first_mr<BSV, double, CTV>), g, t, 0, st, L.n,
                                                             L.dblk, omega, nr, R, X)))
    }
    return hipGetLastError();
}

static hipError_t bj_sweep_mr_shape(int shape, const Level& L, int bs, bool fp32, double omega, int nr,
                                    const ColPtrs& R, const ColPtrs& Xin, const ColPtrs& Xout, hipStream_t st) {
    const dim3 g(grid_for(L.n, kShapes[shape])), t(64 * kTileWaves);
    if (fp32) {
        OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_bj_sweep_mr<BSV, float, CTV>), g, t, 0, st, L.n,
                                                             L.width, L.col, L.ablk32, L.dblk32, (float)omega, nr, R,
                                                             Xin, Xout)))
    } else {
        OMG_MR_SHAPE(shape, OMG_MR_BS(bs, hipLaunchKernelGGL((k_bj_sweep_mr<BSV, double, CTV>), g, t, 0, st, L.n,
                                                             L.width, L.col, L.ablk, L.dblk, omega, nr, R, Xin,
                                                             Xout)))
    }
    return hipGetLastError();
}

// Tuned shape of (op, precision, tile count) on a level; 0 (16 cells per
// tile) until tuned.
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

// Autotuner: time both tile sizes of the three multi-RHS operations on
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
    if (nr < 1 || nr > kMaxCols || !L.ainv || !L.mrpart || n < 1 || L.np < n) return hipErrorInvalidValue;
    const int nkt = (n + kDenseK - 1) / kDenseK;
    hipLaunchKernelGGL(k_dense_mr, dim3((unsigned)((n + kDenseRows - 1) / kDenseRows), (unsigned)nkt), dim3(kDenseK),
                       0, st, n, L.np, L.ainv, nr, X, L.mrpart);
    const int64_t tot = (int64_t)n * kMaxCols;
    hipLaunchKernelGGL(k_dense_mr_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, nr, nkt, L.mrpart,
                       Y);
    return hipGetLastError();
}

// Block-contiguous operator and inverse copies (FP64 and FP32) of a level.
// Levels without a stored operator (a coarsest level below the finest keeps
// only its dense inverse) get none; the inverses exist below the coarsest.
hipError_t build_blocks(Level& L, int bs, int bsh, hipStream_t st) {
    if (L.ainv && !L.mrpart) { // partial products of the coarsest multi-column product
        const int64_t nkt = (L.N + kDenseK - 1) / kDenseK;
        const hipError_t e = hipMalloc((void**)&L.mrpart, sizeof(double) * (size_t)(nkt * L.N * kMaxCols));
        if (e != hipSuccess) return e;
    }
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
