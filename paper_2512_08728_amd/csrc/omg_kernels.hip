// Streaming kernels of the OrthoMG solve for gfx950 (CDNA4, 64-wide waves).
//
// Every kernel here is HBM-bound (block SpMV and smoother ~0.25 flop/byte in
// FP64, vector updates 0.125): one thread owns one cell, reads its block row
// with 16-byte loads that are coalesced across the wavefront (the ELL layout
// is interleaved by cell), and keeps the cell's bs outputs in registers.
// Reductions are deterministic: a fixed grid writes one partial per block,
// and every consumer sums the partials in the same fixed order.
#include "omg_internal.h"

namespace omg {

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

// Operator loads: nontemporal (NT) on levels whose operator is streamed once
// per sweep and does not fit in the last-level cache, so that it does not
// evict the vectors; ordinary loads otherwise.
template <bool NT, typename V> __device__ __forceinline__ V ld_op(const V* p) {
    if constexpr (NT) {
        V v;
        v.x = __builtin_nontemporal_load(&p->x);
        v.y = __builtin_nontemporal_load(&p->y);
        return v;
    } else {
        return *p;
    }
}

// ----------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
    // butterfly: a + b == b + a exactly, so every lane ends with the same value
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the block in a fixed order; every thread returns the same value.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += sh[i];
    __syncthreads();
    return s;
}

// Sum of G partials, same order in every block.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int G, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < G; i += blockDim.x) v += part[i];
    return block_sum(v, sh);
}

// ----------------------------------------------------------------- layout
__global__ void k_to_soa(const double* __restrict__ in, double* __restrict__ out, int n, int bs) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * bs) return;
    int c = (int)(e / bs), k = (int)(e % bs);
    out[(int64_t)k * n + c] = in[e];
}
__global__ void k_from_soa(const double* __restrict__ in, double* __restrict__ out, int n, int bs) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * bs) return;
    int c = (int)(e / bs), k = (int)(e % bs);
    out[e] = in[(int64_t)k * n + c];
}

// ----------------------------------------------------------------- block SpMV
// y = A x, or y = b - A x, for cell i. MT is the storage type of A and the
// arithmetic type (FP32 mixed forms accumulate in float).
template <int BS, typename MT, bool NT>
__device__ __forceinline__ void spmv_cell(int i, int n, int width, const int* __restrict__ col,
                                          const typename Pair<MT>::type* __restrict__ val,
                                          const double* __restrict__ x, const double* __restrict__ b,
                                          double* __restrict__ y) {
    constexpr int BSH = (BS + 1) / 2;
    MT acc[BS];
#pragma unroll
    for (int r = 0; r < BS; ++r) acc[r] = MT(0);
    for (int j = 0; j < width; ++j) {
        const int c = col[(int64_t)j * n + i];
        MT xv[2 * BSH];
#pragma unroll
        for (int k = 0; k < BS; ++k) xv[k] = (MT)x[(int64_t)k * n + c];
        if (BS & 1) xv[BS] = MT(0);
        const typename Pair<MT>::type* vj = val + (int64_t)j * BS * BSH * n + i;
#pragma unroll
        for (int r = 0; r < BS; ++r) {
#pragma unroll
            for (int cp = 0; cp < BSH; ++cp) {
                const typename Pair<MT>::type a = ld_op<NT>(&vj[(int64_t)(r * BSH + cp) * n]);
                acc[r] = fma(a.x, xv[2 * cp], acc[r]);
                acc[r] = fma(a.y, xv[2 * cp + 1], acc[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < BS; ++r) {
        const int64_t o = (int64_t)r * n + i;
        y[o] = b ? (double)((MT)b[o] - acc[r]) : (double)acc[r];
    }
}

// Thread per cell.
template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_spmv(int n, int width, const int* __restrict__ col,
                                                   const typename Pair<MT>::type* __restrict__ val,
                                                   const double* __restrict__ x, const double* __restrict__ b,
                                                   double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    spmv_cell<BS, MT, true>(i, n, width, col, val, x, b, y);
}

// ----------------------------------------------------------------- block-Jacobi
// First iteration from x0 = 0: x = omega D^-1 r.
template <int BS, typename MT, bool NT>
__device__ __forceinline__ void bj_first_cell(int i, int n, const typename Pair<MT>::type* __restrict__ dinv,
                                              MT omega, const double* __restrict__ r, double* __restrict__ x) {
    constexpr int BSH = (BS + 1) / 2;
    MT rv[2 * BSH];
#pragma unroll
    for (int k = 0; k < BS; ++k) rv[k] = (MT)r[(int64_t)k * n + i];
    if (BS & 1) rv[BS] = MT(0);
#pragma unroll
    for (int rr = 0; rr < BS; ++rr) {
        MT s = MT(0);
#pragma unroll
        for (int cp = 0; cp < BSH; ++cp) {
            const typename Pair<MT>::type d = ld_op<NT>(&dinv[(int64_t)(rr * BSH + cp) * n + i]);
            s = fma(d.x, rv[2 * cp], s);
            s = fma(d.y, rv[2 * cp + 1], s);
        }
        x[(int64_t)rr * n + i] = (double)(omega * s);
    }
}

template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_bj_first(int n, const typename Pair<MT>::type* __restrict__ dinv,
                                                       MT omega, const double* __restrict__ r,
                                                       double* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bj_first_cell<BS, MT, true>(i, n, dinv, omega, r, x);
}

// Fused iteration k >= 2: xout = xin + omega D^-1 (r - A xin).
template <int BS, typename MT, bool NT>
__device__ __forceinline__ void bj_sweep_cell(int i, int n, int width, const int* __restrict__ col,
                                              const typename Pair<MT>::type* __restrict__ val,
                                              const typename Pair<MT>::type* __restrict__ dinv, MT omega,
                                              const double* __restrict__ r, const double* __restrict__ xin,
                                              double* __restrict__ xout) {
    constexpr int BSH = (BS + 1) / 2;
    MT acc[BS];
#pragma unroll
    for (int q = 0; q < BS; ++q) acc[q] = MT(0);
    for (int j = 0; j < width; ++j) {
        const int c = col[(int64_t)j * n + i];
        MT xv[2 * BSH];
#pragma unroll
        for (int k = 0; k < BS; ++k) xv[k] = (MT)xin[(int64_t)k * n + c];
        if (BS & 1) xv[BS] = MT(0);
        const typename Pair<MT>::type* vj = val + (int64_t)j * BS * BSH * n + i;
#pragma unroll
        for (int q = 0; q < BS; ++q) {
#pragma unroll
            for (int cp = 0; cp < BSH; ++cp) {
                const typename Pair<MT>::type a = ld_op<NT>(&vj[(int64_t)(q * BSH + cp) * n]);
                acc[q] = fma(a.x, xv[2 * cp], acc[q]);
                acc[q] = fma(a.y, xv[2 * cp + 1], acc[q]);
            }
        }
    }
    MT t[2 * BSH];
#pragma unroll
    for (int q = 0; q < BS; ++q) t[q] = (MT)r[(int64_t)q * n + i] - acc[q];
    if (BS & 1) t[BS] = MT(0);
#pragma unroll
    for (int rr = 0; rr < BS; ++rr) {
        MT s = MT(0);
#pragma unroll
        for (int cp = 0; cp < BSH; ++cp) {
            const typename Pair<MT>::type d = ld_op<NT>(&dinv[(int64_t)(rr * BSH + cp) * n + i]);
            s = fma(d.x, t[2 * cp], s);
            s = fma(d.y, t[2 * cp + 1], s);
        }
        const int64_t o = (int64_t)rr * n + i;
        xout[o] = (double)((MT)xin[o] + omega * s);
    }
}

template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_bj_sweep(int n, int width, const int* __restrict__ col,
                                                       const typename Pair<MT>::type* __restrict__ val,
                                                       const typename Pair<MT>::type* __restrict__ dinv,
                                                       MT omega, const double* __restrict__ r,
                                                       const double* __restrict__ xin, double* __restrict__ xout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bj_sweep_cell<BS, MT, true>(i, n, width, col, val, dinv, omega, r, xin, xout);
}

// ----------------------------------------------------------------- grouped
// One launch over several independent operators (instances): segment q owns
// blocks [blk0[q], blk0[q+1]), one thread per cell of its level, so each
// instance gets a share of the grid proportional to its cells. The per-cell
// arithmetic is the single-instance kernels' (same results bit for bit).
__device__ __forceinline__ int segment_of(const SegTable& T, int block) {
    int q = 0;
    while (q + 1 < T.count && block >= T.blk0[q + 1]) ++q;
    return q;
}

template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_spmv_grouped(SegTable T) {
    const int q = segment_of(T, blockIdx.x);
    const int i = (blockIdx.x - T.blk0[q]) * blockDim.x + threadIdx.x;
    if (i >= T.n[q]) return;
    spmv_cell<BS, MT, false>(i, T.n[q], T.width[q], T.col[q], (const typename Pair<MT>::type*)T.val[q], T.x[q], T.b[q],
                      T.y[q]);
}

template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_bj_first_grouped(SegTable T, MT omega) {
    const int q = segment_of(T, blockIdx.x);
    const int i = (blockIdx.x - T.blk0[q]) * blockDim.x + threadIdx.x;
    if (i >= T.n[q]) return;
    bj_first_cell<BS, MT, false>(i, T.n[q], (const typename Pair<MT>::type*)T.dinv[q], omega, T.b[q], T.y[q]);
}

template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_bj_sweep_grouped(SegTable T, MT omega) {
    const int q = segment_of(T, blockIdx.x);
    const int i = (blockIdx.x - T.blk0[q]) * blockDim.x + threadIdx.x;
    if (i >= T.n[q]) return;
    bj_sweep_cell<BS, MT, false>(i, T.n[q], T.width[q], T.col[q], (const typename Pair<MT>::type*)T.val[q],
                          (const typename Pair<MT>::type*)T.dinv[q], omega, T.b[q], T.x[q], T.y[q]);
}

// Row-split variants for small levels: one thread per (cell, block row), so
// a level with few cells still spreads over the whole GPU. Same FMA order as
// the cell-per-thread kernels, hence the same results bit for bit.
template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_spmv_rows(int n, int width, const int* __restrict__ col,
                                                        const typename Pair<MT>::type* __restrict__ val,
                                                        const double* __restrict__ x, const double* __restrict__ b,
                                                        double* __restrict__ y) {
    constexpr int BSH = (BS + 1) / 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * BS) return;
    const int i = (int)(t % n), r = (int)(t / n);
    MT acc = MT(0);
    for (int j = 0; j < width; ++j) {
        const int c = col[(int64_t)j * n + i];
        const typename Pair<MT>::type* vj = val + ((int64_t)j * BS * BSH + (int64_t)r * BSH) * n + i;
#pragma unroll
        for (int cp = 0; cp < BSH; ++cp) {
            const typename Pair<MT>::type a = vj[(int64_t)cp * n];
            acc = fma(a.x, (MT)x[(int64_t)(2 * cp) * n + c], acc);
            acc = fma(a.y, (2 * cp + 1 < BS) ? (MT)x[(int64_t)(2 * cp + 1) * n + c] : MT(0), acc);
        }
    }
    const int64_t o = (int64_t)r * n + i;
    y[o] = b ? (double)((MT)b[o] - acc) : (double)acc;
}

template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_bj_first_rows(int n, const typename Pair<MT>::type* __restrict__ dinv,
                                                            MT omega, const double* __restrict__ r,
                                                            double* __restrict__ x) {
    constexpr int BSH = (BS + 1) / 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * BS) return;
    const int i = (int)(t % n), rr = (int)(t / n);
    MT s = MT(0);
#pragma unroll
    for (int cp = 0; cp < BSH; ++cp) {
        const typename Pair<MT>::type d = dinv[(int64_t)(rr * BSH + cp) * n + i];
        s = fma(d.x, (MT)r[(int64_t)(2 * cp) * n + i], s);
        s = fma(d.y, (2 * cp + 1 < BS) ? (MT)r[(int64_t)(2 * cp + 1) * n + i] : MT(0), s);
    }
    x[(int64_t)rr * n + i] = (double)(omega * s);
}

// 64 cells x BS rows per block; the residual block t of each cell goes
// through LDS to the D^-1 product.
template <int BS, typename MT>
__global__ __launch_bounds__(64 * BS) void k_bj_sweep_rows(int n, int width, const int* __restrict__ col,
                                                           const typename Pair<MT>::type* __restrict__ val,
                                                           const typename Pair<MT>::type* __restrict__ dinv,
                                                           MT omega, const double* __restrict__ r,
                                                           const double* __restrict__ xin,
                                                           double* __restrict__ xout) {
    constexpr int BSH = (BS + 1) / 2;
    __shared__ MT ts[2 * BSH][64];
    const int lc = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lc;
    const bool ok = i < n;
    MT acc = MT(0);
    if (ok) {
        for (int j = 0; j < width; ++j) {
            const int c = col[(int64_t)j * n + i];
            const typename Pair<MT>::type* vj = val + ((int64_t)j * BS * BSH + (int64_t)q * BSH) * n + i;
#pragma unroll
            for (int cp = 0; cp < BSH; ++cp) {
                const typename Pair<MT>::type a = vj[(int64_t)cp * n];
                acc = fma(a.x, (MT)xin[(int64_t)(2 * cp) * n + c], acc);
                acc = fma(a.y, (2 * cp + 1 < BS) ? (MT)xin[(int64_t)(2 * cp + 1) * n + c] : MT(0), acc);
            }
        }
        ts[q][lc] = (MT)r[(int64_t)q * n + i] - acc;
    }
    if (BS & 1) {
        if (q == 0) ts[BS][lc] = MT(0);
    }
    __syncthreads();
    if (!ok) return;
    MT s = MT(0);
#pragma unroll
    for (int cp = 0; cp < BSH; ++cp) {
        const typename Pair<MT>::type d = dinv[(int64_t)(q * BSH + cp) * n + i];
        s = fma(d.x, ts[2 * cp][lc], s);
        s = fma(d.y, ts[2 * cp + 1][lc], s);
    }
    const int64_t o = (int64_t)q * n + i;
    xout[o] = (double)((MT)xin[o] + omega * s);
}

// ----------------------------------------------------------------- transfers
// Restriction r_c = P^T r: each coarse cell sums E_s^T r_K over its finer
// cells K (slot s), taken from its child list in (slot, K) order. E is
// [8][BS][BS] (fine row, coarse column).
template <int BS, typename MT>
__device__ __forceinline__ void restrict_cell(int I, int fn, int cn, const int* __restrict__ dn_ptr,
                                              const int* __restrict__ dn, const MT* __restrict__ E,
                                              const double* __restrict__ r, double* __restrict__ rc) {
    MT out[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) out[c] = MT(0);
    const int q1 = dn_ptr[I + 1];
    for (int q = dn_ptr[I]; q < q1; ++q) {
        const int e = dn[q];
        const int K = e >> 3, s = e & 7;
        MT rv[BS];
#pragma unroll
        for (int m = 0; m < BS; ++m) rv[m] = (MT)r[(int64_t)m * fn + K];
        const MT* Es = E + s * BS * BS;
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            MT a = MT(0);
#pragma unroll
            for (int m = 0; m < BS; ++m) a = fma(Es[m * BS + c], rv[m], a);
            out[c] += a;
        }
    }
#pragma unroll
    for (int c = 0; c < BS; ++c) rc[(int64_t)c * cn + I] = (double)out[c];
}

// Restriction launch: one thread per (coarse cell, component), BS times the
// parallelism of a thread per coarse cell (the coarse levels have only a few
// thousand cells); each output summed in restrict_cell's order.
template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_restrict_rows(int fn, int cn, const int* __restrict__ dn_ptr,
                                                            const int* __restrict__ dn, const MT* __restrict__ E,
                                                            const double* __restrict__ r, double* __restrict__ rc) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)cn * BS) return;
    const int c = (int)(e / cn), I = (int)(e % cn);
    MT out = MT(0);
    const int q1 = dn_ptr[I + 1];
    for (int q = dn_ptr[I]; q < q1; ++q) {
        const int w = dn[q];
        const int K = w >> 3, s = w & 7;
        const MT* Es = E + s * BS * BS + c;
        MT a = MT(0);
#pragma unroll
        for (int m = 0; m < BS; ++m) a = fma(Es[m * BS], (MT)r[(int64_t)m * fn + K], a);
        out += a;
    }
    rc[(int64_t)c * cn + I] = (double)out;
}

// Prolongation z = P z_c: z_K = E_{slot(K)} z_{parent(K)}.
template <int BS, typename MT>
__device__ __forceinline__ void prolong_cell(int K, int fn, int cn, const int* __restrict__ up,
                                             const MT* __restrict__ E, const double* __restrict__ zc,
                                             double* __restrict__ z) {
    const int e = up[K];
    const int I = e >> 3, s = e & 7;
    MT zv[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) zv[c] = (MT)zc[(int64_t)c * cn + I];
    const MT* Es = E + s * BS * BS;
#pragma unroll
    for (int r = 0; r < BS; ++r) {
        MT a = MT(0);
#pragma unroll
        for (int c = 0; c < BS; ++c) a = fma(Es[r * BS + c], zv[c], a);
        z[(int64_t)r * fn + K] = (double)a;
    }
}

template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_prolong(int fn, int cn, const int* __restrict__ up,
                                                      const MT* __restrict__ E, const double* __restrict__ zc,
                                                      double* __restrict__ z) {
    const int K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= fn) return;
    prolong_cell<BS, MT>(K, fn, cn, up, E, zc, z);
}

// Grouped transfers over several members (segment q: blocks [blk0[q], blk0[q+1])).
template <class TT> __device__ __forceinline__ int seg_of(const TT& T, int block) {
    int q = 0;
    while (q + 1 < T.count && block >= T.blk0[q + 1]) ++q;
    return q;
}

template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_restrict_grouped(XferTable T, const MT* __restrict__ E) {
    const int q = seg_of(T, blockIdx.x);
    const int I = (blockIdx.x - T.blk0[q]) * blockDim.x + threadIdx.x;
    if (I >= T.cn[q]) return;
    restrict_cell<BS, MT>(I, T.fn[q], T.cn[q], T.dn_ptr[q], T.dn[q], E, T.in[q], T.out[q]);
}

template <int BS, typename MT>
__global__ __launch_bounds__(kThreads) void k_prolong_grouped(XferTable T, const MT* __restrict__ E) {
    const int q = seg_of(T, blockIdx.x);
    const int K = (blockIdx.x - T.blk0[q]) * blockDim.x + threadIdx.x;
    if (K >= T.fn[q]) return;
    prolong_cell<BS, MT>(K, T.fn[q], T.cn[q], T.up[q], E, T.in[q], T.out[q]);
}

// Level entry for several members: segment q runs k_level_init's loop on its
// own G_q blocks (same partials as the single launch).
__global__ __launch_bounds__(kThreads) void k_level_init_grouped(InitTable T) {
    __shared__ double sh[kThreads / 64];
    const int q = seg_of(T, blockIdx.x);
    const int bq = blockIdx.x - T.blk0[q];
    const int64_t N = T.N[q];
    const int64_t stride = (int64_t)(T.blk0[q + 1] - T.blk0[q]) * blockDim.x;
    const double* b = T.b[q];
    double* x = T.x[q];
    double* r = T.r[q];
    double s2 = 0.0;
    for (int64_t e = (int64_t)bq * blockDim.x + threadIdx.x; e < N; e += stride) {
        const double v = b[e];
        x[e] = 0.0;
        r[e] = v;
        s2 = fma(v, v, s2);
    }
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) T.part[q][bq] = s2;
}

// ----------------------------------------------------------------- dense GEMV
// y = A x for the coarsest level's dense inverse (row-major, order np >= n);
// one wavefront per row.
__global__ __launch_bounds__(kThreads) void k_gemv(int n, int np, const double* __restrict__ A,
                                                   const double* __restrict__ x, double* __restrict__ y) {
    const int row = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double* a = A + (int64_t)row * np;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s = fma(a[j], x[j], s);
    s = wave_sum(s);
    if (lane == 0) y[row] = s;
}

// Symmetric form: only the lower-triangle 64x64 tiles of A are stored
// (tile (I, J), I >= J, at index I(I+1)/2 + J, row-major, zero beyond n), so
// each visit reads half the matrix. Tile (I, J) contributes A_IJ x_J to y_I
// and, off the diagonal, A_IJ^T x_I to y_J; the contributions go to
// part[I][J][.] and part[J][I][.] and are summed over J in a fixed order.
constexpr int kSymT = 64;
__global__ __launch_bounds__(kThreads) void k_symv_tiles(int n, const double* __restrict__ T,
                                                         const double* __restrict__ x, double* __restrict__ part,
                                                         int nt) {
    __shared__ double xs[2][kSymT];
    __shared__ double cs[kSymT][kSymT + 1];
    // tile index -> (I, J), I >= J
    const int t = blockIdx.x;
    int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    if (threadIdx.x < kSymT) {
        const int gi = J * kSymT + threadIdx.x;
        xs[0][threadIdx.x] = gi < n ? x[gi] : 0.0;
    } else if (threadIdx.x < 2 * kSymT) {
        const int gi = I * kSymT + threadIdx.x - kSymT;
        xs[1][threadIdx.x - kSymT] = gi < n ? x[gi] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
    const double2* rowp = (const double2*)(T + (size_t)t * kSymT * kSymT + (size_t)r * kSymT + c0);
    double a[16];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double2 v = rowp[q];
        a[2 * q] = v.x;
        a[2 * q + 1] = v.y;
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s = fma(a[q], xs[0][c0 + q], s);
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if ((threadIdx.x & 3) == 0) part[((size_t)I * nt + J) * kSymT + r] = s;
    if (I == J) return; // uniform per block
    const double xr = xs[1][r];
#pragma unroll
    for (int q = 0; q < 16; ++q) cs[c0 + q][r] = a[q] * xr;
    __syncthreads();
    if (threadIdx.x < kSymT) {
        double u = 0.0;
        for (int rr = 0; rr < kSymT; ++rr) u += cs[threadIdx.x][rr];
        part[((size_t)J * nt + I) * kSymT + threadIdx.x] = u;
    }
}

// One block per 64-row tile: the four wavefronts sum four contiguous ranges
// of column tiles, then the ranges are added in order.
__global__ __launch_bounds__(kThreads) void k_symv_reduce(int n, int nt, const double* __restrict__ part,
                                                          double* __restrict__ y) {
    __shared__ double sh[kThreads / 64][kSymT];
    const int I = blockIdx.x, il = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int per = (nt + 3) / 4, J0 = q * per, J1 = min(nt, J0 + per);
    const double* p = part + (size_t)I * nt * kSymT + il;
    double s = 0.0;
#pragma unroll 4
    for (int J = J0; J < J1; ++J) s += p[(size_t)J * kSymT];
    sh[q][il] = s;
    __syncthreads();
    const int i = I * kSymT + threadIdx.x;
    if (threadIdx.x < kSymT && i < n) y[i] = ((sh[0][il] + sh[1][il]) + sh[2][il]) + sh[3][il];
}

// Pack the lower-triangle tiles of the dense A (row-major, leading dim np).
__global__ void k_symv_pack(int n, int np, int nt, const double* __restrict__ A, double* __restrict__ T) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntiles = (int64_t)nt * (nt + 1) / 2;
    if (e >= ntiles * kSymT * kSymT) return;
    const int64_t t = e / (kSymT * kSymT);
    const int rc = (int)(e % (kSymT * kSymT)), r = rc / kSymT, c = rc % kSymT;
    int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(I + 1) * (I + 2) / 2 <= t) ++I;
    while ((int64_t)I * (I + 1) / 2 > t) --I;
    const int J = (int)(t - (int64_t)I * (I + 1) / 2);
    const int gr = I * kSymT + r, gc = J * kSymT + c;
    T[e] = (gr < n && gc < n) ? A[(size_t)gr * np + gc] : 0.0;
}

// ----------------------------------------------------------------- RM / MGS
// part_ab[block] = sum a.b over the block's elements; part_cc likewise for c.c
__global__ __launch_bounds__(kThreads) void k_dot2(int64_t N, const double* __restrict__ a,
                                                   const double* __restrict__ b, double* __restrict__ part_ab,
                                                   const double* __restrict__ c, double* __restrict__ part_cc) {
    __shared__ double sh[kThreads / 64];
    double s1 = 0.0, s2 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        if (a) s1 = fma(a[e], b[e], s1);
        if (c) s2 = fma(c[e], c[e], s2);
    }
    if (a) {
        s1 = block_sum(s1, sh);
        if (threadIdx.x == 0) part_ab[blockIdx.x] = s1;
    }
    if (c) {
        s2 = block_sum(s2, sh);
        if (threadIdx.x == 0) part_cc[blockIdx.x] = s2;
    }
}

// One modified Gram-Schmidt step: beta = sum(part_in) (= W_i . w),
// w -= beta W_i, z -= beta Z_i, then partials of W_next . w (or w . w when
// W_next is null) for the following step. Each block updates and then reads
// only its own elements, so the step needs no grid synchronisation.
__global__ __launch_bounds__(kThreads) void k_mgs_step(int64_t N, int G, const double* __restrict__ part_in,
                                                       const double* __restrict__ Wi, const double* __restrict__ Zi,
                                                       double* __restrict__ w, double* __restrict__ z,
                                                       const double* __restrict__ Wnext,
                                                       double* __restrict__ part_out) {
    __shared__ double sh[kThreads / 64];
    const double beta = sum_partials(part_in, G, sh);
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        const double wn = fma(-beta, Wi[e], w[e]);
        w[e] = wn;
        z[e] = fma(-beta, Zi[e], z[e]);
        s = Wnext ? fma(Wnext[e], wn, s) : fma(wn, wn, s);
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part_out[blockIdx.x] = s;
}

// gamma = 1/||w|| (0 if the direction broke down), W_k = gamma w,
// Z_k = gamma z, partials of alpha = W_k . r.
__global__ __launch_bounds__(kThreads) void k_rm_normalize(int64_t N, int G, const double* __restrict__ part_nin,
                                                           const double* __restrict__ part_nout, double breakdown,
                                                           const double* __restrict__ w,
                                                           const double* __restrict__ z, double* __restrict__ Wk,
                                                           double* __restrict__ Zk, const double* __restrict__ r,
                                                           double* __restrict__ part_alpha,
                                                           double* __restrict__ scal) {
    __shared__ double sh[kThreads / 64];
    const double nin = sqrt(sum_partials(part_nin, G, sh));
    const double nout = sqrt(sum_partials(part_nout, G, sh));
    const bool keep = nout > breakdown * nin; // false for NaN and for nout == 0
    const double gamma = keep ? 1.0 / nout : 0.0;
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        const double wk = gamma * w[e];
        Wk[e] = wk;
        Zk[e] = gamma * z[e];
        s = fma(wk, r[e], s);
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        part_alpha[blockIdx.x] = s;
        if (blockIdx.x == 0 && !keep) scal[S_BREAKDOWNS] += 1.0;
    }
}

// alpha = sum(part_alpha); x += alpha Z_k; r -= alpha W_k; partials of r.r
__global__ __launch_bounds__(kThreads) void k_rm_update(int64_t N, int G, const double* __restrict__ part_alpha,
                                                        const double* __restrict__ Wk,
                                                        const double* __restrict__ Zk, double* __restrict__ x,
                                                        double* __restrict__ r, double* __restrict__ part_rn) {
    __shared__ double sh[kThreads / 64];
    const double alpha = sum_partials(part_alpha, G, sh);
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        x[e] = fma(alpha, Zk[e], x[e]);
        const double rn = fma(-alpha, Wk[e], r[e]);
        r[e] = rn;
        s = fma(rn, rn, s);
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part_rn[blockIdx.x] = s;
}

__global__ void k_finish_norm(int G, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sh[kThreads / 64];
    const double s = sum_partials(part, G, sh);
    if (threadIdx.x == 0) out[0] = sqrt(s);
}

// Level entry of Algorithm 2 with x0 = 0: x = 0, r = b, and the partials of
// ||r||^2 (same grid-stride order and block sums as k_dot2, so the norm is
// the same bit for bit).
__global__ __launch_bounds__(kThreads) void k_level_init(int64_t N, const double* __restrict__ b,
                                                         double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ part) {
    __shared__ double sh[kThreads / 64];
    double s2 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        const double v = b[e];
        x[e] = 0.0;
        r[e] = v;
        s2 = fma(v, v, s2);
    }
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s2;
}

// one block per column: the same partial order as k_finish_norm
__global__ void k_finish_norms(NormPack P, double* __restrict__ out) {
    __shared__ double sh[kThreads / 64];
    const int c = blockIdx.x;
    const double s = sum_partials(P.part[c], P.G[c], sh);
    if (threadIdx.x == 0) out[c] = sqrt(s);
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t N) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) dst[e] = src[e];
}
// plain streaming copy (16-byte accesses), the reference kernel for traffic counters
__global__ void k_stream_copy(double2* __restrict__ dst, const double2* __restrict__ src, int64_t N2) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N2; e += stride) dst[e] = src[e];
}
__global__ void k_fill(double* __restrict__ dst, double v, int64_t N) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) dst[e] = v;
}
__global__ void k_axpy(double* __restrict__ y, double a, const double* __restrict__ x, int64_t N) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) y[e] = fma(a, x[e], y[e]);
}

// ----------------------------------------------------------------- launchers
static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

hipError_t launch_to_soa(const double* in, double* out, int n, int bs, hipStream_t st) {
    int64_t N = (int64_t)n * bs;
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_soa, dim3(cdiv(N, kThreads)), dim3(kThreads), 0, st, in, out, n, bs);
    return hipGetLastError();
}
hipError_t launch_from_soa(const double* in, double* out, int n, int bs, hipStream_t st) {
    int64_t N = (int64_t)n * bs;
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_from_soa, dim3(cdiv(N, kThreads)), dim3(kThreads), 0, st, in, out, n, bs);
    return hipGetLastError();
}

#define OMG_BS_DISPATCH(bs, KERNEL_CALL)          \
    switch (bs) {                                 \
    case 1: { constexpr int BSV = 1; KERNEL_CALL; } break;   \
    case 4: { constexpr int BSV = 4; KERNEL_CALL; } break;   \
    case 10: { constexpr int BSV = 10; KERNEL_CALL; } break; \
    case 20: { constexpr int BSV = 20; KERNEL_CALL; } break; \
    default: return hipErrorInvalidValue;         \
    }

hipError_t launch_spmv(const Level& L, int bs, bool fp32, const double* x, const double* b, double* y,
                       hipStream_t st) {
    if (L.rowsplit) {
        dim3 g(cdiv((int64_t)L.n * bs, kThreads)), blk(kThreads);
        if (fp32) {
            OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_spmv_rows<BSV, float>), g, blk, 0, st, L.n, L.width, L.col,
                                                   (const float2*)L.val32, x, b, y));
        } else {
            OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_spmv_rows<BSV, double>), g, blk, 0, st, L.n, L.width, L.col,
                                                   (const double2*)L.val, x, b, y));
        }
        return hipGetLastError();
    }
    dim3 grid(cdiv(L.n, kThreads)), block(kThreads);
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_spmv<BSV, float>), grid, block, 0, st, L.n, L.width, L.col,
                                               (const float2*)L.val32, x, b, y));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_spmv<BSV, double>), grid, block, 0, st, L.n, L.width, L.col,
                                               (const double2*)L.val, x, b, y));
    }
    return hipGetLastError();
}

hipError_t launch_bj_first(const Level& L, int bs, bool fp32, double omega, const double* r, double* x,
                           hipStream_t st) {
    if (L.rowsplit) {
        dim3 g(cdiv((int64_t)L.n * bs, kThreads)), blk(kThreads);
        if (fp32) {
            OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_first_rows<BSV, float>), g, blk, 0, st, L.n,
                                                   (const float2*)L.dinv32, (float)omega, r, x));
        } else {
            OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_first_rows<BSV, double>), g, blk, 0, st, L.n,
                                                   (const double2*)L.dinv, omega, r, x));
        }
        return hipGetLastError();
    }
    dim3 grid(cdiv(L.n, kThreads)), block(kThreads);
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_first<BSV, float>), grid, block, 0, st, L.n,
                                               (const float2*)L.dinv32, (float)omega, r, x));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_first<BSV, double>), grid, block, 0, st, L.n,
                                               (const double2*)L.dinv, omega, r, x));
    }
    return hipGetLastError();
}

hipError_t launch_bj_sweep(const Level& L, int bs, bool fp32, double omega, const double* r, const double* xin,
                           double* xout, hipStream_t st) {
    if (L.rowsplit) {
        dim3 g(cdiv(L.n, 64)), blk(64 * bs);
        if (fp32) {
            OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_sweep_rows<BSV, float>), g, dim3(64 * BSV), 0, st, L.n,
                                                   L.width, L.col, (const float2*)L.val32, (const float2*)L.dinv32,
                                                   (float)omega, r, xin, xout));
        } else {
            OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_sweep_rows<BSV, double>), g, dim3(64 * BSV), 0, st, L.n,
                                                   L.width, L.col, (const double2*)L.val, (const double2*)L.dinv,
                                                   omega, r, xin, xout));
        }
        (void)blk;
        return hipGetLastError();
    }
    dim3 grid(cdiv(L.n, kThreads)), block(kThreads);
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_sweep<BSV, float>), grid, block, 0, st, L.n, L.width, L.col,
                                               (const float2*)L.val32, (const float2*)L.dinv32, (float)omega, r,
                                               xin, xout));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_sweep<BSV, double>), grid, block, 0, st, L.n, L.width, L.col,
                                               (const double2*)L.val, (const double2*)L.dinv, omega, r, xin,
                                               xout));
    }
    return hipGetLastError();
}

static int fill_segments(SegTable& T) {
    int b = 0;
    for (int q = 0; q < T.count; ++q) {
        T.blk0[q] = b;
        b += cdiv(T.n[q], kThreads);
    }
    T.blk0[T.count] = b;
    return b;
}

hipError_t launch_spmv_grouped(int bs, bool fp32, SegTable& T, hipStream_t st) {
    if (T.count < 1 || T.count > kMaxSeg) return hipErrorInvalidValue;
    const int nb = fill_segments(T);
    if (nb == 0) return hipSuccess;
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_spmv_grouped<BSV, float>), dim3(nb), dim3(kThreads), 0, st, T));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_spmv_grouped<BSV, double>), dim3(nb), dim3(kThreads), 0, st, T));
    }
    return hipGetLastError();
}

hipError_t launch_bj_first_grouped(int bs, bool fp32, double omega, SegTable& T, hipStream_t st) {
    if (T.count < 1 || T.count > kMaxSeg) return hipErrorInvalidValue;
    const int nb = fill_segments(T);
    if (nb == 0) return hipSuccess;
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_first_grouped<BSV, float>), dim3(nb), dim3(kThreads), 0, st, T,
                                               (float)omega));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_first_grouped<BSV, double>), dim3(nb), dim3(kThreads), 0, st,
                                               T, omega));
    }
    return hipGetLastError();
}

hipError_t launch_bj_sweep_grouped(int bs, bool fp32, double omega, SegTable& T, hipStream_t st) {
    if (T.count < 1 || T.count > kMaxSeg) return hipErrorInvalidValue;
    const int nb = fill_segments(T);
    if (nb == 0) return hipSuccess;
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_sweep_grouped<BSV, float>), dim3(nb), dim3(kThreads), 0, st, T,
                                               (float)omega));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_bj_sweep_grouped<BSV, double>), dim3(nb), dim3(kThreads), 0, st,
                                               T, omega));
    }
    return hipGetLastError();
}

hipError_t launch_restrict_grouped(int bs, bool fp32, const double* E, const float* E32, XferTable& T,
                                   hipStream_t st) {
    if (T.count < 1 || T.count > kMaxCols) return hipErrorInvalidValue;
    int b = 0;
    for (int q = 0; q < T.count; ++q) {
        T.blk0[q] = b;
        b += cdiv(T.cn[q], kThreads);
    }
    T.blk0[T.count] = b;
    if (b == 0) return hipSuccess;
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_restrict_grouped<BSV, float>), dim3(b), dim3(kThreads), 0, st, T,
                                               E32));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_restrict_grouped<BSV, double>), dim3(b), dim3(kThreads), 0, st, T,
                                               E));
    }
    return hipGetLastError();
}

hipError_t launch_prolong_grouped(int bs, bool fp32, const double* E, const float* E32, XferTable& T,
                                  hipStream_t st) {
    if (T.count < 1 || T.count > kMaxCols) return hipErrorInvalidValue;
    int b = 0;
    for (int q = 0; q < T.count; ++q) {
        T.blk0[q] = b;
        b += cdiv(T.fn[q], kThreads);
    }
    T.blk0[T.count] = b;
    if (b == 0) return hipSuccess;
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_prolong_grouped<BSV, float>), dim3(b), dim3(kThreads), 0, st, T,
                                               E32));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_prolong_grouped<BSV, double>), dim3(b), dim3(kThreads), 0, st, T,
                                               E));
    }
    return hipGetLastError();
}

hipError_t launch_level_init_grouped(InitTable& T, const int* G, hipStream_t st) {
    if (T.count < 1 || T.count > kMaxCols) return hipErrorInvalidValue;
    int b = 0;
    for (int q = 0; q < T.count; ++q) {
        T.blk0[q] = b;
        b += G[q];
    }
    T.blk0[T.count] = b;
    hipLaunchKernelGGL(k_level_init_grouped, dim3(b), dim3(kThreads), 0, st, T);
    return hipGetLastError();
}

hipError_t launch_restrict(const Level& F, const Level& C, int bs, bool fp32, const double* E, const float* E32,
                           const double* r, double* rc, hipStream_t st) {
    dim3 grid(cdiv((int64_t)C.n * bs, kThreads)), block(kThreads);
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_restrict_rows<BSV, float>), grid, block, 0, st, F.n, C.n,
                                               C.dn_ptr, C.dn, E32, r, rc));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_restrict_rows<BSV, double>), grid, block, 0, st, F.n, C.n,
                                               C.dn_ptr, C.dn, E, r, rc));
    }
    return hipGetLastError();
}

hipError_t launch_prolong(const Level& F, const Level& C, int bs, bool fp32, const double* E, const float* E32,
                          const double* zc, double* z, hipStream_t st) {
    dim3 grid(cdiv(F.n, kThreads)), block(kThreads);
    if (fp32) {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_prolong<BSV, float>), grid, block, 0, st, F.n, C.n, F.up, E32,
                                               zc, z));
    } else {
        OMG_BS_DISPATCH(bs, hipLaunchKernelGGL((k_prolong<BSV, double>), grid, block, 0, st, F.n, C.n, F.up, E,
                                               zc, z));
    }
    return hipGetLastError();
}

hipError_t launch_gemv(const Level& L, const double* x, double* y, hipStream_t st) {
    const int n = (int)L.N;
    if (L.atile) {
        const int nt = L.ntile;
        hipLaunchKernelGGL(k_symv_tiles, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(kThreads), 0, st, n, L.atile, x,
                           L.spart, nt);
        hipLaunchKernelGGL(k_symv_reduce, dim3(nt), dim3(kThreads), 0, st, n, nt, L.spart, y);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_gemv, dim3(cdiv(n, kThreads / 64)), dim3(kThreads), 0, st, n, L.np, L.ainv, x, y);
    return hipGetLastError();
}

hipError_t build_symv_tiles(Level& L, hipStream_t st) {
    if (L.atile || !L.ainv) return hipSuccess;
    const int n = (int)L.N;
    const int nt = (n + kSymT - 1) / kSymT;
    const int64_t ntiles = (int64_t)nt * (nt + 1) / 2;
    hipError_t e;
    if ((e = hipMalloc((void**)&L.atile, sizeof(double) * ntiles * kSymT * kSymT)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&L.spart, sizeof(double) * (size_t)nt * nt * kSymT)) != hipSuccess) return e;
    L.ntile = nt;
    const int64_t tot = ntiles * kSymT * kSymT;
    hipLaunchKernelGGL(k_symv_pack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, L.np, nt, L.ainv,
                       L.atile);
    return hipGetLastError();
}

hipError_t launch_dot2(int64_t N, int G, const double* a, const double* b, double* part_ab, const double* c,
                       double* part_cc, hipStream_t st) {
    hipLaunchKernelGGL(k_dot2, dim3(G), dim3(kThreads), 0, st, N, a, b, part_ab, c, part_cc);
    return hipGetLastError();
}

hipError_t launch_mgs_step(int64_t N, int G, const double* part_in, const double* Wi, const double* Zi, double* w,
                           double* z, const double* Wnext, double* part_out, hipStream_t st) {
    hipLaunchKernelGGL(k_mgs_step, dim3(G), dim3(kThreads), 0, st, N, G, part_in, Wi, Zi, w, z, Wnext, part_out);
    return hipGetLastError();
}

hipError_t launch_rm_normalize(int64_t N, int G, const double* part_nin, const double* part_nout,
                               double breakdown, const double* w, const double* z, double* Wk, double* Zk,
                               const double* r, double* part_alpha, double* scal, hipStream_t st) {
    hipLaunchKernelGGL(k_rm_normalize, dim3(G), dim3(kThreads), 0, st, N, G, part_nin, part_nout, breakdown, w, z,
                       Wk, Zk, r, part_alpha, scal);
    return hipGetLastError();
}

hipError_t launch_rm_update(int64_t N, int G, const double* part_alpha, const double* Wk, const double* Zk,
                            double* x, double* r, double* part_rn, hipStream_t st) {
    hipLaunchKernelGGL(k_rm_update, dim3(G), dim3(kThreads), 0, st, N, G, part_alpha, Wk, Zk, x, r, part_rn);
    return hipGetLastError();
}

hipError_t launch_finish_norm(int G, const double* part, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_finish_norm, dim3(1), dim3(kThreads), 0, st, G, part, out);
    return hipGetLastError();
}

hipError_t launch_level_init(int64_t N, int G, const double* b, double* x, double* r, double* part,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_level_init, dim3(G), dim3(kThreads), 0, st, N, b, x, r, part);
    return hipGetLastError();
}

hipError_t launch_finish_norms(int m, const NormPack& P, double* out, hipStream_t st) {
    if (m < 1 || m > kMaxCols) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_finish_norms, dim3(m), dim3(kThreads), 0, st, P, out);
    return hipGetLastError();
}

static inline int stream_blocks(int64_t N) {
    int64_t b = (N + kThreads * 4 - 1) / (kThreads * 4);
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (int)b;
}

// Snapshot / restore of a level's iteration state in one launch: r (N
// entries), x (Nx entries, Nx may be 0) and one scalar.
__global__ void k_snap(double* __restrict__ dr, const double* __restrict__ sr, int64_t N, double* __restrict__ dx,
                       const double* __restrict__ sx, int64_t Nx, double* __restrict__ ds,
                       const double* __restrict__ ss) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t e = t; e < N; e += stride) dr[e] = sr[e];
    for (int64_t e = t; e < Nx; e += stride) dx[e] = sx[e];
    if (t == 0) *ds = *ss;
}
hipError_t launch_snap(double* dr, const double* sr, int64_t N, double* dx, const double* sx, int64_t Nx, double* ds,
                       const double* ss, hipStream_t st) {
    hipLaunchKernelGGL(k_snap, dim3(stream_blocks(std::max(N, Nx))), dim3(kThreads), 0, st, dr, sr, N, dx, sx, Nx,
                       ds, ss);
    return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t N, hipStream_t st) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(stream_blocks(N)), dim3(kThreads), 0, st, dst, src, N);
    return hipGetLastError();
}
hipError_t launch_stream_copy(double* dst, const double* src, int64_t N, hipStream_t st) {
    if (N % 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3(2048), dim3(kThreads), 0, st, (double2*)dst, (const double2*)src, N / 2);
    return hipGetLastError();
}
hipError_t launch_fill(double* dst, double v, int64_t N, hipStream_t st) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(stream_blocks(N)), dim3(kThreads), 0, st, dst, v, N);
    return hipGetLastError();
}
hipError_t launch_axpy(double* y, double a, const double* x, int64_t N, hipStream_t st) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy, dim3(stream_blocks(N)), dim3(kThreads), 0, st, y, a, x, N);
    return hipGetLastError();
}

} // namespace omg
