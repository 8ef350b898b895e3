// Additive Schwarz smoother (Algorithm 3, Sec. 3.2) on a level of the
// hierarchy.
//
// Subdomain i is cell i; its overlap of one cell is every cell its block row
// couples to (the face neighbours of the DG stencil), so a patch holds at most
// `w` cells (7 on the Cartesian levels) and m = w bs unknowns. The local
// matrix A_i = R_i A P_i is assembled from the level's ELL blocks and
// inverted once at setup (one workgroup per patch, Gauss-Jordan in shared
// memory; the patch matrices are SPD, so no pivoting is needed); absent
// neighbours at the boundary are identity rows/columns during the inversion
// and zero in the stored inverse. The inverse is stored transposed,
// [patch][column j][row i], so that the wavefront applying it reads
// consecutive addresses for each j (it is symmetric up to rounding).
//
// One sweep x = omega sum_i P_i A_i^-1 R_i v takes two launches:
//   k_as_apply  one wavefront per patch: gather R_i v (m values) into shared
//               memory, z_i = A_i^-1 (R_i v), store z_i;
//   k_as_gather one thread per (cell, component): sum the contributions of the
//               patches that contain the cell, in the fixed order of the
//               cell's own patch list, and update x (no atomics, so results
//               are deterministic).
// Further sweeps add omega M (v - A x) with the level's residual SpMV.
// In the mixed forms the local solves are single precision, as in the paper:
// the inverse (formed in FP64) is stored rounded to float, the local residual
// is rounded and the products are summed in float; the gather stays FP64.
// Algorithmic bytes per sweep: the stored inverses (n m^2 8), v gathered
// (w N 8), z written and read back (2 n m 8), x written.
#include <vector>

#include "omg_internal.h"

namespace omg {

constexpr int kAsMaxM = 70; // largest patch order in shared memory: 7 cells x 10 (P2)
static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// value of block (slot j, row r, column c) of cell i in the ELL pair layout
__device__ __forceinline__ double ell_val(const double* val, int n, int bs, int bsh, int j, int r, int c, int i) {
    return val[2 * ((((int64_t)j * bs + r) * bsh + (c >> 1)) * n + i) + (c & 1)];
}

template <int BS>
__global__ __launch_bounds__(256) void k_as_build(int n, int width, int w, const int* __restrict__ col,
                                                  const int* __restrict__ dslot, const double* __restrict__ val,
                                                  const int* __restrict__ cells, double* __restrict__ inv) {
    constexpr int BSH = (BS + 1) / 2;
    __shared__ double M[kAsMaxM * kAsMaxM];
    __shared__ double colp[kAsMaxM], rowp[kAsMaxM];
    __shared__ int pc[8];
    const int P = blockIdx.x;
    const int m = w * BS;
    if (threadIdx.x < w) pc[threadIdx.x] = cells[(int64_t)threadIdx.x * n + P];
    __syncthreads();
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int i = e / m, j = e % m;
        const int a = i / BS, r = i % BS, b = j / BS, c = j % BS;
        const int ca = pc[a], cb = pc[b];
        double v = 0.0;
        if (ca < 0 || cb < 0) {
            v = (i == j) ? 1.0 : 0.0;
        } else if (a == b) {
            v = ell_val(val, n, BS, BSH, dslot[ca], r, c, ca);
        } else {
            for (int s = 0; s < width; ++s)
                if (col[(int64_t)s * n + ca] == cb) {
                    v = ell_val(val, n, BS, BSH, s, r, c, ca);
                    break;
                }
        }
        M[i * m + j] = v;
    }
    // in-place Gauss-Jordan inversion
    for (int p = 0; p < m; ++p) {
        __syncthreads();
        const double piv = M[p * m + p];
        for (int t = threadIdx.x; t < m; t += blockDim.x) {
            colp[t] = M[t * m + p];
            rowp[t] = M[p * m + t] / piv;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
            const int i = e / m, j = e % m;
            double v;
            if (i == p) v = (j == p) ? 1.0 / piv : rowp[j];
            else if (j == p) v = -colp[i] / piv;
            else v = M[e] - colp[i] * rowp[j];
            M[e] = v;
        }
    }
    __syncthreads();
    double* out = inv + (int64_t)P * m * m;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int j = e / m, i = e % m; // out[j][i] = inverse(i, j)
        out[e] = (pc[i / BS] < 0 || pc[j / BS] < 0) ? 0.0 : M[i * m + j];
    }
}

// z_i = A_i^-1 R_i v for four patches per block, one wavefront each; T is
// the precision of the stored inverse and of the local solve.
template <int BS, typename T>
__global__ __launch_bounds__(256) void k_as_apply(int n, int w, const int* __restrict__ cells,
                                                  const T* __restrict__ inv, const double* __restrict__ v,
                                                  double* __restrict__ z) {
    __shared__ T rl[4][kAsMaxM];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int P = blockIdx.x * 4 + wid;
    if (P >= n) return; // whole wavefront
    const int m = w * BS;
    int np = 0;
    for (int a = 0; a < w; ++a) np += cells[(int64_t)a * n + P] >= 0 ? 1 : 0; // present cells come first
    const int ma = np * BS;
    for (int t = lane; t < m; t += 64) {
        const int cell = cells[(int64_t)(t / BS) * n + P];
        rl[wid][t] = cell >= 0 ? (T)v[(int64_t)(t % BS) * n + cell] : (T)0;
    }
    __builtin_amdgcn_wave_barrier();
    const T* Ti = inv + (int64_t)P * m * m;
    T acc0 = 0, acc1 = 0;
    const bool two = lane + 64 < ma;
    if (lane < ma) {
        // ma is a multiple of BS: BS independent column loads in flight per step
        for (int j0 = 0; j0 < ma; j0 += BS) {
            T t0[BS], t1[BS];
#pragma unroll
            for (int jj = 0; jj < BS; ++jj) {
                t0[jj] = Ti[(j0 + jj) * m + lane];
                t1[jj] = two ? Ti[(j0 + jj) * m + lane + 64] : (T)0;
            }
#pragma unroll
            for (int jj = 0; jj < BS; ++jj) {
                const T rj = rl[wid][j0 + jj];
                acc0 = fma(t0[jj], rj, acc0);
                acc1 = fma(t1[jj], rj, acc1);
            }
        }
        z[(int64_t)P * m + lane] = (double)acc0;
        if (two) z[(int64_t)P * m + lane + 64] = (double)acc1;
    }
}

// x = omega e (first sweep) or x + omega e, e_cell = sum of the cell's entries
// of the patches that contain it (rev: patch * w + slot, -1 none).
template <int BS>
__global__ __launch_bounds__(256) void k_as_gather(int n, int w, const int* __restrict__ rev,
                                                   const double* __restrict__ z, double omega, int accumulate,
                                                   double* __restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * BS) return;
    const int c = (int)(t / n), cell = (int)(t % n);
    const int m = w * BS;
    double e = 0.0;
    for (int s = 0; s < w; ++s) {
        const int q = rev[(int64_t)s * n + cell];
        if (q >= 0) e += z[(int64_t)(q / w) * m + (q % w) * BS + c];
    }
    x[t] = accumulate ? x[t] + omega * e : omega * e;
}

__global__ void k_as_round(int64_t cnt, const double* __restrict__ in, float* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < cnt) out[e] = (float)in[e];
}

#define OMG_AS_DISPATCH(bs, CALL)                              \
    switch (bs) {                                              \
    case 1: { constexpr int BSV = 1; CALL; } break;            \
    case 4: { constexpr int BSV = 4; CALL; } break;            \
    case 10: { constexpr int BSV = 10; CALL; } break;          \
    default: return OMG_EUNSUPPORTED;                          \
    }

// Patches (host, from the level's pattern), their inverses (device).
omg_status as_setup(omg_solver* s, Level& L) {
    const int n = L.n, bs = s->bs;
    std::vector<std::vector<int>> pc(n);
    int w = 1;
    for (int i = 0; i < n; ++i) {
        pc[i].push_back(i);
        for (int j = 0; j < L.width; ++j) {
            const int c = L.hcol[(size_t)j * n + i];
            bool seen = c == i;
            for (int d : pc[i]) seen = seen || d == c;
            if (!seen) pc[i].push_back(c);
        }
        w = std::max(w, (int)pc[i].size());
    }
    if (w * bs > kAsMaxM || w > 8) return OMG_EUNSUPPORTED;
    const int m = w * bs;
    std::vector<int> cells((size_t)w * n, -1), rev((size_t)w * n, -1);
    for (int i = 0; i < n; ++i)
        for (size_t a = 0; a < pc[i].size(); ++a) cells[a * n + i] = pc[i][a];
    // contributions to cell i: its own patch (slot 0), then the patches of its
    // neighbours in the order of i's patch list, at the slot i holds there
    for (int i = 0; i < n; ++i)
        for (size_t a = 0; a < pc[i].size(); ++a) {
            const int P = pc[i][a];
            int slot = -1;
            for (size_t b = 0; b < pc[P].size(); ++b)
                if (pc[P][b] == i) slot = (int)b;
            if (slot < 0) return OMG_EINVAL; // the pattern is not symmetric
            rev[a * n + i] = P * w + slot;
        }
    L.as_w = w;
    if (hipMalloc((void**)&L.as_cells, sizeof(int) * cells.size()) != hipSuccess ||
        hipMalloc((void**)&L.as_rev, sizeof(int) * rev.size()) != hipSuccess ||
        hipMalloc((void**)&L.as_inv, sizeof(double) * (size_t)n * m * m) != hipSuccess ||
        hipMalloc((void**)&L.as_z, sizeof(double) * (size_t)n * m) != hipSuccess) {
        (void)hipGetLastError();
        return OMG_ENOMEM;
    }
    OMG_TRY_HIP(hipMemcpy(L.as_cells, cells.data(), sizeof(int) * cells.size(), hipMemcpyHostToDevice));
    OMG_TRY_HIP(hipMemcpy(L.as_rev, rev.data(), sizeof(int) * rev.size(), hipMemcpyHostToDevice));
    OMG_AS_DISPATCH(bs, hipLaunchKernelGGL((k_as_build<BSV>), dim3(n), dim3(256), 0, s->stream, n, L.width, w, L.col,
                                           L.dslot, L.val, L.as_cells, L.as_inv));
    OMG_TRY_HIP(hipGetLastError());
    if (s->opt.precision != OMG_FP64) { // single-precision local solves of the mixed forms
        const int64_t cnt = (int64_t)n * m * m;
        if (hipMalloc((void**)&L.as_inv32, sizeof(float) * cnt) != hipSuccess) {
            (void)hipGetLastError();
            return OMG_ENOMEM;
        }
        hipLaunchKernelGGL(k_as_round, dim3(cdiv(cnt, 256)), dim3(256), 0, s->stream, cnt, L.as_inv, L.as_inv32);
        OMG_TRY_HIP(hipGetLastError());
    }
    return OMG_OK;
}

template <int BS>
static void as_sweep(const Level& L, bool fp32, double omega, const double* v, double* out, bool accumulate,
                     hipStream_t st) {
    const int n = L.n, w = L.as_w;
    if (fp32)
        hipLaunchKernelGGL((k_as_apply<BS, float>), dim3(cdiv(n, 4)), dim3(256), 0, st, n, w, L.as_cells, L.as_inv32,
                           v, L.as_z);
    else
        hipLaunchKernelGGL((k_as_apply<BS, double>), dim3(cdiv(n, 4)), dim3(256), 0, st, n, w, L.as_cells, L.as_inv,
                           v, L.as_z);
    hipLaunchKernelGGL((k_as_gather<BS>), dim3(cdiv((int64_t)n * BS, 256)), dim3(256), 0, st, n, w, L.as_rev, L.as_z,
                       omega, (int)accumulate, out);
}

// One sweep: out = omega M v (accumulate = 0) or out + omega M v; fp32
// selects the single-precision local solves.
hipError_t launch_as_sweep(const Level& L, int bs, bool fp32, double omega, const double* v, double* out,
                           bool accumulate, hipStream_t st) {
    if (!L.as_inv || L.as_w * bs > kAsMaxM || (fp32 && !L.as_inv32)) return hipErrorInvalidValue;
    switch (bs) {
    case 1: as_sweep<1>(L, fp32, omega, v, out, accumulate, st); break;
    case 4: as_sweep<4>(L, fp32, omega, v, out, accumulate, st); break;
    case 10: as_sweep<10>(L, fp32, omega, v, out, accumulate, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace omg
