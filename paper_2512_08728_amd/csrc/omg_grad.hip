// Per-cell contraction g_nu[K] = -lambda^T (dA/dnu_K) u for the SIP operator
// assembled by omg_setup_sip. A(nu) = sum_K nu_K S_K + sum_F nu_F(nu-, nu+) B_F
// + sum_{boundary F} nu_K B_F, with nu_F the harmonic mean, so
// dA/dnu_K = S_K + sum_{boundary F of K} B_F
//            + sum_{interior F of K} (2 nu_N^2 / (nu_K + nu_N)^2) B_F.
// Thread per cell; each interior face term is evaluated by both neighbours
// (no atomics, deterministic).
#include "omg_internal.h"

namespace omg {

template <int BS>
__device__ __forceinline__ double qf(const double* __restrict__ M, const double* a, const double* b) {
    double s = 0.0;
    for (int r = 0; r < BS; ++r) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) t = fma(M[r * BS + c], b[c], t);
        s = fma(a[r], t, s);
    }
    return s;
}

template <int BS>
__global__ __launch_bounds__(128) void k_contract(int nx, int ny, int nz, const double* __restrict__ nu,
                                                  const double* __restrict__ refm, const double* __restrict__ lam,
                                                  const double* __restrict__ u, double* __restrict__ g) {
    const int n = nx * ny * nz;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int bb = BS * BS;
    const double* S = refm;
    const double* F = refm + bb;
    const double* B = F + 12 * bb;
    const int ijk[3] = {i % nx, (i / nx) % ny, i / (nx * ny)};
    const int dims[3] = {nx, ny, nz}, stride[3] = {1, nx, nx * ny};
    double li[BS], ui[BS], ln[BS], un[BS];
    for (int k = 0; k < BS; ++k) {
        li[k] = lam[(int64_t)i * BS + k];
        ui[k] = u[(int64_t)i * BS + k];
    }
    const double nk = nu[i];
    double acc = qf<BS>(S, li, ui);
    for (int d = 0; d < 3; ++d) {
        for (int side = 0; side < 2; ++side) {
            const bool up = side == 1;
            const bool inside = up ? (ijk[d] < dims[d] - 1) : (ijk[d] > 0);
            if (!inside) {
                acc += qf<BS>(B + (d * 2 + side) * bb, li, ui);
                continue;
            }
            const int j = up ? i + stride[d] : i - stride[d];
            for (int k = 0; k < BS; ++k) {
                ln[k] = lam[(int64_t)j * BS + k];
                un[k] = u[(int64_t)j * BS + k];
            }
            const double nn = nu[j];
            const double dnf = 2.0 * nn * nn / ((nk + nn) * (nk + nn));
            // face with lower cell lo and upper cell hi
            const double *llo = up ? li : ln, *ulo = up ? ui : un, *lhi = up ? ln : li, *uhi = up ? un : ui;
            const double* Fd = F + (d * 4) * bb;
            const double face = qf<BS>(Fd + 0 * bb, llo, ulo) + qf<BS>(Fd + 1 * bb, llo, uhi) +
                                qf<BS>(Fd + 2 * bb, lhi, ulo) + qf<BS>(Fd + 3 * bb, lhi, uhi);
            acc += dnf * face;
        }
    }
    g[i] = -acc;
}

} // namespace omg

using namespace omg;

hipError_t omg_launch_contract(const omg_solver* s, const double* lam, const double* u, double* g_nu,
                               hipStream_t st) {
    const Level& L = s->lev[0];
    dim3 grid((L.n + 127) / 128), block(128);
    switch (s->bs) {
    case 1: hipLaunchKernelGGL(k_contract<1>, grid, block, 0, st, L.nx, L.ny, L.nz, s->nu, s->refm, lam, u, g_nu); break;
    case 4: hipLaunchKernelGGL(k_contract<4>, grid, block, 0, st, L.nx, L.ny, L.nz, s->nu, s->refm, lam, u, g_nu); break;
    case 10: hipLaunchKernelGGL(k_contract<10>, grid, block, 0, st, L.nx, L.ny, L.nz, s->nu, s->refm, lam, u, g_nu); break;
    case 20: hipLaunchKernelGGL(k_contract<20>, grid, block, 0, st, L.nx, L.ny, L.nz, s->nu, s->refm, lam, u, g_nu); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
