// Setup of the OrthoMG hierarchy on the device: operator ingest into the
// interleaved ELL layout, SIP-DG assembly from a per-cell coefficient,
// Galerkin coarse operators A_{l+1} = P^T A_l P, block-diagonal inverses for
// block-Jacobi (Algorithm 4 with precomputed inverses, Sec. 3.3) and the dense
// Cholesky factor / inverse of the coarsest level.
//
// The element matrices and the embedding blocks are computed here in closed
// form from 1D Legendre identities (exact polynomial integration), not by
// numerical quadrature.
#include <algorithm>
#include <cmath>
#include <cstring>

#include <cstdlib>

#include "omg_internal.h"

namespace omg {

int reduction_blocks(int64_t N) {
    int64_t b = (N + kThreads * 8 - 1) / (kThreads * 8);
    if (b < 1) b = 1;
    if (b > kMaxRedBlocks) b = kMaxRedBlocks;
    return (int)b;
}

// Basis order: total degree d = 0..p, then (a,b,c) lexicographically
// descending with a+b+c = d.
void basis_orders(int p, std::vector<int>& a, std::vector<int>& b, std::vector<int>& c) {
    a.clear();
    b.clear();
    c.clear();
    for (int d = 0; d <= p; ++d)
        for (int i = d; i >= 0; --i)
            for (int j = d - i; j >= 0; --j) {
                a.push_back(i);
                b.push_back(j);
                c.push_back(d - i - j);
            }
}

static double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// Monomial coefficients of psi_m(t) = sqrt(2m+1) P_m(2t-1):
// P_m(2t-1) = sum_k (-1)^{m+k} C(m,k) C(m+k,k) t^k (shifted Legendre).
static std::vector<double> psi_coeffs(int m) {
    std::vector<double> c(m + 1);
    for (int k = 0; k <= m; ++k)
        c[k] = std::sqrt(2.0 * m + 1.0) * (((m + k) & 1) ? -1.0 : 1.0) * binom(m, k) * binom(m + k, k);
    return c;
}

// 1D embedding e^{side}_{n m} = int_child chi_n psi_m^{parent}, child basis
// chi_n(t) = sqrt(2) psi_n(2t - side). With u = 2t - side:
// e_{nm} = (1/sqrt2) int_0^1 psi_m((u + side)/2) psi_n(u) du, integrated exactly.
static double embed1d(int side, int n, int m) {
    std::vector<double> pm = psi_coeffs(m), pn = psi_coeffs(n);
    // q(u) = psi_m((u+side)/2) in monomials of u
    std::vector<double> q(m + 1, 0.0);
    for (int k = 0; k <= m; ++k) {
        double ck = pm[k] / std::pow(2.0, k);
        for (int j = 0; j <= k; ++j) q[j] += ck * binom(k, j) * std::pow((double)side, k - j);
    }
    double s = 0.0;
    for (int i = 0; i <= m; ++i)
        for (int j = 0; j <= n; ++j) s += q[i] * pn[j] / (i + j + 1.0);
    return s / std::sqrt(2.0);
}

void embedding_blocks(int p, std::vector<double>& E) {
    std::vector<int> a, b, c;
    basis_orders(p, a, b, c);
    const int bs = (int)a.size();
    double e[2][8][8];
    for (int side = 0; side < 2; ++side)
        for (int n = 0; n <= p; ++n)
            for (int m = 0; m <= p; ++m) e[side][n][m] = embed1d(side, n, m);
    E.assign((size_t)8 * bs * bs, 0.0);
    for (int s = 0; s < 8; ++s) {
        const int sx = s & 1, sy = (s >> 1) & 1, sz = (s >> 2) & 1;
        for (int r = 0; r < bs; ++r)
            for (int q = 0; q < bs; ++q)
                E[((size_t)s * bs + r) * bs + q] = e[sx][a[r]][a[q]] * e[sy][b[r]][b[q]] * e[sz][c[r]][c[q]];
    }
}

// Unit-coefficient SIP element matrices on a cube of side h (row = test, col
// = trial), in closed form from the 1D values
//   psi_m(0) = sqrt(2m+1)(-1)^m, psi_m(1) = sqrt(2m+1),
//   psi_m'(0) = sqrt(2m+1)(-1)^{m+1} m(m+1), psi_m'(1) = sqrt(2m+1) m(m+1),
//   int_0^1 psi_m' psi_n' = 2 sqrt((2m+1)(2n+1)) k(k+1) [m+n even], k = min(m,n),
// and orthonormality in the tangential directions. Output layout:
// S | F[d][X][Y] (X,Y: 0 lower cell, 1 upper cell; normal +e_d) | B[d][side]
// (side 0: low boundary face, outward -e_d; 1: high), each bs*bs.
//   interior: -int {du/dn}[v] - int {dv/dn}[u] + sigma int [u][v]
//   boundary: -int du/dn v - int dv/dn u + sigma int u v
void reference_matrices(int p, double h, double penalty_c, std::vector<double>& out) {
    std::vector<int> o[3];
    basis_orders(p, o[0], o[1], o[2]);
    const int bs = (int)o[0].size(), bb = bs * bs;
    auto v0 = [](int m) { return std::sqrt(2.0 * m + 1.0) * ((m & 1) ? -1.0 : 1.0); };
    auto v1 = [](int m) { return std::sqrt(2.0 * m + 1.0); };
    auto d0 = [](int m) { return std::sqrt(2.0 * m + 1.0) * ((m & 1) ? 1.0 : -1.0) * m * (m + 1.0); };
    auto d1 = [](int m) { return std::sqrt(2.0 * m + 1.0) * m * (m + 1.0); };
    auto kk = [](int m, int n) {
        if ((m + n) & 1) return 0.0;
        int k = std::min(m, n);
        return 2.0 * std::sqrt((2.0 * m + 1.0) * (2.0 * n + 1.0)) * k * (k + 1.0);
    };
    const double sh = penalty_c * (p + 1.0) * (p + 3.0); // sigma * h
    const double sc = 1.0 / (h * h);
    out.assign((size_t)bb * (1 + 12 + 6), 0.0);
    double* S = out.data();
    double* F = S + bb;
    double* B = F + 12 * bb;
    for (int m = 0; m < bs; ++m)
        for (int n = 0; n < bs; ++n) {
            double s = 0.0;
            for (int d = 0; d < 3; ++d) {
                bool tan_eq = true;
                for (int e = 0; e < 3; ++e)
                    if (e != d && o[e][m] != o[e][n]) tan_eq = false;
                if (tan_eq) s += kk(o[d][m], o[d][n]);
            }
            S[m * bs + n] = sc * s;
        }
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < bs; ++m)
            for (int n = 0; n < bs; ++n) {
                bool tan_eq = true;
                for (int e = 0; e < 3; ++e)
                    if (e != d && o[e][m] != o[e][n]) tan_eq = false;
                if (!tan_eq) continue;
                const int md = o[d][m], nd = o[d][n];
                for (int X = 0; X < 2; ++X)
                    for (int Y = 0; Y < 2; ++Y) {
                        // the lower cell sees the face at t = 1, the upper cell at t = 0;
                        // jump sign +1 for the lower cell, -1 for the upper cell
                        const double vX = X ? v0(md) : v1(md), dX = X ? d0(md) : d1(md), sX = X ? -1.0 : 1.0;
                        const double vY = Y ? v0(nd) : v1(nd), dY = Y ? d0(nd) : d1(nd), sY = Y ? -1.0 : 1.0;
                        F[((size_t)(d * 2 + X) * 2 + Y) * bb + m * bs + n] =
                            sc * (-0.5 * dY * sX * vX - 0.5 * dX * sY * vY + sh * sX * sY * vX * vY);
                    }
                // low face: outward normal -e_d, so du/dn = -u'(0)
                B[(size_t)(d * 2 + 0) * bb + m * bs + n] =
                    sc * (d0(nd) * v0(md) + d0(md) * v0(nd) + sh * v0(md) * v0(nd));
                B[(size_t)(d * 2 + 1) * bb + m * bs + n] =
                    sc * (-d1(nd) * v1(md) - d1(md) * v1(nd) + sh * v1(md) * v1(nd));
            }
}

// ---------------------------------------------------------------- kernels
__device__ __forceinline__ double harm(double a, double b) { return 2.0 * a * b / (a + b); }

// SIP assembly A(nu) into the ELL layout with 7 direction slots
// (-z, -y, -x, self, +x, +y, +z); absent neighbours give zero padding slots
// pointing at the cell itself. Thread per (cell, slot).
__global__ void k_assemble_sip(int nx, int ny, int nz, int bs, int bsh, const double* __restrict__ nu,
                               const double* __restrict__ refm, int* __restrict__ col, double* __restrict__ val) {
    const int n = nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * 7) return;
    const int i = (int)(t % n), j = (int)(t / n);
    const int ijk[3] = {i % nx, (i / nx) % ny, i / (nx * ny)};
    const int dims[3] = {nx, ny, nz};
    const int stride[3] = {1, nx, nx * ny};
    const int bb = bs * bs;
    const double* S = refm;
    const double* F = refm + bb;      // F[d][X][Y]
    const double* B = F + 12 * bb;    // B[d][side]
    double2* out = (double2*)val;
    auto put = [&](int r, int c, double v) {
        double* o = (double*)&out[((int64_t)(j * bs + r) * bsh + (c >> 1)) * n + i];
        o[c & 1] = v;
    };
    // zero the block first (including the padding column of odd bs)
    for (int r = 0; r < bs; ++r)
        for (int cp = 0; cp < bsh; ++cp) out[((int64_t)(j * bs + r) * bsh + cp) * n + i] = make_double2(0.0, 0.0);
    int c = i;
    if (j == 3) {
        const double nk = nu[i];
        for (int r = 0; r < bs; ++r)
            for (int q = 0; q < bs; ++q) {
                double v = nk * S[r * bs + q];
                for (int d = 0; d < 3; ++d) {
                    if (ijk[d] < dims[d] - 1) {
                        v += harm(nk, nu[i + stride[d]]) * F[((d * 2 + 0) * 2 + 0) * bb + r * bs + q];
                    } else {
                        v += nk * B[(d * 2 + 1) * bb + r * bs + q];
                    }
                    if (ijk[d] > 0) {
                        v += harm(nu[i - stride[d]], nk) * F[((d * 2 + 1) * 2 + 1) * bb + r * bs + q];
                    } else {
                        v += nk * B[(d * 2 + 0) * bb + r * bs + q];
                    }
                }
                put(r, q, v);
            }
    } else {
        const int d = (j < 3) ? 2 - j : j - 4; // slot -> direction
        const bool up = j > 3;
        if (up ? (ijk[d] < dims[d] - 1) : (ijk[d] > 0)) {
            c = up ? i + stride[d] : i - stride[d];
            const double nf = up ? harm(nu[i], nu[c]) : harm(nu[c], nu[i]);
            // this cell is the lower one (X=0) for +d, the upper one (X=1) for -d
            const double* M = up ? F + ((d * 2 + 0) * 2 + 1) * bb : F + ((d * 2 + 1) * 2 + 0) * bb;
            for (int r = 0; r < bs; ++r)
                for (int q = 0; q < bs; ++q) put(r, q, nf * M[r * bs + q]);
        }
    }
    col[(int64_t)j * n + i] = c;
}

// Galerkin product: coarse block (slot j, cell I) = sum over its contribution
// list of E_{s(K)}^T A_{K, jf} E_{s(K')}, K' = col(K, jf). One block of
// threads per coarse block; contributions summed in list order (fine cell
// ascending, slot ascending).
__global__ void k_galerkin(int bs, int bsh, const int* __restrict__ fup, int fn, const int* __restrict__ fcol,
                           const double* __restrict__ fval, int cn, const int64_t* __restrict__ cptr,
                           const int* __restrict__ cK, const int* __restrict__ cj, const double* __restrict__ E,
                           double* __restrict__ cval, int cwidth) {
    extern __shared__ double smem[];
    const int bb = bs * bs;
    double* sA = smem;          // bb
    double* sT = sA + bb;       // bb
    double* sE = sT + bb;       // 8*bb
    const int64_t blk = blockIdx.x; // = jc * cn + I
    const int I = (int)(blk % cn), jc = (int)(blk / cn);
    for (int e = threadIdx.x; e < 8 * bb; e += blockDim.x) sE[e] = E[e];
    double acc[4] = {0, 0, 0, 0};  // up to 4 outputs per thread (bs <= 20 with 128+ threads -> 400/256 < 2)
    __syncthreads();
    const double2* fv = (const double2*)fval;
    for (int64_t q = cptr[blk]; q < cptr[blk + 1]; ++q) {
        const int K = cK[q], jf = cj[q];
        const int Kp = fcol[(int64_t)jf * fn + K];
        const int sK = fup[K] & 7;
        const int sKp = fup[Kp] & 7;
        for (int e = threadIdx.x; e < bb; e += blockDim.x) {
            const int r = e / bs, c = e % bs;
            const double2 v = fv[((int64_t)(jf * bs + r) * bsh + (c >> 1)) * fn + K];
            sA[e] = (c & 1) ? v.y : v.x;
        }
        __syncthreads();
        const double* E2 = sE + sKp * bb;
        for (int e = threadIdx.x; e < bb; e += blockDim.x) { // T = A E_{s(K')}
            const int r = e / bs, c = e % bs;
            double s = 0.0;
            for (int m = 0; m < bs; ++m) s = fma(sA[r * bs + m], E2[m * bs + c], s);
            sT[e] = s;
        }
        __syncthreads();
        const double* E1 = sE + sK * bb;
        int slot = 0;
        for (int e = threadIdx.x; e < bb; e += blockDim.x, ++slot) { // acc += E_{s(K)}^T T
            const int r = e / bs, c = e % bs;
            double s = 0.0;
            for (int m = 0; m < bs; ++m) s = fma(E1[m * bs + r], sT[m * bs + c], s);
            acc[slot] += s;
        }
        __syncthreads();
    }
    double* cv = cval;
    int slot = 0;
    for (int e = threadIdx.x; e < bb; e += blockDim.x, ++slot) {
        const int r = e / bs, c = e % bs;
        cv[(((int64_t)(jc * bs + r) * bsh + (c >> 1)) * cn + I) * 2 + (c & 1)] = acc[slot];
    }
    (void)cwidth;
}

// Inverse of each diagonal block by Cholesky (thread per cell); the inverse
// is written in the pair layout. Sets *err on a non-positive pivot.
template <int BS>
__global__ void k_block_inverse(int n, int width, const int* __restrict__ dslot, const double* __restrict__ val,
                                double* __restrict__ dinv, int* __restrict__ err) {
    constexpr int BSH = (BS + 1) / 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int jd = dslot[i];
    if (jd < 0 || jd >= width) {
        *err = 2;
        return;
    }
    double L[BS * BS];
    const double2* v = (const double2*)val;
    for (int r = 0; r < BS; ++r)
        for (int c = 0; c < BS; ++c) {
            const double2 p = v[((int64_t)(jd * BS + r) * BSH + (c >> 1)) * n + i];
            L[r * BS + c] = (c & 1) ? p.y : p.x;
        }
    for (int j = 0; j < BS; ++j) {
        double d = L[j * BS + j];
        for (int q = 0; q < j; ++q) d -= L[j * BS + q] * L[j * BS + q];
        if (!(d > 0.0)) {
            *err = 1;
            d = 1.0;
        }
        const double ljj = sqrt(d);
        L[j * BS + j] = ljj;
        for (int r = j + 1; r < BS; ++r) {
            double s = L[r * BS + j];
            for (int q = 0; q < j; ++q) s -= L[r * BS + q] * L[j * BS + q];
            L[r * BS + j] = s / ljj;
        }
    }
    double X[BS * BS];
    for (int c = 0; c < BS; ++c) { // solve L L^T x = e_c
        double y[BS];
        for (int r = 0; r < BS; ++r) {
            double s = (r == c) ? 1.0 : 0.0;
            for (int q = 0; q < r; ++q) s -= L[r * BS + q] * y[q];
            y[r] = s / L[r * BS + r];
        }
        for (int r = BS - 1; r >= 0; --r) {
            double s = y[r];
            for (int q = r + 1; q < BS; ++q) s -= L[q * BS + r] * y[q];
            y[r] = s / L[r * BS + r];
        }
        for (int r = 0; r < BS; ++r) X[r * BS + c] = y[r];
    }
    double2* o = (double2*)dinv;
    for (int r = 0; r < BS; ++r)
        for (int cp = 0; cp < BSH; ++cp) {
            const double a = X[r * BS + 2 * cp];
            const double b = (2 * cp + 1 < BS) ? X[r * BS + 2 * cp + 1] : 0.0;
            o[(int64_t)(r * BSH + cp) * n + i] = make_double2(a, b);
        }
}

__global__ void k_to_float(const double* __restrict__ in, float* __restrict__ out, int64_t N) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) out[e] = (float)in[e];
}

// Dense SoA-ordered matrix of the coarsest level: row (r*n + i), column
// (c*n + col). Padded rows/columns [N, np) hold the identity.
__global__ void k_densify(int n, int width, int bs, int bsh, int np, const int* __restrict__ col,
                          const double* __restrict__ val, double* __restrict__ D) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * width * bs) return;
    const int i = (int)(t % n);
    const int j = (int)((t / n) % width);
    const int r = (int)(t / ((int64_t)n * width));
    const int cc = col[(int64_t)j * n + i];
    const double2* v = (const double2*)val;
    for (int c = 0; c < bs; ++c) {
        const double2 p = v[((int64_t)(j * bs + r) * bsh + (c >> 1)) * n + i];
        const double a = (c & 1) ? p.y : p.x;
        if (a != 0.0) D[(int64_t)(r * n + i) * np + (int64_t)c * n + cc] += a;
    }
}
__global__ void k_pad_identity(int N, int np, double* D) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x + N;
    if (t < np) D[(int64_t)t * np + t] = 1.0;
}

// ---- blocked dense Cholesky (tile 32) and inverse
constexpr int NB = 32;

// Factor the diagonal tile k in place (lower) and store its inverse in linv[k].
__global__ __launch_bounds__(256) void k_potrf_tile(double* A, int np, int k, double* linv, int* err) {
    __shared__ double T[NB][NB + 1];
    __shared__ double X[NB][NB + 1];
    const int tid = threadIdx.x;
    double* a = A + (int64_t)k * NB * np + (int64_t)k * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) T[e / NB][e % NB] = a[(int64_t)(e / NB) * np + e % NB];
    __syncthreads();
    for (int j = 0; j < NB; ++j) {
        if (tid == 0) {
            double d = T[j][j];
            for (int q = 0; q < j; ++q) d -= T[j][q] * T[j][q];
            if (!(d > 0.0)) {
                *err = 1;
                d = 1.0;
            }
            T[j][j] = sqrt(d);
        }
        __syncthreads();
        if (tid > j && tid < NB) {
            double s = T[tid][j];
            for (int q = 0; q < j; ++q) s -= T[tid][q] * T[j][q];
            T[tid][j] = s / T[j][j];
        }
        __syncthreads();
    }
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int r = e / NB, c = e % NB;
        if (c > r) T[r][c] = 0.0;
    }
    __syncthreads();
    if (tid < NB) { // column tid of T^-1 by forward substitution
        const int c = tid;
        for (int r = 0; r < NB; ++r) {
            if (r < c) {
                X[r][c] = 0.0;
                continue;
            }
            double s = (r == c) ? 1.0 : 0.0;
            for (int q = c; q < r; ++q) s -= T[r][q] * X[q][c];
            X[r][c] = s / T[r][r];
        }
    }
    __syncthreads();
    double* li = linv + (int64_t)k * NB * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        a[(int64_t)(e / NB) * np + e % NB] = T[e / NB][e % NB];
        li[e] = X[e / NB][e % NB];
    }
}

// Panel: L_ik = A_ik (L_kk^-1)^T for the tile rows below k.
__global__ __launch_bounds__(256) void k_trsm_panel(double* A, int np, int k, const double* linv) {
    __shared__ double Bt[NB][NB + 1];
    __shared__ double Li[NB][NB + 1];
    const int i = k + 1 + blockIdx.x;
    const int tid = threadIdx.x;
    double* a = A + (int64_t)i * NB * np + (int64_t)k * NB;
    const double* li = linv + (int64_t)k * NB * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        Bt[e / NB][e % NB] = a[(int64_t)(e / NB) * np + e % NB];
        Li[e / NB][e % NB] = li[e];
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int r = e / NB, c = e % NB;
        double s = 0.0;
        for (int q = 0; q <= c; ++q) s = fma(Bt[r][q], Li[c][q], s);
        a[(int64_t)r * np + c] = s;
    }
}

__device__ __forceinline__ void tri_index(int64_t t, int& i, int& j) {
    int a = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(a + 1) * (a + 2) / 2 <= t) ++a;
    while ((int64_t)a * (a + 1) / 2 > t) --a;
    i = a;
    j = (int)(t - (int64_t)a * (a + 1) / 2);
}

// Trailing update A_ij -= L_ik L_jk^T for k < j <= i.
__global__ __launch_bounds__(256) void k_syrk_update(double* A, int np, int k) {
    __shared__ double Pi[NB][NB + 1];
    __shared__ double Pj[NB][NB + 1];
    int ii, jj;
    tri_index(blockIdx.x, ii, jj);
    const int i = k + 1 + ii, j = k + 1 + jj;
    const int tid = threadIdx.x;
    const double* li = A + (int64_t)i * NB * np + (int64_t)k * NB;
    const double* lj = A + (int64_t)j * NB * np + (int64_t)k * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        Pi[e / NB][e % NB] = li[(int64_t)(e / NB) * np + e % NB];
        Pj[e / NB][e % NB] = lj[(int64_t)(e / NB) * np + e % NB];
    }
    __syncthreads();
    double* a = A + (int64_t)i * NB * np + (int64_t)j * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int r = e / NB, c = e % NB;
        double s = 0.0;
        for (int q = 0; q < NB; ++q) s = fma(Pi[r][q], Pj[c][q], s);
        a[(int64_t)r * np + c] -= s;
    }
}

// X = L^-1 (lower): X_kk = linv[k]; for tile row i, every k < i:
// X_ik = -linv[i] sum_{j=k}^{i-1} L_ij X_jk.
__global__ __launch_bounds__(256) void k_trinv_diag(double* X, int np, const double* linv) {
    const int k = blockIdx.x;
    const double* li = linv + (int64_t)k * NB * NB;
    double* x = X + (int64_t)k * NB * np + (int64_t)k * NB;
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) x[(int64_t)(e / NB) * np + e % NB] = li[e];
}
__global__ __launch_bounds__(256) void k_trinv_row(const double* L, double* X, int np, int i, const double* linv) {
    __shared__ double Ta[NB][NB + 1];
    __shared__ double Tb[NB][NB + 1];
    __shared__ double Acc[NB][NB + 1];
    const int k = blockIdx.x; // k < i
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += blockDim.x) Acc[e / NB][e % NB] = 0.0;
    for (int j = k; j < i; ++j) {
        __syncthreads();
        const double* lij = L + (int64_t)i * NB * np + (int64_t)j * NB;
        const double* xjk = X + (int64_t)j * NB * np + (int64_t)k * NB;
        for (int e = tid; e < NB * NB; e += blockDim.x) {
            Ta[e / NB][e % NB] = lij[(int64_t)(e / NB) * np + e % NB];
            Tb[e / NB][e % NB] = xjk[(int64_t)(e / NB) * np + e % NB];
        }
        __syncthreads();
        for (int e = tid; e < NB * NB; e += blockDim.x) {
            const int r = e / NB, c = e % NB;
            double s = 0.0;
            for (int q = 0; q < NB; ++q) s = fma(Ta[r][q], Tb[q][c], s);
            Acc[r][c] += s;
        }
    }
    __syncthreads();
    const double* li = linv + (int64_t)i * NB * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) Ta[e / NB][e % NB] = li[e];
    __syncthreads();
    double* xik = X + (int64_t)i * NB * np + (int64_t)k * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int r = e / NB, c = e % NB;
        double s = 0.0;
        for (int q = 0; q <= r; ++q) s = fma(Ta[r][q], Acc[q][c], s);
        xik[(int64_t)r * np + c] = -s;
    }
}

// Ainv_IJ = sum_{k >= max(I,J)} X_kI^T X_kJ (full matrix).
__global__ __launch_bounds__(256) void k_xtx(const double* X, double* Ainv, int np, int nt) {
    __shared__ double Ta[NB][NB + 1];
    __shared__ double Tb[NB][NB + 1];
    const int I = blockIdx.x % nt, J = blockIdx.x / nt;
    const int tid = threadIdx.x;
    double acc[(NB * NB + 255) / 256] = {};
    for (int k = max(I, J); k < nt; ++k) {
        __syncthreads();
        const double* xa = X + (int64_t)k * NB * np + (int64_t)I * NB;
        const double* xb = X + (int64_t)k * NB * np + (int64_t)J * NB;
        for (int e = tid; e < NB * NB; e += blockDim.x) {
            Ta[e / NB][e % NB] = xa[(int64_t)(e / NB) * np + e % NB];
            Tb[e / NB][e % NB] = xb[(int64_t)(e / NB) * np + e % NB];
        }
        __syncthreads();
        int s = 0;
        for (int e = tid; e < NB * NB; e += blockDim.x, ++s) {
            const int r = e / NB, c = e % NB;
            double v = 0.0;
            for (int q = 0; q < NB; ++q) v = fma(Ta[q][r], Tb[q][c], v);
            acc[s] += v;
        }
    }
    double* o = Ainv + (int64_t)I * NB * np + (int64_t)J * NB;
    int s = 0;
    for (int e = tid; e < NB * NB; e += blockDim.x, ++s) o[(int64_t)(e / NB) * np + e % NB] = acc[s];
}

} // namespace omg

// ====================================================================== host
using namespace omg;

static inline int cdivi(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

static omg_status dmalloc(void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return OMG_ENOMEM;
    }
    return OMG_OK;
}

omg_status omg_alloc_level_vectors(omg_solver* s, Level& L) {
    const size_t vb = sizeof(double) * (size_t)(std::max<int64_t>(L.N, 1) + kVecPad);
    OMG_TRY(dmalloc((void**)&L.b, vb));
    OMG_TRY(dmalloc((void**)&L.xout, vb));
    OMG_TRY(dmalloc((void**)&L.scal, sizeof(double) * S_COUNT));
    OMG_TRY_HIP(hipMemsetAsync(L.scal, 0, sizeof(double) * S_COUNT, s->stream));
    OMG_TRY(dmalloc((void**)&L.r, vb));
    OMG_TRY(dmalloc((void**)&L.x, vb));
    OMG_TRY(dmalloc((void**)&L.z, vb));
    OMG_TRY(dmalloc((void**)&L.w, vb));
    OMG_TRY(dmalloc((void**)&L.t, vb));
    OMG_TRY(dmalloc((void**)&L.t2, vb));
    OMG_TRY(dmalloc((void**)&L.zcor, vb));
    for (double* v : {L.b, L.xout, L.r, L.x, L.z, L.w, L.t, L.t2, L.zcor}) // zero tails
        OMG_TRY_HIP(hipMemsetAsync(v, 0, vb, s->stream));
    OMG_TRY(dmalloc((void**)&L.part, sizeof(double) * 16 * kMaxRedBlocks));
    return OMG_OK;
}

// Diagonal slot of every cell from the host pattern (padding slots also point
// at the cell itself, so the first valid slot with column == cell is taken).
static omg_status upload_dslot(omg_solver* s, Level& L, const std::vector<unsigned char>& valid) {
    int64_t cnt = 0;
    for (unsigned char v : valid) cnt += v;
    s->nnzb_level[&L - s->lev.data()] = cnt;
    std::vector<int> ds(L.n, -1);
    for (int i = 0; i < L.n; ++i)
        for (int j = 0; j < L.width; ++j)
            if (valid[(size_t)j * L.n + i] && L.hcol[(size_t)j * L.n + i] == i) {
                ds[i] = j;
                break;
            }
    for (int i = 0; i < L.n; ++i)
        if (ds[i] < 0) return OMG_EINVAL;
    OMG_TRY(dmalloc((void**)&L.dslot, sizeof(int) * L.n));
    OMG_TRY_HIP(hipMemcpy(L.dslot, ds.data(), sizeof(int) * L.n, hipMemcpyHostToDevice));
    return OMG_OK;
}

// Allocate the ELL arrays of a level (width already set).
static omg_status alloc_ell(omg_solver* s, Level& L) {
    const int64_t slots = (int64_t)L.width * L.n;
    OMG_TRY(dmalloc((void**)&L.col, sizeof(int) * slots));
    OMG_TRY(dmalloc((void**)&L.val, sizeof(double) * 2 * slots * s->bs * s->bsh));
    return OMG_OK;
}

// Host-side ELL conversion of a caller BSR; rows padded with zero blocks
// pointing at the row's own cell.
omg_status omg_ingest_bsr(omg_solver* s, const omg_bsr* A, std::vector<unsigned char>& valid) {
    Level& L = s->lev[0];
    const int n = A->n_cells, bs = s->bs, bsh = s->bsh;
    int width = 0;
    for (int i = 0; i < n; ++i) width = std::max(width, A->row_ptr[i + 1] - A->row_ptr[i]);
    L.width = width;
    OMG_TRY(alloc_ell(s, L));
    std::vector<int> hcol((size_t)width * n);
    valid.assign((size_t)width * n, 0);
    std::vector<double> hval((size_t)2 * width * n * bs * bsh, 0.0);
    for (int i = 0; i < n; ++i) {
        const int len = A->row_ptr[i + 1] - A->row_ptr[i];
        for (int j = 0; j < width; ++j) {
            const size_t o = (size_t)j * n + i;
            if (j < len) {
                const int64_t q = A->row_ptr[i] + j;
                hcol[o] = A->col_idx[q];
                valid[o] = 1;
                const double* blk = A->val + (size_t)q * bs * bs;
                for (int r = 0; r < bs; ++r)
                    for (int c = 0; c < bs; ++c)
                        hval[((((size_t)j * bs + r) * bsh + (c >> 1)) * n + i) * 2 + (c & 1)] = blk[r * bs + c];
            } else {
                hcol[o] = i;
            }
        }
    }
    L.hcol = hcol;
    OMG_TRY(upload_dslot(s, L, valid));
    OMG_TRY_HIP(hipMemcpyAsync(L.col, hcol.data(), sizeof(int) * hcol.size(), hipMemcpyHostToDevice, s->stream));
    OMG_TRY_HIP(hipMemcpyAsync(L.val, hval.data(), sizeof(double) * hval.size(), hipMemcpyHostToDevice, s->stream));
    OMG_TRY_HIP(hipStreamSynchronize(s->stream));
    return OMG_OK;
}

omg_status omg_assemble_sip(omg_solver* s, const double* nu_dev, std::vector<unsigned char>& valid) {
    Level& L = s->lev[0];
    L.width = 7;
    OMG_TRY(alloc_ell(s, L));
    std::vector<double> refm;
    reference_matrices(s->p, s->grid.h, s->grid.penalty_c, refm);
    OMG_TRY(dmalloc((void**)&s->refm, sizeof(double) * refm.size()));
    OMG_TRY(dmalloc((void**)&s->nu, sizeof(double) * L.n));
    OMG_TRY_HIP(hipMemcpyAsync(s->refm, refm.data(), sizeof(double) * refm.size(), hipMemcpyHostToDevice, s->stream));
    OMG_TRY_HIP(hipMemcpyAsync(s->nu, nu_dev, sizeof(double) * L.n, hipMemcpyDeviceToDevice, s->stream));
    const int64_t nt = (int64_t)L.n * 7;
    hipLaunchKernelGGL(k_assemble_sip, dim3(cdivi(nt, 256)), dim3(256), 0, s->stream, L.nx, L.ny, L.nz, s->bs,
                       s->bsh, s->nu, s->refm, L.col, L.val);
    OMG_TRY_HIP(hipGetLastError());
    // host pattern (same rule as the kernel)
    L.hcol.assign((size_t)7 * L.n, 0);
    valid.assign((size_t)7 * L.n, 0);
    const int dims[3] = {L.nx, L.ny, L.nz}, stride[3] = {1, L.nx, L.nx * L.ny};
    for (int i = 0; i < L.n; ++i) {
        const int ijk[3] = {i % L.nx, (i / L.nx) % L.ny, i / (L.nx * L.ny)};
        for (int j = 0; j < 7; ++j) {
            int c = i, ok = 1;
            if (j != 3) {
                const int d = (j < 3) ? 2 - j : j - 4;
                const bool up = j > 3;
                ok = up ? (ijk[d] < dims[d] - 1) : (ijk[d] > 0);
                if (ok) c = up ? i + stride[d] : i - stride[d];
            }
            L.hcol[(size_t)j * L.n + i] = c;
            valid[(size_t)j * L.n + i] = (unsigned char)ok;
        }
    }
    OMG_TRY(upload_dslot(s, L, valid));
    OMG_TRY_HIP(hipStreamSynchronize(s->stream));
    return OMG_OK;
}

// Agglomeration maps between level l and l+1 (host parent/slot of every cell
// of level l): validated (parents in range, slots 0..7, every coarse cell
// with at least one finer cell) and uploaded as Level::up of level l and the
// child lists Level::dn_ptr / dn of level l+1, children in (slot, index)
// order.
omg_status omg_upload_maps(omg_solver* s, int l, const int32_t* parent, const uint8_t* slot) {
    Level& F = s->lev[l];
    Level& C = s->lev[l + 1];
    const int fn = F.n, cn = C.n;
    if (fn >= (1 << 28) || cn >= (1 << 28)) return OMG_EUNSUPPORTED; // packed with the slot in 3 bits
    F.hup.assign(fn, 0);
    std::vector<int> ptr(cn + 1, 0);
    for (int K = 0; K < fn; ++K) {
        const int I = parent[K], sl = slot[K];
        if (I < 0 || I >= cn || sl > 7) return OMG_EINVAL;
        F.hup[K] = I << 3 | sl;
        ptr[I + 1]++;
    }
    for (int I = 0; I < cn; ++I) {
        if (ptr[I + 1] == 0) return OMG_EINVAL; // a coarse cell with no finer cell
        ptr[I + 1] += ptr[I];
    }
    std::vector<int> dn(fn), fill(ptr.begin(), ptr.end() - 1);
    for (int sl = 0; sl < 8; ++sl)
        for (int K = 0; K < fn; ++K)
            if ((F.hup[K] & 7) == sl) dn[fill[F.hup[K] >> 3]++] = K << 3 | sl;
    OMG_TRY(dmalloc((void**)&F.up, sizeof(int) * fn));
    OMG_TRY(dmalloc((void**)&C.dn_ptr, sizeof(int) * (cn + 1)));
    OMG_TRY(dmalloc((void**)&C.dn, sizeof(int) * fn));
    OMG_TRY_HIP(hipMemcpy(F.up, F.hup.data(), sizeof(int) * fn, hipMemcpyHostToDevice));
    OMG_TRY_HIP(hipMemcpy(C.dn_ptr, ptr.data(), sizeof(int) * (cn + 1), hipMemcpyHostToDevice));
    OMG_TRY_HIP(hipMemcpy(C.dn, dn.data(), sizeof(int) * fn, hipMemcpyHostToDevice));
    return OMG_OK;
}

// Galerkin A_{l+1} = P^T A_l P: symbolic pattern and contribution lists on the
// host, numeric triple products on the device.
omg_status omg_galerkin(omg_solver* s, int l, const std::vector<unsigned char>& fvalid,
                        std::vector<unsigned char>& cvalid) {
    Level& F = s->lev[l];
    Level& C = s->lev[l + 1];
    const int fn = F.n, cn = C.n, bs = s->bs, bsh = s->bsh;
    auto parent = [&](int K) { return F.hup[K] >> 3; };
    // coarse rows: sorted unique parents of the children's columns
    std::vector<std::vector<int>> rows(cn);
    for (int K = 0; K < fn; ++K) {
        const int I = parent(K);
        for (int j = 0; j < F.width; ++j)
            if (fvalid[(size_t)j * fn + K]) rows[I].push_back(parent(F.hcol[(size_t)j * fn + K]));
    }
    int width = 0;
    for (auto& r : rows) {
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        width = std::max(width, (int)r.size());
    }
    C.width = width;
    OMG_TRY(alloc_ell(s, C));
    C.hcol.assign((size_t)width * cn, 0);
    cvalid.assign((size_t)width * cn, 0);
    for (int I = 0; I < cn; ++I)
        for (int j = 0; j < width; ++j) {
            const bool ok = j < (int)rows[I].size();
            C.hcol[(size_t)j * cn + I] = ok ? rows[I][j] : I;
            cvalid[(size_t)j * cn + I] = ok;
        }
    OMG_TRY(upload_dslot(s, C, cvalid));
    // contributions per coarse block (slot jc, cell I), fine cells ascending
    const int64_t nblk = (int64_t)width * cn;
    std::vector<int64_t> cnt(nblk + 1, 0);
    std::vector<int> slot_of((size_t)F.width * fn, -1);
    for (int K = 0; K < fn; ++K) {
        const int I = parent(K);
        for (int j = 0; j < F.width; ++j) {
            if (!fvalid[(size_t)j * fn + K]) continue;
            const int J = parent(F.hcol[(size_t)j * fn + K]);
            const int jc = (int)(std::lower_bound(rows[I].begin(), rows[I].end(), J) - rows[I].begin());
            slot_of[(size_t)j * fn + K] = jc;
            cnt[(int64_t)jc * cn + I + 1]++;
        }
    }
    for (int64_t b = 0; b < nblk; ++b) cnt[b + 1] += cnt[b];
    std::vector<int> cK(cnt[nblk]), cj(cnt[nblk]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int K = 0; K < fn; ++K) {
        const int I = parent(K);
        for (int j = 0; j < F.width; ++j) {
            const int jc = slot_of[(size_t)j * fn + K];
            if (jc < 0) continue;
            const int64_t b = (int64_t)jc * cn + I;
            cK[fill[b]] = K;
            cj[fill[b]] = j;
            fill[b]++;
        }
    }
    int64_t* dptr = nullptr;
    int *dK = nullptr, *dj = nullptr;
    omg_status st = dmalloc((void**)&dptr, sizeof(int64_t) * cnt.size());
    if (st == OMG_OK) st = dmalloc((void**)&dK, sizeof(int) * std::max<size_t>(cK.size(), 1));
    if (st == OMG_OK) st = dmalloc((void**)&dj, sizeof(int) * std::max<size_t>(cj.size(), 1));
    if (st == OMG_OK) {
        hipMemcpyAsync(dptr, cnt.data(), sizeof(int64_t) * cnt.size(), hipMemcpyHostToDevice, s->stream);
        hipMemcpyAsync(dK, cK.data(), sizeof(int) * cK.size(), hipMemcpyHostToDevice, s->stream);
        hipMemcpyAsync(dj, cj.data(), sizeof(int) * cj.size(), hipMemcpyHostToDevice, s->stream);
        hipMemcpyAsync(C.col, C.hcol.data(), sizeof(int) * C.hcol.size(), hipMemcpyHostToDevice, s->stream);
        hipMemsetAsync(C.val, 0, sizeof(double) * 2 * nblk * bs * bsh, s->stream);
        const size_t shm = sizeof(double) * (size_t)bs * bs * 10;
        hipLaunchKernelGGL(k_galerkin, dim3((unsigned)nblk), dim3(256), shm, s->stream, bs, bsh, F.up, fn,
                           F.col, F.val, cn, dptr, dK, dj, s->E, C.val, width);
        if (hipGetLastError() != hipSuccess) st = OMG_EHIP;
        if (hipStreamSynchronize(s->stream) != hipSuccess) st = OMG_EHIP;
    }
    hipFree(dptr);
    hipFree(dK);
    hipFree(dj);
    return st;
}

omg_status omg_block_inverses(omg_solver* s, Level& L) {
    const int bs = s->bs;
    OMG_TRY(dmalloc((void**)&L.dinv, sizeof(double) * 2 * (size_t)L.n * bs * s->bsh));
    OMG_TRY_HIP(hipMemsetAsync(s->err_flag, 0, sizeof(int), s->stream));
    dim3 g(cdivi(L.n, 64)), b(64);
    switch (bs) {
    case 1: hipLaunchKernelGGL(k_block_inverse<1>, g, b, 0, s->stream, L.n, L.width, L.dslot, L.val, L.dinv, s->err_flag); break;
    case 4: hipLaunchKernelGGL(k_block_inverse<4>, g, b, 0, s->stream, L.n, L.width, L.dslot, L.val, L.dinv, s->err_flag); break;
    case 10: hipLaunchKernelGGL(k_block_inverse<10>, g, b, 0, s->stream, L.n, L.width, L.dslot, L.val, L.dinv, s->err_flag); break;
    case 20: hipLaunchKernelGGL(k_block_inverse<20>, g, b, 0, s->stream, L.n, L.width, L.dslot, L.val, L.dinv, s->err_flag); break;
    default: return OMG_EINVAL;
    }
    OMG_TRY_HIP(hipGetLastError());
    int err = 0;
    OMG_TRY_HIP(hipMemcpyAsync(&err, s->err_flag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    OMG_TRY_HIP(hipStreamSynchronize(s->stream));
    if (err == 1) return OMG_ENOTSPD;
    if (err) return OMG_EINVAL;
    return OMG_OK;
}

omg_status omg_fp32_copies(omg_solver* s, Level& L) {
    const int64_t nv = (int64_t)2 * L.width * L.n * s->bs * s->bsh;
    OMG_TRY(dmalloc((void**)&L.val32, sizeof(float) * nv));
    hipLaunchKernelGGL(k_to_float, dim3(2048), dim3(256), 0, s->stream, L.val, L.val32, nv);
    OMG_TRY_HIP(hipGetLastError());
    if (L.dinv) {
        const int64_t nd = (int64_t)2 * L.n * s->bs * s->bsh;
        OMG_TRY(dmalloc((void**)&L.dinv32, sizeof(float) * nd));
        hipLaunchKernelGGL(k_to_float, dim3(2048), dim3(256), 0, s->stream, L.dinv, L.dinv32, nd);
        OMG_TRY_HIP(hipGetLastError());
    }
    return OMG_OK;
}

// Dense Cholesky A = L L^T of the coarsest operator (blocked, right-looking,
// tile 32), then A^-1 = L^-T L^-1 stored in full for the per-visit GEMV.
omg_status omg_coarse_factor(omg_solver* s, Level& L) {
    const int N = (int)L.N;
    const int np = ((N + NB - 1) / NB) * NB, nt = np / NB;
    L.np = np;
    double *D = nullptr, *X = nullptr, *linv = nullptr;
    omg_status st = dmalloc((void**)&D, sizeof(double) * (size_t)np * np);
    if (st == OMG_OK) st = dmalloc((void**)&X, sizeof(double) * (size_t)np * np);
    if (st == OMG_OK) st = dmalloc((void**)&linv, sizeof(double) * (size_t)nt * NB * NB);
    if (st == OMG_OK) st = dmalloc((void**)&L.ainv, sizeof(double) * (size_t)np * np);
    hipStream_t q = s->stream;
    if (st == OMG_OK) {
        hipMemsetAsync(D, 0, sizeof(double) * (size_t)np * np, q);
        hipMemsetAsync(X, 0, sizeof(double) * (size_t)np * np, q);
        hipMemsetAsync(s->err_flag, 0, sizeof(int), q);
        const int64_t nthr = (int64_t)L.n * L.width * s->bs;
        hipLaunchKernelGGL(k_densify, dim3(cdivi(nthr, 256)), dim3(256), 0, q, L.n, L.width, s->bs, s->bsh, np,
                           L.col, L.val, D);
        if (np > N) hipLaunchKernelGGL(k_pad_identity, dim3(cdivi(np - N, 256)), dim3(256), 0, q, N, np, D);
        for (int k = 0; k < nt; ++k) {
            hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(256), 0, q, D, np, k, linv, s->err_flag);
            if (k + 1 < nt) {
                hipLaunchKernelGGL(k_trsm_panel, dim3(nt - k - 1), dim3(256), 0, q, D, np, k, linv);
                const int m = nt - k - 1;
                hipLaunchKernelGGL(k_syrk_update, dim3((unsigned)((int64_t)m * (m + 1) / 2)), dim3(256), 0, q, D,
                                   np, k);
            }
        }
        hipLaunchKernelGGL(k_trinv_diag, dim3(nt), dim3(256), 0, q, X, np, linv);
        for (int i = 1; i < nt; ++i) hipLaunchKernelGGL(k_trinv_row, dim3(i), dim3(256), 0, q, D, X, np, i, linv);
        hipLaunchKernelGGL(k_xtx, dim3((unsigned)nt * nt), dim3(256), 0, q, X, L.ainv, np, nt);
        if (hipGetLastError() != hipSuccess) st = OMG_EHIP;
        if (st == OMG_OK && !std::getenv("OMG_NO_SYMV") && build_symv_tiles(L, q) != hipSuccess) st = OMG_EHIP;
        int err = 0;
        if (hipMemcpyAsync(&err, s->err_flag, sizeof(int), hipMemcpyDeviceToHost, q) != hipSuccess) st = OMG_EHIP;
        if (hipStreamSynchronize(q) != hipSuccess) st = OMG_EHIP;
        if (st == OMG_OK && err) st = OMG_ENOTSPD;
    }
    hipFree(D);
    hipFree(X);
    hipFree(linv);
    return st;
}
