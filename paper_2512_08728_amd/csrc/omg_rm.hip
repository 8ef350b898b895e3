// Persistent residual-minimisation kernel (Algorithm 1 after w = A z).
//
// One launch performs the modified Gram-Schmidt loop of w against the stored
// orthonormal directions W, the normalisation, alpha = w.r and the residual
// update. Each thread keeps the entries of w it owns in registers for the
// whole loop, so every stored direction is read once per launch.
//
// Search directions are kept implicitly: the raw direction z~ handed to RM is
// stored as it is, together with the MGS coefficients beta_{k,i}, gamma_k and
// alpha_k, so that z_k = gamma_k (z~_k - sum_{i<k} beta_{k,i} z_i). Within one
// level solve x is only needed at the end: x = sum_k alpha_k z_k = sum_k d_k z~_k
// with d obtained by a backward recurrence over k (k_recon), then one pass
// over the raw directions (k_combine). Per launch this moves k + 6 vectors
// instead of 2k + 8.
//
// MGS is evaluated B directions per grid-wide exchange: with c_t = W_{j0+t}.w
// (w before the block) and the stored Gram entries G_tm = W_{j0+t}.W_{j0+m},
// the MGS coefficients satisfy beta_t = c_t - sum_{m<t} G_tm beta_m, which is
// the sequential MGS recursion in exact arithmetic. G is recorded when a
// direction is created.
//
// Grid-wide exchange without fences: a device-scope fence on this 8-XCD part
// writes back / invalidates an XCD's L2 and costs tens of microseconds per
// barrier. Each block instead publishes its partial sums as 64-bit
// agent-scope atomic words whose two low mantissa bits carry a phase tag
// (phase mod 3; 3 = empty), and every block reads all G published words with
// agent-scope atomic loads, waiting until each carries the expected tag.
// Phases alternate between two slot sets; a block writes phase g+2 into the
// set of phase g only after it has read every block's phase g+1 words, so
// every block has finished reading phase g. The host keeps each level's phase
// counter across launches, so a stale word always carries the tag of phase
// g-2, never that of g. Clearing the two tag bits perturbs each partial by at
// most 2^-51 relative; all readers see the same words, so the sums are the
// same in every block and deterministic. Waits are bounded: a block that
// waits too long raises an abort flag that ends every other wait, so every
// wave reaches the end of the kernel; the host checks the flag.
//
// The grid is sized from the occupancy query so that every block is resident
// at once; the launch is an ordinary one (cooperative launches carry a large
// per-launch cost on this runtime).
#include <cstdlib>

#include "omg_internal.h"

namespace omg {

constexpr unsigned kSpinMax = 1u << 25;

__device__ __forceinline__ unsigned long long tag_pack(double v, unsigned tag) {
    return ((unsigned long long)__double_as_longlong(v) & ~3ull) | tag;
}
__device__ __forceinline__ double tag_value(unsigned long long b) { return __longlong_as_double(b & ~3ull); }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
// Block sums of nv values at once (one pair of barriers for all of them);
// per value the order is that of bsum. sh holds kMaxVals * (kThreads/64).
constexpr int kMaxVals = kRmBlock + 1;
template <int NV>
__device__ __forceinline__ void bsum_n(double (&v)[NV], int nv, double* sh) {
    constexpr int NW = kThreads / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i)
        if (i < nv) v[i] = wsum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) sh[i * NW + wid] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < nv) {
            double s = 0.0;
            for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += sh[i * NW + q];
            v[i] = s;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ double bsum(double v, double* sh) {
    v = wsum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    __syncthreads();
    return s;
}

// Publish this block's words for phase g: slots[set][block][SW]. All SW words
// are written every phase (unused ones as zero), so the previous value of any
// word is always from phase g-2 and carries a different tag.
template <int SW>
__device__ __forceinline__ void publish(unsigned long long* slots, int G, unsigned long long g, const double* v,
                                        int nw) {
    if (threadIdx.x == 0) {
        unsigned long long* p = slots + ((g & 1) * (unsigned long long)G + blockIdx.x) * SW;
        const unsigned tag = (unsigned)(g % 3);
        for (int i = 0; i < SW; ++i)
            __hip_atomic_store(p + i, tag_pack(i < nw ? v[i] : 0.0, tag), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Sum over blocks of words [0, nw) of phase g; every thread gets the totals.
template <int SW>
__device__ __forceinline__ void collect(unsigned long long* slots, int G, unsigned long long g, int nw, double* out,
                                        double* sh, unsigned* abort_flag) {
    const unsigned tag = (unsigned)(g % 3);
    const unsigned long long* base = slots + (g & 1) * (unsigned long long)G * SW;
    double v[SW];
#pragma unroll
    for (int w = 0; w < SW; ++w) v[w] = 0.0;
    for (int i = threadIdx.x; i < G; i += blockDim.x) {
#pragma unroll
        for (int w = 0; w < SW; ++w) {
            if (w < nw) {
                unsigned long long b = 0;
                unsigned spins = 0;
                for (;;) {
                    b = __hip_atomic_load(base + (unsigned long long)i * SW + w, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                    if ((unsigned)(b & 3ull) == tag) break;
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kSpinMax ||
                        ((spins & 127) == 0 &&
                         __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        b = 0;
                        break;
                    }
                }
                v[w] += tag_value(b);
            }
        }
    }
    bsum_n<SW>(v, nw, sh);
#pragma unroll
    for (int w = 0; w < SW; ++w)
        if (w < nw) out[w] = v[w];
}

// Every vector is handled as a flat array of N entries (RM has no cell
// structure): thread t of a grid of T threads owns entries t + j T, j < EPT,
// so consecutive threads touch consecutive addresses.
template <int EPT, int B>
__global__ __launch_bounds__(kThreads) void k_rm_blk(RmArgs A) {
    constexpr int SW = B + 1;
    __shared__ double sh[kMaxVals * (kThreads / 64)];
    const int G = gridDim.x;
    const int64_t T = (int64_t)G * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = A.N;
    const int k = A.k;
    double w[EPT], a[B][EPT], an[B][EPT];
    bool valid[EPT];
    // w in registers; the raw direction z~ is stored as direction k
    double* Zk = A.Zk;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int64_t e = t0 + j * T;
        valid[j] = e < N;
        w[j] = valid[j] ? A.w[e] : 0.0;
        if (valid[j]) Zk[e] = A.z[e];
    }
    auto load_block = [&](double (&dst)[B][EPT], int j0) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const bool have = j0 + t < k;
            const double* Wt = have ? A.Wp[j0 + t] : nullptr;
#pragma unroll
            for (int j = 0; j < EPT; ++j) dst[t][j] = (have && valid[j]) ? Wt[t0 + j * T] : 0.0;
        }
    };
    const int nblk = (k + B - 1) / B;
    unsigned long long g = A.g0;
    double vals[SW];
    // phase g0: dots of the first block and ||w||^2; the next block is loaded
    // meanwhile. Block b+2 is requested as soon as block b+1 becomes current,
    // so loads stay in flight through every reduction, publish and wait.
    load_block(a, 0);
    if (nblk > 1) load_block(an, B);
    {
        double s_in = 0.0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) s_in = fma(w[j], w[j], s_in);
        vals[B] = s_in;
#pragma unroll
        for (int t = 0; t < B; ++t) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) s = fma(a[t][j], w[j], s);
            vals[t] = s;
        }
        bsum_n<SW>(vals, SW, sh);
        publish<SW>(A.slots, G, g, vals, SW);
    }
    double nin2 = 0.0, nout2 = 0.0;
    double tot[SW];
    for (int b = 0; b < nblk; ++b) {
        const int j0 = b * B;
        const int bb = min(B, k - j0);
        collect<SW>(A.slots, G, g, (b == 0) ? SW : bb, tot, sh, A.abort_flag);
        if (b == 0) nin2 = tot[B];
        double beta[B];
#pragma unroll
        for (int t = 0; t < B; ++t) {
            double bt = 0.0;
            if (t < bb) {
                bt = tot[t];
                for (int m = 0; m < t; ++m) bt = fma(-A.gram[(int64_t)(j0 + t) * kGramStride + m], beta[m], bt);
            }
            beta[t] = bt;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) // row k of the coefficient history
            for (int t = 0; t < bb; ++t) A.hist[(int64_t)k * (k - 1) / 2 + j0 + t] = beta[t];
#pragma unroll
        for (int t = 0; t < B; ++t)
#pragma unroll
            for (int j = 0; j < EPT; ++j) w[j] = fma(-beta[t], a[t][j], w[j]);
        ++g;
        if (b + 1 < nblk) {
#pragma unroll
            for (int t = 0; t < B; ++t)
#pragma unroll
                for (int j = 0; j < EPT; ++j) a[t][j] = an[t][j];
            if (b + 2 < nblk) load_block(an, j0 + 2 * B);
#pragma unroll
            for (int t = 0; t < B; ++t) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < EPT; ++j) s = fma(a[t][j], w[j], s);
                vals[t] = s;
            }
            bsum_n<SW>(vals, B, sh);
            publish<SW>(A.slots, G, g, vals, B);
        } else {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) s = fma(w[j], w[j], s);
            vals[0] = s;
            bsum_n<SW>(vals, 1, sh);
            publish<SW>(A.slots, G, g, vals, 1);
            collect<SW>(A.slots, G, g, 1, tot, sh, A.abort_flag);
            nout2 = tot[0];
        }
    }
    if (k == 0) {
        collect<SW>(A.slots, G, g, SW, tot, sh, A.abort_flag);
        nin2 = tot[B];
        nout2 = nin2;
    }
    const double nin = sqrt(nin2), nout = sqrt(nout2);
    const bool keep = nout > A.breakdown * nin; // false for NaN and for nout == 0
    const double gamma = keep ? 1.0 / nout : 0.0;
    // new direction W_k = gamma w; Gram entries with the earlier directions of its block
    const int jk0 = k - (k % B), gk = k % B;
    load_block(a, jk0); // entries t >= gk are zero (directions not stored yet)
    double s_a = 0.0, s_g[B];
#pragma unroll
    for (int t = 0; t < B; ++t) s_g[t] = 0.0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        w[j] *= gamma;
        double rv = 0.0;
        if (valid[j]) {
            const int64_t e = t0 + j * T;
            A.Wk[e] = w[j];
            rv = A.r[e];
        }
        an[0][j] = rv; // r kept in registers
        s_a = fma(w[j], rv, s_a);
#pragma unroll
        for (int t = 0; t < B; ++t) s_g[t] = fma(a[t][j], w[j], s_g[t]);
    }
    ++g;
    vals[0] = s_a;
#pragma unroll
    for (int t = 0; t < B - 1; ++t) vals[1 + t] = s_g[t];
    bsum_n<SW>(vals, B, sh);
    publish<SW>(A.slots, G, g, vals, B);
    collect<SW>(A.slots, G, g, B, tot, sh, A.abort_flag);
    const double alpha = tot[0];
    double s_r = 0.0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const double rn = fma(-alpha, w[j], an[0][j]);
        if (valid[j]) A.r[t0 + j * T] = rn;
        s_r = fma(rn, rn, s_r);
    }
    s_r = bsum(s_r, sh);
    if (threadIdx.x == 0) {
        A.part_rn[blockIdx.x] = s_r;
        if (blockIdx.x == 0) {
            A.alphas[k] = alpha;
            A.gammas[k] = gamma;
            for (int t = 0; t < B - 1; ++t) A.gram[(int64_t)k * kGramStride + t] = (t < gk) ? tot[1 + t] : 0.0;
            if (!keep) A.scal[S_BREAKDOWNS] += 1.0;
        }
    }
}

// Coefficients of x = sum_k alpha_k z_k in the raw directions: with
// z_k = gamma_k (z~_k - sum_{i<k} beta_{k,i} z_i), walk k downwards keeping the
// coefficient c_i of every z_i still to be expanded: d_k = c_k gamma_k, then
// c_i -= d_k beta_{k,i} for i < k. One wavefront; c lives in LDS.
__global__ __launch_bounds__(64) void k_recon(int K, const double* __restrict__ hist,
                                              const double* __restrict__ gammas, const double* __restrict__ alphas,
                                              double* __restrict__ d) {
    extern __shared__ double c[];
    for (int i = threadIdx.x; i < K; i += blockDim.x) c[i] = alphas[i];
    __syncthreads();
    for (int k = K - 1; k >= 0; --k) {
        const double dk = c[k] * gammas[k];
        __syncthreads();
        if (threadIdx.x == 0) d[k] = dk;
        const double* hk = hist + (int64_t)k * (k - 1) / 2;
        for (int i = threadIdx.x; i < k; i += blockDim.x) c[i] = fma(-dk, hk[i], c[i]);
        __syncthreads();
    }
}

// out = sum_m d[m] V_m (k vectors of length N)
__global__ __launch_bounds__(kThreads) void k_combine(int64_t N, int k, const double* const* __restrict__ V,
                                                      const double* __restrict__ d, double* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        double s = 0.0;
        for (int m = 0; m < k; ++m) s = fma(d[m], V[m][e], s);
        out[e] = s;
    }
}

__global__ void k_zero(double* __restrict__ out, int64_t N) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) out[e] = 0.0;
}

template <int EPT, int B>
static const void* rm_kernel() {
    return reinterpret_cast<const void*>(&k_rm_blk<EPT, B>);
}

// Instantiations: entries per thread EPT, MGS block B in {1, 2, 4}.
constexpr int kEpts[] = {1, 2, 4, 8, 10, 16, 20};
template <int EPT>
static const void* pick_b(int b) {
    if (b == 4) return rm_kernel<EPT, 4>();
    if (b == 2) return rm_kernel<EPT, 2>();
    if (b == 1) return rm_kernel<EPT, 1>();
    return nullptr;
}
static const void* pick(int ept, int b) {
    switch (ept) {
    case 1: return pick_b<1>(b);
    case 2: return pick_b<2>(b);
    case 4: return pick_b<4>(b);
    case 8: return pick_b<8>(b);
    case 10: return pick_b<10>(b);
    case 16: return pick_b<16>(b);
    case 20: return pick_b<20>(b);
    }
    return nullptr;
}

// Co-resident launch configurations for a level of N entries: grids of at
// most kMaxRedBlocks blocks whose blocks all fit at once (occupancy query),
// in order of preference (fewest entries per thread, then the largest MGS
// block, then at most 512 blocks before larger grids).
int rm_persistent_candidates(int64_t N, RmConfig* out, int cap) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    int n = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int e : kEpts) {
            const int64_t need = (N + (int64_t)kThreads * e - 1) / ((int64_t)kThreads * e);
            if (pass == 0 ? need > 512 : (need <= 512 || need > kMaxRedBlocks)) continue;
            for (int b : {4, 2, 1}) {
                const void* f = pick(e, b);
                int per_cu = 0;
                if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kThreads, 0) != hipSuccess ||
                    per_cu < 1 || need > (int64_t)per_cu * cus)
                    continue;
                if (n < cap) out[n++] = RmConfig{(int)need, e, b};
            }
        }
    return n;
}

bool rm_persistent_config(int64_t N, int* G, int* ept, int* B) {
    RmConfig c[64];
    if (rm_persistent_candidates(N, c, 64) < 1) return false;
    *G = c[0].G;
    *ept = c[0].ept;
    *B = c[0].B;
    return true;
}

hipError_t launch_rm_persistent(int G, int ept, int B, const RmArgs& args, hipStream_t st) {
    const void* f = pick(ept, B);
    if (!f) return hipErrorInvalidValue;
    RmArgs a = args;
    void* params[] = {&a};
    return hipLaunchKernel(f, dim3(G), dim3(kThreads), params, 0, st);
}

hipError_t launch_recon(int K, const double* hist, const double* gammas, const double* alphas, double* d,
                        hipStream_t st) {
    if (K == 0) return hipSuccess;
    hipLaunchKernelGGL(k_recon, dim3(1), dim3(64), sizeof(double) * (size_t)K, st, K, hist, gammas, alphas, d);
    return hipGetLastError();
}

hipError_t launch_lincomb(int64_t N, int k, const double* d, const double* const* V, double* out,
                          hipStream_t st) {
    int64_t blocks = (N + kThreads - 1) / kThreads;
    if (blocks > 2048) blocks = 2048;
    if (k == 0) {
        hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kThreads), 0, st, out, N);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_combine, dim3((unsigned)blocks), dim3(kThreads), 0, st, N, k, V, d, out);
    return hipGetLastError();
}

} // namespace omg
