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
#include <algorithm>
#include <cstdint>
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
__device__ __forceinline__ void publish(unsigned long long* slots, int G, int bid, unsigned long long g,
                                        const double* v, int nw) {
    if (threadIdx.x == 0) {
        unsigned long long* p = slots + ((g & 1) * (unsigned long long)G + bid) * SW;
        const unsigned tag = (unsigned)(g % 3);
        for (int i = 0; i < SW; ++i)
            __hip_atomic_store(p + i, tag_pack(i < nw ? v[i] : 0.0, tag), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Wait until the word carries `tag` (bounded; an expired wait raises the
// abort flag, and a raised flag ends every wait). Returns the word (0 after
// an abort).
__device__ __forceinline__ unsigned long long wait_word(const unsigned long long* p, unsigned tag,
                                                        unsigned* abort_flag) {
    unsigned spins = 0;
    for (;;) {
        const unsigned long long b = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((unsigned)(b & 3ull) == tag) return b;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinMax ||
            ((spins & 127) == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
    }
}

// Sum over blocks of words [0, nw) of phase g; every thread gets the totals.
// All-to-all form (LEAD = false): every block reads all G blocks' words.
// Leader form (LEAD = true): block 0 reads them and publishes the totals
// (phase-tagged, two alternating sets after the block words) and the other
// blocks wait for those nw words: 2G word reads per exchange instead of G^2,
// for one more hop of latency. Every block, block 0 included, uses the
// tag-truncated totals, so all blocks hold identical values.
template <int SW, bool LEAD>
__device__ __forceinline__ void collect(unsigned long long* slots, int G, int bid, unsigned long long g, int nw,
                                        double* out, double* sh, unsigned* abort_flag) {
    const unsigned tag = (unsigned)(g % 3);
    const unsigned long long* base = slots + (g & 1) * (unsigned long long)G * SW;
    unsigned long long* tot = slots + 2ull * kMaxRedBlocks * (kRmBlock + 1) + (g & 1) * SW;
    double v[SW];
#pragma unroll
    for (int w = 0; w < SW; ++w) v[w] = 0.0;
    if (!LEAD || bid == 0) {
        for (int i = threadIdx.x; i < G; i += blockDim.x) {
#pragma unroll
            for (int w = 0; w < SW; ++w)
                if (w < nw) v[w] += tag_value(wait_word(base + (unsigned long long)i * SW + w, tag, abort_flag));
        }
        bsum_n<SW>(v, nw, sh);
        if (LEAD) {
            if (threadIdx.x == 0)
                for (int w = 0; w < SW; ++w)
                    __hip_atomic_store(tot + w, tag_pack(w < nw ? v[w] : 0.0, tag), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int w = 0; w < SW; ++w) v[w] = tag_value(tag_pack(v[w], tag));
        }
    } else {
        if (threadIdx.x < nw) sh[threadIdx.x] = tag_value(wait_word(tot + threadIdx.x, tag, abort_flag));
        __syncthreads();
#pragma unroll
        for (int w = 0; w < SW; ++w)
            if (w < nw) v[w] = sh[w];
        __syncthreads();
    }
#pragma unroll
    for (int w = 0; w < SW; ++w)
        if (w < nw) out[w] = v[w];
}

// Every vector is handled as a flat array of N entries (RM has no cell
// structure): thread t of a grid of T threads owns entries t + j T, j < EPT,
// so consecutive threads touch consecutive addresses.
// Vector accesses of the persistent kernel go through raw buffer
// instructions: a resource (base address, size) in scalar registers, the
// uniform part of the offset (entry j of every thread: j T 8 bytes) as a
// scalar offset, and one 32-bit per-thread offset shared by all accesses,
// so no per-entry 64-bit addresses occupy vector registers. The resource's
// fourth word is the raw-buffer format of the gfx9 family.
constexpr int kBufWord3 = 0x00020000;
typedef unsigned int BufData __attribute__((vector_size(2 * sizeof(unsigned int)))); // the 64-bit payload
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* p, int bytes) {
    const uint64_t v = (uint64_t)p; // every lane holds the same pointer: keep it in scalar registers
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0, bytes, kBufWord3);
}

// The RM of one vector set on G blocks; this block is block `bid` of them.
template <int EPT, int B, bool LEAD>
__device__ __forceinline__ void rm_body(const RmArgs& A, const int G, const int bid, double* sh) {
    constexpr int SW = B + 1;
    const int64_t T = (int64_t)G * blockDim.x;
    const int64_t t0 = (int64_t)bid * blockDim.x + threadIdx.x;
    const int64_t N = A.N;
    const int k = A.k;
    // Entry j of this thread is entry t0 + j T of every vector (byte j T 8 +
    // t0 8). The vectors carry kVecPad zero entries past N and this grid
    // covers fewer than N + kVecPad entries, so loads need no masks; stores
    // are masked to [0, N), which keeps the tails zero.
    const int toff = (int)t0 * 8;
    const int stride = (int)T * 8;
    const int bytes = (int)((N + kVecPad) * 8);
    auto ld = [&](__amdgpu_buffer_rsrc_t r, int j) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, toff, j * stride, 0));
    };
    auto st = [&](__amdgpu_buffer_rsrc_t r, int j, double v) {
        if (t0 + j * T < N) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufData, v), r, toff, j * stride, 0);
    };
    double w[EPT], a[B][EPT], an[B][EPT];
    // w in registers; the raw direction z~ is stored as direction k
    {
        const __amdgpu_buffer_rsrc_t rw = buffer_of(A.w, bytes), rz = buffer_of(A.z, bytes),
                                     rk = buffer_of(A.Zk, bytes);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            w[j] = ld(rw, j);
            st(rk, j, ld(rz, j));
        }
    }
    auto load_block = [&](double (&dst)[B][EPT], int j0) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const bool have = j0 + t < k; // uniform
            if (have) {
                const __amdgpu_buffer_rsrc_t rt = buffer_of(A.Wp[j0 + t], bytes);
#pragma unroll
                for (int j = 0; j < EPT; ++j) dst[t][j] = ld(rt, j);
            } else {
#pragma unroll
                for (int j = 0; j < EPT; ++j) dst[t][j] = 0.0;
            }
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
        publish<SW>(A.slots, G, bid, g, vals, SW);
    }
    double nin2 = 0.0, nout2 = 0.0;
    double tot[SW];
    for (int b = 0; b < nblk; ++b) {
        const int j0 = b * B;
        const int bb = min(B, k - j0);
        collect<SW, LEAD>(A.slots, G, bid, g, (b == 0) ? SW : bb, tot, sh, A.abort_flag);
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
        if (bid == 0 && threadIdx.x == 0) // row k of the coefficient history
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
            publish<SW>(A.slots, G, bid, g, vals, B);
        } else {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) s = fma(w[j], w[j], s);
            vals[0] = s;
            bsum_n<SW>(vals, 1, sh);
            publish<SW>(A.slots, G, bid, g, vals, 1);
            collect<SW, LEAD>(A.slots, G, bid, g, 1, tot, sh, A.abort_flag);
            nout2 = tot[0];
        }
    }
    if (k == 0) {
        collect<SW, LEAD>(A.slots, G, bid, g, SW, tot, sh, A.abort_flag);
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
    const __amdgpu_buffer_rsrc_t rwk = buffer_of(A.Wk, bytes), rr = buffer_of(A.r, bytes);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        w[j] *= gamma;
        st(rwk, j, w[j]);
        const double rv = ld(rr, j);
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
    publish<SW>(A.slots, G, bid, g, vals, B);
    collect<SW, LEAD>(A.slots, G, bid, g, B, tot, sh, A.abort_flag);
    const double alpha = tot[0];
    double s_r = 0.0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const double rn = fma(-alpha, w[j], an[0][j]);
        st(rr, j, rn);
        s_r = fma(rn, rn, s_r);
    }
    s_r = bsum(s_r, sh);
    if (threadIdx.x == 0) {
        A.part_rn[bid] = s_r;
        if (bid == 0) {
            A.alphas[k] = alpha;
            A.gammas[k] = gamma;
            for (int t = 0; t < B - 1; ++t) A.gram[(int64_t)k * kGramStride + t] = (t < gk) ? tot[1 + t] : 0.0;
            if (!keep) A.scal[S_BREAKDOWNS] += 1.0;
        }
    }
}

template <int EPT, int B, bool LEAD>
__global__ __launch_bounds__(kThreads) void k_rm_blk(RmArgs A) {
    __shared__ double sh[kMaxVals * (kThreads / 64)];
    rm_body<EPT, B, LEAD>(A, gridDim.x, blockIdx.x, sh);
}

// RM of several vector sets (columns of a batched solve, or independent
// solvers of one level configuration) in one launch: column q owns blocks
// [blk0[q], blk0[q+1]) and exchanges only among them, with its own words,
// phase and storage (table entry idx[q]); all columns share k.
template <int EPT, int B, bool LEAD>
__global__ __launch_bounds__(kThreads) void k_rm_multi(RmMulti M) {
    __shared__ double sh[kMaxVals * (kThreads / 64)];
    int q = 0;
    while (q + 1 < M.ncol && (int)blockIdx.x >= M.blk0[q + 1]) ++q;
    const RmCol& C = M.tab[M.idx[q]];
    RmArgs A;
    A.N = C.N;
    A.k = M.k;
    A.Wp = C.Wp;
    A.Wk = C.Wp[M.k];
    A.Zk = C.Zp[M.k];
    A.w = C.w;
    A.z = M.zcor ? C.zcor : C.z;
    A.r = C.r;
    A.slots = C.slots;
    A.g0 = M.g0[q];
    A.part_rn = C.part_rn;
    A.breakdown = M.breakdown;
    A.scal = C.scal;
    A.abort_flag = M.abort_flag;
    A.hist = C.hist;
    A.gammas = C.gammas;
    A.alphas = C.alphas;
    A.gram = C.gram;
    rm_body<EPT, B, LEAD>(A, M.blk0[q + 1] - M.blk0[q], (int)blockIdx.x - M.blk0[q], sh);
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

// Several members at once: block q of the recombination runs k_recon for
// member q; the combination's segment q runs k_combine's loop for member q.
__global__ __launch_bounds__(64) void k_recon_grouped(RecTable T) {
    extern __shared__ double c[];
    const int q = blockIdx.x;
    const int K = T.K[q];
    const double* hist = T.hist[q];
    const double* gammas = T.gammas[q];
    double* d = T.d[q];
    for (int i = threadIdx.x; i < K; i += blockDim.x) c[i] = T.alphas[q][i];
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

__global__ __launch_bounds__(kThreads) void k_combine_grouped(RecTable T) {
    int q = 0;
    while (q + 1 < T.count && (int)blockIdx.x >= T.blk0[q + 1]) ++q;
    const int64_t N = T.N[q];
    const int k = T.K[q];
    const double* const* V = T.V[q];
    const double* d = T.d[q];
    double* out = T.out[q];
    const int64_t stride = (int64_t)(T.blk0[q + 1] - T.blk0[q]) * blockDim.x;
    for (int64_t e = (int64_t)(blockIdx.x - T.blk0[q]) * blockDim.x + threadIdx.x; e < N; e += stride) {
        double s = 0.0;
        for (int m = 0; m < k; ++m) s = fma(d[m], V[m][e], s);
        out[e] = s;
    }
}

__global__ void k_zero(double* __restrict__ out, int64_t N) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) out[e] = 0.0;
}

template <int EPT, int B, bool LEAD>
static const void* rm_kernel(bool multi) {
    return multi ? reinterpret_cast<const void*>(&k_rm_multi<EPT, B, LEAD>)
                 : reinterpret_cast<const void*>(&k_rm_blk<EPT, B, LEAD>);
}

// Instantiations: entries per thread EPT, MGS block B in {1, 2, 4}, exchange
// form (all-to-all or leader).
constexpr int kEpts[] = {1, 2, 4, 8, 10, 16, 20};
// byte offsets of the buffer accesses are 32-bit
static_assert(((int64_t)kMaxRedBlocks * kThreads * 20 + kVecPad) * 8 < (int64_t)1 << 31, "RM offsets");
template <int EPT, bool LEAD>
static const void* pick_b(int b, bool multi) {
    if (b == 4) return rm_kernel<EPT, 4, LEAD>(multi);
    if (b == 2) return rm_kernel<EPT, 2, LEAD>(multi);
    if (b == 1) return rm_kernel<EPT, 1, LEAD>(multi);
    return nullptr;
}
template <int EPT>
static const void* pick_x(int b, int lead, bool multi) {
    return lead ? pick_b<EPT, true>(b, multi) : pick_b<EPT, false>(b, multi);
}
static const void* pick(int ept, int b, int lead, bool multi = false) {
    switch (ept) {
    case 1: return pick_x<1>(b, lead, multi);
    case 2: return pick_x<2>(b, lead, multi);
    case 4: return pick_x<4>(b, lead, multi);
    case 8: return pick_x<8>(b, lead, multi);
    case 10: return pick_x<10>(b, lead, multi);
    case 16: return pick_x<16>(b, lead, multi);
    case 20: return pick_x<20>(b, lead, multi);
    }
    return nullptr;
}

// Blocks of the multi-column kernel in this configuration that fit at once.
int rm_multi_capacity(int ept, int B, int lead) {
    int dev = 0, cus = 0, per_cu = 0;
    const void* f = pick(ept, B, lead, true);
    if (!f || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kThreads, 0) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_rm_multi(int ept, int B, int lead, const RmMulti& M, hipStream_t st) {
    const void* f = pick(ept, B, lead, true);
    if (!f || M.ncol < 1 || M.ncol > kMaxCols) return hipErrorInvalidValue;
    RmMulti a = M;
    void* params[] = {&a};
    return hipLaunchKernel(f, dim3(M.blk0[M.ncol]), dim3(kThreads), params, 0, st);
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
            for (int b : {4, 2, 1})
                for (int lead : {0, 1}) {
                    const void* f = pick(e, b, lead);
                    int per_cu = 0;
                    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kThreads, 0) != hipSuccess ||
                        per_cu < 1 || need > (int64_t)per_cu * cus)
                        continue;
                    if (n < cap) out[n++] = RmConfig{(int)need, e, b, lead};
                }
        }
    return n;
}

bool rm_persistent_config(int64_t N, RmConfig* cfg) {
    RmConfig c[kMaxRmConfigs];
    if (rm_persistent_candidates(N, c, kMaxRmConfigs) < 1) return false;
    *cfg = c[0];
    return true;
}

// Every word written in a phase g of a fixed layout is overwritten two
// phases later, so a reader waiting for phase g can only meet the tag of g-2
// or g itself. A word last written under another layout (other grid, other
// words per block, other exchange form) can hold any phase's value; the
// words are therefore set to the empty tag (3) whenever the layout changes.
hipError_t prepare_slots(Level& L, const RmConfig& c, hipStream_t st) {
    const int sw = c.B + 1;
    if (L.slot_G == c.G && L.slot_SW == sw && L.slot_lead == c.lead) return hipSuccess;
    hipError_t e = hipMemsetAsync(L.xslots, 0xFF, sizeof(unsigned long long) * kRmSlotWords, st);
    if (e != hipSuccess) return e;
    L.slot_G = c.G;
    L.slot_SW = sw;
    L.slot_lead = c.lead;
    return hipSuccess;
}

hipError_t launch_rm_persistent(const RmConfig& c, const RmArgs& args, hipStream_t st) {
    const void* f = pick(c.ept, c.B, c.lead);
    const int G = c.G;
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

// x of several members: d by the backward recurrence, then x = sum_k d_k z~_k.
hipError_t launch_recon_combine_grouped(RecTable& T, hipStream_t st) {
    if (T.count < 1 || T.count > kMaxCols) return hipErrorInvalidValue;
    int kmax = 0, b = 0;
    for (int q = 0; q < T.count; ++q) {
        if (T.K[q] < 1) return hipErrorInvalidValue; // members with directions only
        kmax = std::max(kmax, T.K[q]);
        T.blk0[q] = b;
        int64_t blocks = (T.N[q] + kThreads - 1) / kThreads;
        if (blocks > 2048) blocks = 2048;
        b += (int)blocks;
    }
    T.blk0[T.count] = b;
    hipLaunchKernelGGL(k_recon_grouped, dim3(T.count), dim3(64), sizeof(double) * (size_t)kmax, st, T);
    hipLaunchKernelGGL(k_combine_grouped, dim3(b), dim3(kThreads), 0, st, T);
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
