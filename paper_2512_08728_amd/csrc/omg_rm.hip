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
#include <type_traits>

#include "omg_internal.h"

namespace omg {

constexpr unsigned kSpinMax = 1u << 22;

__device__ __forceinline__ unsigned long long tag_pack(double v, unsigned tag) {
    return ((unsigned long long)__double_as_longlong(v) & ~3ull) | tag;
}
__device__ __forceinline__ double tag_value(unsigned long long b) { return __longlong_as_double(b & ~3ull); }

// v from another lane of the same row by a DPP permutation (both halves)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// Wavefront sum by pairwise exchanges (each step adds the value of a partner
// lane, the partner relation being symmetric), so every lane ends with the
// same bits: lane i ^ 1, i ^ 2 (quad permutations), 7 - i and 15 - i within
// rows (half-row and row mirrors), then i ^ 16 and i ^ 32.
__device__ __forceinline__ double wsum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
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

// Direction pointers read into shared memory at the start of a launch (the
// first kPtrLds of them), so that requesting a direction costs no global
// memory round trip in the MGS loop.
constexpr int kPtrLds = 1024;

// The lagged form keeps its pointers as a ring: W_j at ptab[j % kPtrLds].
// The first kPtrLds are read at the start of a launch; when direction j0 (a
// multiple of kPtrLds / 2) is about to be requested, directions
// j0 + kPtrLds / 2 .. j0 + kPtrLds - 1 replace the half of the ring already
// passed. Requesting a direction then never reads global memory inside the
// loop: such a read would make the wave wait for every vector load it has in
// flight (loads complete in issue order). The refilled entries are read at
// least kPtrLds / 2 directions later, after the barriers of those steps.
__device__ __forceinline__ void ptr_ring_refill(unsigned long long* ptab, const double* const* Wp, int k, int j0) {
    for (int j = j0 + kPtrLds / 2 + (int)threadIdx.x; j < min(k, j0 + kPtrLds); j += blockDim.x)
        ptab[j % kPtrLds] = (unsigned long long)Wp[j];
}

// The RM of one vector set on G blocks; this block is block `bid` of them.
// MASK: the vectors have no zero tail past N (caller arrays): every access
// of an entry >= N is skipped and such entries count as zero, and Zk may be
// null (the raw direction is not stored).
template <int EPT, int B, bool LEAD, bool MASK = false>
__device__ __forceinline__ void rm_body(const RmArgs& A, const int G, const int bid, double* sh,
                                        unsigned long long* ptab) {
    constexpr int SW = B + 1;
    const int64_t T = (int64_t)G * blockDim.x;
    const int64_t t0 = (int64_t)bid * blockDim.x + threadIdx.x;
    const int64_t N = A.N;
    const int k = A.k;
    // Entry j of this thread is entry t0 + j T of every vector (byte j T 8 +
    // t0 8). The vectors carry kVecPad zero entries past N and this grid
    // covers fewer than N + kVecPad entries, so loads need no masks. Computed
    // values are stored to [0, N) only, which keeps the tails zero whatever
    // the data; the copy of z~ moves its (zero) tail along unmasked, so that
    // its loads are all issued before the first store.
    const int toff = (int)t0 * 8;
    const int stride = (int)T * 8;
    const int bytes = (int)((MASK ? N : N + kVecPad) * 8);
    auto ld = [&](__amdgpu_buffer_rsrc_t r, int j) -> double {
        if (MASK && t0 + j * T >= N) return 0.0;
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, toff, j * stride, 0));
    };
    auto st_all = [&](__amdgpu_buffer_rsrc_t r, int j, double v) {
        if (MASK && t0 + j * T >= N) return;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufData, v), r, toff, j * stride, 0);
    };
    auto st = [&](__amdgpu_buffer_rsrc_t r, int j, double v) {
        if (t0 + j * T < N) st_all(r, j, v);
    };
    double w[EPT], a[B][EPT], an[B][EPT];
    // w in registers; the raw direction z~ is stored as direction k
    {
        const __amdgpu_buffer_rsrc_t rw = buffer_of(A.w, bytes), rz = buffer_of(A.z, bytes);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            w[j] = ld(rw, j);
            an[0][j] = ld(rz, j);
        }
        if (!MASK || A.Zk) { // uniform
            const __amdgpu_buffer_rsrc_t rk = buffer_of(A.Zk, bytes);
#pragma unroll
            for (int j = 0; j < EPT; ++j) st_all(rk, j, an[0][j]);
        }
    }
    for (int i = threadIdx.x; i < min(k, kPtrLds); i += blockDim.x) ptab[i] = (unsigned long long)A.Wp[i];
    __syncthreads();
    auto load_block = [&](double (&dst)[B][EPT], int j0) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const int j = j0 + t;
            if (j < k) { // uniform
                const __amdgpu_buffer_rsrc_t rt =
                    buffer_of(j < kPtrLds ? (const void*)ptab[j] : (const void*)A.Wp[j], bytes);
#pragma unroll
                for (int j = 0; j < EPT; ++j) dst[t][j] = ld(rt, j);
            } else {
#pragma unroll
                for (int j = 0; j < EPT; ++j) dst[t][j] = 0.0;
            }
        }
    };
    const int nblk = (k + B - 1) / B;
    const int gk = k % B; // directions of the new direction's MGS block stored before it
    const __amdgpu_buffer_rsrc_t rr = buffer_of(A.r, bytes);
    unsigned long long g = A.g0;
    double vals[SW];
    // phase g0: dots of the first block and ||w||^2 (with no stored direction:
    // w.r and ||w||^2, the only exchange). The next block is loaded meanwhile;
    // block b+2 is requested as soon as block b+1 becomes current, and r (kept
    // in registers) as soon as no block is left to request.
    load_block(a, 0);
    if (nblk > 1) {
        load_block(an, B);
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) an[0][j] = ld(rr, j);
    }
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
        if (k == 0) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) s = fma(w[j], an[0][j], s);
            vals[0] = s;
        }
        bsum_n<SW>(vals, SW, sh);
        publish<SW>(A.slots, G, bid, g, vals, SW);
    }
    double nin2 = 0.0, nout2 = 0.0, wr = 0.0;
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
                for (int m = 0; m < t; ++m)
                    bt = fma(-A.gram[(int64_t)(j0 + t) * kGramStride + (t - m - 1)], beta[m], bt);
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
            if (b + 2 < nblk) {
                load_block(an, j0 + 2 * B);
            } else {
#pragma unroll
                for (int j = 0; j < EPT; ++j) an[0][j] = ld(rr, j);
            }
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
            // the orthogonalised w: ||w||^2, w.r and the dots with the earlier
            // directions of the new direction's MGS block (a holds that block)
            double s = 0.0, q = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                s = fma(w[j], w[j], s);
                q = fma(w[j], an[0][j], q);
            }
            vals[0] = s;
            vals[1] = q;
#pragma unroll
            for (int t = 0; t < B - 1; ++t) {
                double h = 0.0;
                if (t < gk) {
#pragma unroll
                    for (int j = 0; j < EPT; ++j) h = fma(a[t][j], w[j], h);
                }
                vals[2 + t] = h;
            }
            bsum_n<SW>(vals, SW, sh);
            publish<SW>(A.slots, G, bid, g, vals, SW);
        }
    }
    // the last exchange (phase g0 when no direction is stored)
    collect<SW, LEAD>(A.slots, G, bid, g, SW, tot, sh, A.abort_flag);
    if (k == 0) {
        nin2 = tot[B];
        nout2 = nin2;
        wr = tot[0];
    } else {
        nout2 = tot[0];
        wr = tot[1];
    }
    const double nin = sqrt(nin2), nout = sqrt(nout2);
    const bool keep = nout > A.breakdown * nin; // false for NaN and for nout == 0
    const double gamma = keep ? 1.0 / nout : 0.0;
    const double alpha = gamma * wr; // w_k . r with w_k = gamma w
    const __amdgpu_buffer_rsrc_t rwk = buffer_of(A.Wk, bytes);
    double s_r = 0.0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const double wk = w[j] * gamma;
        st(rwk, j, wk);
        const double rn = fma(-alpha, wk, an[0][j]);
        st(rr, j, rn);
        s_r = fma(rn, rn, s_r);
    }
    s_r = bsum(s_r, sh);
    if (threadIdx.x == 0) {
        A.part_rn[bid] = s_r;
        if (bid == 0) {
            A.alphas[k] = alpha;
            A.gammas[k] = gamma;
            // W_k . W_{k-d} = gamma (w . a[gk-d]) for the gk earlier directions of its block
            for (int d = 1; d <= kGramStride; ++d)
                A.gram[(int64_t)k * kGramStride + d - 1] = (d <= gk) ? gamma * tot[2 + gk - d] : 0.0;
            if (!keep) A.scal[S_BREAKDOWNS] += 1.0;
        }
    }
}

template <int EPT, int B, bool LEAD>
__global__ __launch_bounds__(kThreads) void k_rm_blk(RmArgs A) {
    __shared__ double sh[kMaxVals * (kThreads / 64)];
    __shared__ unsigned long long ptab[kPtrLds];
    rm_body<EPT, B, LEAD>(A, gridDim.x, blockIdx.x, sh, ptab);
}

// The same on vectors without a zero tail (caller arrays).
template <int EPT, int B, bool LEAD>
__global__ __launch_bounds__(kThreads) void k_rm_masked(RmArgs A) {
    __shared__ double sh[kMaxVals * (kThreads / 64)];
    __shared__ unsigned long long ptab[kPtrLds];
    rm_body<EPT, B, LEAD, true>(A, gridDim.x, blockIdx.x, sh, ptab);
}

// ---------------------------------------------------------------------------
// Lagged form. The exchange of an MGS block's dot products is the latency
// that bounds the forms above: block b's dots need w after block b-1's
// update, so every exchange is waited for before the next block's dots. Here
// the dots of block s are taken against w as it stands L blocks earlier (w
// updated through block s-L-1) and published at once; the exchange of block
// s-L, published L steps ago, is collected after that, so L exchanges are in
// flight while the next direction blocks stream in. The exact MGS
// coefficients follow from the lagged dots with the stored Gram entries of
// the directions in between (the MGS recursion in exact arithmetic, as in
// low-synchronisation Gram-Schmidt, Swirydowicz et al., Numer. Linear Algebra
// Appl. 2021):
//   beta_j = W_j . w_{(s-L)} - sum_{m = (s-L) B}^{j-1} (W_j . W_m) beta_m.
// Exchange words rotate over S sets: a block publishes phase s having
// collected phase s-L-1, so every block has read phase s-2L-2 or older when a
// set is reused after S >= 2L+2 phases; with S = 4 (L = 1) or 8 (L = 2) the
// reused set's stale words carry a different phase tag (mod 3).
template <int SW, int S>
__device__ __forceinline__ void publish_lag(unsigned long long* slots, int G, int bid, unsigned long long g,
                                            const double* v, int nw) {
    if (threadIdx.x == 0) {
        unsigned long long* p = slots + ((g % S) * (unsigned long long)G + bid) * SW;
        const unsigned tag = (unsigned)(g % 3);
        for (int i = 0; i < SW; ++i)
            __hip_atomic_store(p + i, tag_pack(i < nw ? v[i] : 0.0, tag), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Phase g's totals for the lagged form, in either exchange form (see
// collect): set g % S of the block words, totals after the S sets.
template <int SW, bool LEAD, int S>
__device__ __forceinline__ void collect_lag(unsigned long long* slots, int G, int bid, unsigned long long g, int nw,
                                            double* out, double* sh, unsigned* abort_flag) {
    const unsigned tag = (unsigned)(g % 3);
    const unsigned long long* base = slots + (g % S) * (unsigned long long)G * SW;
    unsigned long long* tot = slots + (unsigned long long)S * kMaxRedBlocks * SW + (g % S) * SW;
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

// Grids of the lagged form: at most two blocks' words per thread and word
// index in an exchange.
constexpr int kLagMaxBlocks = 2 * kThreads;

// Direction blocks held after their dots for the updates: L for one
// direction per block; L + 1 otherwise, so that the dots of a new direction
// with every direction a later lagged step corrects for are at hand.
template <int B, int L>
constexpr int lag_hold() { return B == 1 ? L : L + 1; }
template <int B, int L>
constexpr int lag_words() { return (2 + lag_hold<B, L>() * B) > (B + 1) ? 2 + lag_hold<B, L>() * B : B + 1; }
template <int L>
constexpr int lag_sets() { return L == 2 ? 8 : 4; }
static_assert(lag_words<kRmBlock, kRmLagMax>() <= kRmLagWords, "lag words");

template <int EPT, int B, int L, bool LEAD>
__device__ __forceinline__ void rm_body_lag(const RmArgs& A, const int G, const int bid, double* sh,
                                            unsigned long long* ptab) {
    constexpr int H = lag_hold<B, L>();
    constexpr int SW = lag_words<B, L>();
    constexpr int S = lag_sets<L>();
    const int64_t T = (int64_t)G * blockDim.x;
    const int64_t t0 = (int64_t)bid * blockDim.x + threadIdx.x;
    const int64_t N = A.N;
    const int k = A.k;
    const int toff = (int)t0 * 8;
    const int stride = (int)T * 8;
    const int bytes = (int)((N + kVecPad) * 8);
    auto ld = [&](__amdgpu_buffer_rsrc_t r, int j) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, toff, j * stride, 0));
    };
    auto st_all = [&](__amdgpu_buffer_rsrc_t r, int j, double v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufData, v), r, toff, j * stride, 0);
    };
    auto st = [&](__amdgpu_buffer_rsrc_t r, int j, double v) {
        if (t0 + j * T < N) st_all(r, j, v);
    };
    // w, and a ring of R direction blocks: block j in ring[j % R] (r, after
    // the last block, in ring[nblk % R]). In step s the ring holds the H
    // blocks before s (awaiting their update, or held for the new
    // direction's Gram dots), block s and block s + 1 streaming in; every
    // role stays in the same registers, so the next block's loads are issued
    // before this block is waited for and no block is copied.
    constexpr int R = H + 2;
    double w[EPT], ring[R][B][EPT];
    {
        const __amdgpu_buffer_rsrc_t rw = buffer_of(A.w, bytes), rz = buffer_of(A.z, bytes),
                                     rk = buffer_of(A.Zk, bytes);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            w[j] = ld(rw, j);
            ring[1][0][j] = ld(rz, j);
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) st_all(rk, j, ring[1][0][j]);
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int t = 0; t < B; ++t)
#pragma unroll
            for (int j = 0; j < EPT; ++j) ring[i][t][j] = 0.0;
    for (int i = threadIdx.x; i < min(k, kPtrLds); i += blockDim.x) ptab[i] = (unsigned long long)A.Wp[i];
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rr = buffer_of(A.r, bytes);
    const int nblk = (k + B - 1) / B;
    // Block blk (zeros past k), or r when blk == nblk. Every call issues the
    // same B EPT loads (a direction past k reads r and is zeroed), so that
    // the compiler can count the loads in flight exactly and wait for one
    // block without waiting for the next.
    auto load_block = [&](double (&dst)[B][EPT], int blk) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const int j = blk * B + t;
            const bool dir = blk < nblk && j < k; // uniform
            const __amdgpu_buffer_rsrc_t rt =
                dir ? buffer_of((const void*)ptab[j % kPtrLds], bytes) : rr;
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const double v = ld(rt, q);
                dst[t][q] = (dir || (blk == nblk && t == 0)) ? v : 0.0;
            }
        }
    };
    unsigned long long g0 = A.g0;
    double nin2 = 0.0;
    double bwin[L][B]; // beta of the L blocks before the one being finished (bwin[0]: the latest)
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
        for (int t = 0; t < B; ++t) bwin[i][t] = 0.0;
    // Gram entries W_{j0+t} . W_{j0+t-d}, d = 1 .. B + L B - 1, of block b2
    // (gram[(j0 + t) kGramStride + d - 1]), read before they are needed
    constexpr int GD = B + L * B - 1;
    auto gram_issue = [&](int b2, double (&gp)[B][GD]) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const int64_t gj = (int64_t)max(0, min(b2 * B + t, k - 1)) * kGramStride;
#pragma unroll
            for (int d = 0; d < GD; ++d) gp[t][d] = A.gram[gj + d];
        }
    };
    // form block b2's MGS coefficients from its exchange totals and update w with blk
    auto finish_block = [&](int b2, const double (&tot)[SW], const double (&gp)[B][GD],
                            const double (&blk)[B][EPT]) {
        if (b2 == 0) nin2 = tot[B];
        const int j0 = b2 * B, nb = min(B, k - j0);
        double beta[B];
#pragma unroll
        for (int t = 0; t < B; ++t) {
            double bt = 0.0;
            if (t < nb) {
                bt = tot[t];
#pragma unroll
                for (int m = 0; m < t; ++m) bt = fma(-gp[t][t - m - 1], beta[m], bt);
                // directions of the L blocks before: W_{j0-e}, e = 1 .. L B
#pragma unroll
                for (int e = 1; e <= L * B; ++e)
                    if (j0 - e >= 0) bt = fma(-gp[t][t + e - 1], bwin[(e - 1) / B][B - 1 - (e - 1) % B], bt);
            }
            beta[t] = bt;
        }
        if (bid == 0 && threadIdx.x == 0)
            for (int t = 0; t < nb; ++t) A.hist[(int64_t)k * (k - 1) / 2 + j0 + t] = beta[t];
#pragma unroll
        for (int t = 0; t < B; ++t)
#pragma unroll
            for (int j = 0; j < EPT; ++j) w[j] = fma(-beta[t], blk[t][j], w[j]);
#pragma unroll
        for (int i = L - 1; i > 0; --i)
#pragma unroll
            for (int t = 0; t < B; ++t) bwin[i][t] = bwin[i - 1][t];
#pragma unroll
        for (int t = 0; t < B; ++t) bwin[0][t] = beta[t];
    };
    // Exchange reads of the main loop. The first read of every word a step
    // needs is issued at the top of the step, before that step's direction
    // loads: a wave's loads complete in issue order, so a word read after
    // them could only be seen once the next block has arrived. The words are
    // normally there by then (published at least one step earlier); a word
    // that is not is read again until it is.
    // All-to-all: every block reads all block words of phase s - L.
    // Leader with two exchanges in flight: block 0 gathers phase s - 1 in
    // step s and publishes its totals, which the other blocks read in step
    // s + 1 as phase (s + 1) - L; block 0 keeps them for that step. With one
    // exchange in flight the leader gathers phase s - L in step s.
    // The number of loads issued does not depend on the block, the phase or
    // the lane (a block index past the grid reads a valid word, ignored).
    // Only the B dot-product words are read early; the first exchange's
    // extra word (||w||^2) is read when it is needed.
    constexpr int NL = B;                       // words read early
    constexpr int P = kLagMaxBlocks / kThreads; // block words per thread and word index
    constexpr bool AHEAD = LEAD && L == 2;
    const bool gather = !LEAD || bid == 0;
    const unsigned tot_off = (unsigned)S * kMaxRedBlocks * SW;
    unsigned long long pw[P][NL];
    auto nw_of = [&](int g) { return g == 0 ? B + 1 : B; };
    auto word_addr = [&](int g, int i, int q) -> const unsigned long long* {
        const unsigned long long ph = g0 + g;
        const int blk = min((int)threadIdx.x + i * kThreads, G - 1);
        return gather ? A.slots + ((ph % S) * (unsigned long long)G + blk) * SW + q
                      : A.slots + tot_off + (ph % S) * SW + q;
    };
    auto poll_issue = [&](int g) { // phase g (relative to g0)
#pragma unroll
        for (int i = 0; i < P; ++i)
#pragma unroll
            for (int q = 0; q < NL; ++q)
                pw[i][q] = __hip_atomic_load(word_addr(g, i, q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // phase g's totals from the words read by poll_issue (the sums of
    // collect_lag); the leader publishes them
    auto poll_finish = [&](int g, double (&tot)[SW]) {
        const unsigned long long ph = g0 + g;
        const unsigned tag = (unsigned)(ph % 3);
        const int nw = nw_of(g);
#pragma unroll
        for (int q = 0; q < SW; ++q) tot[q] = 0.0;
        if (gather) {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                if ((int)threadIdx.x + i * kThreads < G) {
#pragma unroll
                    for (int q = 0; q <= NL; ++q) {
                        if (q < nw) {
                            // the extra word of the first exchange was not read early
                            unsigned long long v = pw[i][q < NL ? q : 0];
                            if (q == NL || (unsigned)(v & 3ull) != tag)
                                v = wait_word(word_addr(g, i, q), tag, A.abort_flag);
                            tot[q] += tag_value(v);
                        }
                    }
                }
            }
            bsum_n<SW>(tot, nw, sh);
            if (LEAD) {
                unsigned long long* tp = A.slots + tot_off + (ph % S) * SW;
                if (threadIdx.x == 0)
                    for (int q = 0; q < SW; ++q)
                        __hip_atomic_store(tp + q, tag_pack(q < nw ? tot[q] : 0.0, tag), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int q = 0; q < SW; ++q) tot[q] = tag_value(tag_pack(tot[q], tag));
            }
        } else {
#pragma unroll
            for (int q = 0; q <= NL; ++q) {
                if (q < nw) {
                    unsigned long long v = pw[0][q < NL ? q : 0];
                    if (q == NL || (unsigned)(v & 3ull) != tag) v = wait_word(word_addr(g, 0, q), tag, A.abort_flag);
                    tot[q] = tag_value(v);
                }
            }
        }
    };
    double ahead[SW]; // leader with two exchanges in flight: totals gathered one step early
#pragma unroll
    for (int q = 0; q < SW; ++q) ahead[q] = 0.0;
    int ahead_g = -1;
    // step s, C = s % R: ring[C] holds block s (arriving), ring[C + 1]
    // receives block s + 1 (or r), ring[C - L] holds block s - L
    auto step = [&](int s, auto cr) {
        constexpr int C = decltype(cr)::value;
        double (&cb)[B][EPT] = ring[C];
        double (&nb)[B][EPT] = ring[(C + 1) % R];
        const int pg = (AHEAD && bid == 0) ? s - 1 : s - L; // the phase whose words are read
        const int fb = s - L;                               // the block finished
        poll_issue(max(pg, 0));
        double gp[B][GD];
        gram_issue(fb, gp);
        if ((s + 1) * B % (kPtrLds / 2) == 0) ptr_ring_refill(ptab, A.Wp, k, (s + 1) * B);
        load_block(nb, s + 1);
        double vals[SW];
#pragma unroll
        for (int i = 0; i < SW; ++i) vals[i] = 0.0;
#pragma unroll
        for (int t = 0; t < B; ++t) {
            double d = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) d = fma(cb[t][j], w[j], d);
            vals[t] = d;
        }
        if (s == 0) {
            double s_in = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) s_in = fma(w[j], w[j], s_in);
            vals[B] = s_in;
        }
        bsum_n<SW>(vals, s == 0 ? B + 1 : B, sh);
        publish_lag<SW, S>(A.slots, G, bid, g0 + s, vals, s == 0 ? B + 1 : B);
        if (pg >= 0) {
            double tot[SW];
            poll_finish(pg, tot);
            if (AHEAD && bid == 0) {
                // finish block s - L with the totals gathered in the previous step
                if (fb >= 0) finish_block(fb, ahead, gp, ring[(C + R - L) % R]);
#pragma unroll
                for (int q = 0; q < SW; ++q) ahead[q] = tot[q];
                ahead_g = pg;
            } else {
                finish_block(fb, tot, gp, ring[(C + R - L) % R]);
            }
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    static_assert(R == 3 || R == 4, "ring of three or four blocks");
    load_block(ring[0], 0); // block 0, or r when there is no direction
    int s = 0;
    for (; s + R <= nblk; s += R) {
        step(s, I0{});
        step(s + 1, I1{});
        step(s + 2, I2{});
        if constexpr (R == 4) step(s + 3, I3{});
    }
    if (s < nblk) step(s, I0{});
    if (s + 1 < nblk) step(s + 1, I1{});
    if constexpr (R == 4)
        if (s + 2 < nblk) step(s + 2, I2{});
    // rotate the ring so that r is in ring[0] and block nblk - 1 - h in
    // ring[R - 1 - h] (one uniform selection per entry, no indexed registers)
    {
        const int rot = nblk % R;
#pragma unroll
        for (int t = 0; t < B; ++t)
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                double v[R];
#pragma unroll
                for (int i = 0; i < R; ++i) v[i] = ring[i][t][j];
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    double x = v[i];
#pragma unroll
                    for (int q = 1; q < R; ++q)
                        if (rot == q) x = v[(i + q) % R];
                    ring[i][t][j] = x;
                }
            }
    }
    double (&nxt)[B][EPT] = ring[0]; // r
    // drain: the last min(L, nblk) blocks, oldest first (block nblk-1-h in ring[R-1-h])
#pragma unroll
    for (int h = L - 1; h >= 0; --h) {
        const int b2 = nblk - 1 - h;
        if (b2 >= 0) {
            double tot[SW], gp[B][GD];
            gram_issue(b2, gp);
            if (AHEAD && bid == 0 && b2 == ahead_g) {
#pragma unroll
                for (int q = 0; q < SW; ++q) tot[q] = ahead[q];
            } else {
                collect_lag<SW, LEAD, S>(A.slots, G, bid, g0 + b2, nw_of(b2), tot, sh, A.abort_flag);
            }
            finish_block(b2, tot, gp, ring[R - 1 - h]);
        }
    }
    // the orthogonalised w: ||w||^2, w.r and its dots with the held directions
    // (ring[R-1-h][t] = direction (nblk-1-h) B + t)
    double vals[SW];
    {
        double s2 = 0.0, q = 0.0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            s2 = fma(w[j], w[j], s2);
            q = fma(w[j], nxt[0][j], q);
        }
        vals[0] = s2;
        vals[1] = q;
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int t = 0; t < B; ++t) {
                double d = 0.0;
#pragma unroll
                for (int j = 0; j < EPT; ++j) d = fma(ring[R - 1 - h][t][j], w[j], d);
                vals[2 + h * B + t] = d;
            }
#pragma unroll
        for (int i = 2 + H * B; i < SW; ++i) vals[i] = 0.0;
    }
    bsum_n<SW>(vals, SW, sh);
    publish_lag<SW, S>(A.slots, G, bid, g0 + nblk, vals, SW);
    double tot[SW];
    collect_lag<SW, LEAD, S>(A.slots, G, bid, g0 + nblk, SW, tot, sh, A.abort_flag);
    const double nout2 = tot[0], wr = tot[1];
    if (k == 0) nin2 = nout2;
    const double nin = sqrt(nin2), nout = sqrt(nout2);
    const bool keep = nout > A.breakdown * nin; // false for NaN and for nout == 0
    const double gamma = keep ? 1.0 / nout : 0.0;
    const double alpha = gamma * wr;
    const __amdgpu_buffer_rsrc_t rwk = buffer_of(A.Wk, bytes);
    double s_r = 0.0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const double wk = w[j] * gamma;
        st(rwk, j, wk);
        const double rn = fma(-alpha, wk, nxt[0][j]);
        st(rr, j, rn);
        s_r = fma(rn, rn, s_r);
    }
    s_r = bsum(s_r, sh);
    if (threadIdx.x == 0) {
        A.part_rn[bid] = s_r;
        if (bid == 0) {
            A.alphas[k] = alpha;
            A.gammas[k] = gamma;
            for (int d = 1; d <= kGramStride; ++d) A.gram[(int64_t)k * kGramStride + d - 1] = 0.0;
            // W_k . W_m = gamma (w . ring[R-1-h][t]) for the held directions m < k
#pragma unroll
            for (int h = 0; h < H; ++h)
#pragma unroll
                for (int t = 0; t < B; ++t) {
                    const int m = (nblk - 1 - h) * B + t;
                    const int d = k - m;
                    if (m >= 0 && d >= 1 && d <= kGramStride)
                        A.gram[(int64_t)k * kGramStride + d - 1] = gamma * tot[2 + h * B + t];
                }
            if (!keep) A.scal[S_BREAKDOWNS] += 1.0;
        }
    }
}

template <int EPT, int B, int L, bool LEAD>
__global__ __launch_bounds__(kThreads) void k_rm_lag(RmArgs A) {
    __shared__ double sh[kRmLagWords * (kThreads / 64)];
    __shared__ unsigned long long ptab[kPtrLds];
    rm_body_lag<EPT, B, L, LEAD>(A, gridDim.x, blockIdx.x, sh, ptab);
}

// Column q of a multi-column launch (the column whose block range holds this
// block) and its RM arguments.
__device__ __forceinline__ RmArgs multi_args(const RmMulti& M, int& q) {
    q = 0;
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
    return A;
}

// RM of several vector sets (columns of a batched solve, or independent
// solvers of one level configuration) in one launch: column q owns blocks
// [blk0[q], blk0[q+1]) and exchanges only among them, with its own words,
// phase and storage (table entry idx[q]); all columns share k.
template <int EPT, int B, bool LEAD>
__global__ __launch_bounds__(kThreads) void k_rm_multi(RmMulti M) {
    __shared__ double sh[kMaxVals * (kThreads / 64)];
    __shared__ unsigned long long ptab[kPtrLds];
    int q = 0;
    const RmArgs A = multi_args(M, q);
    rm_body<EPT, B, LEAD>(A, M.blk0[q + 1] - M.blk0[q], (int)blockIdx.x - M.blk0[q], sh, ptab);
}

// The lagged form of the same (every column tuned to this lagged
// configuration, so that each column runs the arithmetic of its own solve).
template <int EPT, int B, int L, bool LEAD>
__global__ __launch_bounds__(kThreads) void k_rm_multi_lag(RmMulti M) {
    __shared__ double sh[kRmLagWords * (kThreads / 64)];
    __shared__ unsigned long long ptab[kPtrLds];
    int q = 0;
    const RmArgs A = multi_args(M, q);
    rm_body_lag<EPT, B, L, LEAD>(A, M.blk0[q + 1] - M.blk0[q], (int)blockIdx.x - M.blk0[q], sh, ptab);
}


// ---------------------------------------------------------------------------
// Exchange-wave form of the same kernel. The vector memory reads of one wave
// return in issue order, so in the form above a wave's wait for an exchange
// word also waits for every direction load it issued earlier: a direction
// costs a load latency plus an exchange latency. Here each block has a fifth
// wave that issues no vector-stream loads. It performs every grid exchange
// (block sum of the compute waves' partials, publish, wait, grid sum), the
// MGS coefficient recursion and the bookkeeping stores, and it reads the
// direction pointers two MGS blocks ahead into shared memory. The four
// compute waves stream the vectors and meet it at two barriers per exchange
// (partials written, results written), so their direction loads stay in
// flight while it waits. Every sum is formed in the order of the form above
// (per-thread sums over blocks t, t + 256, ..., wave butterflies, then the
// four waves in turn), so both forms give bitwise identical results for the
// same configuration.
// The form is instantiated with NC = 4 compute waves (the plain form's thread
// layout, hence its summation order) and with NC = 3 for the largest
// entries-per-thread counts, where four waves of registers per block would
// leave only one block per compute unit.
constexpr int kCwWaves = kThreads / 64; // lane groups of the exchange wave's gather
// blocks per exchange-wave lane and lane group: grids up to 512 blocks for
// at most 3 words per block, up to 256 blocks for more
template <int SW>
constexpr int cw_rounds() { return SW <= 3 ? 2 : 1; }
int cw_max_blocks(int B) { return 256 * (B + 1 <= 3 ? 2 : 1); }

struct CwShared {
    double part[kMaxVals][kCwWaves];     // wave partials of the compute waves
    double res[kMaxVals];                // results of the last exchange
    unsigned long long ptr[4][kRmBlock]; // direction pointers of MGS blocks (ring of 4)
};

// Grid sums of words [0, nw) of one phase (all-to-all), by the exchange wave:
// lane l reads the words of blocks 64 q + l + 256 r (q < 4, r < R) all at
// once and re-reads only those not yet carrying the tag. Every lane returns
// the same totals.
template <int SW, int R>
__device__ __forceinline__ void cw_gather(const unsigned long long* base, int G, int nw, unsigned tag,
                                          unsigned* abort_flag, double (&tot)[SW]) {
    const int lane = threadIdx.x & 63;
    unsigned long long v[kCwWaves][R][SW];
#pragma unroll
    for (int q = 0; q < kCwWaves; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int w = 0; w < SW; ++w) {
                const int i = 64 * q + lane + 256 * r;
                v[q][r][w] = (i < G && w < nw) ? __hip_atomic_load(base + (int64_t)i * SW + w, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT)
                                               : (unsigned long long)tag; // unused: counts as arrived
            }
    unsigned spins = 0;
    for (;;) {
        bool ready = true;
#pragma unroll
        for (int q = 0; q < kCwWaves; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int w = 0; w < SW; ++w) ready = ready && (unsigned)(v[q][r][w] & 3ull) == tag;
        if (__all(ready)) break;
        __builtin_amdgcn_s_sleep(1);
        ++spins;
        bool stop = spins > kSpinMax;
        if ((spins & 127) == 0)
            stop = stop || __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        if (__any(stop)) {
            if (lane == 0) __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
#pragma unroll
        for (int q = 0; q < kCwWaves; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int w = 0; w < SW; ++w)
                    if ((unsigned)(v[q][r][w] & 3ull) != tag)
                        v[q][r][w] = __hip_atomic_load(base + (int64_t)(64 * q + lane + 256 * r) * SW + w,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int w = 0; w < SW; ++w) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kCwWaves; ++q) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (64 * q + lane + 256 * r < G && w < nw) s += tag_value(v[q][r][w]);
            t += wsum(s);
        }
        tot[w] = t;
    }
}

// Totals of words [0, nw) of phase g by the exchange wave, in either exchange
// form (see collect); every lane returns the same values.
template <int SW, int R, bool LEAD>
__device__ __forceinline__ void cw_collect(unsigned long long* slots, int G, int bid, unsigned long long g, int nw,
                                           unsigned* abort_flag, double (&tot)[SW]) {
    const int lane = threadIdx.x & 63;
    const unsigned tag = (unsigned)(g % 3);
    const unsigned long long* base = slots + (g & 1) * (unsigned long long)G * SW;
    unsigned long long* totw = slots + 2ull * kMaxRedBlocks * (kRmBlock + 1) + (g & 1) * SW;
    if (!LEAD || bid == 0) {
        cw_gather<SW, R>(base, G, nw, tag, abort_flag, tot);
        if (LEAD) {
            double mine = 0.0;
#pragma unroll
            for (int w = 0; w < SW; ++w)
                if (w == lane && w < nw) mine = tot[w];
            if (lane < SW)
                __hip_atomic_store(totw + lane, tag_pack(mine, tag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int w = 0; w < SW; ++w) tot[w] = tag_value(tag_pack(tot[w], tag));
        }
    } else {
        unsigned long long b = (lane < nw) ? __hip_atomic_load(totw + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                           : (unsigned long long)tag;
        unsigned spins = 0;
        while (!__all((unsigned)(b & 3ull) == tag)) {
            __builtin_amdgcn_s_sleep(1);
            ++spins;
            bool stop = spins > kSpinMax;
            if ((spins & 127) == 0)
                stop = stop || __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
            if (__any(stop)) {
                if (lane == 0) __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            if ((unsigned)(b & 3ull) != tag)
                b = __hip_atomic_load(totw + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const double mine = tag_value(b);
#pragma unroll
        for (int w = 0; w < SW; ++w) tot[w] = (w < nw) ? __shfl(mine, w, 64) : 0.0;
    }
}

template <int EPT, int B, bool LEAD, int NC>
__device__ __forceinline__ void rm_body_cw(const RmArgs& A, const int G, const int bid, CwShared& S) {
    constexpr int SW = B + 1;
    constexpr int kThr = 64 * NC; // compute threads per block
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int k = A.k;
    const int nblk = (k + B - 1) / B;
    const int gk = k % B; // directions of the new direction's MGS block stored before it
    if (wid == NC) {
        // ------------------------------------------------ exchange wave
        constexpr int R = cw_rounds<SW>();
        unsigned long long g = A.g0;
        if (lane < B) {
            for (int blk = 0; blk < 2; ++blk) {
                const int j = blk * B + lane;
                if (j < k) S.ptr[blk][lane] = (unsigned long long)A.Wp[j];
            }
        }
        __syncthreads(); // pointers of blocks 0 and 1 in place
        double tot[SW];
        // one exchange of nw words: pointers of MGS block `ahead` are read
        // meanwhile; gram entries of block `blk` (if any) are returned in gm
        auto exchange = [&](int nw, int ahead, int blk, double (&gm)[B][B]) {
            unsigned long long pa = 0;
            const int ja = ahead * B + lane;
            const bool want = lane < B && ahead < nblk && ja < k;
            if (want) pa = (unsigned long long)A.Wp[ja];
#pragma unroll
            for (int t = 0; t < B; ++t)
#pragma unroll
                for (int m = 0; m < B; ++m) gm[t][m] = 0.0;
            if (blk >= 0) {
                const int j0 = blk * B, bb = min(B, k - j0);
#pragma unroll
                for (int t = 1; t < B; ++t)
                    if (t < bb)
#pragma unroll
                        for (int m = 0; m < t; ++m) gm[t][m] = A.gram[(int64_t)(j0 + t) * kGramStride + (t - m - 1)];
            }
            __syncthreads(); // compute waves' partials in place
            const unsigned tag = (unsigned)(g % 3);
            double bs = 0.0;
            if (lane < nw)
                for (int q = 0; q < NC; ++q) bs += S.part[lane][q];
            if (lane < SW)
                __hip_atomic_store(A.slots + ((g & 1) * (unsigned long long)G + bid) * SW + lane, tag_pack(bs, tag),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            cw_collect<SW, R, LEAD>(A.slots, G, bid, g, nw, A.abort_flag, tot);
            if (want) S.ptr[ahead & 3][lane] = pa;
            ++g;
        };
        // MGS coefficients of block blk from its dot products
        auto coefficients = [&](int blk, const double (&gm)[B][B]) {
            const int j0 = blk * B, bb = min(B, k - j0);
            double beta[B];
#pragma unroll
            for (int t = 0; t < B; ++t) {
                double bt = 0.0;
                if (t < bb) {
                    bt = tot[t];
#pragma unroll
                    for (int m = 0; m < t; ++m) bt = fma(-gm[t][m], beta[m], bt);
                }
                beta[t] = bt;
            }
            if (lane == 0) {
#pragma unroll
                for (int t = 0; t < B; ++t) S.res[t] = beta[t];
                if (bid == 0) // row k of the coefficient history
                    for (int t = 0; t < bb; ++t) A.hist[(int64_t)k * (k - 1) / 2 + j0 + t] = beta[t];
            }
        };
        double gm[B][B];
        double nin2 = 0.0, nout2 = 0.0, wr = 0.0;
        // gamma and alpha of the new direction from ||w|| before and after MGS
        // and w.r; the bookkeeping of direction k
        auto finish = [&]() {
            const double nin = sqrt(nin2), nout = sqrt(nout2);
            const bool keep = nout > A.breakdown * nin; // false for NaN and for nout == 0
            const double gamma = keep ? 1.0 / nout : 0.0;
            const double alpha = gamma * wr; // w_k . r with w_k = gamma w
            if (lane == 0) {
                S.res[0] = gamma;
                S.res[1] = alpha;
                if (bid == 0) {
                    A.alphas[k] = alpha;
                    A.gammas[k] = gamma;
                    for (int d = 1; d <= kGramStride; ++d)
                        A.gram[(int64_t)k * kGramStride + d - 1] = (d <= gk) ? gamma * tot[2 + gk - d] : 0.0;
                    if (!keep) A.scal[S_BREAKDOWNS] += 1.0;
                }
            }
        };
        exchange(SW, 2, k > 0 ? 0 : -1, gm); // dots of block 0 and ||w||^2 (no direction: w.r, ||w||^2)
        nin2 = tot[B];
        if (k > 0) {
            coefficients(0, gm);
        } else {
            nout2 = nin2;
            wr = tot[0];
            finish();
        }
        __syncthreads(); // results in place
        for (int b = 0; b < nblk; ++b) {
            if (b + 1 < nblk) {
                exchange(min(B, k - (b + 1) * B), b + 3, b + 1, gm);
                coefficients(b + 1, gm);
            } else {
                exchange(SW, nblk, -1, gm); // ||w||^2 after MGS, w.r, Gram dots
                nout2 = tot[0];
                wr = tot[1];
                finish();
            }
            __syncthreads(); // results in place
        }
        __syncthreads(); // partials of ||r||^2 in place
        if (lane == 0) {
            double s = 0.0;
            for (int q = 0; q < NC; ++q) s += S.part[0][q];
            A.part_rn[bid] = s;
        }
        return;
    }
    // ---------------------------------------------------- compute waves
    const int64_t T = (int64_t)G * kThr;
    const int64_t t0 = (int64_t)bid * kThr + threadIdx.x;
    const int64_t N = A.N;
    const int toff = (int)t0 * 8;
    const int stride = (int)T * 8;
    const int bytes = (int)((N + kVecPad) * 8);
    auto ld = [&](__amdgpu_buffer_rsrc_t r, int j) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, toff, j * stride, 0));
    };
    auto st_all = [&](__amdgpu_buffer_rsrc_t r, int j, double v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufData, v), r, toff, j * stride, 0);
    };
    auto st = [&](__amdgpu_buffer_rsrc_t r, int j, double v) {
        if (t0 + j * T < N) st_all(r, j, v);
    };
    // wave partials of nv values to shared memory (lane 0 of each wave)
    auto partials = [&](const double* v, int nv) {
#pragma unroll
        for (int i = 0; i < kMaxVals; ++i)
            if (i < nv) {
                const double s = wsum(v[i]);
                if (lane == 0) S.part[i][wid] = s;
            }
    };
    double w[EPT], a[B][EPT], an[B][EPT];
    {
        const __amdgpu_buffer_rsrc_t rw = buffer_of(A.w, bytes), rz = buffer_of(A.z, bytes),
                                     rk = buffer_of(A.Zk, bytes);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            w[j] = ld(rw, j);
            an[0][j] = ld(rz, j);
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) st_all(rk, j, an[0][j]);
    }
    __syncthreads(); // pointers of blocks 0 and 1 in place
    auto load_block = [&](double (&dst)[B][EPT], int blk) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            if (blk * B + t < k) { // uniform
                const __amdgpu_buffer_rsrc_t rt = buffer_of((const void*)S.ptr[blk & 3][t], bytes);
#pragma unroll
                for (int j = 0; j < EPT; ++j) dst[t][j] = ld(rt, j);
            } else {
#pragma unroll
                for (int j = 0; j < EPT; ++j) dst[t][j] = 0.0;
            }
        }
    };
    const __amdgpu_buffer_rsrc_t rr = buffer_of(A.r, bytes);
    load_block(a, 0);
    if (nblk > 1) {
        load_block(an, 1);
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) an[0][j] = ld(rr, j);
    }
    double vals[kMaxVals];
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
        if (k == 0) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) s = fma(w[j], an[0][j], s);
            vals[0] = s;
        }
        partials(vals, SW);
    }
    __syncthreads(); // partials in place
    __syncthreads(); // results in place
    for (int b = 0; b < nblk; ++b) {
        double beta[B];
#pragma unroll
        for (int t = 0; t < B; ++t) beta[t] = S.res[t];
#pragma unroll
        for (int t = 0; t < B; ++t)
#pragma unroll
            for (int j = 0; j < EPT; ++j) w[j] = fma(-beta[t], a[t][j], w[j]);
        if (b + 1 < nblk) {
#pragma unroll
            for (int t = 0; t < B; ++t)
#pragma unroll
                for (int j = 0; j < EPT; ++j) a[t][j] = an[t][j];
            if (b + 2 < nblk) {
                load_block(an, b + 2);
            } else {
#pragma unroll
                for (int j = 0; j < EPT; ++j) an[0][j] = ld(rr, j);
            }
#pragma unroll
            for (int t = 0; t < B; ++t) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < EPT; ++j) s = fma(a[t][j], w[j], s);
                vals[t] = s;
            }
            partials(vals, B);
        } else {
            // the orthogonalised w: ||w||^2, w.r and the dots with the earlier
            // directions of the new direction's MGS block (a holds that block)
            double s = 0.0, q = 0.0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                s = fma(w[j], w[j], s);
                q = fma(w[j], an[0][j], q);
            }
            vals[0] = s;
            vals[1] = q;
#pragma unroll
            for (int t = 0; t < B - 1; ++t) {
                double h = 0.0;
                if (t < gk) {
#pragma unroll
                    for (int j = 0; j < EPT; ++j) h = fma(a[t][j], w[j], h);
                }
                vals[2 + t] = h;
            }
            partials(vals, SW);
        }
        __syncthreads(); // partials in place
        __syncthreads(); // results in place
    }
    const double gamma = S.res[0], alpha = S.res[1];
    const __amdgpu_buffer_rsrc_t rwk = buffer_of(A.Wk, bytes);
    double s_r = 0.0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const double wk = w[j] * gamma;
        st(rwk, j, wk);
        const double rn = fma(-alpha, wk, an[0][j]);
        st(rr, j, rn);
        s_r = fma(rn, rn, s_r);
    }
    vals[0] = s_r;
    partials(vals, 1);
    __syncthreads(); // partials of ||r||^2 in place
}

template <int EPT, int B, bool LEAD, int NC>
__global__ __launch_bounds__(64 * (NC + 1)) void k_rm_cw(RmArgs A) {
    __shared__ CwShared S;
    rm_body_cw<EPT, B, LEAD, NC>(A, gridDim.x, blockIdx.x, S);
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

// nc: compute waves of the exchange-wave form, 0 for the plain form
template <int EPT, int B, bool LEAD>
static const void* rm_kernel(bool multi, int nc) {
    if constexpr (EPT > 20) { // three compute waves only
        if constexpr (B <= 2)
            if (!multi && nc == 3) return reinterpret_cast<const void*>(&k_rm_cw<EPT, B, LEAD, 3>);
        return nullptr;
    } else {
        if (multi) return nc ? nullptr : reinterpret_cast<const void*>(&k_rm_multi<EPT, B, LEAD>);
        if (nc == 4) return reinterpret_cast<const void*>(&k_rm_cw<EPT, B, LEAD, 4>);
        return nc ? nullptr : reinterpret_cast<const void*>(&k_rm_blk<EPT, B, LEAD>);
    }
}

// Instantiations: entries per thread EPT, MGS block B in {1, 2, 4}, exchange
// form (all-to-all or leader); the exchange-wave form with four compute waves
// for every EPT of kEpts, with three for kEpts3.
constexpr int kEpts[] = {1, 2, 4, 8, 10, 16, 20};
constexpr int kEpts3[] = {24, 28};
// every grid covers fewer than N + kVecPad entries (64 NC EPT < kVecPad) and
// byte offsets of the buffer accesses are 32-bit
static_assert(kThreads * 20 < kVecPad && 64 * 3 * 28 < kVecPad, "RM grid reach");
static_assert(((int64_t)kMaxRedBlocks * kThreads * 20 + kVecPad) * 8 < (int64_t)1 << 31, "RM offsets");
static_assert(((int64_t)512 * 64 * 3 * 28 + kVecPad) * 8 < (int64_t)1 << 31, "RM offsets");
template <int EPT, bool LEAD>
static const void* pick_b(int b, bool multi, int nc) {
    if (b == 4) return rm_kernel<EPT, 4, LEAD>(multi, nc);
    if (b == 2) return rm_kernel<EPT, 2, LEAD>(multi, nc);
    if (b == 1) return rm_kernel<EPT, 1, LEAD>(multi, nc);
    return nullptr;
}
template <int EPT>
static const void* pick_x(int b, int lead, bool multi, int nc) {
    return lead ? pick_b<EPT, true>(b, multi, nc) : pick_b<EPT, false>(b, multi, nc);
}
static const void* pick(int ept, int b, int lead, bool multi = false, int nc = 0) {
    switch (ept) {
    case 1: return pick_x<1>(b, lead, multi, nc);
    case 2: return pick_x<2>(b, lead, multi, nc);
    case 4: return pick_x<4>(b, lead, multi, nc);
    case 8: return pick_x<8>(b, lead, multi, nc);
    case 10: return pick_x<10>(b, lead, multi, nc);
    case 16: return pick_x<16>(b, lead, multi, nc);
    case 20: return pick_x<20>(b, lead, multi, nc);
    case 24: return nc == 3 ? pick_x<24>(b, lead, multi, nc) : nullptr;
    case 28: return nc == 3 ? pick_x<28>(b, lead, multi, nc) : nullptr;
    }
    return nullptr;
}
// Lagged form instantiations: one direction per exchange with one or two
// exchanges in flight for the entries per thread of bandwidth-bound levels;
// two or four directions per exchange with one in flight for the small,
// exchange-bound levels.
template <int EPT, int B, int L>
static const void* lag_kernel(int lead, bool multi) {
    if (multi)
        return lead ? reinterpret_cast<const void*>(&k_rm_multi_lag<EPT, B, L, true>)
                    : reinterpret_cast<const void*>(&k_rm_multi_lag<EPT, B, L, false>);
    return lead ? reinterpret_cast<const void*>(&k_rm_lag<EPT, B, L, true>)
                : reinterpret_cast<const void*>(&k_rm_lag<EPT, B, L, false>);
}
static const void* pick_lag(int ept, int b, int lag, int lead, bool multi = false) {
    if (b == 1 && lag == 2) {
        switch (ept) {
        case 8: return lag_kernel<8, 1, 2>(lead, multi);
        case 10: return lag_kernel<10, 1, 2>(lead, multi);
        case 16: return lag_kernel<16, 1, 2>(lead, multi);
        case 20: return lag_kernel<20, 1, 2>(lead, multi);
        }
    } else if (b == 1 && lag == 1) {
        switch (ept) {
        case 8: return lag_kernel<8, 1, 1>(lead, multi);
        case 10: return lag_kernel<10, 1, 1>(lead, multi);
        case 16: return lag_kernel<16, 1, 1>(lead, multi);
        case 20: return lag_kernel<20, 1, 1>(lead, multi);
        }
    } else if (b == 2 && lag == 1) {
        switch (ept) {
        case 2: return lag_kernel<2, 2, 1>(lead, multi);
        case 4: return lag_kernel<4, 2, 1>(lead, multi);
        case 8: return lag_kernel<8, 2, 1>(lead, multi);
        }
    } else if (b == 4 && lag == 1) {
        switch (ept) {
        case 1: return lag_kernel<1, 4, 1>(lead, multi);
        case 2: return lag_kernel<2, 4, 1>(lead, multi);
        case 4: return lag_kernel<4, 4, 1>(lead, multi);
        }
    }
    return nullptr;
}
static const void* pick_cfg(const RmConfig& c) {
    return c.lag ? pick_lag(c.ept, c.B, c.lag, c.lead) : pick(c.ept, c.B, c.lead, false, c.cw);
}
// threads per block and compute threads per block of a configuration
static int rm_block_threads(int nc) { return nc ? 64 * (nc + 1) : kThreads; }
static int rm_compute_threads(int nc) { return nc ? 64 * nc : kThreads; }

// Blocks of the multi-column kernel in this configuration that fit at once.
int rm_multi_capacity(int ept, int B, int lead, int lag) {
    int dev = 0, cus = 0, per_cu = 0;
    const void* f = lag ? pick_lag(ept, B, lag, lead, true) : pick(ept, B, lead, true);
    hipFuncAttributes fa;
    if (!f || hipFuncGetAttributes(&fa, f) != hipSuccess || fa.localSizeBytes > 0) return 0; // see candidates
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kThreads, 0) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_rm_multi(int ept, int B, int lead, int lag, const RmMulti& M, hipStream_t st) {
    const void* f = lag ? pick_lag(ept, B, lag, lead, true) : pick(ept, B, lead, true);
    if (!f || M.ncol < 1 || M.ncol > kMaxCols) return hipErrorInvalidValue;
    RmMulti a = M;
    void* params[] = {&a};
    return hipLaunchKernel(f, dim3(M.blk0[M.ncol]), dim3(kThreads), params, 0, st);
}

// Co-resident launch configurations for a level of N entries: grids of at
// most kMaxRedBlocks blocks whose blocks all fit at once (occupancy query),
// in order of preference (fewest entries per thread, then the largest MGS
// block, then at most 512 blocks before larger grids; the exchange-wave form
// before the plain one where both fit). Kernels that need scratch memory are
// left out: the runtime may limit the waves in flight of such a kernel to what
// its scratch allocation covers, below what the occupancy query reports.
int rm_persistent_candidates(int64_t N, RmConfig* out, int cap) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    int n = 0;
    auto consider = [&](int pass, int e, int b, int lead, int nc, int lag) {
        const int64_t per = (int64_t)rm_compute_threads(nc) * e;
        const int64_t need = (N + per - 1) / per;
        if (pass == 0 ? need > 512 : (need <= 512 || need > kMaxRedBlocks)) return;
        if (nc && need > cw_max_blocks(b)) return;
        if (lag && need > kLagMaxBlocks) return;
        const void* f = lag ? pick_lag(e, b, lag, lead) : pick(e, b, lead, false, nc);
        if (!f) return;
        hipFuncAttributes fa;
        int per_cu = 0;
        if (hipFuncGetAttributes(&fa, f) != hipSuccess || fa.localSizeBytes > 0) return;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, rm_block_threads(nc), 0) != hipSuccess ||
            per_cu < 1)
            return;
        // Five-wave blocks do not split evenly over a compute unit's four
        // SIMDs; two of them per unit have failed to be resident together
        // although the occupancy query allowed it, so they get one unit each.
        if (nc == 4) per_cu = 1;
        if (need > (int64_t)per_cu * cus) return;
        if (n < cap) out[n++] = RmConfig{(int)need, e, b, lead, nc, lag};
    };
    for (int pass = 0; pass < 2; ++pass) {
        for (int e : kEpts)
            for (int b : {4, 2, 1})
                for (int lead : {0, 1}) {
                    for (int nc : {4, 0}) consider(pass, e, b, lead, nc, 0);
                    for (int lag : {1, 2}) consider(pass, e, b, lead, 0, lag);
                }
        for (int e : kEpts3)
            for (int b : {2, 1})
                for (int lead : {0, 1}) consider(pass, e, b, lead, 3, 0);
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
    const int sw = rm_slot_words(c), sets = rm_slot_sets(c);
    if (L.slot_G == c.G && L.slot_SW == sw && L.slot_lead == c.lead && L.slot_sets == sets) return hipSuccess;
    hipError_t e = hipMemsetAsync(L.xslots, 0xFF, sizeof(unsigned long long) * kRmSlotWordsMax, st);
    if (e != hipSuccess) return e;
    L.slot_G = c.G;
    L.slot_SW = sw;
    L.slot_lead = c.lead;
    L.slot_sets = sets;
    return hipSuccess;
}

hipError_t launch_rm_persistent(const RmConfig& c, const RmArgs& args, hipStream_t st) {
    const void* f = pick_cfg(c);
    const int G = c.G;
    if (!f || (c.cw && (G > cw_max_blocks(c.B) || c.lag)) || G > kMaxRedBlocks ||
        (int64_t)G * rm_compute_threads(c.cw) * c.ept < args.N) // the grid must cover the vectors
        return hipErrorInvalidValue;
    RmArgs a = args;
    void* params[] = {&a};
    return hipLaunchKernel(f, dim3(G), dim3(rm_block_threads(c.cw)), params, 0, st);
}

// Masked plain-form kernels: MGS blocks of four directions, all-to-all exchange.
static const void* pick_masked(int ept) {
    switch (ept) {
    case 1: return reinterpret_cast<const void*>(&k_rm_masked<1, 4, false>);
    case 2: return reinterpret_cast<const void*>(&k_rm_masked<2, 4, false>);
    case 4: return reinterpret_cast<const void*>(&k_rm_masked<4, 4, false>);
    case 8: return reinterpret_cast<const void*>(&k_rm_masked<8, 4, false>);
    case 10: return reinterpret_cast<const void*>(&k_rm_masked<10, 4, false>);
    case 16: return reinterpret_cast<const void*>(&k_rm_masked<16, 4, false>);
    case 20: return reinterpret_cast<const void*>(&k_rm_masked<20, 4, false>);
    }
    return nullptr;
}

// The co-resident configuration of the masked kernel for N entries: the
// fewest entries per thread whose grid of at most kMaxRedBlocks blocks fits
// at once (occupancy query; kernels that need scratch memory left out).
bool rm_masked_config(int64_t N, RmConfig* cfg) {
    int dev = 0, cus = 0;
    if (N < 1 || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return false;
    for (int e : kEpts) {
        const int64_t need = (N + (int64_t)kThreads * e - 1) / ((int64_t)kThreads * e);
        if (need > kMaxRedBlocks) continue;
        const void* f = pick_masked(e);
        hipFuncAttributes fa;
        int per_cu = 0;
        if (!f || hipFuncGetAttributes(&fa, f) != hipSuccess || fa.localSizeBytes > 0) continue;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kThreads, 0) != hipSuccess || per_cu < 1)
            continue;
        if (need > (int64_t)per_cu * cus) continue;
        *cfg = RmConfig{(int)need, e, 4, 0, 0};
        return true;
    }
    return false;
}

hipError_t launch_rm_masked(const RmConfig& c, const RmArgs& args, hipStream_t st) {
    const void* f = pick_masked(c.ept);
    if (!f || c.B != 4 || c.lead || c.cw || (int64_t)c.G * kThreads * c.ept < args.N || c.G > kMaxRedBlocks)
        return hipErrorInvalidValue;
    RmArgs a = args;
    void* params[] = {&a};
    return hipLaunchKernel(f, dim3(c.G), dim3(kThreads), params, 0, st);
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
