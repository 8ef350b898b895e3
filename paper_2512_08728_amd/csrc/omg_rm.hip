// Persistent residual-minimisation kernel (Algorithm 1 after w = A z).
//
// One launch performs the whole modified Gram-Schmidt loop, the
// normalisation, alpha = w.r and the x/r update. Every thread keeps the
// entries of w and z it owns in registers for the whole loop, so each step
// reads W_i and Z_i exactly once from memory; the k sequential MGS
// coefficients need one grid-wide barrier each (the reductions are two-stage
// and deterministic: every block sums the same partials in the same order).
// A thread owns CPT cells (all bs components of each, component-major
// layout), cells t, t + T, ..., T = total threads.
//
// The grid is sized from the occupancy query so that every block is resident
// at once, and the launch is an ordinary one (cooperative launches carry a
// large per-launch cost on this runtime).
//
// Grid-wide exchange without fences: a device-scope memory fence on this
// 8-XCD part writes back / invalidates an XCD's L2 and costs tens of
// microseconds per barrier. Instead each block publishes its partial sum as
// ONE 64-bit agent-scope atomic store whose two low mantissa bits carry a
// phase tag (phase mod 3; 3 = empty), and every block reads all G published
// words with agent-scope atomic loads, waiting until each carries the
// expected tag. Phases alternate between two slot sets; a block writes phase
// g+2 into the set of phase g only after it has read every block's phase g+1
// word, so every block has finished reading phase g. The host keeps the phase
// counter of each level across launches, so a stale word always carries the
// tag of phase g-2, never that of g. Clearing the two tag bits perturbs each
// partial by at most 2^-51 relative; every reader sees the same words, so the
// sums stay identical across blocks and deterministic. Waits are bounded: a
// block that waits too long raises an abort flag that ends every other wait,
// so every wave reaches the end of the kernel; the host checks the flag.
#include "omg_internal.h"

namespace omg {

constexpr unsigned kSpinMax = 1u << 25;

__device__ __forceinline__ unsigned long long tag_pack(double v, unsigned tag) {
    return ((unsigned long long)__double_as_longlong(v) & ~3ull) | tag;
}
__device__ __forceinline__ double tag_value(unsigned long long b) { return __longlong_as_double(b & ~3ull); }

// Publish (v0, v1) of this block for phase g: slots[set][block][2].
__device__ __forceinline__ void publish(unsigned long long* slots, int G, unsigned long long g, double v0, double v1) {
    if (threadIdx.x == 0) {
        unsigned long long* p = slots + ((g & 1) * G + blockIdx.x) * 2;
        const unsigned tag = (unsigned)(g % 3);
        __hip_atomic_store(p + 1, tag_pack(v1, tag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(p, tag_pack(v0, tag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Wait for word `w` of every block's phase-g slot and return this thread's
// share of their sum (combine with a block reduction).
__device__ __forceinline__ double collect(unsigned long long* slots, int G, unsigned long long g, int w,
                                          unsigned* abort_flag) {
    const unsigned tag = (unsigned)(g % 3);
    const unsigned long long* base = slots + (g & 1) * G * 2 + w;
    double v = 0.0;
    for (int i = threadIdx.x; i < G; i += blockDim.x) {
        unsigned long long b = 0;
        unsigned spins = 0;
        for (;;) {
            b = __hip_atomic_load(base + 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((unsigned)(b & 3ull) == tag) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinMax || ((spins & 127) == 0 &&
                                       __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                b = 0;
                break;
            }
        }
        v += tag_value(b);
    }
    return v;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
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

// slots: exchange words (2 sets x G blocks x 2 words); g0: first phase of this
// launch (the launch uses phases g0 .. g0+k+1); part_rn: plain partials of
// ||r||^2 after the update (read by a later launch).
template <int BS, int CPT>
__global__ __launch_bounds__(kThreads) void k_rm_mgs(int n, int k, const double* const* __restrict__ Wp,
                                                     const double* const* __restrict__ Zp,
                                                     const double* __restrict__ wv, const double* __restrict__ zv,
                                                     double* __restrict__ Wk, double* __restrict__ Zk,
                                                     double* __restrict__ x, double* __restrict__ r,
                                                     unsigned long long* __restrict__ slots, unsigned long long g0,
                                                     double* __restrict__ part_rn, double breakdown,
                                                     double* __restrict__ scal, unsigned* __restrict__ abort_flag) {
    __shared__ double sh[kThreads / 64];
    const int G = gridDim.x;
    const int T = G * blockDim.x;
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    double w[CPT][BS], z[CPT][BS], a[CPT][BS], an[CPT][BS], zi[CPT][BS];
    bool valid[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = t0 + j * T;
        valid[j] = c < n;
#pragma unroll
        for (int q = 0; q < BS; ++q) {
            w[j][q] = valid[j] ? wv[(int64_t)q * n + c] : 0.0;
            z[j][q] = valid[j] ? zv[(int64_t)q * n + c] : 0.0;
        }
    }
    unsigned long long g = g0;
    // phase g0: ||w_in||^2 and W_0 . w
    double s_in = 0.0, s_d = 0.0;
    if (k > 0) {
        const double* W0 = Wp[0];
#pragma unroll
        for (int j = 0; j < CPT; ++j)
#pragma unroll
            for (int q = 0; q < BS; ++q) a[j][q] = valid[j] ? W0[(int64_t)q * n + t0 + j * T] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j)
#pragma unroll
        for (int q = 0; q < BS; ++q) {
            s_in = fma(w[j][q], w[j][q], s_in);
            if (k > 0) s_d = fma(a[j][q], w[j][q], s_d);
        }
    s_in = bsum(s_in, sh);
    s_d = bsum(s_d, sh);
    publish(slots, G, g, k > 0 ? s_d : s_in, s_in);
    const double nin = sqrt(bsum(collect(slots, G, g, 1, abort_flag), sh));
    double nout2 = nin * nin;
    for (int i = 0; i < k; ++i) {
        // loads that do not depend on beta_i go out before the wait
        const double* Zi = Zp[i];
        const bool more = i + 1 < k;
        const double* Wn = more ? Wp[i + 1] : Wp[i];
#pragma unroll
        for (int j = 0; j < CPT; ++j)
#pragma unroll
            for (int q = 0; q < BS; ++q) {
                const int64_t e = (int64_t)q * n + t0 + j * T;
                zi[j][q] = valid[j] ? Zi[e] : 0.0;
                an[j][q] = (valid[j] && more) ? Wn[e] : 0.0;
            }
        const double beta = bsum(collect(slots, G, g, 0, abort_flag), sh);
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < CPT; ++j)
#pragma unroll
            for (int q = 0; q < BS; ++q) {
                w[j][q] = fma(-beta, a[j][q], w[j][q]);
                z[j][q] = fma(-beta, zi[j][q], z[j][q]);
                a[j][q] = an[j][q];
                s = more ? fma(a[j][q], w[j][q], s) : fma(w[j][q], w[j][q], s);
            }
        s = bsum(s, sh);
        ++g;
        publish(slots, G, g, s, 0.0);
        if (!more) nout2 = bsum(collect(slots, G, g, 0, abort_flag), sh);
    }
    const double nout = sqrt(nout2);
    const bool keep = nout > breakdown * nin; // false for NaN and for nout == 0
    const double gamma = keep ? 1.0 / nout : 0.0;
    double s_a = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j)
#pragma unroll
        for (int q = 0; q < BS; ++q) {
            w[j][q] *= gamma;
            z[j][q] *= gamma;
            if (valid[j]) {
                const int64_t e = (int64_t)q * n + t0 + j * T;
                Wk[e] = w[j][q];
                Zk[e] = z[j][q];
                a[j][q] = r[e];
            } else {
                a[j][q] = 0.0;
            }
            s_a = fma(w[j][q], a[j][q], s_a);
        }
    s_a = bsum(s_a, sh);
    ++g;
    publish(slots, G, g, s_a, 0.0);
    const double alpha = bsum(collect(slots, G, g, 0, abort_flag), sh);
    double s_r = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j)
#pragma unroll
        for (int q = 0; q < BS; ++q) {
            const double rn = fma(-alpha, w[j][q], a[j][q]);
            if (valid[j]) {
                const int64_t e = (int64_t)q * n + t0 + j * T;
                x[e] = fma(alpha, z[j][q], x[e]);
                r[e] = rn;
            }
            s_r = fma(rn, rn, s_r);
        }
    s_r = bsum(s_r, sh);
    if (threadIdx.x == 0) {
        part_rn[blockIdx.x] = s_r;
        if (blockIdx.x == 0 && !keep) scal[S_BREAKDOWNS] += 1.0;
    }
}

template <int BS, int CPT>
static const void* rm_kernel() {
    return reinterpret_cast<const void*>(&k_rm_mgs<BS, CPT>);
}

static const void* pick(int bs, int cpt) {
#define OMG_PICK(B)                                   \
    if (bs == B) {                                    \
        if (cpt == 1) return rm_kernel<B, 1>();       \
        if (cpt == 2) return rm_kernel<B, 2>();       \
        if (cpt == 4 && B * 4 <= 40) return rm_kernel<B, (B * 4 <= 40 ? 4 : 1)>(); \
        if (cpt == 8 && B * 8 <= 40) return rm_kernel<B, (B * 8 <= 40 ? 8 : 1)>(); \
        return nullptr;                               \
    }
    OMG_PICK(1)
    OMG_PICK(4)
    OMG_PICK(10)
    OMG_PICK(20)
#undef OMG_PICK
    return nullptr;
}

// Choose the cooperative grid for a level: as many co-resident blocks as the
// device holds (capped by the cells), CPT = cells per thread.
bool rm_persistent_config(int n, int bs, int* G, int* cpt) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    for (int c : {1, 2, 4, 8}) {
        const void* f = pick(bs, c);
        if (!f) continue;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kThreads, 0) != hipSuccess || per_cu < 1)
            continue;
        const int64_t max_blocks = (int64_t)per_cu * cus;
        const int64_t need = ((int64_t)n + (int64_t)kThreads * c - 1) / ((int64_t)kThreads * c);
        // every block reads every block's word per exchange: keep G moderate
        if (need <= max_blocks && need <= 512) {
            *G = (int)need;
            *cpt = c;
            return true;
        }
    }
    return false;
}

hipError_t launch_rm_persistent(int n, int bs, int G, int cpt, int k, const double* const* Wp,
                                const double* const* Zp, const double* w, const double* z, double* Wk, double* Zk,
                                double* x, double* r, unsigned long long* slots, unsigned long long g0,
                                double* part_rn, double breakdown, double* scal, unsigned* abort_flag,
                                hipStream_t st) {
    const void* f = pick(bs, cpt);
    if (!f) return hipErrorInvalidValue;
    void* args[] = {&n, &k, (void*)&Wp, (void*)&Zp, (void*)&w, (void*)&z, &Wk, &Zk, &x, &r, &slots, &g0,
                    &part_rn, &breakdown, &scal, &abort_flag};
    return hipLaunchKernel(f, dim3(G), dim3(kThreads), args, 0, st);
}

} // namespace omg
