// One residual-minimisation step (Algorithm 1 after w = A z) for callers that
// cannot allocate device memory: the persistent RM kernel runs on the
// caller's arrays, and every piece of scratch it needs -- grid-exchange
// words, block partials, the abort flag, the MGS coefficients and the
// direction pointer table -- lives in one file-scope device array of fixed
// size instead of memory the library allocates.
#include <cmath>
#include <mutex>

#include "omg_internal.h"

namespace omg {

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
// layout of the scratch array (byte offsets)
constexpr size_t kStWords = 0;                                                        // kRmSlotWords words
constexpr size_t kStPart = align256(kStWords + sizeof(unsigned long long) * kRmSlotWords); // block partials
constexpr size_t kStScal = align256(kStPart + sizeof(double) * kMaxRedBlocks);        // S_COUNT scalars
constexpr size_t kStFlags = align256(kStScal + sizeof(double) * S_COUNT);             // [1]: abort flag
constexpr size_t kStGam = align256(kStFlags + 2 * sizeof(unsigned));
constexpr size_t kStAlp = align256(kStGam + sizeof(double) * (OMG_NOALLOC_MAX_K + 1));
constexpr size_t kStGram = align256(kStAlp + sizeof(double) * (OMG_NOALLOC_MAX_K + 1));
constexpr size_t kStHist = align256(kStGram + sizeof(double) * (OMG_NOALLOC_MAX_K + 1) * kGramStride);
constexpr size_t kStPtr =
    align256(kStHist + sizeof(double) * ((size_t)(OMG_NOALLOC_MAX_K + 1) * OMG_NOALLOC_MAX_K / 2 + 1));
constexpr size_t kStBytes = align256(kStPtr + sizeof(double*) * (OMG_NOALLOC_MAX_K + 1));
static_assert(kStBytes <= 512 * 1024, "scratch stays modest");
// the kernel's grid (at most kMaxRedBlocks blocks of kThreads threads, at most
// 20 entries each) covers every N up to the limit
static_assert((int64_t)OMG_NOALLOC_MAX_N <= (int64_t)kMaxRedBlocks * kThreads * 20, "grid reach");

// Clear what the step reads before writing it: exchange words to the empty
// tag, the abort flag, the Gram entries of the caller's (orthonormal)
// directions; and the pointer table of the k rows of W.
__global__ void k_noalloc_init(unsigned char* base, const double* W, int64_t N, int k) {
    unsigned long long* words = reinterpret_cast<unsigned long long*>(base + kStWords);
    double* gram = reinterpret_cast<double*>(base + kStGram);
    unsigned* flags = reinterpret_cast<unsigned*>(base + kStFlags);
    double* scal = reinterpret_cast<double*>(base + kStScal);
    const double** ptr = reinterpret_cast<const double**>(base + kStPtr);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)kRmSlotWords; i += stride) {
        words[i] = ~0ull;
        if (i < (int64_t)(k + 1) * kGramStride) gram[i] = 0.0;
        if (i < k) ptr[i] = W + i * N;
        if (i < S_COUNT) scal[i] = 0.0;
        if (i < 2) flags[i] = 0u;
    }
}

} // namespace omg

using namespace omg;

// The scratch array. In host code this name is a host-side stand-in: the
// device address of each GPU's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kStBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

// Device address of this GPU's copy of the scratch array (looked up once
// per device, with that device current).
static omg_status scratch_of_current_device(unsigned char** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return OMG_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OMG_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return OMG_OK;
}

extern "C" omg_status omg_rm_step_noalloc(int64_t N, int32_t k, const double* W, const double* w, const double* z,
                                          const double* r, double breakdown, void* hip_stream, double* Wk,
                                          double* r_new, double* coeff) {
    if (N < 1 || N > OMG_NOALLOC_MAX_N || k < 0 || k > OMG_NOALLOC_MAX_K) return OMG_EINVAL; // beyond the scratch
    if ((k > 0 && !W) || !w || !z || !r || !Wk || !r_new || !coeff || !(breakdown >= 0.0) ||
        !std::isfinite(breakdown))
        return OMG_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    unsigned char* base = nullptr;
    OMG_TRY(scratch_of_current_device(&base));
    RmConfig c;
    if (!rm_masked_config(N, &c)) return OMG_EUNSUPPORTED;
    hipLaunchKernelGGL(k_noalloc_init, dim3(40), dim3(kThreads), 0, st, base, W, N, (int)k);
    OMG_TRY_HIP(hipGetLastError());
    if (r_new != r) OMG_TRY_HIP(launch_copy(r_new, r, N, st)); // the step updates r_new in place
    RmArgs a;
    a.N = N;
    a.k = k;
    a.Wp = reinterpret_cast<const double* const*>(base + kStPtr);
    a.Wk = Wk;
    a.Zk = nullptr; // the raw direction is z itself
    a.w = w;
    a.z = z;
    a.r = r_new;
    a.slots = reinterpret_cast<unsigned long long*>(base + kStWords);
    a.g0 = 0;
    a.part_rn = reinterpret_cast<double*>(base + kStPart);
    a.breakdown = breakdown;
    a.scal = reinterpret_cast<double*>(base + kStScal);
    a.abort_flag = reinterpret_cast<unsigned*>(base + kStFlags) + 1;
    a.hist = reinterpret_cast<double*>(base + kStHist);
    a.gammas = reinterpret_cast<double*>(base + kStGam);
    a.alphas = reinterpret_cast<double*>(base + kStAlp);
    a.gram = reinterpret_cast<double*>(base + kStGram);
    OMG_TRY_HIP(launch_rm_masked(c, a, st));
    unsigned flag = 0;
    if (k > 0)
        OMG_TRY_HIP(hipMemcpyAsync(coeff, a.hist + (size_t)k * (k - 1) / 2, sizeof(double) * k,
                                   hipMemcpyDeviceToHost, st));
    OMG_TRY_HIP(hipMemcpyAsync(coeff + k, a.gammas + k, sizeof(double), hipMemcpyDeviceToHost, st));
    OMG_TRY_HIP(hipMemcpyAsync(coeff + k + 1, a.alphas + k, sizeof(double), hipMemcpyDeviceToHost, st));
    OMG_TRY_HIP(hipMemcpyAsync(&flag, a.abort_flag, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    OMG_TRY_HIP(hipStreamSynchronize(st));
    return flag ? OMG_EHIP : OMG_OK; // an expired bounded wait: results not trustworthy
}
