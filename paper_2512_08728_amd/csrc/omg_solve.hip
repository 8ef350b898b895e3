// OrthoMG solve engine and the C ABI.
//
// Host code drives the level recursion of Algorithm 2 (multiplicative
// synchronous) and of Algorithm 5 in a deterministic form (coarse correction
// from the residual at the start of the cycle, a fixed number of smoother+RM
// steps, then RM of the coarse correction, Sec. 4). All arithmetic runs in
// device kernels; the host reads one residual norm per level iteration for
// the level-local stopping rules of Sec. 4.2.
//
// In the deterministic Algorithm 5 the coarse path of the finest level
// (restriction output -> coarse recursion -> prolongation) runs on a second
// HIP stream while the finest-level smoother and residual minimisation run on
// the caller's stream; the two meet once per cycle (an event) before
// RM(z_cor), which is the paper's single synchronisation per cycle. The coarse
// path works on a private copy of the restricted residual, so the result is
// the same as running both on one stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include <atomic>
#include <map>
#include <tuple>
#include <mutex>
#include <thread>

#include "omg_internal.h"

using namespace omg;

// setup helpers (omg_setup.hip)
omg_status omg_alloc_level_vectors(omg_solver* s, Level& L);
omg_status omg_ingest_bsr(omg_solver* s, const omg_bsr* A, std::vector<unsigned char>& valid);
omg_status omg_assemble_sip(omg_solver* s, const double* nu_dev, std::vector<unsigned char>& valid);
omg_status omg_galerkin(omg_solver* s, int l, const std::vector<unsigned char>& fvalid,
                        std::vector<unsigned char>& cvalid);
omg_status omg_block_inverses(omg_solver* s, Level& L);
omg_status omg_fp32_copies(omg_solver* s, Level& L);
omg_status omg_coarse_factor(omg_solver* s, Level& L);
hipError_t omg_launch_contract(const omg_solver* s, const double* lam, const double* u, double* g_nu,
                               hipStream_t st);

#define HIP_OK(expr)                                   \
    do {                                               \
        if ((expr) != hipSuccess) return OMG_EHIP;     \
    } while (0)

// ------------------------------------------------------------------ options
extern "C" void omg_default_options(omg_options* o) {
    std::memset(o, 0, sizeof(*o));
    o->variant = OMG_SYNC_MULT;
    o->coarse_sync = 0;
    o->s_pre = 1;
    o->s_post = 1;
    o->n_s = 1;
    o->max_iter = 1000;
    o->precision = OMG_FP64;
    o->max_outer = 50;
    o->overlap_streams = 1;
    o->trace = 0;
    o->n_s_max = 0;
    o->smoother = OMG_SMOOTH_BJ;
    o->omega = 0.7;
    o->inner_tol = 1e-5;
    o->breakdown = 1e-14;
    o->crit_rel[0] = 0.1;
    o->crit_max[0] = 20;
    o->crit_rel[1] = 0.5;
    o->crit_max[1] = 2;
    for (int l = 2; l < OMG_MAX_LEVELS; ++l) {
        o->crit_rel[l] = -1.0;
        o->crit_max[l] = 1;
    }
}

extern "C" const char* omg_strerror(omg_status st) {
    switch (st) {
    case OMG_OK: return "ok";
    case OMG_EINVAL: return "invalid argument";
    case OMG_ENOMEM: return "out of memory";
    case OMG_EHIP: return "HIP runtime error";
    case OMG_ENOTSPD: return "matrix not symmetric positive definite";
    case OMG_ENOCONV: return "no convergence within max_iter";
    case OMG_EBREAKDOWN: return "breakdown";
    case OMG_EUNSUPPORTED: return "unsupported for this solver";
    }
    return "unknown status";
}

// ------------------------------------------------------------------ teardown
static void free_level(Level& L) {
    if (!L.shared_op) {
        hipFree(L.col);
        hipFree(L.val);
        hipFree(L.val32);
        hipFree(L.dinv);
        hipFree(L.dinv32);
        hipFree(L.ainv);
        hipFree(L.atile);
        hipFree(L.dslot);
        hipFree(L.ablk);
        hipFree(L.ablk32);
        hipFree(L.mrpart);
        hipFree(L.dblk);
        hipFree(L.as_cells);
        hipFree(L.as_rev);
        hipFree(L.as_inv);
        hipFree(L.as_inv32);
        hipFree(L.as_z);
        hipFree(L.dblk32);
        hipFree(L.up);
        hipFree(L.dn_ptr);
        hipFree(L.dn);
    }
    hipFree(L.b);
    hipFree(L.r);
    hipFree(L.x);
    hipFree(L.z);
    hipFree(L.w);
    hipFree(L.t);
    hipFree(L.t2);
    hipFree(L.zcor);
    hipFree(L.xout);
    hipFree(L.part);
    hipFree(L.scal);
    hipFree(L.spart);
    for (double* c : L.chunks) hipFree(c);
    hipFree(L.dWp);
    hipFree(L.dZp);
    hipFree(L.bar);
    hipFree(L.xslots);
    hipFree(L.hist);
    hipFree(L.alphas);
    hipFree(L.gammas);
    hipFree(L.gram);
    hipFree(L.dvec);
    hipFree(L.rs);
    hipFree(L.xs);
    L = Level();
}

extern "C" void omg_destroy(omg_solver* s) {
    if (!s) return;
    if (s->stream) hipStreamSynchronize(s->stream);
    for (omg_solver* c : s->columns) omg_destroy(c);
    s->columns.clear();
    if (s->bnorm_host) hipHostFree(s->bnorm_host);
    for (auto* t : s->btab) hipFree(t);
    hipFree(s->babort);
    if (s->owner) { // column solver: E, E32 belong to the owner
        s->E = nullptr;
        s->E32 = nullptr;
    }
    if (s->cstream) {
        hipStreamSynchronize(s->cstream);
        hipStreamDestroy(s->cstream);
    }
    if (s->ev_fork) hipEventDestroy(s->ev_fork);
    if (s->ev_join) hipEventDestroy(s->ev_join);
    for (hipEvent_t e : s->ev_step)
        if (e) hipEventDestroy(e);
    for (auto& L : s->lev) free_level(L);
    hipFree(s->E);
    hipFree(s->E32);
    hipFree(s->nu);
    hipFree(s->refm);
    hipFree(s->bufA);
    hipFree(s->bufB);
    hipFree(s->err_flag);
    if (s->host_scal) hipHostFree(s->host_scal);
    if (s->vlog_host) hipHostFree(s->vlog_host);
    for (hipEvent_t e : s->vlog_ev)
        if (e) hipEventDestroy(e);
    delete s;
}

// ------------------------------------------------------------------ setup
// Small host-visible scalars the kernels write directly (mapped, coherent).
static omg_status alloc_host_scalars(omg_solver* s) {
    const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc((void**)&s->host_scal, sizeof(double) * 4 * OMG_MAX_LEVELS, fl) != hipSuccess ||
        hipHostMalloc((void**)&s->bnorm_host, sizeof(double) * kMaxCols, fl) != hipSuccess)
        return OMG_ENOMEM;
    if (hipHostGetDevicePointer((void**)&s->host_scal_dev, s->host_scal, 0) != hipSuccess ||
        hipHostGetDevicePointer((void**)&s->bnorm_dev, s->bnorm_host, 0) != hipSuccess)
        return OMG_EHIP;
    return OMG_OK;
}

static omg_status check_grid(const omg_grid* g) {
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || g->p < 0 || g->p > 3 || g->n_levels < 1 ||
        g->n_levels > OMG_MAX_LEVELS)
        return OMG_EINVAL;
    for (int l = 1; l < g->n_levels; ++l) {
        const int f = 1 << (l - 1);
        if ((g->nx / f) % 2 || (g->ny / f) % 2 || (g->nz / f) % 2 || g->nx % (2 * f) || g->ny % (2 * f) ||
            g->nz % (2 * f))
            return OMG_EINVAL;
    }
    return OMG_OK;
}

static omg_status check_options(const omg_options* o) {
    if (!o) return OMG_OK;
    if (o->variant < OMG_SYNC_MULT || o->variant > OMG_ADD_SYNC || o->precision < OMG_FP64 ||
        o->precision > OMG_MIXED_FLEX || o->n_s < 1 || o->n_s_max < 0 || o->s_pre < 0 || o->s_post < 0 ||
        o->smoother < OMG_SMOOTH_BJ || o->smoother > OMG_SMOOTH_AS || o->m_max < 0)
        return OMG_EINVAL;
    return OMG_OK;
}

// Degree of the total-degree basis with bs functions (the block sizes the
// kernels are built for), -1 otherwise.
static int degree_of(int bs) {
    switch (bs) {
    case 1: return 0;
    case 4: return 1;
    case 10: return 2;
    case 20: return 3;
    }
    return -1;
}

static omg_status check_hierarchy(const omg_hierarchy* H, int n0) {
    if (!H || H->n_levels < 1 || H->n_levels > OMG_MAX_LEVELS || !H->n_cells || H->n_cells[0] != n0)
        return OMG_EINVAL;
    for (int l = 0; l < H->n_levels; ++l)
        if (H->n_cells[l] < 1) return OMG_EINVAL;
    if (H->n_levels > 1 && (!H->parent || !H->slot)) return OMG_EINVAL;
    for (int l = 0; l + 1 < H->n_levels; ++l)
        if (!H->parent[l] || !H->slot[l]) return OMG_EINVAL;
    return OMG_OK;
}

// Solver shell: level sizes from the hierarchy, streams, events, host
// scalars, layout buffers. The maps and the embedding come next.
static omg_status create(int nlev, const int32_t* n_cells, int bs, const omg_options* opt, void* stream,
                         omg_solver** out) {
    *out = nullptr;
    OMG_TRY(check_options(opt));
    const int p = degree_of(bs);
    if (p < 0) return OMG_EUNSUPPORTED;
    omg_solver* s = new omg_solver();
    *out = s;
    if (opt) s->opt = *opt;
    else omg_default_options(&s->opt);
    std::memset(&s->grid, 0, sizeof(s->grid));
    s->p = p;
    s->bs = bs;
    s->bsh = (s->bs + 1) / 2;
    s->nlev = nlev;
    s->stream = (hipStream_t)stream;
    s->lev.resize(s->nlev);
    const char* rs = std::getenv("OMG_ROWSPLIT_MAX_CELLS");
    for (int l = 0; l < s->nlev; ++l) {
        Level& L = s->lev[l];
        L.n = n_cells[l];
        L.N = (int64_t)L.n * s->bs;
        L.coarsest = (l == s->nlev - 1);
        L.G = reduction_blocks(L.N);
        // few cells: split block rows over threads so the launch covers the GPU
        L.rowsplit = s->bs <= 16 && L.n <= (rs ? std::atoi(rs) : 65536); // 64*bs threads per smoother block
    }
    if (hipMalloc((void**)&s->err_flag, sizeof(int)) != hipSuccess) return OMG_ENOMEM;
    OMG_TRY(alloc_host_scalars(s));
    const size_t vb = sizeof(double) * (size_t)s->lev[0].N;
    if (hipMalloc((void**)&s->bufA, vb) != hipSuccess) return OMG_ENOMEM;
    if (hipMalloc((void**)&s->bufB, vb) != hipSuccess) return OMG_ENOMEM;
    HIP_OK(hipStreamCreateWithFlags(&s->cstream, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&s->ev_step[0], hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&s->ev_step[1], hipEventDisableTiming));
    return OMG_OK;
}

omg_status omg_upload_maps(omg_solver* s, int l, const int32_t* parent, const uint8_t* slot);

// Embedding blocks (host [8][bs][bs]) and the agglomeration maps of every level.
static omg_status set_hierarchy(omg_solver* s, const omg_hierarchy* H, const double* E) {
    const size_t ne = (size_t)8 * s->bs * s->bs;
    for (size_t t = 0; t < ne; ++t)
        if (!std::isfinite(E[t])) return OMG_EINVAL;
    s->hE.assign(E, E + ne);
    std::vector<float> E32(E, E + ne);
    if (hipMalloc((void**)&s->E, sizeof(double) * ne) != hipSuccess) return OMG_ENOMEM;
    if (hipMalloc((void**)&s->E32, sizeof(float) * ne) != hipSuccess) return OMG_ENOMEM;
    HIP_OK(hipMemcpy(s->E, E, sizeof(double) * ne, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(s->E32, E32.data(), sizeof(float) * ne, hipMemcpyHostToDevice));
    for (int l = 0; l + 1 < s->nlev; ++l) OMG_TRY(omg_upload_maps(s, l, H->parent[l], H->slot[l]));
    return OMG_OK;
}

// The 2x2x2 agglomeration of a Cartesian grid, as host arrays owned here.
struct GridHierarchy {
    std::vector<int32_t> n_cells;
    std::vector<std::vector<int32_t>> parent;
    std::vector<std::vector<uint8_t>> slot;
    std::vector<const int32_t*> pp;
    std::vector<const uint8_t*> sp;
    std::vector<double> E;
    omg_hierarchy H;
};

static omg_status grid_maps(const omg_grid* g, int level, int32_t* parent, uint8_t* slot) {
    const int nx = g->nx >> level, ny = g->ny >> level, nz = g->nz >> level;
    const int cx = nx / 2, cy = ny / 2;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int K = i + nx * (j + ny * k);
                parent[K] = (i >> 1) + cx * ((j >> 1) + cy * (k >> 1));
                slot[K] = (uint8_t)((i & 1) + 2 * (j & 1) + 4 * (k & 1));
            }
    return OMG_OK;
}

static omg_status make_grid_hierarchy(const omg_grid* g, GridHierarchy& G) {
    OMG_TRY(check_grid(g));
    const int nl = g->n_levels;
    G.n_cells.resize(nl);
    G.parent.resize(nl > 1 ? nl - 1 : 0);
    G.slot.resize(nl > 1 ? nl - 1 : 0);
    for (int l = 0; l < nl; ++l) G.n_cells[l] = (g->nx >> l) * (g->ny >> l) * (g->nz >> l);
    for (int l = 0; l + 1 < nl; ++l) {
        G.parent[l].resize(G.n_cells[l]);
        G.slot[l].resize(G.n_cells[l]);
        OMG_TRY(grid_maps(g, l, G.parent[l].data(), G.slot[l].data()));
        G.pp.push_back(G.parent[l].data());
        G.sp.push_back(G.slot[l].data());
    }
    embedding_blocks(g->p, G.E);
    G.H.n_levels = nl;
    G.H.pad = 0;
    G.H.n_cells = G.n_cells.data();
    G.H.parent = G.pp.empty() ? nullptr : G.pp.data();
    G.H.slot = G.sp.empty() ? nullptr : G.sp.data();
    G.H.embed = G.E.data();
    return OMG_OK;
}

extern "C" omg_status omg_grid_hierarchy(const omg_grid* g, int32_t level, int32_t* parent, uint8_t* slot) {
    OMG_TRY(check_grid(g));
    if (level < 0 || level >= g->n_levels - 1 || !parent || !slot) return OMG_EINVAL;
    return grid_maps(g, level, parent, slot);
}

extern "C" omg_status omg_embedding(int32_t p, double* E) {
    if (p < 0 || p > 3 || !E) return OMG_EINVAL;
    std::vector<double> v;
    embedding_blocks(p, v);
    std::memcpy(E, v.data(), sizeof(double) * v.size());
    return OMG_OK;
}

// Storage of the persistent RM kernel on one level: exchange words, abort
// flag, MGS coefficient history (sized for the level's iteration cap).
static omg_status alloc_rm_state(omg_solver* s, Level& L, int l) {
    const int per_it = std::max(3, std::max(s->opt.n_s, s->opt.n_s_max) + 1); // RMs per level iteration
    const int its = (l == 0) ? s->opt.max_iter : s->opt.crit_max[l - 1];
    L.ucap = per_it * std::max(its, 1) + 4;
    if (hipMalloc((void**)&L.bar, 2 * sizeof(unsigned)) != hipSuccess) return OMG_ENOMEM;
    HIP_OK(hipMemset(L.bar, 0, 2 * sizeof(unsigned)));
    const size_t xs = sizeof(unsigned long long) * kRmSlotWordsMax;
    if (hipMalloc((void**)&L.xslots, xs) != hipSuccess) return OMG_ENOMEM;
    HIP_OK(hipMemset(L.xslots, 0xFF, xs)); // every word starts with tag 3 = empty
    L.phase = 0;
    const size_t uc = (size_t)L.ucap;
    if (hipMalloc((void**)&L.hist, sizeof(double) * (uc * (uc - 1) / 2 + 1)) != hipSuccess ||
        hipMalloc((void**)&L.alphas, sizeof(double) * uc) != hipSuccess ||
        hipMalloc((void**)&L.gammas, sizeof(double) * uc) != hipSuccess ||
        hipMalloc((void**)&L.dvec, sizeof(double) * uc) != hipSuccess ||
        hipMalloc((void**)&L.gram, sizeof(double) * uc * kGramStride) != hipSuccess)
        return OMG_ENOMEM;
    HIP_OK(hipMemset(L.gram, 0, sizeof(double) * uc * kGramStride));
    return OMG_OK;
}

static omg_status ensure_dir(omg_solver* s, Level& L, int k);

// Launch configuration of the persistent RM kernel on level l: time every
// co-resident configuration (entries per thread, MGS block, exchange form,
// grid) with kt stored directions, half the level's capacity (at most 256:
// the exchange latency and the streaming share depend on k), zero data (the
// traffic and exchanges do not depend on the values), best of two trials,
// and keep the fastest. The directions' storage is the level's own; the
// solve overwrites everything these launches write.
//
// The configuration sets the order of the kernel's partial sums, so it is
// chosen once per (device, level size) for the whole process: every solver
// of that size then runs the same arithmetic, and results do not depend on
// which solver was timed.
static std::mutex g_rm_mu;
// keyed by (device, level size, stored directions the tuner times with): a
// level of the same size deep in one hierarchy (a few directions per visit)
// and finest in another (hundreds) need not share a configuration
static std::map<std::tuple<int, int64_t, int>, RmConfig> g_rm_cache;

// Tuning record file (JSON lines, path in the environment variable
// OMG_RM_TUNE_FILE): one line per (device architecture, compute units, level
// size, stored directions timed with) with the configuration the tuner chose
// and its time. A level with a record uses that configuration (if it is
// still co-resident) without timing, so that every process on that device
// kind runs the same arithmetic; a newly tuned level is appended.
struct TuneRecord {
    std::string arch;
    int cus = 0;
    int64_t N = 0;
    int k = 0;
    RmConfig c;
};
static std::vector<TuneRecord> g_tune_file;
static bool g_tune_loaded = false;

static const char* tune_path() { return std::getenv("OMG_RM_TUNE_FILE"); }

static void device_kind(int dev, std::string& arch, int& cus) {
    hipDeviceProp_t p;
    arch = "?";
    cus = 0;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return;
    arch = p.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    cus = p.multiProcessorCount;
}

static void tune_file_load() { // under g_rm_mu
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = tune_path();
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char arch[64];
        TuneRecord r;
        long long n = 0;
        if (std::sscanf(line,
                        " {\"arch\": \"%63[^\"]\", \"cus\": %d, \"N\": %lld, \"k\": %d, \"G\": %d, \"ept\": %d, "
                        "\"B\": %d, \"lead\": %d, \"cw\": %d, \"lag\": %d",
                        arch, &r.cus, &n, &r.k, &r.c.G, &r.c.ept, &r.c.B, &r.c.lead, &r.c.cw, &r.c.lag) == 10) {
            r.arch = arch;
            r.N = n;
            g_tune_file.push_back(r);
        }
    }
    std::fclose(f);
}

static void tune_file_append(const std::string& arch, int cus, int64_t N, int k, const RmConfig& c, double us) {
    const char* path = tune_path();
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"arch\": \"%s\", \"cus\": %d, \"N\": %lld, \"k\": %d, \"G\": %d, \"ept\": %d, \"B\": %d, "
                 "\"lead\": %d, \"cw\": %d, \"lag\": %d, \"us\": %.1f}\n",
                 arch.c_str(), cus, (long long)N, k, c.G, c.ept, c.B, c.lead, c.cw, c.lag, us);
    std::fclose(f);
    g_tune_file.push_back(TuneRecord{arch, cus, N, k, c});
}

static omg_status tune_rm(omg_solver* s, int l) {
    Level& L = s->lev[l];
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    // the tuner times RM with kt stored directions: half the level's
    // direction capacity, at most 256
    const int kt = std::max(1, std::min((L.ucap - 1) / 2, 256));
    const std::tuple<int, int64_t, int> key(dev, L.N, kt);
    std::string arch;
    int cus = 0;
    device_kind(dev, arch, cus);
    RmConfig c[kMaxRmConfigs];
    const int nc = rm_persistent_candidates(L.N, c, kMaxRmConfigs);
    {
        std::lock_guard<std::mutex> lk(g_rm_mu);
        auto it = g_rm_cache.find(key);
        if (it != g_rm_cache.end()) {
            L.rmc = it->second;
            return OMG_OK;
        }
        tune_file_load();
        for (const TuneRecord& r : g_tune_file) {
            if (r.arch != arch || r.cus != cus || r.N != L.N || r.k != kt) continue;
            for (int q = 0; q < nc; ++q)
                if (c[q].G == r.c.G && c[q].ept == r.c.ept && c[q].B == r.c.B && c[q].lead == r.c.lead &&
                    c[q].cw == r.c.cw && c[q].lag == r.c.lag) {
                    L.rmc = c[q];
                    g_rm_cache.emplace(key, c[q]);
                    return OMG_OK;
                }
        }
    }
    if (nc <= 1 || std::getenv("OMG_RM_NOTUNE")) {
        std::lock_guard<std::mutex> lk(g_rm_mu);
        g_rm_cache.emplace(key, L.rmc);
        return OMG_OK;
    }
    OMG_TRY(ensure_dir(s, L, kt));
    if ((int)L.W.size() <= kt || (int)L.dcap <= kt) return OMG_EINVAL;
    hipStream_t st = s->stream;
    for (int i = 0; i <= kt; ++i) HIP_OK(launch_fill(L.W[i], 0.0, L.N, st));
    HIP_OK(launch_fill(L.w, 0.0, L.N, st));
    HIP_OK(launch_fill(L.z, 0.0, L.N, st));
    HIP_OK(launch_fill(L.r, 0.0, L.N, st));
    RmArgs a;
    a.N = L.N;
    a.k = kt;
    a.Wp = L.dWp;
    a.Wk = L.W[kt];
    a.Zk = L.Z[kt];
    a.w = L.w;
    a.z = L.z;
    a.r = L.r;
    a.slots = L.xslots;
    a.part_rn = L.part + 4 * kMaxRedBlocks;
    a.breakdown = s->opt.breakdown;
    a.scal = L.scal;
    a.abort_flag = L.bar + 1;
    a.hist = L.hist;
    a.gammas = L.gammas;
    a.alphas = L.alphas;
    a.gram = L.gram;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    float best = 1e30f;
    int bi = 0;
    omg_status res = OMG_OK;
    const bool log = std::getenv("OMG_RM_TUNE_LOG") != nullptr;
    for (int q = 0; q < nc && res == OMG_OK; ++q) {
        float tbest = 1e30f;
        for (int trial = 0; trial < 2 && res == OMG_OK; ++trial) {
            const int reps = 3;
            for (int r = 0; r <= reps && res == OMG_OK; ++r) {
                if (r == 1 && hipEventRecord(e0, st) != hipSuccess) res = OMG_EHIP;
                a.g0 = L.phase;
                if (res == OMG_OK && prepare_slots(L, c[q], st) != hipSuccess) res = OMG_EHIP;
                if (res == OMG_OK && launch_rm_persistent(c[q], a, st) != hipSuccess) res = OMG_EHIP;
                L.phase += rm_phases(kt, c[q].B);
            }
            float ms = 0.f;
            if (res == OMG_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                res = OMG_EHIP;
            tbest = std::min(tbest, ms);
        }
        if (res == OMG_OK) { // a configuration whose bounded waits expired is not used
            unsigned flags[2] = {0, 0};
            if (hipMemcpy(flags, L.bar, sizeof(flags), hipMemcpyDeviceToHost) != hipSuccess) res = OMG_EHIP;
            if (res == OMG_OK && flags[1]) {
                if (log) std::fprintf(stderr, "[omg] RM tuning: configuration %d aborted\n", q);
                L.rm_dropped++;
                tbest = 1e30f;
                L.slot_G = 0; // words in unknown state: reset before the next launch
                if (hipMemset(L.bar + 1, 0, sizeof(unsigned)) != hipSuccess) res = OMG_EHIP;
            }
        }
        if (log)
            std::fprintf(stderr, "[omg] RM tuning N=%lld k=%d: G=%d ept=%d B=%d lead=%d cw=%d lag=%d: %.1f us\n",
                         (long long)L.N, kt, c[q].G, c[q].ept, c[q].B, c[q].lead, c[q].cw, c[q].lag,
                         1e3 * tbest / 3);
        if (res == OMG_OK && tbest < best) {
            best = tbest;
            bi = q;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    OMG_TRY(res);
    unsigned flags[2] = {0, 0};
    HIP_OK(hipMemcpy(flags, L.bar, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags[1]) return OMG_EHIP; // a bounded wait expired
    std::lock_guard<std::mutex> lk(g_rm_mu);
    auto ins = g_rm_cache.emplace(key, c[bi]); // first tuner of this size wins
    if (ins.second) tune_file_append(arch, cus, L.N, kt, c[bi], 1e3 * best / 3);
    L.rmc = ins.first->second;
    return OMG_OK;
}

static omg_status build_hierarchy(omg_solver* s, std::vector<unsigned char>& valid0) {
    std::vector<unsigned char> fvalid = valid0, cvalid;
    for (int l = 0; l + 1 < s->nlev; ++l) {
        OMG_TRY(omg_galerkin(s, l, fvalid, cvalid));
        fvalid.swap(cvalid);
    }
    for (int l = 0; l < s->nlev; ++l) {
        Level& L = s->lev[l];
        OMG_TRY(omg_alloc_level_vectors(s, L));
        if (!L.coarsest) {
            OMG_TRY(omg_block_inverses(s, L));
            if (s->opt.smoother == OMG_SMOOTH_AS) OMG_TRY(as_setup(s, L));
            OMG_TRY(omg_fp32_copies(s, L));
            // the persistent RM runs on the caller's stream only: levels below
            // the forking level (second stream) keep the per-step kernels
            const int fl = cycle_fork_level(s->opt);
            const bool eligible = !std::getenv("OMG_NO_PERSISTENT_RM") && !(fl >= 0 && l > fl);
            if (eligible) L.persist = rm_persistent_config(L.N, &L.rmc);
            if (L.persist) {
                OMG_TRY(alloc_rm_state(s, L, l));
                OMG_TRY(tune_rm(s, l));
            }
        } else {
            OMG_TRY(omg_coarse_factor(s, L));
        }
    }
    HIP_OK(hipStreamSynchronize(s->stream));
    return OMG_OK;
}

extern "C" omg_status omg_setup(const omg_bsr* A, const omg_hierarchy* H, const omg_options* opt,
                                void* hip_stream, omg_solver** out) {
    if (!out) return OMG_EINVAL;
    *out = nullptr;
    if (!A || !A->row_ptr || !A->col_idx || !A->val || !H || !H->embed) return OMG_EINVAL;
    const int n = A->n_cells, bs = A->bs;
    if (n < 1 || bs < 1) return OMG_EINVAL;
    OMG_TRY(check_hierarchy(H, n));
    if (A->row_ptr[0] != 0 || A->row_ptr[n] != A->nnzb) return OMG_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (A->row_ptr[i + 1] < A->row_ptr[i]) return OMG_EINVAL;
        bool diag = false;
        for (int64_t q = A->row_ptr[i]; q < A->row_ptr[i + 1]; ++q) {
            const int c = A->col_idx[q];
            if (c < 0 || c >= n) return OMG_EINVAL;
            if (q > A->row_ptr[i] && c <= A->col_idx[q - 1]) return OMG_EINVAL;
            if (c == i) diag = true;
        }
        if (!diag) return OMG_EINVAL;
    }
    for (int64_t t = 0; t < A->nnzb * bs * bs; ++t)
        if (!std::isfinite(A->val[t])) return OMG_EINVAL;
    omg_solver* s = nullptr;
    omg_status st = create(H->n_levels, H->n_cells, bs, opt, hip_stream, &s);
    if (st == OMG_OK) st = set_hierarchy(s, H, H->embed);
    std::vector<unsigned char> valid;
    if (st == OMG_OK) st = omg_ingest_bsr(s, A, valid);
    if (st == OMG_OK) st = build_hierarchy(s, valid);
    if (st != OMG_OK) {
        omg_destroy(s);
        return st;
    }
    *out = s;
    return OMG_OK;
}

extern "C" omg_status omg_setup_sip(const omg_grid* grid, const double* nu, const omg_hierarchy* H,
                                    const omg_options* opt, void* hip_stream, omg_solver** out) {
    if (!out) return OMG_EINVAL;
    *out = nullptr;
    if (!grid || !nu || !(grid->h > 0) || !std::isfinite(grid->penalty_c) || grid->nx < 1 || grid->ny < 1 ||
        grid->nz < 1 || grid->p < 0 || grid->p > 3)
        return OMG_EINVAL;
    const int n = grid->nx * grid->ny * grid->nz;
    GridHierarchy GH;
    std::vector<double> E;
    if (!H) {
        OMG_TRY(make_grid_hierarchy(grid, GH));
        H = &GH.H;
    } else {
        OMG_TRY(check_hierarchy(H, n));
    }
    const double* Eh = H->embed;
    if (!Eh) {
        embedding_blocks(grid->p, E);
        Eh = E.data();
    }
    const int bs = (grid->p + 1) * (grid->p + 2) * (grid->p + 3) / 6;
    omg_solver* s = nullptr;
    omg_status st = create(H->n_levels, H->n_cells, bs, opt, hip_stream, &s);
    if (st == OMG_OK) {
        s->grid = *grid;
        s->grid.n_levels = H->n_levels;
        Level& L0 = s->lev[0];
        L0.nx = grid->nx;
        L0.ny = grid->ny;
        L0.nz = grid->nz;
        st = set_hierarchy(s, H, Eh);
    }
    if (st == OMG_OK) {
        // nu must be positive and finite
        std::vector<double> hnu(n);
        if (hipMemcpy(hnu.data(), nu, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) st = OMG_EHIP;
        for (int i = 0; st == OMG_OK && i < n; ++i)
            if (!(hnu[i] > 0.0) || !std::isfinite(hnu[i])) st = OMG_EINVAL;
    }
    std::vector<unsigned char> valid;
    if (st == OMG_OK) st = omg_assemble_sip(s, nu, valid);
    if (st == OMG_OK) {
        s->has_sip = 1;
        st = build_hierarchy(s, valid);
    }
    if (st != OMG_OK) {
        if (s) omg_destroy(s);
        return st;
    }
    *out = s;
    return OMG_OK;
}

// ------------------------------------------------------------------ solve
static inline bool use32(const omg_solver* s, int l, bool is_rm) {
    if (s->mode32 == 1) return true;
    if (s->mode32 == 2) return !(l == 0 && is_rm);
    return false;
}

// Kernel probe: bracket one launch with a pair of events when armed.
static void probe_begin(omg_solver* s, int kind, int l, hipStream_t st) {
    if (s->probe_kind != kind || s->probe_level != l || s->probe_n >= s->probe_max) return;
    const size_t i = 2 * (size_t)s->probe_n;
    while (s->probe_ev.size() < i + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        s->probe_ev.push_back(e);
    }
    hipEventRecord(s->probe_ev[i], st);
}
static void probe_end(omg_solver* s, int kind, int l, hipStream_t st, double bytes) {
    if (s->probe_kind != kind || s->probe_level != l || s->probe_n >= s->probe_max) return;
    const size_t i = 2 * (size_t)s->probe_n;
    if (s->probe_ev.size() < i + 2) return;
    hipEventRecord(s->probe_ev[i + 1], st);
    s->probe_n++;
    s->probe_bytes += bytes;
}

// Algorithmic bytes of one launch: operator values and column indices of the
// stored blocks, block-diagonal inverses, and every vector read or written once.
static double alg_bytes(const omg_solver* s, int kind, int l, int k) {
    const Level& L = s->lev[l];
    const double N = (double)L.N, nnzb = (double)s->nnzb_level[l], bb = (double)s->bs * s->bs;
    switch (kind) {
    case OMG_K_SPMV: return nnzb * bb * 8 + nnzb * 4 + 2 * N * 8;
    case OMG_K_SPMV32: return nnzb * bb * 4 + nnzb * 4 + 2 * N * 8;
    case OMG_K_BJ: return nnzb * bb * 8 + nnzb * 4 + L.n * bb * 8 + 3 * N * 8;
    case OMG_K_BJ32: return nnzb * bb * 4 + nnzb * 4 + L.n * bb * 4 + 3 * N * 8;
    case OMG_K_BJFIRST: return L.n * bb * 8 + 2 * N * 8;
    case OMG_K_MGS: return 2 * N * 8;                 // W_i and Z_i; w and z stay resident
    case OMG_K_RMP: return (k + 6.0) * N * 8; // W_i (i < k), w, z~ in, W_k, Z~_k out, r in/out
    case OMG_K_RMFIN: return 8 * N * 8;
    case OMG_K_COARSE: return N * N * 8 + 2 * N * 8;
    }
    return 0.0;
}

// Make room for direction index k on level l (chunks of 32 directions).
static omg_status ensure_dir(omg_solver* s, Level& L, int k) {
    if (k < 0) return OMG_EINVAL;
    if (k < (int)L.W.size()) return OMG_OK;
    const int chunk = 32;
    const size_t vn = (size_t)(L.N + kVecPad); // with the zero tail
    while (k >= (int)L.W.size()) { // as many chunks as index k needs
        double* mem = nullptr;
        if (hipMalloc((void**)&mem, sizeof(double) * vn * 2 * chunk) != hipSuccess) {
            (void)hipGetLastError();
            return OMG_ENOMEM;
        }
        // zero tails; finished before any stream (the overlap form's coarse
        // stream included) can use the chunk
        HIP_OK(hipMemsetAsync(mem, 0, sizeof(double) * vn * 2 * chunk, s->stream));
        HIP_OK(hipStreamSynchronize(s->stream));
        L.chunks.push_back(mem);
        for (int c = 0; c < chunk; ++c) {
            L.W.push_back(mem + vn * (2 * c));
            L.Z.push_back(mem + vn * (2 * c + 1));
        }
    }
    // device copies of the pointer arrays (read by the persistent RM kernel)
    double **dW = nullptr, **dZ = nullptr;
    if (hipMalloc((void**)&dW, sizeof(double*) * L.W.size()) != hipSuccess ||
        hipMalloc((void**)&dZ, sizeof(double*) * L.Z.size()) != hipSuccess) {
        (void)hipGetLastError();
        return OMG_ENOMEM;
    }
    HIP_OK(hipMemcpy(dW, L.W.data(), sizeof(double*) * L.W.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dZ, L.Z.data(), sizeof(double*) * L.Z.size(), hipMemcpyHostToDevice));
    HIP_OK(hipFree(L.dWp)); // hipFree waits for work that may still read the old arrays
    HIP_OK(hipFree(L.dZp));
    L.dWp = dW;
    L.dZp = dZ;
    L.dcap = L.W.size();
    return OMG_OK;
}

// Residual minimisation (Algorithm 1) on level l with the direction z
// (overwritten): w = A z, MGS against W with the same coefficients on z,
// normalise, append, alpha = w.r, x += alpha z, r -= alpha w. Leaves the
// partials of ||r||^2 in part slot 4 (L.Grn of them).
static omg_status rm_apply(omg_solver* s, int l, double* z, hipStream_t st);
// Restart of a level solve that holds m_max directions (bounded storage;
// the paper sets no limit): x0 = x, r0 = r, W = Z = {}. On a level with
// implicit directions the share of x carried by the dropped directions is
// formed now and accumulated in L.x (zero since level entry), which the
// level's result adds at the end; elsewhere x is explicit already.
static omg_status restart_level(omg_solver* s, int l, hipStream_t st) {
    Level& L = s->lev[l];
    if (L.persist && L.k > 0) {
        HIP_OK(launch_recon(L.k, L.hist, L.gammas, L.alphas, L.dvec, st));
        HIP_OK(launch_lincomb(L.N, L.k, L.dvec, L.dZp, L.t2, st));
        HIP_OK(launch_axpy(L.x, 1.0, L.t2, L.N, st));
        L.restarted = 1;
    }
    L.k = 0;
    return OMG_OK;
}

static omg_status rm(omg_solver* s, int l, double* z, hipStream_t st) {
    Level& L = s->lev[l];
    if (s->opt.m_max > 0 && L.k >= s->opt.m_max) OMG_TRY(restart_level(s, l, st));
    const int kspmv = use32(s, l, true) ? OMG_K_SPMV32 : OMG_K_SPMV;
    probe_begin(s, kspmv, l, st);
    HIP_OK(launch_spmv(L, s->bs, use32(s, l, true), z, nullptr, L.w, st));
    probe_end(s, kspmv, l, st, alg_bytes(s, kspmv, l, 0));
    s->kcount[kspmv][l]++;
    return rm_apply(s, l, z, st);
}

// The part of RM after w = A z (w in L.w).
static omg_status rm_apply(omg_solver* s, int l, double* z, hipStream_t st) {
    Level& L = s->lev[l];
    const int G = L.G;
    const int64_t N = L.N;
    OMG_TRY(ensure_dir(s, L, L.k));
    double* P_nin = L.part;
    double* P_a = L.part + kMaxRedBlocks;
    double* P_b = L.part + 2 * kMaxRedBlocks;
    double* P_alpha = L.part + 3 * kMaxRedBlocks;
    double* P_rn = L.part + 4 * kMaxRedBlocks;
    if (L.persist) {
        if (L.k + 1 > L.ucap) return OMG_ENOMEM;
        RmArgs a;
        a.N = L.N;
        a.k = L.k;
        a.Wp = L.dWp;
        a.Wk = L.W[L.k];
        a.Zk = L.Z[L.k];
        a.w = L.w;
        a.z = z;
        a.r = L.r;
        a.slots = L.xslots;
        a.g0 = L.phase;
        a.part_rn = P_rn;
        a.breakdown = s->opt.breakdown;
        a.scal = L.scal;
        a.abort_flag = L.bar + 1;
        a.hist = L.hist;
        a.gammas = L.gammas;
        a.alphas = L.alphas;
        a.gram = L.gram;
        probe_begin(s, OMG_K_RMP, l, st);
        HIP_OK(prepare_slots(L, L.rmc, st));
        HIP_OK(launch_rm_persistent(L.rmc, a, st));
        probe_end(s, OMG_K_RMP, l, st, alg_bytes(s, OMG_K_RMP, l, L.k));
        L.phase += rm_phases(L.k, L.rmc.B);
        s->kcount[OMG_K_RMP][l]++;
        L.Grn = L.rmc.G;
        L.k++;
        return OMG_OK;
    }
    s->kcount[OMG_K_MGS][l] += L.k;
    s->kcount[OMG_K_RMFIN][l]++;
    const double* P_nout = P_nin;
    if (L.k == 0) {
        HIP_OK(launch_dot2(N, G, nullptr, nullptr, nullptr, L.w, P_nin, st));
    } else {
        HIP_OK(launch_dot2(N, G, L.W[0], L.w, P_a, L.w, P_nin, st));
        for (int i = 0; i < L.k; ++i) {
            double* pin = (i & 1) ? P_b : P_a;
            double* pout = (i & 1) ? P_a : P_b;
            const double* next = (i + 1 < L.k) ? L.W[i + 1] : nullptr;
            probe_begin(s, OMG_K_MGS, l, st);
            HIP_OK(launch_mgs_step(N, G, pin, L.W[i], L.Z[i], L.w, z, next, pout, st));
            probe_end(s, OMG_K_MGS, l, st, alg_bytes(s, OMG_K_MGS, l, 0));
            P_nout = pout;
        }
    }
    HIP_OK(launch_rm_normalize(N, G, P_nin, P_nout, s->opt.breakdown, L.w, z, L.W[L.k], L.Z[L.k], L.r, P_alpha,
                               L.scal, st));
    HIP_OK(launch_rm_update(N, G, P_alpha, L.W[L.k], L.Z[L.k], L.x, L.r, P_rn, st));
    L.Grn = G;
    L.k++;
    return OMG_OK;
}

// Read ||r|| of level l (from the partials of the last update) to the host.
// The finishing kernel writes straight into mapped, coherent pinned host
// memory, so the read costs one kernel and one wait (no copy command).
static omg_status read_rnorm(omg_solver* s, int l, hipStream_t st, double* out) {
    Level& L = s->lev[l];
    HIP_OK(launch_finish_norm(L.Grn, L.part + 4 * kMaxRedBlocks, s->host_scal_dev + l, st));
    HIP_OK(hipStreamSynchronize(st));
    *out = s->host_scal[l];
    return OMG_OK;
}

static omg_status vec_norm(omg_solver* s, int l, const double* v, hipStream_t st, double* out) {
    Level& L = s->lev[l];
    HIP_OK(launch_dot2(L.N, L.G, nullptr, nullptr, nullptr, v, L.part + 4 * kMaxRedBlocks, st));
    L.Grn = L.G;
    return read_rnorm(s, l, st, out);
}

// Block-Jacobi smoother (Algorithm 4) from x0 = 0 with `sweeps` iterations;
// result in out (ping-pong through t).
static omg_status smoother(omg_solver* s, int l, const double* r, int sweeps, double* out, hipStream_t st) {
    Level& L = s->lev[l];
    const bool f32 = use32(s, l, false);
    if (sweeps < 1) sweeps = 1;
    if (s->opt.smoother == OMG_SMOOTH_AS) { // additive Schwarz (Algorithm 3), damped sweeps from zero
        HIP_OK(launch_as_sweep(L, s->bs, f32, s->opt.omega, r, out, false, st));
        for (int it = 1; it < sweeps; ++it) {
            HIP_OK(launch_spmv(L, s->bs, f32, out, r, L.t, st)); // t = r - A x
            HIP_OK(launch_as_sweep(L, s->bs, f32, s->opt.omega, L.t, out, true, st));
        }
        return OMG_OK;
    }
    // place the last sweep's output in `out`
    double* bufs[2] = {out, L.t};
    int cur = (sweeps % 2 == 1) ? 0 : 1;
    HIP_OK(launch_bj_first(L, s->bs, f32, s->opt.omega, r, bufs[cur], st));
    s->kcount[OMG_K_BJFIRST][l]++;
    s->kcount[f32 ? OMG_K_BJ32 : OMG_K_BJ][l] += sweeps - 1;
    const int kbj = f32 ? OMG_K_BJ32 : OMG_K_BJ;
    for (int it = 1; it < sweeps; ++it) {
        probe_begin(s, kbj, l, st);
        HIP_OK(launch_bj_sweep(L, s->bs, f32, s->opt.omega, r, bufs[cur], bufs[cur ^ 1], st));
        probe_end(s, kbj, l, st, alg_bytes(s, kbj, l, 0));
        cur ^= 1;
    }
    return OMG_OK;
}

static void log_trace(omg_solver* s, double rn, int type) {
    s->trace.push_back(Trace{(double)s->step, rn, (double)type});
}

static omg_status trace_rm(omg_solver* s, int l, hipStream_t st, int type) {
    if (l != 0 || !s->opt.trace) return OMG_OK;
    double rn;
    OMG_TRY(read_rnorm(s, l, st, &rn));
    s->step++;
    log_trace(s, rn, type);
    return OMG_OK;
}


static bool stop_level(const omg_solver* s, int l, double rn, double r0n, double bn, int it, double tol,
                       int replay_count) {
    if (!std::isfinite(rn)) return true;
    if (replay_count >= 0) return it >= replay_count;
    if (l == 0) return (rn <= tol * bn) || it >= s->opt.max_iter;
    const int idx = l - 1;
    const double rel = s->opt.crit_rel[idx];
    if (rel >= 0.0 && rn <= rel * r0n) return true;
    return it >= s->opt.crit_max[idx];
}

static omg_status mg(omg_solver* s, int l, const double* b, double* xout, double tol, int variant, hipStream_t st);

// z = P_l MG_{l+1}(P_l^T r, 0): the coarse-grid correction of level l.
static omg_status coarse_path(omg_solver* s, int l, int variant, hipStream_t st, double* z) {
    Level& F = s->lev[l];
    Level& C = s->lev[l + 1];
    OMG_TRY(mg(s, l + 1, C.b, C.xout, 0.0, variant, st));
    HIP_OK(launch_prolong(F, C, s->bs, use32(s, l, false), s->E, s->E32, C.xout, z, st));
    s->kcount[OMG_K_PROLONG][l]++;
    s->kcount[OMG_K_RESTRICT][l]++;
    return OMG_OK;
}

// Timing-adaptive cycle of the forking level (adaptive loops, Sec. 4.3;
// Algorithm 5). The coarse group (coarse recursion on the restricted
// residual, prolongation into zcor; second stream) is driven by a host thread
// of its own, because the coarse recursion waits for one residual norm per
// coarse iteration. Meanwhile the smoother group keeps issuing smoothing +
// RM steps on the caller's stream until the coarse group has signalled that
// its correction is complete on the device: at least n_s steps, at most
// n_s_max. One step is kept queued ahead of the GPU, and the decision to stop
// is taken when the step before it has finished, so at most one step is
// issued after the signal. The count is returned in *steps.
static omg_status adaptive_cycle(omg_solver* s, int l, int sub_variant, hipStream_t st, int* steps) {
    Level& L = s->lev[l];
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipStreamWaitEvent(s->cstream, s->ev_fork, 0));
    std::atomic<int> done_c{0};
    omg_status cst = OMG_OK;
    std::thread coarse;
    try {
        coarse = std::thread([&]() {
            if (hipSetDevice(dev) != hipSuccess) cst = OMG_EHIP;
            if (cst == OMG_OK) cst = coarse_path(s, l, sub_variant, s->cstream, L.zcor);
            if (cst == OMG_OK && hipEventRecord(s->ev_join, s->cstream) != hipSuccess) cst = OMG_EHIP;
            if (cst == OMG_OK && hipEventSynchronize(s->ev_join) != hipSuccess) cst = OMG_EHIP;
            done_c.store(1, std::memory_order_release);
        });
    } catch (...) {
        return OMG_EHIP; // no thread: nothing was queued on the coarse stream but the wait
    }
    omg_status sst = OMG_OK;
    int t = 0;
    for (;;) {
        sst = smoother(s, l, L.r, s->opt.s_post, L.z, st);
        if (sst == OMG_OK) sst = rm(s, l, L.z, st);
        if (sst == OMG_OK && hipEventRecord(s->ev_step[t & 1], st) != hipSuccess) sst = OMG_EHIP;
        if (sst != OMG_OK) break;
        ++t;
        if (t >= s->opt.n_s_max) break;
        // step t is queued; wait for step t - 1 before deciding on step t + 1
        if (t >= 2 && hipEventSynchronize(s->ev_step[t & 1]) != hipSuccess) {
            sst = OMG_EHIP;
            break;
        }
        if (t >= s->opt.n_s && done_c.load(std::memory_order_acquire)) break;
    }
    coarse.join();
    *steps = t;
    OMG_TRY(sst);
    OMG_TRY(cst);
    HIP_OK(hipStreamWaitEvent(st, s->ev_join, 0));
    return OMG_OK;
}

// ---------------------------------------------------------------- norm log
// Residual norms of the level tests go to consecutive positions of a mapped
// host buffer: norm_async queues the finishing reduction of level l's last
// update (and an event behind it) and returns the position; norm_wait blocks
// until that event and returns the value. Positions past the buffer are
// read at once (the value kept on the host).
constexpr int64_t kVlogCap = 1 << 18;
constexpr int kVlogEvents = 64;

static omg_status vlog_init(omg_solver* s) {
    if (s->vlog_host) return OMG_OK;
    const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc((void**)&s->vlog_host, sizeof(double) * kVlogCap, fl) != hipSuccess) return OMG_ENOMEM;
    HIP_OK(hipHostGetDevicePointer((void**)&s->vlog_dev, s->vlog_host, 0));
    s->vlog_ev.assign(kVlogEvents, nullptr);
    for (auto& e : s->vlog_ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return OMG_OK;
}

static omg_status norm_async(omg_solver* s, int l, hipStream_t st, int64_t* pos) {
    Level& L = s->lev[l];
    const int64_t p = s->vlog_pos++;
    if (p < kVlogCap) {
        HIP_OK(launch_finish_norm(L.Grn, L.part + 4 * kMaxRedBlocks, s->vlog_dev + p, st));
        HIP_OK(hipEventRecord(s->vlog_ev[p % kVlogEvents], st));
    } else { // past the buffer: read now
        double v;
        HIP_OK(launch_finish_norm(L.Grn, L.part + 4 * kMaxRedBlocks, s->host_scal_dev + l, st));
        HIP_OK(hipStreamSynchronize(st));
        v = s->host_scal[l];
        s->vlog_over.push_back(v);
    }
    *pos = p;
    return OMG_OK;
}

static omg_status norm_wait(omg_solver* s, int64_t p, double* out) {
    if (p >= kVlogCap) {
        *out = s->vlog_over[(size_t)(p - kVlogCap)];
        return OMG_OK;
    }
    HIP_OK(hipEventSynchronize(s->vlog_ev[p % kVlogEvents]));
    *out = s->vlog_host[p];
    return OMG_OK;
}

// Per-visit residual log entry whose norms are filled in when the solve ends.
static void log_visit_norms(omg_solver* s, int l, int it, int64_t p0, const std::vector<int64_t>& ps) {
    s->vnorm.push_back(l);
    s->vnorm.push_back(it);
    s->vfix.push_back({s->vnorm.size(), p0});
    s->vnorm.push_back(0.0);
    for (int64_t p : ps) {
        s->vfix.push_back({s->vnorm.size(), p});
        s->vnorm.push_back(0.0);
    }
}

static omg_status vlog_resolve(omg_solver* s) {
    HIP_OK(hipStreamSynchronize(s->stream));
    for (auto& f : s->vfix) {
        double v;
        OMG_TRY(norm_wait(s, f.second, &v));
        if (f.first < s->vnorm.size()) s->vnorm[f.first] = v;
    }
    s->vfix.clear();
    return OMG_OK;
}

// Snapshot of a level before a speculative iteration: r, x (where it holds
// anything besides the implicit directions), the dropped-direction counter,
// the direction count and the logs' lengths. The stored directions below
// that count are not touched by the iteration (it only appends), so the
// count restores them.
struct Snap {
    int k = 0, restarted = 0;
    size_t visits = 0, vnorm = 0, vfix = 0, steps = 0;
};

static omg_status snap_take(omg_solver* s, int l, hipStream_t st, Snap& sp) {
    Level& L = s->lev[l];
    if (!L.rs && (hipMalloc((void**)&L.rs, sizeof(double) * L.N) != hipSuccess ||
                  hipMalloc((void**)&L.xs, sizeof(double) * L.N) != hipSuccess))
        return OMG_ENOMEM;
    const int64_t nx = (!L.persist || s->opt.m_max > 0) ? L.N : 0; // persistent: x is zero unless restarted
    HIP_OK(launch_snap(L.rs, L.r, L.N, L.xs, L.x, nx, L.scal + S_TMP, L.scal + S_BREAKDOWNS, st));
    sp.k = L.k;
    sp.restarted = L.restarted;
    sp.visits = s->visits.size();
    sp.vnorm = s->vnorm.size();
    sp.vfix = s->vfix.size();
    sp.steps = s->steps.size();
    return OMG_OK;
}

static omg_status snap_restore(omg_solver* s, int l, hipStream_t st, const Snap& sp) {
    Level& L = s->lev[l];
    const int64_t nx = (!L.persist || s->opt.m_max > 0) ? L.N : 0;
    HIP_OK(launch_snap(L.r, L.rs, L.N, L.x, L.xs, nx, L.scal + S_BREAKDOWNS, L.scal + S_TMP, st));
    L.k = sp.k;
    L.restarted = sp.restarted;
    s->visits.resize(sp.visits);
    s->vnorm.resize(sp.vnorm);
    s->vfix.resize(sp.vfix);
    s->steps.resize(sp.steps);
    return OMG_OK;
}

// One iteration of level l's cycle (Algorithm 2, or the deterministic /
// timing-adaptive Algorithm 5 form), x and r updated in place.
static omg_status level_iteration(omg_solver* s, int l, int variant, int sub_variant, hipStream_t st) {
    Level& L = s->lev[l];
    Level& C = s->lev[l + 1];
    if (cycle_multiplicative(variant)) {
        OMG_TRY(smoother(s, l, L.r, s->opt.s_pre, L.z, st));
        OMG_TRY(rm(s, l, L.z, st));
        OMG_TRY(trace_rm(s, l, st, 1));
        HIP_OK(launch_restrict(L, C, s->bs, use32(s, l, false), s->E, s->E32, L.r, C.b, st));
        OMG_TRY(coarse_path(s, l, sub_variant, st, L.z));
        OMG_TRY(rm(s, l, L.z, st));
        OMG_TRY(trace_rm(s, l, st, 2));
        OMG_TRY(smoother(s, l, L.r, s->opt.s_post, L.z, st));
        OMG_TRY(rm(s, l, L.z, st));
        OMG_TRY(trace_rm(s, l, st, 1));
        return OMG_OK;
    }
    // coarse group: restriction of the residual at the start of the cycle
    HIP_OK(launch_restrict(L, C, s->bs, use32(s, l, false), s->E, s->E32, L.r, C.b, st));
    const bool forking = (l == cycle_fork_level(s->opt));
    const bool fork = forking && s->opt.overlap_streams && !s->opt.trace;
    if (fork && s->opt.n_s_max > s->opt.n_s) {
        HIP_OK(hipEventRecord(s->ev_fork, st));
        int steps = 0;
        OMG_TRY(adaptive_cycle(s, l, sub_variant, st, &steps));
        s->steps.push_back(steps);
    } else if (fork) {
        s->steps.push_back(s->opt.n_s);
        HIP_OK(hipEventRecord(s->ev_fork, st));
        // smoother group: queue the fine work first (asynchronous)
        for (int t = 0; t < s->opt.n_s; ++t) {
            OMG_TRY(smoother(s, l, L.r, s->opt.s_post, L.z, st));
            OMG_TRY(rm(s, l, L.z, st));
        }
        HIP_OK(hipStreamWaitEvent(s->cstream, s->ev_fork, 0));
        OMG_TRY(coarse_path(s, l, sub_variant, s->cstream, L.zcor));
        HIP_OK(hipEventRecord(s->ev_join, s->cstream));
        HIP_OK(hipStreamWaitEvent(st, s->ev_join, 0));
    } else {
        if (forking) s->steps.push_back(s->opt.n_s);
        OMG_TRY(coarse_path(s, l, sub_variant, st, L.zcor));
        for (int t = 0; t < s->opt.n_s; ++t) {
            OMG_TRY(smoother(s, l, L.r, s->opt.s_post, L.z, st));
            OMG_TRY(rm(s, l, L.z, st));
            OMG_TRY(trace_rm(s, l, st, 1));
        }
    }
    OMG_TRY(rm(s, l, L.zcor, st));
    OMG_TRY(trace_rm(s, l, st, 2));
    return OMG_OK;
}

// (x, r) = MG_l(b, 0): the level loop of Algorithm 2 / 5 with the level tests
// of Sec. 4.2. On a coarse level (l >= 1) the next iteration is queued before
// the norm that decides on it has been read (speculation): the host then
// waits while the GPU already works on that iteration, and if the test says
// stop, the iteration is undone exactly (r, x, direction count, logs and the
// dropped-direction counter restored from a snapshot), so the results are
// those of the plain loop. A replayed visit (omg_set_replay) reads no norm
// at all while it runs.
static omg_status mg(omg_solver* s, int l, const double* b, double* xout, double tol, int variant, hipStream_t st) {
    Level& L = s->lev[l];
    if (L.coarsest) {
        HIP_OK(launch_gemv(L, b, xout, st));
        s->kcount[OMG_K_COARSE][l]++;
        return OMG_OK;
    }
    L.k = 0;
    L.restarted = 0;
    HIP_OK(launch_level_init(L.N, L.G, b, L.x, L.r, L.part + 4 * kMaxRedBlocks, st));
    L.Grn = L.G;
    int replay_count = -1; // replayed iteration count of this visit (omg_set_replay)
    if (s->replaying && l < (int)s->replay_q.size() && s->replay_pos[l] < s->replay_q[l].size())
        replay_count = s->replay_q[l][s->replay_pos[l]++];
    const int sub_variant = cycle_sub_variant(variant, s->opt.coarse_sync);
    const bool adaptive_here = l == cycle_fork_level(s->opt) && !cycle_multiplicative(variant) &&
                               s->opt.overlap_streams && !s->opt.trace && s->opt.n_s_max > s->opt.n_s;
    // (an m_max restart inside the speculative iteration would overwrite the
    // stored directions the snapshot keeps by count only: no speculation then)
    const bool speculate = l > 0 && !s->opt.trace && !adaptive_here && s->opt.m_max == 0;
    int64_t p0;
    OMG_TRY(norm_async(s, l, st, &p0));
    std::vector<int64_t> ps; // positions of ||r|| after each iteration
    int it = 0;
    double r0n = 0.0, rn = 0.0;
    omg_status status = OMG_OK;
    if (l == 0) { // ||b|| of the finest level: one read per solve
        OMG_TRY(norm_wait(s, p0, &r0n));
        log_trace(s, r0n, 0);
    }
    if (replay_count >= 0) {
        for (; it < replay_count; ++it) {
            OMG_TRY(level_iteration(s, l, variant, sub_variant, st));
            int64_t p;
            OMG_TRY(norm_async(s, l, st, &p));
            ps.push_back(p);
        }
    } else if (!speculate) {
        OMG_TRY(norm_wait(s, p0, &r0n));
        rn = r0n;
        while (!stop_level(s, l, rn, r0n, r0n, it, tol, -1)) {
            OMG_TRY(level_iteration(s, l, variant, sub_variant, st));
            it++;
            int64_t p;
            OMG_TRY(norm_async(s, l, st, &p));
            ps.push_back(p);
            OMG_TRY(norm_wait(s, p, &rn));
            if (!std::isfinite(rn)) {
                status = OMG_EINVAL;
                break;
            }
        }
    } else {
        const int cap = s->opt.crit_max[l - 1];
        int64_t pq = p0; // position of the norm after iteration `it`
        for (;;) {
            const bool ahead = it + 1 <= cap; // stop_level stops at the cap whatever the norm
            Snap sp;
            int64_t pn = -1;
            if (ahead) {
                OMG_TRY(snap_take(s, l, st, sp));
                OMG_TRY(level_iteration(s, l, variant, sub_variant, st));
                OMG_TRY(norm_async(s, l, st, &pn));
            }
            OMG_TRY(norm_wait(s, pq, &rn));
            if (it == 0) r0n = rn;
            const bool bad = !std::isfinite(rn);
            if (bad || stop_level(s, l, rn, r0n, r0n, it, tol, -1)) {
                if (ahead) OMG_TRY(snap_restore(s, l, st, sp));
                if (bad && it > 0) status = OMG_EINVAL;
                break;
            }
            it++;
            ps.push_back(pn);
            pq = pn;
        }
    }
    if (l == 0 && status == OMG_OK && rn > tol * r0n && replay_count < 0) status = OMG_ENOCONV;
    s->visits.push_back(l);
    s->visits.push_back(it);
    log_visit_norms(s, l, it, p0, ps);
    if (L.persist) { // x = sum_k d_k z~_k: the search directions are implicit
        HIP_OK(launch_recon(L.k, L.hist, L.gammas, L.alphas, L.dvec, st));
        HIP_OK(launch_lincomb(L.N, L.k, L.dvec, L.dZp, xout, st));
        if (L.restarted) HIP_OK(launch_axpy(xout, 1.0, L.x, L.N, st)); // directions dropped at restarts
    }
    else
        HIP_OK(launch_copy(xout, L.x, L.N, st));
    return status;
}

static omg_status solve_soa(omg_solver* s, const double* b, double* x, double tol, omg_report* R) {
    Level& L = s->lev[0];
    hipStream_t st = s->stream;
    double* rr = L.t2;   // outer residual
    double* e = L.xout;  // correction
    double bn;
    OMG_TRY(vec_norm(s, 0, b, st, &bn));
    if (!std::isfinite(bn)) return OMG_EINVAL;
    if (bn == 0.0) {
        HIP_OK(launch_fill(x, 0.0, L.N, st));
        return OMG_OK;
    }
    if (L.coarsest) { // one level: direct solve
        HIP_OK(launch_spmv(L, s->bs, false, x, b, rr, st));
        HIP_OK(launch_gemv(L, rr, e, st));
        HIP_OK(launch_axpy(x, 1.0, e, L.N, st));
        return OMG_OK;
    }
    omg_status status = OMG_OK;
    if (s->opt.precision == OMG_MIXED_IR) {
        int outer = 0;
        for (;;) {
            HIP_OK(launch_spmv(L, s->bs, false, x, b, rr, st));
            double rn;
            OMG_TRY(vec_norm(s, 0, rr, st, &rn));
            R->rel_res_rec = rn / bn;
            if (!std::isfinite(rn)) {
                status = OMG_EINVAL;
                break;
            }
            if (rn <= tol * bn) break;
            if (outer >= s->opt.max_outer) {
                status = OMG_ENOCONV;
                break;
            }
            s->mode32 = 1;
            omg_status st2 = mg(s, 0, rr, e, s->opt.inner_tol, s->opt.variant, st);
            s->mode32 = 0;
            R->iters_fine += s->visits.back();
            if (st2 == OMG_EINVAL || st2 == OMG_EHIP || st2 == OMG_ENOMEM) {
                status = st2;
                break;
            }
            HIP_OK(launch_axpy(x, 1.0, e, L.N, st));
            outer++;
        }
        R->outer_iters = outer;
    } else {
        HIP_OK(launch_spmv(L, s->bs, false, x, b, rr, st));
        double rn;
        OMG_TRY(vec_norm(s, 0, rr, st, &rn));
        if (!std::isfinite(rn)) return OMG_EINVAL;
        s->mode32 = (s->opt.precision == OMG_MIXED_FLEX) ? 2 : 0;
        if (rn > 0.0) {
            status = mg(s, 0, rr, e, tol * bn / rn, s->opt.variant, st);
            s->mode32 = 0;
            HIP_OK(launch_axpy(x, 1.0, e, L.N, st));
            R->iters_fine = s->visits.back();
            double rrec;
            OMG_TRY(vec_norm(s, 0, L.r, st, &rrec));
            R->rel_res_rec = rrec / bn;
            log_trace(s, rrec, 3);
        }
        s->mode32 = 0;
    }
    return status;
}

static omg_status finish_report(omg_solver* s, const double* b, const double* x, omg_report* R) {
    Level& L = s->lev[0];
    hipStream_t st = s->stream;
    double bn, rn;
    OMG_TRY(vec_norm(s, 0, b, st, &bn));
    HIP_OK(launch_spmv(L, s->bs, false, x, b, L.t2, st));
    OMG_TRY(vec_norm(s, 0, L.t2, st, &rn));
    R->rel_res_true = bn > 0 ? rn / bn : 0.0;
    R->n_dirs_fine = L.coarsest ? 0 : L.k;
    double nb = 0;
    for (auto& Lv : s->lev)
        if (!Lv.coarsest) {
            double v;
            HIP_OK(hipMemcpyAsync(&v, Lv.scal + S_BREAKDOWNS, sizeof(double), hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            nb += v;
        }
    R->n_breakdowns = (int)nb;
    for (auto& Lv : s->lev)
        if (Lv.bar) {
            unsigned flags[2];
            HIP_OK(hipMemcpyAsync(flags, Lv.bar, sizeof(flags), hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            if (flags[1]) { // a grid barrier timed out: results are not trustworthy
                Lv.persist = 0;
                return OMG_EHIP;
            }
        }
    R->n_visits = (int)s->visits.size() / 2;
    R->n_trace = (int)s->trace.size();
    return OMG_OK;
}

static void reset_logs(omg_solver* s) {
    s->visits.clear();
    s->vnorm.clear();
    s->steps.clear();
    s->trace.clear();
    s->step = 0;
    for (auto& L : s->lev)
        if (L.scal) hipMemsetAsync(L.scal, 0, sizeof(double) * S_COUNT, s->stream);
}

// A raised abort flag on a persistent level means a bounded wait of one of
// its RM launches expired (a block was not resident in time): the results of
// the solve are not trustworthy. The flag is cleared and the level's exchange
// words are reset before its next launch.
static omg_status check_rm_abort(omg_solver* s) {
    HIP_OK(hipStreamSynchronize(s->stream));
    omg_status st = OMG_OK;
    for (Level& L : s->lev) {
        if (!L.persist || !L.bar) continue;
        unsigned f = 0;
        HIP_OK(hipMemcpy(&f, L.bar + 1, sizeof(unsigned), hipMemcpyDeviceToHost));
        if (f) {
            if (std::getenv("OMG_RM_TUNE_LOG"))
                std::fprintf(stderr, "[omg] level %d: a bounded wait of the persistent RM expired\n",
                             (int)(&L - s->lev.data()));
            HIP_OK(hipMemset(L.bar + 1, 0, sizeof(unsigned)));
            L.slot_G = -1;
            st = OMG_EHIP;
        }
    }
    return st;
}

static omg_status solve_internal(omg_solver* s, const double* b_soa, double* x_soa, double tol, omg_report* R) {
    reset_logs(s);
    OMG_TRY(vlog_init(s));
    s->vlog_pos = 0;
    s->vlog_over.clear();
    s->vfix.clear();
    s->replay_q.assign(s->nlev, {});
    s->replay_pos.assign(s->nlev, 0);
    s->replaying = !s->replay.empty();
    for (size_t i = 0; i + 1 < s->replay.size(); i += 2)
        if (s->replay[i] >= 0 && s->replay[i] < s->nlev) s->replay_q[s->replay[i]].push_back(s->replay[i + 1]);
    omg_status st = solve_soa(s, b_soa, x_soa, tol, R);
    s->replaying = 0;
    const omg_status lg = vlog_resolve(s);
    if (lg != OMG_OK && st == OMG_OK) st = lg;
    const omg_status ab = check_rm_abort(s);
    return ab != OMG_OK ? ab : st;
}

extern "C" omg_status omg_solve(omg_solver* s, const double* b, double* x, double tol, double* r_out,
                                omg_report* rep) {
    if (!s || !b || !x || !(tol >= 0.0)) return OMG_EINVAL;
    auto t0 = std::chrono::steady_clock::now();
    omg_report R;
    std::memset(&R, 0, sizeof(R));
    Level& L = s->lev[0];
    hipStream_t st = s->stream;
    HIP_OK(launch_to_soa(b, s->bufA, L.n, s->bs, st));
    HIP_OK(launch_to_soa(x, s->bufB, L.n, s->bs, st));
    omg_status status = solve_internal(s, s->bufA, s->bufB, tol, &R);
    if (status == OMG_OK || status == OMG_ENOCONV) {
        HIP_OK(launch_from_soa(s->bufB, x, L.n, s->bs, st));
        if (r_out && !L.coarsest) HIP_OK(launch_from_soa(L.r, r_out, L.n, s->bs, st));
        OMG_TRY(finish_report(s, s->bufA, s->bufB, &R));
    }
    HIP_OK(hipStreamSynchronize(st));
    R.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    R.status = status;
    if (rep) *rep = R;
    return status;
}

// ------------------------------------------------------------------ engine
// entry points shared with the batched driver
namespace omg {
bool engine_use32(const omg_solver* s, int l, bool is_rm) { return use32(s, l, is_rm); }
bool engine_stop_level(const omg_solver* s, int l, double rn, double r0n, int it, double tol) {
    return stop_level(s, l, rn, r0n, r0n, it, tol, -1);
}
omg_status engine_rm_apply(omg_solver* s, int l, double* z, hipStream_t st) { return rm_apply(s, l, z, st); }
omg_status engine_finish_report(omg_solver* s, const double* b, const double* x, omg_report* R) {
    return finish_report(s, b, x, R);
}
omg_status engine_ensure_dir(omg_solver* s, int l) {
    Level& L = s->lev[l];
    OMG_TRY(ensure_dir(s, L, L.k));
    if (L.persist && L.k + 1 > L.ucap) return OMG_ENOMEM;
    return OMG_OK;
}
void engine_reset_logs(omg_solver* s) { reset_logs(s); }

// A column solver: the owner's operator arrays (shared, not copied), its own
// work vectors, search directions and persistent-RM state on every level.
omg_status engine_make_column(omg_solver* o, omg_solver** out) {
    omg_solver* s = new omg_solver();
    *out = s;
    s->owner = o;
    s->opt = o->opt;
    s->grid = o->grid;
    s->bs = o->bs;
    s->bsh = o->bsh;
    s->p = o->p;
    s->nlev = o->nlev;
    s->stream = o->stream;
    s->E = o->E;
    s->E32 = o->E32;
    for (int l = 0; l < OMG_MAX_LEVELS; ++l) s->nnzb_level[l] = o->nnzb_level[l];
    s->lev.resize(s->nlev);
    for (int l = 0; l < s->nlev; ++l) {
        const Level& P = o->lev[l];
        Level& L = s->lev[l];
        L.nx = P.nx;
        L.ny = P.ny;
        L.nz = P.nz;
        L.n = P.n;
        L.N = P.N;
        L.width = P.width;
        L.coarsest = P.coarsest;
        L.rowsplit = P.rowsplit;
        L.G = P.G;
        L.shared_op = 1;
        L.col = P.col;
        L.val = P.val;
        L.val32 = P.val32;
        L.dinv = P.dinv;
        L.dinv32 = P.dinv32;
        L.ainv = P.ainv;
        L.np = P.np;
        L.atile = P.atile;
        L.ntile = P.ntile;
        if (L.atile && hipMalloc((void**)&L.spart, sizeof(double) * (size_t)L.ntile * L.ntile * 64) != hipSuccess)
            return OMG_ENOMEM;
        L.dslot = P.dslot;
        L.up = P.up;
        L.dn_ptr = P.dn_ptr;
        L.dn = P.dn;
        L.ablk = P.ablk;
        L.ablk32 = P.ablk32;
        L.dblk = P.dblk;
        L.dblk32 = P.dblk32;
        OMG_TRY(omg_alloc_level_vectors(s, L));
        if (!L.coarsest && P.persist) {
            L.persist = 1;
            L.rmc = P.rmc;
            OMG_TRY(alloc_rm_state(s, L, l));
        }
    }
    const size_t vb = sizeof(double) * (size_t)s->lev[0].N;
    if (hipMalloc((void**)&s->bufA, vb) != hipSuccess) return OMG_ENOMEM;
    if (hipMalloc((void**)&s->bufB, vb) != hipSuccess) return OMG_ENOMEM;
    OMG_TRY(alloc_host_scalars(s));
    HIP_OK(hipStreamSynchronize(s->stream));
    return OMG_OK;
}
} // namespace omg

extern "C" omg_status omg_solve_backward(omg_solver* s, const double* u, const double* g_u, double* g_f,
                                         double* g_nu, double tol, omg_report* rep) {
    if (!s || !u || !g_u) return OMG_EINVAL;
    if (g_nu && !s->has_sip) return OMG_EUNSUPPORTED;
    Level& L = s->lev[0];
    double* lam = nullptr;
    if (hipMalloc((void**)&lam, sizeof(double) * L.N) != hipSuccess) return OMG_ENOMEM;
    omg_status st = OMG_OK;
    if (launch_fill(lam, 0.0, L.N, s->stream) != hipSuccess) st = OMG_EHIP;
    if (st == OMG_OK) st = omg_solve(s, g_u, lam, tol, nullptr, rep); // adjoint: A symmetric
    // gradients only from a converged adjoint
    if (st == OMG_OK && g_f &&
        hipMemcpyAsync(g_f, lam, sizeof(double) * L.N, hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
        st = OMG_EHIP;
    if (st == OMG_OK && g_nu && omg_launch_contract(s, lam, u, g_nu, s->stream) != hipSuccess) st = OMG_EHIP;
    if (hipStreamSynchronize(s->stream) != hipSuccess && st == OMG_OK) st = OMG_EHIP;
    hipFree(lam);
    return st;
}

// ------------------------------------------------------------------ inspection
// One RM step of level l's persistent kernel on caller data (flat vectors:
// RM has no cell structure): k directions W (rows of a k x N device array,
// orthonormal), w = A z, z, r; configuration cfg[4] = (blocks, entries per
// thread, directions per exchange, leader exchange) or NULL for the tuned
// one. Outputs: Wk (new direction), r_new, and host coeff[k + 2] =
// (beta_0..beta_{k-1}, gamma, alpha).
extern "C" omg_status omg_level_rm_step(omg_solver* s, int32_t level, int32_t k, const double* W, const double* w,
                                        const double* z, const double* r, const int32_t* cfg, double* Wk,
                                        double* r_new, double* coeff) {
    if (!s || level < 0 || level >= s->nlev || k < 0 || !w || !z || !r || !Wk || !r_new || !coeff || (k > 0 && !W))
        return OMG_EINVAL;
    Level& L = s->lev[level];
    if (!L.persist || k + 1 > L.ucap) return OMG_EUNSUPPORTED;
    RmConfig c = L.rmc;
    if (cfg) {
        RmConfig cand[kMaxRmConfigs];
        const int nc = rm_persistent_candidates(L.N, cand, kMaxRmConfigs);
        bool found = false;
        for (int q = 0; q < nc && !found; ++q)
            if (cand[q].G == cfg[0] && cand[q].ept == cfg[1] && cand[q].B == cfg[2] && cand[q].lead == cfg[3] &&
                cand[q].cw == cfg[4] && cand[q].lag == cfg[5]) {
                c = cand[q];
                found = true;
            }
        if (!found) return OMG_EINVAL; // only co-resident configurations are launched
    }
    hipStream_t st = s->stream;
    OMG_TRY(ensure_dir(s, L, k));
    if ((int)L.W.size() <= k) return OMG_EINVAL;
    for (int i = 0; i < k; ++i)
        HIP_OK(hipMemcpyAsync(L.W[i], W + (size_t)i * L.N, sizeof(double) * L.N, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(L.w, w, sizeof(double) * L.N, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(L.z, z, sizeof(double) * L.N, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(L.r, r, sizeof(double) * L.N, hipMemcpyDeviceToDevice, st));
    // the stored intra-block Gram entries of orthonormal directions are zero
    HIP_OK(launch_fill(L.gram, 0.0, (int64_t)L.ucap * kGramStride, st));
    RmArgs a;
    a.N = L.N;
    a.k = k;
    a.Wp = L.dWp;
    a.Wk = L.W[k];
    a.Zk = L.Z[k];
    a.w = L.w;
    a.z = L.z;
    a.r = L.r;
    a.slots = L.xslots;
    a.g0 = L.phase;
    a.part_rn = L.part + 4 * kMaxRedBlocks;
    a.breakdown = s->opt.breakdown;
    a.scal = L.scal;
    a.abort_flag = L.bar + 1;
    a.hist = L.hist;
    a.gammas = L.gammas;
    a.alphas = L.alphas;
    a.gram = L.gram;
    HIP_OK(hipMemsetAsync(L.bar + 1, 0, sizeof(unsigned), st)); // each call starts with the abort flag clear
    HIP_OK(prepare_slots(L, c, st));
    HIP_OK(launch_rm_persistent(c, a, st));
    L.phase += rm_phases(k, c.B);
    HIP_OK(hipMemcpyAsync(Wk, L.W[k], sizeof(double) * L.N, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(r_new, L.r, sizeof(double) * L.N, hipMemcpyDeviceToDevice, st));
    std::vector<double> h((size_t)k + 2);
    if (k > 0) HIP_OK(hipMemcpyAsync(h.data(), L.hist + (size_t)k * (k - 1) / 2, sizeof(double) * k,
                                     hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&h[k], L.gammas + k, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&h[k + 1], L.alphas + k, sizeof(double), hipMemcpyDeviceToHost, st));
    unsigned flags[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(flags, L.bar, sizeof(flags), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (flags[1]) {
        L.slot_G = 0; // words in unknown state: reset before the next launch
        return OMG_EHIP;
    }
    for (int i = 0; i < k + 2; ++i) coeff[i] = h[i];
    return OMG_OK;
}

extern "C" omg_status omg_level_set_rm_config(omg_solver* s, int32_t level, const int32_t* cfg) {
    if (!s || level < 0 || level >= s->nlev || !cfg) return OMG_EINVAL;
    Level& L = s->lev[level];
    if (!L.persist) return OMG_EUNSUPPORTED;
    RmConfig cand[kMaxRmConfigs];
    const int nc = rm_persistent_candidates(L.N, cand, kMaxRmConfigs);
    for (int q = 0; q < nc; ++q)
        if (cand[q].G == cfg[0] && cand[q].ept == cfg[1] && cand[q].B == cfg[2] && cand[q].lead == cfg[3] &&
            cand[q].cw == cfg[4] && cand[q].lag == cfg[5]) {
            L.rmc = cand[q];
            return OMG_OK;
        }
    return OMG_EINVAL;
}

// Co-resident RM launch configurations of level l (host out[6*cap]: blocks,
// entries per thread, directions per exchange, leader, exchange wave, lag);
// count in *n.
extern "C" omg_status omg_level_rm_configs(const omg_solver* s, int32_t level, int32_t* out, int32_t cap,
                                           int32_t* n) {
    if (!s || level < 0 || level >= s->nlev || !n) return OMG_EINVAL;
    const Level& L = s->lev[level];
    RmConfig cand[kMaxRmConfigs];
    const int nc = L.persist ? rm_persistent_candidates(L.N, cand, kMaxRmConfigs) : 0;
    *n = nc;
    for (int q = 0; q < nc && q < cap && out; ++q) {
        out[6 * q] = cand[q].G;
        out[6 * q + 1] = cand[q].ept;
        out[6 * q + 2] = cand[q].B;
        out[6 * q + 3] = cand[q].lead;
        out[6 * q + 4] = cand[q].cw;
        out[6 * q + 5] = cand[q].lag;
    }
    return OMG_OK;
}
extern "C" omg_status omg_level_info(const omg_solver* s, int32_t level, int32_t* n_cells, int32_t* ell_width,
                                     int32_t* k_dirs) {
    if (!s || level < 0 || level >= s->nlev) return OMG_EINVAL;
    const Level& L = s->lev[level];
    if (n_cells) *n_cells = L.n;
    if (ell_width) *ell_width = L.width;
    if (k_dirs) *k_dirs = L.k;
    return OMG_OK;
}

extern "C" omg_status omg_level_matrix(const omg_solver* s, int32_t level, int32_t* row_ptr, int32_t* col_idx,
                                       double* val, int64_t* nnzb) {
    if (!s || level < 0 || level >= s->nlev || !row_ptr || !col_idx || !val) return OMG_EINVAL;
    const Level& L = s->lev[level];
    const int n = L.n, bs = s->bs, bsh = s->bsh;
    std::vector<int> hcol((size_t)L.width * n);
    std::vector<double> hval((size_t)2 * L.width * n * bs * bsh);
    HIP_OK(hipMemcpy(hcol.data(), L.col, sizeof(int) * hcol.size(), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hval.data(), L.val, sizeof(double) * hval.size(), hipMemcpyDeviceToHost));
    std::vector<int> ds(n);
    HIP_OK(hipMemcpy(ds.data(), L.dslot, sizeof(int) * n, hipMemcpyDeviceToHost));
    int64_t q = 0;
    row_ptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        // padding slots point at the cell itself; keep only the recorded diagonal slot among those
        std::vector<std::pair<int, int>> ent;
        for (int j = 0; j < L.width; ++j) {
            const int c = hcol[(size_t)j * n + i];
            if (c == i && j != ds[i]) continue;
            ent.push_back({c, j});
        }
        std::sort(ent.begin(), ent.end());
        for (auto& e : ent) {
            col_idx[q] = e.first;
            for (int r = 0; r < bs; ++r)
                for (int cc = 0; cc < bs; ++cc)
                    val[(size_t)q * bs * bs + r * bs + cc] =
                        hval[((((size_t)e.second * bs + r) * bsh + (cc >> 1)) * n + i) * 2 + (cc & 1)];
            ++q;
        }
        row_ptr[i + 1] = (int)q;
    }
    if (nnzb) *nnzb = q;
    return OMG_OK;
}

// level operations on cell-major vectors (converted through bufA/bufB and t/t2)
extern "C" omg_status omg_level_spmv(omg_solver* s, int32_t level, int32_t fp32, const double* x, const double* b,
                                     double* y) {
    if (!s || level < 0 || level >= s->nlev || !x || !y) return OMG_EINVAL;
    Level& L = s->lev[level];
    if (L.coarsest && level > 0) return OMG_EUNSUPPORTED;
    if (fp32 && !L.val32) return OMG_EUNSUPPORTED;
    hipStream_t st = s->stream;
    double *xs = s->bufA, *bs_ = nullptr, *ys = s->bufB;
    HIP_OK(launch_to_soa(x, xs, L.n, s->bs, st));
    if (b) {
        bs_ = L.coarsest ? nullptr : L.t;
        if (!bs_) return OMG_EUNSUPPORTED;
        HIP_OK(launch_to_soa(b, bs_, L.n, s->bs, st));
    }
    HIP_OK(launch_spmv(L, s->bs, fp32 != 0, xs, bs_, ys, st));
    HIP_OK(launch_from_soa(ys, y, L.n, s->bs, st));
    HIP_OK(hipStreamSynchronize(st));
    return OMG_OK;
}

extern "C" omg_status omg_level_smoother(omg_solver* s, int32_t level, int32_t fp32, const double* r,
                                         int32_t sweeps, double* out) {
    if (!s || level < 0 || level >= s->nlev - 1 || !r || !out || sweeps < 1) return OMG_EINVAL;
    Level& L = s->lev[level];
    if (fp32 && (!L.val32 || !L.dinv32 || (s->opt.smoother == OMG_SMOOTH_AS && !L.as_inv32)))
        return OMG_EUNSUPPORTED;
    hipStream_t st = s->stream;
    HIP_OK(launch_to_soa(r, s->bufA, L.n, s->bs, st));
    const int saved = s->mode32;
    s->mode32 = fp32 ? 1 : 0;
    const omg_status res = smoother(s, level, s->bufA, sweeps, s->bufB, st);
    s->mode32 = saved;
    OMG_TRY(res);
    HIP_OK(launch_from_soa(s->bufB, out, L.n, s->bs, st));
    HIP_OK(hipStreamSynchronize(st));
    return OMG_OK;
}

extern "C" omg_status omg_level_restrict(omg_solver* s, int32_t level, int32_t fp32, const double* r,
                                         double* rc) {
    if (!s || level < 0 || level >= s->nlev - 1 || !r || !rc) return OMG_EINVAL;
    Level& F = s->lev[level];
    Level& C = s->lev[level + 1];
    hipStream_t st = s->stream;
    HIP_OK(launch_to_soa(r, s->bufA, F.n, s->bs, st));
    HIP_OK(launch_restrict(F, C, s->bs, fp32 != 0, s->E, s->E32, s->bufA, s->bufB, st));
    HIP_OK(launch_from_soa(s->bufB, rc, C.n, s->bs, st));
    HIP_OK(hipStreamSynchronize(st));
    return OMG_OK;
}

extern "C" omg_status omg_level_prolong(omg_solver* s, int32_t level, int32_t fp32, const double* zc, double* z) {
    if (!s || level < 0 || level >= s->nlev - 1 || !zc || !z) return OMG_EINVAL;
    Level& F = s->lev[level];
    Level& C = s->lev[level + 1];
    hipStream_t st = s->stream;
    HIP_OK(launch_to_soa(zc, s->bufA, C.n, s->bs, st));
    HIP_OK(launch_prolong(F, C, s->bs, fp32 != 0, s->E, s->E32, s->bufA, s->bufB, st));
    HIP_OK(launch_from_soa(s->bufB, z, F.n, s->bs, st));
    HIP_OK(hipStreamSynchronize(st));
    return OMG_OK;
}

extern "C" omg_status omg_coarse_solve(omg_solver* s, const double* b, double* x) {
    if (!s || !b || !x) return OMG_EINVAL;
    Level& L = s->lev[s->nlev - 1];
    hipStream_t st = s->stream;
    HIP_OK(launch_to_soa(b, s->bufA, L.n, s->bs, st));
    HIP_OK(launch_gemv(L, s->bufA, s->bufB, st));
    HIP_OK(launch_from_soa(s->bufB, x, L.n, s->bs, st));
    HIP_OK(hipStreamSynchronize(st));
    return OMG_OK;
}

extern "C" omg_status omg_get_dirs(const omg_solver* s, int32_t level, double* W, double* Z) {
    if (!s || level < 0 || level >= s->nlev) return OMG_EINVAL;
    const Level& L = s->lev[level];
    const size_t K = (size_t)L.k;
    std::vector<double> U; // persistent levels: z_j = sum_q U[q,j] z~_q, from the coefficient history
    double* dcol = nullptr;
    if (Z && L.persist && K > 0) {
        std::vector<double> hh(K * (K - 1) / 2 + 1), gg(K);
        HIP_OK(hipMemcpy(hh.data(), L.hist, sizeof(double) * hh.size(), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(gg.data(), L.gammas, sizeof(double) * K, hipMemcpyDeviceToHost));
        U.assign(K * K, 0.0); // column j: gamma_j (e_j - sum_{m<j} beta_{j,m} U[:,m])
        for (size_t j = 0; j < K; ++j) {
            for (size_t m = 0; m < j; ++m) {
                const double b = hh[j * (j - 1) / 2 + m];
                for (size_t q = 0; q <= m; ++q) U[q + j * K] -= b * U[q + m * K];
            }
            U[j + j * K] += 1.0;
            for (size_t q = 0; q <= j; ++q) U[q + j * K] *= gg[j];
        }
        HIP_OK(hipMalloc((void**)&dcol, sizeof(double) * K));
    }
    for (size_t i = 0; i < K; ++i) {
        if (W) HIP_OK(launch_from_soa(L.W[i], W + i * L.N, L.n, s->bs, s->stream));
        if (Z && !L.persist) HIP_OK(launch_from_soa(L.Z[i], Z + i * L.N, L.n, s->bs, s->stream));
        if (Z && L.persist) {
            HIP_OK(hipMemcpyAsync(dcol, U.data() + i * K, sizeof(double) * (i + 1), hipMemcpyHostToDevice,
                                  s->stream));
            HIP_OK(launch_lincomb(L.N, (int)i + 1, dcol, L.dZp, s->bufB, s->stream));
            HIP_OK(launch_from_soa(s->bufB, Z + i * L.N, L.n, s->bs, s->stream));
            HIP_OK(hipStreamSynchronize(s->stream));
        }
    }
    HIP_OK(hipStreamSynchronize(s->stream));
    if (dcol) HIP_OK(hipFree(dcol));
    return OMG_OK;
}

extern "C" omg_status omg_get_visits(const omg_solver* s, int32_t* out, int32_t cap, int32_t* n) {
    if (!s || !n) return OMG_EINVAL;
    const int cnt = (int)s->visits.size() / 2;
    *n = cnt;
    if (out)
        for (int i = 0; i < cnt && i < cap; ++i) {
            out[2 * i] = s->visits[2 * i];
            out[2 * i + 1] = s->visits[2 * i + 1];
        }
    return OMG_OK;
}

extern "C" omg_status omg_get_visit_norms(const omg_solver* s, double* out, int32_t cap, int32_t* n) {
    if (!s || !n) return OMG_EINVAL;
    const int cnt = (int)s->vnorm.size();
    *n = cnt;
    if (out)
        for (int i = 0; i < cnt && i < cap; ++i) out[i] = s->vnorm[i];
    return OMG_OK;
}

extern "C" omg_status omg_get_step_counts(const omg_solver* s, int32_t* out, int32_t cap, int32_t* n) {
    if (!s || !n) return OMG_EINVAL;
    const int cnt = (int)s->steps.size();
    *n = cnt;
    if (out)
        for (int i = 0; i < cnt && i < cap; ++i) out[i] = s->steps[i];
    return OMG_OK;
}

extern "C" omg_status omg_get_trace(const omg_solver* s, double* out, int32_t cap, int32_t* n) {
    if (!s || !n) return OMG_EINVAL;
    const int cnt = (int)s->trace.size();
    *n = cnt;
    if (out)
        for (int i = 0; i < cnt && i < cap; ++i) {
            out[3 * i] = s->trace[i].step;
            out[3 * i + 1] = s->trace[i].rnorm;
            out[3 * i + 2] = s->trace[i].type;
        }
    return OMG_OK;
}

extern "C" omg_status omg_set_replay(omg_solver* s, const int32_t* visits, int32_t n) {
    if (!s || n < 0 || (n > 0 && !visits)) return OMG_EINVAL;
    s->replay.assign(visits, visits + 2 * (size_t)n);
    return OMG_OK;
}

// ------------------------------------------------------------------ kernel timing
extern "C" omg_status omg_get_kernel_counts(omg_solver* s, int64_t* out) {
    if (!s || !out) return OMG_EINVAL;
    for (int k = 0; k < OMG_K_COUNT; ++k)
        for (int l = 0; l < OMG_MAX_LEVELS; ++l) {
            out[k * OMG_MAX_LEVELS + l] = s->kcount[k][l];
            s->kcount[k][l] = 0;
        }
    return OMG_OK;
}

extern "C" omg_status omg_bench_kernel(omg_solver* s, int32_t kind, int32_t level, int32_t reps, double* avg_ms,
                                       double* bytes_out) {
    if (!s || level < 0 || level >= s->nlev || reps < 1 || !avg_ms || kind < 0 || kind >= OMG_K_COUNT)
        return OMG_EINVAL;
    Level& L = s->lev[level];
    hipStream_t st = s->stream;
    const int bs = s->bs;
    const double N = (double)L.N, nnzb = (double)s->nnzb_level[level], bb = (double)bs * bs;
    const bool needs_fine = kind != OMG_K_COARSE;
    if (needs_fine && L.coarsest && kind != OMG_K_SPMV && kind != OMG_K_COPY) return OMG_EINVAL;
    if ((kind == OMG_K_RESTRICT || kind == OMG_K_PROLONG) && level + 1 >= s->nlev) return OMG_EINVAL;
    if (kind == OMG_K_COARSE && !L.coarsest) return OMG_EINVAL;
    HIP_OK(launch_fill(L.z, 1.0, L.N, st));
    HIP_OK(launch_fill(L.w, 0.5, L.N, st));
    HIP_OK(launch_fill(L.b, 0.5, L.N, st));
    if (L.r) HIP_OK(launch_fill(L.r, 0.25, L.N, st));
    if (L.x) HIP_OK(launch_fill(L.x, 0.0, L.N, st));
    double bytes = 0.0;
    if (kind == OMG_K_RMFIN) OMG_TRY(ensure_dir(s, L, 0));
    const int kb = 16; // directions used by the persistent RM benchmark
    if (kind == OMG_K_RMP) {
        if (!L.persist || L.ucap < kb + 1) return OMG_EUNSUPPORTED;
        OMG_TRY(ensure_dir(s, L, kb));
        if ((int)L.W.size() <= kb) return OMG_EINVAL;
        for (int i = 0; i <= kb; ++i) {
            HIP_OK(launch_fill(L.W[i], 1.0 / std::sqrt(N), L.N, st));
            HIP_OK(launch_fill(L.Z[i], 0.0, L.N, st));
        }
    }
    if (kind == OMG_K_MGS) {
        OMG_TRY(ensure_dir(s, L, 1));
        HIP_OK(launch_fill(L.W[0], 1.0 / std::sqrt(N), L.N, st));
        HIP_OK(launch_fill(L.Z[0], 0.0, L.N, st));
        HIP_OK(launch_fill(L.W[1], 1.0 / std::sqrt(N), L.N, st));
        HIP_OK(launch_dot2(L.N, L.G, L.W[0], L.w, L.part + kMaxRedBlocks, nullptr, nullptr, st));
    }
    auto launch = [&](int rep) -> hipError_t {
        switch (kind) {
        case OMG_K_SPMV: bytes = nnzb * bb * 8 + nnzb * 4 + 2 * N * 8;
            return launch_spmv(L, bs, false, L.z, nullptr, L.w, st);
        case OMG_K_SPMV32: bytes = nnzb * bb * 4 + nnzb * 4 + 2 * N * 8;
            return launch_spmv(L, bs, true, L.z, nullptr, L.w, st);
        case OMG_K_BJ: bytes = nnzb * bb * 8 + nnzb * 4 + L.n * bb * 8 + 3 * N * 8;
            return launch_bj_sweep(L, bs, false, s->opt.omega, L.r, L.z, L.w, st);
        case OMG_K_BJ32: bytes = nnzb * bb * 4 + nnzb * 4 + L.n * bb * 4 + 3 * N * 8;
            return launch_bj_sweep(L, bs, true, s->opt.omega, L.r, L.z, L.w, st);
        case OMG_K_BJFIRST: bytes = L.n * bb * 8 + 2 * N * 8;
            return launch_bj_first(L, bs, false, s->opt.omega, L.r, L.w, st);
        case OMG_K_MGS: { // w, z stay resident in the method: one read of W_i and Z_i
            bytes = 2 * N * 8;
            double* pin = L.part + ((rep & 1) ? 2 : 1) * kMaxRedBlocks;
            double* pout = L.part + ((rep & 1) ? 1 : 2) * kMaxRedBlocks;
            return launch_mgs_step(L.N, L.G, pin, L.W[0], L.Z[0], L.w, L.z, L.W[1], pout, st);
        }
        case OMG_K_RESTRICT: {
            const Level& C = s->lev[level + 1];
            bytes = (N + (double)C.N) * 8;
            return launch_restrict(L, C, bs, false, s->E, s->E32, L.r, C.b, st);
        }
        case OMG_K_PROLONG: {
            const Level& C = s->lev[level + 1];
            bytes = (N + (double)C.N) * 8;
            return launch_prolong(L, C, bs, false, s->E, s->E32, C.b, L.w, st);
        }
        case OMG_K_COARSE: bytes = N * N * 8 + 2 * N * 8;
            return launch_gemv(L, L.b, L.xout, st);
        case OMG_K_COPY: bytes = 2 * N * 8;
            return launch_stream_copy(L.w, L.z, L.N, st);
        case OMG_K_RMP: {
            bytes = alg_bytes(s, OMG_K_RMP, level, kb);
            RmArgs a;
            a.N = L.N;
            a.k = kb;
            a.Wp = L.dWp;
            a.Wk = L.W[kb];
            a.Zk = L.Z[kb];
            a.w = L.w;
            a.z = L.z;
            a.r = L.r;
            a.slots = L.xslots;
            a.g0 = L.phase;
            a.part_rn = L.part + 4 * kMaxRedBlocks;
            a.breakdown = s->opt.breakdown;
            a.scal = L.scal;
            a.abort_flag = L.bar + 1;
            a.hist = L.hist;
            a.gammas = L.gammas;
            a.alphas = L.alphas;
            a.gram = L.gram;
            hipError_t e = prepare_slots(L, L.rmc, st);
            if (e == hipSuccess) e = launch_rm_persistent(L.rmc, a, st);
            L.phase += rm_phases(kb, L.rmc.B);
            return e;
        }
        }
        return hipErrorInvalidValue;
    };
    HIP_OK(launch(0)); // warm-up
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) HIP_OK(launch(r + 1));
    HIP_OK(hipEventRecord(e1, st));
    HIP_OK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *avg_ms = ms / reps;
    if (bytes_out) *bytes_out = bytes;
    return OMG_OK;
}

extern "C" omg_status omg_probe_kernel(omg_solver* s, int32_t kind, int32_t level, int32_t max_launches) {
    if (!s || kind < 0 || kind >= OMG_K_COUNT || level < 0 || level >= s->nlev || max_launches < 0)
        return OMG_EINVAL;
    s->probe_kind = kind;
    s->probe_level = level;
    s->probe_max = max_launches;
    s->probe_n = 0;
    s->probe_bytes = 0.0;
    return OMG_OK;
}

extern "C" omg_status omg_probe_result(omg_solver* s, int64_t* launches, double* avg_ms, double* alg_bytes_out) {
    if (!s || !launches || !avg_ms) return OMG_EINVAL;
    double tot = 0.0;
    for (int64_t i = 0; i < s->probe_n; ++i) {
        HIP_OK(hipEventSynchronize(s->probe_ev[2 * i + 1]));
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, s->probe_ev[2 * i], s->probe_ev[2 * i + 1]));
        tot += ms;
    }
    *launches = s->probe_n;
    *avg_ms = s->probe_n ? tot / s->probe_n : 0.0;
    if (alg_bytes_out) *alg_bytes_out = s->probe_n ? s->probe_bytes / s->probe_n : 0.0;
    for (hipEvent_t e : s->probe_ev) hipEventDestroy(e);
    s->probe_ev.clear();
    s->probe_kind = -1;
    s->probe_n = 0;
    return OMG_OK;
}
