// Internal declarations of the MI355X OrthoMG library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/omg.h"
#include "../../include/omg_inspect.h"

namespace omg {

// Threads per block of every streaming kernel, and the fixed grid of the
// deterministic two-stage reductions (partials are always summed in the same
// order, so a result does not depend on timing).
constexpr int kThreads = 256;
// Every level work vector and stored direction has kVecPad zero entries past
// N: the persistent RM kernel covers G * kThreads * EPT >= N entries with
// EPT <= 20 and reads and writes all of them without masks.
constexpr int64_t kVecPad = 32 * kThreads;
constexpr int kMaxRedBlocks = 1024;
// largest number of stored directions per grid-wide exchange in the
// persistent RM kernel; the lagged form keeps up to kRmLagMax exchanges in
// flight. Every stored direction j keeps its dots with the directions just
// before it: gram[j * kGramStride + d - 1] = W_j . W_{j-d}, d = 1 ..
// kGramStride (the lagged form with 4 directions per exchange and two
// exchanges in flight needs 4 * 2 + 3 of them).
constexpr int kRmBlock = 4;
constexpr int kRmLagMax = 2;
constexpr int kGramStride = kRmBlock * kRmLagMax + kRmBlock - 1;
// right-hand sides advanced together by the batched solve (two 16-wide
// matrix-core tiles), and the pointers of their vectors passed by value
constexpr int kMaxCols = 32;
struct ColPtrs {
    double* p[kMaxCols];
};
struct NormPack {
    const double* part[kMaxCols];
    int G[kMaxCols];
};
// Independent operators (instances) advanced together by one grouped launch
// per operation; segment q covers blocks [blk0[q], blk0[q+1]).
constexpr int kMaxSeg = 16;
struct SegTable {
    int count;
    int blk0[kMaxSeg + 1];
    int n[kMaxSeg], width[kMaxSeg];
    const int* col[kMaxSeg];
    const void* val[kMaxSeg];          // pair layout of the level (FP64 or FP32 copy)
    const void* dinv[kMaxSeg];
    const double* x[kMaxSeg];
    const double* b[kMaxSeg];
    double* y[kMaxSeg];
};

// Device-resident scalars of one level (indices into Level::scal).
enum Scal : int {
    S_RNORM = 0,      // ||r|| after the last update
    S_BREAKDOWNS = 1, // directions dropped by RM on this level
    S_TMP = 2,
    S_COUNT = 8
};

// Launch configuration of the persistent RM kernel on one level.
struct RmConfig {
    int G = 0;    // blocks (all co-resident)
    int ept = 0;  // vector entries per thread
    int B = 1;    // MGS directions resolved per grid exchange
    int lead = 0; // exchange form: 0 all-to-all, 1 leader block
    int cw = 0;   // compute waves per block of the exchange-wave form (0: plain form)
    int lag = 0;  // lagged form: exchanges in flight (1, 2; 0: not lagged)
};
// Exchange phases of one launch with k stored directions: one per MGS block of
// B directions, then the final one (every form).
// Words per block of a configuration's exchanges and its slot sets.
inline int rm_slot_words(const RmConfig& c) {
    if (!c.lag) return c.B + 1;
    const int held = c.B == 1 ? c.lag : c.lag + 1; // as the lagged kernel's final exchange
    return 2 + held * c.B > c.B + 1 ? 2 + held * c.B : c.B + 1;
}
inline int rm_slot_sets(const RmConfig& c) { return c.lag == 2 ? 8 : c.lag == 1 ? 4 : 2; }
// Grid exchanges (phases) of one persistent RM launch with k stored
// directions: one per MGS block of B directions, then one for the norm of
// the orthogonalised vector, its dot product with r and its Gram entries.
inline unsigned long long rm_phases(int k, int B) { return (unsigned long long)((k + B - 1) / B) + 1; }

// Cycle schedule per level under the configurations of Table 1. A level runs
// the multiplicative cycle of Algorithm 2 or the additive (deterministic
// Algorithm 5) cycle; the variant handed to the next coarser level follows.
inline bool cycle_multiplicative(int variant) { return variant == OMG_SYNC_MULT || variant == OMG_HYBRID; }
inline int cycle_sub_variant(int variant, int coarse_sync) {
    if (variant == OMG_HYBRID) return OMG_OVERLAP_DET;
    if ((variant == OMG_OVERLAP_DET || variant == OMG_ADD_SYNC) && coarse_sync) return OMG_SYNC_MULT;
    return variant;
}
// The level whose coarse path runs on the second stream (levels below it
// stay there); -1 if every level runs on the caller's stream.
inline int cycle_fork_level(const omg_options& o) {
    if (o.variant == OMG_OVERLAP_DET) return 0;
    if (o.variant == OMG_HYBRID) return 1;
    return -1;
}
// exchange words: two sets of [kMaxRedBlocks][kRmBlock + 1] block words, then
// two sets of kRmBlock + 1 total words (leader form)
constexpr size_t kRmSlotWords = 2 * (size_t)kMaxRedBlocks * (kRmBlock + 1) + 2 * (kRmBlock + 1);
// the lagged form: up to eight sets of up to (kRmLagMax + 1) kRmBlock + 1
// words per block, then eight sets of totals
constexpr int kRmLagSets = 8;
constexpr int kRmLagWords = (kRmLagMax + 1) * kRmBlock + 2;
constexpr size_t kRmSlotWordsLag = (size_t)kRmLagSets * kMaxRedBlocks * kRmLagWords + kRmLagSets * kRmLagWords;
constexpr size_t kRmSlotWordsMax = kRmSlotWordsLag > kRmSlotWords ? kRmSlotWordsLag : kRmSlotWords;

// Per-column state of the multi-column RM kernel (device table entry).
struct RmCol {
    int64_t N;
    double* const* Wp;                 // direction pointer arrays (device)
    double* const* Zp;
    const double* w;                   // A z
    const double* z;                   // the direction handed to RM (z or zcor)
    const double* zcor;
    double* r;
    unsigned long long* slots;
    double* part_rn;
    double* scal;
    double* hist;
    double* gammas;
    double* alphas;
    double* gram;
};
// One level of the hierarchy. Vectors are stored component-major inside the
// library ("SoA"): entry k of cell c at k*n + c, so that a wavefront of
// consecutive cells reads consecutive addresses.
// The operator is stored in an ELL-of-blocks layout: `width` block slots per
// cell; slot j of cell i holds column cell col[j*n+i] (padding slots point to
// the cell itself with zero values). Values are interleaved by column pairs:
// element (slot j, row r, column 2cp+h) of cell i is component h of the
// 2-vector at index ((j*bs + r)*bsh + cp)*n + i, bsh = ceil(bs/2).
struct Level {
    int nx = 0, ny = 0, nz = 0, n = 0; // cells
    int64_t N = 0;                     // DOFs = n*bs
    int width = 0;                     // ELL block slots per cell
    int coarsest = 0;
    int rowsplit = 0;                  // small level: one thread per (cell, block row) in SpMV / smoother
    int G = 1;                         // reduction grid for this level

    int* col = nullptr;                // [width][n]
    double* val = nullptr;             // pairs, see above
    float* val32 = nullptr;            // FP32 copy (mixed precision)
    double* dinv = nullptr;            // [bs][bsh][n] pairs: block-diagonal inverses
    float* dinv32 = nullptr;
    double* ainv = nullptr;            // coarsest: dense inverse, [np][np] SoA DOF order
    int np = 0;                        // padded dense order
    double* atile = nullptr;           // coarsest: lower-triangle 64x64 tiles of ainv (symmetric GEMV)
    double* spart = nullptr;           // [ntile][ntile][64] partial products of the symmetric GEMV
    double* mrpart = nullptr;          // [k tile][N][32] partial products of the multi-column product (built on first use)
    int ntile = 0;

    std::vector<int> hcol;             // host copy of col (Galerkin symbolic phase)
    // agglomeration maps (R and P of Algorithm 2). On a level with a coarser
    // one: up[K] = parent(K) << 3 | slot(K) (device) and its host copy hup.
    // On a level with a finer one: the finer cells of coarse cell I are
    // dn[dn_ptr[I] .. dn_ptr[I+1]) (device), each K << 3 | slot(K), ordered by
    // (slot, K) -- the order in which restriction sums them.
    int* up = nullptr;
    std::vector<int> hup;
    int* dn_ptr = nullptr;
    int* dn = nullptr;
    int* dslot = nullptr;              // [n] slot of the diagonal block of each cell
    // block-contiguous copies for the multi-right-hand-side kernels (built on
    // first use): blocks [n][width][bs][bs], inverses [n][bs][bs]
    double* ablk = nullptr;
    float* ablk32 = nullptr;
    double* dblk = nullptr;
    float* dblk32 = nullptr;
    // additive Schwarz smoother (built when selected): patch of cell i = i and
    // the cells its row couples to, as_w cells at most
    int as_w = 0;
    int* as_cells = nullptr;           // [as_w][n] cells of each patch (-1: none; present ones first)
    int* as_rev = nullptr;             // [as_w][n] contributions to cell i: patch * as_w + slot (-1: none)
    double* as_inv = nullptr;          // [n][m][m] patch inverses, transposed (m = as_w bs)
    float* as_inv32 = nullptr;         // the same rounded to float (mixed forms)
    double* as_z = nullptr;            // [n][m] local corrections of one sweep
    int shared_op = 0;                 // operator arrays belong to another solver (column solvers)
    // autotuned launch shape + 1 of the multi-RHS kernels [op: spmv, bj_first,
    // bj_sweep][FP64, FP32][one tile, two tiles]; 0 = not tuned
    int mr_shape[3][2][2] = {};
    int rm_dropped = 0; // RM configurations the tuner dropped (bounded waits expired)

    // work vectors (SoA, N each)
    double *b = nullptr, *r = nullptr, *x = nullptr, *z = nullptr, *w = nullptr;
    double *t = nullptr, *t2 = nullptr, *zcor = nullptr, *xout = nullptr;
    // reduction partials
    double* part = nullptr;            // [8][kMaxRedBlocks]
    double* scal = nullptr;            // [S_COUNT]

    // residual-minimisation storage: pointers to direction vectors
    int k = 0;
    std::vector<double*> W, Z;         // size = allocated capacity
    std::vector<double*> chunks;       // backing allocations
    double** dWp = nullptr;            // device copies of the W / Z pointer arrays
    double** dZp = nullptr;
    size_t dcap = 0;
    // persistent residual minimisation (one co-resident grid)
    int persist = 0;
    RmConfig rmc;                      // launch configuration (tuned at setup)
    RmConfig rmc_multi;                // configuration for multi-column launches of rmc_multi_m columns
    int rmc_multi_m = 0;
    unsigned* bar = nullptr;           // [2]: [1] = abort flag of the persistent kernel's waits
    unsigned long long* xslots = nullptr; // exchange words (kRmSlotWords)
    // layout (blocks, words per block, exchange form) of the last launch on
    // xslots: a stale word is only guaranteed to carry a foreign tag while
    // the layout stays the same, so the words are reset when it changes
    int slot_G = -1, slot_SW = -1, slot_lead = -1, slot_sets = -1;
    unsigned long long phase = 0;      // next exchange phase of this level (host counter)
    // implicit search directions (persistent levels): raw directions + MGS coefficients
    double* hist = nullptr;            // packed beta rows, ucap*(ucap-1)/2
    int ucap = 0;                      // maximum directions of one level solve
    double *alphas = nullptr, *gammas = nullptr, *gram = nullptr, *dvec = nullptr;
    int Grn = 1;                       // number of ||r||^2 partials written by the last update
    int restarted = 0;                 // the current level solve restarted (m_max): x holds the
                                       // share of the directions dropped at the restarts
    double *rs = nullptr, *xs = nullptr; // snapshot of r and x before a speculative iteration
};

struct Trace {
    double step, rnorm, type;
};

} // namespace omg

struct omg_solver {
    omg_options opt;
    omg_grid grid;                     // SIP geometry (omg_setup_sip); nx*ny*nz = level 0's cells
    int bs = 0, bsh = 0, p = 0, nlev = 0;
    hipStream_t stream = nullptr;      // caller's stream
    hipStream_t cstream = nullptr;     // coarse-path stream (OVERLAP_DET)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_step[2] = {nullptr, nullptr}; // smoother steps of a timing-adaptive cycle
    std::vector<omg::Level> lev;
    double* E = nullptr;               // [8][bs][bs] embedding blocks (device)
    float* E32 = nullptr;
    std::vector<double> hE;            // host copy
    // SIP data (omg_setup_sip)
    int has_sip = 0;
    double* nu = nullptr;              // [n_cells] device
    double* refm = nullptr;            // reference matrices: S, F[3][2][2], B[3][2] (device)
    // external <-> internal layout buffers (fine level)
    double *bufA = nullptr, *bufB = nullptr;
    double* host_scal = nullptr;       // pinned, mapped: residual norms per level
    double* host_scal_dev = nullptr;   // its device address
    int* err_flag = nullptr;           // device error flag (setup kernels)
    // logs of the last solve
    std::vector<int> visits;
    std::vector<int> steps;            // smoother+RM steps per cycle of the forking level
    std::vector<omg::Trace> trace;
    std::vector<int> replay;           // (level, iterations) pairs set by omg_set_replay
    // per-level queues of the replay during a solve (one host thread touches
    // one level's queue at a time; the outer vectors are sized before it)
    std::vector<std::vector<int>> replay_q;
    std::vector<size_t> replay_pos;
    int replaying = 0;
    // per-visit residual log of the last solve, in completion order: level,
    // iterations, ||r0||, then ||r|| after each iteration (what the level
    // tests of Sec. 4.2 read); appended under vnorm_mu (the adaptive cycle's
    // coarse thread logs its visits too)
    std::vector<double> vnorm;
    // residual norms computed during a solve, written by the device into mapped
    // host memory at consecutive positions (vlog_pos); a norm is read when a
    // level test needs it (after an event recorded behind it), and the log
    // entries above are filled from these positions when the solve ends
    double* vlog_host = nullptr;
    double* vlog_dev = nullptr;
    int64_t vlog_pos = 0;
    std::vector<hipEvent_t> vlog_ev;               // ring of events, one per position modulo its size
    std::vector<std::pair<size_t, int64_t>> vfix;  // (index into vnorm, position)
    std::vector<double> vlog_over;                 // values of positions past the buffer
    int mode32 = 0;                    // 0 FP64, 1 FP32 everywhere, 2 FP32 except finest-level RM
    int64_t kcount[OMG_K_COUNT][OMG_MAX_LEVELS] = {};  // launches per kernel kind and level
    int64_t nnzb_level[OMG_MAX_LEVELS] = {};           // stored (non-padding) blocks per level
    // kernel probe: events around launches of one kernel kind on one level
    int probe_kind = -1, probe_level = -1, probe_max = 0;
    std::vector<hipEvent_t> probe_ev;                  // begin/end pairs
    int64_t probe_n = 0;
    double probe_bytes = 0.0;                          // algorithmic bytes summed over probed launches
    int step = 0;
    int status = 0;
    // batched solves: column solvers that share this solver's operator arrays
    // (work vectors and search directions of their own), created on demand
    omg_solver* owner = nullptr;       // set on a column solver: the solver whose operator it uses
    std::vector<omg_solver*> columns;
    // batched RM launches led by this solver: per level, the device table of
    // the members' RM state and what it holds; the launches' abort flag
    omg::RmCol* btab[OMG_MAX_LEVELS] = {};
    std::vector<omg::RmCol> btab_host[OMG_MAX_LEVELS];
    unsigned* babort = nullptr;
    int batch_rm_off = 0;              // set when a batched RM launch's wait expired
    double* bnorm_host = nullptr;      // [kMaxCols] pinned, mapped: norms of batched members
    double* bnorm_dev = nullptr;       // its device address
};

namespace omg {

// ---------------------------------------------------------------- kernels
// (omg_kernels.hip). Every launcher enqueues on `st` and returns the launch
// status.
hipError_t launch_to_soa(const double* in, double* out, int n, int bs, hipStream_t st);
hipError_t launch_from_soa(const double* in, double* out, int n, int bs, hipStream_t st);
hipError_t launch_spmv(const Level& L, int bs, bool fp32, const double* x, const double* b, double* y,
                       hipStream_t st);
hipError_t launch_bj_first(const Level& L, int bs, bool fp32, double omega, const double* r, double* x,
                           hipStream_t st);
omg_status as_setup(omg_solver* s, Level& L);
hipError_t launch_as_sweep(const Level& L, int bs, bool fp32, double omega, const double* v, double* out,
                           bool accumulate, hipStream_t st);
hipError_t launch_bj_sweep(const Level& L, int bs, bool fp32, double omega, const double* r, const double* xin,
                           double* xout, hipStream_t st);
hipError_t launch_restrict(const Level& F, const Level& C, int bs, bool fp32, const double* E, const float* E32,
                           const double* r, double* rc, hipStream_t st);
hipError_t launch_prolong(const Level& F, const Level& C, int bs, bool fp32, const double* E, const float* E32,
                          const double* zc, double* z, hipStream_t st);
hipError_t launch_gemv(const Level& L, const double* x, double* y, hipStream_t st);
hipError_t build_symv_tiles(Level& L, hipStream_t st);

// reductions: partial sums into part[0..G) (deterministic fixed-order)
hipError_t launch_dot2(int64_t N, int G, const double* a, const double* b, double* part_ab, const double* c,
                       double* part_cc, hipStream_t st);
hipError_t launch_mgs_step(int64_t N, int G, const double* part_in, const double* Wi, const double* Zi, double* w,
                           double* z, const double* Wnext, double* part_out, hipStream_t st);
hipError_t launch_rm_normalize(int64_t N, int G, const double* part_nin, const double* part_nout,
                               double breakdown, const double* w, const double* z, double* Wk, double* Zk,
                               const double* r, double* part_alpha, double* scal, hipStream_t st);
hipError_t launch_rm_update(int64_t N, int G, const double* part_alpha, const double* Wk, const double* Zk,
                            double* x, double* r, double* part_rn, hipStream_t st);
hipError_t launch_finish_norm(int G, const double* part, double* out, hipStream_t st);
// x = 0, r = b, partials of ||b||^2 into part[0..G) (as launch_dot2)
hipError_t launch_level_init(int64_t N, int G, const double* b, double* x, double* r, double* part,
                             hipStream_t st);
hipError_t launch_copy(double* dst, const double* src, int64_t N, hipStream_t st);
hipError_t launch_snap(double* dr, const double* sr, int64_t N, double* dx, const double* sx, int64_t Nx, double* ds,
                       const double* ss, hipStream_t st);
hipError_t launch_fill(double* dst, double v, int64_t N, hipStream_t st);
hipError_t launch_stream_copy(double* dst, const double* src, int64_t N, hipStream_t st);
hipError_t launch_axpy(double* y, double a, const double* x, int64_t N, hipStream_t st);

// persistent RM (omg_rm.hip)
struct RmArgs {
    int64_t N;                         // vector entries
    int k;                             // directions stored before this RM
    const double* const* Wp;           // stored orthonormal directions
    double* Wk;                        // receives the new direction w_k
    double* Zk;                        // receives the raw direction z~_k
    const double* w;                   // A z~
    const double* z;                   // z~
    double* r;                         // residual (updated)
    unsigned long long* slots;         // exchange words
    unsigned long long g0;             // first exchange phase of this launch
    double* part_rn;                   // partials of ||r||^2 (one per block)
    double breakdown;
    double* scal;
    unsigned* abort_flag;
    double* hist;                      // packed rows: beta_{k,i} at k(k-1)/2 + i
    double* gammas;                    // gamma of every direction (0 = dropped)
    double* alphas;                    // alpha of every direction
    double* gram;                      // [.][kRmBlock-1] intra-block Gram entries
};
struct RmMulti {
    const RmCol* tab;                  // device table
    int k;                             // directions stored before this RM (same for all columns)
    int zcor;                          // 1: the direction is zcor
    double breakdown;
    unsigned* abort_flag;
    int ncol;
    int idx[kMaxCols];                 // table entry of column q
    int blk0[kMaxCols + 1];            // block range of column q
    unsigned long long g0[kMaxCols];   // first exchange phase of column q
};
int rm_multi_capacity(int ept, int B, int lead, int lag = 0);
hipError_t launch_rm_multi(int ept, int B, int lead, int lag, const RmMulti& M, hipStream_t st);

// co-resident configurations for N entries, most preferred first; returns the count
constexpr int kMaxRmConfigs = 192;
int rm_persistent_candidates(int64_t N, RmConfig* out, int cap);
bool rm_persistent_config(int64_t N, RmConfig* cfg);
hipError_t launch_rm_persistent(const RmConfig& c, const RmArgs& args, hipStream_t st);
// the persistent kernel on vectors without a zero tail past N (entries >= N
// neither read nor written; Zk may be null): its co-resident configuration
// and launch
bool rm_masked_config(int64_t N, RmConfig* cfg);
hipError_t launch_rm_masked(const RmConfig& c, const RmArgs& args, hipStream_t st);
// Reset L's exchange words to "empty" if configuration c lays them out
// differently from the last launch on them (call before every launch).
hipError_t prepare_slots(Level& L, const RmConfig& c, hipStream_t st);
// d = coefficients of x = sum_k alpha_k z_k in the raw directions
hipError_t launch_recon(int K, const double* hist, const double* gammas, const double* alphas, double* d,
                        hipStream_t st);
// out = sum_m d[m] V_m
hipError_t launch_lincomb(int64_t N, int k, const double* d, const double* const* V, double* out,
                          hipStream_t st);
// launch_recon + launch_lincomb for several members (K[q] >= 1 directions each)
struct RecTable {
    int count;
    int blk0[kMaxCols + 1];
    int K[kMaxCols];
    int64_t N[kMaxCols];
    const double* hist[kMaxCols];
    const double* gammas[kMaxCols];
    const double* alphas[kMaxCols];
    double* d[kMaxCols];
    const double* const* V[kMaxCols];
    double* out[kMaxCols];
};
hipError_t launch_recon_combine_grouped(RecTable& T, hipStream_t st);

// multi-right-hand-side kernels (omg_multi.hip): nr <= kMaxCols columns that
// share the operator of L; B may be null (then Y = A X, else Y = B - A X)
hipError_t build_blocks(Level& L, int bs, int bsh, hipStream_t st);
hipError_t launch_spmv_mr(const Level& L, int bs, bool fp32, int nr, const ColPtrs& X, const ColPtrs* B,
                          const ColPtrs& Y, hipStream_t st);
hipError_t launch_bj_first_mr(const Level& L, int bs, bool fp32, double omega, int nr, const ColPtrs& R,
                              const ColPtrs& X, hipStream_t st);
hipError_t launch_bj_sweep_mr(const Level& L, int bs, bool fp32, double omega, int nr, const ColPtrs& R,
                              const ColPtrs& Xin, const ColPtrs& Xout, hipStream_t st);
hipError_t launch_dense_mr(const Level& L, int nr, const ColPtrs& X, const ColPtrs& Y, hipStream_t st);
// time every launch shape of the multi-RHS kernels on L for nr columns and keep
// the fastest per (operation, precision, tile count); best_us[6] (nullable)
hipError_t tune_mr(Level& L, int bs, int nr, const ColPtrs& X, const ColPtrs& Y, const ColPtrs& T, int reps,
                   hipStream_t st, double* best_us);
// Grid transfers of several members in one launch (segment per member).
struct XferTable {
    int count;
    int blk0[kMaxCols + 1];
    int fn[kMaxCols], cn[kMaxCols];
    const int* up[kMaxCols];           // the fine level's maps (Level::up)
    const int* dn_ptr[kMaxCols];       // the coarse level's child lists
    const int* dn[kMaxCols];
    const double* in[kMaxCols];
    double* out[kMaxCols];
};
// Level entry (x = 0, r = b, ||b||^2 partials) of several members.
struct InitTable {
    int count;
    int blk0[kMaxCols + 1];
    int64_t N[kMaxCols];
    const double* b[kMaxCols];
    double* x[kMaxCols];
    double* r[kMaxCols];
    double* part[kMaxCols];
};
hipError_t launch_restrict_grouped(int bs, bool fp32, const double* E, const float* E32, XferTable& T,
                                   hipStream_t st);
hipError_t launch_prolong_grouped(int bs, bool fp32, const double* E, const float* E32, XferTable& T,
                                  hipStream_t st);
// G[q]: reduction blocks of member q (its partials as launch_level_init's)
hipError_t launch_level_init_grouped(InitTable& T, const int* G, hipStream_t st);
// grouped forms over T.count instances of one block size (blk0 is filled in):
// SpMV y = A x or b - A x; first block-Jacobi iteration y = omega D^-1 b;
// fused iteration y = x + omega D^-1 (b - A x)
hipError_t launch_spmv_grouped(int bs, bool fp32, SegTable& T, hipStream_t st);
hipError_t launch_bj_first_grouped(int bs, bool fp32, double omega, SegTable& T, hipStream_t st);
hipError_t launch_bj_sweep_grouped(int bs, bool fp32, double omega, SegTable& T, hipStream_t st);
// out[c] = sqrt(sum of the G[c] partials of column c), same order as launch_finish_norm
hipError_t launch_finish_norms(int m, const NormPack& P, double* out, hipStream_t st);

// ---------------------------------------------------------------- setup
// (omg_setup.hip)
int reduction_blocks(int64_t N);
void basis_orders(int p, std::vector<int>& a, std::vector<int>& b, std::vector<int>& c);
void embedding_blocks(int p, std::vector<double>& E);
void reference_matrices(int p, double h, double penalty_c, std::vector<double>& out);

// ---------------------------------------------------------------- engine
// (omg_solve.hip), shared with the batched driver (omg_batch.hip)
bool engine_use32(const omg_solver* s, int l, bool is_rm);
bool engine_stop_level(const omg_solver* s, int l, double rn, double r0n, int it, double tol);
// RM of Algorithm 1 with w = A z already in the level's w vector
omg_status engine_rm_apply(omg_solver* s, int l, double* z, hipStream_t st);
// a column solver for batched solves: shares the operator of `owner`
omg_status engine_make_column(omg_solver* owner, omg_solver** out);
omg_status engine_finish_report(omg_solver* s, const double* b, const double* x, omg_report* R);
// storage for direction L.k of level l (and the k + 1 <= capacity check)
omg_status engine_ensure_dir(omg_solver* s, int l);
void engine_reset_logs(omg_solver* s);

} // namespace omg

// error helpers
#define OMG_TRY_HIP(expr)                                  \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return OMG_EHIP;             \
    } while (0)
#define OMG_TRY(expr)                                      \
    do {                                                   \
        omg_status s_ = (expr);                            \
        if (s_ != OMG_OK) return s_;                       \
    } while (0)
