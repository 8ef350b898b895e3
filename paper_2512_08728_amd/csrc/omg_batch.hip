// Batched solves: several right-hand sides on one operator advanced in
// lockstep, and several independent solvers called together.
//
// Lockstep (one solver, nrhs > 1): every right-hand side gets a column solver
// that shares the operator arrays and keeps its own work vectors, search
// directions W, Z and stopping state on every level. Each step of the cycle
// (Algorithm 2, or the deterministic form of Algorithm 5) runs for all
// columns that are still iterating on that level: the block-Jacobi sweeps
// (Algorithm 4), the SpMV inside RM and the coarsest solve are one
// matrix-core launch for up to 32 columns, so the operator is read once per
// sweep instead of once per column; the orthogonalisation of Algorithm 1
// runs per column (its inner products are per column). Each column keeps the
// level-local stopping rules of Sec. 4.2 on its own residual: a column that
// has stopped on a level is masked out of that level's remaining steps.
#include <chrono>
#include <cmath>
#include <cstring>

#include "omg_internal.h"

using namespace omg;

#define HIP_OK(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) {                        \
            (void)hipGetLastError();                   \
            return OMG_EHIP;                           \
        }                                              \
    } while (0)

namespace {

__global__ void k_gather_cols(const double* __restrict__ in, ColPtrs out, int n, int bs, int nrhs, int c0, int m) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * bs * m) return;
    const int j = (int)(t % m);
    const int64_t e = t / m;
    const int c = (int)(e / bs), k = (int)(e % bs);
    out.p[j][(int64_t)k * n + c] = in[e * nrhs + c0 + j];
}
__global__ void k_scatter_cols(ColPtrs in, double* __restrict__ out, int n, int bs, int nrhs, int c0, int m) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * bs * m) return;
    const int j = (int)(t % m);
    const int64_t e = t / m;
    const int c = (int)(e / bs), k = (int)(e % bs);
    out[e * nrhs + c0 + j] = in.p[j][(int64_t)k * n + c];
}

// One lockstep group. Either up to kMaxCols column solvers that share the
// operator of P (matrix-core multi-RHS kernels), or up to kMaxSeg
// independent solvers (grouped launches, one segment per solver). The cycle
// options (variant, sweeps, omega, precision) are those of P for every member.
struct Group {
    omg_solver* P = nullptr;           // operator owner (shared) or first member; counts, norm buffers
    bool shared = false;
    std::vector<omg_solver*> col;
    std::vector<double> tol;           // per member: finest-level tolerance of the current mg call
    std::vector<omg_status> stat;      // per member: finest-level status of the current mg call
    hipStream_t st = nullptr;
};

inline Level& LV(omg_solver* c, int l) { return c->lev[l]; }

template <typename F> ColPtrs pack(const std::vector<int>& act, F f) {
    ColPtrs p;
    std::memset(&p, 0, sizeof(p));
    for (size_t i = 0; i < act.size(); ++i) p.p[i] = f(act[i], (int)i);
    return p;
}

template <typename F> SegTable segs(Group& g, const std::vector<int>& act, int l, bool fp32, F f) {
    SegTable T;
    std::memset(&T, 0, sizeof(T));
    T.count = (int)act.size();
    for (size_t i = 0; i < act.size(); ++i) {
        Level& L = LV(g.col[act[i]], l);
        T.n[i] = L.n;
        T.width[i] = L.width;
        T.col[i] = L.col;
        T.val[i] = fp32 ? (const void*)L.val32 : (const void*)L.val;
        T.dinv[i] = fp32 ? (const void*)L.dinv32 : (const void*)L.dinv;
        f(T, (int)i, act[i]);
    }
    return T;
}

// ---- operations over the active members -----------------------------------
// Y = A X or B - A X (B nullable)
omg_status op_spmv(Group& g, const std::vector<int>& act, int l, bool fp32, const ColPtrs& X, const ColPtrs* B,
                   const ColPtrs& Y) {
    omg_solver* P = g.P;
    if (g.shared) {
        HIP_OK(launch_spmv_mr(P->lev[l], P->bs, fp32, (int)act.size(), X, B, Y, g.st));
    } else {
        SegTable T = segs(g, act, l, fp32, [&](SegTable& t, int i, int) {
            t.x[i] = X.p[i];
            t.b[i] = B ? B->p[i] : nullptr;
            t.y[i] = Y.p[i];
        });
        HIP_OK(launch_spmv_grouped(P->bs, fp32, T, g.st));
    }
    P->kcount[fp32 ? OMG_K_SPMV32 : OMG_K_SPMV][l]++;
    return OMG_OK;
}

// O = omega D^-1 R (first block-Jacobi iteration from zero)
omg_status op_bj_first(Group& g, const std::vector<int>& act, int l, bool fp32, const ColPtrs& R, const ColPtrs& O) {
    omg_solver* P = g.P;
    if (g.shared) {
        HIP_OK(launch_bj_first_mr(P->lev[l], P->bs, fp32, P->opt.omega, (int)act.size(), R, O, g.st));
    } else {
        SegTable T = segs(g, act, l, fp32, [&](SegTable& t, int i, int) {
            t.b[i] = R.p[i];
            t.y[i] = O.p[i];
        });
        HIP_OK(launch_bj_first_grouped(P->bs, fp32, P->opt.omega, T, g.st));
    }
    P->kcount[OMG_K_BJFIRST][l]++;
    return OMG_OK;
}

// O = I + omega D^-1 (R - A I)
omg_status op_bj_sweep(Group& g, const std::vector<int>& act, int l, bool fp32, const ColPtrs& R, const ColPtrs& I,
                       const ColPtrs& O) {
    omg_solver* P = g.P;
    if (g.shared) {
        HIP_OK(launch_bj_sweep_mr(P->lev[l], P->bs, fp32, P->opt.omega, (int)act.size(), R, I, O, g.st));
    } else {
        SegTable T = segs(g, act, l, fp32, [&](SegTable& t, int i, int) {
            t.b[i] = R.p[i];
            t.x[i] = I.p[i];
            t.y[i] = O.p[i];
        });
        HIP_OK(launch_bj_sweep_grouped(P->bs, fp32, P->opt.omega, T, g.st));
    }
    P->kcount[fp32 ? OMG_K_BJ32 : OMG_K_BJ][l]++;
    return OMG_OK;
}

// Y = A_c^-1 X on members whose level l is their coarsest
omg_status op_coarse(Group& g, const std::vector<int>& act, int l, const ColPtrs& X, const ColPtrs& Y) {
    omg_solver* P = g.P;
    if (g.shared) {
        HIP_OK(launch_dense_mr(P->lev[l], (int)act.size(), X, Y, g.st));
    } else {
        for (size_t i = 0; i < act.size(); ++i) HIP_OK(launch_gemv(LV(g.col[act[i]], l), X.p[i], Y.p[i], g.st));
    }
    P->kcount[OMG_K_COARSE][l]++;
    return OMG_OK;
}

// Norms of the members in `act` from the partials their last reduction left
// in part slot 4 (L.Grn of them): one launch into mapped host memory, one wait.
omg_status read_norms(Group& g, const std::vector<int>& act, int l, std::vector<double>& out) {
    NormPack np;
    std::memset(&np, 0, sizeof(np));
    for (size_t i = 0; i < act.size(); ++i) {
        Level& L = LV(g.col[act[i]], l);
        np.part[i] = L.part + 4 * kMaxRedBlocks;
        np.G[i] = L.Grn;
    }
    HIP_OK(launch_finish_norms((int)act.size(), np, g.P->bnorm_dev, g.st)); // mapped host memory
    HIP_OK(hipStreamSynchronize(g.st));
    out.assign(g.P->bnorm_host, g.P->bnorm_host + act.size());
    return OMG_OK;
}

// ||v_i|| for the members in act (v given per active index).
omg_status vec_norms(Group& g, const std::vector<int>& act, int l, const ColPtrs& v, std::vector<double>& out) {
    for (size_t i = 0; i < act.size(); ++i) {
        Level& L = LV(g.col[act[i]], l);
        HIP_OK(launch_dot2(L.N, L.G, nullptr, nullptr, nullptr, v.p[i], L.part + 4 * kMaxRedBlocks, g.st));
        L.Grn = L.G;
    }
    return read_norms(g, act, l, out);
}

// z_i (or zcor_i) = BJ(r_i, sweeps) (Algorithm 4 from zero).
omg_status smoother_b(Group& g, const std::vector<int>& act, int l, int sweeps, bool zcor) {
    const bool f32 = engine_use32(g.col[act[0]], l, false);
    if (sweeps < 1) sweeps = 1;
    const ColPtrs R = pack(act, [&](int c, int) { return LV(g.col[c], l).r; });
    const ColPtrs O = pack(act, [&](int c, int) { return zcor ? LV(g.col[c], l).zcor : LV(g.col[c], l).z; });
    const ColPtrs T = pack(act, [&](int c, int) { return LV(g.col[c], l).t; });
    const ColPtrs* bufs[2] = {&O, &T};
    int cur = (sweeps % 2 == 1) ? 0 : 1;
    OMG_TRY(op_bj_first(g, act, l, f32, R, *bufs[cur]));
    for (int it = 1; it < sweeps; ++it) {
        OMG_TRY(op_bj_sweep(g, act, l, f32, R, *bufs[cur], *bufs[cur ^ 1]));
        cur ^= 1;
    }
    return OMG_OK;
}

// Launch configuration of the multi-column RM for m columns of N entries:
// the tuned single-column form (entries per thread, directions per exchange,
// exchange form) with entries per thread raised until all m columns' blocks
// are co-resident in one launch, else the most columns per launch.
RmConfig multi_config(const RmConfig& tuned, int64_t N, int m) {
    static const int epts[] = {1, 2, 4, 8, 10, 16, 20};
    RmConfig best = tuned;
    int best_cols = 0;
    for (int e : epts) {
        if (e < std::min(tuned.ept, 20)) continue;
        for (int b : {tuned.B, 2, 1}) {
            if (b > tuned.B) continue;
            const int G = (int)((N + (int64_t)kThreads * e - 1) / ((int64_t)kThreads * e));
            const int cap = rm_multi_capacity(e, b, tuned.lead);
            if (G > kMaxRedBlocks || cap < G) continue;
            const int cols = std::min(m, cap / G);
            if (cols > best_cols) {
                best_cols = cols;
                best = RmConfig{G, e, b, tuned.lead};
            }
            if (cols == m) return best;
        }
    }
    return best;
}

// The RM state of every group member at level l in the level's device table
// (uploaded when it changed: a new direction chunk moves the pointer arrays).
omg_status refresh_rm_table(Group& g, int l) {
    omg_solver* P = g.P;
    const int m = (int)g.col.size();
    if (!P->btab[l] && hipMalloc((void**)&P->btab[l], sizeof(RmCol) * kMaxCols) != hipSuccess) return OMG_ENOMEM;
    std::vector<RmCol> h(m);
    for (int i = 0; i < m; ++i) {
        RmCol& c = h[i];
        std::memset(&c, 0, sizeof(c));
        if (l >= g.col[i]->nlev || !g.col[i]->lev[l].persist) continue; // member has no RM state here
        Level& L = LV(g.col[i], l);
        c.N = L.N;
        c.Wp = L.dWp;
        c.Zp = L.dZp;
        c.w = L.w;
        c.z = L.z;
        c.zcor = L.zcor;
        c.r = L.r;
        c.slots = L.xslots;
        c.part_rn = L.part + 4 * kMaxRedBlocks;
        c.scal = L.scal;
        c.hist = L.hist;
        c.gammas = L.gammas;
        c.alphas = L.alphas;
        c.gram = L.gram;
    }
    std::vector<RmCol>& H = P->btab_host[l];
    const bool same = H.size() == h.size() && std::memcmp(H.data(), h.data(), sizeof(RmCol) * h.size()) == 0;
    if (!same) { // rare (a new chunk of directions): copy and wait, so the source may change afterwards
        H = h;
        HIP_OK(hipMemcpyAsync(P->btab[l], H.data(), sizeof(RmCol) * m, hipMemcpyHostToDevice, g.st));
        HIP_OK(hipStreamSynchronize(g.st));
    }
    return OMG_OK;
}

// Launch configuration of member c's RM in a batched launch at level l.
// The multi-column kernels have no exchange wave: a tuned exchange-wave
// configuration contributes its grid, entries per thread, block and exchange
// form (the two forms sum in the same order). A lagged configuration keeps
// its lag (the multi-column lagged kernel), so that an instance runs the
// arithmetic of its own solve.
inline RmConfig member_config(const Group& g, int c, int l) {
    RmConfig r = g.shared ? g.P->lev[l].rmc_multi : g.col[c]->lev[l].rmc;
    r.cw = 0;
    if (g.shared) r.lag = 0;
    return r;
}

// RM of the active persistent members in multi-column launches: members with
// the same launch configuration share a launch as long as their blocks are
// co-resident; each keeps its own exchange words, phase and storage.
omg_status rm_multi(Group& g, const std::vector<int>& act, int l, bool zcor) {
    omg_solver* P = g.P;
    for (int c : act) OMG_TRY(engine_ensure_dir(g.col[c], l));
    OMG_TRY(refresh_rm_table(g, l));
    const int k = LV(g.col[act[0]], l).k;
    for (int c : act)
        if ((int)LV(g.col[c], l).dcap <= k) return OMG_EINVAL; // direction k must have storage
    std::vector<RmConfig> cfg(act.size());
    for (size_t i = 0; i < act.size(); ++i) {
        const Level& L = LV(g.col[act[i]], l);
        if (L.k != k) return OMG_EINVAL; // lockstep members share k
        cfg[i] = member_config(g, act[i], l);
    }
    std::vector<int> done(act.size(), 0);
    for (size_t i0 = 0; i0 < act.size(); ++i0) {
        if (done[i0]) continue;
        const RmConfig c0 = cfg[i0];
        const int cap = rm_multi_capacity(c0.ept, c0.B, c0.lead, c0.lag);
        RmMulti M;
        std::memset(&M, 0, sizeof(M));
        M.tab = P->btab[l];
        M.k = k;
        M.zcor = zcor ? 1 : 0;
        M.breakdown = P->opt.breakdown;
        M.abort_flag = P->babort;
        std::vector<int> members;
        int blocks = 0;
        for (size_t i = i0; i < act.size() && M.ncol < kMaxCols; ++i) {
            if (done[i] || cfg[i].ept != c0.ept || cfg[i].B != c0.B || cfg[i].lead != c0.lead ||
                cfg[i].lag != c0.lag)
                continue;
            if (M.ncol > 0 && blocks + cfg[i].G > cap) continue;
            HIP_OK(prepare_slots(LV(g.col[act[i]], l), cfg[i], g.st));
            M.idx[M.ncol] = act[i];
            M.blk0[M.ncol] = blocks;
            M.g0[M.ncol] = LV(g.col[act[i]], l).phase;
            blocks += cfg[i].G;
            M.ncol++;
            done[i] = 1;
            members.push_back((int)i);
        }
        M.blk0[M.ncol] = blocks;
        if (blocks > cap) return OMG_EINVAL; // a single member larger than the device
        HIP_OK(launch_rm_multi(c0.ept, c0.B, c0.lead, c0.lag, M, g.st));
        P->kcount[OMG_K_RMP][l]++;
        for (int i : members) {
            Level& L = LV(g.col[act[i]], l);
            L.phase += rm_phases(k, c0.B);
            L.Grn = cfg[i].G;
            L.k++;
        }
    }
    return OMG_OK;
}

// RM (Algorithm 1) of every active member with its direction z (or zcor):
// one SpMV launch for all, then the orthogonalisation and update of the
// persistent members in multi-column launches (others one by one).
omg_status rm_b(Group& g, const std::vector<int>& act, int l, bool zcor) {
    const bool f32 = engine_use32(g.col[act[0]], l, true);
    const ColPtrs Z = pack(act, [&](int c, int) { return zcor ? LV(g.col[c], l).zcor : LV(g.col[c], l).z; });
    const ColPtrs W = pack(act, [&](int c, int) { return LV(g.col[c], l).w; });
    OMG_TRY(op_spmv(g, act, l, f32, Z, nullptr, W));
    std::vector<int> multi;
    for (size_t i = 0; i < act.size(); ++i) {
        omg_solver* s = g.col[act[i]];
        bool ok = LV(s, l).persist && g.P->babort && !g.P->batch_rm_off;
        if (ok && g.shared) ok = g.P->lev[l].rmc_multi_m > 0;
        if (ok) {
            const RmConfig c = member_config(g, act[i], l);
            ok = c.G <= rm_multi_capacity(c.ept, c.B, c.lead, c.lag);
        }
        if (ok) multi.push_back(act[i]);
        else OMG_TRY(engine_rm_apply(s, l, Z.p[i], g.st));
    }
    if (!multi.empty()) OMG_TRY(rm_multi(g, multi, l, zcor));
    return OMG_OK;
}

omg_status mg_b(Group& g, std::vector<int> act, int l, int variant);

// z_i (or zcor_i) = P_l MG_{l+1}(P_l^T r_i, 0) for the active members.
// Transfer table of the active members between levels l and l+1.
XferTable xfer_table(Group& g, const std::vector<int>& act, int l, bool up, bool zcor) {
    XferTable T;
    std::memset(&T, 0, sizeof(T));
    T.count = (int)act.size();
    for (size_t i = 0; i < act.size(); ++i) {
        const Level& F = LV(g.col[act[i]], l);
        const Level& C = LV(g.col[act[i]], l + 1);
        T.fn[i] = F.n;
        T.cn[i] = C.n;
        T.up[i] = F.up;
        T.dn_ptr[i] = C.dn_ptr;
        T.dn[i] = C.dn;
        T.in[i] = up ? F.r : C.xout;
        T.out[i] = up ? C.b : (zcor ? F.zcor : F.z);
    }
    return T;
}

omg_status coarse_path(Group& g, const std::vector<int>& act, int l, int variant, bool zcor) {
    omg_solver* P = g.P;
    omg_solver* s0 = g.col[act[0]];
    const bool f32 = engine_use32(s0, l, false);
    XferTable up = xfer_table(g, act, l, true, zcor);
    HIP_OK(launch_restrict_grouped(s0->bs, f32, s0->E, s0->E32, up, g.st));
    OMG_TRY(mg_b(g, act, l + 1, variant));
    XferTable down = xfer_table(g, act, l, false, zcor);
    HIP_OK(launch_prolong_grouped(s0->bs, f32, s0->E, s0->E32, down, g.st));
    P->kcount[OMG_K_RESTRICT][l]++;
    P->kcount[OMG_K_PROLONG][l]++;
    return OMG_OK;
}

// MG_l(b, 0) for every active member: input LV(c,l).b, output LV(c,l).xout.
// On the finest level member c stops at ||r|| <= g.tol[c] ||r0|| (Sec. 4.2
// criteria below it) and its status goes to g.stat[c].
omg_status mg_b(Group& g, std::vector<int> act, int l, int variant) {
    omg_solver* P = g.P;
    {   // members for which level l is the coarsest: direct solve
        std::vector<int> co, rest;
        for (int c : act) (LV(g.col[c], l).coarsest ? co : rest).push_back(c);
        if (!co.empty()) {
            const ColPtrs X = pack(co, [&](int c, int) { return LV(g.col[c], l).b; });
            const ColPtrs Y = pack(co, [&](int c, int) { return LV(g.col[c], l).xout; });
            OMG_TRY(op_coarse(g, co, l, X, Y));
        }
        act.swap(rest);
    }
    const int m = (int)act.size();
    if (m == 0) return OMG_OK;
    {
        InitTable T;
        std::memset(&T, 0, sizeof(T));
        int G[kMaxCols];
        T.count = m;
        for (int i = 0; i < m; ++i) {
            Level& L = LV(g.col[act[i]], l);
            L.k = 0;
            T.N[i] = L.N;
            T.b[i] = L.b;
            T.x[i] = L.x;
            T.r[i] = L.r;
            T.part[i] = L.part + 4 * kMaxRedBlocks;
            G[i] = L.G;
            L.Grn = L.G;
        }
        HIP_OK(launch_level_init_grouped(T, G, g.st));
    }
    std::vector<double> r0;
    OMG_TRY(read_norms(g, act, l, r0));
    std::vector<double> rn = r0;
    std::vector<int> its(m, 0), live(m, 1);
    std::vector<std::vector<double>> rns(m); // ||r|| after each iteration, per member
    const int sub_variant = cycle_sub_variant(variant, P->opt.coarse_sync);
    for (;;) {
        std::vector<int> cur, pos;
        for (int i = 0; i < m; ++i) {
            if (!live[i]) continue;
            omg_solver* s = g.col[act[i]];
            const double tl = (l == 0) ? g.tol[act[i]] : 0.0;
            if (!std::isfinite(rn[i]) || engine_stop_level(s, l, rn[i], r0[i], its[i], tl)) {
                live[i] = 0;
                continue;
            }
            cur.push_back(act[i]);
            pos.push_back(i);
        }
        if (cur.empty()) break;
        if (cycle_multiplicative(variant)) {
            OMG_TRY(smoother_b(g, cur, l, P->opt.s_pre, false));
            OMG_TRY(rm_b(g, cur, l, false));
            OMG_TRY(coarse_path(g, cur, l, sub_variant, false));
            OMG_TRY(rm_b(g, cur, l, false));
            OMG_TRY(smoother_b(g, cur, l, P->opt.s_post, false));
            OMG_TRY(rm_b(g, cur, l, false));
        } else {
            // deterministic Algorithm 5: coarse correction from the residual at
            // the start of the cycle, n_s smoother+RM steps, then RM(z_cor)
            OMG_TRY(coarse_path(g, cur, l, sub_variant, true));
            for (int t = 0; t < P->opt.n_s; ++t) {
                OMG_TRY(smoother_b(g, cur, l, P->opt.s_post, false));
                OMG_TRY(rm_b(g, cur, l, false));
            }
            OMG_TRY(rm_b(g, cur, l, true));
        }
        std::vector<double> nv;
        OMG_TRY(read_norms(g, cur, l, nv));
        for (size_t q = 0; q < cur.size(); ++q) {
            its[pos[q]]++;
            rn[pos[q]] = nv[q];
            rns[pos[q]].push_back(nv[q]);
        }
    }
    RecTable T;
    std::memset(&T, 0, sizeof(T));
    for (int i = 0; i < m; ++i) {
        const int c = act[i];
        omg_solver* s = g.col[c];
        Level& L = LV(s, l);
        s->visits.push_back(l);
        s->visits.push_back(its[i]);
        s->vnorm.push_back(l);
        s->vnorm.push_back(its[i]);
        s->vnorm.push_back(r0[i]);
        s->vnorm.insert(s->vnorm.end(), rns[i].begin(), rns[i].end());
        if (l == 0) {
            if (!std::isfinite(rn[i])) g.stat[c] = OMG_EINVAL;
            else if (rn[i] > g.tol[c] * r0[i]) g.stat[c] = OMG_ENOCONV;
        }
        if (L.persist && L.k > 0) { // x = sum_k d_k z~_k, all such members in one pair of launches
            const int q = T.count++;
            T.K[q] = L.k;
            T.N[q] = L.N;
            T.hist[q] = L.hist;
            T.gammas[q] = L.gammas;
            T.alphas[q] = L.alphas;
            T.d[q] = L.dvec;
            T.V[q] = L.dZp;
            T.out[q] = L.xout;
        } else if (L.persist) {
            HIP_OK(launch_lincomb(L.N, 0, L.dvec, L.dZp, L.xout, g.st)); // no directions: x = 0
        } else {
            HIP_OK(launch_copy(L.xout, L.x, L.N, g.st));
        }
    }
    if (T.count > 0) HIP_OK(launch_recon_combine_grouped(T, g.st));
    return OMG_OK;
}

// Outer solve of the members of one group: b in bufA, x (in/out) in bufB of
// every member (component-major). Mirrors the single solve: FP64 (or
// flexible mixed) correction solve from the outer residual, or FP64 iterative
// refinement around FP32 inner solves. Fills R[i].iters_fine/outer_iters/
// rel_res_rec and stat[i].
omg_status solve_group(Group& g, double tol, std::vector<omg_report>& R, std::vector<omg_status>& stat) {
    omg_solver* P = g.P;
    const int m = (int)g.col.size();
    g.tol.assign(m, 0.0);
    g.stat.assign(m, OMG_OK);
    std::vector<int> all(m);
    for (int i = 0; i < m; ++i) all[i] = i;
    for (omg_solver* s : g.col) engine_reset_logs(s);
    std::vector<double> bn;
    OMG_TRY(vec_norms(g, all, 0, pack(all, [&](int c, int) { return g.col[c]->bufA; }), bn));
    std::vector<int> act;
    for (int i = 0; i < m; ++i) {
        if (!std::isfinite(bn[i])) stat[i] = OMG_EINVAL;
        else if (bn[i] == 0.0) HIP_OK(launch_fill(g.col[i]->bufB, 0.0, LV(g.col[i], 0).N, g.st));
        else act.push_back(i);
    }
    if (act.empty()) return OMG_OK;
    auto outer_residual = [&](const std::vector<int>& a, std::vector<double>& rn) -> omg_status {
        const ColPtrs X = pack(a, [&](int c, int) { return g.col[c]->bufB; });
        const ColPtrs B = pack(a, [&](int c, int) { return g.col[c]->bufA; });
        const ColPtrs Y = pack(a, [&](int c, int) { return LV(g.col[c], 0).t2; });
        OMG_TRY(op_spmv(g, a, 0, false, X, &B, Y));
        return vec_norms(g, a, 0, Y, rn);
    };
    auto add_correction = [&](const std::vector<int>& a) -> omg_status {
        for (int c : a) HIP_OK(launch_axpy(g.col[c]->bufB, 1.0, LV(g.col[c], 0).xout, LV(g.col[c], 0).N, g.st));
        return OMG_OK;
    };
    auto inner = [&](const std::vector<int>& a, int mode) -> omg_status {
        for (int c : a) {
            HIP_OK(launch_copy(LV(g.col[c], 0).b, LV(g.col[c], 0).t2, LV(g.col[c], 0).N, g.st));
            g.col[c]->mode32 = mode;
        }
        omg_status e = mg_b(g, a, 0, P->opt.variant);
        for (int c : a) g.col[c]->mode32 = 0;
        return e;
    };
    if (P->opt.precision == OMG_MIXED_IR) {
        std::vector<int> outer(m, 0);
        while (!act.empty()) {
            std::vector<double> rn;
            OMG_TRY(outer_residual(act, rn));
            std::vector<int> next;
            for (size_t q = 0; q < act.size(); ++q) {
                const int i = act[q];
                R[i].rel_res_rec = rn[q] / bn[i];
                if (!std::isfinite(rn[q])) stat[i] = OMG_EINVAL;
                else if (rn[q] <= tol * bn[i]) continue;
                else if (outer[i] >= P->opt.max_outer) stat[i] = OMG_ENOCONV;
                else {
                    next.push_back(i);
                    g.tol[i] = P->opt.inner_tol;
                    g.stat[i] = OMG_OK;
                }
            }
            if (next.empty()) break;
            OMG_TRY(inner(next, 1));
            for (int i : next) {
                R[i].iters_fine += g.col[i]->visits.back();
                if (g.stat[i] == OMG_EINVAL) stat[i] = OMG_EINVAL;
            }
            OMG_TRY(add_correction(next));
            std::vector<int> keep;
            for (int i : next) {
                outer[i]++;
                if (stat[i] == OMG_OK) keep.push_back(i);
            }
            act.swap(keep);
        }
        for (int i = 0; i < m; ++i) R[i].outer_iters = outer[i];
        return OMG_OK;
    }
    std::vector<double> rn;
    OMG_TRY(outer_residual(act, rn));
    std::vector<int> go;
    for (size_t q = 0; q < act.size(); ++q) {
        const int i = act[q];
        if (!std::isfinite(rn[q])) stat[i] = OMG_EINVAL;
        else if (rn[q] > 0.0) {
            go.push_back(i);
            g.tol[i] = tol * bn[i] / rn[q];
        }
    }
    if (go.empty()) return OMG_OK;
    OMG_TRY(inner(go, (P->opt.precision == OMG_MIXED_FLEX) ? 2 : 0));
    OMG_TRY(add_correction(go));
    std::vector<double> rr;
    // members whose finest level is their coarsest were solved directly
    std::vector<int> ml;
    for (int i : go)
        if (!LV(g.col[i], 0).coarsest) ml.push_back(i);
    if (!ml.empty()) OMG_TRY(vec_norms(g, ml, 0, pack(ml, [&](int c, int) { return LV(g.col[c], 0).r; }), rr));
    for (size_t q = 0; q < ml.size(); ++q) {
        const int i = ml[q];
        R[i].iters_fine = g.col[i]->visits.back();
        R[i].rel_res_rec = rr[q] / bn[i];
    }
    for (int i : go)
        if (g.stat[i] != OMG_OK) stat[i] = g.stat[i];
    return OMG_OK;
}

// The abort flag of batched RM launches led by P (zero while all is well).
omg_status ensure_batch_flag(omg_solver* P) {
    if (P->babort) return OMG_OK;
    if (hipMalloc((void**)&P->babort, sizeof(unsigned)) != hipSuccess) return OMG_ENOMEM;
    HIP_OK(hipMemsetAsync(P->babort, 0, sizeof(unsigned), P->stream));
    return OMG_OK;
}

// After a batched solve: a raised abort flag means a bounded wait of a
// batched RM launch expired; the results are not trustworthy and later
// batched solves of P run RM one member at a time.
omg_status check_batch_flag(omg_solver* P) {
    unsigned f = 0;
    HIP_OK(hipMemcpy(&f, P->babort, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (f) {
        P->batch_rm_off = 1;
        return OMG_EHIP;
    }
    return OMG_OK;
}

// Column solvers and block copies of solver s for m columns.
omg_status prepare_columns(omg_solver* s, int m) {
    for (Level& L : s->lev) HIP_OK(build_blocks(L, s->bs, s->bsh, s->stream));
    while ((int)s->columns.size() < m) {
        omg_solver* c = nullptr;
        omg_status e = engine_make_column(s, &c);
        if (e != OMG_OK) {
            omg_destroy(c);
            return e;
        }
        s->columns.push_back(c);
    }
    // multi-column RM configuration for m columns
    for (int l = 0; l < s->nlev; ++l) {
        Level& L = s->lev[l];
        if (L.coarsest || !L.persist || L.rmc_multi_m == m) continue;
        L.rmc_multi = multi_config(L.rmc, L.N, m);
        L.rmc_multi_m = m;
    }
    // launch shapes of the multi-RHS kernels, tuned once per level and tile count
    const int ti = m > 16 ? 1 : 0;
    for (int l = 0; l < s->nlev; ++l) {
        Level& L = s->lev[l];
        if (L.coarsest || !L.dblk || L.mr_shape[0][0][ti]) continue;
        std::vector<int> all(m);
        for (int i = 0; i < m; ++i) all[i] = i;
        const ColPtrs X = pack(all, [&](int c, int) { return s->columns[c]->lev[l].t; });
        const ColPtrs Y = pack(all, [&](int c, int) { return s->columns[c]->lev[l].w; });
        const ColPtrs T = pack(all, [&](int c, int) { return s->columns[c]->lev[l].t2; });
        HIP_OK(tune_mr(L, s->bs, m, X, Y, T, 3, s->stream, nullptr));
        for (omg_solver* c : s->columns) std::memcpy(c->lev[l].mr_shape, L.mr_shape, sizeof(L.mr_shape));
    }
    return OMG_OK;
}

// (the lockstep engines run the block-Jacobi smoother, fixed smoother step
// counts and no restarts; other solvers are solved column by column)
bool lockstep_supported(const omg_solver* s) {
    return s->bs <= 16 && !s->owner && s->opt.smoother == OMG_SMOOTH_BJ && s->opt.n_s_max <= s->opt.n_s &&
           s->opt.m_max == 0;
}

// nrhs columns of one solver, in lockstep groups of up to kMaxCols.
omg_status solve_columns(omg_solver* s, const double* b, double* x, int nrhs, double tol, omg_report* rep,
                         omg_status* worst) {
    Level& L0 = s->lev[0];
    const int n = L0.n, bs = s->bs;
    for (int c0 = 0; c0 < nrhs; c0 += kMaxCols) {
        const int m = std::min(kMaxCols, nrhs - c0);
        auto t0 = std::chrono::steady_clock::now();
        OMG_TRY(prepare_columns(s, m));
        OMG_TRY(ensure_batch_flag(s));
        Group g;
        g.P = s;
        g.shared = true;
        g.st = s->stream;
        g.col.assign(s->columns.begin(), s->columns.begin() + m);
        std::vector<int> all(m);
        for (int i = 0; i < m; ++i) all[i] = i;
        const ColPtrs Bc = pack(all, [&](int c, int) { return g.col[c]->bufA; });
        const ColPtrs Xc = pack(all, [&](int c, int) { return g.col[c]->bufB; });
        const int64_t tot = (int64_t)n * bs * m;
        const dim3 gg((unsigned)((tot + 255) / 256)), blk(256);
        hipLaunchKernelGGL(k_gather_cols, gg, blk, 0, g.st, b, Bc, n, bs, nrhs, c0, m);
        hipLaunchKernelGGL(k_gather_cols, gg, blk, 0, g.st, x, Xc, n, bs, nrhs, c0, m);
        HIP_OK(hipGetLastError());
        std::vector<omg_report> R(m);
        for (auto& r : R) std::memset(&r, 0, sizeof(r));
        std::vector<omg_status> stat(m, OMG_OK);
        omg_status e = solve_group(g, tol, R, stat);
        if (e == OMG_OK) e = check_batch_flag(s);
        for (omg_solver* c : g.col) // launch counts of the per-column kernels
            for (int k = 0; k < OMG_K_COUNT; ++k)
                for (int l = 0; l < OMG_MAX_LEVELS; ++l) {
                    s->kcount[k][l] += c->kcount[k][l];
                    c->kcount[k][l] = 0;
                }
        OMG_TRY(e);
        hipLaunchKernelGGL(k_scatter_cols, gg, blk, 0, g.st, Xc, x, n, bs, nrhs, c0, m);
        HIP_OK(hipGetLastError());
        for (int i = 0; i < m; ++i)
            if (stat[i] == OMG_OK || stat[i] == OMG_ENOCONV)
                OMG_TRY(engine_finish_report(g.col[i], g.col[i]->bufA, g.col[i]->bufB, &R[i]));
        HIP_OK(hipStreamSynchronize(g.st));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int i = 0; i < m; ++i) {
            R[i].status = stat[i];
            R[i].t_solve_ms = ms;
            if (rep) rep[c0 + i] = R[i];
            if (stat[i] != OMG_OK && *worst == OMG_OK) *worst = stat[i];
        }
    }
    return OMG_OK;
}

// Cycle options that must agree for solvers advanced in lockstep.
bool same_cycle(const omg_solver* a, const omg_solver* b) {
    return a->bs == b->bs && a->stream == b->stream && a->opt.variant == b->opt.variant &&
           a->opt.s_pre == b->opt.s_pre && a->opt.s_post == b->opt.s_post && a->opt.n_s == b->opt.n_s &&
           a->opt.omega == b->opt.omega && a->opt.precision == b->opt.precision &&
           a->opt.coarse_sync == b->opt.coarse_sync && a->opt.max_outer == b->opt.max_outer &&
           a->opt.inner_tol == b->opt.inner_tol && a->opt.smoother == OMG_SMOOTH_BJ &&
           b->opt.smoother == OMG_SMOOTH_BJ && a->opt.n_s_max <= a->opt.n_s && b->opt.n_s_max <= b->opt.n_s &&
           a->opt.m_max == 0 && b->opt.m_max == 0 &&
           !a->owner && !b->owner;
}

// Independent solvers with one right-hand side each (b[i], x[i] cell-major),
// in lockstep groups of up to kMaxSeg: the streaming kernels of a step are one
// grouped launch over all members, each member getting a share of the grid
// proportional to its cells; RM runs per member.
omg_status solve_instances(omg_solver* const* s, int n, const double* const* b, double* const* x, double tol,
                           omg_report* rep, omg_status* worst) {
    for (int i0 = 0; i0 < n; i0 += kMaxSeg) {
        const int m = std::min(kMaxSeg, n - i0);
        auto t0 = std::chrono::steady_clock::now();
        Group g;
        g.P = s[i0];
        g.shared = false;
        g.st = g.P->stream;
        OMG_TRY(ensure_batch_flag(g.P));
        for (int i = 0; i < m; ++i) {
            omg_solver* si = s[i0 + i];
            g.col.push_back(si);
            HIP_OK(launch_to_soa(b[i0 + i], si->bufA, si->lev[0].n, si->bs, g.st));
            HIP_OK(launch_to_soa(x[i0 + i], si->bufB, si->lev[0].n, si->bs, g.st));
        }
        std::vector<omg_report> R(m);
        for (auto& r : R) std::memset(&r, 0, sizeof(r));
        std::vector<omg_status> stat(m, OMG_OK);
        OMG_TRY(solve_group(g, tol, R, stat));
        OMG_TRY(check_batch_flag(g.P));
        for (int i = 0; i < m; ++i) {
            omg_solver* si = g.col[i];
            HIP_OK(launch_from_soa(si->bufB, x[i0 + i], si->lev[0].n, si->bs, g.st));
            if (stat[i] == OMG_OK || stat[i] == OMG_ENOCONV)
                OMG_TRY(engine_finish_report(si, si->bufA, si->bufB, &R[i]));
        }
        HIP_OK(hipStreamSynchronize(g.st));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int i = 0; i < m; ++i) {
            R[i].status = stat[i];
            R[i].t_solve_ms = ms;
            if (rep) rep[i0 + i] = R[i];
            if (stat[i] != OMG_OK && *worst == OMG_OK) *worst = stat[i];
        }
    }
    return OMG_OK;
}

// One column at a time through the single-solve path (bs > 16).
__global__ void k_gather_col(const double* __restrict__ in, double* __restrict__ out, int n, int bs, int nrhs,
                             int col) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * bs) return;
    out[e] = in[e * nrhs + col];
}
__global__ void k_scatter_col(const double* __restrict__ in, double* __restrict__ out, int n, int bs, int nrhs,
                              int col) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * bs) return;
    out[e * nrhs + col] = in[e];
}

} // namespace

extern "C" omg_status omg_solve_batched(omg_solver* const* s, int32_t n_inst, int32_t nrhs, const double* const* b,
                                        double* const* x, double tol, omg_report* rep) {
    if (!s || n_inst < 1 || nrhs < 1 || !b || !x || !(tol >= 0.0)) return OMG_EINVAL;
    for (int i = 0; i < n_inst; ++i)
        if (!s[i] || !b[i] || !x[i]) return OMG_EINVAL;
    omg_status worst = OMG_OK;
    if (nrhs == 1 && n_inst > 1) {
        bool lock = true;
        for (int i = 1; i < n_inst; ++i) lock = lock && same_cycle(s[0], s[i]);
        for (int i = 0; i < n_inst && lock; ++i)
            for (int j = 0; j < i && lock; ++j) lock = s[i] != s[j]; // members need their own work vectors
        if (lock) {
            OMG_TRY(solve_instances(s, n_inst, b, x, tol, rep, &worst));
            return worst;
        }
    }
    for (int i = 0; i < n_inst; ++i) {
        omg_solver* si = s[i];
        omg_report* ri = rep ? rep + (size_t)i * nrhs : nullptr;
        if (lockstep_supported(si) && nrhs > 1) {
            OMG_TRY(solve_columns(si, b[i], x[i], nrhs, tol, ri, &worst));
            continue;
        }
        Level& L = si->lev[0];
        const int64_t N = L.N;
        double *bc = nullptr, *xc = nullptr;
        if (hipMalloc((void**)&bc, sizeof(double) * N) != hipSuccess) return OMG_ENOMEM;
        if (hipMalloc((void**)&xc, sizeof(double) * N) != hipSuccess) {
            hipFree(bc);
            return OMG_ENOMEM;
        }
        const dim3 g((unsigned)((N + 255) / 256)), blk(256);
        omg_status e = OMG_OK;
        for (int c = 0; c < nrhs && e == OMG_OK; ++c) {
            hipLaunchKernelGGL(k_gather_col, g, blk, 0, si->stream, b[i], bc, L.n, si->bs, nrhs, c);
            hipLaunchKernelGGL(k_gather_col, g, blk, 0, si->stream, x[i], xc, L.n, si->bs, nrhs, c);
            omg_report R;
            omg_status st = omg_solve(si, bc, xc, tol, nullptr, &R);
            if (st == OMG_EINVAL || st == OMG_EHIP || st == OMG_ENOMEM) e = st;
            hipLaunchKernelGGL(k_scatter_col, g, blk, 0, si->stream, xc, x[i], L.n, si->bs, nrhs, c);
            if (hipStreamSynchronize(si->stream) != hipSuccess) e = OMG_EHIP;
            if (ri) ri[c] = R;
            if (st != OMG_OK && worst == OMG_OK) worst = st;
        }
        hipFree(bc);
        hipFree(xc);
        OMG_TRY(e);
    }
    return worst;
}

// ------------------------------------------------------------------ inspection
extern "C" omg_status omg_level_tuning(const omg_solver* s, int32_t level, int32_t* shapes) {
    if (!s || level < 0 || level >= s->nlev || !shapes) return OMG_EINVAL;
    const Level& L = s->lev[level];
    int q = 0;
    for (int op = 0; op < 3; ++op)
        for (int f = 0; f < 2; ++f)
            for (int t = 0; t < 2; ++t) shapes[q++] = L.mr_shape[op][f][t] - 1;
    shapes[q++] = L.persist ? L.rmc.G : -1;
    shapes[q++] = L.persist ? L.rmc.ept : -1;
    shapes[q++] = L.persist ? L.rmc.B : -1;
    shapes[q++] = L.persist ? L.rmc.lead : -1;
    shapes[q++] = L.persist ? L.rmc.cw : -1;
    shapes[q++] = L.persist ? L.rmc.lag : -1;
    shapes[q++] = L.rm_dropped;
    return OMG_OK;
}

extern "C" omg_status omg_level_multi(omg_solver* s, int32_t level, int32_t op, int32_t nrhs, int32_t sweeps,
                                      int32_t fp32, const double* X, const double* B, double* Y) {
    if (!s || level < 0 || level >= s->nlev || nrhs < 1 || nrhs > kMaxCols || !X || !Y) return OMG_EINVAL;
    if (s->bs > 16 || s->owner) return OMG_EUNSUPPORTED;
    Level& L = s->lev[level];
    if (op == OMG_MR_SPMV) {
        if (L.coarsest && level > 0) return OMG_EUNSUPPORTED;
    } else if (op == OMG_MR_SMOOTHER) {
        if (L.coarsest || sweeps < 1) return OMG_EINVAL;
    } else if (op == OMG_MR_COARSE) {
        if (!L.coarsest || fp32) return OMG_EINVAL;
    } else {
        return OMG_EINVAL;
    }
    hipStream_t st = s->stream;
    HIP_OK(build_blocks(L, s->bs, s->bsh, st));
    const int64_t N = L.N;
    double* mem = nullptr;
    if (hipMalloc((void**)&mem, sizeof(double) * (size_t)N * 4 * nrhs) != hipSuccess) return OMG_ENOMEM;
    ColPtrs xs, bv, ys, ts;
    std::memset(&xs, 0, sizeof(xs));
    std::memset(&bv, 0, sizeof(bv));
    std::memset(&ys, 0, sizeof(ys));
    std::memset(&ts, 0, sizeof(ts));
    for (int j = 0; j < nrhs; ++j) {
        xs.p[j] = mem + (size_t)N * (4 * j);
        bv.p[j] = mem + (size_t)N * (4 * j + 1);
        ys.p[j] = mem + (size_t)N * (4 * j + 2);
        ts.p[j] = mem + (size_t)N * (4 * j + 3);
    }
    const int64_t tot = N * nrhs;
    const dim3 gg((unsigned)((tot + 255) / 256)), blk(256);
    omg_status res = OMG_OK;
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(k_gather_cols, gg, blk, 0, st, X, xs, L.n, s->bs, nrhs, 0, nrhs);
    if (B) hipLaunchKernelGGL(k_gather_cols, gg, blk, 0, st, B, bv, L.n, s->bs, nrhs, 0, nrhs);
    e = hipGetLastError();
    if (e == hipSuccess) {
        if (op == OMG_MR_SPMV) {
            e = launch_spmv_mr(L, s->bs, fp32 != 0, nrhs, xs, B ? &bv : nullptr, ys, st);
        } else if (op == OMG_MR_COARSE) {
            e = launch_dense_mr(L, nrhs, xs, ys, st);
        } else {
            const ColPtrs* bufs[2] = {&ys, &ts};
            int cur = (sweeps % 2 == 1) ? 0 : 1;
            e = launch_bj_first_mr(L, s->bs, fp32 != 0, s->opt.omega, nrhs, xs, *bufs[cur], st);
            for (int it = 1; it < sweeps && e == hipSuccess; ++it) {
                e = launch_bj_sweep_mr(L, s->bs, fp32 != 0, s->opt.omega, nrhs, xs, *bufs[cur], *bufs[cur ^ 1], st);
                cur ^= 1;
            }
        }
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_scatter_cols, gg, blk, 0, st, ys, Y, L.n, s->bs, nrhs, 0, nrhs);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        res = OMG_EHIP;
    }
    hipFree(mem);
    return res;
}
