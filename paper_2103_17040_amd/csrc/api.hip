// Host runtime of libtsm: validation, device buffers, setup, the per-step
// launch sequence (captured once in a hipGraph and replayed), outputs.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "tsm_internal.h"

using namespace tsm;

namespace {
// A roctx range over a library call, so that a marker trace of a profiler
// (rocprofv3 --marker-trace) shows set-up, steps, gradients and solves
// around their kernels.  Without a profiler attached the calls do nothing.
struct Range {
    explicit Range(const char* name) { roctxRangePush(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};
}  // namespace

namespace {

// Micro kernel classes: SLOTS nodes per lane with 256 lanes per workgroup.
const int kSlotClasses[] = {1, 2, 3, 5, 9, 17};

int slots_for(int n) {
    for (int s : kSlotClasses)
        if (s * kMicroThreads >= n) return s;
    return -1;
}

// Coarse levels of the multigrid hierarchy of an N-cell mesh: N = c 2^L with
// c <= kMgCoarsest and L >= 1, else 0 (no hierarchy).
int mg_levels_for(int N) {
    int L = 0, c = N;
    while (c > kMgCoarsest && c % 2 == 0 && L < kMgMaxLevels) {
        c /= 2;
        ++L;
    }
    return (L >= 1 && c <= kMgCoarsest) ? L : 0;
}

struct Group {
    int first;      // first task in the order array
    int count;
    int slots;
    int mode;       // 0 FP64 resident, 1 FP64 streamed, 2 refine resident, 3 refine streamed
    int max_level;
};

template <typename T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc((void**)p, count * sizeof(T));
}
template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace

struct tsm_ctx {
    tsm_params prm{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    int NM = 0, n_macro_int = 0;
    int64_t n_inst = 0, total = 0;
    std::vector<int32_t> level_h;
    std::vector<int64_t> off_h;
    std::vector<int32_t> order_h;
    std::vector<Group> groups;        // generic kernels: one launch per slot class
    int n_packs = 0;                  // packed kernels: one launch per mesh size
    std::vector<std::array<int, 3>> pack_groups;   // (level, first pack, pack count)
    int32_t *pk_first = nullptr, *pk_count = nullptr, *pk_level = nullptr, *queue = nullptr;
    int32_t* pk_slot_inst = nullptr;
    int64_t* pk_slot_off = nullptr;
    size_t pack_lds_max = 0;
    int64_t n_packed_tasks = 0;
    int n_cu = 0;

    // per instance
    int32_t *level = nullptr, *order = nullptr, *iters = nullptr, *sweeps = nullptr, *counters = nullptr;
    int64_t* order_off = nullptr;   // offsets[order[t]]
    int64_t *cell_off = nullptr, *bnd_off = nullptr;   // Jacobian tables per instance
    bool geom_tables = false;       // geometry from tsm_set_jacobians (no amplitude gradient)
    int64_t* offsets = nullptr;
    double *amp = nullptr, *beta = nullptr, *len = nullptr, *jmin = nullptr, *bx = nullptr,
           *alpha = nullptr, *F = nullptr, *u = nullptr;
    // ragged
    double *S64 = nullptr, *M64 = nullptr, *b = nullptr, *w = nullptr, *v0 = nullptr;
    double* Mw = nullptr;          // M_i w_i (packed step solves start from v0)
    // b at the boundary nodes, compact (kBndStride per instance, bnd_node order)
    double* bcomp = nullptr;
    // instances above kMaxLevel cells per side: the large-mesh kernel's
    // vectors (r, p, q: three ragged vectors per set; one set per stream
    // that runs micro solves side by side)
    double* lg_ws = nullptr;
    int lg_sets = 0;
    // FP64 recovery of packed refinement solves that miss rtol: the list
    // the packed kernels fill, and one workspace slot per workgroup
    int32_t* fb_list = nullptr;
    double* fb_ws = nullptr;
    int64_t fb_slot = 0;
    // history of the extrapolated start of the forward refinement solves:
    // the previous X0 and the two increments before it (FP32 per micro DoF)
    // and the number of steps they cover (device counter, advanced inside
    // the step graph)
    float* hx = nullptr;
    float* he = nullptr;
    float* he2 = nullptr;
    int32_t* hn = nullptr;
    // multigrid-preconditioned micro solves (stationary contexts with
    // TSM_FLAG_MULTIGRID): per-instance coarse levels, Galerkin operators,
    // coarsest inverses, damping, and per-stream workspaces
    int32_t* mg_nlev = nullptr;
    int64_t *mg_coff = nullptr, *mg_ioff = nullptr;
    double *mg_Ac = nullptr, *mg_inv = nullptr, *mg_omega = nullptr, *mg_ws = nullptr, *mg_cws = nullptr;
    int64_t mg_ctotal = 0;
    int mg_sets = 0;
    bool mg_ready = false;
    // an N-cell instance of this context is solved on the multigrid path:
    // by default the meshes above kMaxLevel cells per side (there the
    // alternative is one-workgroup Jacobi CG, whose iteration count grows
    // like N), every mesh with a hierarchy under TSM_FLAG_MULTIGRID, none
    // under TSM_FLAG_NO_MULTIGRID; stationary contexts only
    bool mg_use(int N) const {
        if (!stationary || (prm.flags & TSM_FLAG_NO_MULTIGRID) || mg_levels_for(N) == 0) return false;
        return N > kMaxLevel || (prm.flags & TSM_FLAG_MULTIGRID);
    }
    MgArgs mg_args(int set) const {
        MgArgs G{};
        G.nlev = mg_nlev;
        G.coff = mg_coff;
        G.ioff = mg_ioff;
        G.Ac = mg_Ac;
        G.inv = mg_inv;
        G.omega = mg_omega;
        G.ws = mg_ws + (int64_t)set * 5 * total;
        G.ws_stride = total;
        G.cws = mg_cws + (int64_t)set * 3 * mg_ctotal;
        G.cws_stride = mg_ctotal;
        G.nu = 2;
        return G;
    }
    void free_mg() {
        dfree(mg_nlev); dfree(mg_coff); dfree(mg_ioff); dfree(mg_Ac); dfree(mg_inv); dfree(mg_omega);
        dfree(mg_ws); dfree(mg_cws);
        mg_ctotal = 0;
        mg_sets = 0;
        mg_ready = false;
    }
    float *S32 = nullptr, *Slo = nullptr;
    // symmetric upper-half planes [kSym][n] of S, K = S - M/dt, M (FP32), S split in FP32
    double *Ss64 = nullptr, *Ks64 = nullptr;
    float *Ss32 = nullptr, *Sslo = nullptr;
    // tables
    int32_t* tab_off = nullptr;
    double *tab_y = nullptr, *tab_s = nullptr, *tab_c = nullptr;
    double* tab_m = nullptr;        // separable mass tables (MicroArgs::mass1d)
    // macro solver
    double *rhs = nullptr, *R = nullptr, *T1 = nullptr, *T2 = nullptr, *Q = nullptr, *lam = nullptr;
    int macro_sweeps = 2;
    double rho = 0.0;
    // macro PCG (sine-basis preconditioner): z, p (full grid), q, (r, z);
    // iteration count from the condition bound (0: A_M not shown SPD)
    double *mp_z = nullptr, *mp_p = nullptr, *mp_q = nullptr, *mp_s = nullptr;
    int macro_pcg_iters = 0;
    bool macro_pcg_cheaper = false;   // fewer operations than the sweeps at this contraction bound
    bool macro_pcg() const {
        return macro_pcg_iters > 0 && (rho >= 0.5 || macro_pcg_cheaper || (prm.flags & TSM_FLAG_MACRO_PCG));
    }
    // alternating (fixed-point) coupling: macro operator with beta = kappa p
    // (eigenvalues lam_fp), full micro state vf, rhs M v^n, previous macro
    // state, per-instance residual norms, the residual sum (2 values)
    double *lam_fp = nullptr, *beta_fp = nullptr, *vf = nullptr, *rvec = nullptr, *u_prev = nullptr,
           *resn = nullptr, *fpm = nullptr;
    int fp_iters_last = 0, fp_iters_max = 0;

    // adjoint work vectors (first tsm_gradient)
    double *lam0 = nullptr, *mu = nullptr, *coef = nullptr, *grad = nullptr, *Jd = nullptr;
    // history of the extrapolated start of the adjoint micro solves (lam0)
    float *lhx = nullptr, *lhe = nullptr, *lhe2 = nullptr;
    int32_t* lhn = nullptr;
    double grad_fwd_ms = 0.0, grad_bwd_ms = 0.0;

    // stationary three-field system (tsm_stationary_create): b holds b_I and
    // len |G^I|; b_O, |G^O|, the three micro solutions, the five
    // products per instance, w, the macro scratch and the iterations of the
    // three solves
    bool stationary = false;
    tsm_stationary_params sp{};
    double *st_bO = nullptr, *st_lenO = nullptr, *st_zI = nullptr, *st_zO = nullptr,
           *st_z0 = nullptr, *st_dots = nullptr, *st_w = nullptr, *st_work = nullptr, *st_info = nullptr;
    int32_t *st_iters = nullptr, *st_sweeps = nullptr;
    // loads: point weights of the geometry (wq J, wb |F tau|) and their
    // offsets, the micro load, part integrals, macro loads and Dirichlet
    // values; data at quadrature points given by tsm_stationary_set_data
    double *st_wcell = nullptr, *st_wbnd = nullptr, *st_Fv = nullptr, *st_GI = nullptr, *st_GO = nullptr,
           *st_Fu = nullptr, *st_Fw = nullptr, *st_uDn = nullptr;
    int64_t *st_wcoff = nullptr, *st_wboff = nullptr;
    int64_t st_ncell = 0, st_nbnd = 0;
    double *st_dfv = nullptr, *st_dgv = nullptr, *st_dfu = nullptr, *st_dfw = nullptr, *st_dgu = nullptr,
           *st_dgw = nullptr, *st_duD = nullptr;
    bool st_has[7] = {false, false, false, false, false, false, false};
    // the three micro solves run side by side: two more streams (default
    // priority), their work counters and the fork/join events
    hipStream_t st_side[2] = {nullptr, nullptr};
    int32_t* st_queue = nullptr;
    hipEvent_t st_ev[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_mid = nullptr;
    tsm_stationary_stats st_stats{};

    bool have_mesh = false, have_geom = false, have_state = false;
    hipGraphExec_t graph = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int64_t steps_taken = 0;
    double setup_ms = 0.0, step_ms = 0.0, micro_ms = 0.0, macro_ms = 0.0;
    int timed_steps = 0;
    std::vector<hipEvent_t> tev;   // TSM_FLAG_TIMING: 3 events per step

    tsm_status fail(tsm_status s, const std::string& m) {
        err = m;
        return s;
    }
    void free_mesh() {
        dfree(level); dfree(order); dfree(order_off); dfree(iters); dfree(sweeps); dfree(offsets);
        dfree(cell_off); dfree(bnd_off);
        geom_tables = false;
        dfree(Ss64); dfree(Ks64); dfree(Ss32); dfree(Sslo);
        dfree(amp); dfree(beta); dfree(len); dfree(jmin); dfree(bx); dfree(alpha); dfree(F); dfree(u);
        dfree(S64); dfree(M64); dfree(b); dfree(w); dfree(Mw); dfree(v0); dfree(S32); dfree(Slo);
        dfree(bcomp); dfree(lg_ws); dfree(fb_list); dfree(fb_ws); dfree(hx); dfree(he); dfree(he2); dfree(hn);
        lg_sets = 0;
        fb_slot = 0;
        free_mg();
        dfree(tab_off); dfree(tab_y); dfree(tab_s); dfree(tab_c); dfree(tab_m);
        dfree(pk_first); dfree(pk_count); dfree(pk_level); dfree(pk_slot_inst); dfree(pk_slot_off);
        dfree(lam0); dfree(mu); dfree(coef); dfree(grad); dfree(Jd); dfree(lhx); dfree(lhe); dfree(lhe2); dfree(lhn);
        dfree(st_bO); dfree(st_lenO); dfree(st_zI); dfree(st_zO); dfree(st_z0); dfree(st_dots);
        dfree(st_w); dfree(st_work); dfree(st_info); dfree(st_iters); dfree(st_sweeps);
        dfree(st_wcell); dfree(st_wbnd); dfree(st_Fv); dfree(st_GI); dfree(st_GO); dfree(st_Fu); dfree(st_Fw);
        dfree(st_uDn); dfree(st_wcoff); dfree(st_wboff);
        dfree(st_dfv); dfree(st_dgv); dfree(st_dfu); dfree(st_dfw); dfree(st_dgu); dfree(st_dgw); dfree(st_duD);
        for (bool& h : st_has) h = false;
        drop_graph();
        have_mesh = have_geom = have_state = false;
    }
    void free_macro() {
        dfree(rhs); dfree(R); dfree(T1); dfree(T2); dfree(Q); dfree(lam);
        dfree(mp_z); dfree(mp_p); dfree(mp_q); dfree(mp_s);
        dfree(lam_fp); dfree(beta_fp); dfree(vf); dfree(rvec); dfree(u_prev); dfree(resn); dfree(fpm);
    }
    void drop_graph() {
        if (graph) (void)hipGraphExecDestroy(graph);
        graph = nullptr;
    }
    MacroArgs macro_args() const {
        MacroArgs m;
        const double H = 1.0 / NM;
        m.NM = NM;
        m.n = NM - 1;
        m.mass_c = H * H / (36.0 * prm.dt);
        m.lap_c = prm.D / 3.0;
        m.sig_h2 = prm.source_sign * H * H;
        m.kappa = prm.kappa;
        m.p = prm.p;
        m.beta = beta;
        m.len = len;
        return m;
    }
};

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return c->fail(TSM_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define HIPALLOC(p, n)                                                                     \
    do {                                                                                   \
        hipError_t e_ = dalloc(&(p), (n));                                                 \
        if (e_ != hipSuccess) {                                                            \
            (void)hipGetLastError();                                                       \
            return c->fail(TSM_ENOMEM, std::string("allocation of ") + #p + " failed: " + hipGetErrorString(e_)); \
        }                                                                                  \
    } while (0)

namespace {

// One batched micro solve: the packed launch (16/32/64 cells) and one
// generic launch per remaining slot class.  setup: FP64 whatever the precision.
// On stream st with the persistent work counter queue (the context's own,
// or another for launches that run beside it).
tsm_status enqueue_micro(tsm_ctx* c, MicroArgs base, bool setup, hipStream_t st, int32_t* queue, int set = 0) {
    const bool refine = c->prm.precision == TSM_FP32_REFINE && !setup;
    // the packed refinement kernels read the operator assembled at setup;
    // per-size plans evaluate it from the amplitudes instead when asked
    // (TSM_FLAG_MATRIX_FREE; time-step form: right-hand side M x0/dt with
    // M w).  The persistent plans never do: a run of their matrix-free form
    // faulted the GPU and its cause is not found.
    const bool mf = refine && base.rhs_vec == nullptr && base.Mw != nullptr && !base.zero_init && !c->geom_tables &&
                    !c->stationary && (c->prm.flags & TSM_FLAG_MATRIX_FREE) &&
                    !(c->prm.flags & TSM_FLAG_PERSISTENT);
    const int pmode = refine ? (mf ? 3 : 2) : 1;
    // the packed kernels leave b^T x to one boundary pass over their instances
    MicroArgs pbase = base;
    pbase.bx_out = nullptr;
    // the extrapolated start (history of the forward step) belongs to the
    // packed kernels that read the assembled operator (FP64 and refinement)
    if (pmode == 3 || c->n_packs == 0) {
        pbase.hx = nullptr;
        pbase.he = nullptr;
        pbase.he2 = nullptr;
        pbase.hn = nullptr;
    }
    // the start residual of the packed kernels on the assembled operator
    // takes M x0 from the separable mass tables where the geometry is the
    // analytic family (not for Jacobian tables or the stationary system)
    pbase.mass1d = (pmode != 3 && !c->geom_tables && !c->stationary && !(c->prm.flags & TSM_FLAG_ASSEMBLED_START))
                       ? c->tab_m
                       : nullptr;
    // refinement solves that miss rtol are listed and solved again in FP64
    const bool fb = refine && c->n_packs > 0 && c->fb_list != nullptr && c->fb_ws != nullptr;
    if (fb) {
        pbase.fb_list = c->fb_list;
        HIPCHK(launch_fill_i32(c->fb_list, 0, 1, st));
    }
    if ((c->prm.flags & TSM_FLAG_PERSISTENT) && c->n_packs > 0) {
        // one persistent launch over every pack; the queue is reset by a
        // kernel so the sequence can be captured in a graph
        PackList pl{c->n_packs, c->pk_first, c->pk_count, c->pk_slot_inst, c->pk_slot_off};
        MicroArgs a = pbase;
        a.n_tasks = (int)c->n_inst;
        a.order = c->order;
        a.order_off = c->order_off;
        a.queue = queue;
        HIPCHK(launch_fill_i32(queue, 0, 1, st));
        const int grid = std::min(c->n_packs, c->n_cu);
        if (c->pack_groups.size() == 1)   // one mesh size: its own kernel, same queue
            HIPCHK(launch_packed(a, pl, c->pack_groups[0][0], pmode, grid, st));
        else
            HIPCHK(launch_packed_mixed(a, pl, c->pk_level, pmode, grid, c->pack_lds_max, st));
    } else {
        for (const auto& pg : c->pack_groups) {
            PackList pl{pg[2], c->pk_first + pg[1], c->pk_count + pg[1], c->pk_slot_inst + (int64_t)pg[1] * kPackSlots,
                        c->pk_slot_off + (int64_t)pg[1] * kPackSlots};
            MicroArgs a = pbase;
            a.n_tasks = (int)c->n_inst;
            a.order = c->order;
            a.order_off = c->order_off;
            HIPCHK(launch_packed(a, pl, pg[0], pmode, pg[2], st));
        }
    }
    if (pbase.hx != nullptr) HIPCHK(launch_history_advance(const_cast<int32_t*>(pbase.hn), st));
    if (fb) HIPCHK(launch_micro_fallback(pbase, c->fb_ws, c->fb_slot, c->n_cu, c->counters, st));
    if (c->n_packs > 0 && base.bx_out != nullptr)
        HIPCHK(launch_bdot_boundary((int)c->n_packed_tasks, c->order, c->level, c->offsets, c->bcomp, base.X_out,
                                    base.bx_out, st));
    for (const Group& g : c->groups) {
        MicroArgs a = base;
        a.n_tasks = g.count;
        a.order = c->order + g.first;
        if (g.slots == -2) {
            if (!c->mg_ready || set >= c->mg_sets) return c->fail(TSM_ESTATE, "multigrid hierarchy not built");
            MgArgs G = c->mg_args(set);
            HIPCHK(launch_micro_mg(a, G, st));
            continue;
        }
        if (g.slots < 0) {
            if (set >= c->lg_sets) return c->fail(TSM_EINVAL, "no large-mesh workspace for this stream");
            a.ws = c->lg_ws + (int64_t)set * 3 * c->total;
            a.ws_stride = c->total;
            HIPCHK(launch_micro_large(a, st));
            continue;
        }
        int mode = g.mode;
        if (setup) mode = (g.slots <= 5 && !(c->prm.flags & TSM_FLAG_STENCIL_STREAM)) ? 0 : 1;
        const int NP = g.max_level + 1;
        const size_t n_pad = (size_t)NP * NP + 2 * (size_t)(NP + 1);
        const size_t lds = n_pad * (sizeof(double) + sizeof(float));
        HIPCHK(launch_micro(a, g.slots, mode, g.count, lds, st));
    }
    return TSM_OK;
}

tsm_status enqueue_micro(tsm_ctx* c, MicroArgs base, bool setup) {
    return enqueue_micro(c, base, setup, c->stream, c->queue);
}

// Task order, packs and generic groups for the current mesh and flags.
tsm_status plan_tasks(tsm_ctx* c) {
    const int64_t n_inst = c->n_inst;
    const uint64_t fl = c->prm.flags;
    const bool use_packs = !(fl & TSM_FLAG_GENERIC);
    auto size_ok = [&](int lvl) {
        return !((lvl == 16 && (fl & TSM_FLAG_GENERIC_16)) || (lvl == 32 && (fl & TSM_FLAG_GENERIC_32)) ||
                 (lvl == 64 && (fl & TSM_FLAG_GENERIC_64)));
    };
    auto packable = [&](int32_t i) {
        const int lvl = c->level_h[i];
        return use_packs && packed_capacity(lvl) > 0 && size_ok(lvl) && !c->mg_use(lvl);
    };
    c->order_h.resize(n_inst);
    for (int64_t i = 0; i < n_inst; ++i) c->order_h[i] = (int32_t)i;
    // packable instances first, then by descending mesh size (largest first), stable
    std::stable_sort(c->order_h.begin(), c->order_h.end(), [&](int32_t x, int32_t y) {
        const bool px = packable(x), py = packable(y);
        if (px != py) return px;
        return c->level_h[x] > c->level_h[y];
    });
    std::vector<int32_t> pf, pc, pv;
    int64_t t = 0;
    c->pack_groups.clear();
    c->pack_lds_max = 0;
    while (t < n_inst && packable(c->order_h[t])) {
        const int lvl = c->level_h[c->order_h[t]];
        const int cap = packed_capacity(lvl);
        int cnt = 0;
        while (t + cnt < n_inst && cnt < cap && packable(c->order_h[t + cnt]) && c->level_h[c->order_h[t + cnt]] == lvl)
            ++cnt;
        if (c->pack_groups.empty() || c->pack_groups.back()[0] != lvl)
            c->pack_groups.push_back({lvl, (int)pf.size(), 0});
        c->pack_groups.back()[2]++;
        pf.push_back((int32_t)t);
        pc.push_back(cnt);
        pv.push_back(lvl);
        c->pack_lds_max = std::max(c->pack_lds_max, packed_lds_bytes(lvl));
        t += cnt;
    }
    c->n_packs = (int)pf.size();
    c->n_packed_tasks = t;     // the packed instances are order[0, t)
    c->groups.clear();
    const bool refine = c->prm.precision == TSM_FP32_REFINE;
    const bool stream_all = (c->prm.flags & TSM_FLAG_STENCIL_STREAM) != 0;
    for (; t < n_inst; ++t) {
        const int lvl = c->level_h[c->order_h[t]];
        // slots -2: the multigrid kernel; -1: above kMaxLevel, the large-mesh kernel
        const int sl = c->mg_use(lvl) ? -2
                       : lvl > kMaxLevel               ? -1
                                                       : slots_for((lvl + 1) * (lvl + 1));
        if (c->groups.empty() || c->groups.back().slots != sl) {
            Group g;
            g.first = (int)t;
            g.count = 0;
            g.slots = sl;
            const bool resident = !stream_all && (refine ? sl <= 9 : sl <= 5);
            g.mode = (refine ? 2 : 0) + (resident ? 0 : 1);
            g.max_level = lvl;
            c->groups.push_back(g);
        }
        c->groups.back().count++;
    }
    dfree(c->pk_first); dfree(c->pk_count); dfree(c->pk_level); dfree(c->pk_slot_inst); dfree(c->pk_slot_off);
    if (c->n_packs > 0) {
        HIPALLOC(c->pk_first, c->n_packs); HIPALLOC(c->pk_count, c->n_packs); HIPALLOC(c->pk_level, c->n_packs);
        const int64_t ns = (int64_t)c->n_packs * kPackSlots;
        std::vector<int32_t> si(ns, 0);
        std::vector<int64_t> so(ns, 0);
        for (int k = 0; k < c->n_packs; ++k)
            for (int q = 0; q < pc[k]; ++q) {
                const int32_t inst = c->order_h[pf[k] + q];
                si[(int64_t)k * kPackSlots + q] = inst;
                so[(int64_t)k * kPackSlots + q] = c->off_h[inst];
            }
        HIPALLOC(c->pk_slot_inst, ns); HIPALLOC(c->pk_slot_off, ns);
        HIPCHK(hipMemcpy(c->pk_slot_inst, si.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->pk_slot_off, so.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->pk_level, pv.data(), pv.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->pk_first, pf.data(), pf.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->pk_count, pc.data(), pc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    if (!c->order) HIPALLOC(c->order, n_inst);
    if (!c->order_off) HIPALLOC(c->order_off, n_inst);
    std::vector<int64_t> oo(n_inst);
    for (int64_t i = 0; i < n_inst; ++i) oo[i] = c->off_h[c->order_h[i]];
    HIPCHK(hipMemcpy(c->order, c->order_h.data(), n_inst * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->order_off, oo.data(), n_inst * sizeof(int64_t), hipMemcpyHostToDevice));
    return TSM_OK;
}

MicroArgs micro_base(tsm_ctx* c) {
    MicroArgs a{};
    a.level = c->level;
    a.offsets = c->offsets;
    a.S64 = c->S64;
    a.S32 = c->S32;
    a.Slo = c->Slo;
    a.M64 = c->M64;
    a.Ss64 = c->Ss64;
    a.Ks64 = c->Ks64;
    a.Ss32 = c->Ss32;
    a.Sslo = c->Sslo;
    a.b = c->b;
    a.w = c->w;
    a.bx_out = c->bx;
    a.iters_out = c->iters;
    a.sweeps_out = c->sweeps;
    a.nonconv = c->counters;
    a.inv_dt = 1.0 / c->prm.dt;
    a.rtol = c->prm.rtol;
    a.inner_rtol = c->prm.inner_rtol;
    a.max_iter = c->prm.max_iter;
    a.max_refine = c->prm.max_refine;
    a.queue = nullptr;
    a.amp = c->amp;
    a.tab = Tables{c->tab_off, c->tab_y, c->tab_s, c->tab_c};
    a.d = c->prm.d;
    a.kappa = c->prm.kappa;
    return a;
}

// Macro solve of A_M u = rhs in place (u holds the initial guess).
// Sweeps u <- u + A0^{-1} (rhs - A_M u) of the macro solve; A_M from m (its
// beta), A0^{-1} by the sine basis and the eigenvalues lam.
tsm_status enqueue_macro_solve(tsm_ctx* c, double* u, const MacroArgs& m, const double* lam, int sweeps) {
    const int n = m.n;
    for (int s = 0; s < sweeps; ++s) {
        HIPCHK(launch_macro_residual(m, u, c->rhs, c->R, c->stream));
        HIPCHK(launch_gemm(n, c->Q, c->R, c->T1, 0, nullptr, nullptr, c->NM, c->stream));
        HIPCHK(launch_gemm(n, c->T1, c->Q, c->T2, 1, lam, nullptr, c->NM, c->stream));
        HIPCHK(launch_gemm(n, c->Q, c->T2, c->T1, 0, nullptr, nullptr, c->NM, c->stream));
        HIPCHK(launch_gemm(n, c->T1, c->Q, nullptr, 2, nullptr, u, c->NM, c->stream));
    }
    return TSM_OK;
}

// Macro solve of A_M u = rhs in place by PCG with A0^{-1} (sine basis) as
// preconditioner, a fixed number of iterations (from the condition bound,
// so the sequence can be captured in a graph).
tsm_status enqueue_macro_pcg(tsm_ctx* c, double* u) {
    const MacroArgs m = c->macro_args();
    const int n = m.n, NM = c->NM;
    hipStream_t s = c->stream;
    if (macro_pcg_fused_fits(NM)) {
        HIPCHK(launch_macro_pcg_fused(m, u, c->rhs, c->Q, c->lam, c->macro_pcg_iters, s));
        return TSM_OK;
    }
    auto precondition = [&]() -> hipError_t {     // z = A0^{-1} r
        hipError_t e = launch_gemm(n, c->Q, c->R, c->T1, 0, nullptr, nullptr, NM, s);
        if (e == hipSuccess) e = launch_gemm(n, c->T1, c->Q, c->T2, 1, c->lam, nullptr, NM, s);
        if (e == hipSuccess) e = launch_gemm(n, c->Q, c->T2, c->T1, 0, nullptr, nullptr, NM, s);
        if (e == hipSuccess) e = launch_gemm(n, c->T1, c->Q, c->mp_z, 0, nullptr, nullptr, NM, s);
        return e;
    };
    HIPCHK(launch_macro_residual(m, u, c->rhs, c->R, s));
    HIPCHK(precondition());
    HIPCHK(launch_macro_pcg_start(NM, c->R, c->mp_z, c->mp_p, c->mp_s, s));
    for (int it = 0; it < c->macro_pcg_iters; ++it) {
        HIPCHK(launch_macro_pcg_step(m, c->mp_p, c->mp_q, c->R, u, c->mp_s, s));
        if (it + 1 == c->macro_pcg_iters) break;
        HIPCHK(precondition());
        HIPCHK(launch_macro_pcg_direction(NM, c->R, c->mp_z, c->mp_p, c->mp_s, s));
    }
    return TSM_OK;
}

tsm_status enqueue_macro_solve(tsm_ctx* c, double* u) {
    if (c->macro_pcg()) return enqueue_macro_pcg(c, u);
    return enqueue_macro_solve(c, u, c->macro_args(), c->lam, c->macro_sweeps);
}

// One forward step: micro solves (state v = v0 + u w in place), macro solve, fluxes.
// ev (optional, 3 events) brackets the micro and macro phases.
tsm_status enqueue_step(tsm_ctx* c, const hipEvent_t* ev = nullptr) {
    if (ev) HIPCHK(hipEventRecord(ev[0], c->stream));
    MicroArgs a = micro_base(c);
    a.X0 = c->v0;
    a.coef = c->u;
    a.Mw = c->Mw;
    a.rhs_vec = nullptr;
    a.zero_init = 0;
    a.X_out = c->v0;
    if (c->hx != nullptr && !(c->prm.flags & TSM_FLAG_NO_EXTRAPOLATION)) {
        a.hx = c->hx;
        a.he = c->he;
        a.he2 = c->he2;
        a.hn = c->hn;
    }
    tsm_status st = enqueue_micro(c, a, false);
    if (st != TSM_OK) return st;
    if (ev) HIPCHK(hipEventRecord(ev[1], c->stream));
    const MacroArgs m = c->macro_args();
    HIPCHK(launch_macro_rhs_forward(m, c->u, c->bx, c->rhs, c->alpha, c->stream));
    st = enqueue_macro_solve(c, c->u);
    if (st != TSM_OK) return st;
    HIPCHK(launch_macro_finalize(m, c->u, c->alpha, c->F, c->stream));
    if (ev) HIPCHK(hipEventRecord(ev[2], c->stream));
    return TSM_OK;
}

// One step of the paper's alternating coupling (Section 3.3): the macro
// solve with the micro data lagged (A_fp u = M_H u^n/dt + sign L alpha(v^k),
// A_fp = M_H/dt + D K_H - sign kappa p L, solved exactly by the sine basis),
// then every micro solve with the new macro values
// (S_i v_i = M_i v_i^n/dt + kappa p u_i b_i, previous iterate as the guess),
// until the residual sum (macro residual norm + mean micro residual norm)
// changes by less than fp_rtol times its first value.  The test runs on the
// host: one synchronisation per iteration.
tsm_status step_fixed_point(tsm_ctx* c) {
    const int64_t ni = c->n_inst, tot = c->total;
    if (!c->vf) {
        HIPALLOC(c->vf, tot); HIPALLOC(c->rvec, tot); HIPALLOC(c->u_prev, ni);
        HIPALLOC(c->resn, ni); HIPALLOC(c->fpm, 2);
    }
    hipStream_t s = c->stream;
    MacroArgs m = c->macro_args();
    m.beta = c->beta_fp;
    const int nR = m.n * m.n;
    HIPCHK(launch_state_join((int)ni, c->offsets, c->u, c->v0, c->w, c->vf, s));          // v^n
    HIPCHK(launch_apply((int)ni, c->level, c->offsets, c->M64, c->vf, c->rvec, s));       // M v^n
    HIPCHK(hipMemcpyAsync(c->u_prev, c->u, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_bdot((int)ni, c->offsets, c->b, c->vf, c->bx, s));
    double first = 0.0, prev = 0.0;
    int it = 0;
    while (it < c->prm.fp_max_iter) {
        ++it;
        HIPCHK(launch_macro_rhs_forward(m, c->u_prev, c->bx, c->rhs, c->alpha, s));
        tsm_status st = enqueue_macro_solve(c, c->u, m, c->lam_fp, 2);
        if (st != TSM_OK) return st;
        MicroArgs a = micro_base(c);
        a.X0 = c->vf;
        a.coef = nullptr;
        a.zero_init = 0;
        a.rhs_vec = c->rvec;
        a.rhs_scale = 1.0 / c->prm.dt;
        a.rhs_bcoef = c->u;
        a.rhs_bscale = c->prm.kappa * c->prm.p;
        a.X_out = c->vf;
        a.res_out = c->resn;
        st = enqueue_micro(c, a, false);
        if (st != TSM_OK) return st;
        // residual sum of (u^{k+1}, v^{k+1}); alpha is left for the fluxes
        HIPCHK(launch_macro_rhs_forward(m, c->u_prev, c->bx, c->rhs, c->alpha, s));
        HIPCHK(launch_macro_residual(m, c->u, c->rhs, c->R, s));
        HIPCHK(launch_coupling_residual(nR, c->R, (int)ni, c->resn, c->fpm, s));
        double h[2];
        HIPCHK(hipMemcpyAsync(h, c->fpm, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double res = h[0] + h[1];
        if (!std::isfinite(res)) return c->fail(TSM_ENOCONV, "fixed-point coupling: residual sum is not finite");
        if (it == 1) first = res;
        else if (std::fabs(res - prev) <= c->prm.fp_rtol * first) break;
        prev = res;
    }
    HIPCHK(launch_macro_finalize(m, c->u, c->alpha, c->F, s));                         // F = kappa p u + alpha
    HIPCHK(launch_state_split((int)ni, c->offsets, c->u, c->vf, c->w, c->v0, s));       // back to (v0, u)
    c->fp_iters_last = it;
    c->fp_iters_max = std::max(c->fp_iters_max, it);
    return TSM_OK;
}

// The history of the extrapolated start no longer follows the state: the
// next steps start without it (a fill kernel on the context's stream).
tsm_status reset_history(tsm_ctx* c) {
    if (c->hn != nullptr) HIPCHK(launch_fill_i32(c->hn, 0, 1, c->stream));
    return TSM_OK;
}

tsm_status build_graph(tsm_ctx* c) {
    c->drop_graph();
    if (c->prm.flags & (TSM_FLAG_NO_GRAPH | TSM_FLAG_TIMING | TSM_FLAG_FIXED_POINT)) return TSM_OK;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    tsm_status st = enqueue_step(c);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st != TSM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HIPCHK(e);
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    return TSM_OK;
}

bool finite_all(const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

}  // namespace

extern "C" {

void tsm_default_params(tsm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->macro_cells = 8;
    p->D = 1.0;
    p->d = 0.5;
    p->kappa = 1.0;
    p->p = 1.0;
    p->dt = 0.01;
    p->source_sign = -1;
    p->precision = TSM_FP64;
    p->rtol = 1e-12;
    p->inner_rtol = 1e-2;
    p->setup_rtol = 1e-14;
    p->max_iter = 1000;
    p->max_refine = 12;
    p->checkpoint_every = 10;
    p->flags = 0;
    p->fp_rtol = 1e-10;
    p->fp_max_iter = 50;
    p->grad_rtol = 0.0;
}

namespace {
thread_local std::string g_create_error = "no error";   // tsm_last_error(NULL)

tsm_status create_failed(tsm_ctx* c, tsm_status st, const std::string& msg) {
    g_create_error = msg;
    if (c) tsm_destroy(c);
    return st;
}
}  // namespace

extern "C++" {
namespace tsm {
tsm_status call_failed(tsm_status st, const std::string& msg) {
    g_create_error = msg;
    return st;
}
}  // namespace tsm
}  // extern "C++"

tsm_status tsm_create(const tsm_params* p, void* stream, tsm_ctx** out) {
    if (!out) return create_failed(nullptr, TSM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return create_failed(nullptr, TSM_EINVAL, "params is NULL");
    const bool ok = p->macro_cells >= 2 && p->macro_cells <= 1024 && p->D > 0 && p->d > 0 && p->kappa >= 0 &&
                    p->p > 0 && p->dt > 0 && (p->source_sign == 1 || p->source_sign == -1) &&
                    (p->precision == TSM_FP64 || p->precision == TSM_FP32_REFINE) && p->rtol > 0 &&
                    p->inner_rtol > 0 && p->inner_rtol < 1 && p->setup_rtol > 0 && p->max_iter >= 1 &&
                    p->max_refine >= 1 && p->checkpoint_every >= 1 && p->fp_rtol > 0 && p->fp_max_iter >= 2 && p->grad_rtol >= 0 && std::isfinite(p->grad_rtol) && std::isfinite(p->D) &&
                    std::isfinite(p->d) && std::isfinite(p->kappa) && std::isfinite(p->p) && std::isfinite(p->dt);
    if (!ok) return create_failed(nullptr, TSM_EINVAL, "parameter out of range");
    tsm_ctx* c = new tsm_ctx();
    c->prm = *p;
    c->NM = p->macro_cells;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        const hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return create_failed(nullptr, TSM_EHIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
        }
        c->own_stream = true;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return create_failed(c, TSM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || c->n_cu <= 0)
        return create_failed(c, TSM_EHIP, std::string("compute unit count: ") + hipGetErrorString(e));
    if ((e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess ||
        (e = dalloc(&c->counters, 4)) != hipSuccess || (e = dalloc(&c->queue, 1)) != hipSuccess) {
        (void)hipGetLastError();
        return create_failed(c, TSM_EHIP, std::string("context resources: ") + hipGetErrorString(e));
    }
    g_create_error = "no error";
    *out = c;
    return TSM_OK;
}

tsm_status tsm_set_reference_mesh(tsm_ctx* c, const int32_t* micro_cells, int64_t n_inst) {
    const Range range("tsm_set_reference_mesh");
    if (!c) return TSM_EINVAL;
    if (!micro_cells) return c->fail(TSM_EINVAL, "micro_cells is NULL");
    const int64_t expect = (int64_t)(c->NM + 1) * (c->NM + 1);
    if (n_inst != expect)
        return c->fail(TSM_EINVAL, "n_inst must equal (macro_cells+1)^2 = " + std::to_string(expect));
    for (int64_t i = 0; i < n_inst; ++i)
        if (micro_cells[i] < kMinLevel || micro_cells[i] > kMaxMesh)
            return c->fail(TSM_EINVAL, "micro_cells[" + std::to_string(i) + "] = " + std::to_string(micro_cells[i]) +
                                           " outside 2..256");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->free_mesh();
    c->free_macro();
    c->n_inst = n_inst;
    c->level_h.assign(micro_cells, micro_cells + n_inst);
    c->off_h.assign(n_inst + 1, 0);
    for (int64_t i = 0; i < n_inst; ++i) c->off_h[i + 1] = c->off_h[i] + (int64_t)(micro_cells[i] + 1) * (micro_cells[i] + 1);
    c->total = c->off_h[n_inst];

    // level tables
    std::vector<int32_t> toff(kMaxMesh + 1, 0);
    std::vector<double> ty, ts, tc;
    std::vector<bool> present(kMaxMesh + 1, false);
    for (int32_t l : c->level_h) present[l] = true;
    const double g0 = 0.5 - 0.5 / std::sqrt(3.0), g1 = 0.5 + 0.5 / std::sqrt(3.0);
    for (int N = kMinLevel; N <= kMaxMesh; ++N) {
        if (!present[N]) continue;
        toff[N] = (int32_t)ty.size();
        const double h = 2.0 / N;
        for (int t = 0; t < 2 * N + 2; ++t) {
            double y;
            if (t < 2 * N) y = -1.0 + ((t / 2) + ((t % 2) ? g1 : g0)) * h;
            else y = (t == 2 * N) ? -1.0 : 1.0;
            ty.push_back(y);
            ts.push_back(0.25 * std::sin(M_PI * y));
            tc.push_back(0.25 * M_PI * std::cos(M_PI * y));
        }
    }
    // separable mass tables (MicroArgs::mass1d), 16 (N+1) = 8 (2N+2) doubles
    // a level, so level N starts at 8 tab_off[N]: for each weight function f
    // (1, c, y, c y, s of the Gauss abscissa) the 1D Q1 mass
    // m_jk = (h/2) sum_g f(y_g) phi_j(y_g) phi_k(y_g) over the cells, stored
    // per node j as the planes (3 f + d + 1) of k = j + d
    std::vector<double> tm(8 * ty.size(), 0.0);
    for (int N = kMinLevel; N <= kMaxMesh; ++N) {
        if (!present[N]) continue;
        const int NP = N + 1, t0 = toff[N];
        double* m = tm.data() + 8 * (size_t)t0;
        const double wh = 1.0 / N;     // h / 2
        for (int f = 0; f < 5; ++f)
            for (int e = 0; e < N; ++e) {
                double m00 = 0.0, m01 = 0.0, m11 = 0.0;
                for (int g = 0; g < 2; ++g) {
                    const int t = t0 + 2 * e + g;
                    const double y = ty[t], fv = f == 0 ? 1.0 : f == 1 ? tc[t] : f == 2 ? y : f == 3 ? tc[t] * y : ts[t];
                    const double p1 = g ? g1 : g0, p0 = 1.0 - p1;
                    m00 += wh * fv * p0 * p0;
                    m01 += wh * fv * p0 * p1;
                    m11 += wh * fv * p1 * p1;
                }
                m[(3 * f + 1) * NP + e] += m00;
                m[(3 * f + 2) * NP + e] = m01;
                m[(3 * f + 0) * NP + e + 1] = m01;
                m[(3 * f + 1) * NP + e + 1] += m11;
            }
    }

    const int64_t ni = n_inst, tot = c->total;
    HIPALLOC(c->level, ni); HIPALLOC(c->iters, ni); HIPALLOC(c->sweeps, ni);
    HIPALLOC(c->offsets, ni + 1);
    HIPALLOC(c->amp, ni); HIPALLOC(c->beta, ni); HIPALLOC(c->len, ni); HIPALLOC(c->jmin, ni);
    HIPALLOC(c->bx, ni); HIPALLOC(c->alpha, ni); HIPALLOC(c->F, ni); HIPALLOC(c->u, ni);
    HIPALLOC(c->S64, kStencil * tot); HIPALLOC(c->M64, kStencil * tot); HIPALLOC(c->S32, kStencil * tot);
    HIPALLOC(c->Slo, kStencil * tot);
    // symmetric planes: kPlanePad zeroed entries past the last instance
    // (the packed kernels read past an instance's block for strip rows past
    // its mesh and discard the products)
    const int64_t np = kSym * tot + kPlanePad;
    HIPALLOC(c->Ss64, np); HIPALLOC(c->Ks64, np);
    HIPALLOC(c->Ss32, np); HIPALLOC(c->Sslo, np);
    const int64_t pe = kSym * tot;     // the assembly writes every entry before it
    HIPCHK(hipMemset(c->Ss64 + pe, 0, kPlanePad * sizeof(double)));
    HIPCHK(hipMemset(c->Ks64 + pe, 0, kPlanePad * sizeof(double)));
    HIPCHK(hipMemset(c->Ss32 + pe, 0, kPlanePad * sizeof(float)));
    HIPCHK(hipMemset(c->Sslo + pe, 0, kPlanePad * sizeof(float)));
    HIPALLOC(c->b, tot); HIPALLOC(c->w, tot); HIPALLOC(c->v0, tot); HIPALLOC(c->Mw, tot);
    HIPALLOC(c->bcomp, ni * kBndStride);
    if (*std::max_element(c->level_h.begin(), c->level_h.end()) > kMaxLevel) {
        // the three micro solves of a stationary context run side by side
        c->lg_sets = c->stationary ? 3 : 1;
        HIPALLOC(c->lg_ws, (size_t)c->lg_sets * 3 * tot);
    }
    if (c->prm.precision == TSM_FP32_REFINE) {
        int nmax = 0;
        for (int32_t l : c->level_h)
            if (l <= kMaxLevel) nmax = std::max(nmax, (l + 1) * (l + 1));
        c->fb_slot = nmax;
        HIPALLOC(c->fb_list, ni + 1);
        if (nmax > 0) HIPALLOC(c->fb_ws, (size_t)c->n_cu * 3 * nmax);
    }
    if (!c->stationary) {
        HIPALLOC(c->hx, tot); HIPALLOC(c->he, tot); HIPALLOC(c->he2, tot); HIPALLOC(c->hn, 1);
        HIPCHK(launch_fill_i32(c->hn, 0, 1, c->stream));
    }
    if (c->stationary) {
        HIPALLOC(c->st_bO, tot); HIPALLOC(c->st_lenO, ni);
        HIPALLOC(c->st_zI, tot); HIPALLOC(c->st_zO, tot); HIPALLOC(c->st_z0, tot);
        HIPALLOC(c->st_dots, 5 * ni); HIPALLOC(c->st_w, ni); HIPALLOC(c->st_work, 11 * ni);
        HIPALLOC(c->st_info, 2); HIPALLOC(c->st_iters, 3 * ni); HIPALLOC(c->st_sweeps, 3 * ni);
        std::vector<int64_t> wco(ni), wbo(ni);
        int64_t nc = 0, nb = 0;
        for (int64_t i = 0; i < ni; ++i) {
            const int64_t N = c->level_h[i];
            wco[i] = nc;
            wbo[i] = nb;
            nc += 4 * N * N;
            nb += 8 * N;
        }
        c->st_ncell = nc;
        c->st_nbnd = nb;
        HIPALLOC(c->st_wcell, nc); HIPALLOC(c->st_wbnd, nb); HIPALLOC(c->st_wcoff, ni); HIPALLOC(c->st_wboff, ni);
        HIPCHK(hipMemcpy(c->st_wcoff, wco.data(), ni * sizeof(int64_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->st_wboff, wbo.data(), ni * sizeof(int64_t), hipMemcpyHostToDevice));
        HIPALLOC(c->st_Fv, tot); HIPALLOC(c->st_GI, ni); HIPALLOC(c->st_GO, ni);
        HIPALLOC(c->st_Fu, ni); HIPALLOC(c->st_Fw, ni); HIPALLOC(c->st_uDn, ni);
    }
    HIPALLOC(c->tab_off, kMaxMesh + 1); HIPALLOC(c->tab_y, ty.size()); HIPALLOC(c->tab_s, ts.size());
    HIPALLOC(c->tab_c, tc.size()); HIPALLOC(c->tab_m, tm.size());
    HIPCHK(hipMemcpy(c->level, c->level_h.data(), ni * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->offsets, c->off_h.data(), (ni + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->tab_off, toff.data(), toff.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->tab_y, ty.data(), ty.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->tab_s, ts.data(), ts.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->tab_c, tc.data(), tc.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->tab_m, tm.data(), tm.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(c->u, 0, ni * sizeof(double)));
    HIPCHK(hipMemset(c->F, 0, ni * sizeof(double)));
    HIPCHK(hipMemset(c->v0, 0, tot * sizeof(double)));

    {
        tsm_status ps = plan_tasks(c);
        if (ps != TSM_OK) return ps;
    }
    const int n = c->NM - 1;
    HIPALLOC(c->rhs, (size_t)n * n); HIPALLOC(c->R, (size_t)n * n); HIPALLOC(c->T1, (size_t)n * n);
    HIPALLOC(c->T2, (size_t)n * n); HIPALLOC(c->Q, (size_t)n * n); HIPALLOC(c->lam, (size_t)n * n);
    HIPALLOC(c->lam_fp, (size_t)n * n);
    HIPALLOC(c->mp_z, (size_t)n * n); HIPALLOC(c->mp_q, (size_t)n * n);
    HIPALLOC(c->mp_p, (size_t)(n + 2) * (n + 2)); HIPALLOC(c->mp_s, 4);
    c->have_mesh = true;
    return TSM_OK;
}

tsm_status tsm_get_offsets(const tsm_ctx* c, int64_t* out) {
    if (!c || !out) return TSM_EINVAL;
    if (!c->have_mesh) return TSM_ESTATE;
    std::memcpy(out, c->off_h.data(), (c->n_inst + 1) * sizeof(int64_t));
    return TSM_OK;
}

extern "C++" {
namespace {

// Everything after the assembly, shared by both geometry inputs: the det
// check, the responses w_i, beta, the macro solver and the step graph.
// what(i) describes instance i for the geometry error message.
// Assembly arguments of the context's operator: S = M/dt + d A + kappa B
// with b = B 1 (time-dependent system), or S = Dv A + k2 B^I + k4 B^O with
// b = b_I, b2 = b_O and the point weights for the loads (stationary system).
AssembleArgs assemble_base(tsm_ctx* c) {
    AssembleArgs as{};
    as.n_inst = (int)c->n_inst;
    as.level = c->level;
    as.offsets = c->offsets;
    as.amp = c->amp;
    as.tab = Tables{c->tab_off, c->tab_y, c->tab_s, c->tab_c};
    as.S64 = c->S64; as.S32 = c->S32; as.Slo = c->Slo; as.M64 = c->M64; as.b = c->b; as.len = c->len; as.jmin = c->jmin;
    as.Ss64 = c->Ss64; as.Ks64 = c->Ks64; as.Ss32 = c->Ss32; as.Sslo = c->Sslo;
    if (!c->stationary) {
        as.d = c->prm.d;
        as.inv_dt = 1.0 / c->prm.dt;
        for (int s = 0; s < 4; ++s) {
            as.kside[s] = c->prm.kappa;
            as.bw[s] = 1.0;
            as.bw2[s] = 0.0;
        }
    } else {
        as.d = c->sp.Dv;
        as.inv_dt = 0.0;
        for (int s = 0; s < 4; ++s) {
            const int part = c->sp.parts[s];
            as.kside[s] = part == TSM_PART_I ? c->sp.kappa2 : part == TSM_PART_O ? c->sp.kappa4 : 0.0;
            as.bw[s] = part == TSM_PART_I ? 1.0 : 0.0;
            as.bw2[s] = part == TSM_PART_O ? 1.0 : 0.0;
        }
        as.b2 = c->st_bO;
        as.len2 = c->st_lenO;
        as.wcell = c->st_wcell;
        as.wbnd = c->st_wbnd;
        as.wc_off = c->st_wcoff;
        as.wb_off = c->st_wboff;
    }
    return as;
}

// The multigrid hierarchy of a stationary context from its assembled
// operators: levels, offsets, Galerkin operators, damping, coarsest inverses.
tsm_status mg_setup(tsm_ctx* c) {
    c->free_mg();
    const int64_t ni = c->n_inst;
    std::vector<int32_t> nl(ni);
    std::vector<int64_t> co(ni), io(ni);
    int64_t ct = 0, it = 0;
    int lmax = 0;
    for (int64_t i = 0; i < ni; ++i) {
        const int N = c->level_h[i];
        const int L = c->mg_use(N) ? mg_levels_for(N) : 0;
        nl[i] = L;
        co[i] = ct;
        io[i] = it;
        for (int l = 1; l <= L; ++l) ct += (int64_t)((N >> l) + 1) * ((N >> l) + 1);
        if (L > 0) {
            const int64_t nc = (int64_t)((N >> L) + 1) * ((N >> L) + 1);
            it += nc * nc;
        }
        lmax = std::max(lmax, L);
    }
    if (lmax == 0) return TSM_OK;      // no instance has a hierarchy: nothing runs on this path
    HIPALLOC(c->mg_nlev, ni); HIPALLOC(c->mg_coff, ni); HIPALLOC(c->mg_ioff, ni);
    HIPALLOC(c->mg_Ac, (size_t)kStencil * ct); HIPALLOC(c->mg_inv, (size_t)it);
    HIPALLOC(c->mg_omega, (size_t)ni * (kMgMaxLevels + 1));
    c->mg_sets = 3;                    // the three micro solves run side by side
    c->mg_ctotal = ct;
    HIPALLOC(c->mg_ws, (size_t)c->mg_sets * 5 * c->total); HIPALLOC(c->mg_cws, (size_t)c->mg_sets * 3 * ct);
    HIPCHK(hipMemcpy(c->mg_nlev, nl.data(), ni * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->mg_coff, co.data(), ni * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->mg_ioff, io.data(), ni * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(c->mg_omega, 0, (size_t)ni * (kMgMaxLevels + 1) * sizeof(double)));
    HIPCHK(launch_mg_setup(micro_base(c), c->mg_args(0), (int)ni, lmax, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->mg_ready = true;
    return TSM_OK;
}

template <class What>
tsm_status finish_setup(tsm_ctx* c, std::chrono::steady_clock::time_point t0, What what) {
    const int64_t n_inst = c->n_inst;
    HIPCHK(launch_bnd_gather((int)n_inst, c->level, c->offsets, c->b, c->bcomp, c->stream));
    std::vector<double> jm(n_inst);
    HIPCHK(hipMemcpyAsync(jm.data(), c->jmin, n_inst * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n_inst; ++i)
        if (!(jm[i] > 0.0)) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "det D zeta = %.3e <= 0 at a quadrature point of instance %lld (%s)",
                          jm[i], (long long)i, what(i).c_str());
            return c->fail(TSM_EGEOM, buf);
        }
    if (c->stationary) {   // the solves belong to tsm_stationary_solve
        const tsm_status ms = mg_setup(c);   // (frees a hierarchy of an earlier geometry)
        if (ms != TSM_OK) return ms;
        c->have_geom = true;
        c->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return TSM_OK;
    }

    // responses w_i = kappa p S_i^{-1} b_i (FP64, zero initial guess)
    HIPCHK(hipMemsetAsync(c->counters, 0, 4 * sizeof(int32_t), c->stream));
    MicroArgs ma = micro_base(c);
    ma.X0 = nullptr;
    ma.coef = nullptr;
    ma.rhs_vec = c->b;
    ma.rhs_scale = c->prm.kappa * c->prm.p;
    ma.zero_init = 1;
    ma.X_out = c->w;
    ma.rtol = c->prm.setup_rtol;
    ma.max_iter = std::max(c->prm.max_iter, 50000);   // setup must converge whatever the step budget
    tsm_status st = enqueue_micro(c, ma, true);
    if (st != TSM_OK) return st;
    // M w, so that the packed step solves can start from v0 alone (the
    // homogeneous part changes by O(dt) per step; v = v0 + u w does not
    // settle while u does)
    HIPCHK(launch_apply((int)n_inst, c->level, c->offsets, c->M64, c->w, c->Mw, c->stream));
    HIPCHK(launch_beta((int)n_inst, c->prm.kappa, c->prm.p, c->len, c->bx, c->beta, c->stream));
    {
        std::vector<double> kp_h(n_inst, c->prm.kappa * c->prm.p);
        if (!c->beta_fp) HIPALLOC(c->beta_fp, n_inst);
        HIPCHK(hipMemcpyAsync(c->beta_fp, kp_h.data(), n_inst * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    std::vector<double> bh(n_inst);
    int32_t nc = 0;
    HIPCHK(hipMemcpyAsync(bh.data(), c->beta, n_inst * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&nc, c->counters, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (nc > 0) return c->fail(TSM_ENOCONV, std::to_string(nc) + " response solves missed setup_rtol");

    // macro solver: reference beta, eigenvalues, sine basis, sweep count
    const int NM = c->NM, n = NM - 1;
    const double H = 1.0 / NM;
    double bmin = 1e300, bmax = -1e300;
    for (int k2 = 1; k2 < NM; ++k2)
        for (int k1 = 1; k1 < NM; ++k1) {
            const double v = bh[(size_t)k2 * (NM + 1) + k1];
            bmin = std::min(bmin, v);
            bmax = std::max(bmax, v);
        }
    const double bref = 0.5 * (bmin + bmax);
    std::vector<double> mk(n), kk(n), Qh((size_t)n * n), lh((size_t)n * n);
    for (int k = 0; k < n; ++k) {
        const double th_k = M_PI * (k + 1) * H;
        mk[k] = H / 6.0 * (4.0 + 2.0 * std::cos(th_k));
        kk[k] = (2.0 - 2.0 * std::cos(th_k)) / H;
    }
    double lmin = 1e300;
    const double sg = c->prm.source_sign;
    const double kp = c->prm.kappa * c->prm.p;
    std::vector<double> lf((size_t)n * n);
    for (int l2 = 0; l2 < n; ++l2)
        for (int l1 = 0; l1 < n; ++l1) {
            const double a0 = mk[l1] * mk[l2] / c->prm.dt + c->prm.D * (kk[l1] * mk[l2] + mk[l1] * kk[l2]);
            const double v = a0 - sg * bref * H * H;
            lh[(size_t)l2 * n + l1] = v;
            lf[(size_t)l2 * n + l1] = a0 - sg * kp * H * H;   // lagged coupling: beta = kappa p, exact
            lmin = std::min(lmin, std::fabs(v));
        }
    const double qs = std::sqrt(2.0 / (n + 1));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Qh[(size_t)i * n + j] = qs * std::sin(M_PI * (double)(i + 1) * (j + 1) / (n + 1));
    c->rho = H * H * 0.5 * (bmax - bmin) / lmin;
    // PCG bound: with A_M = A(0) + diag(c_k), c_k = -sign H^2 beta_k, and the
    // preconditioner A(0) + c_ref I, the generalised Rayleigh quotient is
    // (t + cbar) / (t + c_ref) with t in [tmin, tmax] (the eigenvalues of the
    // tensor operator A(0)) and cbar in [cmin, cmax]; it is monotone in t, so
    // its range -- and the condition number -- follow from the end points.
    {
        double tmin = 1e300, tmax = -1e300;
        for (int l2 = 0; l2 < n; ++l2)
            for (int l1 = 0; l1 < n; ++l1) {
                const double a0 = lh[(size_t)l2 * n + l1] + sg * bref * H * H;
                tmin = std::min(tmin, a0);
                tmax = std::max(tmax, a0);
            }
        const double c_lo = std::min(-sg * H * H * bmin, -sg * H * H * bmax);
        const double c_hi = std::max(-sg * H * H * bmin, -sg * H * H * bmax);
        const double c_ref = -sg * H * H * bref;
        c->macro_pcg_iters = 0;
        if (tmin + c_lo > 0 && tmin + c_ref > 0) {
            const double lo = std::min((tmin + c_lo) / (tmin + c_ref), (tmax + c_lo) / (tmax + c_ref));
            const double hi = std::max((tmin + c_hi) / (tmin + c_ref), (tmax + c_hi) / (tmax + c_ref));
            const double sk = std::sqrt(hi / lo);
            const double q = (sk - 1.0) / (sk + 1.0);
            // ||e_k||_A <= 2 q^k ||e_0||_A; a quarter more for finite precision
            int k = q > 0 ? (int)std::ceil(std::log(0.5e-17) / std::log(q)) : 1;
            k = std::max(2, k + k / 4 + 2);
            c->macro_pcg_iters = std::min(k, 400);
        }
    }
    if (!(c->rho < 0.5) && c->macro_pcg_iters == 0)
        return c->fail(TSM_EINVAL, "macro operator not shown positive definite (sweep contraction bound " +
                                       std::to_string(c->rho) + ")");
    int sweeps = 2;
    if (c->rho > 0) sweeps = std::max(2, (int)std::ceil(std::log(1e-17) / std::log(std::min(c->rho, 0.5))));
    c->macro_sweeps = std::min(sweeps, 64);
    // a PCG iteration costs about 1.2 sweeps (the same four GEMMs, two
    // one-workgroup kernels instead of the residual kernel)
    const int sweeps_needed = c->rho > 0 ? (int)std::ceil(std::log(1e-17) / std::log(c->rho)) : 2;
    c->macro_pcg_cheaper = c->rho < 1.0 && c->macro_pcg_iters > 0 && 6 * c->macro_pcg_iters < 5 * sweeps_needed;
    HIPCHK(hipMemcpy(c->Q, Qh.data(), Qh.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->lam, lh.data(), lh.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->lam_fp, lf.data(), lf.size() * sizeof(double), hipMemcpyHostToDevice));

    c->have_geom = true;
    tsm_status gs = build_graph(c);
    if (gs != TSM_OK) return gs;
    c->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return TSM_OK;
}

}  // namespace
}  // extern "C++"

tsm_status tsm_set_deformation(tsm_ctx* c, const double* a, const double* theta, int64_t n_inst) {
    const Range range("tsm_set_deformation");
    if (!c) return TSM_EINVAL;
    if (!c->have_mesh) return c->fail(TSM_ESTATE, "set_reference_mesh first");
    if (!a) return c->fail(TSM_EINVAL, "a is NULL");
    if (n_inst != c->n_inst) return c->fail(TSM_EINVAL, "n_inst does not match the reference mesh");
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipDeviceSynchronize());   // caller's producers of a, theta
    std::vector<double> ah(n_inst), th(n_inst, 0.0);
    HIPCHK(hipMemcpy(ah.data(), a, n_inst * sizeof(double), hipMemcpyDeviceToHost));
    if (theta) HIPCHK(hipMemcpy(th.data(), theta, n_inst * sizeof(double), hipMemcpyDeviceToHost));
    if (!finite_all(ah) || !finite_all(th)) return c->fail(TSM_EINVAL, "non-finite deformation parameter");
    c->have_geom = false;
    c->have_state = false;
    c->geom_tables = false;
    c->drop_graph();
    HIPCHK(hipMemcpyAsync(c->amp, a, n_inst * sizeof(double), hipMemcpyDeviceToDevice, c->stream));

    const AssembleArgs as = assemble_base(c);
    HIPCHK(launch_assemble(as, c->stream));
    return finish_setup(c, t0, [&](int64_t i) {
        char b[48];
        std::snprintf(b, sizeof b, "a = %.6g", ah[i]);
        return std::string(b);
    });
}

tsm_status tsm_set_jacobians(tsm_ctx* c, const double* Fcell, int64_t n_cell, const double* Fbnd, int64_t n_bnd) {
    const Range range("tsm_set_jacobians");
    if (!c) return TSM_EINVAL;
    if (!c->have_mesh) return c->fail(TSM_ESTATE, "set_reference_mesh first");
    if (!Fcell || !Fbnd) return c->fail(TSM_EINVAL, "Jacobian table is NULL");
    const int64_t n_inst = c->n_inst;
    std::vector<int64_t> co(n_inst), bo(n_inst);
    int64_t nc = 0, nb = 0;
    for (int64_t i = 0; i < n_inst; ++i) {
        const int64_t N = c->level_h[i];
        co[i] = nc;
        bo[i] = nb;
        nc += 16 * N * N;
        nb += 32 * N;
    }
    if (n_cell != nc || n_bnd != nb)
        return c->fail(TSM_EINVAL, "Jacobian tables must hold 16 sum N_i^2 = " + std::to_string(nc) +
                                       " and 32 sum N_i = " + std::to_string(nb) + " values");
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipDeviceSynchronize());   // caller's producers of the tables
    c->have_geom = false;
    c->have_state = false;
    c->drop_graph();
    if (!c->cell_off) HIPALLOC(c->cell_off, n_inst);
    if (!c->bnd_off) HIPALLOC(c->bnd_off, n_inst);
    HIPCHK(hipMemcpy(c->cell_off, co.data(), n_inst * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->bnd_off, bo.data(), n_inst * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemsetAsync(c->amp, 0, n_inst * sizeof(double), c->stream));

    AssembleArgs as = assemble_base(c);
    as.Fcell = Fcell; as.Fbnd = Fbnd; as.cell_off = c->cell_off; as.bnd_off = c->bnd_off;
    HIPCHK(launch_assemble_tables(as, c->stream));
    c->geom_tables = true;
    return finish_setup(c, t0, [](int64_t) { return std::string("Jacobian tables; -1: non-finite entry"); });
}

tsm_status tsm_set_state(tsm_ctx* c, const double* u, int64_t n_u, const double* v, int64_t n_v) {
    if (!c) return TSM_EINVAL;
    if (c->stationary) return c->fail(TSM_ESTATE, "stationary context: no time stepping (tsm_stationary_solve)");
    if (!c->have_geom) return c->fail(TSM_ESTATE, "set_deformation first");
    if (!u) return c->fail(TSM_EINVAL, "u is NULL");
    if (n_u != c->n_inst) return c->fail(TSM_EINVAL, "u has " + std::to_string(n_u) + " entries, n_inst is " + std::to_string(c->n_inst));
    if (v && n_v != c->total)
        return c->fail(TSM_EINVAL, "v has " + std::to_string(n_v) + " entries, the ragged micro layout has " +
                                       std::to_string(c->total));
    HIPCHK(hipDeviceSynchronize());
    std::vector<double> uh(c->n_inst);
    HIPCHK(hipMemcpy(uh.data(), u, c->n_inst * sizeof(double), hipMemcpyDeviceToHost));
    if (!finite_all(uh)) return c->fail(TSM_EINVAL, "non-finite macro state");
    const int W = c->NM + 1;
    for (int k2 = 0; k2 < W; ++k2)
        for (int k1 = 0; k1 < W; ++k1)
            if (k1 == 0 || k2 == 0 || k1 == c->NM || k2 == c->NM) uh[(size_t)k2 * W + k1] = 0.0;
    HIPCHK(hipMemcpy(c->u, uh.data(), c->n_inst * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(launch_state_split((int)c->n_inst, c->offsets, c->u, v, c->w, c->v0, c->stream));
    HIPCHK(hipMemsetAsync(c->F, 0, c->n_inst * sizeof(double), c->stream));
    if (reset_history(c) != TSM_OK) return TSM_EHIP;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->steps_taken = 0;
    c->have_state = true;
    return TSM_OK;
}

tsm_status tsm_step(tsm_ctx* c, int32_t n_steps) {
    const Range range("tsm_step");
    if (!c) return TSM_EINVAL;
    if (!c->have_state) return c->fail(TSM_ESTATE, "set_state first");
    if (n_steps < 0) return c->fail(TSM_EINVAL, "n_steps < 0");
    // per-phase events bracket the exact step only (the alternating step times as a whole)
    const bool timing = (c->prm.flags & TSM_FLAG_TIMING) && !(c->prm.flags & TSM_FLAG_FIXED_POINT);
    if (timing) {
        while ((int)c->tev.size() < 3 * n_steps) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            c->tev.push_back(e);
        }
    }
    HIPCHK(hipMemsetAsync(c->counters, 0, 4 * sizeof(int32_t), c->stream));
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    const bool fixed_point = (c->prm.flags & TSM_FLAG_FIXED_POINT) != 0;
    if (fixed_point) c->fp_iters_max = 0;
    for (int s = 0; s < n_steps; ++s) {
        if (fixed_point) {
            tsm_status st = step_fixed_point(c);
            if (st != TSM_OK) return st;
        } else if (c->graph) {
            HIPCHK(hipGraphLaunch(c->graph, c->stream));
        } else {
            tsm_status st = enqueue_step(c, timing ? &c->tev[3 * s] : nullptr);
            if (st != TSM_OK) return st;
        }
    }
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    // the alternating step moves the state without the history
    if (fixed_point && n_steps > 0 && reset_history(c) != TSM_OK) return TSM_EHIP;
    int32_t nc = 0;
    HIPCHK(hipMemcpyAsync(&nc, c->counters, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->step_ms = ms;
    c->micro_ms = c->macro_ms = 0.0;
    c->timed_steps = 0;
    if (timing) {
        for (int s = 0; s < n_steps; ++s) {
            float a = 0.0f, b = 0.0f;
            HIPCHK(hipEventElapsedTime(&a, c->tev[3 * s], c->tev[3 * s + 1]));
            HIPCHK(hipEventElapsedTime(&b, c->tev[3 * s + 1], c->tev[3 * s + 2]));
            c->micro_ms += a;
            c->macro_ms += b;
        }
        c->timed_steps = n_steps;
    }
    c->steps_taken += n_steps;
    if (nc > 0) return c->fail(TSM_ENOCONV, std::to_string(nc) + " micro solves missed rtol");
    return TSM_OK;
}

tsm_status tsm_get_macro(const tsm_ctx* cc, double* out, int64_t n) {
    tsm_ctx* c = const_cast<tsm_ctx*>(cc);
    if (!c || !out) return TSM_EINVAL;
    if (!c->have_state) return c->fail(TSM_ESTATE, "no state");
    if (n != c->n_inst) return c->fail(TSM_EINVAL, "u_out must hold n_inst = " + std::to_string(c->n_inst) + " entries");
    HIPCHK(hipDeviceSynchronize());   // the caller's pending work on the output buffer
    HIPCHK(hipMemcpyAsync(out, c->u, c->n_inst * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TSM_OK;
}

tsm_status tsm_get_fluxes(const tsm_ctx* cc, double* out, int64_t n) {
    tsm_ctx* c = const_cast<tsm_ctx*>(cc);
    if (!c || !out) return TSM_EINVAL;
    if (!c->have_state) return c->fail(TSM_ESTATE, "no state");
    if (n != c->n_inst) return c->fail(TSM_EINVAL, "F_out must hold n_inst = " + std::to_string(c->n_inst) + " entries");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpyAsync(out, c->F, c->n_inst * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TSM_OK;
}

tsm_status tsm_get_micro(const tsm_ctx* cc, double* out, int64_t n) {
    tsm_ctx* c = const_cast<tsm_ctx*>(cc);
    if (!c || !out) return TSM_EINVAL;
    if (!c->have_state) return c->fail(TSM_ESTATE, "no state");
    if (n != c->total) return c->fail(TSM_EINVAL, "v_out must hold the " + std::to_string(c->total) + " ragged entries");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(launch_state_join((int)c->n_inst, c->offsets, c->u, c->v0, c->w, out, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TSM_OK;
}

tsm_status tsm_get_setup(const tsm_ctx* cc, double* beta_out, double* len_out, int64_t n_inst, double* w_out,
                         int64_t n_w) {
    tsm_ctx* c = const_cast<tsm_ctx*>(cc);
    if (!c) return TSM_EINVAL;
    if (!c->have_geom) return c->fail(TSM_ESTATE, "set_deformation first");
    if (c->stationary) return c->fail(TSM_ESTATE, "stationary context: no response functionals");
    if ((beta_out || len_out) && n_inst != c->n_inst)
        return c->fail(TSM_EINVAL, "beta_out and len_out must hold n_inst = " + std::to_string(c->n_inst) + " entries");
    if (w_out && n_w != c->total)
        return c->fail(TSM_EINVAL, "w_out must hold the " + std::to_string(c->total) + " ragged entries");
    HIPCHK(hipDeviceSynchronize());
    if (beta_out) HIPCHK(hipMemcpyAsync(beta_out, c->beta, c->n_inst * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (len_out) HIPCHK(hipMemcpyAsync(len_out, c->len, c->n_inst * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (w_out) HIPCHK(hipMemcpyAsync(w_out, c->w, c->total * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TSM_OK;
}

tsm_status tsm_apply_operator(tsm_ctx* c, const double* x, double* y, int64_t n) {
    if (!c || !x || !y) return TSM_EINVAL;
    if (!c->have_geom) return c->fail(TSM_ESTATE, "set_deformation first");
    if (n != c->total) return c->fail(TSM_EINVAL, "x and y must hold the " + std::to_string(c->total) + " ragged entries");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(launch_apply((int)c->n_inst, c->level, c->offsets, c->S64, x, y, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TSM_OK;
}

tsm_status tsm_gradient(tsm_ctx* c, int32_t n_steps, double* J_out, double* dJda_out, int64_t n) {
    const Range range("tsm_gradient");
    if (!c) return TSM_EINVAL;
    if (!c->have_state) return c->fail(TSM_ESTATE, "set_state first");
    if (n_steps < 1) return c->fail(TSM_EINVAL, "n_steps < 1");
    if (!J_out || !dJda_out) return c->fail(TSM_EINVAL, "J_out and dJda_out are required");
    if (n != c->n_inst) return c->fail(TSM_EINVAL, "dJda_out must hold n_inst = " + std::to_string(c->n_inst) + " entries");
    if (c->geom_tables)
        return c->fail(TSM_ESTATE, "tsm_gradient differentiates with respect to the deformation amplitudes; "
                                   "the geometry came from Jacobian tables");
    const int64_t ni = c->n_inst, tot = c->total;
    const int N = n_steps, K = c->prm.checkpoint_every;
    const int nseg = (N + K - 1) / K;
    HIPCHK(hipDeviceSynchronize());
    // --- adjoint state (the derivative forms are evaluated matrix-free)
    if (!c->lam0) {
        HIPALLOC(c->lam0, tot); HIPALLOC(c->mu, ni); HIPALLOC(c->coef, ni); HIPALLOC(c->grad, ni);
        HIPALLOC(c->Jd, 1);
        if (c->hx != nullptr) {
            HIPALLOC(c->lhx, tot); HIPALLOC(c->lhe, tot); HIPALLOC(c->lhe2, tot); HIPALLOC(c->lhn, 1);
        }
    }
    const bool extrap = c->hx != nullptr && !(c->prm.flags & TSM_FLAG_NO_EXTRAPOLATION);
    // --- work buffers of this call
    double *U = nullptr, *ck_u = nullptr, *ck_v = nullptr, *V = nullptr, *save_u = nullptr, *save_v = nullptr,
           *save_F = nullptr;
    // the history of the extrapolated start at every checkpoint, so that a
    // recomputed segment repeats its steps bitwise
    float *ck_hx = nullptr, *ck_he = nullptr, *ck_he2 = nullptr;
    int32_t* ck_hn = nullptr;
    auto release = [&]() {
        dfree(U); dfree(ck_u); dfree(ck_v); dfree(V); dfree(save_u); dfree(save_v); dfree(save_F);
        dfree(ck_hx); dfree(ck_he); dfree(ck_he2); dfree(ck_hn);
    };
    const size_t nh = extrap ? (size_t)nseg : 0;
    if (dalloc(&U, (size_t)(N + 1) * ni) != hipSuccess || dalloc(&ck_u, (size_t)nseg * ni) != hipSuccess ||
        dalloc(&ck_v, (size_t)nseg * tot) != hipSuccess || dalloc(&V, (size_t)(K + 1) * tot) != hipSuccess ||
        dalloc(&save_u, ni) != hipSuccess || dalloc(&save_v, tot) != hipSuccess || dalloc(&save_F, ni) != hipSuccess ||
        dalloc(&ck_hx, nh * tot) != hipSuccess || dalloc(&ck_he, nh * tot) != hipSuccess ||
        dalloc(&ck_he2, nh * tot) != hipSuccess ||
        dalloc(&ck_hn, nh) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return c->fail(TSM_ENOMEM, "gradient work buffers");
    }
    tsm_status st = TSM_OK;
    auto run = [&]() -> tsm_status {
        hipStream_t s = c->stream;
        HIPCHK(hipMemcpyAsync(save_u, c->u, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(save_v, c->v0, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(save_F, c->F, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemsetAsync(c->counters, 0, 4 * sizeof(int32_t), s));
        HIPCHK(hipEventRecord(c->ev0, s));
        // forward with checkpoints; u of every step kept (n_inst doubles per
        // step).  The tape's history of the extrapolated start begins empty
        // and is kept with every checkpoint.
        HIPCHK(hipMemcpyAsync(U, c->u, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (reset_history(c) != TSM_OK) return TSM_EHIP;
        for (int n = 0; n < N; ++n) {
            if (n % K == 0) {
                const size_t q = (size_t)(n / K);
                HIPCHK(hipMemcpyAsync(ck_u + q * ni, c->u, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(ck_v + q * tot, c->v0, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
                if (extrap) {
                    HIPCHK(hipMemcpyAsync(ck_hx + q * tot, c->hx, tot * sizeof(float), hipMemcpyDeviceToDevice, s));
                    HIPCHK(hipMemcpyAsync(ck_he + q * tot, c->he, tot * sizeof(float), hipMemcpyDeviceToDevice, s));
                    HIPCHK(hipMemcpyAsync(ck_he2 + q * tot, c->he2, tot * sizeof(float), hipMemcpyDeviceToDevice, s));
                    HIPCHK(hipMemcpyAsync(ck_hn + q, c->hn, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
                }
            }
            if (c->graph) {
                HIPCHK(hipGraphLaunch(c->graph, s));
            } else {
                tsm_status e = enqueue_step(c);
                if (e != TSM_OK) return e;
            }
            HIPCHK(hipMemcpyAsync(U + (size_t)(n + 1) * ni, c->u, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        const MacroArgs m = c->macro_args();
        HIPCHK(launch_observable(m, U + (size_t)N * ni, c->Jd, s));
        HIPCHK(hipEventRecord(c->ev1, s));
        // backward: lambda^{N+1} = 0, mu^{N+1} = 0; the history of the
        // adjoint solves' extrapolated start begins empty
        HIPCHK(hipMemsetAsync(c->lam0, 0, tot * sizeof(double), s));
        if (extrap) HIPCHK(launch_fill_i32(c->lhn, 0, 1, s));
        HIPCHK(hipMemsetAsync(c->coef, 0, ni * sizeof(double), s));
        HIPCHK(hipMemsetAsync(c->mu, 0, ni * sizeof(double), s));
        HIPCHK(hipMemsetAsync(c->grad, 0, ni * sizeof(double), s));
        for (int sg = nseg - 1; sg >= 0; --sg) {
            const int a = sg * K, e = std::min(a + K, N);
            // recompute the segment's states v^a .. v^e (same kernels: bitwise equal)
            HIPCHK(hipMemcpyAsync(c->u, ck_u + (size_t)sg * ni, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(c->v0, ck_v + (size_t)sg * tot, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
            if (extrap) {
                HIPCHK(hipMemcpyAsync(c->hx, ck_hx + (size_t)sg * tot, tot * sizeof(float), hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(c->he, ck_he + (size_t)sg * tot, tot * sizeof(float), hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(c->he2, ck_he2 + (size_t)sg * tot, tot * sizeof(float), hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(c->hn, ck_hn + sg, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            }
            HIPCHK(launch_state_join((int)ni, c->offsets, c->u, c->v0, c->w, V, s));
            for (int n = a + 1; n <= e; ++n) {
                if (c->graph) {
                    HIPCHK(hipGraphLaunch(c->graph, s));
                } else {
                    tsm_status e2 = enqueue_step(c);
                    if (e2 != TSM_OK) return e2;
                }
                HIPCHK(launch_state_join((int)ni, c->offsets, c->u, c->v0, c->w, V + (size_t)(n - a) * tot, s));
            }
            for (int mstep = e; mstep > a; --mstep) {
                // micro adjoint solves: lam0^m = S^{-1} M (lam0^{m+1} + coef^{m+1} w) / dt
                MicroArgs ma = micro_base(c);
                ma.X0 = c->lam0;
                ma.coef = c->coef;
                ma.Mw = c->Mw;
                ma.rhs_vec = nullptr;
                ma.zero_init = 0;
                ma.X_out = c->lam0;
                if (extrap) {
                    ma.hx = c->lhx;
                    ma.he = c->lhe;
                    ma.he2 = c->lhe2;
                    ma.hn = c->lhn;
                }
                tsm_status e3 = enqueue_micro(c, ma, false);
                if (e3 != TSM_OK) return e3;
                // macro adjoint: A_M mu^m = M_H mu^{m+1}/dt + kappa p (b^T lam0^m) (+ 2 M_H u^N)
                HIPCHK(launch_macro_rhs_adjoint(m, c->mu, c->bx, U + (size_t)N * ni, mstep == N ? 1 : 0, c->rhs, s));
                e3 = enqueue_macro_solve(c, c->mu);
                if (e3 != TSM_OK) return e3;
                HIPCHK(launch_adjoint_coef(m, c->mu, c->coef, s));
                GradArgs ga;
                ga.n_inst = (int)ni;
                ga.NM = c->NM;
                ga.level = c->level;
                ga.offsets = c->offsets;
                ga.amp = c->amp;
                ga.tab = Tables{c->tab_off, c->tab_y, c->tab_s, c->tab_c};
                ga.len = c->len;
                ga.d = c->prm.d;
                ga.lam0 = c->lam0; ga.coef = c->coef; ga.w = c->w;
                ga.v_now = V + (size_t)(mstep - a) * tot;
                ga.v_prev = V + (size_t)(mstep - a - 1) * tot;
                ga.u_now = U + (size_t)mstep * ni;
                ga.mu = c->mu;
                ga.kappa = c->prm.kappa; ga.p = c->prm.p; ga.sign = c->prm.source_sign; ga.inv_dt = 1.0 / c->prm.dt;
                ga.g = c->grad;
                HIPCHK(launch_gradient_step(ga, s));
            }
        }
        hipEvent_t e_end;
        HIPCHK(hipEventCreate(&e_end));
        HIPCHK(hipEventRecord(e_end, s));
        HIPCHK(hipMemcpyAsync(dJda_out, c->grad, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(J_out, c->Jd, sizeof(double), hipMemcpyDeviceToHost, s));
        // restore the state
        HIPCHK(hipMemcpyAsync(c->u, save_u, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(c->v0, save_v, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(c->F, save_F, ni * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (reset_history(c) != TSM_OK) return TSM_EHIP;
        int32_t nc = 0;
        HIPCHK(hipMemcpyAsync(&nc, c->counters, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        float f1 = 0.0f, f2 = 0.0f;
        HIPCHK(hipEventElapsedTime(&f1, c->ev0, c->ev1));
        HIPCHK(hipEventElapsedTime(&f2, c->ev1, e_end));
        (void)hipEventDestroy(e_end);
        c->grad_fwd_ms = f1;
        c->grad_bwd_ms = f2;
        if (nc > 0) return c->fail(TSM_ENOCONV, std::to_string(nc) + " solves missed rtol during the gradient");
        return TSM_OK;
    };
    // every solve of the gradient at its own tolerance (the step graph is
    // rebuilt for it and restored afterwards)
    const double step_rtol = c->prm.rtol;
    const bool own_rtol = c->prm.grad_rtol > 0.0 && c->prm.grad_rtol != step_rtol;
    if (own_rtol) {
        c->prm.rtol = c->prm.grad_rtol;
        st = build_graph(c);
    }
    if (st == TSM_OK) st = run();
    (void)hipStreamSynchronize(c->stream);
    if (own_rtol) {
        c->prm.rtol = step_rtol;
        const std::string err = c->err;
        const tsm_status gs = build_graph(c);
        if (st == TSM_OK) st = gs;
        else c->err = err;
    }
    release();
    return st;
}

tsm_status tsm_set_flags(tsm_ctx* c, uint64_t flags) {
    if (!c) return TSM_EINVAL;
    const bool replan = ((flags ^ c->prm.flags) & (TSM_FLAG_STENCIL_STREAM | TSM_FLAG_GENERIC | TSM_FLAG_GENERIC_16 |
                                                    TSM_FLAG_GENERIC_32 | TSM_FLAG_GENERIC_64 |
                                                    TSM_FLAG_MULTIGRID | TSM_FLAG_NO_MULTIGRID)) != 0;
    if (flags & ~(TSM_FLAG_NO_GRAPH | TSM_FLAG_STENCIL_STREAM | TSM_FLAG_TIMING | TSM_FLAG_GENERIC | TSM_FLAG_PERSISTENT |
                  TSM_FLAG_FIXED_POINT | TSM_FLAG_GENERIC_16 | TSM_FLAG_GENERIC_32 | TSM_FLAG_GENERIC_64 |
                  TSM_FLAG_MATRIX_FREE | TSM_FLAG_MACRO_PCG | TSM_FLAG_MULTIGRID | TSM_FLAG_NO_MULTIGRID |
                  TSM_FLAG_NO_EXTRAPOLATION | TSM_FLAG_ASSEMBLED_START))
        return c->fail(TSM_EINVAL, "unknown flag bits");
    const bool mg_changed = ((flags ^ c->prm.flags) & (TSM_FLAG_MULTIGRID | TSM_FLAG_NO_MULTIGRID)) != 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->prm.flags = flags;
    if (reset_history(c) != TSM_OK) return TSM_EHIP;
    if (replan && c->have_mesh) {
        tsm_status st = plan_tasks(c);
        if (st != TSM_OK) return st;
    }
    if (c->stationary && c->have_geom && mg_changed) {
        const tsm_status ms = mg_setup(c);
        if (ms != TSM_OK) return ms;
    }
    if (c->have_geom && !c->stationary) return build_graph(c);
    return TSM_OK;
}

tsm_status tsm_autotune(tsm_ctx* c, int32_t steps, double* ms_out, uint64_t* flags_out) {
    const Range range("tsm_autotune");
    if (!c) return TSM_EINVAL;
    if (!c->have_state) return c->fail(TSM_ESTATE, "set_state first");
    if (steps < 1) return c->fail(TSM_EINVAL, "steps < 1");
    const int64_t ni = c->n_inst, tot = c->total;
    // plans are timed with the whole-step events (TSM_FLAG_TIMING would turn the graph off)
    const uint64_t plan_bits = TSM_FLAG_GENERIC | TSM_FLAG_PERSISTENT | TSM_FLAG_GENERIC_16 | TSM_FLAG_GENERIC_32 |
                               TSM_FLAG_GENERIC_64 | TSM_FLAG_MATRIX_FREE;
    const uint64_t timing = c->prm.flags & TSM_FLAG_TIMING;
    const uint64_t keep = c->prm.flags & ~(plan_bits | TSM_FLAG_TIMING);
    const uint64_t entry_flags = c->prm.flags;
    // stages 1 and 2 keep the caller's operator form; stage 3 tries the
    // assembled one when the caller asked for the matrix-free form
    const uint64_t op_form = c->prm.flags & TSM_FLAG_MATRIX_FREE;
    double ms[5] = {-1.0, -1.0, -1.0, -1.0, -1.0};
    double *su = nullptr, *sv = nullptr, *sF = nullptr;
    if (dalloc(&su, ni) != hipSuccess || dalloc(&sv, tot) != hipSuccess || dalloc(&sF, ni) != hipSuccess) {
        (void)hipGetLastError();
        dfree(su); dfree(sv); dfree(sF);
        return c->fail(TSM_ENOMEM, "autotune state copy");
    }
    auto copy = [&](double* du, double* dv, double* dF, const double* u, const double* v, const double* F) {
        return hipMemcpyAsync(du, u, ni * sizeof(double), hipMemcpyDeviceToDevice, c->stream) == hipSuccess &&
               hipMemcpyAsync(dv, v, tot * sizeof(double), hipMemcpyDeviceToDevice, c->stream) == hipSuccess &&
               hipMemcpyAsync(dF, F, ni * sizeof(double), hipMemcpyDeviceToDevice, c->stream) == hipSuccess;
    };
    tsm_status st = TSM_OK;
    const int64_t taken = c->steps_taken;
    if (!copy(su, sv, sF, c->u, c->v0, c->F)) st = c->fail(TSM_EHIP, "autotune: state copy");
    // time one plan from the saved state, then restore it
    auto trial = [&](uint64_t plan, double& out) {
        if (st != TSM_OK) return;
        st = tsm_set_flags(c, keep | plan);
        if (st != TSM_OK) return;
        tsm_status s1 = tsm_step(c, 1);                  // warm-up (and code load)
        if (s1 == TSM_OK || s1 == TSM_ENOCONV) s1 = tsm_step(c, steps);
        if (s1 != TSM_OK && s1 != TSM_ENOCONV) { st = s1; return; }
        out = c->step_ms / steps;
        if (!copy(c->u, c->v0, c->F, su, sv, sF)) st = c->fail(TSM_EHIP, "autotune: state restore");
    };
    // the packed mesh sizes present
    bool present[3] = {false, false, false};
    for (int32_t l : c->level_h) {
        if (l == 16) present[0] = true;
        if (l == 32) present[1] = true;
        if (l == 64) present[2] = true;
    }
    const bool packs = present[0] || present[1] || present[2];
    // stage 1: whole plans
    trial(op_form, ms[0]);
    if (packs) {
        trial(TSM_FLAG_PERSISTENT | op_form, ms[1]);
        trial(TSM_FLAG_GENERIC | op_form, ms[2]);
    }
    uint64_t best = op_form;
    double best_ms = ms[0];
    if (ms[1] >= 0 && ms[1] < best_ms) { best = TSM_FLAG_PERSISTENT | op_form; best_ms = ms[1]; }
    // stage 2: from the better packed plan, move one mesh size at a time to
    // the generic kernel while that helps
    const uint64_t size_bit[3] = {TSM_FLAG_GENERIC_16, TSM_FLAG_GENERIC_32, TSM_FLAG_GENERIC_64};
    int packed_sizes = (int)present[0] + (int)present[1] + (int)present[2];
    for (int k = 0; k < 3 && st == TSM_OK && packed_sizes > 1; ++k) {
        if (!present[k]) continue;
        double t = -1.0;
        trial(best | size_bit[k], t);
        if (t >= 0 && t < best_ms) {
            best |= size_bit[k];
            best_ms = t;
            --packed_sizes;
        }
    }
    if (ms[2] >= 0 && ms[2] < best_ms) { best = TSM_FLAG_GENERIC | op_form; best_ms = ms[2]; }
    // stage 3 (the caller asked for the matrix-free operator): the chosen
    // plan with the assembled operator instead
    const bool op_choice = op_form != 0 && packs && !(best & TSM_FLAG_GENERIC) &&
                           c->prm.precision == TSM_FP32_REFINE && !c->geom_tables;
    if (op_choice && st == TSM_OK) {
        trial(best & ~TSM_FLAG_MATRIX_FREE, ms[4]);
        if (ms[4] >= 0 && ms[4] < best_ms) {
            std::swap(best_ms, ms[4]);
            best &= ~TSM_FLAG_MATRIX_FREE;
        }
    }
    ms[3] = best_ms;
    if (st == TSM_OK) {
        st = tsm_set_flags(c, keep | timing | best);
        (void)hipStreamSynchronize(c->stream);
        c->steps_taken = taken;
        if (ms_out) std::memcpy(ms_out, ms, sizeof(ms));
        if (flags_out) *flags_out = best;
    } else {
        // a trial failed: back to the caller's plan (its error stays reported)
        const std::string err = c->err;
        (void)tsm_set_flags(c, entry_flags);
        c->err = err;
    }
    (void)hipStreamSynchronize(c->stream);
    dfree(su); dfree(sv); dfree(sF);
    return st;
}

tsm_status tsm_get_stats(const tsm_ctx* cc, tsm_stats* s) {
    tsm_ctx* c = const_cast<tsm_ctx*>(cc);
    if (!c || !s) return TSM_EINVAL;
    std::memset(s, 0, sizeof(*s));
    s->n_inst = c->n_inst;
    s->n_micro_dofs = c->total;
    s->steps_taken = c->steps_taken;
    s->macro_sweeps = c->macro_pcg() ? 0 : c->macro_sweeps;
    s->macro_pcg_iters = c->macro_pcg() ? c->macro_pcg_iters : 0;
    s->macro_contraction = c->rho;
    s->setup_ms = c->setup_ms;
    s->step_ms = c->step_ms;
    s->micro_ms = c->micro_ms;
    s->macro_ms = c->macro_ms;
    s->timed_steps = c->timed_steps;
    const size_t packed = ((c->prm.flags & TSM_FLAG_PERSISTENT) && !c->pack_groups.empty()) ? 1 : c->pack_groups.size();
    s->micro_launches = (int32_t)(c->groups.size() + packed);
    s->fp_iters_last = c->fp_iters_last;
    s->fp_iters_max = c->fp_iters_max;
    s->grad_forward_ms = c->grad_fwd_ms;
    s->grad_backward_ms = c->grad_bwd_ms;
    if (c->have_geom && c->n_inst > 0) {
        std::vector<int32_t> it(c->n_inst), sw(c->n_inst);
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipMemcpy(it.data(), c->iters, c->n_inst * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(sw.data(), c->sweeps, c->n_inst * sizeof(int32_t), hipMemcpyDeviceToHost));
        int32_t cnt[4] = {0, 0, 0, 0};
        HIPCHK(hipMemcpy(cnt, c->counters, sizeof(cnt), hipMemcpyDeviceToHost));
        const int32_t nc = cnt[0];
        s->fp64_fallbacks = cnt[2];
        s->iters_min = *std::min_element(it.begin(), it.end());
        s->iters_max = *std::max_element(it.begin(), it.end());
        double sum = 0;
        for (int32_t v : it) sum += v;
        s->iters_mean = sum / c->n_inst;
        s->sweeps_max = *std::max_element(sw.begin(), sw.end());
        double ssum = 0;
        for (int32_t v : sw) ssum += v;
        s->sweeps_mean = ssum / c->n_inst;
        s->unconverged = nc;
    }
    return TSM_OK;
}

const char* tsm_last_error(const tsm_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

tsm_status tsm_error_indicator(tsm_ctx* c, double* eta2_out, int64_t n) {
    const Range range("tsm_error_indicator");
    if (!c) return TSM_EINVAL;
    if (!eta2_out) return c->fail(TSM_EINVAL, "eta2_out is NULL");
    if (n != c->n_inst) return c->fail(TSM_EINVAL, "eta2_out must hold n_inst = " + std::to_string(c->n_inst) + " entries");
    if (c->stationary) return c->fail(TSM_ESTATE, "stationary context: no time-stepped micro state");
    if (!c->have_state) return c->fail(TSM_ESTATE, "set_state first");
    if (c->geom_tables) return c->fail(TSM_ESTATE, "indicator needs the amplitude geometry (not Jacobian tables)");
    IndicatorArgs a{};
    a.n_inst = (int)c->n_inst;
    a.level = c->level;
    a.offsets = c->offsets;
    a.amp = c->amp;
    a.u = c->u;
    a.v0 = c->v0;
    a.w = c->w;
    a.d = c->prm.d;
    a.eta2 = eta2_out;
    HIPCHK(launch_indicator(a, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TSM_OK;
}

tsm_status tsm_mark_refine(int64_t n_inst, const double* eta2, const int32_t* level, double theta, int32_t max_level,
                           int32_t* level_new, int64_t* n_marked) {
    if (n_inst < 0 || (n_inst > 0 && (!eta2 || !level || !level_new)))
        return create_failed(nullptr, TSM_EINVAL, "tsm_mark_refine: bad arguments");
    if (!(theta >= 0.0 && theta <= 1.0)) return create_failed(nullptr, TSM_EINVAL, "tsm_mark_refine: theta outside [0, 1]");
    double total = 0.0;
    std::vector<int64_t> cand;
    for (int64_t i = 0; i < n_inst; ++i) {
        if (!(eta2[i] >= 0.0) || !std::isfinite(eta2[i]))
            return create_failed(nullptr, TSM_EINVAL, "tsm_mark_refine: eta2 negative or not finite");
        if (level[i] < kMinLevel || level[i] > kMaxMesh)
            return create_failed(nullptr, TSM_EINVAL, "tsm_mark_refine: level outside 2..256");
        total += eta2[i];
        if (2 * level[i] <= max_level) cand.push_back(i);
        level_new[i] = level[i];
    }
    std::sort(cand.begin(), cand.end(), [&](int64_t x, int64_t y) {
        if (eta2[x] != eta2[y]) return eta2[x] > eta2[y];
        return x < y;
    });
    double acc = 0.0;
    int64_t nm = 0;
    for (int64_t i : cand) {
        if (acc >= theta * total) break;
        level_new[i] = 2 * level[i];
        acc += eta2[i];
        ++nm;
    }
    if (n_marked) *n_marked = nm;
    return TSM_OK;
}

tsm_status tsm_prolong(int64_t n_inst, const int32_t* lo, const int32_t* ln, const double* vo, int64_t n_old,
                       double* vn, int64_t n_new, void* stream) {
    if (n_inst < 1 || !lo || !ln || !vo || !vn) return create_failed(nullptr, TSM_EINVAL, "tsm_prolong: bad arguments");
    std::vector<int64_t> oo(n_inst + 1, 0), on(n_inst + 1, 0);
    for (int64_t i = 0; i < n_inst; ++i) {
        if (lo[i] < kMinLevel || lo[i] > kMaxMesh || !(ln[i] == lo[i] || ln[i] == 2 * lo[i]) || ln[i] > kMaxMesh)
            return create_failed(nullptr, TSM_EINVAL,
                                 "tsm_prolong: level_new[" + std::to_string(i) + "] is neither level_old nor twice it (<= 256)");
        oo[i + 1] = oo[i] + (int64_t)(lo[i] + 1) * (lo[i] + 1);
        on[i + 1] = on[i] + (int64_t)(ln[i] + 1) * (ln[i] + 1);
    }
    if (n_old != oo[n_inst] || n_new != on[n_inst])
        return create_failed(nullptr, TSM_EINVAL,
                             "tsm_prolong: v_old must hold " + std::to_string(oo[n_inst]) + " and v_new " +
                                 std::to_string(on[n_inst]) + " entries");
    hipStream_t s = (hipStream_t)stream;
    int32_t *dlo = nullptr, *dln = nullptr;
    int64_t *doo = nullptr, *don = nullptr;
    hipError_t e = dalloc(&dlo, n_inst);
    if (e == hipSuccess) e = dalloc(&dln, n_inst);
    if (e == hipSuccess) e = dalloc(&doo, n_inst + 1);
    if (e == hipSuccess) e = dalloc(&don, n_inst + 1);
    if (e == hipSuccess) e = hipMemcpy(dlo, lo, n_inst * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dln, ln, n_inst * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(doo, oo.data(), (n_inst + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(don, on.data(), (n_inst + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_prolong((int)n_inst, dlo, dln, doo, don, vo, vn, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(dlo);
    dfree(dln);
    dfree(doo);
    dfree(don);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return create_failed(nullptr, TSM_EHIP, std::string("tsm_prolong: ") + hipGetErrorString(e));
    }
    return TSM_OK;
}

void tsm_stationary_default_params(tsm_stationary_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->macro_cells = 8;
    p->Dv = 1.0;
    p->Dw = 0.1;
    p->kappa1 = 0.5;
    p->kappa2 = 1.0;
    p->kappa3 = 0.25;
    p->kappa4 = 1.0;
    p->u_dirichlet = 1.0;
    p->parts[0] = TSM_PART_N;
    p->parts[1] = TSM_PART_N;
    p->parts[2] = TSM_PART_I;
    p->parts[3] = TSM_PART_O;
    p->dirichlet[2] = 1;
    p->rtol = 1e-12;
    p->macro_rtol = 1e-14;
    p->max_iter = 20000;
    p->macro_max_iter = 200000;
    p->flags = 0;
}

tsm_status tsm_stationary_create(const tsm_stationary_params* sp, void* stream, tsm_ctx** out) {
    if (!out) return create_failed(nullptr, TSM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!sp) return create_failed(nullptr, TSM_EINVAL, "params is NULL");
    int n_in = 0, n_out = 0, n_dir = 0;
    bool parts_ok = true;
    for (int s = 0; s < 4; ++s) {
        parts_ok = parts_ok && sp->parts[s] >= TSM_PART_N && sp->parts[s] <= TSM_PART_O;
        n_in += sp->parts[s] == TSM_PART_I;
        n_out += sp->parts[s] == TSM_PART_O;
        n_dir += sp->dirichlet[s] != 0;
    }
    const uint64_t plan = TSM_FLAG_NO_GRAPH | TSM_FLAG_STENCIL_STREAM | TSM_FLAG_GENERIC | TSM_FLAG_PERSISTENT |
                          TSM_FLAG_GENERIC_16 | TSM_FLAG_GENERIC_32 | TSM_FLAG_GENERIC_64 | TSM_FLAG_MULTIGRID |
                          TSM_FLAG_NO_MULTIGRID;
    const double pos[] = {sp->Dv, sp->Dw, sp->kappa1, sp->kappa2, sp->kappa3, sp->kappa4, sp->rtol, sp->macro_rtol};
    bool ok = sp->macro_cells >= 2 && sp->macro_cells <= 256 && parts_ok && n_in >= 1 && n_out >= 1 && n_dir >= 1 &&
              sp->max_iter >= 1 && sp->macro_max_iter >= 1 && !(sp->flags & ~plan) && std::isfinite(sp->fu) &&
              std::isfinite(sp->fv) && std::isfinite(sp->fw) && std::isfinite(sp->u_dirichlet);
    for (double v : pos) ok = ok && v > 0 && std::isfinite(v);
    if (!ok) return create_failed(nullptr, TSM_EINVAL, "stationary parameter out of range");
    tsm_params p;
    tsm_default_params(&p);
    p.macro_cells = sp->macro_cells;
    p.d = sp->Dv;
    p.rtol = sp->rtol;
    p.setup_rtol = sp->rtol;
    p.max_iter = sp->max_iter;
    p.flags = sp->flags;
    const tsm_status st = tsm_create(&p, stream, out);
    if (st != TSM_OK) return st;
    tsm_ctx* c = *out;
    c->stationary = true;
    c->sp = *sp;
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&c->st_side[k], hipStreamNonBlocking);
    for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&c->st_ev[k], hipEventDisableTiming);
    if (e == hipSuccess) e = dalloc(&c->st_queue, 2);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return create_failed(c, TSM_EHIP, std::string("stationary context resources: ") + hipGetErrorString(e));
    }
    return TSM_OK;
}

tsm_status tsm_stationary_solve(tsm_ctx* c, double* u_out, double* w_out, int64_t n_inst, double* v_out,
                                int64_t n_v) {
    const Range range("tsm_stationary_solve");
    if (!c) return TSM_EINVAL;
    if (!c->stationary) return c->fail(TSM_ESTATE, "not a stationary context (tsm_stationary_create)");
    if (!c->have_geom) return c->fail(TSM_ESTATE, "set_deformation or set_jacobians first");
    if (!u_out || !w_out) return c->fail(TSM_EINVAL, "u_out or w_out is NULL");
    if (n_inst != c->n_inst)
        return c->fail(TSM_EINVAL, "u_out and w_out must hold n_inst = " + std::to_string(c->n_inst) + " entries");
    if (v_out && n_v != c->total)
        return c->fail(TSM_EINVAL, "v_out must hold the " + std::to_string(c->total) + " ragged entries");
    const int64_t ni = c->n_inst;
    const tsm_stationary_params& sp = c->sp;
    if (!c->ev_mid) HIPCHK(hipEventCreate(&c->ev_mid));
    HIPCHK(hipMemsetAsync(c->counters, 0, 4 * sizeof(int32_t), c->stream));
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    // loads: micro F^v (bulk source and Robin/Neumann data), the part
    // integrals of the data, the macro loads and the Dirichlet values
    StationaryLoadArgs la{};
    la.n_inst = (int)ni;
    la.level = c->level;
    la.offsets = c->offsets;
    la.wc_off = c->st_wcoff;
    la.wb_off = c->st_wboff;
    la.wcell = c->st_wcell;
    la.wbnd = c->st_wbnd;
    la.fv = c->st_has[0] ? c->st_dfv : nullptr;
    la.gv = c->st_has[1] ? c->st_dgv : nullptr;
    la.fv_const = sp.fv;
    for (int s = 0; s < 4; ++s) {
        la.parts[s] = sp.parts[s];
        la.dirichlet[s] = sp.dirichlet[s] != 0;
    }
    la.Fv = c->st_Fv;
    la.GI = c->st_GI;
    la.GO = c->st_GO;
    la.NM = c->NM;
    la.fu = c->st_has[2] ? c->st_dfu : nullptr;
    la.fw = c->st_has[3] ? c->st_dfw : nullptr;
    la.gu = c->st_has[4] ? c->st_dgu : nullptr;
    la.gw = c->st_has[5] ? c->st_dgw : nullptr;
    la.uD = c->st_has[6] ? c->st_duD : nullptr;
    la.fu_const = sp.fu;
    la.fw_const = sp.fw;
    la.uD_const = sp.u_dirichlet;
    la.Fu = c->st_Fu;
    la.Fw = c->st_Fw;
    la.uDn = c->st_uDn;
    HIPCHK(launch_stationary_loads(la, c->stream));
    // the three batched micro solves (FP64, zero initial guess) are
    // independent: they run side by side on the context's stream and the two
    // side streams, each with its own work counter, so that a small batch
    // still fills the chip.  Each leaves b_I^T x (the kernels' b is b_I):
    // b_I^T z^I, b_I^T z^O and b_I^T z^0 come with the solves.
    const bool with_f = sp.fv != 0.0 || c->st_has[0] || c->st_has[1];
    const int n_solve = with_f ? 3 : 2;
    const double* rhs[3] = {c->b, c->st_bO, c->st_Fv};
    const double scale[3] = {1.0, 1.0, 1.0};
    double* sol[3] = {c->st_zI, c->st_zO, c->st_z0};
    double* bx[3] = {c->st_dots, c->st_dots + 2 * ni, c->st_dots + 3 * ni};
    hipStream_t strm[3] = {c->stream, c->st_side[0], c->st_side[1]};
    int32_t* queue[3] = {c->queue, c->st_queue, c->st_queue + 1};
    if (!with_f) {
        HIPCHK(launch_fill_i32(c->st_iters + 2 * ni, 0, (int)ni, c->stream));
        HIPCHK(hipMemsetAsync(c->st_dots + 3 * ni, 0, 2 * ni * sizeof(double), c->stream));
    }
    HIPCHK(hipEventRecord(c->st_ev[0], c->stream));
    for (int q = 1; q < n_solve; ++q) HIPCHK(hipStreamWaitEvent(strm[q], c->st_ev[0], 0));
    MicroArgs ma = micro_base(c);
    ma.X0 = nullptr;
    ma.coef = nullptr;
    ma.zero_init = 1;
    ma.inv_dt = 0.0;
    ma.rtol = sp.rtol;
    ma.max_iter = sp.max_iter;
    for (int q = 0; q < n_solve; ++q) {
        ma.rhs_vec = rhs[q];
        ma.rhs_scale = scale[q];
        ma.X_out = sol[q];
        ma.bx_out = bx[q];
        ma.iters_out = c->st_iters + q * ni;
        ma.sweeps_out = c->st_sweeps + q * ni;
        const tsm_status st = enqueue_micro(c, ma, true, strm[q], queue[q], q);
        if (st != TSM_OK) {
            (void)hipDeviceSynchronize();   // nothing left running on the side streams
            return st;
        }
    }
    for (int q = 1; q < n_solve; ++q) {
        HIPCHK(hipEventRecord(c->st_ev[q], strm[q]));
        HIPCHK(hipStreamWaitEvent(c->stream, c->st_ev[q], 0));
    }
    HIPCHK(hipEventRecord(c->ev_mid, c->stream));
    // b_O^T z^O and b_O^T z^0
    HIPCHK(launch_bdot((int)ni, c->offsets, c->st_bO, c->st_zO, c->st_dots + ni, c->stream));
    if (with_f) HIPCHK(launch_bdot((int)ni, c->offsets, c->st_bO, c->st_z0, c->st_dots + 4 * ni, c->stream));
    StationaryMacroArgs m{};
    m.NM = c->NM;
    m.Dw = sp.Dw;
    m.k1 = sp.kappa1;
    m.k2 = sp.kappa2;
    m.k3 = sp.kappa3;
    m.k4 = sp.kappa4;
    m.Fu = c->st_Fu;
    m.Fw = c->st_Fw;
    m.uDn = c->st_uDn;
    m.GI = c->st_GI;
    m.GO = c->st_GO;
    for (int s = 0; s < 4; ++s) m.dirichlet[s] = sp.dirichlet[s] != 0;
    m.lenI = c->len;
    m.lenO = c->st_lenO;
    m.dots = c->st_dots;
    m.u = c->u;
    m.w = c->st_w;
    m.work = c->st_work;
    m.rtol = sp.macro_rtol;
    m.max_iter = sp.macro_max_iter;
    m.info = c->st_info;
    HIPCHK(launch_stationary_macro(m, c->stream));
    if (v_out)
        HIPCHK(launch_stationary_micro((int)ni, c->offsets, with_f ? c->st_z0 : nullptr, c->st_zI, c->st_zO, c->u,
                                       c->st_w, sp.kappa1, sp.kappa3, v_out, c->stream));
    HIPCHK(hipMemcpyAsync(u_out, c->u, ni * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(w_out, c->st_w, ni * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));

    std::vector<int32_t> it(3 * ni);
    double info[2];
    int32_t nc = 0;
    HIPCHK(hipMemcpy(it.data(), c->st_iters, 3 * ni * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(info, c->st_info, sizeof(info), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&nc, c->counters, sizeof(int32_t), hipMemcpyDeviceToHost));
    tsm_stationary_stats& S = c->st_stats;
    std::memset(&S, 0, sizeof(S));
    for (int q = 0; q < 3; ++q) {
        double sum = 0.0;
        int32_t mx = 0;
        for (int64_t i = 0; i < ni; ++i) {
            sum += it[q * ni + i];
            mx = std::max(mx, it[q * ni + i]);
        }
        S.micro_iters_max[q] = mx;
        S.micro_iters_mean[q] = sum / (double)ni;
    }
    S.unconverged = nc;
    S.macro_iters = (int32_t)info[0];
    S.macro_rel_residual = info[1];
    float ms = 0.0f, ms_micro = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    HIPCHK(hipEventElapsedTime(&ms_micro, c->ev0, c->ev_mid));
    S.solve_ms = ms;
    S.micro_ms = ms_micro;
    if (nc > 0) return c->fail(TSM_ENOCONV, std::to_string(nc) + " micro solves missed rtol");
    if (!(info[1] <= sp.macro_rtol))
        return c->fail(TSM_ENOCONV, "macro solve stopped at relative residual " + std::to_string(info[1]));
    return TSM_OK;
}

tsm_status tsm_stationary_set_data(tsm_ctx* c, const double* fv_cell, int64_t n_fv, const double* gv_bnd,
                                    int64_t n_gv, const double* fu_cell, int64_t n_fu, const double* fw_cell,
                                    int64_t n_fw, const double* gu_bnd, int64_t n_gu, const double* gw_bnd,
                                    int64_t n_gw, const double* uD, int64_t n_uD) {
    if (!c) return TSM_EINVAL;
    if (!c->stationary) return c->fail(TSM_ESTATE, "not a stationary context (tsm_stationary_create)");
    if (!c->have_mesh) return c->fail(TSM_ESTATE, "set_reference_mesh first");
    const int64_t nM = c->NM, ni = c->n_inst;
    const double* src[7] = {fv_cell, gv_bnd, fu_cell, fw_cell, gu_bnd, gw_bnd, uD};
    const int64_t given[7] = {n_fv, n_gv, n_fu, n_fw, n_gu, n_gw, n_uD};
    const char* name[7] = {"fv_cell", "gv_bnd", "fu_cell", "fw_cell", "gu_bnd", "gw_bnd", "uD"};
    double** dst[7] = {&c->st_dfv, &c->st_dgv, &c->st_dfu, &c->st_dfw, &c->st_dgu, &c->st_dgw, &c->st_duD};
    const int64_t len[7] = {c->st_ncell, c->st_nbnd, 4 * nM * nM, 4 * nM * nM, 8 * nM, 8 * nM, ni};
    for (int q = 0; q < 7; ++q)
        if (src[q] && given[q] != len[q])
            return c->fail(TSM_EINVAL, std::string(name[q]) + " has " + std::to_string(given[q]) + " values, expected " +
                                           std::to_string(len[q]));
    HIPCHK(hipDeviceSynchronize());   // the caller's producers of the data
    for (int q = 0; q < 7; ++q) {
        c->st_has[q] = src[q] != nullptr;
        if (!src[q]) continue;
        if (!*dst[q]) HIPALLOC(*dst[q], len[q]);
        HIPCHK(hipMemcpyAsync(*dst[q], src[q], len[q] * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return TSM_OK;
}

tsm_status tsm_stationary_get_stats(const tsm_ctx* c, tsm_stationary_stats* s) {
    if (!c || !s) return TSM_EINVAL;
    *s = c->st_stats;
    return TSM_OK;
}

void tsm_destroy(tsm_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    c->free_mesh();
    c->free_macro();
    dfree(c->counters);
    dfree(c->queue);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev_mid) (void)hipEventDestroy(c->ev_mid);
    for (hipEvent_t e : c->st_ev)
        if (e) (void)hipEventDestroy(e);
    dfree(c->st_queue);
    for (hipStream_t s : c->st_side)
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
