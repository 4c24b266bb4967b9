// Internal declarations shared by the HIP sources of libtsm (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

#include "tsm.h"

namespace tsm {

constexpr int kMicroThreads = 256;        // lanes per micro workgroup (4 waves), generic kernels
constexpr int kPackThreads = 768;         // lanes per packed workgroup (12 waves)
constexpr int kWave = 64;
constexpr int kMaxLevel = 64;             // largest micro mesh N of the packed, register- and
                                          // LDS-resident kernels, the indicator and refinement
constexpr int kMaxMesh = 256;             // largest micro mesh N (cells per side) of a batch
constexpr int kMinLevel = 2;
constexpr int kStencil = 9;               // 9-point Q1 stencil, k = (dj2+1)*3 + (dj1+1)
// The operators are symmetric, so the packed kernels read only the upper half
// of each row, k = 4..8 (centre, E, NW, N, NE), stored as planes p = k - 4;
// the lower coefficients of node j are upper ones of its neighbours:
//   k=3 (W) = E of j-1,   k=1 (S) = N of j-NP,
//   k=0 (SW) = NE of j-NP-1,   k=2 (SE) = NW of j-NP+1.
constexpr int kSym = 5;
// Zeroed entries after the last instance's planes: a packed kernel reads up
// to 2(N+1) entries past an instance's block (strip rows past its mesh, on
// lanes that own mesh rows; the other lanes address from the block's start).
constexpr int kPlanePad = 4 * (kMaxLevel + 1);

// Boundary nodes of an N x N instance in a compact order: the bottom row
// (N+1 nodes), the top row (N+1), then the first and the last column of the
// interior rows (N-1 each), 4N in all; per instance at stride kBndStride.
constexpr int kBndStride = 4 * kMaxLevel;
__host__ __device__ inline int bnd_node(int N, int k) {
    const int NP = N + 1;
    if (k < NP) return k;
    if (k < 2 * NP) return N * NP + (k - NP);
    if (k < 2 * NP + N - 1) return (k - 2 * NP + 1) * NP;
    return (k - 2 * NP - N + 2) * NP + N;
}

// Tightest relative tolerance asked of an FP32 inner solve (2^-17, 64 FP32
// ulps).  The correction of an FP32 solve is accurate to about cond(S)
// FP32 ulps whatever its own residual says, so iterating further only
// costs iterations (measured on 64x64 instances: 2^-20 -> 2^-18 saved two
// of 24 iterations per step, and with the extrapolated start 2^-18 ->
// 2^-17 saves 0.4 of 12.1, no refinement sweep added either time).
constexpr double kInnerFloor = 7.62939453125e-06;

// Squared relative tolerance of one FP32 inner solve in the refinement: half
// of what the outer test still needs (tol2 = rtol^2 ||b||^2 against the
// current squared FP64 residual rr), no tighter than kInnerFloor and no
// looser than cap.  A correction solved this far usually ends the
// refinement; a looser one would cost another FP64 residual pass, a tighter
// one iterations that the outer test does not need.
__host__ __device__ inline float inner_tol2(double tol2, double rr, double cap) {
    double t = 0.25 * tol2 / rr;
    const double lo = kInnerFloor * kInnerFloor, hi = cap * cap;
    t = t < lo ? lo : t;
    t = t > hi ? hi : t;
    return (float)t;
}

// Per-level quadrature tables: for level N, entries [tab_off[N], tab_off[N] + 2N + 2).
// Entry t < 2N is the Gauss abscissa y_t = -1 + (t/2 + g_{t%2}) h of cell t/2;
// entries 2N and 2N+1 are the edges y = -1 and y = +1.
// s_t = sin(pi y_t)/4 and c_t = pi cos(pi y_t)/4, so the displacement
// gradient is G = [[c(y1) y2, s(y1)], [s(y2), c(y2) y1]].
struct Tables {
    const int32_t* off;   // [kMaxMesh + 1]
    const double* y;
    const double* s;
    const double* c;
};

struct AssembleArgs {
    int n_inst;
    const int32_t* level;
    const int64_t* offsets;
    const double* amp;
    Tables tab;
    double d, inv_dt;
    // sides of Z in the order bottom (y2 = -1), top (y2 = +1), left (y1 = -1), right (y1 = +1)
    double kside[4];      // Robin coefficient of each side in S (kappa on every side: whole-boundary exchange)
    double bw[4];         // b = sum over sides of bw[side] (B_side 1)
    double* b2;           // optional second load sum bw2[side] (B_side 1) (null: none)
    double bw2[4];
    double* len2;         // [n_inst] 1^T b2 (with b2)
    // optional (null: none): the quadrature weights times the geometry at every
    // point, for load assembly -- wq J at the cell points (per instance at
    // wc_off[i], cells c2*N+c1, points g2*2+g1) and wb |F tau| at the
    // boundary points (at wb_off[i], sides bottom, top, left, right; edges; 2 points)
    double* wcell;
    double* wbnd;
    const int64_t* wc_off;
    const int64_t* wb_off;
    double* S64;          // [9 * total] : instance block at 9*off, coefficient-major [k][n]
    float* S32;           // S rounded to FP32
    float* Slo;           // S - S32 rounded to FP32: S32 + Slo equals S to about 2^-48 relative
    double* M64;
    // upper-half planes [kSym][n] at kSym*off (symmetric storage, see kSym)
    double* Ss64;         // S
    double* Ks64;         // K = d A + kappa B = S - M/dt, accumulated on its own
    float* Ss32;          // S rounded to FP32
    float* Sslo;          // S - Ss32 rounded to FP32
    double* b;            // boundary load B 1 (ragged)
    double* len;          // [n_inst] 1^T b
    double* jmin;         // [n_inst] minimum det over all quadrature points (-1: non-finite Jacobian)
    // general maps (launch_assemble_tables): D zeta at the quadrature points,
    // per instance at cell_off[i] (cells c2*N+c1, points g2*2+g1, 4 entries
    // F11 F12 F21 F22) and bnd_off[i] (sides bottom, top, left, right; edges;
    // 2 points; 4 entries)
    const double* Fcell;
    const double* Fbnd;
    const int64_t* cell_off;
    const int64_t* bnd_off;
};

// One batched micro solve: for every task t, instance i = order[t] solves
//   S_i x = rhs_i,   rhs_i = rhs_scale * rhs_vec_i [+ rhs_bscale * rhs_bcoef_i * b_i]   (rhs_vec != null)
//                    rhs_i = M_i x0_i / dt                (otherwise)
// from the initial guess x0_i = X0_i + coef_i * w_i (zero if zero_init; X0_i
// alone with Mw, see there).
// Writes x to X_out and b_i^T x to bx_out[i].
struct MicroArgs {
    int n_tasks;
    const int32_t* order;
    const int64_t* order_off;   // offsets[order[t]] (packed kernels)
    const int32_t* level;
    const int64_t* offsets;
    const double* S64;
    const float* S32;
    const float* Slo;
    const double* M64;
    const double* Ss64;   // symmetric upper-half planes (packed kernels)
    const double* Ks64;
    const float* Ss32;
    const float* Sslo;
    const double* b;
    const double* X0;
    const double* w;
    const double* coef;
    const double* rhs_vec;
    double rhs_scale;
    // M_i w_i per node (packed kernels, time-step form, may be null): with it
    // the iteration starts from X0 instead of X0 + coef w; the right-hand side
    // is unchanged, M (X0 + coef w)/dt, so r = -K X0 + coef Mw / dt
    const double* Mw;
    const double* rhs_bcoef;   // with rhs_vec: rhs_i += rhs_bscale * rhs_bcoef[i] * b_i (may be null)
    double rhs_bscale;
    double* res_out;           // optional: final FP64 residual norm ||rhs - S x||_2 per instance
    int zero_init;
    double* X_out;
    double* bx_out;       // b_i^T x_i per instance (packed kernels: null, a separate boundary pass)
    int32_t* iters_out;
    int32_t* sweeps_out;
    int32_t* nonconv;     // device counter, incremented by instances that miss rtol
    double inv_dt;
    double rtol, inner_rtol;
    int max_iter, max_refine;
    int32_t* queue;       // persistent work counter (null: task = blockIdx.x)
    // matrix-free operator of the time-step solves (packed kernels, mode 3):
    // the amplitudes, the per-level quadrature tables and the coefficients of
    // S = M/dt + d A + kappa B (inv_dt above)
    const double* amp;
    Tables tab;
    double d, kappa;
    // meshes above kMaxLevel (launch_micro_large): workspace of three ragged
    // vectors (r, p, q), ws_stride doubles apart
    double* ws;
    int64_t ws_stride;
    // FP64 recovery of the packed refinement solves (may be null): an
    // instance that misses rtol after max_refine sweeps is not stored but
    // appended to fb_list ([0] count, then instance indices), and
    // launch_micro_fallback solves it again in FP64 from X0
    int32_t* fb_list;
    // extrapolated start of the forward time-step solves (packed kernels on
    // the assembled operator, all null elsewhere): hx holds the X0 of the
    // previous step, he the increment before it and he2 the one before that
    // (FP32, ragged like X0), *hn the number of steps that history covers
    // (0 .. 3).  The solve starts from X0 + 3 e1 - 3 e2 + e3 (e1 = X0 - hx,
    // e2 = he, e3 = he2), X0 + 2 e1 - e2 with two steps known, X0 + e1 with
    // one (the refinement form: its first inner solve)
    float* hx;
    float* he;
    float* he2;
    const int32_t* hn;
    // separable mass of the analytic deformation family (packed kernels on
    // the assembled operator, time-step form; null: none).  For level N the
    // table starts at mass1d + 8 tab.off[N]: 15 planes of N+1 doubles, plane
    // 3 f + d + 1 the 1D Q1 mass weighted at the Gauss points by function f
    // (1, c, y, c y, s) between node j and node j + d (d = -1, 0, +1; zero
    // past the ends).  With it the start residual is coef M w/dt + M x0/dt
    // - S x0 (S from the stencil the solve holds) instead of -K x0 + coef
    // M w/dt with K read from the assembled planes.
    const double* mass1d;
};

// Packs of instances of one mesh size solved by one kPackThreads-lane workgroup.
constexpr int kPackSlots = 16;             // slot stride of a pack (the most instances a pack holds)

struct PackList {
    int n_packs;
    const int32_t* first;   // first task (index into MicroArgs::order)
    const int32_t* count;   // instances in the pack
    // per pack slot (pack * kPackSlots + sub): the instance and its offset,
    // so a workgroup finds its instances in one dependent load
    const int32_t* slot_inst;
    const int64_t* slot_off;
};

struct MacroArgs {
    int NM;               // macro cells per side
    int n;                // interior nodes per side = NM - 1
    double mass_c;        // H^2 / (36 dt)
    double lap_c;         // D / 3
    double sig_h2;        // source_sign * H^2 (nodal weight L_kk of interior nodes times sign)
    double kappa, p;
    const double* beta;   // [n_inst]
    const double* len;    // [n_inst]
};

// The eliminated macro system of the stationary three-field model, solved by
// one workgroup (Jacobi-PCG).
struct StationaryMacroArgs {
    int NM;                       // macro cells per side of [-1,1]^2
    double Dw, k1, k2, k3, k4;
    int dirichlet[4];             // sides bottom, top, left, right: u prescribed
    const double* lenI;           // [n] |G^I| = 1^T b_I per node
    const double* lenO;           // [n] |G^O|
    const double* dots;           // [5][n] b_I^T z^I, b_O^T z^O, b_I^T z^O, b_I^T z^0, b_O^T z^0
    const double* Fu;             // [n] int f^u xi_k + the Neumann load of u (non-Dirichlet sides)
    const double* Fw;             // [n] int f^w xi_k + the Neumann load of w
    const double* uDn;            // [n] u at the Dirichlet nodes
    const double* GI;             // [n] int over G^I of g^v_1 at node k
    const double* GO;             // [n] int over G^O of g^v_2
    double* u;                    // [n] out
    double* w;                    // [n] out
    double* work;                 // [11 n] scratch
    double rtol;
    int max_iter;
    double* info;                 // [2] out: iterations, final ||r|| / ||b||
};

// launchers (return hipError_t of the launch)
hipError_t launch_assemble(const AssembleArgs& a, hipStream_t s);
// same gather for maps given by their Jacobian tables (a.Fcell, a.Fbnd)
hipError_t launch_assemble_tables(const AssembleArgs& a, hipStream_t s);
hipError_t launch_micro(const MicroArgs& a, int slots, int mode, int grid, size_t lds_bytes, hipStream_t s);
// instances with more than kMaxLevel cells per side: one 1024-lane workgroup
// per task, vectors in the workspace a.ws (FP64 in either precision mode)
hipError_t launch_micro_large(const MicroArgs& a, hipStream_t s);
// FP64 Jacobi PCG of the instances in a.fb_list (the same right-hand sides
// and outputs as the packed kernels, b^T x left to the boundary pass), one
// 1024-lane workgroup per listed instance, `grid` workgroups looping over
// the list; vectors r, p, q at ws + (3 blockIdx.x + k) * slot.  Adds the
// list's count to counters[2]; an instance that misses rtol again counts in
// a.nonconv.
hipError_t launch_micro_fallback(const MicroArgs& a, double* ws, int64_t slot, int grid, int32_t* counters,
                                 hipStream_t s);

// Multigrid-preconditioned micro solves (mg.hip).  An instance with
// N = c 2^L cells per side, c <= kMgCoarsest, L >= 1, has coarse levels
// 1..L (N >> l cells per side), their Galerkin operators in Ac (9
// coefficient-major planes per level at 9 * (coff + level offset)), the
// coarsest operator's dense inverse at inv + ioff, and a Jacobi damping per
// smoothed level.
constexpr int kMgMaxLevels = 8;
constexpr int kMgCoarsest = 8;
struct MgArgs {
    const int32_t* nlev;   // [n_inst] L (0: not on the multigrid path)
    const int64_t* coff;   // [n_inst] offset of the instance's coarse levels (vectors; x9 for operators)
    const int64_t* ioff;   // [n_inst] offset of the coarsest inverse
    double* Ac;
    double* inv;
    double* omega;         // [n_inst][kMgMaxLevels + 1]
    double* ws;            // fine-level vectors r, z, t, p, q: ws + k * ws_stride + offset
    int64_t ws_stride;
    double* cws;           // coarse-level vectors x, r, t: cws + k * cws_stride + coarse offset
    int64_t cws_stride;
    int nu;                // smoothing sweeps before and after the coarse correction
};
hipError_t launch_micro_mg(const MicroArgs& a, const MgArgs& g, hipStream_t s);
// Galerkin operators (levels 0 -> max_levels), damping, coarsest inverses
hipError_t launch_mg_setup(const MicroArgs& a, const MgArgs& g, int n_inst, int max_levels, hipStream_t s);
// packs of one mesh size (16, 32 or 64); mode 1 FP64, 2 refinement, 3 refinement
// with the operator evaluated matrix-free from the amplitudes (time-step form only)
hipError_t launch_packed(const MicroArgs& a, const PackList& p, int level, int mode, int grid, hipStream_t s);
// every pack of every size in one persistent launch (work queue a.queue, reset to 0 beforehand)
hipError_t launch_packed_mixed(const MicroArgs& a, const PackList& p, const int32_t* pack_level, int mode,
                               int grid, size_t lds, hipStream_t s);
int packed_capacity(int level);          // instances per pack (0: no packed kernel for this size)
size_t packed_lds_bytes(int level);      // dynamic LDS of one pack
hipError_t launch_apply(int n_inst, const int32_t* level, const int64_t* offsets,
                        const double* S64, const double* x, double* y, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int n, hipStream_t s);
// *hn = min(*hn + 1, 2): the forward step just taken extends the history of
// the extrapolated start
hipError_t launch_history_advance(int32_t* hn, hipStream_t s);
// out_i = b_i^T x_i for every instance
hipError_t launch_bdot(int n_inst, const int64_t* offsets, const double* b, const double* x, double* out,
                       hipStream_t s);
// out[order[t]] = b^T x over the boundary nodes of instance order[t], t < n_tasks
// (b vanishes at interior nodes), with b in the compact boundary order
hipError_t launch_bdot_boundary(int n_tasks, const int32_t* order, const int32_t* level, const int64_t* offsets,
                                const double* bc, const double* x, double* out, hipStream_t s);
// bc[i * kBndStride + k] = b_i at boundary node bnd_node(N_i, k)
hipError_t launch_stationary_macro(const StationaryMacroArgs& a, hipStream_t s);
// Micro loads of the stationary system: Fv_i = int f^v eta J + int g^v eta |F tau|
// (f^v and g^v at the quadrature points, or fv_const / 0 where null), and the
// part integrals GI_i, GO_i of g^v; from the weights of AssembleArgs::wcell/wbnd.
struct StationaryLoadArgs {
    int n_inst;
    const int32_t* level;
    const int64_t* offsets;
    const int64_t* wc_off;
    const int64_t* wb_off;
    const double* wcell;
    const double* wbnd;
    const double* fv;             // [4 sum N^2] or null
    const double* gv;             // [8 sum N] or null
    double fv_const;
    int parts[4];
    double* Fv;                   // ragged out
    double* GI;                   // [n_inst] out
    double* GO;                   // [n_inst] out
    // macro loads (one extra block): f^u, f^w at the macro cell points and
    // grad u . n, Dw grad w . n at the macro boundary points (null: constants, 0),
    // u at the nodes (null: uD_const)
    int NM;
    const double* fu;
    const double* fw;
    const double* gu;
    const double* gw;
    const double* uD;
    double fu_const, fw_const, uD_const;
    int dirichlet[4];
    double* Fu;
    double* Fw;
    double* uDn;
};
hipError_t launch_stationary_loads(const StationaryLoadArgs& a, hipStream_t s);

// Error indicator eta_i^2 of the micro fields v = v0 + u_i w (refine.hip).
struct IndicatorArgs {
    int n_inst;
    const int32_t* level;
    const int64_t* offsets;
    const double* amp;
    const double* u;
    const double* v0;
    const double* w;
    double d;
    double* eta2;          // [n_inst] out
};
hipError_t launch_indicator(const IndicatorArgs& a, hipStream_t s);
// Nested Q1 interpolation of ragged fields: level ln[i] is lo[i] or 2 lo[i]
hipError_t launch_prolong(int n_inst, const int32_t* lo, const int32_t* ln, const int64_t* oo, const int64_t* on,
                          const double* vo, double* vn, hipStream_t s);
// v_i = z0_i + k1 u_i zI_i + k3 w_i zO_i (z0 may be null: zero), ragged
hipError_t launch_stationary_micro(int n_inst, const int64_t* offsets, const double* z0, const double* zI,
                                   const double* zO, const double* u, const double* w, double k1, double k3,
                                   double* v, hipStream_t s);
hipError_t launch_bnd_gather(int n_inst, const int32_t* level, const int64_t* offsets, const double* b, double* bc,
                             hipStream_t s);
// residual sum of the alternating coupling: out[0] = ||R||_2 (nR interior macro rows),
// out[1] = mean over instances of res (per-instance micro residual norms)
hipError_t launch_coupling_residual(int nR, const double* R, int n_inst, const double* res, double* out,
                                    hipStream_t s);
// Failure of a call that has no context: the message becomes
// tsm_last_error(NULL) of the calling thread; returns st.
tsm_status call_failed(tsm_status st, const std::string& msg);

// macro kernels
hipError_t launch_macro_rhs_forward(const MacroArgs& m, const double* u, const double* bx,
                                    double* rhs, double* alpha, hipStream_t s);
hipError_t launch_macro_rhs_adjoint(const MacroArgs& m, const double* mu_next, const double* blam,
                                    const double* u_final, int add_terminal, double* rhs, hipStream_t s);
hipError_t launch_macro_residual(const MacroArgs& m, const double* u, const double* rhs, double* R, hipStream_t s);
// C = A * B (n x n row-major); epilogue 0: C stored; 1: C ./= lam; 2: u[interior] += C
hipError_t launch_gemm(int n, const double* A, const double* B, double* C, int epilogue,
                       const double* lam, double* u, int NM, hipStream_t s);
hipError_t launch_observable(const MacroArgs& m, const double* u, double* J, hipStream_t s);
// macro PCG with the sine-basis preconditioner: r, z, q interior (n x n), p
// full grid (zero boundary), s[0] = (r, z)
hipError_t launch_macro_pcg_start(int NM, const double* r, const double* z, double* p, double* s, hipStream_t st);
// The whole macro PCG (residual, preconditioner, iters steps) in one
// single-workgroup launch for NM - 1 <= 64 interior nodes per side
// (macro_pcg_fused_fits); u (full grid, zero boundary) in place.
bool macro_pcg_fused_fits(int NM);
hipError_t launch_macro_pcg_fused(const MacroArgs& m, double* u, const double* rhs, const double* Q,
                                  const double* lam, int iters, hipStream_t st);
hipError_t launch_macro_pcg_step(const MacroArgs& m, const double* p, double* q, double* r, double* u,
                                 const double* s, hipStream_t st);
hipError_t launch_macro_pcg_direction(int NM, const double* r, const double* z, double* p, double* s,
                                      hipStream_t st);
hipError_t launch_adjoint_coef(const MacroArgs& m, const double* mu, double* coef, hipStream_t s);

// Gradient contribution of one adjoint step m (one workgroup per instance):
//   g_i -= lam_i^T (dS_i v_i^m - kappa p u_i^m db_i - dM_i v_i^{m-1} / dt)
//          - sign mu_i L_ii dF_i,   dF_i = -kappa (db_i^T v_i^m / |dY_i| - (b_i^T v_i^m) d|dY_i| / |dY_i|^2)
// with lam_i = lam0_i + coef_i w_i; the derivative forms are evaluated
// matrix-free from the amplitudes and the quadrature tables.
struct GradArgs {
    int n_inst, NM;
    const int32_t* level;
    const int64_t* offsets;
    const double* amp;
    Tables tab;
    const double* len;
    const double *lam0, *coef, *w;
    const double *v_now, *v_prev, *u_now, *mu;
    double d, kappa, p, sign, inv_dt;
    double* g;
};
hipError_t launch_gradient_step(const GradArgs& a, hipStream_t s);

hipError_t launch_macro_finalize(const MacroArgs& m, const double* u, const double* alpha,
                                 double* F, hipStream_t s);
hipError_t launch_beta(int n_inst, double kappa, double p, const double* len, const double* bx,
                       double* beta, hipStream_t s);
hipError_t launch_state_split(int n_inst, const int64_t* offsets, const double* u, const double* v,
                              const double* w, double* v0, hipStream_t s);
hipError_t launch_state_join(int n_inst, const int64_t* offsets, const double* u, const double* v0,
                             const double* w, double* v, hipStream_t s);

}  // namespace tsm
