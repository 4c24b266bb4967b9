// Packed micro solves for the common mesh sizes (16, 32 and 64 cells per
// side): Jacobi-preconditioned CG (paper Section 3.5: CG on every micro
// system, the systems distributed over the processors), laid out for a
// 768-lane workgroup (12 waves, 3 per SIMD: 168 VGPRs per lane) that
// solves a pack of instances of one size in lockstep:
//     64x64: 1 instance on 12 waves (strips of 6 rows),
//     32x32: 3 instances on 4 waves each,  16x16: 12 instances on 1 wave each.
// (1024 lanes would give 4 waves per SIMD but only 128 VGPRs, and 64x64 would
// take 14 waves in strips of 5 rows: the busiest SIMD then carries 4 waves x
// 5 rows against 3 x 6 here, and the solver state spills.)
// Within an instance, lane l owns column l % (N+1) and a strip of R
// consecutive rows.  Each iteration it reads only the left/right neighbour
// columns and the two rows past its strip from LDS (2R+6 reads for R nodes,
// against 9R for one node per lane); its own column comes from registers.
// Vectors live in an LDS grid with a zero halo (rows past the mesh included),
// so boundary rows need no bounds checks.
//
// Operators are read from their symmetric upper-half planes (kSym): 5 stored
// coefficients per node instead of 9, so each operator read costs 40 (FP64)
// or 20 (FP32) bytes per node; the lower coefficients are loaded from the
// neighbours' planes (same cache lines as the neighbours' own loads).  Every
// operator is read once per solve: the solver's stencil into registers (FP32
// planes through an asynchronous LDS copy), and for the start residual
// either K or, for the analytic deformation family, nothing: its mass term
// comes from per-level 1D tables (mass_apply) and S x0 from the stencil.
//
// Register budget (768 lanes: 168 VGPRs per lane) decides the data flow:
//   FP64 form     the FP64 stencil rows resident in registers for the whole
//                 solve, r, p, q in FP64 registers, x in LDS, diag^{-1} in
//                 FP32 (the preconditioner need not be exact).
//   REFINE form   FP32 stencil and diag^{-1} resident in registers for the
//                 whole solve; FP32 PCG on S d = r/||r||; the FP64 residual
//                 is formed once as r = -K x0 (K = S - M/dt), or as
//                 M x0/dt - S32 x0 with the separable mass (the low part
//                 -Slo x0 joins at the first update), then updated
//                 as r <- r - ||r|| S d with the FP64 stencil (FP32 part in
//                 registers plus the FP32 low part from LDS), x <- x + ||r|| d,
//                 until ||r|| <= rtol ||b||.
//
// Lockstep: all instances of a pack pass the same barriers; an instance
// that has met its tolerance freezes while the others go on.  Dot products:
// a DPP wavefront sum ending in lane 63, one LDS exchange (ping-pong buffer,
// one barrier), a DPP sum over the waves of each instance; fixed order, so
// every wave of an instance holds the same bits.
#include <cmath>

#include "device_common.h"

namespace tsm {

namespace {

constexpr int NTP = kPackThreads;
constexpr int NWP = 16;                    // reduction slots: at most 16 waves
constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int N_, int TPI_, int R_>
struct Lvl {
    static constexpr int N = N_, NP = N_ + 1, W2 = N_ + 3, R = R_;
    static constexpr int NS = (NP + R_ - 1) / R_;          // strips per instance
    static constexpr int H2 = NS * R_ + 2;                  // grid rows: strips plus halo
    static constexpr int TPI = TPI_, WPI = TPI_ / kWave;    // lanes / waves per instance
    static constexpr int IPP = NTP / TPI_;                  // instances per pack
    static constexpr int GRID = H2 * W2;                    // LDS cells per instance
    static constexpr int n = NP * NP;
    // LDS stride of one instance's copied FP32 planes (planes_copy_start):
    // kSym*n floats shifted by up to 3, rounded up to whole 16-byte words
    static constexpr int PS = (kSym * NP * NP + 8 + 3) / 4 * 4;
    // DPP group of the second reduction level: the waves of one instance
    static constexpr int G = IPP == 1 ? 16 : WPI;
    static_assert(NS * NP <= TPI, "strips do not fit the lanes of an instance");
    static_assert(TPI % kWave == 0, "an instance owns whole waves");
    static_assert(IPP * WPI <= NWP && WPI <= G, "instances must fit one 16-lane DPP row");
    static_assert(IPP <= kPackSlots, "pack slots");
};
using L16 = Lvl<16, 64, 6>;
using L32 = Lvl<32, 256, 5>;
using L64 = Lvl<64, 768, 6>;

// Workgroup barrier for LDS traffic only.  __syncthreads() is also a memory
// fence, which makes every wave wait for all of its global loads, the
// asynchronous global->LDS plane copies included; this barrier waits only for
// the wave's own LDS operations, so a plane copy stays in flight across it.
// Every use orders LDS accesses alone.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Per-instance sums of NV values (NV <= 4).  Level 1: every wave reduces its
// lanes into lane 63 (wave_total_last), which writes the NV totals to LDS.
// Level 2, after the one barrier: lane l < IPP*WPI reads wave l's totals and
// a DPP sum over groups of G lanes gives every lane of a group its
// instance's totals; each wave takes them from lane w0 (its first wave).
// `tail` keeps, per lane of row 0, the group total of value NV-1 for the
// convergence vote (any_above).  All lanes must call.
template <int NV, typename T>
struct PackRed {
    T (*buf)[NWP][4];
    int phase = 0;
    T tail = T(0);
    __device__ PackRed(T (*b)[NWP][4]) : buf(b) {}
    template <class L>
    __device__ __forceinline__ void sum(T (&v)[NV], int w0) {
        static_assert(NV <= 4, "at most 4 values");
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = wave_total_last(v[i]);
        if (lane == kWave - 1) {
#pragma unroll
            for (int i = 0; i < NV; ++i) buf[phase][wid][i] = v[i];
        }
        lds_barrier();
        const bool has = lane < L::IPP * L::WPI;
        const T* slot = buf[phase][lane & (NWP - 1)];   // in bounds for every lane
        T t[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) t[i] = slot[i];
#pragma unroll
        for (int i = 0; i < NV; ++i) t[i] = has ? t[i] : T(0);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            t[i] = group_sum<L::G>(t[i]);
            v[i] = lane_read(t[i], w0);
        }
        tail = t[NV - 1];
        phase ^= 1;
    }
    // Some instance's value NV-1 (of the last sum) exceeds its threshold
    // (thr: per lane, see lane_threshold).  Uniform over the workgroup.
    __device__ __forceinline__ bool any_above(T thr) const { return __ballot(tail > thr) != 0; }
};

// Per-lane threshold for any_above: the group leaders (lane q*WPI of
// instance q of the pack) hold instance q's threshold, all others +inf.
template <class L, typename T>
__device__ __forceinline__ T lane_threshold(const T* thr_s, int cnt) {
    const int lane = threadIdx.x & (kWave - 1);
    const int q = lane / L::WPI;
    const bool lead = lane % L::WPI == 0 && q < L::IPP && q < cnt;
    return lead ? thr_s[lead ? q : 0] : T(INFINITY);
}

struct Lane {
    int sub, lt, col, r0, inst, w0;     // w0: first wave of the instance (0 for spare lanes)
    bool live, act;
    int64_t off;
};

// A pack's metadata, copied into LDS ahead of its solve (meta_copy_start):
// slot instances [0, 16), slot offsets as int64 [16, 48), instance count 48,
// mesh size 49.
constexpr int kMetaInst = 0, kMetaOff = 16, kMetaCount = 48, kMetaLevel = 49, kMetaWords = 64;

template <class L>
__device__ __forceinline__ Lane lane_of(const int32_t* meta, int cnt) {
    Lane z;
    // the lane geometry is recomputed for every pack: hidden from the
    // compiler, so that it is not hoisted out of the work-queue loop and
    // held (or spilled) across every solve
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    z.sub = tid / L::TPI;
    z.lt = tid - z.sub * L::TPI;
    z.w0 = (z.sub < L::IPP ? z.sub : 0) * L::WPI;
    z.live = z.sub < L::IPP && z.sub < cnt;
    // every wave belongs to one instance: instance and offset are wave-uniform
    // and come from the pack's slot in the LDS copy of its metadata
    const int t = z.live ? z.sub : 0;
    const int inst = z.live ? meta[kMetaInst + t] : 0;
    const int64_t off = z.live ? *reinterpret_cast<const int64_t*>(meta + kMetaOff + 2 * t) : 0;
    z.inst = __builtin_amdgcn_readfirstlane(inst);
    z.col = z.lt % L::NP;
    const int strip = z.lt / L::NP;
    z.r0 = strip * L::R;
    z.act = z.live && strip < L::NS;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)off & 0xffffffffu));
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)off >> 32));
    z.off = (int64_t)(((uint64_t)hi << 32) | lo);
    return z;
}

template <class L>
__device__ __forceinline__ bool row_ok(const Lane& z, int i) { return z.act && z.r0 + i < L::NP; }
template <class L>
__device__ __forceinline__ int node_of(const Lane& z, int i) { return (z.r0 + i) * L::NP + z.col; }
template <class L>
__device__ __forceinline__ int cell_of(const Lane& z, int i) { return (z.r0 + i + 1) * L::W2 + z.col + 1; }

// Zero the halo of one instance's grid: row 0, rows NP+1 .. H2-1 and the
// first and last column.
template <class L, typename T>
__device__ __forceinline__ void zero_halo(T* g, const Lane& z) {
    if (z.sub >= L::IPP) return;
    constexpr int NROWS = L::H2 - L::NP;                    // row 0 and rows NP+1..H2-1
    constexpr int NH = NROWS * L::W2 + 2 * L::H2;
    for (int t = z.lt; t < NH; t += L::TPI) {
        int idx;
        if (t < NROWS * L::W2) {
            const int hr = t / L::W2, e = t % L::W2;
            idx = (hr == 0 ? 0 : L::NP + hr) * L::W2 + e;
        } else {
            const int u = t - NROWS * L::W2;
            idx = (u % L::H2) * L::W2 + ((u / L::H2) ? L::W2 - 1 : 0);
        }
        g[idx] = T(0);
    }
}

// Write the lane's strip values to the grid.  Rows past the mesh carry 0 in
// every vector the kernels write, so they land on the zero halo unchanged.
template <class L, typename T>
__device__ __forceinline__ void strip_store(T* g, const Lane& z, const T (&v)[L::R]) {
    if (z.act) {
#pragma unroll
        for (int i = 0; i < L::R; ++i) g[cell_of<L>(z, i)] = v[i];
    }
}

// The plane bases of a streamed stencil pass through an empty asm at every
// application (SymStencil::prepare), so the compiler cannot hoist the
// coefficient loads out of the work loop and keep them live across solves.
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Coefficient k of the 9-point row of the lane's strip row i is read from the
// upper-half planes of the instance ([kSym][n]).  The lower couplings index a
// neighbour node; for mesh row 0 such an index falls at most NP+1 entries
// into the previous plane (never before the block).  Wrapped reads at the
// left and right edges hit coefficients that are structurally zero (E and NE
// of the last column, NW of the first column, N of the top row), so only the
// bottom mesh row needs a mask (sym_mask).
template <class L, typename T>
__device__ __forceinline__ T sym_mask(const Lane& z, int i, int k, T v) {
    if (i == 0 && k <= 3) {
        // strip row 0 may be mesh row 0: no southern neighbours, and node 0 has no W
        const bool ok = (k == 3) ? (z.r0 > 0 || z.col > 0) : (z.r0 > 0);
        return ok ? v : T(0);
    }
    return v;
}


// The same coefficients from a copy of the instance's planes in LDS, read
// from two per-lane base addresses (planes 0-1 from the lane's node in strip
// row 0, planes 2-4 from one plane further) plus compile-time offsets, all
// non-negative and below 64 KiB (the instruction's offset field): no
// per-coefficient address arithmetic.  Strip rows past the mesh read up to
// 2(N+1) floats past the instance's planes (the buffer is padded for the last
// one); their products are discarded.
template <class L>
struct LdsPlanes {
    const float* lo;
    const float* hi;
    __device__ __forceinline__ LdsPlanes(const float* planes, const Lane& z) {
        const int j0 = z.r0 * L::NP + z.col;
        lo = planes + j0;
        hi = planes + L::n + j0;
    }
    __device__ __forceinline__ float at(const Lane& z, int i, int k) const {
        int p, d;
        switch (k) {
            case 0: p = 4; d = -L::NP - 1; break;    // SW = NE of j-NP-1
            case 1: p = 3; d = -L::NP; break;        // S  = N  of j-NP
            case 2: p = 2; d = -L::NP + 1; break;    // SE = NW of j-NP+1
            case 3: p = 1; d = -1; break;            // W  = E  of j-1
            default: p = k - 4; d = 0; break;        // own C, E, NW, N, NE
        }
        const float v = p < 2 ? lo[p * L::n + i * L::NP + d] : hi[(p - 1) * L::n + i * L::NP + d];
        return sym_mask<L>(z, i, k, v);
    }
    static_assert((3 * L::n + L::R * L::NP) * 4 < 65536, "offsets fit the instruction");
};

// Asynchronous copy of one instance's symmetric FP32 planes (kSym * n floats
// at src, global) into LDS, issued by the waves of the instance (lt: lane
// within the instance), without passing through registers.  Each instruction
// moves 16 bytes per lane, 1 KiB per wave, from a 16-byte aligned address:
// the copy starts `shift` = (src / 4) mod 4 floats before src, so element e
// of the block lands at region + shift + e (region: 16-byte aligned, L::PS
// floats).  It ends at most 3 floats past the block (inside the planes'
// zeroed pad after the last instance).
template <class L>
__device__ __forceinline__ void planes_copy_start(const float* src, float* region, int lt, int shift) {
    using gptr = __attribute__((address_space(1))) void*;
    using lptr = __attribute__((address_space(3))) void*;
    constexpr int chunk = kWave * 4;
    const float* g = src - shift;
    const int total = shift + kSym * L::n;
    const int lane = lt & (kWave - 1);
    for (int c = lt / kWave; c * chunk < total; c += L::WPI) {
        const int e = c * chunk + 4 * lane;
        if (e < total) __builtin_amdgcn_global_load_lds((gptr)(g + e), (lptr)(region + c * chunk), 16, 0, 0);
    }
}

// Every wave waits for its own copies, then for the others'.
__device__ __forceinline__ void planes_copy_wait() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

// Asynchronous copy of pack `task`'s metadata into LDS (kMetaWords words at
// dst), one instruction of the first wave: lane l copies word l.  pack_level
// may be null (one mesh size); unused words repeat the count.
__device__ __forceinline__ void meta_copy_start(const PackList& P, const int32_t* pack_level, int task,
                                                int32_t* dst) {
    using gptr = __attribute__((address_space(1))) void*;
    using lptr = __attribute__((address_space(3))) void*;
    const int l = threadIdx.x & (kWave - 1);
    const int32_t* src = P.count + task;
    if (l < kMetaOff) src = P.slot_inst + task * kPackSlots + l;
    else if (l < kMetaCount) src = reinterpret_cast<const int32_t*>(P.slot_off + task * kPackSlots) + (l - kMetaOff);
    else if (l == kMetaLevel && pack_level != nullptr) src = pack_level + task;
    __builtin_amdgcn_global_load_lds((gptr)src, (lptr)dst, 4, 0, 0);
}

// Stencil sources.  A source gives, for row i of the lane's strip and
// coefficient k, a raw value (load) and the coefficient (value):
//   RegStencil     stencil resident in registers (FP32, or FP64)
//   SymStencil     symmetric planes in global memory, read per application
//   SplitStencil   FP64 operator as resident FP32 part + FP32 low part read
//                  from an LDS copy of its planes: S32 + Slo spans at most 48
//                  significant bits, so the FP64 sum is exact and equals S to
//                  about 2^-48 relative.
template <class L, typename TS>
struct RegStencil {
    static constexpr bool kGlobal = false;
    using raw_t = TS;
    const TS (&S)[L::R][kStencil];
    __device__ __forceinline__ TS load(const Lane&, int i, int k) const { return S[i][k]; }
    __device__ __forceinline__ TS value(int, int, TS raw) const { return raw; }
};

// FP64 stencil of the lane's rows with the two lower corner couplings (SW,
// SE) in LDS slots of the lane ([corner][row][lane]: each lane reads only
// what it wrote, so no barrier) and the other seven in registers: 12 fewer
// FP64 values held through the solve.
template <class L>
struct RegLdsStencil {
    static constexpr bool kGlobal = false;
    using raw_t = double;
    const double (&S)[L::R][kStencil];
    const double* cs;
    __device__ __forceinline__ double load(const Lane&, int i, int k) const {
        if (k == 0) return cs[i * NTP + threadIdx.x];
        if (k == 2) return cs[(L::R + i) * NTP + threadIdx.x];
        return S[i][k];
    }
    __device__ __forceinline__ double value(int, int, double raw) const { return raw; }
};

// Streamed planes are addressed with one VGPR per lane: each load is plane
// k's base (wave-uniform, SGPRs) + the byte offset of the lane's node in
// strip row 0 (VGPR) + a compile-time offset for the row and the neighbour
// (the instruction's immediate), so a whole batch of loads is in flight with
// no address registers of its own.  Strip rows past the mesh of active lanes
// read at most 2(N+1) entries past the instance's block (the planes carry
// kPlanePad zeroed entries at the end); their products are discarded.
template <class L, typename TS>
struct SymStencil {
    static constexpr bool kGlobal = true;
    using raw_t = TS;
    const TS* __restrict__ base;   // instance block: kSym planes of n
    const TS* pb[kSym] = {};       // plane bases, set by prepare()
    uint32_t vofs = 0;
    __device__ __forceinline__ SymStencil(const TS* b) : base(b) {}
    __device__ __forceinline__ void prepare(const Lane& z) {
#pragma unroll
        for (int p = 0; p < kSym; ++p) pb[p] = opaque(base + p * L::n);
        // lanes past the last strip address from the block's start instead
        // (their strip would lie up to 2 strips past the mesh; what they
        // load is discarded)
        vofs = z.act ? (uint32_t)((z.r0 * L::NP + z.col) * (int)sizeof(TS)) : 0u;
    }
    __device__ __forceinline__ TS load(const Lane& z, int i, int k) const {
        int p, d;
        switch (k) {
            case 0: p = 4; d = -L::NP - 1; break;    // SW = NE of j-NP-1
            case 1: p = 3; d = -L::NP; break;        // S  = N  of j-NP
            case 2: p = 2; d = -L::NP + 1; break;    // SE = NW of j-NP+1
            case 3: p = 1; d = -1; break;            // W  = E  of j-1
            default: p = k - 4; d = 0; break;        // own C, E, NW, N, NE
        }
        using gchar = const __attribute__((address_space(1))) char;
        using gT = const __attribute__((address_space(1))) TS;
        const TS v = *reinterpret_cast<gT*>((gchar*)pb[p] + vofs + (i * L::NP + d) * (int)sizeof(TS));
        return sym_mask<L>(z, i, k, v);
    }
    __device__ __forceinline__ TS value(int, int, TS raw) const { return raw; }
};

template <class L>
struct SplitStencil {
    static constexpr bool kGlobal = false;
    using raw_t = float;
    const float (&S)[L::R][kStencil];
    LdsPlanes<L> planes;              // low parts, symmetric planes, copied to LDS
    __device__ __forceinline__ float load(const Lane& z, int i, int k) const { return planes.at(z, i, k); }
    __device__ __forceinline__ double value(int i, int k, float raw) const { return (double)S[i][k] + (double)raw; }
};

// The low parts alone (the LDS planes of SplitStencil), applied in FP64.
template <class L>
struct LowStencil {
    static constexpr bool kGlobal = false;
    using raw_t = float;
    LdsPlanes<L> planes;
    __device__ __forceinline__ float load(const Lane& z, int i, int k) const { return planes.at(z, i, k); }
    __device__ __forceinline__ double value(int, int, float raw) const { return (double)raw; }
};

// y_i = sum_k S_ik g(row r0+i + dr, col + dc) in k order 0..8, one product
// at a time; own-column values come from mine[].  Streamed coefficients are
// loaded B rows at a time, all loads of a batch in flight before the first
// use (scheduling barriers keep the batches apart without draining memory);
// coefficient 1 (S) of row i > 0 is coefficient 7 (N) of row i-1, already
// loaded.  Rows past the mesh give 0.  Active lanes only.
template <class L, int B, typename TA, typename TG, class ST>
__device__ __forceinline__ void strip_apply(const ST& S0, const TG* g, const Lane& z,
                                            const TG (&mine)[L::R], TA (&y)[L::R]) {
    ST S = S0;
    if constexpr (ST::kGlobal) S.prepare(z);
    constexpr int W2 = L::W2;
    const int base = (z.r0 + 1) * W2 + (z.col + 1);
    TG lf[L::R + 2], rt[L::R + 2];
#pragma unroll
    for (int i = 0; i < L::R + 2; ++i) {
        lf[i] = g[base + (i - 1) * W2 - 1];
        rt[i] = g[base + (i - 1) * W2 + 1];
    }
    const TG up = g[base - W2];
    const TG dn = g[base + L::R * W2];
    typename ST::raw_t carry7 = typename ST::raw_t(0);
#pragma unroll
    for (int i0 = 0; i0 < L::R; i0 += B) {
        typename ST::raw_t c[B][kStencil];
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int k = 0; k < kStencil; ++k) {
                if (i0 + b >= L::R) continue;
                if (k == 1 && i0 + b > 0) c[b][1] = (b > 0) ? c[b - 1][7] : carry7;
                else c[b][k] = S.load(z, i0 + b, k);
            }
        if constexpr (ST::kGlobal) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            if (i >= L::R) break;
            const TG cm = (i == 0) ? up : mine[i - 1];
            const TG cp = (i == L::R - 1) ? dn : mine[i + 1];
            TA t = TA(S.value(i, 0, c[b][0])) * TA(lf[i]);
            t += TA(S.value(i, 1, c[b][1])) * TA(cm);
            t += TA(S.value(i, 2, c[b][2])) * TA(rt[i]);
            t += TA(S.value(i, 3, c[b][3])) * TA(lf[i + 1]);
            t += TA(S.value(i, 4, c[b][4])) * TA(mine[i]);
            t += TA(S.value(i, 5, c[b][5])) * TA(rt[i + 1]);
            t += TA(S.value(i, 6, c[b][6])) * TA(lf[i + 2]);
            t += TA(S.value(i, 7, c[b][7])) * TA(cp);
            t += TA(S.value(i, 8, c[b][8])) * TA(rt[i + 2]);
            y[i] = (z.r0 + i < L::NP) ? t : TA(0);
            carry7 = c[b][7];
        }
        if constexpr (ST::kGlobal) __builtin_amdgcn_sched_barrier(0);
    }
}

// As strip_apply, but the neighbour columns are read from LDS row by row (six
// reads per row instead of 2R+4 values held through the whole apply), which
// leaves registers for a larger batch of streamed coefficients: fewer
// dependent memory round trips in the start and residual phases.
template <class L, int B, typename TA, typename TG, class ST>
__device__ __forceinline__ void strip_apply_lean(const ST& S0, const TG* g, const Lane& z,
                                                 const TG (&mine)[L::R], TA (&y)[L::R]) {
    ST S = S0;
    if constexpr (ST::kGlobal) S.prepare(z);
    constexpr int W2 = L::W2;
    const int base = (z.r0 + 1) * W2 + (z.col + 1);
    typename ST::raw_t carry7 = typename ST::raw_t(0);
#pragma unroll
    for (int i0 = 0; i0 < L::R; i0 += B) {
        typename ST::raw_t c[B][kStencil];
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int k = 0; k < kStencil; ++k) {
                if (i0 + b >= L::R) continue;
                if (k == 1 && i0 + b > 0) c[b][1] = (b > 0) ? c[b - 1][7] : carry7;
                else c[b][k] = S.load(z, i0 + b, k);
            }
        if constexpr (ST::kGlobal) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            if (i >= L::R) break;
            const int rb = base + (i - 1) * W2;
            const TG l0 = g[rb - 1], l1 = g[rb + W2 - 1], l2 = g[rb + 2 * W2 - 1];
            const TG q0 = g[rb + 1], q1 = g[rb + W2 + 1], q2 = g[rb + 2 * W2 + 1];
            const TG cm = (i == 0) ? g[base - W2] : mine[i - 1];
            const TG cp = (i == L::R - 1) ? g[base + L::R * W2] : mine[i + 1];
            TA t = TA(S.value(i, 0, c[b][0])) * TA(l0);
            t += TA(S.value(i, 1, c[b][1])) * TA(cm);
            t += TA(S.value(i, 2, c[b][2])) * TA(q0);
            t += TA(S.value(i, 3, c[b][3])) * TA(l1);
            t += TA(S.value(i, 4, c[b][4])) * TA(mine[i]);
            t += TA(S.value(i, 5, c[b][5])) * TA(q1);
            t += TA(S.value(i, 6, c[b][6])) * TA(l2);
            t += TA(S.value(i, 7, c[b][7])) * TA(cp);
            t += TA(S.value(i, 8, c[b][8])) * TA(q2);
            y[i] = (z.r0 + i < L::NP) ? t : TA(0);
            carry7 = c[b][7];
        }
        if constexpr (ST::kGlobal) __builtin_amdgcn_sched_barrier(0);
    }
}

// x to X_out and the per-instance results.  b^T x (the flux) only when
// A.bx_out is set: the step leaves it to a boundary-only pass after the
// launch (b vanishes in the interior), which spares the b loads and a
// reduction at the end of every solve.
template <class L>
__device__ __forceinline__ void pack_store(const MicroArgs& A, const Lane& z, const double (&x)[L::R],
                                           int iters, int sweeps, bool conv, double rr, PackRed<1, double>& red1) {
    // an instance that missed rtol goes to the FP64 recovery (when there is
    // one) with X0 untouched; conv is uniform over the instance's lanes
    const bool hand_off = !conv && A.fb_list != nullptr;
    if (!hand_off) {
#pragma unroll
        for (int i = 0; i < L::R; ++i)
            if (row_ok<L>(z, i)) A.X_out[z.off + node_of<L>(z, i)] = x[i];
    }
    double bx[1] = {0.0};
    if (A.bx_out != nullptr) {
#pragma unroll
        for (int i = 0; i < L::R; ++i)
            if (row_ok<L>(z, i)) bx[0] += A.b[z.off + node_of<L>(z, i)] * x[i];
        red1.sum<L>(bx, z.w0);
    }
    if (z.live && z.lt == 0) {
        if (A.bx_out != nullptr) A.bx_out[z.inst] = bx[0];
        if (A.iters_out) A.iters_out[z.inst] = iters;
        if (A.sweeps_out) A.sweeps_out[z.inst] = sweeps;
        if (A.res_out) A.res_out[z.inst] = sqrt(rr);
        if (hand_off) A.fb_list[1 + atomicAdd(A.fb_list, 1)] = z.inst;
        else if (!conv) atomicAdd(A.nonconv, 1);
    }
}

// Steps of history of the extrapolated start for this solve (-1: none; the
// time-step form with a history only).
__device__ __forceinline__ int history_steps(const MicroArgs& A) {
    return (A.rhs_vec == nullptr && A.Mw != nullptr && !A.zero_init && A.hx != nullptr) ? *A.hn : -1;
}

// Issue the loads of the history of the lane's rows (hx; he with two steps;
// he2 with three), all in one block: rows past the mesh read node 0
// (discarded).
template <class L>
__device__ __forceinline__ void history_load(const MicroArgs& A, const Lane& z, int hn, float (&lh)[L::R],
                                             float (&le)[L::R], float (&le2)[L::R]) {
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        lh[i] = 0.0f;
        le[i] = 0.0f;
        le2[i] = 0.0f;
    }
    if (hn >= 1) {
#pragma unroll
        for (int i = 0; i < L::R; ++i) lh[i] = A.hx[z.off + (row_ok<L>(z, i) ? node_of<L>(z, i) : 0)];
    }
    if (hn >= 2) {
#pragma unroll
        for (int i = 0; i < L::R; ++i) le[i] = A.he[z.off + (row_ok<L>(z, i) ? node_of<L>(z, i) : 0)];
    }
    if (hn >= 3) {
#pragma unroll
        for (int i = 0; i < L::R; ++i) le2[i] = A.he2[z.off + (row_ok<L>(z, i) ? node_of<L>(z, i) : 0)];
    }
}

// From the loaded history and the current X0 (xc): the predicted increment
// of the lane's rows into g -- 3 e1 - 3 e2 + e3 with three steps of history
// (the increments extrapolated quadratically), 2 e1 - e2 with two, e1 with
// one, 0 with none (e1 = X0 - hx, where hx is X0 rounded to FP32, ~2^-24
// |X0| absolute, far below the increment) -- then the history moves on
// (hx = X0, he = e1, he2 = the previous he).  The caller has waited for the
// loads (vmcnt), so no store overtakes a load of its address.
template <class L, typename TG>
__device__ __forceinline__ void history_step(const MicroArgs& A, const Lane& z, int hn, const double (&xc)[L::R],
                                             const float (&lh)[L::R], const float (&le)[L::R],
                                             const float (&le2)[L::R], TG (&g)[L::R]) {
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        const float e1 = hn >= 1 ? (float)(xc[i] - (double)lh[i]) : 0.0f;
        const float pr = hn >= 3 ? 3.0f * (e1 - le[i]) + le2[i] : hn >= 2 ? 2.0f * e1 - le[i] : e1;
        g[i] = row_ok<L>(z, i) ? (TG)pr : TG(0);
        if (row_ok<L>(z, i)) {
            const int j = node_of<L>(z, i);
            A.hx[z.off + j] = (float)xc[i];
            A.he[z.off + j] = e1;
            A.he2[z.off + j] = le[i];
        }
    }
}

// Time-step solve whose start residual takes M x0 from the separable mass
// tables (MicroArgs::mass1d) instead of K x0 from the assembled planes.
__device__ __forceinline__ bool mass_free(const MicroArgs& A) {
    return A.mass1d != nullptr && A.rhs_vec == nullptr && A.Mw != nullptr && !A.zero_init;
}

// Separable mass of the analytic family.  J = det(I + a G) at the point
// (y1, y2) is 1 + a (c(y1) y2 + y1 c(y2)) + a^2 (c(y1) y1 c(y2) y2 -
// s(y1) s(y2)): five terms f_T(y1) g_T(y2), and the 2x2 Gauss rule is the
// tensor product of the 1D rule, so the J-weighted Q1 mass (Section 3.1) is
//   M = sum_T kappa_T  M1[g_T] (x) M1[f_T],   kappa = (1, a, a, a^2, -a^2),
//   (f_T, g_T) = (1, 1), (c, y), (y, c), (c y, c y), (s, s),
// with M1[f] the 1D Q1 mass weighted by f at the Gauss points (table planes
// per level; Section 3.4 caches J per quadrature point, here its factors
// per level).  The lane applies M1[f_T] of its column along the rows r0-1 ..
// r0+R (three grid reads a row), then M1[g_T] of each of its rows across
// three consecutive such rows: 35 FP64 FMAs per node.  mt: the level's
// table in LDS (mass_table_copy); x0 in the grid (zero halo); active lanes
// only; rows past the mesh give 0.
constexpr int kMassF = 5;
constexpr int kMassG[kMassF] = {0, 2, 1, 3, 4};     // g_T as a function index
// Asynchronous copy of the level's table (16 planes of N+1 doubles, the
// last one padding) into LDS at dst, 16 bytes a lane, without registers; it
// has landed once the wave has waited for its loads.
template <class L>
__device__ __forceinline__ void mass_table_copy(const MicroArgs& A, double* dst) {
    using gptr = __attribute__((address_space(1))) void*;
    using lptr = __attribute__((address_space(3))) void*;
    constexpr int pieces = 8 * L::NP;
    const double* src = A.mass1d + 8 * A.tab.off[L::N];
    const int lane = threadIdx.x & (kWave - 1), w0 = threadIdx.x - lane;
    if (w0 + lane < pieces) __builtin_amdgcn_global_load_lds((gptr)(src + 2 * (w0 + lane)), (lptr)(dst + 2 * w0), 16, 0, 0);
}

template <class L>
__device__ __forceinline__ void mass_apply(const double* mt, const Lane& z, const double* xg, double a,
                                           double (&mx)[L::R]) {
    constexpr int NP = L::NP, W2 = L::W2;
    const double a2 = a * a;
    const double kap[kMassF] = {1.0, a, a, a2, -a2};
    double fk[kMassF][3];     // kappa_T M1[f_T] of the lane's column
#pragma unroll
    for (int t = 0; t < kMassF; ++t)
#pragma unroll
        for (int d = 0; d < 3; ++d) fk[t][d] = kap[t] * mt[(3 * t + d) * NP + z.col];
    auto across = [&](int rho, double (&v)[kMassF]) {
        const int cb = (rho + 1) * W2 + z.col + 1;
        const double xl = xg[cb - 1], xm = xg[cb], xr = xg[cb + 1];
#pragma unroll
        for (int t = 0; t < kMassF; ++t) v[t] = fk[t][0] * xl + fk[t][1] * xm + fk[t][2] * xr;
    };
    double vm[kMassF], v0[kMassF], vp[kMassF];
    across(z.r0 - 1, vm);
    across(z.r0, v0);
    // one row's coefficients in flight at a time (hoisting all of them
    // would spill)
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        __builtin_amdgcn_sched_barrier(0);
        const int rho = z.r0 + i;
        across(rho + 1, vp);
        const double* gp = mt + (rho < NP ? rho : NP - 1);
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < kMassF; ++t) {
            const double* gt = gp + 3 * kMassG[t] * NP;
            s += gt[0] * vm[t] + gt[NP] * v0[t] + gt[2 * NP] * vp[t];
        }
        mx[i] = rho < NP ? s : 0.0;
#pragma unroll
        for (int t = 0; t < kMassF; ++t) {
            vm[t] = v0[t];
            v0[t] = vp[t];
        }
    }
}

// x0 into registers and the (double) grid, then the FP64 residual:
//   given right-hand side:  b = rhs_scale rhs [+ rhs_bscale c_i b_i],  r = b - S x0,
//                           and the partial ||b||^2 in bb
//   time step:              b = M x0 / dt,      r = b - S x0 = -K x0
//   time step with Mw:      the iterate starts from y0 = X0 (x0 = y0 + coef w)
//                           and r = b - S y0 = -K y0 + coef M w / dt
// (K = S - M/dt is stored on its own, so the residual carries no
// cancellation; the separable-mass start below forms b - S y0 instead, a
// difference of two terms of size ||b|| that is exact to ~1e-16 ||b||, far
// below rtol ||b||).  The time-step forms leave ||b||^2 to the caller (bb = 0),
// which forms b = S y0 + r from its register stencil (y0 stays in the
// double grid) instead of reading M.
// copy_src/copy_dst (non-null): start the asynchronous copy of the instance's
// FP32 planes into LDS (planes_copy_start) once x0 is in the grid, so that it
// overlaps the operator application; the caller waits for it
// (planes_copy_wait).
// mtab (non-null, LDS for the level's table) with mass_free: the separable
// mass; r leaves with coef M w/dt + M x0/dt, the right-hand side b itself,
// and the caller subtracts S x0.
// hslot (non-null) with hist >= 0 (history_steps of the launch): the
// history of the lane's rows is read with X0, the predicted increment goes
// to the lane's slots hslot[i * NTP + lane] (history_step; every lane writes
// all of its slots), and the history moves on after the barrier that waits
// for those loads.
template <class L>
__device__ __forceinline__ void pack_start(const MicroArgs& A, const Lane& z, double* xg, double (&x)[L::R],
                                           double (&r)[L::R], double& bb, const float* copy_src = nullptr,
                                           float* copy_dst = nullptr, int copy_shift = 0, float* hslot = nullptr,
                                           int hist = -1, double* mtab = nullptr) {
    const bool sep = mtab != nullptr && mass_free(A);
    if (sep) mass_table_copy<L>(A, mtab);
    zero_halo<L, double>(xg, z);
    const double cf = (z.live && A.coef != nullptr) ? A.coef[z.inst] : 0.0;
    // the amplitude of the separable mass, loaded with the rows (no load
    // can pass the barrier that follows them)
    const double am = (sep && z.live) ? A.amp[z.inst] : 0.0;
    // time step with M w: start from X0 alone; the right-hand side keeps
    // coef w through cm[i] = coef (M w)_j / dt
    const bool use_mw = A.rhs_vec == nullptr && A.Mw != nullptr && !A.zero_init;
    const int hn = hslot != nullptr ? hist : -1;
    double cm[L::R];
    float lh[L::R], le[L::R], le2[L::R];
    // the rows' loads: no arithmetic and no uniform branch inside a row's
    // branch, so that every row's loads are in flight before the first wait
    // (M w, or w, in wv)
    double wv[L::R];
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        x[i] = 0.0;
        wv[i] = 0.0;
        lh[i] = 0.0f;
        le[i] = 0.0f;
        le2[i] = 0.0f;
    }
    if (!A.zero_init) {
        const double* ws = use_mw ? A.Mw : A.w;
#pragma unroll
        for (int i = 0; i < L::R; ++i)
            if (row_ok<L>(z, i)) {
                x[i] = A.X0[z.off + node_of<L>(z, i)];
                wv[i] = ws[z.off + node_of<L>(z, i)];
            }
        if (hn >= 1) {
#pragma unroll
            for (int i = 0; i < L::R; ++i)
                if (row_ok<L>(z, i)) lh[i] = A.hx[z.off + node_of<L>(z, i)];
        }
        if (hn >= 2) {
#pragma unroll
            for (int i = 0; i < L::R; ++i)
                if (row_ok<L>(z, i)) le[i] = A.he[z.off + node_of<L>(z, i)];
        }
        if (hn >= 3) {
#pragma unroll
            for (int i = 0; i < L::R; ++i)
                if (row_ok<L>(z, i)) le2[i] = A.he2[z.off + node_of<L>(z, i)];
        }
    }
    const double cmf = use_mw ? cf * A.inv_dt : 0.0, cw = use_mw ? 0.0 : cf;
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        cm[i] = cmf * wv[i];
        x[i] += cw * wv[i];
    }
    strip_store<L>(xg, z, x);
    // (the mass table copy has landed in every wave past this barrier)
    if (sep) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (hn >= 0) {
        float g[L::R];
        history_step<L>(A, z, hn, x, lh, le, le2, g);
#pragma unroll
        for (int i = 0; i < L::R; ++i) hslot[i * NTP + threadIdx.x] = g[i];
    }
    if (copy_src != nullptr && z.live) planes_copy_start<L>(copy_src, copy_dst, z.lt, copy_shift);
    double b[L::R], sx[L::R];
#pragma unroll
    for (int i = 0; i < L::R; ++i) { b[i] = 0.0; sx[i] = 0.0; }
    bb = 0.0;
    if (A.rhs_vec != nullptr) {
#pragma unroll
        for (int i = 0; i < L::R; ++i)
            b[i] = row_ok<L>(z, i) ? A.rhs_scale * A.rhs_vec[z.off + node_of<L>(z, i)] : 0.0;
        if (A.rhs_bcoef != nullptr) {
            const double bc = z.live ? A.rhs_bscale * A.rhs_bcoef[z.inst] : 0.0;
#pragma unroll
            for (int i = 0; i < L::R; ++i)
                if (row_ok<L>(z, i)) b[i] += bc * A.b[z.off + node_of<L>(z, i)];
        }
        if (z.act) strip_apply_lean<L, L::R>(SymStencil<L, double>{A.Ss64 + kSym * z.off}, xg, z, x, sx);
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            r[i] = b[i] - sx[i];
            bb += b[i] * b[i];
        }
    } else if (sep) {
        if (z.act) mass_apply<L>(mtab, z, xg, am, sx);
#pragma unroll
        for (int i = 0; i < L::R; ++i) r[i] = cm[i] + A.inv_dt * sx[i];
    } else {
        if (z.act) strip_apply_lean<L, L::R>(SymStencil<L, double>{A.Ks64 + kSym * z.off}, xg, z, x, sx);
#pragma unroll
        for (int i = 0; i < L::R; ++i) r[i] = cm[i] - sx[i];
    }
}


// ------------------------------------------------------------ matrix-free
// The time-step operator S = M/dt + d A + kappa B of a pack's instances,
// evaluated at the start of every solve from the amplitude a_i and the
// level's quadrature tables instead of read from assembled planes (paper
// Section 3.1: J and K K^T J at every quadrature point, |cof(F) nu| on the
// boundary; Section 3.4 caches them per point, here they are recomputed).
//
// Lane (col c, strip rows r0..r0+R-1) integrates the cells (c, r) for
// r = r0-1 .. r0+R-1 -- the cells to the right of and above its nodes; the
// first one is also integrated by the strip below -- into element matrices
// (2x2 Gauss), and the Robin edge terms of boundary cells.  A node's 9-point
// row takes the entries of its four cells: the two to its right are the
// lane's own, the two to its left belong to lane c-1, which passes six FP64
// values one lane to the right per node row (a DPP wave shift; the first
// lane of a wave takes them from LDS, written by the last lane of the wave
// before): the centre and north parts of its cells, the north-west
// coupling, its cells' part of K x0, its own east coupling (the receiver's
// west) and its previous row's north-east coupling (the receiver's
// south-west).  South and south-east come from the lane's own previous row.
// So every coupling is one FP64 value whichever of its two nodes uses it,
// and the FP32 stencil fl32(S) -- in registers -- is exactly symmetric; the
// low parts fl32(S - fl32(S)) of the upper couplings go to the LDS planes
// for the FP64 residual updates; the start residual r = -K x0 + coef M w/dt
// stays in FP64.

// Boundary weights of every instance of a pack (kappa wb |F tau| at the 8N
// edge points) and the level's tables, in LDS.
constexpr int kMfBw = cmax(cmax(L16::IPP * 8 * 16, L32::IPP * 8 * 32), L64::IPP * 8 * 64);
constexpr int kMfX = 6;      // FP64 values passed to the right per node row
struct MfShared {
    double ty[2 * kMaxLevel + 2], ts[2 * kMaxLevel + 2], tc[2 * kMaxLevel + 2];
    double bw[kMfBw];
    double xb[2][NWP][kMfX];
};

// Lane l takes lane l-1's value (DPP wave_shr:1); lane 0 of the wave takes 0.
__device__ __forceinline__ double lane_from_left(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Each lane receives the kMfX values of the lane on its left; lanes of
// column 0 (nothing to their left) and inactive lanes receive 0.  One LDS
// barrier (the last lane of every wave hands its values over through LDS,
// double-buffered by par).  All lanes must call.
template <class L>
__device__ __forceinline__ void mf_pass_right(const Lane& z, double (*xb)[NWP][kMfX], int par,
                                              const double (&snd)[kMfX], double (&rcv)[kMfX]) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < kMfX; ++q) rcv[q] = lane_from_left(snd[q]);
    if (lane == kWave - 1) {
#pragma unroll
        for (int q = 0; q < kMfX; ++q) xb[par][wid][q] = snd[q];
    }
    lds_barrier();
    if (lane == 0) {
        const int src = wid > 0 ? wid - 1 : 0;
#pragma unroll
        for (int q = 0; q < kMfX; ++q) rcv[q] = xb[par][src][q];
    }
    const bool none = !z.act || z.col == 0;
#pragma unroll
    for (int q = 0; q < kMfX; ++q) rcv[q] = none ? 0.0 : rcv[q];
}

// Element matrices of one cell (2x2 Gauss) from the geometry at its points:
// M = I + a G with M11 = 1 + a c(y1) y2, M12 = a s(y1), M21 = a s(y2),
// M22 = 1 + a c(y2) y1 (A1 = a c(y1), S1 = a s(y1), likewise A2, S2 per
// abscissa of the cell); J = det M, C = adj(M) adj(M)^T / J.  Entries in
// the order (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3) of
// the local nodes q = l2*2 + l1:
//   K_lm = d sum_g wq grad eta_l . C grad eta_m   (wq / h^2 = 1/4)
//   S_lm = K_lm + (1/dt) sum_g wq J eta_l eta_m
// The stiffness entries come from the moments of C11 along y2, C22 along
// y1 and C12 against one basis factor in each direction; the mass entries
// from the moments of J.
constexpr int kPairL[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
constexpr int kPairM[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
__device__ __forceinline__ void mf_cell(double d4, double wq_dt, const double (&y1)[2], const double (&A1)[2],
                                        const double (&S1)[2], const double (&y2)[2], const double (&A2)[2],
                                        const double (&S2)[2], double (&K)[10], double (&S)[10]) {
    double q11[3] = {0.0, 0.0, 0.0}, q22[3] = {0.0, 0.0, 0.0};
    double q12[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    double mm[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
    for (int g2 = 0; g2 < 2; ++g2)
#pragma unroll
        for (int g1 = 0; g1 < 2; ++g1) {
            const double M11 = fma(A1[g1], y2[g2], 1.0);
            const double M22 = fma(A2[g2], y1[g1], 1.0);
            const double M12 = S1[g1], M21 = S2[g2];
            const double J = M11 * M22 - M12 * M21;
            // d/(4J): reciprocal estimate refined by two Newton steps
            // x <- x + x (1 - J x) (J > 0: the setup checked det D zeta)
            double iJ = __builtin_amdgcn_rcp(J);
            iJ = fma(iJ, fma(-J, iJ, 1.0), iJ);
            iJ = fma(iJ, fma(-J, iJ, 1.0), iJ);
            const double s = d4 * iJ;
            const double C11 = (M22 * M22 + M12 * M12) * s;
            const double C12 = -(M22 * M21 + M12 * M11) * s;
            const double C22 = (M21 * M21 + M11 * M11) * s;
            const double f1[2] = {lin(0, g1), lin(1, g1)};
            const double f2[2] = {lin(0, g2), lin(1, g2)};
            const double F1[3] = {f1[0] * f1[0], f1[0] * f1[1], f1[1] * f1[1]};
            const double F2[3] = {f2[0] * f2[0], f2[0] * f2[1], f2[1] * f2[1]};
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                q11[p] = fma(C11, F2[p], q11[p]);
                q22[p] = fma(C22, F1[p], q22[p]);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) q12[u][v] = fma(C12, f2[u] * f1[v], q12[u][v]);
#pragma unroll
            for (int p1 = 0; p1 < 3; ++p1)
#pragma unroll
                for (int p2 = 0; p2 < 3; ++p2) mm[p1][p2] = fma(J, F1[p1] * F2[p2], mm[p1][p2]);
        }
#pragma unroll
    for (int e = 0; e < 10; ++e) {
        const int l1 = kPairL[e] & 1, l2 = kPairL[e] >> 1, m1 = kPairM[e] & 1, m2 = kPairM[e] >> 1;
        const double s11 = (l1 == m1) ? 1.0 : -1.0;     // sigma(l1) sigma(m1)
        const double s12 = (l1 == m2) ? 1.0 : -1.0;     // sigma(l1) sigma(m2)
        const double s21 = (l2 == m1) ? 1.0 : -1.0;     // sigma(l2) sigma(m1)
        const double s22 = (l2 == m2) ? 1.0 : -1.0;     // sigma(l2) sigma(m2)
        const double a = s11 * q11[l2 + m2] + s12 * q12[l2][m1] + s21 * q12[m2][l1] + s22 * q22[l1 + m1];
        K[e] = a;
        S[e] = fma(mm[l1 + m1][l2 + m2], wq_dt, a);
    }
}

// Matrix-free start of a time-step solve in the refinement form: x0 to the
// (double) grid, the FP32 stencil of the lane's rows to S, the FP32 low
// parts of their upper couplings to the LDS planes slo ([kSym][n]),
// r = -K x0 + coef M w/dt to r64.  The caller reads x0 back from the grid.
// All lanes must call.
template <class L>
__device__ __forceinline__ void mf_start(const MicroArgs& A, const Lane& z, double* xg, MfShared& ms, float* slo,
                                         float (&S)[L::R][kStencil], double (&r64)[L::R]) {
    constexpr int N = L::N, W2 = L::W2;
    constexpr double h = 2.0 / N;
    constexpr double wq = 0.25 * h * h, wb = 0.5 * h;
    zero_halo<L, double>(xg, z);
    const double cf = (z.live && A.coef != nullptr) ? A.coef[z.inst] : 0.0;
    const double a = z.live ? A.amp[z.inst] : 0.0;
    {
        double x[L::R];
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            double v = 0.0, m = 0.0;
            if (row_ok<L>(z, i)) {
                const int j = node_of<L>(z, i);
                v = A.X0[z.off + j];
                m = cf * A.inv_dt * A.Mw[z.off + j];
            }
            x[i] = v;
            r64[i] = m;
        }
        strip_store<L>(xg, z, x);
    }
    // the level's tables, and kappa wb |F tau| at the boundary points of
    // every instance of the pack (sides bottom, top, left, right; edges; 2
    // points): bottom/top edges run along y1, |M e1| = sqrt(M11^2 + M21^2);
    // left/right edges along y2, |M e2| = sqrt(M12^2 + M22^2)
    const int tb = A.tab.off[N];
    for (int t = threadIdx.x; t < 2 * N + 2; t += NTP) {
        ms.ty[t] = A.tab.y[tb + t];
        ms.ts[t] = A.tab.s[tb + t];
        ms.tc[t] = A.tab.c[tb + t];
    }
    if (z.live) {
        for (int t = z.lt; t < 8 * N; t += L::TPI) {
            const int side = t / (2 * N), e = (t >> 1) % N, g = t & 1;
            const int tf = tb + 2 * N + (side & 1);        // the edge's coordinate: -1 or +1
            const int tg = tb + 2 * e + g;                 // the Gauss point along the edge
            const double yf = A.tab.y[tf], sf = A.tab.s[tf];
            const double along = fma(a * A.tab.c[tg], yf, 1.0);   // M11 (bottom/top) or M22 (left/right)
            const double across = a * sf;                          // M21 or M12
            ms.bw[z.sub * 8 * N + t] = A.kappa * wb * sqrt(along * along + across * across);
        }
    }
    __syncthreads();
    const double* bw = ms.bw + (z.sub < L::IPP ? z.sub : 0) * 8 * N;
    const int c = z.col;
    const bool colc = z.act && c < N;
    const int t1 = 2 * (c < N ? c : 0);

    // carries from the previous cell row: its entries (2,2) (2,3) (3,3) of S,
    // its K x0 parts for the row above, its north-east and north-west
    // couplings, and the previous node row's complete north coupling
    double cS22 = 0.0, cS23 = 0.0, cS33 = 0.0, ck2 = 0.0, ck3 = 0.0, cNE = 0.0, cN = 0.0, cNW = 0.0;
    // one node row at a time (not unrolled: the cell arithmetic of several
    // rows in flight would not fit the registers)
#pragma unroll 1
    for (int k = -1; k < L::R; ++k) {
        const int r = z.r0 + k;
        const bool valid = colc && r >= 0 && r < N;
        const int t2 = 2 * (valid ? r : 0);
        double y2[2], A2[2], S2[2], y1[2], A1[2], S1[2];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            y1[g] = ms.ty[t1 + g];
            A1[g] = a * ms.tc[t1 + g];
            S1[g] = a * ms.ts[t1 + g];
            y2[g] = ms.ty[t2 + g];
            A2[g] = a * ms.tc[t2 + g];
            S2[g] = a * ms.ts[t2 + g];
        }
        // a cell outside the mesh gets zero weights (its geometry, from the
        // first table entries, is finite)
        const double on = valid ? 1.0 : 0.0;
        double Ke[10], Se[10];
        mf_cell(on * 0.25 * A.d, on * wq * A.inv_dt, y1, A1, S1, y2, A2, S2, Ke, Se);
        // Robin terms of the cell's boundary edges: entries of the edge's two
        // nodes, sum over its points of kappa wb |F tau| eta_l eta_m
        auto edge = [&](const double* w, int ea, int eb, int ec) {
            const double w0 = w[0], w1 = w[1];
            const double va = w0 * (lin(0, 0) * lin(0, 0)) + w1 * (lin(0, 1) * lin(0, 1));
            const double vb = w0 * (lin(0, 0) * lin(1, 0)) + w1 * (lin(0, 1) * lin(1, 1));
            const double vc = w0 * (lin(1, 0) * lin(1, 0)) + w1 * (lin(1, 1) * lin(1, 1));
            Ke[ea] += va; Se[ea] += va;
            Ke[eb] += vb; Se[eb] += vb;
            Ke[ec] += vc; Se[ec] += vc;
        };
        if (valid && r == 0) edge(bw + (0 * N + c) * 2, 0, 1, 4);          // bottom: nodes 0, 1
        if (valid && r == N - 1) edge(bw + (1 * N + c) * 2, 7, 8, 9);      // top: nodes 2, 3
        if (valid && c == 0) edge(bw + (2 * N + r) * 2, 0, 2, 7);          // left: nodes 0, 2
        if (valid && c == N - 1) edge(bw + (3 * N + r) * 2, 4, 6, 9);      // right: nodes 1, 3
        // K x0 on the cell's corners (c, r), (c+1, r), (c, r+1), (c+1, r+1)
        // (lanes without a cell read the grid's first cells: zero entries)
        const int gb = valid ? (r + 1) * W2 + c + 1 : 0;
        const double x0 = xg[gb], x1 = xg[gb + 1], x2 = xg[gb + W2], x3 = xg[gb + W2 + 1];
        const double k0 = Ke[0] * x0 + Ke[1] * x1 + Ke[2] * x2 + Ke[3] * x3;    // to (c, r)
        const double k1 = Ke[1] * x0 + Ke[4] * x1 + Ke[5] * x2 + Ke[6] * x3;    // to (c+1, r)
        const double k2 = Ke[2] * x0 + Ke[5] * x1 + Ke[7] * x2 + Ke[8] * x3;    // to (c, r+1)
        const double k3 = Ke[3] * x0 + Ke[6] * x1 + Ke[8] * x2 + Ke[9] * x3;    // to (c+1, r+1)
        // node row k: the lane's own parts, and what it passes to lane c+1
        const double Eown = Se[1] + cS23;
        double snd[kMfX] = {Se[4] + cS33,   // centre part of (c+1, r) from the cells (c, r), (c, r-1)
                            Se[6],          // north part of (c+1, r)
                            Se[5],          // north-west coupling of (c+1, r)
                            k1 + ck3,       // K x0 part of (c+1, r)
                            Eown,           // west coupling of (c+1, r) = east of (c, r)
                            cNE};           // south-west of (c+1, r) = north-east of (c, r-1)
        double rcv[kMfX];
        mf_pass_right<L>(z, ms.xb, (k + 1) & 1, snd, rcv);
        const double Nc = Se[2] + rcv[1];
        if (k >= 0) {
            // the 9-point row of node row k (k = (dj2+1)*3 + (dj1+1))
            const double cpl[kStencil] = {rcv[5], cN, cNW, rcv[4], Se[0] + cS22 + rcv[0], Eown, rcv[2], Nc, Se[3]};
            const double kx = (k0 + ck2) + rcv[3];
            const bool ok = row_ok<L>(z, k);
            const int j = node_of<L>(z, k);
            // row k of the register arrays (static indices keep them in registers)
#pragma unroll
            for (int i = 0; i < L::R; ++i)
                if (i == k) {
                    r64[i] -= kx;
#pragma unroll
                    for (int q = 0; q < kStencil; ++q) S[i][q] = (float)cpl[q];
                }
#pragma unroll
            for (int p = 0; p < kSym; ++p) {
                const double v = cpl[4 + p];
                if (ok) slo[p * L::n + j] = (float)(v - (double)(float)v);
            }
        }
        cS22 = Se[7];
        cS23 = Se[8];
        cS33 = Se[9];
        ck2 = k2;
        ck3 = k3;
        cNE = Se[3];
        cN = Nc;
        cNW = Se[5];
    }
    lds_barrier();
}

// ------------------------------------------------------------------ FP64
// meta: this pack's metadata in LDS; prefetch(): starts the copy of the next
// pack's metadata (all waves call it once, early in the solve).
// xs: LDS for the iterate, kFp64Rows slots per lane ([row][lane]): x is only
// read and written once per iteration, so it waits there instead of holding
// registers that the resident stencil needs.
template <class L, bool CS = false, class Prefetch>
__device__ void pack_fp64(const MicroArgs& A, const int32_t* meta, int cnt, double* lds, double* xs,
                          PackRed<1, double>& red1, PackRed<2, double>& red2, PackRed<3, double>& red3,
                          Prefetch prefetch, double* cs = nullptr, int hist = -1, double* mtab = nullptr) {
    const Lane z = lane_of<L>(meta, cnt);
    double* xg = lds + (z.sub < L::IPP ? z.sub : 0) * L::GRID;
    double x[L::R], r[L::R], p[L::R];
    float dinv[L::R];
    double bb;
    pack_start<L>(A, z, xg, x, r, bb, nullptr, nullptr, 0, nullptr, -1, mtab);
    prefetch();
#pragma unroll
    for (int i = 0; i < L::R; ++i) xs[i * NTP + threadIdx.x] = x[i];
    // the FP64 stencil of the lane's rows, resident for the solve: in
    // registers, or (cs given) its corner couplings in LDS
    double Sr[L::R][kStencil];
    {
        SymStencil<L, double> Sg{A.Ss64 + kSym * z.off};
        Sg.prepare(z);
#pragma unroll
        for (int i = 0; i < L::R; ++i)
#pragma unroll
            for (int k = 0; k < kStencil; ++k) {
                if (CS && (k == 0 || k == 2)) cs[((k >> 1) * L::R + i) * NTP + threadIdx.x] = Sg.load(z, i, k);
                else Sr[i][k] = (k == 1 && i > 0) ? Sr[i - 1][7] : Sg.load(z, i, k);
            }
    }
    const RegStencil<L, double> S{Sr};
    const RegLdsStencil<L> SL{Sr, cs};
    if (A.rhs_vec == nullptr) {
        // ||b|| of the time step from b = S x0 + r with the resident stencil
        // (x0 is still in the grid): no pass over M
        double sb[L::R];
#pragma unroll
        for (int i = 0; i < L::R; ++i) sb[i] = 0.0;
        if (z.act) {
            if constexpr (CS) strip_apply_lean<L, 1>(SL, xg, z, x, sb);
            else strip_apply_lean<L, 1>(S, xg, z, x, sb);
        }
        // (separable mass: r holds b, and r = b - S x0 from here on)
        const bool mfree = mtab != nullptr && mass_free(A);
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            const double bi = mfree ? r[i] : sb[i] + r[i];
            if (mfree) r[i] -= sb[i];
            bb += row_ok<L>(z, i) ? bi * bi : 0.0;
        }
    }
    // Extrapolated start (time-step form with a history): x0 = X0 + the
    // predicted increment (3 e1 - 3 e2 + e3, 2 e1 - e2 or e1), r -= S (that increment) with
    // the resident FP64 stencil, kept only where it lowers ||r||.  The
    // history is read here rather than with X0 (the LDS has no room to hold
    // the prediction until the stencil is resident) and moves on once its
    // loads have returned.
    const int hn = hist;
    if (hn >= 0) {
        float lh[L::R], le[L::R], le2[L::R];
        history_load<L>(A, z, hn, lh, le, le2);
        double xc[L::R], g[L::R];
#pragma unroll
        for (int i = 0; i < L::R; ++i) xc[i] = xs[i * NTP + threadIdx.x];
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        history_step<L>(A, z, hn, xc, lh, le, le2, g);
        if (hn >= 1) {
            __syncthreads();     // the reads of x0 in the grid are done
            strip_store<L>(xg, z, g);
            __syncthreads();
            double sg[L::R];
#pragma unroll
            for (int i = 0; i < L::R; ++i) sg[i] = 0.0;
            if (z.act) {
                if constexpr (CS) strip_apply_lean<L, 1>(SL, xg, z, g, sg);
                else strip_apply_lean<L, 1>(S, xg, z, g, sg);
            }
            double a2[2] = {0.0, 0.0};     // guessed and plain ||r||^2
#pragma unroll
            for (int i = 0; i < L::R; ++i) {
                sg[i] = r[i] - sg[i];
                a2[0] += sg[i] * sg[i];
                a2[1] += r[i] * r[i];
            }
            red2.sum<L>(a2, z.w0);     // its barrier also ends the reads of the guess in the grid
            const bool keep = a2[0] < a2[1];
#pragma unroll
            for (int i = 0; i < L::R; ++i) {
                r[i] = keep ? sg[i] : r[i];
                xs[i * NTP + threadIdx.x] += keep ? g[i] : 0.0;
            }
        }
    }
    double acc[3] = {bb, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        dinv[i] = row_ok<L>(z, i) ? (float)(1.0 / Sr[i][4]) : 0.0f;
        p[i] = (double)dinv[i] * r[i];
        acc[1] += r[i] * p[i];
        acc[2] += r[i] * r[i];
    }
    red3.sum<L>(acc, z.w0);
    __shared__ double tol_s[L::IPP];
    const double tol2 = A.rtol * A.rtol * acc[0];
    if (z.live && z.lt == 0) tol_s[z.sub] = tol2;
    double rz = acc[1], rr = acc[2];
    bool conv = acc[2] <= tol2;
    int it = 0;
    __syncthreads();
    const double thr = lane_threshold<L>(tol_s, cnt);
    bool go = red3.any_above(thr);
    int k = 0;
    while (go && k < A.max_iter) {
        const bool me = !conv;
        strip_store<L>(xg, z, p);
        __syncthreads();
        double q[L::R];
#pragma unroll
        for (int i = 0; i < L::R; ++i) q[i] = 0.0;
        if (z.act) {
            if constexpr (CS) strip_apply_lean<L, 1>(SL, xg, z, p, q);
            else strip_apply_lean<L, 1>(S, xg, z, p, q);
        }
        double pq[1] = {0.0};
#pragma unroll
        for (int i = 0; i < L::R; ++i) pq[0] += p[i] * q[i];
        red1.sum<L>(pq, z.w0);
        const double alpha = me ? rz / pq[0] : 0.0;
        double a2[2] = {0.0, 0.0};     // (r, D^-1 r), (r, r)
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            xs[i * NTP + threadIdx.x] += alpha * p[i];
            r[i] -= alpha * q[i];
            a2[0] += r[i] * (double)dinv[i] * r[i];
            a2[1] += r[i] * r[i];
        }
        red2.sum<L>(a2, z.w0);
        rr = a2[1];
        ++k;
        if (me) {
            ++it;
            if (a2[1] <= tol2) {
                conv = true;
            } else {
                const double beta = a2[0] / rz;
                rz = a2[0];
#pragma unroll
                for (int i = 0; i < L::R; ++i) p[i] = (double)dinv[i] * r[i] + beta * p[i];
            }
        }
        go = red2.any_above(thr);
    }
#pragma unroll
    for (int i = 0; i < L::R; ++i) x[i] = xs[i * NTP + threadIdx.x];
    pack_store<L>(A, z, x, it, 1, conv, rr, red1);
}

// --------------------------------------------------------------- REFINE
// planes: LDS for the FP32 planes of the pack's instances (IPP * kSym * n
// floats).  It holds S32 while the register stencil is loaded, then the low
// parts Slo, copied while the first inner solve runs, for the FP64 residual
// updates.  Between the start of a copy and its wait, barriers are
// lds_barrier() (LDS ordering only) so that the copy stays in flight.
// hslot: per-lane slots of the predicted increment (extrapolated start of
// the stored-operator form; null: none); hist: history_steps of the launch.
template <class L, bool MF, class Prefetch>
__device__ void pack_refine(const MicroArgs& A, const int32_t* meta, int cnt, double* lds, float* planes,
                            MfShared* ms, PackRed<1, double>& red1, PackRed<3, double>& red3,
                            PackRed<2, float>& rf2, Prefetch prefetch, float* hslot, int hist,
                            double* mtab = nullptr) {
    const Lane z = lane_of<L>(meta, cnt);
    double* xg = lds + (z.sub < L::IPP ? z.sub : 0) * L::GRID;
    float* pg = reinterpret_cast<float*>(xg);
    // spare instances of a partial pack read instance 0's planes (results
    // discarded); pl: element 0 of the instance's copied planes
    float* region = planes + (z.live ? z.sub : 0) * L::PS;
    const int shift = MF ? 0 : (int)((kSym * z.off) & 3);
    const float* pl = region + shift;
    double x[L::R], r64[L::R];
    double bb = 0.0;
    float S[L::R][kStencil], dinv[L::R];
    int hn = -1;
    if constexpr (MF) {
        // the operator from the amplitude: FP32 stencil to registers, low
        // parts to the planes buffer, r = -K x0 + coef M w / dt
        mf_start<L>(A, z, xg, *ms, region, S, r64);
#pragma unroll
        for (int i = 0; i < L::R; ++i) dinv[i] = row_ok<L>(z, i) ? 1.0f / S[i][4] : 0.0f;
#pragma unroll
        for (int i = 0; i < L::R; ++i) x[i] = row_ok<L>(z, i) ? xg[cell_of<L>(z, i)] : 0.0;
        prefetch();
    } else {
        pack_start<L>(A, z, xg, x, r64, bb, A.Ss32 + kSym * z.off, region, shift, hslot, hist, mtab);
        if (hslot != nullptr) hn = hist;
        planes_copy_wait();
        const LdsPlanes<L> plc(pl, z);
        // coefficient 1 of row i > 0 is coefficient 7 of row i-1; rows past
        // the mesh give products that are discarded and diag^{-1} = 0
#pragma unroll
        for (int i = 0; i < L::R; ++i)
#pragma unroll
            for (int k = 0; k < kStencil; ++k)
                S[i][k] = (k == 1 && i > 0) ? S[i - 1][7] : plc.at(z, i, k);
#pragma unroll
        for (int i = 0; i < L::R; ++i) dinv[i] = row_ok<L>(z, i) ? 1.0f / S[i][4] : 0.0f;
        // every wave has its stencil: the planes buffer takes the low parts next
        lds_barrier();
        if (z.live) planes_copy_start<L>(A.Sslo + kSym * z.off, region, z.lt, shift);
        prefetch();
    }
    const LdsPlanes<L> plv(pl, z);
    const RegStencil<L, float> SR{S};
    const SplitStencil<L> S64{S, plv};
    // separable mass (stored-operator form): r64 holds b = coef M w/dt +
    // M x0/dt and becomes b - S32 x0 here; the low part -Slo x0 joins at the
    // first FP64 update (the low parts arrive during the first inner solve)
    const bool mfree = !MF && mtab != nullptr && mass_free(A);
    if (A.rhs_vec == nullptr) {
        // ||b|| of the time step from b = S x0 + r (S in FP32: the norm only
        // sizes the tolerance, ~1e-7 relative is plenty); x0 is in the grid
        double sb[L::R];
#pragma unroll
        for (int i = 0; i < L::R; ++i) sb[i] = 0.0;
        if (z.act) strip_apply<L, L::R>(SR, xg, z, x, sb);
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            const double bi = mfree ? r64[i] : sb[i] + r64[i];
            if (mfree) r64[i] -= sb[i];
            bb += row_ok<L>(z, i) ? bi * bi : 0.0;
        }
    }
    // ||b||^2, ||r||^2 and the residual of the start test: without the low
    // part, r64 is exact only where x0 = 0, so an instance with x0 != 0
    // takes at least one sweep (its test value is huge)
    bool nz = false;
#pragma unroll
    for (int i = 0; i < L::R; ++i) nz = nz || x[i] != 0.0;
    double acc[3] = {bb, 0.0, (mfree && nz) ? 1e300 : 0.0};
#pragma unroll
    for (int i = 0; i < L::R; ++i) acc[1] += r64[i] * r64[i];
    acc[2] += acc[1];
    red3.sum<L>(acc, z.w0);
    __shared__ double otol_s[L::IPP];
    __shared__ float itol_s[L::IPP];
    const double tol2 = A.rtol * A.rtol * acc[0];
    if (z.live && z.lt == 0) otol_s[z.sub] = tol2;
    double rr = acc[1];
    bool conv = acc[2] <= tol2;
    int sweeps = 1, iters = 0;
    zero_halo<L, float>(pg, z);     // the float view of the grid from here on
    // second float grid (the upper half of the double one): x0 in FP32 for
    // the low-part term of the first update
    float* pg2 = pg + L::GRID;
    if (mfree) zero_halo<L, float>(pg2, z);
    lds_barrier();
    const double othr = lane_threshold<L>(otol_s, cnt);
    bool ogo = red3.any_above(othr);
    while (ogo && sweeps <= A.max_refine) {
        // Inner FP32 solve of S d = r / ||r|| by the Chronopoulos-Gear form of
        // PCG: s = S p is carried by a recurrence, so each iteration needs one
        // operator application (w = S u, u = D^{-1} r) and ONE fused reduction
        // of (w,u) and (r,u); two barriers per iteration.  The inner test is
        // on the preconditioned norm: (r,u) <= itol2 (r0,u0), with each
        // instance's own itol2 (inner_tol2); outer-converged instances enter
        // with r = 0 and sit out.  Frozen instances take alpha = beta = 0,
        // which leaves d and r unchanged, so the update needs no branch.
        const bool me = !conv;
        const double rn = sqrt(rr);
        const double isc = me ? 1.0 / rn : 0.0;
        float r[L::R], d[L::R], p[L::R], sv[L::R];
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            r[i] = (float)(r64[i] * isc);
            d[i] = 0.0f;
            p[i] = 0.0f;
            sv[i] = 0.0f;
        }
        const float itol2 = me ? inner_tol2(tol2, rr, A.inner_rtol) : 0.0f;
        if (z.live && z.lt == 0) itol_s[z.sub] = itol2;
        lds_barrier();
        const float ithr = lane_threshold<L>(itol_s, cnt);
        float vthr = ithr, gam0 = 0.0f;
        float gam_prev = 1.0f, alpha_prev = 1.0f;
        bool iconv = !me;
        int k = 0;
        // Extrapolated start of the first inner solve: d0 = (predicted
        // increment) / ||r||, r = r/||r|| - S d0.  The inner test stays
        // relative to the residual without the guess, and an instance whose
        // guessed residual is not smaller drops the guess (d0 = 0).  The FP64
        // update below takes the whole d, the guess included, so the outer
        // residual stays exact.  One operator application and one reduction.
        const bool guessed = hn >= 1 && sweeps == 1;
        if (guessed) {
            const float fs = (float)isc;
#pragma unroll
            for (int i = 0; i < L::R; ++i) d[i] = hslot[i * NTP + threadIdx.x] * fs;
            strip_store<L>(pg, z, d);
            lds_barrier();
            float sd[L::R];
            strip_apply<L, L::R>(SR, pg, z, d, sd);
            float g2[2] = {0.0f, 0.0f};     // guessed and plain (r, D^-1 r)
#pragma unroll
            for (int i = 0; i < L::R; ++i) {
                sd[i] = r[i] - sd[i];
                g2[0] += sd[i] * dinv[i] * sd[i];
                g2[1] += r[i] * dinv[i] * r[i];
            }
            rf2.sum<L>(g2, z.w0);     // its barrier also ends the reads of d in the grid
            const bool keep = g2[0] < g2[1];
#pragma unroll
            for (int i = 0; i < L::R; ++i) {
                r[i] = keep ? sd[i] : r[i];
                d[i] = keep ? d[i] : 0.0f;
            }
            gam0 = g2[1];
            vthr = (ithr < INFINITY) ? ithr * rf2.tail : ithr;
        }
        // One iteration, from the direction pair (pi, si) to (po, so): u and
        // w are formed in po and so, which then become the new p and s.  Two
        // iterations per loop trip with the pairs swapped, so the new p and s
        // are never copied back into the old registers.  True: stop.
        auto iterate = [&](const float (&pi)[L::R], const float (&si)[L::R], float (&po)[L::R],
                           float (&so)[L::R]) -> bool {
#pragma unroll
            for (int i = 0; i < L::R; ++i) po[i] = dinv[i] * r[i];     // u
            strip_store<L>(pg, z, po);
            lds_barrier();
            // every lane applies (no branch): the reads of inactive and spare
            // lanes stay inside the LDS block, rows past the mesh give 0, and
            // spare waves never enter a sum
            strip_apply<L, L::R>(SR, pg, z, po, so);                    // w = S u
            float g2[2] = {0.0f, 0.0f};     // (w,u), (r,u)
#pragma unroll
            for (int i = 0; i < L::R; ++i) {
                g2[0] += so[i] * po[i];
                g2[1] += r[i] * po[i];
            }
            rf2.sum<L>(g2, z.w0);
            if (k == 0 && !guessed) {
                gam0 = g2[1];
                vthr = (ithr < INFINITY) ? ithr * rf2.tail : ithr;
            }
            if (!iconv && g2[1] <= itol2 * gam0) iconv = true;
            if (!rf2.any_above(vthr) || k >= A.max_iter) return true;
            const float gam = g2[1];
            const float beta = (k == 0 || iconv) ? 0.0f : gam * __builtin_amdgcn_rcpf(gam_prev);
            const float den = (k == 0) ? g2[0] : g2[0] - beta * gam * __builtin_amdgcn_rcpf(alpha_prev);
            const float alpha = iconv ? 0.0f : gam * __builtin_amdgcn_rcpf(den);
#pragma unroll
            for (int i = 0; i < L::R; ++i) {
                po[i] = po[i] + beta * pi[i];     // p = u + beta p
                so[i] = so[i] + beta * si[i];     // s = w + beta s
                d[i] += alpha * po[i];
                r[i] -= alpha * so[i];
            }
            if (!iconv) {
                gam_prev = gam;
                alpha_prev = alpha;
                ++iters;
            }
            ++k;
            return false;
        };
        float p2[L::R], sv2[L::R];
        for (;;) {
            if (iterate(p, sv, p2, sv2)) break;
            if (iterate(p2, sv2, p, sv)) break;
        }
        // x += ||r|| d;  r64 -= ||r|| S d  (FP64 stencil, d exact in FP64)
        const double sc = me ? rn : 0.0;
        // separable mass, first update: also r64 -= Slo x0 (x0 in FP32 in the
        // second grid: the low parts are ~2^-24 of S, so this rounding is
        // ~2^-48 of S x0, the size of the split's own)
        const bool low0 = mfree && sweeps == 1;
        if (low0) {
            float x0f[L::R];
#pragma unroll
            for (int i = 0; i < L::R; ++i) x0f[i] = (float)x[i];
            strip_store<L>(pg2, z, x0f);
        }
#pragma unroll
        for (int i = 0; i < L::R; ++i) x[i] += sc * (double)d[i];
        strip_store<L>(pg, z, d);
        planes_copy_wait();     // the low parts are in LDS from here on
        if (low0 && z.act) {
            float x0f[L::R];
#pragma unroll
            for (int i = 0; i < L::R; ++i) x0f[i] = pg2[cell_of<L>(z, i)];
            double s0[L::R];
#pragma unroll
            for (int i = 0; i < L::R; ++i) s0[i] = 0.0;
            strip_apply_lean<L, 1>(LowStencil<L>{plv}, pg2, z, x0f, s0);
#pragma unroll
            for (int i = 0; i < L::R; ++i) r64[i] -= s0[i];
        }
        double sd[L::R];
#pragma unroll
        for (int i = 0; i < L::R; ++i) sd[i] = 0.0;
        // Once the residual is within 2^12 of the tolerance, the FP32 stencil
        // alone is exact enough for the update: its rounding error is about
        // 2^-24 of the update (which is about the residual), i.e. below 2^-12
        // of the tolerance, and the low part need not be read.
        const bool lo = rr > 16777216.0 * tol2;
        if (z.act) {
            if (lo) strip_apply_lean<L, L::R>(S64, pg, z, d, sd);
            else strip_apply<L, L::R>(SR, pg, z, d, sd);
        }
        double a1[1] = {0.0};
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            r64[i] -= sc * sd[i];
            a1[0] += r64[i] * r64[i];
        }
        red1.sum<L>(a1, z.w0);
        ogo = red1.any_above(othr);
        ++sweeps;
        rr = a1[0];
        if (!conv && rr <= tol2) conv = true;
    }
    // the copy must end before the next pack's copy reuses the buffer (a pack
    // that needs no sweep never waited for it)
    planes_copy_wait();
    pack_store<L>(A, z, x, iters, sweeps, conv, rr, red1);
}

// Iterate slots of the FP64 solves (xs of pack_fp64): the most rows per lane.
constexpr int kFp64Rows = cmax(cmax(L16::R, L32::R), L64::R);

// FP32 planes buffer of the refinement (one pack's instances), in LDS, with
// room for the reads past the last instance's planes (LdsPlanes).
constexpr int kPlaneFloats =
    cmax(cmax(L16::IPP * L16::PS, L32::IPP * L32::PS), L64::IPP * L64::PS) + 2 * (kMaxLevel + 1);

// Reduction buffers and pack metadata of one packed workgroup.
struct PackShared {
    double r1[2][NWP][4];
    double r2[2][NWP][4];
    double r3[2][NWP][4];
    float f3[2][NWP][4];
    int32_t meta[2][kMetaWords];   // this pack's and the next one's
    int task;
    int hist;                      // steps of history of the extrapolated start (history_steps)
};

// The work loop of a packed workgroup.  With a queue, packs are popped one
// ahead: while pack t is solved, the first wave pops the next pack and copies
// its metadata into the other half of sh.meta (the solve calls prefetch()
// once it has its own data in flight), so that the next solve starts from
// LDS instead of three dependent global round trips.  Without a queue the
// workgroup solves pack blockIdx.x.  solve(meta, cnt, level, prefetch).
template <class Solve>
__device__ __forceinline__ void pack_loop(const MicroArgs& A, const PackList& P, const int32_t* pack_level,
                                          PackShared& sh, Solve solve) {
    int task;
    if (A.queue != nullptr) {
        if (threadIdx.x == 0) sh.task = atomicAdd(A.queue, 1);
        __syncthreads();
        task = sh.task;
    } else {
        task = blockIdx.x;
    }
    if (task < P.n_packs && threadIdx.x < kWave) meta_copy_start(P, pack_level, task, sh.meta[0]);
    // the history count is fixed during the launch: read once, here, so that
    // no wait for it lands behind a pack's plane copy
    if (threadIdx.x == 0) sh.hist = history_steps(A);
    planes_copy_wait();
    int buf = 0;
    while (task < P.n_packs) {
        int nxt = P.n_packs;
        if (A.queue != nullptr && threadIdx.x == 0) nxt = atomicAdd(A.queue, 1);
        const int32_t* meta = sh.meta[buf];
        int32_t* meta_next = sh.meta[buf ^ 1];
        auto prefetch = [&]() {
            if (A.queue != nullptr && threadIdx.x < kWave) {
                const int n = __builtin_amdgcn_readfirstlane(nxt);
                if (threadIdx.x == 0) sh.task = n;
                if (n < P.n_packs) meta_copy_start(P, pack_level, n, meta_next);
            }
        };
        solve(meta, meta[kMetaCount], meta[kMetaLevel], prefetch);
        if (A.queue == nullptr) break;
        planes_copy_wait();     // the next pack's metadata has landed
        task = sh.task;
        buf ^= 1;
        __syncthreads();        // every wave has read sh.task before it is rewritten
    }
}

// MODE: 1 FP64, 2 refine.  One instantiation per mesh size (LV), so each
// gets its own register allocation.
template <int MODE, class L>
__global__ __launch_bounds__(NTP) void packed_kernel(MicroArgs A, PackList P) {
    extern __shared__ double lds[];
    __shared__ PackShared sh;
    PackRed<1, double> red1(sh.r1);
    PackRed<2, double> red2(sh.r2);
    PackRed<3, double> red3(sh.r3);
    PackRed<2, float> rf2(sh.f3);
    if constexpr (MODE == 2) {
        __shared__ __attribute__((aligned(16))) float planes[L::PS * L::IPP + 2 * L::NP];
        __shared__ float hslot[L::R * NTP];
        __shared__ __attribute__((aligned(16))) double mtab[16 * L::NP];
        pack_loop(A, P, nullptr, sh, [&](const int32_t* meta, int cnt, int, auto prefetch) {
            pack_refine<L, false>(A, meta, cnt, lds, planes, nullptr, red1, red3, rf2, prefetch, hslot, sh.hist,
                                  mtab);
        });
    } else if constexpr (MODE == 3) {
        __shared__ __attribute__((aligned(16))) float planes[L::PS * L::IPP + 2 * L::NP];
        __shared__ MfShared ms;
        pack_loop(A, P, nullptr, sh, [&](const int32_t* meta, int cnt, int, auto prefetch) {
            pack_refine<L, true>(A, meta, cnt, lds, planes, &ms, red1, red3, rf2, prefetch, nullptr, -1);
        });
    } else {
        __shared__ double xs[L::R * NTP];
        // the corner couplings of the resident stencil (2 x R doubles a lane)
        __shared__ double cs[2 * L::R * NTP];
        __shared__ __attribute__((aligned(16))) double mtab[16 * L::NP];
        pack_loop(A, P, nullptr, sh, [&](const int32_t* meta, int cnt, int, auto prefetch) {
            pack_fp64<L, true>(A, meta, cnt, lds, xs, red1, red2, red3, prefetch, cs, sh.hist, mtab);
        });
    }
}

// All mesh sizes in ONE persistent launch: every workgroup pops packs from a
// work queue (packs in largest-first order) until the queue is empty; the
// register allocation is the largest of the three size paths.
template <int MODE>
__global__ __launch_bounds__(NTP) void packed_mixed_kernel(MicroArgs A, PackList P, const int32_t* pack_level) {
    extern __shared__ double lds[];
    __shared__ PackShared sh;
    PackRed<1, double> red1(sh.r1);
    PackRed<2, double> red2(sh.r2);
    PackRed<3, double> red3(sh.r3);
    PackRed<2, float> rf2(sh.f3);
    if constexpr (MODE == 2) {
        __shared__ __attribute__((aligned(16))) float planes[kPlaneFloats];
        __shared__ float hslot[kFp64Rows * NTP];
        __shared__ __attribute__((aligned(16))) double mtab[16 * (kMaxLevel + 1)];
        pack_loop(A, P, pack_level, sh, [&](const int32_t* meta, int cnt, int lvl, auto prefetch) {
            if (lvl == 64)
                pack_refine<L64, false>(A, meta, cnt, lds, planes, nullptr, red1, red3, rf2, prefetch, hslot, sh.hist,
                                        mtab);
            else if (lvl == 32)
                pack_refine<L32, false>(A, meta, cnt, lds, planes, nullptr, red1, red3, rf2, prefetch, hslot, sh.hist,
                                        mtab);
            else pack_refine<L16, false>(A, meta, cnt, lds, planes, nullptr, red1, red3, rf2, prefetch, hslot, sh.hist,
                                         mtab);
        });
    } else if constexpr (MODE == 3) {
        __shared__ __attribute__((aligned(16))) float planes[kPlaneFloats];
        __shared__ MfShared ms;
        pack_loop(A, P, pack_level, sh, [&](const int32_t* meta, int cnt, int lvl, auto prefetch) {
            if (lvl == 64)
                pack_refine<L64, true>(A, meta, cnt, lds, planes, &ms, red1, red3, rf2, prefetch, nullptr, -1);
            else if (lvl == 32)
                pack_refine<L32, true>(A, meta, cnt, lds, planes, &ms, red1, red3, rf2, prefetch, nullptr, -1);
            else pack_refine<L16, true>(A, meta, cnt, lds, planes, &ms, red1, red3, rf2, prefetch, nullptr, -1);
        });
    } else {
        __shared__ double xs[kFp64Rows * NTP];
        __shared__ double cs[2 * kFp64Rows * NTP];
        __shared__ __attribute__((aligned(16))) double mtab[16 * (kMaxLevel + 1)];
        pack_loop(A, P, pack_level, sh, [&](const int32_t* meta, int cnt, int lvl, auto prefetch) {
            if (lvl == 64) pack_fp64<L64, true>(A, meta, cnt, lds, xs, red1, red2, red3, prefetch, cs, sh.hist, mtab);
            else if (lvl == 32)
                pack_fp64<L32, true>(A, meta, cnt, lds, xs, red1, red2, red3, prefetch, cs, sh.hist, mtab);
            else pack_fp64<L16, true>(A, meta, cnt, lds, xs, red1, red2, red3, prefetch, cs, sh.hist, mtab);
        });
    }
}

template <class L>
hipError_t launch_level(const MicroArgs& a, const PackList& p, int mode, int grid, hipStream_t s) {
    const size_t lds = sizeof(double) * L::GRID * L::IPP;
    if (mode == 3) hipLaunchKernelGGL((packed_kernel<3, L>), dim3(grid), dim3(NTP), lds, s, a, p);
    else if (mode == 2) hipLaunchKernelGGL((packed_kernel<2, L>), dim3(grid), dim3(NTP), lds, s, a, p);
    else hipLaunchKernelGGL((packed_kernel<1, L>), dim3(grid), dim3(NTP), lds, s, a, p);
    return hipGetLastError();
}

}  // namespace

int packed_capacity(int level) {
    switch (level) {
        case 16: return L16::IPP;
        case 32: return L32::IPP;
        case 64: return L64::IPP;
        default: return 0;
    }
}

size_t packed_lds_bytes(int level) {
    switch (level) {
        case 16: return sizeof(double) * L16::GRID * L16::IPP;
        case 32: return sizeof(double) * L32::GRID * L32::IPP;
        case 64: return sizeof(double) * L64::GRID * L64::IPP;
        default: return 0;
    }
}

hipError_t launch_packed_mixed(const MicroArgs& a, const PackList& p, const int32_t* pack_level, int mode,
                               int grid, size_t lds, hipStream_t s) {
    if (p.n_packs <= 0 || grid <= 0 || a.queue == nullptr) return hipSuccess;
    if (mode == 3) hipLaunchKernelGGL(packed_mixed_kernel<3>, dim3(grid), dim3(NTP), lds, s, a, p, pack_level);
    else if (mode == 2) hipLaunchKernelGGL(packed_mixed_kernel<2>, dim3(grid), dim3(NTP), lds, s, a, p, pack_level);
    else if (mode == 1) hipLaunchKernelGGL(packed_mixed_kernel<1>, dim3(grid), dim3(NTP), lds, s, a, p, pack_level);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_packed(const MicroArgs& a, const PackList& p, int level, int mode, int grid, hipStream_t s) {
    if (p.n_packs <= 0 || grid <= 0) return hipSuccess;
    if (mode < 1 || mode > 3) return hipErrorInvalidValue;
    switch (level) {
        case 16: return launch_level<L16>(a, p, mode, grid, s);
        case 32: return launch_level<L32>(a, p, mode, grid, s);
        case 64: return launch_level<L64>(a, p, mode, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tsm
