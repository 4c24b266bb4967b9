// Packed micro solves for the common mesh sizes (16, 32 and 64 cells per
// side): Jacobi-preconditioned CG (paper Section 3.3: CG on every micro
// system, the systems distributed over the processors), laid out for a
// 1024-lane workgroup that solves a pack of instances of one size in
// lockstep:
//     64x64: 1 instance on 14 waves,  32x32: 4 instances on 4 waves each,
//     16x16: 16 instances on 1 wave each.
// Within an instance, lane l owns column l % (N+1) and a strip of R
// consecutive rows.  Each iteration it reads only the left/right neighbour
// columns and the two rows past its strip from LDS (2R+6 reads for R nodes,
// against 9R for one node per lane); its own column comes from registers.
// Vectors live in an LDS grid with a zero halo (rows past the mesh included),
// so boundary rows need no bounds checks.
//
// Register budget (1024 lanes: 128 VGPRs per lane) decides the data flow:
//   FP64 form     x, r, p, q in FP64 registers, diag^{-1} in FP32 (the
//                 preconditioner need not be exact), FP64 stencil re-read
//                 from global memory every iteration.
//   REFINE form   FP32 stencil and diag^{-1} resident in registers for the
//                 whole solve; FP32 PCG on S d = r/||r||; the FP64 residual
//                 is formed once from b = M x0/dt and S x0, then updated as
//                 r <- r - ||r|| S d with the FP64 stencil (read once per
//                 sweep), x <- x + ||r|| d, until ||r|| <= rtol ||b||.
//
// Lockstep: all instances of a pack pass the same barriers; an instance
// that has met its tolerance freezes while the others go on.  Dot products:
// wavefront butterfly, one LDS exchange per reduction (ping-pong buffer,
// one barrier), per-instance sums in a fixed order.
#include "device_common.h"

namespace tsm {

namespace {

constexpr int NTP = kPackThreads;
constexpr int NWP = NTP / kWave;

template <int N_, int TPI_, int R_>
struct Lvl {
    static constexpr int N = N_, NP = N_ + 1, W2 = N_ + 3, R = R_;
    static constexpr int NS = (NP + R_ - 1) / R_;          // strips per instance
    static constexpr int H2 = NS * R_ + 2;                  // grid rows: strips plus halo
    static constexpr int TPI = TPI_, WPI = TPI_ / kWave;    // lanes / waves per instance
    static constexpr int IPP = NTP / TPI_;                  // instances per pack
    static constexpr int GRID = H2 * W2;                    // LDS cells per instance
    static constexpr int n = NP * NP;
    static_assert(NS * NP <= TPI, "strips do not fit the lanes of an instance");
    static_assert(TPI % kWave == 0, "an instance owns whole waves");
};
using L16 = Lvl<16, 64, 6>;
using L32 = Lvl<32, 256, 5>;
using L64 = Lvl<64, 896, 5>;

template <int NV, typename T>
struct PackRed {
    T (*buf)[NV][NWP];
    int phase = 0;
    __device__ PackRed(T (*b)[NV][NWP]) : buf(b) {}
    // Per-instance sums (instance = waves [w0, w0+wpi)).  All lanes call.
    __device__ __forceinline__ void sum(T (&v)[NV], int w0, int wpi) {
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
        if (lane == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) buf[phase][i][wid] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            T s = buf[phase][i][w0];
            for (int w = 1; w < wpi; ++w) s += buf[phase][i][w0 + w];
            v[i] = s;
        }
        phase ^= 1;
    }
    // value NV-1 of instance k from the last sum
    __device__ __forceinline__ T last_of(int k, int wpi) const {
        const int ph = phase ^ 1;
        T s = buf[ph][NV - 1][k * wpi];
        for (int w = 1; w < wpi; ++w) s += buf[ph][NV - 1][k * wpi + w];
        return s;
    }
};

struct Lane {
    int sub, lt, col, r0, inst, w0;     // w0: first wave of the instance (0 for spare lanes)
    bool live, act;
    int64_t off;
};

template <class L>
__device__ __forceinline__ Lane lane_of(const MicroArgs& A, int first, int cnt) {
    Lane z;
    z.sub = threadIdx.x / L::TPI;
    z.lt = threadIdx.x - z.sub * L::TPI;
    z.w0 = (z.sub < L::IPP ? z.sub : 0) * L::WPI;
    z.live = z.sub < L::IPP && z.sub < cnt;
    // every wave belongs to one instance: instance and offset are wave-uniform
    int inst = z.live ? A.order[first + z.sub] : 0;
    inst = __builtin_amdgcn_readfirstlane(inst);
    z.inst = inst;
    z.col = z.lt % L::NP;
    const int strip = z.lt / L::NP;
    z.r0 = strip * L::R;
    z.act = z.live && strip < L::NS;
    const int64_t off = z.live ? A.offsets[inst] : 0;
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

// Stencil sources.  A source gives, for row i of the lane's strip and
// coefficient k, a raw value (load) and the coefficient (value):
//   RegStencil     FP32 stencil resident in registers
//   GlobalStencil  stencil in global memory, coefficient-major [k][n]
//   SplitStencil   FP64 operator as resident FP32 part + streamed FP32 low
//                  part: S32 + Slo spans at most 48 significant bits, so the
//                  FP64 sum is exact and equals S to about 2^-48 relative.
template <class L, typename TS>
struct RegStencil {
    static constexpr bool kGlobal = false;
    using raw_t = TS;
    const TS (&S)[L::R][kStencil];
    __device__ __forceinline__ TS load(const Lane&, int i, int k) const { return S[i][k]; }
    __device__ __forceinline__ TS value(int, int, TS raw) const { return raw; }
};

// The base pointer of a streamed stencil passes through an empty asm at
// every use, so the compiler cannot hoist the loop-invariant coefficient
// loads out of the solver loops and keep them live across them.
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// wave-uniform base + zero-extended 32-bit byte offset (scalar-base
// addressing); rows past the mesh read the last mesh row, in bounds, and
// their results are discarded
template <class L, typename T>
__device__ __forceinline__ T stencil_load(const T* base, const Lane& z, int i, int k) {
    const int row = min(z.r0 + i, L::NP - 1);
    const uint32_t byte = (uint32_t)(k * L::n + row * L::NP + z.col) * (uint32_t)sizeof(T);
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte);
}

template <class L, typename TS>
struct GlobalStencil {
    static constexpr bool kGlobal = true;
    using raw_t = TS;
    const TS* __restrict__ base;
    __device__ __forceinline__ TS load(const Lane& z, int i, int k) const { return stencil_load<L>(base, z, i, k); }
    __device__ __forceinline__ TS value(int, int, TS raw) const { return raw; }
    __device__ __forceinline__ TS at(const Lane& z, int i, int k) const { return load(z, i, k); }
};

template <class L>
struct SplitStencil {
    static constexpr bool kGlobal = true;
    using raw_t = float;
    const float (&S)[L::R][kStencil];
    const float* __restrict__ base;   // Slo
    __device__ __forceinline__ float load(const Lane& z, int i, int k) const { return stencil_load<L>(base, z, i, k); }
    __device__ __forceinline__ double value(int i, int k, float raw) const { return (double)S[i][k] + (double)raw; }
};

// y_i = sum_k S_ik g(row r0+i + dr, col + dc) in k order 0..8, one product
// at a time; own-column values come from mine[].  Streamed coefficients are
// loaded B rows at a time, all loads of a batch in flight before the first
// use (scheduling barriers keep the batches apart without draining memory).
// Rows past the mesh give 0.  Active lanes only.
template <class L, int B, typename TA, typename TG, class ST>
__device__ __forceinline__ void strip_apply(const ST& S0, const TG* g, const Lane& z,
                                            const TG (&mine)[L::R], TA (&y)[L::R]) {
    ST S = S0;
    if constexpr (ST::kGlobal) S.base = opaque(S.base);
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
#pragma unroll
    for (int i0 = 0; i0 < L::R; i0 += B) {
        typename ST::raw_t c[B][kStencil];
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int k = 0; k < kStencil; ++k)
                if (i0 + b < L::R) c[b][k] = S.load(z, i0 + b, k);
        if constexpr (ST::kGlobal) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            if (i >= L::R) break;
            const TG cm = (i == 0) ? up : mine[i - 1];
            const TG cp = (i == L::R - 1) ? dn : mine[i + 1];
            TA t = TA(0);
            t += TA(S.value(i, 0, c[b][0])) * TA(lf[i]);
            t += TA(S.value(i, 1, c[b][1])) * TA(cm);
            t += TA(S.value(i, 2, c[b][2])) * TA(rt[i]);
            t += TA(S.value(i, 3, c[b][3])) * TA(lf[i + 1]);
            t += TA(S.value(i, 4, c[b][4])) * TA(mine[i]);
            t += TA(S.value(i, 5, c[b][5])) * TA(rt[i + 1]);
            t += TA(S.value(i, 6, c[b][6])) * TA(lf[i + 2]);
            t += TA(S.value(i, 7, c[b][7])) * TA(cp);
            t += TA(S.value(i, 8, c[b][8])) * TA(rt[i + 2]);
            y[i] = (z.r0 + i < L::NP) ? t : TA(0);
        }
        if constexpr (ST::kGlobal) __builtin_amdgcn_sched_barrier(0);
    }
}

template <class L>
__device__ __forceinline__ void pack_store(const MicroArgs& A, const Lane& z, const double (&x)[L::R],
                                           int iters, int sweeps, bool conv, PackRed<1, double>& red1) {
    double bx[1] = {0.0};
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        if (row_ok<L>(z, i)) {
            const int j = node_of<L>(z, i);
            A.X_out[z.off + j] = x[i];
            bx[0] += A.b[z.off + j] * x[i];
        }
    }
    red1.sum(bx, z.w0, L::WPI);
    if (z.live && z.lt == 0) {
        A.bx_out[z.inst] = bx[0];
        if (A.iters_out) A.iters_out[z.inst] = iters;
        if (A.sweeps_out) A.sweeps_out[z.inst] = sweeps;
        if (!conv) atomicAdd(A.nonconv, 1);
    }
}

// x0 into registers and the (double) grid; b = M x0/dt or the given
// right-hand side; r = b - S x0 with the FP64 stencil; bb = partial ||b||^2.
template <class L>
__device__ __forceinline__ void pack_start(const MicroArgs& A, const Lane& z, double* xg, double (&x)[L::R],
                                           double (&r)[L::R], double& bb) {
    zero_halo<L, double>(xg, z);
    const double cf = (z.live && A.coef != nullptr) ? A.coef[z.inst] : 0.0;
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        double v = 0.0;
        if (row_ok<L>(z, i) && !A.zero_init) {
            const int j = node_of<L>(z, i);
            v = A.X0[z.off + j] + cf * A.w[z.off + j];
        }
        x[i] = v;
        if (row_ok<L>(z, i)) xg[cell_of<L>(z, i)] = v;
    }
    __syncthreads();
    double b[L::R], sx[L::R];
#pragma unroll
    for (int i = 0; i < L::R; ++i) { b[i] = 0.0; sx[i] = 0.0; }
    if (A.rhs_vec != nullptr) {
#pragma unroll
        for (int i = 0; i < L::R; ++i)
            b[i] = row_ok<L>(z, i) ? A.rhs_scale * A.rhs_vec[z.off + node_of<L>(z, i)] : 0.0;
    } else if (z.act) {
        strip_apply<L, 3>(GlobalStencil<L, double>{A.M64 + kStencil * z.off}, xg, z, x, b);
#pragma unroll
        for (int i = 0; i < L::R; ++i) b[i] *= A.inv_dt;
    }
    if (z.act) strip_apply<L, 3>(GlobalStencil<L, double>{A.S64 + kStencil * z.off}, xg, z, x, sx);
    bb = 0.0;
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        r[i] = row_ok<L>(z, i) ? b[i] - sx[i] : 0.0;
        bb += row_ok<L>(z, i) ? b[i] * b[i] : 0.0;
    }
}

// ------------------------------------------------------------------ FP64
template <class L>
__device__ void pack_fp64(const MicroArgs& A, int first, int cnt, double* lds, PackRed<1, double>& red1,
                          PackRed<3, double>& red3) {
    const Lane z = lane_of<L>(A, first, cnt);
    double* xg = lds + (z.sub < L::IPP ? z.sub : 0) * L::GRID;
    const GlobalStencil<L, double> S{A.S64 + kStencil * z.off};
    double x[L::R], r[L::R], p[L::R];
    float dinv[L::R];
    double bb;
    pack_start<L>(A, z, xg, x, r, bb);
    double acc[3] = {bb, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < L::R; ++i) {
        dinv[i] = row_ok<L>(z, i) ? (float)(1.0 / S.at(z, i, 4)) : 0.0f;
        p[i] = (double)dinv[i] * r[i];
        acc[1] += r[i] * p[i];
        acc[2] += r[i] * r[i];
    }
    red3.sum(acc, z.w0, L::WPI);
    __shared__ double tol_s[L::IPP];
    const double tol2 = A.rtol * A.rtol * acc[0];
    if (z.live && z.lt == 0) tol_s[z.sub] = tol2;
    double rz = acc[1];
    bool conv = acc[2] <= tol2;
    int it = 0;
    __syncthreads();
    auto any_active = [&]() {
        bool any = false;
        for (int s = 0; s < L::IPP && s < cnt; ++s) any |= red3.last_of(s, L::WPI) > tol_s[s];
        return any;
    };
    bool go = any_active();
    int k = 0;
    while (go && k < A.max_iter) {
        const bool me = !conv;
#pragma unroll
        for (int i = 0; i < L::R; ++i)
            if (row_ok<L>(z, i)) xg[cell_of<L>(z, i)] = p[i];
        __syncthreads();
        double q[L::R];
#pragma unroll
        for (int i = 0; i < L::R; ++i) q[i] = 0.0;
        if (z.act) strip_apply<L, 2>(S, xg, z, p, q);
        double pq[1] = {0.0};
#pragma unroll
        for (int i = 0; i < L::R; ++i) pq[0] += p[i] * q[i];
        red1.sum(pq, z.w0, L::WPI);
        const double alpha = me ? rz / pq[0] : 0.0;
        double a3[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            a3[1] += r[i] * (double)dinv[i] * r[i];
            a3[2] += r[i] * r[i];
        }
        red3.sum(a3, z.w0, L::WPI);
        ++k;
        if (me) {
            ++it;
            if (a3[2] <= tol2) {
                conv = true;
            } else {
                const double beta = a3[1] / rz;
                rz = a3[1];
#pragma unroll
                for (int i = 0; i < L::R; ++i) p[i] = (double)dinv[i] * r[i] + beta * p[i];
            }
        }
        go = any_active();
    }
    pack_store<L>(A, z, x, it, 1, conv, red1);
}

// --------------------------------------------------------------- REFINE
template <class L>
__device__ void pack_refine(const MicroArgs& A, int first, int cnt, double* lds, PackRed<1, double>& red1,
                            PackRed<3, double>& red3, PackRed<1, float>& rf1, PackRed<3, float>& rf3) {
    const Lane z = lane_of<L>(A, first, cnt);
    double* xg = lds + (z.sub < L::IPP ? z.sub : 0) * L::GRID;
    float* pg = reinterpret_cast<float*>(xg);
    double x[L::R], r64[L::R];
    double bb;
    pack_start<L>(A, z, xg, x, r64, bb);
    float S[L::R][kStencil], dinv[L::R];
    {
        // branch-free: every row's loads in flight at once (rows past the
        // mesh read in bounds and are zeroed)
        const float* Sf = A.S32 + kStencil * z.off;
#pragma unroll
        for (int i = 0; i < L::R; ++i)
#pragma unroll
            for (int k = 0; k < kStencil; ++k) S[i][k] = stencil_load<L>(Sf, z, i, k);
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            const bool ok = row_ok<L>(z, i);
#pragma unroll
            for (int k = 0; k < kStencil; ++k) S[i][k] = ok ? S[i][k] : 0.0f;
            dinv[i] = ok ? 1.0f / S[i][4] : 0.0f;
        }
    }
    const RegStencil<L, float> SR{S};
    const SplitStencil<L> S64{S, A.Slo + kStencil * z.off};
    double acc[3] = {bb, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < L::R; ++i) acc[2] += r64[i] * r64[i];
    red3.sum(acc, z.w0, L::WPI);
    __shared__ double otol_s[L::IPP];
    const double tol2 = A.rtol * A.rtol * acc[0];
    if (z.live && z.lt == 0) otol_s[z.sub] = tol2;
    double rr = acc[2];
    bool conv = rr <= tol2;
    int sweeps = 1, iters = 0;
    zero_halo<L, float>(pg, z);     // the float view of the grid from here on
    __syncthreads();
    auto outer_any = [&]() {
        bool any = false;
        for (int s = 0; s < L::IPP && s < cnt; ++s) any |= red3.last_of(s, L::WPI) > otol_s[s];
        return any;
    };
    while (outer_any() && sweeps <= A.max_refine) {
        // Inner FP32 solve of S d = r / ||r|| by the Chronopoulos-Gear form of
        // PCG: s = S p is carried by a recurrence, so each iteration needs one
        // operator application (w = S u, u = D^{-1} r) and ONE fused reduction
        // of (r,u), (w,u), (r,r); two barriers per iteration.  The normalised
        // residual starts at ||r|| = 1, so the inner stopping test is
        // (r,r) <= inner_rtol^2 for every instance; outer-converged instances
        // enter with r = 0 and sit out.
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
        const float itol2 = (float)(A.inner_rtol * A.inner_rtol);
        float gam_prev = 1.0f, alpha_prev = 1.0f;
        bool iconv = !me;
        int k = 0;
        for (;;) {
            float u[L::R], w[L::R];
#pragma unroll
            for (int i = 0; i < L::R; ++i) {
                u[i] = dinv[i] * r[i];
                w[i] = 0.0f;
                if (row_ok<L>(z, i)) pg[cell_of<L>(z, i)] = u[i];
            }
            __syncthreads();
            if (z.act) strip_apply<L, L::R>(SR, pg, z, u, w);
            float g3[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < L::R; ++i) {
                g3[0] += r[i] * u[i];
                g3[1] += w[i] * u[i];
                g3[2] += r[i] * r[i];
            }
            rf3.sum(g3, z.w0, L::WPI);
            if (!iconv && g3[2] <= itol2) iconv = true;
            bool go;
            if constexpr (L::IPP == 1) {
                go = !iconv;
            } else {
                go = false;
                for (int q = 0; q < L::IPP && q < cnt; ++q) go |= rf3.last_of(q, L::WPI) > itol2;
            }
            if (!go || k >= A.max_iter) break;
            if (!iconv) {
                const float beta = (k == 0) ? 0.0f : g3[0] * __builtin_amdgcn_rcpf(gam_prev);
                const float den = (k == 0) ? g3[1] : g3[1] - beta * g3[0] * __builtin_amdgcn_rcpf(alpha_prev);
                const float alpha = g3[0] * __builtin_amdgcn_rcpf(den);
#pragma unroll
                for (int i = 0; i < L::R; ++i) {
                    p[i] = u[i] + beta * p[i];
                    sv[i] = w[i] + beta * sv[i];
                    d[i] += alpha * p[i];
                    r[i] -= alpha * sv[i];
                }
                gam_prev = g3[0];
                alpha_prev = alpha;
                ++iters;
            }
            ++k;
        }
        // x += ||r|| d;  r64 -= ||r|| S d  (FP64 stencil, d exact in FP64)
        const double sc = me ? rn : 0.0;
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            x[i] += sc * (double)d[i];
            if (row_ok<L>(z, i)) pg[cell_of<L>(z, i)] = d[i];
        }
        __syncthreads();
        double sd[L::R];
#pragma unroll
        for (int i = 0; i < L::R; ++i) sd[i] = 0.0;
        if (z.act) strip_apply<L, 3>(S64, pg, z, d, sd);
        double a1[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < L::R; ++i) {
            r64[i] -= sc * sd[i];
            a1[2] += r64[i] * r64[i];
        }
        red3.sum(a1, z.w0, L::WPI);
        ++sweeps;
        rr = a1[2];
        if (!conv && rr <= tol2) conv = true;
    }
    pack_store<L>(A, z, x, iters, sweeps, conv, red1);
}

// MODE: 1 FP64, 2 refine.  One instantiation per mesh size (LV), so each
// gets its own register allocation.
template <int MODE, class L>
__global__ __launch_bounds__(NTP) void packed_kernel(MicroArgs A, PackList P) {
    extern __shared__ double lds[];
    __shared__ double r1[2][1][NWP];
    __shared__ double r3[2][3][NWP];
    __shared__ float f1[2][1][NWP];
    __shared__ float f3[2][3][NWP];
    __shared__ int task_s;
    PackRed<1, double> red1(r1);
    PackRed<3, double> red3(r3);
    PackRed<1, float> rf1(f1);
    PackRed<3, float> rf3(f3);
    int task = blockIdx.x;
    for (;;) {
        if (A.queue != nullptr) {
            if (threadIdx.x == 0) task_s = atomicAdd(A.queue, 1);
            __syncthreads();
            task = task_s;
            __syncthreads();
        }
        if (task >= P.n_packs) break;
        const int first = P.first[task], cnt = P.count[task];
        if constexpr (MODE == 2) pack_refine<L>(A, first, cnt, lds, red1, red3, rf1, rf3);
        else pack_fp64<L>(A, first, cnt, lds, red1, red3);
        if (A.queue == nullptr) break;
        __syncthreads();
    }
}

// All mesh sizes in ONE persistent launch: every workgroup pops packs from a
// work queue (packs in largest-first order) until the queue is empty; the
// register allocation is the largest of the three size paths.
template <int MODE>
__global__ __launch_bounds__(NTP) void packed_mixed_kernel(MicroArgs A, PackList P, const int32_t* pack_level) {
    extern __shared__ double lds[];
    __shared__ double r1[2][1][NWP];
    __shared__ double r3[2][3][NWP];
    __shared__ float f1[2][1][NWP];
    __shared__ float f3[2][3][NWP];
    __shared__ int task_s;
    PackRed<1, double> red1(r1);
    PackRed<3, double> red3(r3);
    PackRed<1, float> rf1(f1);
    PackRed<3, float> rf3(f3);
    for (;;) {
        if (threadIdx.x == 0) task_s = atomicAdd(A.queue, 1);
        __syncthreads();
        const int task = task_s;
        __syncthreads();
        if (task >= P.n_packs) break;
        const int lvl = pack_level[task], first = P.first[task], cnt = P.count[task];
        if constexpr (MODE == 2) {
            if (lvl == 64) pack_refine<L64>(A, first, cnt, lds, red1, red3, rf1, rf3);
            else if (lvl == 32) pack_refine<L32>(A, first, cnt, lds, red1, red3, rf1, rf3);
            else pack_refine<L16>(A, first, cnt, lds, red1, red3, rf1, rf3);
        } else {
            if (lvl == 64) pack_fp64<L64>(A, first, cnt, lds, red1, red3);
            else if (lvl == 32) pack_fp64<L32>(A, first, cnt, lds, red1, red3);
            else pack_fp64<L16>(A, first, cnt, lds, red1, red3);
        }
        __syncthreads();
    }
}

template <class L>
hipError_t launch_level(const MicroArgs& a, const PackList& p, int mode, int grid, hipStream_t s) {
    const size_t lds = sizeof(double) * L::GRID * L::IPP;
    if (mode == 2) hipLaunchKernelGGL((packed_kernel<2, L>), dim3(grid), dim3(NTP), lds, s, a, p);
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
    if (mode == 2) hipLaunchKernelGGL(packed_mixed_kernel<2>, dim3(grid), dim3(NTP), lds, s, a, p, pack_level);
    else if (mode == 1) hipLaunchKernelGGL(packed_mixed_kernel<1>, dim3(grid), dim3(NTP), lds, s, a, p, pack_level);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_packed(const MicroArgs& a, const PackList& p, int level, int mode, int grid, hipStream_t s) {
    if (p.n_packs <= 0 || grid <= 0) return hipSuccess;
    if (mode != 1 && mode != 2) return hipErrorInvalidValue;
    switch (level) {
        case 16: return launch_level<L16>(a, p, mode, grid, s);
        case 32: return launch_level<L32>(a, p, mode, grid, s);
        case 64: return launch_level<L64>(a, p, mode, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tsm
