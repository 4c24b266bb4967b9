// Device helpers: wavefront/workgroup reductions and the pulled-back Q1
// quadrature of one node's stencil row.
#pragma once

#include <hip/hip_runtime.h>

#include "tsm_internal.h"

namespace tsm {

// 2-point Gauss-Legendre abscissae on [0,1]
__device__ constexpr double kGX0 = 0.21132486540518711775;   // 1/2 - 1/(2 sqrt 3)
__device__ constexpr double kGX1 = 0.78867513459481288225;   // 1/2 + 1/(2 sqrt 3)

__device__ __forceinline__ double gauss_x(int g) { return g ? kGX1 : kGX0; }
// 1D linear basis on [0,1]: local node l at abscissa g
__device__ __forceinline__ double lin(int l, int g) { return l ? gauss_x(g) : 1.0 - gauss_x(g); }

// Wavefront sum with DPP lane permutations (no LDS traffic):
//   quad_perm [1,0,3,2], quad_perm [2,3,0,1]  -> every lane holds its quad sum
//   row_half_mirror, row_mirror               -> every lane holds its 16-lane row sum
// then the four row sums are read as scalars and added in a fixed order.
// Every lane returns the same bits: each step adds two operands whose order
// differs between partner lanes only, and IEEE addition commutes.
// All 64 lanes must be active.
// DPP move of v under control CTRL; lanes without a source lane (and rows
// outside ROWMASK) read 0 (bound_ctrl), which lets v + dpp(v) become one
// v_add_f32 with a DPP operand.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, true));
}
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, ROWMASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWMASK, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float lane_read(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_read(double v, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);   // row_half_mirror
    v += dpp<0x140>(v);   // row_mirror
    return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

// Wavefront sum that ends in lane 63 only (other lanes hold partial sums):
// the four in-row steps above, then row_bcast:15 adds the sum of each row
// into the next row (row 3 gets r3 + r2) and row_bcast:31 adds lane 31
// (r1 + r0) into rows 2 and 3, so lane 63 holds (r3 + r2) + (r1 + r0).  Two
// DPP steps and no lane reads in place of the four lane reads and three adds
// of wave_sum.
template <typename T>
__device__ __forceinline__ T wave_total_last(T v) {
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    v += dpp<0x142>(v);   // row_bcast:15
    v += dpp<0x143>(v);   // row_bcast:31
    return v;
}

// Sum over aligned groups of G lanes (G = 1, 2, 4, 8 or 16) within each
// 16-lane row; every lane of a group ends with the same bits.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
    if constexpr (G > 1) v += dpp<0xB1>(v);
    if constexpr (G > 2) v += dpp<0x4E>(v);
    if constexpr (G > 4) v += dpp<0x141>(v);
    if constexpr (G > 8) v += dpp<0x140>(v);
    return v;
}

// Sum of NV values over a workgroup of NW waves.  red is a [2][NV][NW] LDS
// ping-pong buffer; consecutive calls alternate halves so one barrier per call
// suffices (the next write to a half happens after another barrier).
template <int NW, int NV, typename T>
struct BlockReducer {
    T (*red)[NV][NW];
    int phase = 0;
    __device__ BlockReducer(T (*r)[NV][NW]) : red(r) {}
    __device__ __forceinline__ void sum(T (&v)[NV]) {
        const int lane = threadIdx.x & (kWave - 1);
        const int wid = threadIdx.x / kWave;
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
        if (lane == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) red[phase][i][wid] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            T s = red[phase][i][0];
#pragma unroll
            for (int w = 1; w < NW; ++w) s += red[phase][i][w];
            v[i] = s;
        }
        phase ^= 1;
    }
};

// Geometry of the workloads' deformation at one reference point:
// M = I + a G (the rotation drops out of K K^T J and |cof(F) nu|).
struct Pull {
    double J, C11, C12, C22;
};

// J = det M and C = adj(M) adj(M)^T / J (= K K^T J with K = M^{-1}) for a
// Jacobian M; any rotation in front of M drops out of both.
__device__ __forceinline__ Pull pull_from(double M11, double M12, double M21, double M22) {
    Pull g;
    g.J = M11 * M22 - M12 * M21;
    const double iJ = 1.0 / g.J;
    g.C11 = (M22 * M22 + M12 * M12) * iJ;
    g.C12 = -(M22 * M21 + M12 * M11) * iJ;
    g.C22 = (M21 * M21 + M11 * M11) * iJ;
    return g;
}

__device__ __forceinline__ Pull pullback_at(double a, double y1, double y2,
                                            double s1, double c1, double s2, double c2) {
    const double M11 = 1.0 + a * c1 * y2;
    const double M12 = a * s1;
    const double M21 = a * s2;
    const double M22 = 1.0 + a * c2 * y1;
    Pull g;
    g.J = M11 * M22 - M12 * M21;
    const double iJ = 1.0 / g.J;
    // C = adj(M) adj(M)^T / J  ( = K K^T J with K = M^{-1} )
    g.C11 = (M22 * M22 + M12 * M12) * iJ;
    g.C12 = -(M22 * M21 + M12 * M11) * iJ;
    g.C22 = (M21 * M21 + M11 * M11) * iJ;
    return g;
}

// a-derivatives of J and C at one reference point (M = I + a G, dM/da = G)
__device__ __forceinline__ Pull pullback_da_at(double a, double y1, double y2,
                                               double s1, double c1, double s2, double c2) {
    const double G11 = c1 * y2, G12 = s1, G21 = s2, G22 = c2 * y1;
    const double M11 = 1.0 + a * G11, M12 = a * G12, M21 = a * G21, M22 = 1.0 + a * G22;
    const double J = M11 * M22 - M12 * M21;
    const double iJ = 1.0 / J;
    const double dJ = G11 * M22 + M11 * G22 - G12 * M21 - M12 * G21;
    const double C11 = (M22 * M22 + M12 * M12) * iJ;
    const double C12 = -(M22 * M21 + M12 * M11) * iJ;
    const double C22 = (M21 * M21 + M11 * M11) * iJ;
    Pull d;
    d.J = dJ;
    d.C11 = 2.0 * (M22 * G22 + M12 * G12) * iJ - C11 * dJ * iJ;
    d.C12 = -(G22 * M21 + M22 * G21 + G12 * M11 + M12 * G11) * iJ - C12 * dJ * iJ;
    d.C22 = 2.0 * (M21 * G21 + M11 * G11) * iJ - C22 * dJ * iJ;
    return d;
}

}  // namespace tsm
