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

// Butterfly reduction: every lane ends with the same bitwise value
// (each stage adds two operands in either order, and IEEE addition commutes).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
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

}  // namespace tsm
