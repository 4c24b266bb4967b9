// Setup kernel: the pulled-back Q1 operator of every micro instance.
//
// For node j of instance i the kernel integrates, over the (at most four)
// cells around j with the 2x2 Gauss rule, the row of
//     S_i = M_i/dt + d A_i + sum over sides kappa_side B_side,   M_i = int eta eta J,
//     A_i = int grad eta . (K K^T J) grad eta
// (discrete weak form on the reference cell, paper Section 3.1) and over the
// (at most two) boundary edges at j, with the 2-point rule, the row of
//     B_side = int_side eta eta |cof(F) nu|      (boundary change of variables).
// The time-dependent system has kappa on every side; the stationary system
// has its exchange rates on the sides that form G^I and G^O and none on G^N.
// Each node gathers its own row -- no atomics, fixed summation order.
// Besides the full rows (generic kernels) it stores the upper half
// of S, of K = d A + kappa B and of M (FP32) as symmetric planes for the
// packed kernels.
// K K^T J and |cof F nu| are evaluated at each point from the amplitude a_i
// and the per-level sin/cos tables (the paper caches J and K K^T J per
// quadrature point; here they cost a few flops, so nothing is cached).
#include "device_common.h"

namespace tsm {

namespace {

// MODE 0: the sinusoidal family from the amplitude a_i.
// MODE 2: a general map given by its Jacobian F at every quadrature point
//   (the paper caches J and K K^T J per quadrature point; here the caller
//   supplies F and the same formulas give J, C and |F tau|).
template <int MODE>
__global__ __launch_bounds__(kMicroThreads) void assemble_kernel(AssembleArgs A) {
    constexpr bool TAB = MODE == 2;
    __shared__ double red_s[2][2][kMicroThreads / kWave];
    __shared__ double mins[kMicroThreads / kWave];
    BlockReducer<kMicroThreads / kWave, 2, double> red(red_s);

    const int inst = blockIdx.x;
    const int N = A.level[inst];
    const int NP = N + 1;
    const int n = NP * NP;
    const int64_t off = A.offsets[inst];
    const double a = A.amp[inst];
    const double h = 2.0 / N;
    const double wq = 0.25 * h * h;      // 2x2 Gauss weight on an h x h cell
    const double wb = 0.5 * h;           // 2-point Gauss weight on an edge of length h
    const int tb = A.tab.off[N];
    const double* ys = A.tab.y + tb;
    const double* ss = A.tab.s + tb;
    const double* cs = A.tab.c + tb;
    const int tm = 2 * N, tp = 2 * N + 1;  // table entries at y = -1, y = +1
    const double* Fc = TAB ? A.Fcell + A.cell_off[inst] : nullptr;
    const double* Fb = TAB ? A.Fbnd + A.bnd_off[inst] : nullptr;
    bool bad = false;                      // TAB: a non-finite Jacobian entry

    double len_part = 0.0, len2_part = 0.0;
    double jmin = 1e300;
    for (int j = threadIdx.x; j < n; j += kMicroThreads) {
        const int j1 = j % NP, j2 = j / NP;
        double S[kStencil], M[kStencil], K[kStencil];
#pragma unroll
        for (int k = 0; k < kStencil; ++k) { S[k] = 0.0; M[k] = 0.0; K[k] = 0.0; }
        double bj = 0.0, bj2 = 0.0;
        // ---- cells around node j
        for (int dc2 = -1; dc2 <= 0; ++dc2) {
            const int c2 = j2 + dc2;
            if (c2 < 0 || c2 >= N) continue;
            const int l2 = j2 - c2;
            for (int dc1 = -1; dc1 <= 0; ++dc1) {
                const int c1 = j1 + dc1;
                if (c1 < 0 || c1 >= N) continue;
                const int l1 = j1 - c1;
                for (int g2 = 0; g2 < 2; ++g2) {
                    const int t2 = 2 * c2 + g2;
                    for (int g1 = 0; g1 < 2; ++g1) {
                        const int t1 = 2 * c1 + g1;
                        Pull P;
                        if constexpr (TAB) {
                            const double* F = Fc + 4 * ((int64_t)(c2 * N + c1) * 4 + g2 * 2 + g1);
                            P = pull_from(F[0], F[1], F[2], F[3]);
                            bad |= !isfinite(P.J) || !isfinite(P.C11) || !isfinite(P.C12) || !isfinite(P.C22);
                        } else {
                            P = pullback_at(a, ys[t1], ys[t2], ss[t1], cs[t1], ss[t2], cs[t2]);
                        }
                        jmin = fmin(jmin, P.J);
                        // each cell's point weights are kept by its first node
                        if (A.wcell != nullptr && l1 == 0 && l2 == 0)
                            A.wcell[A.wc_off[inst] + (int64_t)(c2 * N + c1) * 4 + g2 * 2 + g1] = wq * P.J;
                        // basis of local node (l1,l2) and its reference gradient
                        const double f1 = lin(l1, g1), f2 = lin(l2, g2);
                        const double phl = f1 * f2;
                        const double gl1 = (l1 ? 1.0 : -1.0) * f2 / h;
                        const double gl2 = f1 * (l2 ? 1.0 : -1.0) / h;
                        const double Cg1 = P.C11 * gl1 + P.C12 * gl2;
                        const double Cg2 = P.C12 * gl1 + P.C22 * gl2;
#pragma unroll
                        for (int m2 = 0; m2 < 2; ++m2) {
#pragma unroll
                            for (int m1 = 0; m1 < 2; ++m1) {
                                const double e1 = lin(m1, g1), e2 = lin(m2, g2);
                                const double phm = e1 * e2;
                                const double gm1 = (m1 ? 1.0 : -1.0) * e2 / h;
                                const double gm2 = e1 * (m2 ? 1.0 : -1.0) / h;
                                const int k = (m2 - l2 + 1) * 3 + (m1 - l1 + 1);
                                const double mass = wq * P.J * phl * phm;
                                const double stiff = wq * (Cg1 * gm1 + Cg2 * gm2);
                                M[k] += mass;
                                S[k] += A.d * stiff + A.inv_dt * mass;
                                K[k] += A.d * stiff;
                            }
                        }
                    }
                }
            }
        }
        // ---- boundary edges at node j: weight |F tau|
        // bottom / top edges run along y1 (tangent (1,0)): |M e1| = sqrt(M11^2 + M21^2)
        for (int side = 0; side < 2; ++side) {
            if (j2 != (side ? N : 0)) continue;
            const int tf = side ? tp : tm;
            const double yf = ys[tf];
            for (int e = j1 - 1; e <= j1; ++e) {
                if (e < 0 || e >= N) continue;
                const int l1 = j1 - e;
                for (int g = 0; g < 2; ++g) {
                    const int t1 = 2 * e + g;
                    double M11, M21;
                    if constexpr (TAB) {
                        const double* F = Fb + 4 * ((int64_t)(side * N + e) * 2 + g);
                        M11 = F[0];
                        M21 = F[2];
                    } else {
                        M11 = 1.0 + a * cs[t1] * yf;
                        M21 = a * ss[tf];
                    }
                    double om = sqrt(M11 * M11 + M21 * M21);
                    if constexpr (TAB) bad |= !isfinite(om);
                    if (A.wbnd != nullptr && l1 == 0) A.wbnd[A.wb_off[inst] + (int64_t)(side * N + e) * 2 + g] = wb * om;
                    for (int m1 = 0; m1 < 2; ++m1) {
                        const double v = wb * om * lin(l1, g) * lin(m1, g);
                        S[3 + (m1 - l1 + 1)] += A.kside[side] * v;
                        K[3 + (m1 - l1 + 1)] += A.kside[side] * v;
                        bj += A.bw[side] * v;
                        bj2 += A.bw2[side] * v;
                    }
                }
            }
        }
        // left / right edges run along y2 (tangent (0,1)): |M e2| = sqrt(M12^2 + M22^2)
        for (int side = 0; side < 2; ++side) {
            if (j1 != (side ? N : 0)) continue;
            const int tf = side ? tp : tm;
            const double yf = ys[tf];
            for (int e = j2 - 1; e <= j2; ++e) {
                if (e < 0 || e >= N) continue;
                const int l2 = j2 - e;
                for (int g = 0; g < 2; ++g) {
                    const int t2 = 2 * e + g;
                    double M12, M22;
                    if constexpr (TAB) {
                        const double* F = Fb + 4 * ((int64_t)((2 + side) * N + e) * 2 + g);
                        M12 = F[1];
                        M22 = F[3];
                    } else {
                        M12 = a * ss[tf];
                        M22 = 1.0 + a * cs[t2] * yf;
                    }
                    double om = sqrt(M12 * M12 + M22 * M22);
                    if constexpr (TAB) bad |= !isfinite(om);
                    if (A.wbnd != nullptr && l2 == 0)
                        A.wbnd[A.wb_off[inst] + (int64_t)((2 + side) * N + e) * 2 + g] = wb * om;
                    for (int m2 = 0; m2 < 2; ++m2) {
                        const double v = wb * om * lin(l2, g) * lin(m2, g);
                        S[(m2 - l2 + 1) * 3 + 1] += A.kside[2 + side] * v;
                        K[(m2 - l2 + 1) * 3 + 1] += A.kside[2 + side] * v;
                        bj += A.bw[2 + side] * v;
                        bj2 += A.bw2[2 + side] * v;
                    }
                }
            }
        }
        double* Sd = A.S64 + kStencil * off;
        double* Md = A.M64 + kStencil * off;
#pragma unroll
        for (int k = 0; k < kStencil; ++k) {
            Sd[(int64_t)k * n + j] = S[k];
            Md[(int64_t)k * n + j] = M[k];
            const float hi = (float)S[k];
            A.S32[kStencil * off + (int64_t)k * n + j] = hi;
            A.Slo[kStencil * off + (int64_t)k * n + j] = (float)(S[k] - (double)hi);
        }
#pragma unroll
        for (int q = 0; q < kSym; ++q) {
            const int k = 4 + q;
            const int64_t e = kSym * off + (int64_t)q * n + j;
            const float hi = (float)S[k];
            A.Ss64[e] = S[k];
            A.Ks64[e] = K[k];
            A.Ss32[e] = hi;
            A.Sslo[e] = (float)(S[k] - (double)hi);
        }
        A.b[off + j] = bj;
        len_part += bj;
        if (A.b2 != nullptr) {
            A.b2[off + j] = bj2;
            len2_part += bj2;
        }
    }
    double v[2] = {len_part, len2_part};
    red.sum(v);
    double m = bad ? -1.0 : jmin;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) mins[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = mins[0];
        for (int w = 1; w < kMicroThreads / kWave; ++w) mm = fmin(mm, mins[w]);
        A.len[inst] = v[0];
        if (A.b2 != nullptr) A.len2[inst] = v[1];
        A.jmin[inst] = mm;
    }
}

}  // namespace

hipError_t launch_assemble(const AssembleArgs& a, hipStream_t s) {
    if (a.n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(assemble_kernel<0>, dim3(a.n_inst), dim3(kMicroThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_assemble_tables(const AssembleArgs& a, hipStream_t s) {
    if (a.n_inst <= 0) return hipSuccess;
    if (a.Fcell == nullptr || a.Fbnd == nullptr || a.cell_off == nullptr || a.bnd_off == nullptr)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(assemble_kernel<2>, dim3(a.n_inst), dim3(kMicroThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace tsm
