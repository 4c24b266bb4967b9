// Refinement of the micro meshes from an error indicator (an extension the
// paper's conclusions propose: an indicator over all micro grids driving
// the refinement of the reference mesh).
//
// Indicator of instance i (gradient-jump form, the estimator deal.II
// provides): the jump of the pulled-back flux d (C grad_z v) . nu across
// every interior edge of the reference mesh, squared, integrated along the
// edge with the 2-point rule and weighted by h/12:
//     eta_i^2 = sum_e (h/12) int_e [[ d (C grad_z v_i) . nu_e ]]^2 ds.
// The tangential derivative of a Q1 field is continuous, so across a line
// z1 = const the jump is C11 [[d_z1 v]] and across z2 = const C22 [[d_z2 v]];
// C = K K^T J at the edge's points (Section 3.1), from the amplitude.
// Refinement doubles the cells per side of an instance; its field is carried
// to the nested mesh by Q1 interpolation.
#include "device_common.h"

namespace tsm {

namespace {

constexpr int NT = 256;

constexpr int kCoords = 3 * kMaxLevel + 1;   // N+1 node and 2N Gauss coordinates of a side

// one workgroup per instance; the micro state v = v0 + u w is formed once
// into LDS, and sin/cos of every node and Gauss coordinate of the mesh
// (the only points the indicator visits) are tabulated there too
__global__ __launch_bounds__(NT) void indicator_kernel(IndicatorArgs A) {
    __shared__ double red_s[2][1][NT / kWave];
    __shared__ double vs[(kMaxLevel + 1) * (kMaxLevel + 1)];
    __shared__ double ycoord[kCoords], ysin[kCoords], ycos[kCoords];
    BlockReducer<NT / kWave, 1, double> red(red_s);
    const int inst = blockIdx.x;
    const int N = A.level[inst], NP = N + 1;
    const int64_t off = A.offsets[inst];
    const double a = A.amp[inst], u = A.u[inst];
    const double* v0 = A.v0 + off;
    const double* w = A.w + off;
    const double h = 2.0 / N;
    for (int j = threadIdx.x; j < NP * NP; j += NT) vs[j] = v0[j] + u * w[j];
    // coordinate k: node k (k <= N), or Gauss point g of cell c at N + 1 + 2c + g
    for (int k = threadIdx.x; k < 3 * N + 1; k += NT) {
        const double y = k <= N ? -1.0 + k * h : -1.0 + (((k - NP) >> 1) + gauss_x((k - NP) & 1)) * h;
        double s, c;
        sincospi(y, &s, &c);
        ycoord[k] = y;
        ysin[k] = 0.25 * s;
        ycos[k] = 0.25 * M_PI * c;
    }
    __syncthreads();
    auto V = [&](int j1, int j2) { return vs[j2 * NP + j1]; };
    // C at (node coordinate kn along one axis, Gauss coordinate kg along the other)
    auto pull = [&](int k1, int k2) {
        return pullback_at(a, ycoord[k1], ycoord[k2], ysin[k1], ycos[k1], ysin[k2], ycos[k2]);
    };
    // work items: direction x interior line (1..N-1) x segment (0..N-1) x point
    const int lines = N - 1;
    const int n_items = 2 * lines * N * 2;
    double s = 0.0;
    for (int t = threadIdx.x; t < n_items; t += NT) {
        const int g = t & 1;
        const int seg = (t >> 1) % N;
        const int line = ((t >> 1) / N) % lines + 1;
        const int dir = (t >> 1) / (N * lines);
        const double gx = gauss_x(g);
        double jump;
        if (dir == 0) {
            // line z1 = -1 + line h between the cells (line-1, seg) and (line, seg)
            const int j1 = line, c2 = seg;
            const double left =
                ((V(j1, c2) - V(j1 - 1, c2)) * (1 - gx) + (V(j1, c2 + 1) - V(j1 - 1, c2 + 1)) * gx) / h;
            const double right =
                ((V(j1 + 1, c2) - V(j1, c2)) * (1 - gx) + (V(j1 + 1, c2 + 1) - V(j1, c2 + 1)) * gx) / h;
            const Pull P = pull(j1, NP + 2 * c2 + g);
            jump = A.d * P.C11 * (right - left);
        } else {
            // line z2 = -1 + line h between the cells (seg, line-1) and (seg, line)
            const int j2 = line, c1 = seg;
            const double below =
                ((V(c1, j2) - V(c1, j2 - 1)) * (1 - gx) + (V(c1 + 1, j2) - V(c1 + 1, j2 - 1)) * gx) / h;
            const double above =
                ((V(c1, j2 + 1) - V(c1, j2)) * (1 - gx) + (V(c1 + 1, j2 + 1) - V(c1 + 1, j2)) * gx) / h;
            const Pull P = pull(NP + 2 * c1 + g, j2);
            jump = A.d * P.C22 * (above - below);
        }
        s += (h / 12.0) * 0.5 * h * jump * jump;
    }
    double v[1] = {s};
    red.sum(v);
    if (threadIdx.x == 0) A.eta2[inst] = v[0];
}

// Nested Q1 interpolation: a fine node is a coarse corner, the midpoint of
// a coarse edge or the centre of a coarse cell (mean of 1, 2 or 4 values);
// instances whose mesh is kept are copied.
__global__ __launch_bounds__(NT) void prolong_kernel(int n_inst, const int32_t* lo, const int32_t* ln,
                                                     const int64_t* oo, const int64_t* on, const double* vo,
                                                     double* vn) {
    const int inst = blockIdx.x;
    if (inst >= n_inst) return;
    const int No = lo[inst], Nn = ln[inst];
    const int NPo = No + 1, NPn = Nn + 1;
    const double* src = vo + oo[inst];
    double* dst = vn + on[inst];
    for (int j = threadIdx.x; j < NPn * NPn; j += NT) {
        if (Nn == No) {
            dst[j] = src[j];
            continue;
        }
        const int i1 = j % NPn, i2 = j / NPn;
        const int a1 = i1 >> 1, b1 = i1 & 1, a2 = i2 >> 1, b2 = i2 & 1;
        double s = 0.0;
        for (int q2 = 0; q2 <= b2; ++q2)
            for (int q1 = 0; q1 <= b1; ++q1) s += src[(a2 + q2) * NPo + a1 + q1];
        dst[j] = s / ((b1 + 1) * (b2 + 1));
    }
}

}  // namespace

hipError_t launch_indicator(const IndicatorArgs& a, hipStream_t s) {
    if (a.n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(indicator_kernel, dim3(a.n_inst), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prolong(int n_inst, const int32_t* lo, const int32_t* ln, const int64_t* oo, const int64_t* on,
                          const double* vo, double* vn, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(prolong_kernel, dim3(n_inst), dim3(NT), 0, s, n_inst, lo, ln, oo, on, vo, vn);
    return hipGetLastError();
}

}  // namespace tsm
