// Gradient contributions of the discrete adjoint (no counterpart in the
// paper: the exact derivative of the discrete time-stepping map with respect
// to the per-instance deformation amplitudes).  One workgroup per instance;
// the amplitude-derivative stencils dS/da, dM/da and db/da come from the
// derivative assembly.  Block sums in a fixed order: deterministic.
#include "device_common.h"

namespace tsm {

namespace {

constexpr int NT = kMicroThreads;
constexpr int NW = NT / kWave;

__global__ __launch_bounds__(NT) void gradient_step_kernel(GradArgs A) {
    __shared__ double red_s[2][5][NW];
    BlockReducer<NW, 5, double> red(red_s);
    const int inst = blockIdx.x;
    const int NP = A.level[inst] + 1;
    const int n = NP * NP;
    const int64_t off = A.offsets[inst];
    const double* dS = A.dS + kStencil * off;
    const double* dM = A.dM + kStencil * off;
    const double cf = A.coef[inst];
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < n; j += NT) {
        const double lam = A.lam0[off + j] + cf * A.w[off + j];
        double sv = 0.0, mv = 0.0;
#pragma unroll
        for (int k = 0; k < kStencil; ++k) {
            const int jj = j + (k / 3 - 1) * NP + (k % 3 - 1);
            if (jj >= 0 && jj < n) {
                sv += dS[(int64_t)k * n + j] * A.v_now[off + jj];
                mv += dM[(int64_t)k * n + j] * A.v_prev[off + jj];
            }
        }
        const double dbj = A.db[off + j], vj = A.v_now[off + j];
        t[0] += lam * sv;
        t[1] += lam * dbj;
        t[2] += lam * mv;
        t[3] += dbj * vj;
        t[4] += A.b[off + j] * vj;
    }
    red.sum(t);
    if (threadIdx.x == 0) {
        const int k1 = inst % (A.NM + 1), k2 = inst / (A.NM + 1);
        const bool interior = k1 > 0 && k2 > 0 && k1 < A.NM && k2 < A.NM;
        const double L = interior ? 1.0 / ((double)A.NM * A.NM) : 0.0;
        const double ln = A.len[inst];
        const double dF = -A.kappa * (t[3] / ln - t[4] * A.dlen[inst] / (ln * ln));
        const double dR = t[0] - A.kappa * A.p * A.u_now[inst] * t[1] - t[2] * A.inv_dt;
        A.g[inst] -= dR - A.sign * A.mu[inst] * L * dF;
    }
}

}  // namespace

hipError_t launch_gradient_step(const GradArgs& a, hipStream_t s) {
    if (a.n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(gradient_step_kernel, dim3(a.n_inst), dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace tsm
