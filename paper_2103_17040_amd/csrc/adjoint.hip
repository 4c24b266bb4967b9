// Gradient contributions of the discrete adjoint (no counterpart in the
// paper: the exact derivative of the discrete time-stepping map with respect
// to the per-instance deformation amplitudes).  Matrix-free: the bilinear
// forms with the amplitude derivatives of the operators,
//     lam^T dS v = d lam^T dA v + kappa lam^T dB v + lam^T dM v / dt,
//     lam^T dM v_prev,  lam^T db,  db^T v,  b^T v,  d|dY| = 1^T db,
// are sums over the cells (2x2 Gauss points) and boundary edges (2 Gauss
// points) of the element forms, with dJ, dC and d|M tau| evaluated at each
// point from the amplitude and the per-level tables -- the same quadrature
// and formulas as the operator assembly (Section 3.1 weak form), so no
// derivative operator is stored or read: one pass reads lam0, w, v and
// v_prev.  One workgroup per instance; block sums in a fixed order.
#include "device_common.h"

namespace tsm {

namespace {

constexpr int NT = kMicroThreads;
constexpr int NW = NT / kWave;

__global__ __launch_bounds__(NT) void gradient_step_kernel(GradArgs A) {
    __shared__ double red_s[2][5][NW];
    BlockReducer<NW, 5, double> red(red_s);
    const int inst = blockIdx.x;
    const int N = A.level[inst], NP = N + 1;
    const int64_t off = A.offsets[inst];
    const double a = A.amp[inst];
    const double h = 2.0 / N, ih = 1.0 / h;
    const double wq = 0.25 * h * h;      // 2x2 Gauss weight on an h x h cell
    const double wb = 0.5 * h;           // 2-point Gauss weight on an edge of length h
    const int tb = A.tab.off[N];
    const double* ys = A.tab.y + tb;
    const double* ss = A.tab.s + tb;
    const double* cs = A.tab.c + tb;
    const double cf = A.coef[inst];
    const double* lam0 = A.lam0 + off;
    const double* w = A.w + off;
    const double* vn = A.v_now + off;
    const double* vp = A.v_prev + off;
    // t[0]: lam^T (d dA + kappa dB) v + lam^T dM (v - v_prev) / dt
    // t[1]: lam^T db   t[2]: db^T v   t[3]: b^T v   t[4]: 1^T db
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double stiff = 0.0, mass = 0.0;
    for (int c = threadIdx.x; c < N * N; c += NT) {
        const int c1 = c % N, c2 = c / N;
        const int j00 = c2 * NP + c1;
        // nodal values, local node (l1, l2) at index l2 * 2 + l1
        double L[4], V[4], D[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j00 + (q >> 1) * NP + (q & 1);
            L[q] = lam0[j] + cf * w[j];
            V[q] = vn[j];
            D[q] = vn[j] - vp[j];
        }
#pragma unroll
        for (int g2 = 0; g2 < 2; ++g2) {
            const int t2 = 2 * c2 + g2;
#pragma unroll
            for (int g1 = 0; g1 < 2; ++g1) {
                const int t1 = 2 * c1 + g1;
                const Pull P = pullback_da_at(a, ys[t1], ys[t2], ss[t1], cs[t1], ss[t2], cs[t2]);
                double lv = 0.0, dv = 0.0, l1 = 0.0, l2 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m1 = q & 1, m2 = q >> 1;
                    const double e1 = lin(m1, g1), e2 = lin(m2, g2);
                    const double ph = e1 * e2;
                    const double d1 = (m1 ? ih : -ih) * e2, d2 = e1 * (m2 ? ih : -ih);
                    lv += ph * L[q];
                    dv += ph * D[q];
                    l1 += d1 * L[q];
                    l2 += d2 * L[q];
                    v1 += d1 * V[q];
                    v2 += d2 * V[q];
                }
                stiff += wq * (l1 * (P.C11 * v1 + P.C12 * v2) + l2 * (P.C12 * v1 + P.C22 * v2));
                mass += wq * P.J * lv * dv;
            }
        }
    }
    t[0] = A.d * stiff + A.inv_dt * mass;
    // boundary edges: bottom, top (along y1), left, right (along y2)
    for (int e = threadIdx.x; e < 4 * N; e += NT) {
        const int side = e / N, k = e % N;
        const bool horiz = side < 2;
        const int tf = (side & 1) ? 2 * N + 1 : 2 * N;   // table entry of y = +1 or -1
        const double yf = ys[tf];
        int ja, jb;
        if (horiz) {
            ja = ((side & 1) ? N * NP : 0) + k;
            jb = ja + 1;
        } else {
            ja = k * NP + ((side & 1) ? N : 0);
            jb = ja + NP;
        }
        const double La = lam0[ja] + cf * w[ja], Lb = lam0[jb] + cf * w[jb];
        const double Va = vn[ja], Vb = vn[jb];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int tt = 2 * k + g;
            double om, dom;
            if (horiz) {
                const double M11 = 1.0 + a * cs[tt] * yf, M21 = a * ss[tf];
                om = sqrt(M11 * M11 + M21 * M21);
                dom = (M11 * cs[tt] * yf + M21 * ss[tf]) / om;
            } else {
                const double M12 = a * ss[tf], M22 = 1.0 + a * cs[tt] * yf;
                om = sqrt(M12 * M12 + M22 * M22);
                dom = (M12 * ss[tf] + M22 * cs[tt] * yf) / om;
            }
            const double pa = lin(0, g), pb = lin(1, g);
            const double lg = pa * La + pb * Lb, vg = pa * Va + pb * Vb;
            t[0] += A.kappa * wb * dom * lg * vg;
            t[1] += wb * dom * lg;
            t[2] += wb * dom * vg;
            t[3] += wb * om * vg;
            t[4] += wb * dom;
        }
    }
    red.sum(t);
    if (threadIdx.x == 0) {
        const int k1 = inst % (A.NM + 1), k2 = inst / (A.NM + 1);
        const bool interior = k1 > 0 && k2 > 0 && k1 < A.NM && k2 < A.NM;
        const double Lw = interior ? 1.0 / ((double)A.NM * A.NM) : 0.0;
        const double ln = A.len[inst];
        const double dF = -A.kappa * (t[2] / ln - t[3] * t[4] / (ln * ln));
        const double dR = t[0] - A.kappa * A.p * A.u_now[inst] * t[1];
        A.g[inst] -= dR - A.sign * A.mu[inst] * Lw * dF;
    }
}

}  // namespace

hipError_t launch_gradient_step(const GradArgs& a, hipStream_t s) {
    if (a.n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(gradient_step_kernel, dim3(a.n_inst), dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace tsm
