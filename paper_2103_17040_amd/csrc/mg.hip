// Geometric multigrid as the preconditioner of the micro CG (Section 3.5:
// the micro systems are solved by CG; the preconditioner is this library's
// choice).  The stationary micro operator S = Dv A + k2 B^I + k4 B^O has no
// mass term, so the Jacobi-preconditioned CG needs O(N) iterations on an
// N x N reference mesh (630 at 64, 1272 at 128 cells per side); one V-cycle
// per iteration makes the count independent of N.
//
// Hierarchy of an instance with N = c 2^L cells per side (c <= kMgCoarsest,
// L >= 1): the nested vertex meshes N, N/2, ..., c of the reference cell Z,
// bilinear interpolation P between consecutive meshes, Galerkin coarse
// operators A_{l+1} = P^T A_l P (9-point again), built once per geometry;
// the coarsest operator (at most 81 unknowns) is inverted densely.  Smoother:
// nu sweeps of damped Jacobi before and after the coarse correction, damping
// omega_l = 1.6 / g_l with g_l the largest Gershgorin row ratio
// sum_k |a_jk| / a_jj of level l, so omega lambda_max(D^{-1} A) <= 1.6 < 2:
// the V-cycle is then a fixed symmetric positive definite operator, as CG
// needs.  One 1024-lane workgroup per instance; vectors in global memory
// (cached: an instance's level vectors are at most 0.5 MB).
#include "device_common.h"

namespace tsm {

namespace {

constexpr int NTM = 1024;
constexpr int NWM = NTM / kWave;

// Level l of instance (N, fine offset off, coarse offset coff): operator,
// vectors x (the correction), r (its right-hand side), t (scratch).
struct MgLevel {
    const double* S;   // 9 coefficient-major planes of n entries
    int NP, n;
    double *x, *r, *t;
    double om;
};

__device__ __forceinline__ int64_t coarse_level_offset(int N, int l) {
    int64_t o = 0;
    for (int m = 1; m < l; ++m) {
        const int64_t np = (N >> m) + 1;
        o += np * np;
    }
    return o;
}

__device__ __forceinline__ MgLevel mg_level(const MicroArgs& A, const MgArgs& G, int inst, int N, int64_t off,
                                            int l, double* z, double* r, double* t) {
    MgLevel v;
    v.NP = (N >> l) + 1;
    v.n = v.NP * v.NP;
    v.om = G.omega[(int64_t)inst * (kMgMaxLevels + 1) + l];
    if (l == 0) {
        v.S = A.S64 + kStencil * off;
        v.x = z;
        v.r = r;
        v.t = t;
    } else {
        const int64_t c = G.coff[inst] + coarse_level_offset(N, l);
        v.S = G.Ac + kStencil * c;
        v.x = G.cws + c;
        v.r = G.cws + G.cws_stride + c;
        v.t = G.cws + 2 * G.cws_stride + c;
    }
    return v;
}

// (A_l y)_j; a neighbour outside the mesh has a zero coefficient and is read
// at a clamped index
__device__ __forceinline__ double level_apply(const MgLevel& L, const double* y, int j) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kStencil; ++k) {
        int jj = j + (k / 3 - 1) * L.NP + (k % 3 - 1);
        jj = jj < 0 ? 0 : (jj >= L.n ? L.n - 1 : jj);
        s += L.S[(int64_t)k * L.n + j] * y[jj];
    }
    return s;
}

// x = omega D^{-1} r (the first sweep from a zero guess)
__device__ void smooth_first(const MgLevel& L) {
    for (int j = threadIdx.x; j < L.n; j += NTM) L.x[j] = L.om * L.r[j] / L.S[4 * (int64_t)L.n + j];
    __syncthreads();
}

// x += omega D^{-1} (r - A x)
__device__ void smooth_sweep(const MgLevel& L) {
    for (int j = threadIdx.x; j < L.n; j += NTM) L.t[j] = L.r[j] - level_apply(L, L.x, j);
    __syncthreads();
    for (int j = threadIdx.x; j < L.n; j += NTM) L.x[j] += L.om * L.t[j] / L.S[4 * (int64_t)L.n + j];
    __syncthreads();
}

// r_c = P^T (r - A x): coarse node J gathers the fine nodes within one of
// 2J, weight (1 - |d1|/2)(1 - |d2|/2)
__device__ void restrict_residual(const MgLevel& F, const MgLevel& C) {
    for (int j = threadIdx.x; j < F.n; j += NTM) F.t[j] = F.r[j] - level_apply(F, F.x, j);
    __syncthreads();
    const int Nf = F.NP - 1;
    for (int J = threadIdx.x; J < C.n; J += NTM) {
        const int J1 = J % C.NP, J2 = J / C.NP;
        double s = 0.0;
        for (int d2 = -1; d2 <= 1; ++d2) {
            const int i2 = 2 * J2 + d2;
            if (i2 < 0 || i2 > Nf) continue;
            for (int d1 = -1; d1 <= 1; ++d1) {
                const int i1 = 2 * J1 + d1;
                if (i1 < 0 || i1 > Nf) continue;
                const double w = (d1 == 0 ? 1.0 : 0.5) * (d2 == 0 ? 1.0 : 0.5);
                s += w * F.t[i2 * F.NP + i1];
            }
        }
        C.r[J] = s;
    }
    __syncthreads();
}

// x_f += P x_c (bilinear interpolation of the nested coarse mesh)
__device__ void prolong_add(const MgLevel& F, const MgLevel& C) {
    for (int j = threadIdx.x; j < F.n; j += NTM) {
        const int j1 = j % F.NP, j2 = j / F.NP;
        const int a1 = j1 >> 1, b1 = (j1 + 1) >> 1, a2 = j2 >> 1, b2 = (j2 + 1) >> 1;
        const double v = 0.25 * (C.x[a2 * C.NP + a1] + C.x[a2 * C.NP + b1] + C.x[b2 * C.NP + a1] +
                                 C.x[b2 * C.NP + b1]);
        F.x[j] += v;
    }
    __syncthreads();
}

// x_c = A_c^{-1} r_c (dense inverse, row-major)
__device__ void coarsest_solve(const MgLevel& C, const double* inv) {
    for (int i = threadIdx.x; i < C.n; i += NTM) {
        double s = 0.0;
        for (int j = 0; j < C.n; ++j) s += inv[(int64_t)i * C.n + j] * C.r[j];
        C.x[i] = s;
    }
    __syncthreads();
}

// z = V r (levels 0..L)
__device__ void vcycle(const MicroArgs& A, const MgArgs& G, int inst, int N, int64_t off, int L, double* z,
                       double* r, double* t) {
    for (int l = 0; l < L; ++l) {
        const MgLevel F = mg_level(A, G, inst, N, off, l, z, r, t);
        smooth_first(F);
        for (int s = 1; s < G.nu; ++s) smooth_sweep(F);
        restrict_residual(F, mg_level(A, G, inst, N, off, l + 1, z, r, t));
    }
    coarsest_solve(mg_level(A, G, inst, N, off, L, z, r, t), G.inv + G.ioff[inst]);
    for (int l = L - 1; l >= 0; --l) {
        const MgLevel F = mg_level(A, G, inst, N, off, l, z, r, t);
        prolong_add(F, mg_level(A, G, inst, N, off, l + 1, z, r, t));
        for (int s = 0; s < G.nu; ++s) smooth_sweep(F);
    }
}

// The micro solve with the V-cycle as preconditioner (same right-hand sides,
// initial guesses, stopping test and outputs as the other micro kernels).
__global__ __launch_bounds__(NTM) void micro_mg_kernel(MicroArgs A, MgArgs G) {
    __shared__ double r1[2][1][NWM];
    __shared__ double r3[2][3][NWM];
    BlockReducer<NWM, 1, double> red1(r1);
    BlockReducer<NWM, 3, double> red3(r3);
    const int inst = A.order[blockIdx.x];
    const int N = A.level[inst];
    const int NP = N + 1, n = NP * NP;
    const int64_t off = A.offsets[inst];
    const int L = G.nlev[inst];
    const double* __restrict__ M = A.M64 + kStencil * off;
    double* x = A.X_out + off;
    double* r = G.ws + off;
    double* z = G.ws + G.ws_stride + off;
    double* t = G.ws + 2 * G.ws_stride + off;
    double* p = G.ws + 3 * G.ws_stride + off;
    double* q = G.ws + 4 * G.ws_stride + off;
    const MgLevel L0 = mg_level(A, G, inst, N, off, 0, z, r, t);
    const double cf = (A.coef != nullptr) ? A.coef[inst] : 0.0;
    for (int j = threadIdx.x; j < n; j += NTM) x[j] = A.zero_init ? 0.0 : A.X0[off + j] + cf * A.w[off + j];
    __syncthreads();
    const double bc = (A.rhs_vec != nullptr && A.rhs_bcoef != nullptr) ? A.rhs_bscale * A.rhs_bcoef[inst] : 0.0;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < n; j += NTM) {
        double bj;
        if (A.rhs_vec != nullptr) {
            bj = A.rhs_scale * A.rhs_vec[off + j];
            if (A.rhs_bcoef != nullptr) bj += bc * A.b[off + j];
        } else {
            MgLevel Ml = L0;
            Ml.S = M;
            bj = level_apply(Ml, x, j) * A.inv_dt;
        }
        const double rj = bj - level_apply(L0, x, j);
        r[j] = rj;
        acc[0] += bj * bj;
        acc[1] += rj * rj;
    }
    red3.sum(acc);
    const double tol2 = A.rtol * A.rtol * acc[0];
    double rr = acc[1];
    bool conv = rr <= tol2;
    int it = 0;
    double rz = 0.0;
    if (!conv) {
        vcycle(A, G, inst, N, off, L, z, r, t);
        double a1[1] = {0.0};
        for (int j = threadIdx.x; j < n; j += NTM) {
            p[j] = z[j];
            a1[0] += r[j] * z[j];
        }
        red1.sum(a1);     // (its barrier orders the p stores before the first product)
        rz = a1[0];
    }
    while (!conv && it < A.max_iter) {
        double pq[1] = {0.0};
        for (int j = threadIdx.x; j < n; j += NTM) {
            const double v = level_apply(L0, p, j);
            q[j] = v;
            pq[0] += p[j] * v;
        }
        red1.sum(pq);
        const double alpha = pq[0] > 0.0 ? rz / pq[0] : 0.0;
        double a2[3] = {0.0, 0.0, 0.0};
        for (int j = threadIdx.x; j < n; j += NTM) {
            x[j] += alpha * p[j];
            const double rj = r[j] - alpha * q[j];
            r[j] = rj;
            a2[1] += rj * rj;
        }
        red3.sum(a2);
        ++it;
        rr = a2[1];
        if (rr <= tol2) {
            conv = true;
            break;
        }
        vcycle(A, G, inst, N, off, L, z, r, t);
        double a3[1] = {0.0};
        for (int j = threadIdx.x; j < n; j += NTM) a3[0] += r[j] * z[j];
        red1.sum(a3);
        const double beta = rz > 0.0 ? a3[0] / rz : 0.0;
        rz = a3[0];
        for (int j = threadIdx.x; j < n; j += NTM) p[j] = z[j] + beta * p[j];
        __syncthreads();
    }
    double bx[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += NTM) bx[0] += A.b[off + j] * x[j];
    red1.sum(bx);
    if (threadIdx.x == 0) {
        if (A.bx_out) A.bx_out[inst] = bx[0];
        if (A.iters_out) A.iters_out[inst] = it;
        if (A.sweeps_out) A.sweeps_out[inst] = 1;
        if (A.res_out) A.res_out[inst] = sqrt(rr);
        if (!conv) atomicAdd(A.nonconv, 1);
    }
}

// A_{l+1} = P^T A_l P for every instance with more than l coarse levels
// (one workgroup per instance, one lane per coarse node; a coarse
// neighbour outside the mesh gets a zero coefficient).
__global__ __launch_bounds__(256) void mg_galerkin_kernel(MicroArgs A, MgArgs G, int l) {
    const int inst = blockIdx.x;
    if (l >= G.nlev[inst]) return;
    const int N = A.level[inst];
    const int64_t off = A.offsets[inst];
    const MgLevel F = mg_level(A, G, inst, N, off, l, nullptr, nullptr, nullptr);
    const int64_t c = G.coff[inst] + coarse_level_offset(N, l + 1);
    double* Acc = G.Ac + kStencil * c;
    const int NPc = (N >> (l + 1)) + 1, nc = NPc * NPc, Nf = F.NP - 1;
    for (int J = threadIdx.x; J < nc; J += blockDim.x) {
        const int J1 = J % NPc, J2 = J / NPc;
        double out[kStencil];
#pragma unroll
        for (int k = 0; k < kStencil; ++k) out[k] = 0.0;
        for (int d2 = -1; d2 <= 1; ++d2) {
            const int i2 = 2 * J2 + d2;
            if (i2 < 0 || i2 > Nf) continue;
            for (int d1 = -1; d1 <= 1; ++d1) {
                const int i1 = 2 * J1 + d1;
                if (i1 < 0 || i1 > Nf) continue;
                const double wi = (d1 == 0 ? 1.0 : 0.5) * (d2 == 0 ? 1.0 : 0.5);
                const int i = i2 * F.NP + i1;
                for (int k = 0; k < kStencil; ++k) {
                    const int j1 = i1 + k % 3 - 1, j2 = i2 + k / 3 - 1;
                    if (j1 < 0 || j1 > Nf || j2 < 0 || j2 > Nf) continue;
                    const double a = wi * F.S[(int64_t)k * F.n + i];
                    // coarse nodes interpolating fine node j: floor and ceil of j/2
                    const int c1a = j1 >> 1, c1b = (j1 + 1) >> 1, c2a = j2 >> 1, c2b = (j2 + 1) >> 1;
                    const double w1 = c1a == c1b ? 1.0 : 0.5, w2 = c2a == c2b ? 1.0 : 0.5;
                    for (int e2 = 0; e2 < (c2a == c2b ? 1 : 2); ++e2) {
                        const int K2 = e2 ? c2b : c2a;
                        for (int e1 = 0; e1 < (c1a == c1b ? 1 : 2); ++e1) {
                            const int K1 = e1 ? c1b : c1a;
                            out[(K2 - J2 + 1) * 3 + (K1 - J1 + 1)] += a * w1 * w2;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kStencil; ++k) Acc[(int64_t)k * nc + J] = out[k];
    }
}

// omega_l = 1.6 / max_j sum_k |a_jk| / a_jj for the smoothed levels 0..L-1
__global__ __launch_bounds__(256) void mg_omega_kernel(MicroArgs A, MgArgs G) {
    __shared__ double red_s[256 / kWave];
    const int inst = blockIdx.x;
    const int L = G.nlev[inst];
    const int N = A.level[inst];
    const int64_t off = A.offsets[inst];
    for (int l = 0; l < L; ++l) {
        MgLevel F = mg_level(A, G, inst, N, off, l, nullptr, nullptr, nullptr);
        double g = 0.0;
        for (int j = threadIdx.x; j < F.n; j += blockDim.x) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < kStencil; ++k) s += fabs(F.S[(int64_t)k * F.n + j]);
            g = fmax(g, s / F.S[4 * (int64_t)F.n + j]);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o));
        if ((threadIdx.x & (kWave - 1)) == 0) red_s[threadIdx.x / kWave] = g;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = red_s[0];
            for (int w = 1; w < (int)(blockDim.x / kWave); ++w) m = fmax(m, red_s[w]);
            G.omega[(int64_t)inst * (kMgMaxLevels + 1) + l] = 1.6 / m;
        }
        __syncthreads();
    }
}

// Dense inverse of the coarsest operator (Gauss-Jordan in place, no
// pivoting: the operator is symmetric positive definite).
constexpr int kMgInvMax = (kMgCoarsest + 1) * (kMgCoarsest + 1);
__global__ __launch_bounds__(256) void mg_inverse_kernel(MicroArgs A, MgArgs G) {
    __shared__ double a[kMgInvMax * kMgInvMax];
    const int inst = blockIdx.x;
    const int L = G.nlev[inst];
    if (L <= 0) return;
    const int N = A.level[inst];
    const MgLevel C = mg_level(A, G, inst, N, A.offsets[inst], L, nullptr, nullptr, nullptr);
    const int n = C.n;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        const int d1 = j % C.NP - i % C.NP, d2 = j / C.NP - i / C.NP;
        a[e] = (d1 >= -1 && d1 <= 1 && d2 >= -1 && d2 <= 1) ? C.S[(int64_t)((d2 + 1) * 3 + d1 + 1) * n + i] : 0.0;
    }
    __syncthreads();
    constexpr int kPer = (kMgInvMax * kMgInvMax + 255) / 256;
    for (int k = 0; k < n; ++k) {
        const double piv = 1.0 / a[k * n + k];
        __syncthreads();
        // row k: a[k][j] *= piv (j != k), a[k][k] = piv
        for (int j = threadIdx.x; j < n; j += blockDim.x) a[k * n + j] = (j == k) ? piv : a[k * n + j] * piv;
        __syncthreads();
        double nv[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + q * 256;
            nv[q] = 0.0;
            if (e < n * n) {
                const int i = e / n, j = e % n;
                if (i != k) {
                    const double f = a[i * n + k];
                    nv[q] = (j == k) ? -f * a[k * n + k] : a[e] - f * a[k * n + j];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + q * 256;
            if (e < n * n && e / n != k) a[e] = nv[q];
        }
        __syncthreads();
    }
    double* out = G.inv + G.ioff[inst];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) out[e] = a[e];
}

}  // namespace

hipError_t launch_micro_mg(const MicroArgs& a, const MgArgs& g, hipStream_t s) {
    if (a.n_tasks <= 0) return hipSuccess;
    if (g.ws == nullptr || g.cws == nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL(micro_mg_kernel, dim3(a.n_tasks), dim3(NTM), 0, s, a, g);
    return hipGetLastError();
}

hipError_t launch_mg_setup(const MicroArgs& a, const MgArgs& g, int n_inst, int max_levels, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    for (int l = 0; l < max_levels; ++l) {
        hipLaunchKernelGGL(mg_galerkin_kernel, dim3(n_inst), dim3(256), 0, s, a, g, l);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mg_omega_kernel, dim3(n_inst), dim3(256), 0, s, a, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mg_inverse_kernel, dim3(n_inst), dim3(256), 0, s, a, g);
    return hipGetLastError();
}

}  // namespace tsm
