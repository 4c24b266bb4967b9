// Batched micro solves: Jacobi-preconditioned conjugate gradients on every
// instance's S_i = M_i/dt + d A_i + kappa B_i (paper Section 3.5: every system
// solved by CG, the micro systems distributed over the processors).
//
// Layout and mapping (one workgroup of 256 lanes per instance):
//   - lane t owns nodes j = t + 256 s for s < SLOTS; its x, r, diag^{-1}
//     stay in registers for the whole solve;
//   - the search direction lives in LDS with N+2 zero entries on both sides,
//     so the 9-point neighbour reads of the boundary rows stay in bounds and
//     read zeros where the stencil coefficient is zero anyway;
//   - the stencil row (9 coefficients, coefficient-major in HBM so that a
//     wavefront reads it coalesced) is either held in registers across all
//     iterations (resident forms) or re-read every iteration (streamed forms,
//     for meshes whose rows do not fit in registers);
//   - dot products: butterfly wavefront sums, then one LDS exchange per call
//     (ping-pong buffer, one barrier per reduction), identical on all lanes,
//     so every lane takes the same convergence decision.
//
// Precision forms:
//   FP64      PCG in FP64 until ||b - S x||_2 <= rtol ||b||_2.
//   REFINE    FP64 residual r = b - S x (FP64 stencil), FP32 PCG on
//             S d = r / ||r|| to its own tolerance (inner_tol2) with the FP32
//             stencil, x += ||r|| d,
//             repeated until the FP64 residual meets rtol.
#include "device_common.h"

namespace tsm {

namespace {

constexpr int NT = kMicroThreads;
constexpr int NW = NT / kWave;

struct Geo {
    int n, NP, PAD;
    int64_t off;
    int dj[kStencil];
};

__device__ __forceinline__ Geo instance_geo(const MicroArgs& A, int inst) {
    Geo g;
    const int N = A.level[inst];
    g.NP = N + 1;
    g.n = g.NP * g.NP;
    g.PAD = g.NP + 1;
    g.off = A.offsets[inst];
#pragma unroll
    for (int k = 0; k < kStencil; ++k) g.dj[k] = (k / 3 - 1) * g.NP + (k % 3 - 1);
    return g;
}

// x0 into registers and LDS; right-hand side b.
template <int SLOTS>
__device__ __forceinline__ void load_initial(const MicroArgs& A, int inst, const Geo& g,
                                             double* xs, double (&x)[SLOTS], double (&b)[SLOTS]) {
    const int tid = threadIdx.x;
    for (int t = tid; t < g.PAD; t += NT) {
        xs[t] = 0.0;
        xs[g.PAD + g.n + t] = 0.0;
    }
    const double cf = (A.coef != nullptr) ? A.coef[inst] : 0.0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = tid + s * NT;
        double v = 0.0;
        if (j < g.n && !A.zero_init) v = A.X0[g.off + j] + cf * A.w[g.off + j];
        x[s] = v;
        if (j < g.n) xs[g.PAD + j] = v;
    }
    __syncthreads();
    const double* __restrict__ Mm = A.M64 + kStencil * g.off;
    const double bc = (A.rhs_vec != nullptr && A.rhs_bcoef != nullptr) ? A.rhs_bscale * A.rhs_bcoef[inst] : 0.0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = tid + s * NT;
        double v = 0.0;
        if (j < g.n) {
            if (A.rhs_vec != nullptr) {
                v = A.rhs_scale * A.rhs_vec[g.off + j];
                if (A.rhs_bcoef != nullptr) v += bc * A.b[g.off + j];
            } else {
                double m = 0.0;
#pragma unroll
                for (int k = 0; k < kStencil; ++k) m += Mm[(int64_t)k * g.n + j] * xs[g.PAD + j + g.dj[k]];
                v = m * A.inv_dt;
            }
        }
        b[s] = v;
    }
}

template <int SLOTS>
__device__ __forceinline__ void write_result(const MicroArgs& A, int inst, const Geo& g,
                                             const double (&x)[SLOTS], int iters, int sweeps, bool conv,
                                             double rr, BlockReducer<NW, 1, double>& red1) {
    const int tid = threadIdx.x;
    double bx[1] = {0.0};
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = tid + s * NT;
        if (j < g.n) {
            A.X_out[g.off + j] = x[s];
            bx[0] += A.b[g.off + j] * x[s];
        }
    }
    red1.sum(bx);
    if (tid == 0) {
        A.bx_out[inst] = bx[0];
        if (A.iters_out) A.iters_out[inst] = iters;
        if (A.sweeps_out) A.sweeps_out[inst] = sweeps;
        if (A.res_out) A.res_out[inst] = sqrt(rr);
        if (!conv) atomicAdd(A.nonconv, 1);
    }
}

// ---------------------------------------------------------------- FP64 PCG
template <int SLOTS, bool RES>
__device__ void solve_fp64(const MicroArgs& A, int inst, double* xs,
                           BlockReducer<NW, 1, double>& red1, BlockReducer<NW, 3, double>& red3) {
    const Geo g = instance_geo(A, inst);
    const int tid = threadIdx.x;
    const double* __restrict__ S = A.S64 + kStencil * g.off;
    double x[SLOTS], b[SLOTS], r[SLOTS], dinv[SLOTS], p[SLOTS];
    double Sr[RES ? SLOTS : 1][kStencil];
    load_initial<SLOTS>(A, inst, g, xs, x, b);

    double acc[3] = {0.0, 0.0, 0.0};   // ||b||^2, ||r||^2, r.z
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = tid + s * NT;
        r[s] = 0.0; dinv[s] = 0.0;
        if (j < g.n) {
            double sx = 0.0;
#pragma unroll
            for (int k = 0; k < kStencil; ++k) {
                const double c = S[(int64_t)k * g.n + j];
                if constexpr (RES) Sr[s][k] = c;
                sx += c * xs[g.PAD + j + g.dj[k]];
            }
            r[s] = b[s] - sx;
            dinv[s] = 1.0 / S[4 * (int64_t)g.n + j];
            acc[0] += b[s] * b[s];
            acc[1] += r[s] * r[s];
            acc[2] += r[s] * dinv[s] * r[s];
        } else if constexpr (RES) {
#pragma unroll
            for (int k = 0; k < kStencil; ++k) Sr[s][k] = 0.0;
        }
        p[s] = dinv[s] * r[s];
    }
    red3.sum(acc);
    const double tol2 = A.rtol * A.rtol * acc[0];
    double rr = acc[1], rz = acc[2];
    bool conv = rr <= tol2;
    int it = 0;
    while (!conv && it < A.max_iter) {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int j = tid + s * NT;
            if (j < g.n) xs[g.PAD + j] = p[s];
        }
        __syncthreads();
        double q[SLOTS];
        double pq[1] = {0.0};
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int j = tid + s * NT;
            double t = 0.0;
            if (j < g.n) {
#pragma unroll
                for (int k = 0; k < kStencil; ++k) {
                    const double c = RES ? Sr[s][k] : S[(int64_t)k * g.n + j];
                    t += c * xs[g.PAD + j + g.dj[k]];
                }
            }
            q[s] = t;
            pq[0] += p[s] * t;
        }
        red1.sum(pq);
        const double alpha = rz / pq[0];
        double a2[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            x[s] += alpha * p[s];
            r[s] -= alpha * q[s];
            a2[0] += r[s] * dinv[s] * r[s];
            a2[1] += r[s] * r[s];
        }
        red3.sum(a2);
        ++it;
        rr = a2[1];
        if (rr <= tol2) { conv = true; break; }
        const double beta = a2[0] / rz;
        rz = a2[0];
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) p[s] = dinv[s] * r[s] + beta * p[s];
    }
    write_result<SLOTS>(A, inst, g, x, it, 1, conv, rr, red1);
}

// ------------------------------------------- FP32 PCG inside FP64 refinement
template <int SLOTS, bool RES>
__device__ void solve_refine(const MicroArgs& A, int inst, double* xs, float* ps,
                             BlockReducer<NW, 1, double>& red1, BlockReducer<NW, 3, double>& red3,
                             BlockReducer<NW, 1, float>& rf1, BlockReducer<NW, 2, float>& rf2) {
    const Geo g = instance_geo(A, inst);
    const int tid = threadIdx.x;
    const double* __restrict__ S = A.S64 + kStencil * g.off;
    const float* __restrict__ Sf = A.S32 + kStencil * g.off;
    double x[SLOTS], b[SLOTS];
    float dinv[SLOTS];
    float Sr[RES ? SLOTS : 1][kStencil];
    for (int t = tid; t < g.PAD; t += NT) {
        ps[t] = 0.0f;
        ps[g.PAD + g.n + t] = 0.0f;
    }
    load_initial<SLOTS>(A, inst, g, xs, x, b);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int j = tid + s * NT;
        dinv[s] = 0.0f;
        if (j < g.n) {
            if constexpr (RES) {
#pragma unroll
                for (int k = 0; k < kStencil; ++k) Sr[s][k] = Sf[(int64_t)k * g.n + j];
            }
            dinv[s] = 1.0f / Sf[4 * (int64_t)g.n + j];
        } else if constexpr (RES) {
#pragma unroll
            for (int k = 0; k < kStencil; ++k) Sr[s][k] = 0.0f;
        }
    }
    double bn2 = 0.0, rr_last = 0.0;
    int sweeps = 0, iters = 0;
    bool conv = false;
    for (;;) {
        if (sweeps > 0) {
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int j = tid + s * NT;
                if (j < g.n) xs[g.PAD + j] = x[s];
            }
            __syncthreads();
        }
        // FP64 residual
        double r64[SLOTS];
        double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int j = tid + s * NT;
            double t = 0.0;
            if (j < g.n) {
                double sx = 0.0;
#pragma unroll
                for (int k = 0; k < kStencil; ++k) sx += S[(int64_t)k * g.n + j] * xs[g.PAD + j + g.dj[k]];
                t = b[s] - sx;
            }
            r64[s] = t;
            acc[0] += b[s] * b[s];
            acc[1] += t * t;
        }
        red3.sum(acc);
        if (sweeps == 0) bn2 = acc[0];
        ++sweeps;
        rr_last = acc[1];
        if (acc[1] <= A.rtol * A.rtol * bn2) { conv = true; break; }
        if (sweeps > A.max_refine) break;
        // inner FP32 solve of S d = r / ||r||, zero initial guess
        const double rn = sqrt(acc[1]);
        const double isc = 1.0 / rn;
        float r[SLOTS], d[SLOTS], p[SLOTS];
        float f2[2] = {0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            r[s] = (float)(r64[s] * isc);
            d[s] = 0.0f;
            p[s] = dinv[s] * r[s];
            f2[0] += r[s] * p[s];
            f2[1] += r[s] * r[s];
        }
        rf2.sum(f2);
        float rz = f2[0];
        const float itol2 = inner_tol2(A.rtol * A.rtol * bn2, acc[1], A.inner_rtol) * f2[1];
        int it = 0;
        for (;;) {
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int j = tid + s * NT;
                if (j < g.n) ps[g.PAD + j] = p[s];
            }
            __syncthreads();
            float q[SLOTS];
            float pq[1] = {0.0f};
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int j = tid + s * NT;
                float t = 0.0f;
                if (j < g.n) {
#pragma unroll
                    for (int k = 0; k < kStencil; ++k) {
                        const float c = RES ? Sr[s][k] : Sf[(int64_t)k * g.n + j];
                        t += c * ps[g.PAD + j + g.dj[k]];
                    }
                }
                q[s] = t;
                pq[0] += p[s] * t;
            }
            rf1.sum(pq);
            const float alpha = rz / pq[0];
            float a2[2] = {0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                d[s] += alpha * p[s];
                r[s] -= alpha * q[s];
                a2[0] += r[s] * dinv[s] * r[s];
                a2[1] += r[s] * r[s];
            }
            rf2.sum(a2);
            ++it;
            if (a2[1] <= itol2 || it >= A.max_iter) break;
            const float beta = a2[0] / rz;
            rz = a2[0];
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) p[s] = dinv[s] * r[s] + beta * p[s];
        }
        iters += it;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) x[s] += rn * (double)d[s];
    }
    write_result<SLOTS>(A, inst, g, x, iters, sweeps, conv, rr_last, red1);
}

// MODE: 0 FP64 resident stencil, 1 FP64 streamed, 2 refine resident, 3 refine streamed
template <int SLOTS, int MODE>
__global__ __launch_bounds__(NT) void micro_kernel(MicroArgs A, int max_n_pad) {
    extern __shared__ double lds[];
    __shared__ double r1[2][1][NW];
    __shared__ double r3[2][3][NW];
    __shared__ float f1[2][1][NW];
    __shared__ float f2[2][2][NW];
    __shared__ int task_s;
    BlockReducer<NW, 1, double> red1(r1);
    BlockReducer<NW, 3, double> red3(r3);
    BlockReducer<NW, 1, float> rf1(f1);
    BlockReducer<NW, 2, float> rf2(f2);
    double* xs = lds;
    float* ps = reinterpret_cast<float*>(lds + max_n_pad);

    int task = blockIdx.x;
    for (;;) {
        if (A.queue != nullptr) {
            if (threadIdx.x == 0) task_s = atomicAdd(A.queue, 1);
            __syncthreads();
            task = task_s;
            __syncthreads();
        }
        if (task >= A.n_tasks) break;
        const int inst = A.order[task];
        if constexpr (MODE == 0) solve_fp64<SLOTS, true>(A, inst, xs, red1, red3);
        if constexpr (MODE == 1) solve_fp64<SLOTS, false>(A, inst, xs, red1, red3);
        if constexpr (MODE == 2) solve_refine<SLOTS, true>(A, inst, xs, ps, red1, red3, rf1, rf2);
        if constexpr (MODE == 3) solve_refine<SLOTS, false>(A, inst, xs, ps, red1, red3, rf1, rf2);
        if (A.queue == nullptr) break;
    }
}

template <int SLOTS, int MODE>
hipError_t launch_one(const MicroArgs& a, int grid, size_t lds, hipStream_t s) {
    const int max_n_pad = (int)(lds / (sizeof(double) + sizeof(float)));
    hipLaunchKernelGGL((micro_kernel<SLOTS, MODE>), dim3(grid), dim3(NT), lds, s, a, max_n_pad);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(const MicroArgs& a, int slots, int grid, size_t lds, hipStream_t s) {
    switch (slots) {
        case 1: return launch_one<1, MODE>(a, grid, lds, s);
        case 2: return launch_one<2, MODE>(a, grid, lds, s);
        case 3: return launch_one<3, MODE>(a, grid, lds, s);
        case 5: return launch_one<5, MODE>(a, grid, lds, s);
        case 9: return launch_one<9, MODE>(a, grid, lds, s);
        case 17:
            if constexpr (MODE == 1 || MODE == 3) return launch_one<17, MODE>(a, grid, lds, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------- meshes above 64 cells
// Reference meshes finer than the register- and LDS-resident kernels hold
// (64 < N <= 256, up to 66049 nodes): one 1024-lane workgroup per instance,
// every vector in global memory -- x in X_out, the residual r, the search
// direction p and the product q = S p in a workspace at the instance's
// ragged offset (ws, ws + ws_stride, ws + 2 ws_stride) -- and the full FP64
// rows streamed every iteration.  FP64 Jacobi-PCG to rtol in either
// precision mode; the starting point and right-hand side are those of the
// generic kernels (x0 = X0 + coef w, b = M x0 / dt or the given
// right-hand side).  A node reads its neighbours at indices clamped into the
// instance: the coefficient of a missing neighbour is zero.
constexpr int NTL = 1024;
constexpr int NWL = NTL / kWave;

// FP64 Jacobi PCG of one instance by the whole workgroup, vectors r, p, q
// given (instance-sized).
__device__ void pcg_fp64_instance(const MicroArgs& A, int inst, double* r, double* p, double* q,
                                  BlockReducer<NWL, 1, double>& red1, BlockReducer<NWL, 3, double>& red3) {
    const Geo g = instance_geo(A, inst);
    const int tid = threadIdx.x;
    const double* __restrict__ S = A.S64 + kStencil * g.off;
    const double* __restrict__ M = A.M64 + kStencil * g.off;
    double* x = A.X_out + g.off;
    auto nb = [&](int j, int k) {
        const int jj = j + g.dj[k];
        return jj < 0 ? 0 : (jj >= g.n ? g.n - 1 : jj);
    };
    // x0 (in place when X_out is X0: each node is read and written by its lane)
    const double cf = (A.coef != nullptr) ? A.coef[inst] : 0.0;
    for (int j = tid; j < g.n; j += NTL)
        x[j] = A.zero_init ? 0.0 : A.X0[g.off + j] + cf * A.w[g.off + j];
    __syncthreads();
    // b, r = b - S x0, p = D^-1 r; b^T-norm, ||r||^2, (r, D^-1 r)
    const double bc = (A.rhs_vec != nullptr && A.rhs_bcoef != nullptr) ? A.rhs_bscale * A.rhs_bcoef[inst] : 0.0;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = tid; j < g.n; j += NTL) {
        double bj;
        if (A.rhs_vec != nullptr) {
            bj = A.rhs_scale * A.rhs_vec[g.off + j];
            if (A.rhs_bcoef != nullptr) bj += bc * A.b[g.off + j];
        } else {
            double m = 0.0;
#pragma unroll
            for (int k = 0; k < kStencil; ++k) m += M[(int64_t)k * g.n + j] * x[nb(j, k)];
            bj = m * A.inv_dt;
        }
        double sx = 0.0;
#pragma unroll
        for (int k = 0; k < kStencil; ++k) sx += S[(int64_t)k * g.n + j] * x[nb(j, k)];
        const double rj = bj - sx;
        const double zj = rj / S[4 * (int64_t)g.n + j];
        r[j] = rj;
        p[j] = zj;
        acc[0] += bj * bj;
        acc[1] += rj * rj;
        acc[2] += rj * zj;
    }
    red3.sum(acc);     // (its barrier also orders the p stores before the first product)
    const double tol2 = A.rtol * A.rtol * acc[0];
    double rr = acc[1], rz = acc[2];
    bool conv = rr <= tol2;
    int it = 0;
    while (!conv && it < A.max_iter) {
        double pq[1] = {0.0};
        for (int j = tid; j < g.n; j += NTL) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < kStencil; ++k) t += S[(int64_t)k * g.n + j] * p[nb(j, k)];
            q[j] = t;
            pq[0] += p[j] * t;
        }
        red1.sum(pq);
        const double alpha = rz / pq[0];
        double a2[3] = {0.0, 0.0, 0.0};
        for (int j = tid; j < g.n; j += NTL) {
            x[j] += alpha * p[j];
            const double rj = r[j] - alpha * q[j];
            r[j] = rj;
            a2[0] += rj * rj / S[4 * (int64_t)g.n + j];
            a2[1] += rj * rj;
        }
        red3.sum(a2);
        ++it;
        rr = a2[1];
        if (rr <= tol2) { conv = true; break; }
        const double beta = a2[0] / rz;
        rz = a2[0];
        // every lane's p reads of this iteration are done (the reductions'
        // barriers): p may be overwritten
        for (int j = tid; j < g.n; j += NTL) p[j] = r[j] / S[4 * (int64_t)g.n + j] + beta * p[j];
        __syncthreads();
    }
    double bx[1] = {0.0};
    for (int j = tid; j < g.n; j += NTL) bx[0] += A.b[g.off + j] * x[j];
    red1.sum(bx);
    if (tid == 0) {
        if (A.bx_out) A.bx_out[inst] = bx[0];
        if (A.iters_out) A.iters_out[inst] = it;
        if (A.sweeps_out) A.sweeps_out[inst] = 1;
        if (A.res_out) A.res_out[inst] = sqrt(rr);
        if (!conv) atomicAdd(A.nonconv, 1);
    }
}

__global__ __launch_bounds__(NTL) void micro_large_kernel(MicroArgs A) {
    __shared__ double r1[2][1][NWL];
    __shared__ double r3[2][3][NWL];
    BlockReducer<NWL, 1, double> red1(r1);
    BlockReducer<NWL, 3, double> red3(r3);
    const int inst = A.order[blockIdx.x];
    const int64_t off = A.offsets[inst];
    pcg_fp64_instance(A, inst, A.ws + off, A.ws + A.ws_stride + off, A.ws + 2 * A.ws_stride + off, red1, red3);
}

// The FP64 recovery of the packed refinement solves: the instances the
// packed kernels listed (missed rtol after max_refine sweeps; their X0 is
// untouched) solved again from X0 in FP64, each by one workgroup with its
// own slot of the workspace.
__global__ __launch_bounds__(NTL) void micro_fallback_kernel(MicroArgs A, double* ws, int64_t slot,
                                                             int32_t* counters) {
    __shared__ double r1[2][1][NWL];
    __shared__ double r3[2][3][NWL];
    BlockReducer<NWL, 1, double> red1(r1);
    BlockReducer<NWL, 3, double> red3(r3);
    const int cnt = A.fb_list[0];
    if (blockIdx.x == 0 && threadIdx.x == 0 && cnt > 0) atomicAdd(counters + 2, cnt);
    double* r = ws + (int64_t)3 * blockIdx.x * slot;
    for (int t = blockIdx.x; t < cnt; t += gridDim.x) {
        pcg_fp64_instance(A, A.fb_list[1 + t], r, r + slot, r + 2 * slot, red1, red3);
        __syncthreads();     // every lane is done with the vectors before the next instance
    }
}

// y = S x for every instance (FP64 stencil), one workgroup per instance.
__global__ __launch_bounds__(NT) void apply_kernel(const int32_t* level, const int64_t* offsets,
                                                   const double* S64, const double* x, double* y) {
    const int inst = blockIdx.x;
    const int NP = level[inst] + 1;
    const int n = NP * NP;
    const int64_t off = offsets[inst];
    const double* S = S64 + kStencil * off;
    for (int j = threadIdx.x; j < n; j += NT) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < kStencil; ++k) {
            const int jj = j + (k / 3 - 1) * NP + (k % 3 - 1);
            const double c = S[(int64_t)k * n + j];
            if (jj >= 0 && jj < n) t += c * x[off + jj];
        }
        y[off + j] = t;
    }
}

// out_i = b_i^T x_i (one workgroup per instance, fixed summation order)
__global__ __launch_bounds__(NT) void bdot_kernel(const int64_t* offsets, const double* b, const double* x,
                                                  double* out) {
    __shared__ double red_s[2][1][NW];
    BlockReducer<NW, 1, double> red(red_s);
    const int inst = blockIdx.x;
    const int64_t off = offsets[inst], n = offsets[inst + 1] - off;
    double v[1] = {0.0};
    for (int64_t j = threadIdx.x; j < n; j += NT) v[0] += b[off + j] * x[off + j];
    red.sum(v);
    if (threadIdx.x == 0) out[inst] = v[0];
}

// b_i^T x_i over the boundary nodes only (b is the boundary load B 1, zero at
// every interior node), with b in the compact boundary order, gathered once at
// set-up, so only x is read at strided nodes: one wave per task, 4N nodes per
// N x N instance.
constexpr int kBdotWaves = 4;
__global__ __launch_bounds__(kBdotWaves * kWave) void bdot_boundary_kernel(int n_tasks, const int32_t* order,
                                                                           const int32_t* level,
                                                                           const int64_t* offsets, const double* bc,
                                                                           const double* x, double* out) {
    const int t = blockIdx.x * kBdotWaves + (int)(threadIdx.x / kWave);
    if (t >= n_tasks) return;                // whole waves leave together
    const int lane = threadIdx.x & (kWave - 1);
    const int inst = order[t];
    const int N = level[inst];
    const int64_t o = (int64_t)inst * kBndStride;
    const double* xi = x + offsets[inst];
    double v = 0.0;
    for (int k = lane; k < 4 * N; k += kWave) v += bc[o + k] * xi[bnd_node(N, k)];
    v = wave_total_last(v);
    if (lane == kWave - 1) out[inst] = v;
}

__global__ void bnd_gather_kernel(int n_inst, const int32_t* level, const int64_t* offsets, const double* b,
                                  double* bc) {
    const int inst = blockIdx.x;
    if (inst >= n_inst) return;
    const int N = level[inst];
    if (N > kMaxLevel) return;              // only the packed sizes (<= 64) use the compact copy
    for (int k = threadIdx.x; k < 4 * N; k += blockDim.x)
        bc[(int64_t)inst * kBndStride + k] = b[offsets[inst] + bnd_node(N, k)];
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// One more step of history for the extrapolated start (at most two are used).
__global__ void history_advance_kernel(int32_t* hn) {
    if (threadIdx.x == 0) hn[0] = hn[0] < 3 ? hn[0] + 1 : 3;
}

}  // namespace

hipError_t launch_micro(const MicroArgs& a, int slots, int mode, int grid, size_t lds, hipStream_t s) {
    if (a.n_tasks <= 0 || grid <= 0) return hipSuccess;
    switch (mode) {
        case 0: return launch_mode<0>(a, slots, grid, lds, s);
        case 1: return launch_mode<1>(a, slots, grid, lds, s);
        case 2: return launch_mode<2>(a, slots, grid, lds, s);
        case 3: return launch_mode<3>(a, slots, grid, lds, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_micro_large(const MicroArgs& a, hipStream_t s) {
    if (a.n_tasks <= 0) return hipSuccess;
    if (a.ws == nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL(micro_large_kernel, dim3(a.n_tasks), dim3(NTL), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_micro_fallback(const MicroArgs& a, double* ws, int64_t slot, int grid, int32_t* counters,
                                 hipStream_t s) {
    if (a.fb_list == nullptr || ws == nullptr || grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(micro_fallback_kernel, dim3(grid), dim3(NTL), 0, s, a, ws, slot, counters);
    return hipGetLastError();
}

hipError_t launch_apply(int n_inst, const int32_t* level, const int64_t* offsets,
                        const double* S64, const double* x, double* y, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(apply_kernel, dim3(n_inst), dim3(NT), 0, s, level, offsets, S64, x, y);
    return hipGetLastError();
}

hipError_t launch_bdot(int n_inst, const int64_t* offsets, const double* b, const double* x, double* out,
                       hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(bdot_kernel, dim3(n_inst), dim3(NT), 0, s, offsets, b, x, out);
    return hipGetLastError();
}

hipError_t launch_bdot_boundary(int n_tasks, const int32_t* order, const int32_t* level, const int64_t* offsets,
                                const double* bc, const double* x, double* out, hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(bdot_boundary_kernel, dim3((n_tasks + kBdotWaves - 1) / kBdotWaves), dim3(kBdotWaves * kWave),
                       0, s, n_tasks, order, level, offsets, bc, x, out);
    return hipGetLastError();
}

hipError_t launch_bnd_gather(int n_inst, const int32_t* level, const int64_t* offsets, const double* b, double* bc,
                             hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(bnd_gather_kernel, dim3(n_inst), dim3(256), 0, s, n_inst, level, offsets, b, bc);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_history_advance(int32_t* hn, hipStream_t s) {
    hipLaunchKernelGGL(history_advance_kernel, dim3(1), dim3(64), 0, s, hn);
    return hipGetLastError();
}

}  // namespace tsm
