// The stationary three-field system (Section 2.1 model) once the micro
// unknowns are eliminated.
//
// With the three micro solutions z^I = S^{-1} b_I, z^O = S^{-1} b_O and
// z^0 = S^{-1} F^v of instance k (F^v the load of f^v and g^v), the micro field is
// v_k = z^0 + k1 u_k z^I + k3 w_k z^O, and the macro rows of u and w
// (exchange integrals at the nodes with weights L_k) become, after scaling
// the u rows by k1/k2 and the w rows by k3/k4,
//   (k1/k2) (K u)_k + c_uu,k u_k + c_uw,k w_k        = (k1/k2) (F^u_k - L_k G_I,k + k2 L_k q_I,k)
//   (k3/k4) Dw (K w)_k + c_ww,k w_k + c_uw,k u_k     = (k3/k4) (F^w_k - L_k G_O,k + k4 L_k q_O,k)
//   c_uu = L (k1^2/k2) (|G^I| - k2 b_I^T z^I),  c_ww = L (k3^2/k4) (|G^O| - k4 b_O^T z^O),
//   c_uw = -L k1 k3 b_I^T z^O,  q_I = b_I^T z^0,  q_O = b_O^T z^0,
// with F^u, F^w the bulk and Neumann loads of u and w and G_I, G_O the part
// integrals of the Robin data g^v_1, g^v_2 (zero in the model; the
// manufactured form of Section 4.1 has them),
// a symmetric positive definite system (Dirichlet rows of u removed):
// its energy is the scaled energy of the whole coupled system, in which the
// exchange terms form the squares (k1/sqrt k2 u - sqrt k2 v)^2 and
// (k3/sqrt k4 w - sqrt k4 v)^2 on G^I and G^O.  K is the Q1 stiffness of
// the uniform macro mesh, applied matrix-free.  The system is small (two
// values per macro node), so one workgroup runs the whole Jacobi-PCG with
// block reductions in a fixed order; its vectors live in global memory,
// except the search direction -- the one vector read at neighbouring nodes
// -- which sits in LDS when it fits (up to kMacroLdsNodes nodes).
#include "device_common.h"

namespace tsm {

namespace {

constexpr int NT = 1024;
constexpr int NW = NT / kWave;
constexpr int kMacroLdsNodes = 9216;    // 2 x 9216 doubles = 144 KB of LDS

// (K p)_k: the rows of the Q1 element stiffness of the cells at node
// (k1, k2).  On a square cell it is 2/3 on the diagonal, -1/6 between
// corners that share an edge and -1/3 between opposite corners, whatever
// the cell size (two dimensions).
__device__ double stiff_row(const double* p, int NM, int k1, int k2) {
    const int W = NM + 1;
    double s = 0.0;
    for (int dc2 = -1; dc2 <= 0; ++dc2) {
        const int c2 = k2 + dc2;
        if (c2 < 0 || c2 >= NM) continue;
        const int l2 = k2 - c2;
        for (int dc1 = -1; dc1 <= 0; ++dc1) {
            const int c1 = k1 + dc1;
            if (c1 < 0 || c1 >= NM) continue;
            const int l1 = k1 - c1;
            for (int m2 = 0; m2 < 2; ++m2)
                for (int m1 = 0; m1 < 2; ++m1) {
                    const bool s1 = m1 == l1, s2 = m2 == l2;
                    const double e = (s1 && s2) ? 2.0 / 3.0 : ((s1 || s2) ? -1.0 / 6.0 : -1.0 / 3.0);
                    s += e * p[(c2 + m2) * W + (c1 + m1)];
                }
        }
    }
    return s;
}

__device__ int cells_at(int NM, int k1, int k2) {
    const int a = (k1 > 0) + (k1 < NM), b = (k2 > 0) + (k2 < NM);
    return a * b;
}

__device__ bool dirichlet_node(const StationaryMacroArgs& A, int k1, int k2) {
    return (A.dirichlet[0] && k2 == 0) || (A.dirichlet[1] && k2 == A.NM) || (A.dirichlet[2] && k1 == 0) ||
           (A.dirichlet[3] && k1 == A.NM);
}

template <bool LDSP>
__global__ __launch_bounds__(NT) void stationary_macro_kernel(StationaryMacroArgs A) {
    __shared__ double red_s[2][2][NW];
    __shared__ double p_s[LDSP ? 2 * kMacroLdsNodes : 1];
    BlockReducer<NW, 2, double> red(red_s);
    const int NM = A.NM, W = NM + 1, n = W * W;
    const double H = 2.0 / NM;
    const double au = A.k1 / A.k2, aw = A.k3 / A.k4;
    double* xu = A.u;
    double* xw = A.w;
    double* ru = A.work;
    double* rw = ru + n;
    double* pu = LDSP ? p_s : rw + n;
    double* pw = LDSP ? p_s + kMacroLdsNodes : rw + 2 * n;
    double* qu = rw + 3 * n;
    double* qw = qu + n;
    double* cuu = qw + n;
    double* cww = cuu + n;
    double* cuw = cww + n;
    double* bu = cuw + n;
    double* bw = bu + n;
    const double* pI = A.dots;           // b_I^T z^I
    const double* pO = A.dots + n;       // b_O^T z^O
    const double* pIO = A.dots + 2 * n;  // b_I^T z^O
    const double* qI = A.dots + 3 * n;   // b_I^T z^0
    const double* qO = A.dots + 4 * n;   // b_O^T z^0

    // coefficients, right-hand side, initial iterate (u_D on Dirichlet nodes)
    for (int k = threadIdx.x; k < n; k += NT) {
        const int k1 = k % W, k2 = k / W;
        const double L = 0.25 * H * H * cells_at(NM, k1, k2);
        cuu[k] = L * (A.k1 * A.k1 / A.k2) * (A.lenI[k] - A.k2 * pI[k]);
        cww[k] = L * (A.k3 * A.k3 / A.k4) * (A.lenO[k] - A.k4 * pO[k]);
        cuw[k] = -L * A.k1 * A.k3 * pIO[k];
        bu[k] = au * (A.Fu[k] - L * A.GI[k] + L * A.k2 * qI[k]);
        bw[k] = aw * (A.Fw[k] - L * A.GO[k] + L * A.k4 * qO[k]);
        xu[k] = dirichlet_node(A, k1, k2) ? A.uDn[k] : 0.0;
        xw[k] = 0.0;
    }
    __syncthreads();
    // r = b - A x (zero in the Dirichlet rows of u), p = D^{-1} r
    double s0[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < n; k += NT) {
        const int k1 = k % W, k2 = k / W;
        const double kd = (2.0 / 3.0) * cells_at(NM, k1, k2);
        const bool dn = dirichlet_node(A, k1, k2);
        const double r1 = dn ? 0.0 : bu[k] - (au * stiff_row(xu, NM, k1, k2) + cuu[k] * xu[k] + cuw[k] * xw[k]);
        const double r2 = bw[k] - (aw * A.Dw * stiff_row(xw, NM, k1, k2) + cww[k] * xw[k] + cuw[k] * xu[k]);
        ru[k] = r1;
        rw[k] = r2;
        pu[k] = dn ? 0.0 : r1 / (au * kd + cuu[k]);
        pw[k] = r2 / (aw * A.Dw * kd + cww[k]);
        s0[0] += r1 * pu[k] + r2 * pw[k];
        s0[1] += r1 * r1 + r2 * r2;
    }
    red.sum(s0);
    double rz = s0[0];
    const double bb = s0[1];
    double rr = bb;
    int it = 0;
    while (rr > A.rtol * A.rtol * bb && it < A.max_iter) {
        // q = A p
        double s1[2] = {0.0, 0.0};
        for (int k = threadIdx.x; k < n; k += NT) {
            const int k1 = k % W, k2 = k / W;
            const bool dn = dirichlet_node(A, k1, k2);
            const double q1 = dn ? 0.0 : au * stiff_row(pu, NM, k1, k2) + cuu[k] * pu[k] + cuw[k] * pw[k];
            const double q2 = aw * A.Dw * stiff_row(pw, NM, k1, k2) + cww[k] * pw[k] + cuw[k] * pu[k];
            qu[k] = q1;
            qw[k] = q2;
            s1[0] += pu[k] * q1 + pw[k] * q2;
        }
        red.sum(s1);
        const double alpha = rz / s1[0];
        // x += alpha p, r -= alpha q; the new r^T D^{-1} r and r^T r
        double s2[2] = {0.0, 0.0};
        for (int k = threadIdx.x; k < n; k += NT) {
            const int k1 = k % W, k2 = k / W;
            const double kd = (2.0 / 3.0) * cells_at(NM, k1, k2);
            xu[k] += alpha * pu[k];
            xw[k] += alpha * pw[k];
            const double r1 = ru[k] - alpha * qu[k];
            const double r2 = rw[k] - alpha * qw[k];
            ru[k] = r1;
            rw[k] = r2;
            s2[0] += r1 * r1 / (au * kd + cuu[k]) + r2 * r2 / (aw * A.Dw * kd + cww[k]);
            s2[1] += r1 * r1 + r2 * r2;
        }
        red.sum(s2);
        ++it;
        rr = s2[1];
        const double beta = s2[0] / rz;
        rz = s2[0];
        // p = D^{-1} r + beta p at the thread's own nodes; the barrier below
        // orders these writes before the next apply reads p at neighbours
        for (int k = threadIdx.x; k < n; k += NT) {
            const int k1 = k % W, k2 = k / W;
            const double kd = (2.0 / 3.0) * cells_at(NM, k1, k2);
            const bool dn = dirichlet_node(A, k1, k2);
            pu[k] = dn ? 0.0 : ru[k] / (au * kd + cuu[k]) + beta * pu[k];
            pw[k] = rw[k] / (aw * A.Dw * kd + cww[k]) + beta * pw[k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        A.info[0] = (double)it;
        A.info[1] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    }
}

// v_k = z^0 + k1 u_k z^I + k3 w_k z^O over every instance (z^0 may be null: zero)
__global__ void stationary_micro_kernel(int n_inst, const int64_t* offsets, const double* z0, const double* zI,
                                        const double* zO, const double* u, const double* w, double k1, double k3,
                                        double* v) {
    const int inst = blockIdx.x;
    if (inst >= n_inst) return;
    const int64_t o = offsets[inst], e = offsets[inst + 1];
    const double cu = k1 * u[inst], cw = k3 * w[inst];
    for (int64_t j = o + threadIdx.x; j < e; j += blockDim.x)
        v[j] = (z0 != nullptr ? z0[j] : 0.0) + cu * zI[j] + cw * zO[j];
}

// Q1 basis of local corner (l1, l2) at the Gauss point (g1, g2) of a cell
__device__ double basis_at(int l1, int l2, int g1, int g2) { return lin(l1, g1) * lin(l2, g2); }

// Micro loads, one workgroup per instance: node j gathers the points of its
// cells and boundary edges; the part integrals sum over edges.  The last
// workgroup assembles the macro loads.
__global__ __launch_bounds__(256) void stationary_loads_kernel(StationaryLoadArgs A) {
    __shared__ double red_s[2][2][256 / kWave];
    BlockReducer<256 / kWave, 2, double> red(red_s);
    if ((int)blockIdx.x == A.n_inst) {
        // macro loads on [-1,1]^2: int f xi_k (2x2 Gauss, weight H^2/4) and
        // the Neumann loads (2-point Gauss, weight H/2)
        const int NM = A.NM, W = NM + 1;
        const double H = 2.0 / NM;
        for (int k = threadIdx.x; k < W * W; k += blockDim.x) {
            const int k1 = k % W, k2 = k / W;
            double fu = 0.0, fw = 0.0;
            for (int dc2 = -1; dc2 <= 0; ++dc2) {
                const int c2 = k2 + dc2;
                if (c2 < 0 || c2 >= NM) continue;
                for (int dc1 = -1; dc1 <= 0; ++dc1) {
                    const int c1 = k1 + dc1;
                    if (c1 < 0 || c1 >= NM) continue;
                    for (int q = 0; q < 4; ++q) {
                        const int g1 = q & 1, g2 = q >> 1;
                        const double wphi = 0.25 * H * H * basis_at(k1 - c1, k2 - c2, g1, g2);
                        const int64_t e = (int64_t)(c2 * NM + c1) * 4 + q;
                        fu += wphi * (A.fu != nullptr ? A.fu[e] : A.fu_const);
                        fw += wphi * (A.fw != nullptr ? A.fw[e] : A.fw_const);
                    }
                }
            }
            // sides bottom (k2 = 0), top (k2 = NM) along x1; left, right along x2
            for (int side = 0; side < 4; ++side) {
                const bool horiz = side < 2;
                const int fixed = horiz ? k2 : k1, along = horiz ? k1 : k2;
                if (fixed != ((side & 1) ? NM : 0)) continue;
                for (int e = along - 1; e <= along; ++e) {
                    if (e < 0 || e >= NM) continue;
                    for (int g = 0; g < 2; ++g) {
                        const double wphi = 0.5 * H * lin(along - e, g);
                        const int64_t b = (int64_t)(side * NM + e) * 2 + g;
                        if (!A.dirichlet[side] && A.gu != nullptr) fu += wphi * A.gu[b];
                        if (A.gw != nullptr) fw += wphi * A.gw[b];
                    }
                }
            }
            A.Fu[k] = fu;
            A.Fw[k] = fw;
            A.uDn[k] = A.uD != nullptr ? A.uD[k] : A.uD_const;
        }
        return;
    }
    const int inst = blockIdx.x;
    const int N = A.level[inst], NP = N + 1;
    const int64_t off = A.offsets[inst];
    const double* wc = A.wcell + A.wc_off[inst];
    const double* wb = A.wbnd + A.wb_off[inst];
    const double* fv = A.fv != nullptr ? A.fv + A.wc_off[inst] : nullptr;
    const double* gv = A.gv != nullptr ? A.gv + A.wb_off[inst] : nullptr;
    for (int j = threadIdx.x; j < NP * NP; j += blockDim.x) {
        const int j1 = j % NP, j2 = j / NP;
        double f = 0.0;
        for (int dc2 = -1; dc2 <= 0; ++dc2) {
            const int c2 = j2 + dc2;
            if (c2 < 0 || c2 >= N) continue;
            for (int dc1 = -1; dc1 <= 0; ++dc1) {
                const int c1 = j1 + dc1;
                if (c1 < 0 || c1 >= N) continue;
                for (int q = 0; q < 4; ++q) {
                    const int64_t e = (int64_t)(c2 * N + c1) * 4 + q;
                    f += wc[e] * basis_at(j1 - c1, j2 - c2, q & 1, q >> 1) * (fv != nullptr ? fv[e] : A.fv_const);
                }
            }
        }
        if (gv != nullptr) {
            for (int side = 0; side < 4; ++side) {
                const bool horiz = side < 2;
                const int fixed = horiz ? j2 : j1, along = horiz ? j1 : j2;
                if (fixed != ((side & 1) ? N : 0)) continue;
                for (int e = along - 1; e <= along; ++e) {
                    if (e < 0 || e >= N) continue;
                    for (int g = 0; g < 2; ++g) {
                        const int64_t b = (int64_t)(side * N + e) * 2 + g;
                        f += wb[b] * lin(along - e, g) * gv[b];
                    }
                }
            }
        }
        A.Fv[off + j] = f;
    }
    double s[2] = {0.0, 0.0};     // G_I, G_O
    if (gv != nullptr) {
        for (int b = threadIdx.x; b < 8 * N; b += blockDim.x) {
            const int part = A.parts[b / (2 * N)];
            const double v = wb[b] * gv[b];
            if (part == 1) s[0] += v;
            if (part == 2) s[1] += v;
        }
    }
    red.sum(s);
    if (threadIdx.x == 0) {
        A.GI[inst] = s[0];
        A.GO[inst] = s[1];
    }
}

}  // namespace

hipError_t launch_stationary_loads(const StationaryLoadArgs& a, hipStream_t s) {
    if (a.n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(stationary_loads_kernel, dim3(a.n_inst + 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stationary_macro(const StationaryMacroArgs& a, hipStream_t s) {
    const int n = (a.NM + 1) * (a.NM + 1);
    if (n <= kMacroLdsNodes)
        hipLaunchKernelGGL(stationary_macro_kernel<true>, dim3(1), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL(stationary_macro_kernel<false>, dim3(1), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stationary_micro(int n_inst, const int64_t* offsets, const double* z0, const double* zI,
                                   const double* zO, const double* u, const double* w, double k1, double k3,
                                   double* v, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(stationary_micro_kernel, dim3(n_inst), dim3(256), 0, s, n_inst, offsets, z0, zI, zO, u, w, k1,
                       k3, v);
    return hipGetLastError();
}

}  // namespace tsm
