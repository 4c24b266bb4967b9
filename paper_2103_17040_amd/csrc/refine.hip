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
#include <mutex>
#include <string>

#include "device_common.h"

namespace tsm {

namespace {

constexpr int NT = 256;

constexpr int kCoords = 3 * kMaxLevel + 1;   // N+1 node and 2N Gauss coordinates of a side

// one workgroup per instance; up to kMaxLevel cells per side the micro state
// v = v0 + u w is formed once into LDS, and sin/cos of every node and Gauss
// coordinate of the mesh (the only points the indicator visits) are
// tabulated there too; larger meshes read v0 and w at every point and
// evaluate the coordinates where they are used
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
    const bool big = N > kMaxLevel;      // uniform over the workgroup
    // coordinate k: node k (k <= N), or Gauss point g of cell c at N + 1 + 2c + g
    auto coord = [&](int k, double& y, double& sn, double& cs) {
        y = k <= N ? -1.0 + k * h : -1.0 + (((k - NP) >> 1) + gauss_x((k - NP) & 1)) * h;
        double s, c;
        sincospi(y, &s, &c);
        sn = 0.25 * s;
        cs = 0.25 * M_PI * c;
    };
    if (!big) {
        for (int j = threadIdx.x; j < NP * NP; j += NT) vs[j] = v0[j] + u * w[j];
        for (int k = threadIdx.x; k < 3 * N + 1; k += NT) coord(k, ycoord[k], ysin[k], ycos[k]);
    }
    __syncthreads();
    auto V = [&](int j1, int j2) {
        const int j = j2 * NP + j1;
        return big ? v0[j] + u * w[j] : vs[j];
    };
    // C at (node coordinate kn along one axis, Gauss coordinate kg along the other)
    auto pull = [&](int k1, int k2) {
        if (big) {
            double y1, s1, c1, y2, s2, c2;
            coord(k1, y1, s1, c1);
            coord(k2, y2, s2, c2);
            return pullback_at(a, y1, y2, s1, c1, s2, c2);
        }
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

// ---------------------------------------------------------------------------
// Interpolation without device allocation (tsm_prolong_noalloc): the level
// arrays are staged, and the ragged offsets formed, in one static device
// array per GPU instead of buffers allocated per call.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kNoAllocMaxInst = 131072;
// layout: level_old int32[MAX], level_new int32[MAX], offsets_old int64[MAX+1], offsets_new int64[MAX+1]
constexpr size_t kScratchLoOff = 0;
constexpr size_t kScratchLnOff = kScratchLoOff + 4 * kNoAllocMaxInst;
constexpr size_t kScratchOoOff = kScratchLnOff + 4 * kNoAllocMaxInst;
constexpr size_t kScratchOnOff = kScratchOoOff + 8 * (kNoAllocMaxInst + 1);
constexpr size_t kScratchBytes = kScratchOnOff + 8 * (kNoAllocMaxInst + 1);
static_assert(kScratchOoOff % 8 == 0 && kScratchOnOff % 8 == 0, "int64 regions aligned");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Exclusive prefix sums of (N+1)^2 over both level arrays, offsets[n] the
// total: one workgroup, each lane a contiguous chunk of instances.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void level_offsets_kernel(int n, const int32_t* lo, const int32_t* ln,
                                                                   int64_t* oo, int64_t* on) {
    __shared__ int64_t part[2][kScanThreads];
    const int t = threadIdx.x;
    const int per = (n + kScanThreads - 1) / kScanThreads;
    const int b = t * per;
    const int e = b + per < n ? b + per : n;
    int64_t so = 0, sn = 0;
    for (int i = b; i < e; ++i) {
        so += (int64_t)(lo[i] + 1) * (lo[i] + 1);
        sn += (int64_t)(ln[i] + 1) * (ln[i] + 1);
    }
    part[0][t] = so;
    part[1][t] = sn;
    __syncthreads();
    if (t == 0) {
        int64_t ao = 0, an = 0;
        for (int k = 0; k < kScanThreads; ++k) {
            const int64_t xo = part[0][k], xn = part[1][k];
            part[0][k] = ao;
            part[1][k] = an;
            ao += xo;
            an += xn;
        }
        oo[n] = ao;
        on[n] = an;
    }
    __syncthreads();
    so = part[0][t];
    sn = part[1][t];
    for (int i = b; i < e; ++i) {
        oo[i] = so;
        on[i] = sn;
        so += (int64_t)(lo[i] + 1) * (lo[i] + 1);
        sn += (int64_t)(ln[i] + 1) * (ln[i] + 1);
    }
}

}  // namespace

// Stand-in on the host for the device array; its device address is taken
// with hipGetSymbolAddress once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

extern "C" tsm_status tsm_prolong_noalloc(int64_t n_inst, const int32_t* lo, const int32_t* ln, const double* vo,
                                          int64_t n_old, double* vn, int64_t n_new, void* stream) {
    using namespace tsm;
    if (n_inst < 1 || !lo || !ln || !vo || !vn) return call_failed(TSM_EINVAL, "tsm_prolong_noalloc: bad arguments");
    if (n_inst > kNoAllocMaxInst)
        return call_failed(TSM_ENOMEM, "tsm_prolong_noalloc: " + std::to_string(n_inst) +
                                           " instances exceed its static workspace of " +
                                           std::to_string(kNoAllocMaxInst));
    int64_t to = 0, tn = 0;
    for (int64_t i = 0; i < n_inst; ++i) {
        if (lo[i] < kMinLevel || lo[i] > kMaxMesh || !(ln[i] == lo[i] || ln[i] == 2 * lo[i]) || ln[i] > kMaxMesh)
            return call_failed(TSM_EINVAL, "tsm_prolong_noalloc: level_new[" + std::to_string(i) +
                                               "] is neither level_old nor twice it (<= 256)");
        to += (int64_t)(lo[i] + 1) * (lo[i] + 1);
        tn += (int64_t)(ln[i] + 1) * (ln[i] + 1);
    }
    if (n_old != to || n_new != tn)
        return call_failed(TSM_EINVAL, "tsm_prolong_noalloc: v_old must hold " + std::to_string(to) + " and v_new " +
                                           std::to_string(tn) + " entries");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return call_failed(TSM_EHIP, std::string("tsm_prolong_noalloc: hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return call_failed(TSM_EINVAL, "tsm_prolong_noalloc: device index out of range");
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return call_failed(TSM_EHIP, std::string("tsm_prolong_noalloc: hipGetSymbolAddress: ") +
                                                 hipGetErrorString(e));
            g_scratch_ptr[dev] = p;
        }
        base = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    }
    int32_t* dlo = reinterpret_cast<int32_t*>(base + kScratchLoOff);
    int32_t* dln = reinterpret_cast<int32_t*>(base + kScratchLnOff);
    int64_t* doo = reinterpret_cast<int64_t*>(base + kScratchOoOff);
    int64_t* don = reinterpret_cast<int64_t*>(base + kScratchOnOff);
    hipStream_t s = (hipStream_t)stream;
    // every scratch entry the kernels read is written first in this call
    e = hipMemcpyAsync(dlo, lo, n_inst * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dln, ln, n_inst * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(level_offsets_kernel, dim3(1), dim3(kScanThreads), 0, s, (int)n_inst, dlo, dln, doo, don);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_prolong((int)n_inst, dlo, dln, doo, don, vo, vn, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return call_failed(TSM_EHIP, std::string("tsm_prolong_noalloc: ") + hipGetErrorString(e));
    }
    return TSM_OK;
}
