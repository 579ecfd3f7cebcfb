// HIP kernels for gfx950 (CDNA4): the fused DG right-hand side + Runge-Kutta
// stage (Sections 5.2-5.3), the period filter accumulation (Section 5.4) and
// the FP64 vector kernels of the CG iteration (Algorithm 3).
//
// Stage kernel layout: one workgroup = one 64-lane wavefront = 10 elements.
//   * the 10 x 6 x Np stage-input values are staged in LDS with coalesced
//     loads;
//   * face-node lanes compute the upwind flux (own trace from LDS, the
//     neighbour's from LDS when it belongs to the same workgroup, otherwise
//     from global memory through the connectivity code) into an LDS tile
//     laid out [face node][lane];
//   * lanes 0..59 own one (element, component) column: the reference
//     derivatives D_a y are formed with the matrix entries as wave-uniform
//     scalar operands (constant memory -> SGPRs), the two physical
//     derivatives a component contributes to the curl are exchanged between
//     the six lanes of an element with cross-lane permutes, and the lift
//     M^-1 E_f of the face fluxes is applied the same way;
//   * the RK stage update, source term, conductivity and the FP64 filter
//     accumulation run as one coalesced pass over the 10-element chunk.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "launch.h"

namespace cmcg {

namespace {

template <int Q> struct Dim {
    static constexpr int NP = (Q + 1) * (Q + 2) * (Q + 3) / 6;
    static constexpr int NFP = (Q + 1) * (Q + 2) / 2;
};

// per-q offsets into the constant tables
__host__ __device__ constexpr int mat_size(int q) {
    return 3 * ((q + 1) * (q + 2) * (q + 3) / 6) * ((q + 1) * (q + 2) * (q + 3) / 6) +
           ((q + 1) * (q + 2) * (q + 3) / 6) * 4 * ((q + 1) * (q + 2) / 2) +
           ((q + 1) * (q + 2) * (q + 3) / 6) * ((q + 1) * (q + 2) * (q + 3) / 6);
}
__host__ __device__ constexpr int mat_off(int q) { return q <= 1 ? 0 : mat_off(q - 1) + mat_size(q - 1); }
constexpr int kMatTotal = mat_off(4);
__host__ __device__ constexpr int fn_off(int q) { return q <= 1 ? 0 : fn_off(q - 1) + 4 * ((q) * (q + 1) / 2); }
__host__ __device__ constexpr int fp_off(int q) { return q <= 1 ? 0 : fp_off(q - 1) + 6 * ((q) * (q + 1) / 2); }
constexpr int kFnTotal = fn_off(4);
constexpr int kFpTotal = fp_off(4);

__constant__ double cMat64[kMatTotal];
__constant__ float cMat32[kMatTotal];
__constant__ int cFnode[kFnTotal];
__constant__ int cFperm[kFpTotal];

template <typename T> __device__ __forceinline__ const T* mats();
template <> __device__ __forceinline__ const double* mats<double>() { return cMat64; }
template <> __device__ __forceinline__ const float* mats<float>() { return cMat32; }

constexpr int EPW = 10;  // elements per 64-lane workgroup (60 active column lanes)

template <typename T, int Q>
__global__ __launch_bounds__(64) void k_stage(StageArgs a) {
    constexpr int NP = Dim<Q>::NP, NFP = Dim<Q>::NFP, NF4 = 4 * NFP;
    constexpr int MO = mat_off(Q);
    constexpr int LO = MO + 3 * NP * NP;  // LIFT [NP][NF4]
    __shared__ T sY[EPW * 6 * NP];
    __shared__ T sR[EPW * 6 * NP];
    __shared__ T sF[NF4 * 64];
    __shared__ T sG[EPW * kGeo];

    const T* __restrict__ Y = (const T*)a.Y;
    const int lane = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * EPW;
    const int ne = (int)((a.K - e0) < EPW ? (a.K - e0) : EPW);
    const int nv = ne * 6 * NP;
    const int64_t base = e0 * 6 * NP;

    for (int v = lane; v < nv; v += 64) sY[v] = Y[base + v];
    const T* geo = (const T*)a.geo + e0 * kGeo;
    for (int v = lane; v < ne * kGeo; v += 64) sG[v] = geo[v];
    __syncthreads();

    // ---- upwind flux at every face node: sF[face node][el * 6 + comp]
    const int* fnode = cFnode + fn_off(Q);
    const int* fperm = cFperm + fp_off(Q);
    for (int it = lane; it < ne * NF4; it += 64) {
        const int el = it / NF4;
        const int r = it - el * NF4;
        const int f = r / NFP;
        const int k = r - f * NFP;
        const int own = fnode[f * NFP + k];
        T Em[3], Hm[3], Ep[3], Hp[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Em[c] = sY[(el * 6 + c) * NP + own];
            Hm[c] = sY[(el * 6 + 3 + c) * NP + own];
        }
        const int code = a.conn[(e0 + el) * 4 + f];
        if (code >= 0) {
            const int64_t nb = code >> 5;
            const int f2 = (code >> 3) & 3;
            const int p = code & 7;
            const int nn = fnode[f2 * NFP + fperm[p * NFP + k]];
            if (nb >= e0 && nb < e0 + ne) {
                const int l = (int)(nb - e0);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Ep[c] = sY[(l * 6 + c) * NP + nn];
                    Hp[c] = sY[(l * 6 + 3 + c) * NP + nn];
                }
            } else {
                const T* q = Y + nb * 6 * NP + nn;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Ep[c] = q[c * NP];
                    Hp[c] = q[(3 + c) * NP];
                }
            }
        } else if (code == -1) {  // PEC ghost: E+ = -E-, H+ = H-
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Ep[c] = -Em[c];
                Hp[c] = Hm[c];
            }
        } else {  // impedance ghost (homogeneous part): zero exterior state
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Ep[c] = T(0);
                Hp[c] = T(0);
            }
        }
        const T* g = &sG[el * kGeo + 9 + 7 * f];
        const T n0 = g[0], n1 = g[1], n2 = g[2];
        const T cE1 = g[3], cE2 = g[4], cH1 = g[5], cH2 = g[6];
        const T dE0 = Ep[0] - Em[0], dE1 = Ep[1] - Em[1], dE2 = Ep[2] - Em[2];
        const T dH0 = Hp[0] - Hm[0], dH1 = Hp[1] - Hm[1], dH2 = Hp[2] - Hm[2];
        const T ndE = n0 * dE0 + n1 * dE1 + n2 * dE2;
        const T ndH = n0 * dH0 + n1 * dH1 + n2 * dH2;
        // n x dH, n x dE
        const T xH0 = n1 * dH2 - n2 * dH1, xH1 = n2 * dH0 - n0 * dH2, xH2 = n0 * dH1 - n1 * dH0;
        const T xE0 = n1 * dE2 - n2 * dE1, xE1 = n2 * dE0 - n0 * dE2, xE2 = n0 * dE1 - n1 * dE0;
        T* o = &sF[(f * NFP + k) * 64 + el * 6];
        o[0] = cE1 * (dE0 - ndE * n0) - cE2 * xH0;
        o[1] = cE1 * (dE1 - ndE * n1) - cE2 * xH1;
        o[2] = cE1 * (dE2 - ndE * n2) - cE2 * xH2;
        o[3] = cH1 * (dH0 - ndH * n0) + cH2 * xE0;
        o[4] = cH1 * (dH1 - ndH * n1) + cH2 * xE1;
        o[5] = cH1 * (dH2 - ndH * n2) + cH2 * xE2;
    }

    // ---- volume term: lane = (element, component) column
    const int el = lane / 6;
    const int c = lane - 6 * el;
    const bool act = el < ne;
    const int elc = act ? el : 0;
    const int row = elc * 6 + c;
    T y[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) y[j] = sY[row * NP + j];
    const T* gg = &sG[elc * kGeo];
    const int c3 = c < 3 ? c : c - 3;
    const int kp = c3 == 0 ? 2 : c3 - 1;  // (c3 + 2) % 3
    const int km = c3 == 2 ? 0 : c3 + 1;  // (c3 + 1) % 3
    T pv[NP], mv[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        pv[i] = T(0);
        mv[i] = T(0);
    }
    const T* Mt = mats<T>();
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const T gp = gg[3 * ax + kp];
        const T gm = gg[3 * ax + km];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            T d = T(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) d = fma(Mt[MO + (ax * NP + i) * NP + j], y[j], d);
            pv[i] = fma(gp, d, pv[i]);
            mv[i] = fma(-gm, d, mv[i]);
        }
    }
    // curl component c3 of the other field: +d_{c3+1} V_{c3+2} from lane
    // (c3+2), -d_{c3+2} V_{c3+1} from lane (c3+1)
    const int sb = elc * 6 + (c < 3 ? 3 : 0);
    const int lane_p = sb + (c3 == 0 ? 2 : c3 - 1);
    const int lane_m = sb + (c3 == 2 ? 0 : c3 + 1);
    T curl[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) curl[i] = __shfl(pv[i], lane_p) + __shfl(mv[i], lane_m);
    __syncthreads();  // flux tile complete

    // ---- lift and scaling
    T fl[NF4];
#pragma unroll
    for (int kk = 0; kk < NF4; ++kk) fl[kk] = sF[kk * 64 + lane];
    const T inv = c < 3 ? gg[37] : gg[38];
    const T sgn = c < 3 ? T(-1) : T(1);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        T s = T(0);
#pragma unroll
        for (int kk = 0; kk < NF4; ++kk) s = fma(Mt[LO + i * NF4 + kk], fl[kk], s);
        const T rv = inv * fma(sgn, curl[i], s);
        if (act) sR[row * NP + i] = rv;
    }
    __syncthreads();

    // ---- coalesced stage update
    const T* __restrict__ Ub = (const T*)a.U;
    const T* __restrict__ Sre = (const T*)a.Sre;
    const T* __restrict__ Sim = (const T*)a.Sim;
    const T scos = (T)a.scos, ssin = (T)a.ssin;
    const T cy = (T)a.cy, ca = (T)a.ca, cu = (T)a.cu;
    for (int v = lane; v < nv; v += 64) {
        const int rw = v / NP;
        const int comp = rw % 6;
        const int e = rw / 6;
        const T yv = sY[v];
        T k = sR[v];
        if (comp < 3) k = fma(-sG[e * kGeo + 39], yv, k);
        const int64_t gi = base + v;
        if (comp < a.src_rows) k += scos * Sre[gi] - ssin * Sim[gi];
        T u = yv;
        switch (a.mode) {
            case RK2_S1:
                ((T*)a.Ynext)[gi] = fma(cy, k, yv);
                break;
            case RK2_S2:
                u = Ub[gi];
                ((T*)a.Uout)[gi] = fma(cu, k, u);
                break;
            case RK4_S1:
                ((T*)a.Ynext)[gi] = fma(cy, k, yv);
                ((T*)a.Acc)[gi] = fma(ca, k, yv);
                break;
            case RK4_S2:
            case RK4_S3: {
                u = Ub[gi];
                ((T*)a.Ynext)[gi] = fma(cy, k, u);
                T* acc = (T*)a.Acc;
                acc[gi] = fma(ca, k, acc[gi]);
                break;
            }
            case RK4_S4:
                ((T*)a.Uout)[gi] = fma(cu, k, ((const T*)a.Acc)[gi]);
                break;
            default:
                ((T*)a.Kout)[gi] = k;
                break;
        }
        if (a.filter) {
            const double ud = (double)u, kd = (double)k;
            a.Fre[gi] += a.fa_re * ud + a.fb_re * kd;
            a.Fim[gi] += a.fa_im * ud + a.fb_im * kd;
        }
    }
}

template <typename T>
__global__ void k_to_field(const double* __restrict__ X, T* __restrict__ U, int64_t n, int Np, int flipH) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double x = X[i];
        if (flipH && ((i / Np) % 6) >= 3) x = -x;
        U[i] = (T)x;
    }
}

template <typename T>
__global__ void k_from_field(const T* __restrict__ U, double* __restrict__ Yo, const double* __restrict__ sub,
                             int64_t n, int Np, int flipH) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double x = (double)U[i];
        if (flipH && ((i / Np) % 6) >= 3) x = -x;
        if (sub) x -= sub[i];
        Yo[i] = x;
    }
}

template <typename T>
__global__ void k_copy(const T* __restrict__ s, T* __restrict__ d, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

__global__ void k_zero(uint32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_axpby(double a, const double* x, double b, const double* y, double* z, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = a * x[i] + b * y[i];
}

template <typename T>
__global__ void k_filter_add(const T* __restrict__ U, double wr, double wi, double* Fre, double* Fim, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double u = (double)U[i];
        Fre[i] += wr * u;
        Fim[i] += wi * u;
    }
}

constexpr int kDotBlocks = 1024;
constexpr int kDotThreads = 256;

template <int Q>
__global__ __launch_bounds__(kDotThreads) void k_dot(const double* __restrict__ U, const double* __restrict__ V,
                                                     const double* __restrict__ wE, const double* __restrict__ wH,
                                                     int64_t K, double* __restrict__ partial) {
    constexpr int NP = Dim<Q>::NP;
    constexpr int MMO = mat_off(Q) + 3 * NP * NP + NP * 4 * Dim<Q>::NFP;
    __shared__ double sm[kDotThreads];
    double acc = 0.0;
    const int64_t rows = 6 * K;
    for (int64_t r = blockIdx.x * (int64_t)kDotThreads + threadIdx.x; r < rows; r += (int64_t)gridDim.x * kDotThreads) {
        const double* u = U + r * NP;
        const double* v = V + r * NP;
        double vv[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) vv[j] = v[j];
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            double mvv = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) mvv = fma(cMat64[MMO + i * NP + j], vv[j], mvv);
            s = fma(u[i], mvv, s);
        }
        const int64_t e = r / 6;
        acc = fma(s, (r - 6 * e) < 3 ? wE[e] : wH[e], acc);
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kDotThreads) void k_dot_final(const double* __restrict__ partial, int n,
                                                           double* __restrict__ out) {
    __shared__ double sm[kDotThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kDotThreads) acc += partial[i];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

__global__ void k_nonfinite(const double* X, int64_t n, int* flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = X[i];
        if (!(x == x) || x - x != 0.0) flag[0] = 1;
    }
}

inline int grid_for(int64_t n, int threads = 256) {
    int64_t g = (n + threads - 1) / threads;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

template <typename T, int Q>
void stage_launch(const StageArgs& a, hipStream_t s) {
    const int64_t blocks = (a.K + EPW - 1) / EPW;
    hipLaunchKernelGGL((k_stage<T, Q>), dim3((unsigned)blocks), dim3(64), 0, s, a);
}

void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(CMCG_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

}  // namespace

void upload_constants(int q, int precision, const double* D, const double* LIFT, const double* M,
                      const int* fnode, const int* fperm) {
    (void)precision;
    const int NP = np_of(q), NFP = nfp_of(q);
    const int n = mat_size(q);
    std::vector<double> buf(n);
    std::copy(D, D + 3 * NP * NP, buf.begin());
    std::copy(LIFT, LIFT + NP * 4 * NFP, buf.begin() + 3 * NP * NP);
    std::copy(M, M + NP * NP, buf.begin() + 3 * NP * NP + 4 * NP * NFP);
    std::vector<float> bf(buf.begin(), buf.end());
    const size_t off = mat_off(q);
    CMCG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cMat64), buf.data(), n * sizeof(double), off * sizeof(double),
                               hipMemcpyHostToDevice));
    CMCG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cMat32), bf.data(), n * sizeof(float), off * sizeof(float),
                               hipMemcpyHostToDevice));
    CMCG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cFnode), fnode, 4 * NFP * sizeof(int), fn_off(q) * sizeof(int),
                               hipMemcpyHostToDevice));
    CMCG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cFperm), fperm, 6 * NFP * sizeof(int), fp_off(q) * sizeof(int),
                               hipMemcpyHostToDevice));
}

void launch_stage(int q, int precision, const StageArgs& a, hipStream_t s) {
    if (precision == CMCG_FP64) {
        if (q == 1) stage_launch<double, 1>(a, s);
        else if (q == 2) stage_launch<double, 2>(a, s);
        else stage_launch<double, 3>(a, s);
    } else {
        if (q == 1) stage_launch<float, 1>(a, s);
        else if (q == 2) stage_launch<float, 2>(a, s);
        else stage_launch<float, 3>(a, s);
    }
    check_launch();
}

void launch_to_field(int precision, int Np, const double* X, void* U, int64_t n, int flipH, hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_to_field<double>, dim3(grid_for(n)), dim3(256), 0, s, X, (double*)U, n, Np, flipH);
    else
        hipLaunchKernelGGL(k_to_field<float>, dim3(grid_for(n)), dim3(256), 0, s, X, (float*)U, n, Np, flipH);
    check_launch();
}

void launch_from_field(int precision, int Np, const void* U, double* Y, const double* sub, int64_t n, int flipH,
                       hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_from_field<double>, dim3(grid_for(n)), dim3(256), 0, s, (const double*)U, Y, sub, n,
                           Np, flipH);
    else
        hipLaunchKernelGGL(k_from_field<float>, dim3(grid_for(n)), dim3(256), 0, s, (const float*)U, Y, sub, n,
                           Np, flipH);
    check_launch();
}

void launch_copy_field(int precision, const void* src, void* dst, int64_t n, hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_copy<double>, dim3(grid_for(n)), dim3(256), 0, s, (const double*)src, (double*)dst, n);
    else
        hipLaunchKernelGGL(k_copy<float>, dim3(grid_for(n)), dim3(256), 0, s, (const float*)src, (float*)dst, n);
    check_launch();
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(256), 0, s, (uint32_t*)p, n);
    check_launch();
}

void launch_axpby(double a, const double* x, double b, const double* y, double* z, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, s, a, x, b, y, z, n);
    check_launch();
}

void launch_filter_add(int precision, const void* U, double wr, double wi, double* Fre, double* Fim, int64_t n,
                       hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_filter_add<double>, dim3(grid_for(n)), dim3(256), 0, s, (const double*)U, wr, wi, Fre,
                           Fim, n);
    else
        hipLaunchKernelGGL(k_filter_add<float>, dim3(grid_for(n)), dim3(256), 0, s, (const float*)U, wr, wi, Fre,
                           Fim, n);
    check_launch();
}

int dot_partials() { return kDotBlocks; }

void launch_dot(int q, const double* U, const double* V, const double* wE, const double* wH, int64_t K,
                double* partial, double* out_dev, hipStream_t s) {
    int64_t rows = 6 * K;
    int blocks = (int)((rows + kDotThreads - 1) / kDotThreads);
    if (blocks > kDotBlocks) blocks = kDotBlocks;
    if (q == 1)
        hipLaunchKernelGGL(k_dot<1>, dim3(blocks), dim3(kDotThreads), 0, s, U, V, wE, wH, K, partial);
    else if (q == 2)
        hipLaunchKernelGGL(k_dot<2>, dim3(blocks), dim3(kDotThreads), 0, s, U, V, wE, wH, K, partial);
    else
        hipLaunchKernelGGL(k_dot<3>, dim3(blocks), dim3(kDotThreads), 0, s, U, V, wE, wH, K, partial);
    check_launch();
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kDotThreads), 0, s, partial, blocks, out_dev);
    check_launch();
}

void launch_nonfinite(const double* X, int64_t n, int* out_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n)), dim3(256), 0, s, X, n, out_dev);
    check_launch();
}

}  // namespace cmcg
