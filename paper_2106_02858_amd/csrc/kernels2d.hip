// Kernels of the 2-D transverse-magnetic path (Section 5.2.1, two-dimensional
// setting; Section 5.2.2 DG scheme on triangles; Section 5.3 Runge-Kutta
// stages): fields (e, h1, h2), dof layout [K][3][Np].
//
// Stage kernel: one 64-lane workgroup per block of 21 triangles, lane =
// (triangle, component).  The block's stage input is staged in LDS with one
// coalesced load, together with the order's D and LIFT (read afterwards as
// LDS broadcasts, which shortens the chain of scalar-cache loads a lone wave
// otherwise waits on); each lane differentiates its own component, and the
// curl terms are exchanged between the three lanes of a triangle:
//   e row:  -scurl h = -(d1 h2 - d2 h1),   h1 row: d2 e,   h2 row: -d1 e.
// The upwind flux of the lane's component is formed at the Nfp nodes of each
// edge (own traces from LDS, neighbour traces from the field) and lifted with
// LIFT.  The Runge-Kutta update, the compensated FP32 state and the filter
// accumulation follow the stage modes of launch.h, as in the 3-D kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "launch.h"

namespace cmcg {

namespace {

template <int Q> struct Dim2 {
    static constexpr int NP = (Q + 1) * (Q + 2) / 2;
    static constexpr int NFP = Q + 1;
    static constexpr int MAT = 2 * NP * NP + NP * 3 * NFP + NP * NP;  // D | LIFT | M
};
constexpr int mat2_off(int q) { return q <= 1 ? 0 : q == 2 ? Dim2<1>::MAT : Dim2<1>::MAT + Dim2<2>::MAT; }
constexpr int kMat2Total = Dim2<1>::MAT + Dim2<2>::MAT + Dim2<3>::MAT;

__constant__ double c2Mat64[kMat2Total];
__constant__ float c2Mat32[kMat2Total];

template <typename T> __device__ __forceinline__ const T* mats2();
template <> __device__ __forceinline__ const double* mats2<double>() { return c2Mat64; }
template <> __device__ __forceinline__ const float* mats2<float>() { return c2Mat32; }

constexpr int EPB = 21;  // triangles per 64-lane workgroup (63 active lanes)
constexpr int64_t kEarlyBlocks = 2048;

// Element node of edge node k of edge f (nodes (i, j)/q, j slowest; edge 0 runs
// from vertex 1 to vertex 2, edge 1 from 0 to 2, edge 2 from 0 to 1).
template <int Q> __device__ __host__ constexpr int edge_node(int f, int k) {
    // node (i, j) has index j (Q + 1) - j (j - 1) / 2 + i
    return f == 0 ? k * (Q + 1) - k * (k - 1) / 2 + (Q - k) : f == 1 ? k * (Q + 1) - k * (k - 1) / 2 : k;
}

__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint32_t h) { return __uint_as_float(h << 16); }

// NP contiguous values of one row in pairs: 8-byte accesses for FP32 rows,
// 16-byte for FP64 rows, when rows start on such boundaries (they start at
// multiples of NP sizeof(T) bytes: P2 and P3), single accesses otherwise;
// bfloat16 rows likewise in 4-byte pairs.
template <typename T, int NP> struct Row2 {
    static constexpr bool V2 = NP % 2 == 0;
    using P2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    __device__ __forceinline__ static void load(const T* __restrict__ p, T (&r)[NP]) {
        if constexpr (V2) {
            const P2* q = reinterpret_cast<const P2*>(p);
#pragma unroll
            for (int c = 0; c < NP / 2; ++c) {
                const P2 v = q[c];
                r[2 * c] = v.x;
                r[2 * c + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NP; ++i) r[i] = p[i];
        }
    }
    __device__ __forceinline__ static void store(T* __restrict__ p, const T (&r)[NP]) {
        if constexpr (V2) {
            P2* q = reinterpret_cast<P2*>(p);
#pragma unroll
            for (int c = 0; c < NP / 2; ++c) {
                P2 v;
                v.x = r[2 * c];
                v.y = r[2 * c + 1];
                q[c] = v;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NP; ++i) p[i] = r[i];
        }
    }
};
template <int NP> struct RowLo2 {
    static constexpr bool V2 = (NP * 2) % 4 == 0;
    __device__ __forceinline__ static void load(const uint16_t* __restrict__ p, float (&r)[NP]);
    __device__ __forceinline__ static void store(uint16_t* __restrict__ p, const float (&r)[NP]);
};
template <int NP>
__device__ __forceinline__ void RowLo2<NP>::load(const uint16_t* __restrict__ p, float (&r)[NP]) {
    if constexpr (V2) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
        for (int c = 0; c < NP / 2; ++c) {
            const uint32_t w = q[c];
            r[2 * c] = __uint_as_float(w << 16);
            r[2 * c + 1] = __uint_as_float(w & 0xffff0000u);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NP; ++i) r[i] = __uint_as_float((uint32_t)p[i] << 16);
    }
}

template <int NP>
__device__ __forceinline__ void RowLo2<NP>::store(uint16_t* __restrict__ p, const float (&r)[NP]) {
    if constexpr (V2) {
        uint32_t* q = reinterpret_cast<uint32_t*>(p);
#pragma unroll
        for (int c = 0; c < NP / 2; ++c) q[c] = (uint32_t)to_bf16(r[2 * c]) | ((uint32_t)to_bf16(r[2 * c + 1]) << 16);
    } else {
#pragma unroll
        for (int i = 0; i < NP; ++i) p[i] = to_bf16(r[i]);
    }
}

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Arguments of this workgroup's member in a batched launch (grid.y = member):
// field, geometry and source pointers move by whole members, the stage
// scalars come from the member table; false when the member is idle (its CG
// has converged, or its period has fewer steps than this launch's).
template <typename T>
__device__ __forceinline__ bool member_args2d(const StageArgs& in, StageArgs& a) {
    a = in;
    a.smask = nullptr;
    if (!in.mtab) return true;
    const int b = blockIdx.y;
    if (!in.active[b]) return false;
    if (in.step >= 0 && in.step >= in.msteps[b]) return false;
    const double* p = in.mtab + (int64_t)b * kMemberParams;
    a.cy = p[0];
    a.ca = p[1];
    a.cu = p[2];
    a.scos = p[3];
    a.ssin = p[4];
    a.fa_re = p[5];
    a.fa_im = p[6];
    a.fb_re = p[7];
    a.fb_im = p[8];
    const int64_t fo = (int64_t)b * in.bstride;
    if (in.Y) a.Y = (const T*)in.Y + fo;
    if (in.U) a.U = (const T*)in.U + fo;
    if (in.Ynext) a.Ynext = (T*)in.Ynext + fo;
    if (in.Acc) a.Acc = (T*)in.Acc + fo;
    if (in.Uout) a.Uout = (T*)in.Uout + fo;
    if (in.Kout) a.Kout = (T*)in.Kout + fo;
    if (in.Ulo) a.Ulo = (uint16_t*)in.Ulo + fo;
    if (in.Fre) a.Fre = in.Fre + fo;
    if (in.Fim) a.Fim = in.Fim + fo;
    a.geo = (const T*)in.geo + (int64_t)b * in.gstride;
    if (in.Sre) a.Sre = (const T*)in.Sre + (int64_t)b * in.sstride;
    if (in.Sim) a.Sim = (const T*)in.Sim + (int64_t)b * in.sstride;
    return true;
}

template <typename T, int Q, bool EARLY>
__global__ __launch_bounds__(64) void k_stage2d(StageArgs args, int64_t per) {
    constexpr int NP = Dim2<Q>::NP, NFP = Dim2<Q>::NFP, NF3 = 3 * NFP;
    constexpr int MO = 0;                 // D [2][NP][NP] in sM
    constexpr int LO = 2 * NP * NP;       // LIFT [NP][3 NFP] in sM
    constexpr int NM = 2 * NP * NP + NP * NF3;
    constexpr int ROWS = EPB * 3;
    __shared__ __align__(16) T sY[ROWS * NP];
    __shared__ __align__(16) T sG[EPB * kGeo2];
    __shared__ int sC[EPB * 3];
    __shared__ T sM[NM];  // the order's D and LIFT, read as LDS broadcasts

    StageArgs a;
    if (!member_args2d<T>(args, a)) return;  // uniform per workgroup
    const int64_t b = blockIdx.x;
    const int64_t blk = (b & 7) * per + (b >> 3);  // consecutive blocks on one XCD
    const int64_t e0 = blk * EPB;
    if (e0 >= a.K) return;
    const int lane = threadIdx.x;
    const int ne = (int)((a.K - e0) < EPB ? (a.K - e0) : EPB);
    const T* __restrict__ Y = (const T*)a.Y;
    const T* __restrict__ geo = (const T*)a.geo;
    {
        // every staging load is issued before the first is consumed (loops of
        // a compile-time trip count; a loop that stored each value as it
        // arrived waited for one load at a time), then written to LDS.  The
        // stage input goes in pairs when the chunk starts on a pair boundary
        // and holds whole pairs, the geometry records (28 values) in 16-byte
        // groups.
        constexpr int PV = Row2<T, NP>::V2 ? 2 : 1;
        constexpr int GV = 16 / (int)sizeof(T);
        // native vectors: arrays of them stay in registers
        typedef T VY __attribute__((ext_vector_type(PV)));
        typedef T VG __attribute__((ext_vector_type(GV)));
        static_assert(kGeo2 % GV == 0, "geometry records split into 16-byte groups");
        constexpr int NYL = (EPB * 3 * NP / PV + 63) / 64, NGL = (EPB * kGeo2 / GV + 63) / 64;
        constexpr int NML = (NM + 63) / 64, NCL = (EPB * 3 + 63) / 64;
        const int nyl = ne * 3 * NP / PV, ngl = ne * kGeo2 / GV;
        const VY* ys = reinterpret_cast<const VY*>(Y + e0 * 3 * NP);
        const VG* gs = reinterpret_cast<const VG*>(geo + e0 * kGeo2);
        const T* gm = mats2<T>() + mat2_off(Q);
        VY ry[NYL];
        VG rg[NGL];
        T rm[NML];
        int rc[NCL];
#pragma unroll
        for (int i = 0; i < NYL; ++i)
            if (lane + 64 * i < nyl) ry[i] = ys[lane + 64 * i];
#pragma unroll
        for (int i = 0; i < NGL; ++i)
            if (lane + 64 * i < ngl) rg[i] = gs[lane + 64 * i];
#pragma unroll
        for (int i = 0; i < NCL; ++i)
            if (lane + 64 * i < ne * 3) rc[i] = a.conn[e0 * 3 + lane + 64 * i];
#pragma unroll
        for (int i = 0; i < NML; ++i)
            if (lane + 64 * i < NM) rm[i] = gm[lane + 64 * i];
        VY* yd = reinterpret_cast<VY*>(sY);
        VG* gd = reinterpret_cast<VG*>(sG);
#pragma unroll
        for (int i = 0; i < NYL; ++i)
            if (lane + 64 * i < nyl) yd[lane + 64 * i] = ry[i];
#pragma unroll
        for (int i = 0; i < NGL; ++i)
            if (lane + 64 * i < ngl) gd[lane + 64 * i] = rg[i];
#pragma unroll
        for (int i = 0; i < NCL; ++i)
            if (lane + 64 * i < ne * 3) sC[lane + 64 * i] = rc[i];
#pragma unroll
        for (int i = 0; i < NML; ++i)
            if (lane + 64 * i < NM) sM[lane + 64 * i] = rm[i];
    }
    __syncthreads();

    const int el = lane / 3;
    const int c = lane - 3 * el;
    const bool act = el < ne;
    const int elc = act ? el : 0;
    const int row = elc * 3 + c;
    const int64_t grow = (e0 * 3 + row) * NP;
    const int mode = a.mode;
    constexpr bool COMP = std::is_same<T, float>::value;
    const bool needL = COMP && (mode == RK2_S2 || mode == RK4_S4);
    const bool needU = mode == RK2_S2 || mode == RK4_S2 || mode == RK4_S3 || needL;
    const bool needA = mode == RK4_S2 || mode == RK4_S3 || mode == RK4_S4;
    const T* Mt = sM;
    const T* gg = &sG[elc * kGeo2];

    // ---- EARLY: every global load of the stage is requested here, before the
    // volume work (neighbour traces of the three edges, update operands,
    // source rows): for launches of about one wave per SIMD, where each wave's
    // chain of dependent loads sets the time.  Otherwise the traces are
    // gathered per edge and the update operands loaded after the lift, which
    // keeps the registers (and so the occupancy) of large launches in check.
    // Each lane gathers its own component of the neighbour's edge trace; the
    // triangle's three lanes then exchange them (lanes 3 el + c), so every
    // trace value is loaded once.
    const int base = 3 * elc;
    T nv[3][NFP];
    auto gather = [&](int f, T (&own)[NFP]) {
        const int code = sC[elc * 3 + f];
#pragma unroll
        for (int k = 0; k < NFP; ++k) {
            if (code >= 0) {
                const int64_t nb = code >> 5;
                const int nf = (code >> 3) & 3;
                const int kk = (code & 7) ? NFP - 1 - k : k;
                own[k] = Y[nb * 3 * NP + c * NP + edge_node<Q>(nf, kk)];
            } else {
                own[k] = T(0);
            }
        }
    };
    auto expand = [&](const T (&own)[NFP], T (&tr)[NFP][3]) {
#pragma unroll
        for (int k = 0; k < NFP; ++k) {
            tr[k][0] = __shfl(own[k], base);
            tr[k][1] = __shfl(own[k], base + 1);
            tr[k][2] = __shfl(own[k], base + 2);
        }
    };
    T up[NP], ap[NP], sr[NP], si[NP];
    float lo[NP];
    const bool src = act && c < a.src_rows;
    auto operands = [&]() {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            up[i] = ap[i] = sr[i] = si[i] = T(0);
            lo[i] = 0.f;
        }
        if (act && needU) Row2<T, NP>::load((const T*)a.U + grow, up);
        if (act && needA) Row2<T, NP>::load((const T*)a.Acc + grow, ap);
        if (act && needL) RowLo2<NP>::load((const uint16_t*)a.Ulo + grow, lo);
        if (src) {
            Row2<T, NP>::load((const T*)a.Sre + grow, sr);
            Row2<T, NP>::load((const T*)a.Sim + grow, si);
        }
    };
    if constexpr (EARLY) {
#pragma unroll
        for (int f = 0; f < 3; ++f) gather(f, nv[f]);
        operands();
    }

    // ---- volume: physical derivatives of the lane's component
    T y[NP], d1[NP], d2[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) y[j] = sY[row * NP + j];
    const T g00 = gg[0], g01 = gg[1], g10 = gg[2], g11 = gg[3];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        T r0 = T(0), r1 = T(0);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            r0 = fma(Mt[MO + i * NP + j], y[j], r0);
            r1 = fma(Mt[MO + NP * NP + i * NP + j], y[j], r1);
        }
        d1[i] = fma(g00, r0, g10 * r1);
        d2[i] = fma(g01, r0, g11 * r1);
    }
    // curl exchange between the triangle's lanes (3 el: e, 3 el + 1: h1, 3 el + 2: h2)
    const int srcA = c == 0 ? base + 2 : base;  // lane whose d1 is taken
    const int srcB = c == 0 ? base + 1 : base;  // lane whose d2 is taken
    const T sa = c == 1 ? T(0) : T(-1);
    const T sb = c == 2 ? T(0) : T(1);
    T acc[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const T A = __shfl(d1[i], srcA);
        const T B = __shfl(d2[i], srcB);
        acc[i] = sa * A + sb * B;
    }

    // ---- upwind flux of the lane's component on each edge, lifted
    auto face = [&](int f, const T (&tr)[NFP][3]) {
        const int code = sC[elc * 3 + f];
        const T* g = &gg[4 + 6 * f];
        const T n0 = g[0], n1 = g[1];
        const T cE1 = g[2], cE2 = g[3], cH1 = g[4], cH2 = g[5];
        T fl[NFP];
#pragma unroll
        for (int k = 0; k < NFP; ++k) {
            const int own = edge_node<Q>(f, k);
            const T em = sY[(elc * 3) * NP + own];
            const T h1m = sY[(elc * 3 + 1) * NP + own];
            const T h2m = sY[(elc * 3 + 2) * NP + own];
            T ep = tr[k][0], h1p = tr[k][1], h2p = tr[k][2];
            if (code == -1) {  // PEC ghost: e+ = -e-, h+ = h-
                ep = -em;
                h1p = h1m;
                h2p = h2m;
            }  // impedance ghost (homogeneous part): zero exterior state, as gathered
            const T de = ep - em, dh1 = h1p - h1m, dh2 = h2p - h2m;
            if (c == 0) {
                fl[k] = cE1 * de - cE2 * (n0 * dh2 - n1 * dh1);
            } else {
                const T ndh = n0 * dh1 + n1 * dh2;
                fl[k] = c == 1 ? cH1 * (dh1 - ndh * n0) + cH2 * (n1 * de) : cH1 * (dh2 - ndh * n1) - cH2 * (n0 * de);
            }
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            T t = acc[i];
#pragma unroll
            for (int k = 0; k < NFP; ++k) t = fma(Mt[LO + i * NF3 + f * NFP + k], fl[k], t);
            acc[i] = t;
        }
    };
    if constexpr (EARLY) {
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            T tr[NFP][3];
            expand(nv[f], tr);
            face(f, tr);
        }
    } else {
#pragma unroll 1
        for (int f = 0; f < 3; ++f) {
            T own[NFP], tr[NFP][3];
            gather(f, own);
            expand(own, tr);
            face(f, tr);
        }
    }
    if (!act) return;
    if constexpr (!EARLY) operands();

    // ---- stage update of the lane's row
    const T inv = c == 0 ? gg[22] : gg[23];
    const T sig = c == 0 ? gg[24] : T(0);
    T kv[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) kv[i] = fma(inv, acc[i], -sig * y[i]);
    if (src) {
        const T scos = (T)a.scos, ssin = (T)a.ssin;
#pragma unroll
        for (int i = 0; i < NP; ++i) kv[i] += scos * sr[i] - ssin * si[i];
        // further harmonics of a several-frequency source (single launches only,
        // so the kernel arguments hold this problem's tables; they are indexed
        // there, not in the local copy, which would go to scratch)
#pragma unroll 1
        for (int h = 1; h < args.nharm; ++h) {
            Row2<T, NP>::load((const T*)args.Sre + h * args.hstride + grow, sr);
            Row2<T, NP>::load((const T*)args.Sim + h * args.hstride + grow, si);
            const T hc = (T)args.hcos[h], hs = (T)args.hsin[h];
#pragma unroll
            for (int i = 0; i < NP; ++i) kv[i] += hc * sr[i] - hs * si[i];
        }
    }
    const T cy = (T)a.cy, ca = (T)a.ca, cu = (T)a.cu;
    T o1[NP], o2[NP];
    float lo2[NP];
    switch (mode) {
        case RK2_S1:
#pragma unroll
            for (int i = 0; i < NP; ++i) o1[i] = fma(cy, kv[i], y[i]);
            Row2<T, NP>::store((T*)a.Ynext + grow, o1);
            break;
        case RK2_S2:
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                if constexpr (COMP)
                    two_sum(up[i], fma(cu, kv[i], lo[i]), o1[i], lo2[i]);
                else
                    o1[i] = fma(cu, kv[i], up[i]);
            }
            Row2<T, NP>::store((T*)a.Uout + grow, o1);
            if constexpr (COMP) RowLo2<NP>::store((uint16_t*)a.Ulo + grow, lo2);
            break;
        case RK4_S1:
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                o1[i] = fma(cy, kv[i], y[i]);
                o2[i] = COMP ? ca * kv[i] : fma(ca, kv[i], y[i]);
            }
            Row2<T, NP>::store((T*)a.Ynext + grow, o1);
            Row2<T, NP>::store((T*)a.Acc + grow, o2);
            break;
        case RK4_S2:
        case RK4_S3:
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                o1[i] = fma(cy, kv[i], up[i]);
                o2[i] = fma(ca, kv[i], ap[i]);
            }
            Row2<T, NP>::store((T*)a.Ynext + grow, o1);
            Row2<T, NP>::store((T*)a.Acc + grow, o2);
            break;
        case RK4_S4:
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                if constexpr (COMP)
                    two_sum(up[i], fma(cu, kv[i], ap[i]) + lo[i], o1[i], lo2[i]);
                else
                    o1[i] = fma(cu, kv[i], ap[i]);
            }
            Row2<T, NP>::store((T*)a.Uout + grow, o1);
            if constexpr (COMP) RowLo2<NP>::store((uint16_t*)a.Ulo + grow, lo2);
            break;
        default:
            Row2<T, NP>::store((T*)a.Kout + grow, kv);
            break;
    }
    if (a.filter) {
        double* fr = a.Fre + grow;
        double* fi = a.Fim + grow;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const double ud = (double)y[i], kd = (double)kv[i];
            fr[i] += a.fa_re * ud + a.fb_re * kd;
            fi[i] += a.fa_im * ud + a.fb_im * kd;
        }
#pragma unroll 1
        for (int h = 1; h < args.nharm; ++h) {  // each harmonic filtered at its own frequency
            double* hr = args.Fre + h * args.hstride + grow;
            double* hi = args.Fim + h * args.hstride + grow;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const double ud = (double)y[i], kd = (double)kv[i];
                hr[i] += args.hfa_re[h] * ud + args.hfb_re[h] * kd;
                hi[i] += args.hfa_im[h] * ud + args.hfb_im[h] * kd;
            }
        }
    }
}

template <typename T>
__global__ void k_to_field2d(const double* __restrict__ X, T* __restrict__ U, uint16_t* __restrict__ Ulo, int64_t n,
                             int Np, int flipH) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double x = X[i];
        if (flipH && ((i / Np) % 3) >= 1) x = -x;
        const T hi = (T)x;
        U[i] = hi;
        if constexpr (std::is_same<T, float>::value)
            if (Ulo) Ulo[i] = to_bf16((float)(x - (double)hi));
    }
}

template <typename T>
__global__ void k_from_field2d(const T* __restrict__ U, const uint16_t* __restrict__ Ulo, double* __restrict__ Yo,
                               const double* __restrict__ sub, int64_t n, int Np, int flipH) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double x = (double)U[i];
        if constexpr (std::is_same<T, float>::value)
            if (Ulo) x += (double)from_bf16(Ulo[i]);
        if (flipH && ((i / Np) % 3) >= 1) x = -x;
        if (sub) x -= sub[i];
        Yo[i] = x;
    }
}

constexpr int kDot2Blocks = 1024;
constexpr int kDot2Threads = 256;

// (U, V)_{eps,mu} per block over rows r = 3 e + c (weight wE for c = 0, wH
// otherwise), fixed decomposition; k_dot2d_final sums the partials in a
// fixed order, so the result does not depend on scheduling.
template <int Q>
__global__ __launch_bounds__(kDot2Threads) void k_dot2d(const double* __restrict__ U, const double* __restrict__ V,
                                                        const double* __restrict__ wE, const double* __restrict__ wH,
                                                        int64_t K, double* __restrict__ partial) {
    constexpr int NP = Dim2<Q>::NP;
    constexpr int MMO = mat2_off(Q) + 2 * NP * NP + NP * 3 * Dim2<Q>::NFP;
    __shared__ double sm[kDot2Threads];
    double acc = 0.0;
    const int64_t rows = 3 * K;
    for (int64_t r = blockIdx.x * (int64_t)kDot2Threads + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * kDot2Threads) {
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
            for (int j = 0; j < NP; ++j) mvv = fma(c2Mat64[MMO + i * NP + j], vv[j], mvv);
            s = fma(u[i], mvv, s);
        }
        const int64_t e = r / 3;
        acc = fma(s, (r - 3 * e) == 0 ? wE[e] : wH[e], acc);
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kDot2Threads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

// Batched form: member b = blockIdx.y, the same block decomposition and
// summation order per member (a member's inner product equals its single one).
template <int Q>
__global__ __launch_bounds__(kDot2Threads) void k_dot2d_batch(const double* __restrict__ U,
                                                              const double* __restrict__ V,
                                                              const double* __restrict__ wE,
                                                              const double* __restrict__ wH, int64_t wstride,
                                                              int64_t K, double* __restrict__ partial) {
    constexpr int NP = Dim2<Q>::NP;
    constexpr int MMO = mat2_off(Q) + 2 * NP * NP + NP * 3 * Dim2<Q>::NFP;
    __shared__ double sm[kDot2Threads];
    const int64_t bm = blockIdx.y;
    const int64_t n = 3 * K * NP;
    U += bm * n;
    V += bm * n;
    wE += bm * wstride;
    wH += bm * wstride;
    double acc = 0.0;
    const int64_t rows = 3 * K;
    for (int64_t r = blockIdx.x * (int64_t)kDot2Threads + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * kDot2Threads) {
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
            for (int j = 0; j < NP; ++j) mvv = fma(c2Mat64[MMO + i * NP + j], vv[j], mvv);
            s = fma(u[i], mvv, s);
        }
        const int64_t e = r / 3;
        acc = fma(s, (r - 3 * e) == 0 ? wE[e] : wH[e], acc);
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kDot2Threads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[bm * kDot2Blocks + blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kDot2Threads) void k_dot2d_final_batch(const double* __restrict__ partial, int n,
                                                                    double* __restrict__ out) {
    __shared__ double sm[kDot2Threads];
    const int bm = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kDot2Threads) acc += partial[(int64_t)bm * kDot2Blocks + i];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kDot2Threads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[bm] = sm[0];
}

__global__ __launch_bounds__(kDot2Threads) void k_dot2d_final(const double* __restrict__ partial, int n,
                                                              double* __restrict__ out) {
    __shared__ double sm[kDot2Threads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kDot2Threads) acc += partial[i];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kDot2Threads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

unsigned grid2_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (unsigned)g;
}

void check2() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(CMCG_ERR_DEVICE, std::string("2-D kernel launch: ") + hipGetErrorString(e));
}

template <typename T, int Q>
void stage2d(const StageArgs& a, hipStream_t s) {
    const int64_t nb = (a.K + EPB - 1) / EPB;
    const int64_t per = (nb + 7) / 8;
    if (8 * per > 0x7fffffffLL) fail(CMCG_ERR_ARG, "stage2d: too many element blocks");
    if (a.mtab && (a.nmembers < 1 || a.nmembers > 65535)) fail(CMCG_ERR_ARG, "stage2d: 1 to 65535 members");
    const dim3 grid((unsigned)(8 * per), (unsigned)(a.mtab ? a.nmembers : 1));
    // early loads pay off while the launch has at most about two single-wave
    // workgroups per SIMD (1024 SIMDs); FP64 always takes the lean form
    const int64_t total = nb * (a.mtab ? a.nmembers : 1);
    if constexpr (std::is_same<T, float>::value) {
        if (total <= kEarlyBlocks) {
            hipLaunchKernelGGL((k_stage2d<T, Q, true>), grid, dim3(64), 0, s, a, per);
            return;
        }
    }
    hipLaunchKernelGGL((k_stage2d<T, Q, false>), grid, dim3(64), 0, s, a, per);
}

}  // namespace

void upload_constants2d(int q, const double* D, const double* LIFT, const double* M, const int* fnode) {
    const int NP = np2_of(q), NFP = nfp2_of(q);
    for (int f = 0; f < 3; ++f)
        for (int k = 0; k < NFP; ++k) {
            const int want = q == 1 ? edge_node<1>(f, k) : q == 2 ? edge_node<2>(f, k) : edge_node<3>(f, k);
            if (fnode[f * NFP + k] != want) fail(CMCG_ERR_ARG, "2-D edge-node table does not match the kernels");
        }
    const int n = 2 * NP * NP + NP * 3 * NFP + NP * NP;
    std::vector<double> buf(n);
    std::copy(D, D + 2 * NP * NP, buf.begin());
    std::copy(LIFT, LIFT + NP * 3 * NFP, buf.begin() + 2 * NP * NP);
    std::copy(M, M + NP * NP, buf.begin() + 2 * NP * NP + 3 * NP * NFP);
    std::vector<float> bf(buf.begin(), buf.end());
    const size_t off = mat2_off(q);
    CMCG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c2Mat64), buf.data(), n * sizeof(double), off * sizeof(double),
                               hipMemcpyHostToDevice));
    CMCG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c2Mat32), bf.data(), n * sizeof(float), off * sizeof(float),
                               hipMemcpyHostToDevice));
}

void launch_stage2d(int q, int precision, const StageArgs& a, hipStream_t s) {
    if (precision == CMCG_FP64) {
        if (q == 1) stage2d<double, 1>(a, s);
        else if (q == 2) stage2d<double, 2>(a, s);
        else stage2d<double, 3>(a, s);
    } else {
        if (q == 1) stage2d<float, 1>(a, s);
        else if (q == 2) stage2d<float, 2>(a, s);
        else stage2d<float, 3>(a, s);
    }
    check2();
}

void launch_to_field2d(int precision, int Np, const double* X, void* U, void* Ulo, int64_t n, int flipH,
                       hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_to_field2d<double>, dim3(grid2_for(n)), dim3(256), 0, s, X, (double*)U, nullptr, n, Np,
                           flipH);
    else
        hipLaunchKernelGGL(k_to_field2d<float>, dim3(grid2_for(n)), dim3(256), 0, s, X, (float*)U, (uint16_t*)Ulo, n,
                           Np, flipH);
    check2();
}

void launch_from_field2d(int precision, int Np, const void* U, const void* Ulo, double* Y, const double* sub,
                         int64_t n, int flipH, hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_from_field2d<double>, dim3(grid2_for(n)), dim3(256), 0, s, (const double*)U, nullptr, Y,
                           sub, n, Np, flipH);
    else
        hipLaunchKernelGGL(k_from_field2d<float>, dim3(grid2_for(n)), dim3(256), 0, s, (const float*)U,
                           (const uint16_t*)Ulo, Y, sub, n, Np, flipH);
    check2();
}

void launch_dot_batch2d(int q, const double* U, const double* V, const double* wE, const double* wH,
                        int64_t wstride, int64_t K, int B, double* partial, double* out_dev, hipStream_t s) {
    const dim3 grid(kDot2Blocks, (unsigned)B);
    if (q == 1)
        hipLaunchKernelGGL(k_dot2d_batch<1>, grid, dim3(kDot2Threads), 0, s, U, V, wE, wH, wstride, K, partial);
    else if (q == 2)
        hipLaunchKernelGGL(k_dot2d_batch<2>, grid, dim3(kDot2Threads), 0, s, U, V, wE, wH, wstride, K, partial);
    else
        hipLaunchKernelGGL(k_dot2d_batch<3>, grid, dim3(kDot2Threads), 0, s, U, V, wE, wH, wstride, K, partial);
    hipLaunchKernelGGL(k_dot2d_final_batch, dim3((unsigned)B), dim3(kDot2Threads), 0, s, partial, kDot2Blocks,
                       out_dev);
    check2();
}

int dot2d_partials() { return kDot2Blocks; }

void launch_dot2d(int q, const double* U, const double* V, const double* wE, const double* wH, int64_t K,
                  double* partial, double* out_dev, hipStream_t s) {
    if (q == 1)
        hipLaunchKernelGGL(k_dot2d<1>, dim3(kDot2Blocks), dim3(kDot2Threads), 0, s, U, V, wE, wH, K, partial);
    else if (q == 2)
        hipLaunchKernelGGL(k_dot2d<2>, dim3(kDot2Blocks), dim3(kDot2Threads), 0, s, U, V, wE, wH, K, partial);
    else
        hipLaunchKernelGGL(k_dot2d<3>, dim3(kDot2Blocks), dim3(kDot2Threads), 0, s, U, V, wE, wH, K, partial);
    hipLaunchKernelGGL(k_dot2d_final, dim3(1), dim3(kDot2Threads), 0, s, partial, kDot2Blocks, out_dev);
    check2();
}

}  // namespace cmcg
