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

#include <mutex>
#include <type_traits>

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
// face-node tables as packed bytes in 32-bit words: [fnode (4 Nfp) | nnode (24 Nfp)]
__host__ __device__ constexpr int ft_words(int q) { return (28 * ((q + 1) * (q + 2) / 2) + 3) / 4; }
__host__ __device__ constexpr int ft_off(int q) { return q <= 1 ? 0 : ft_off(q - 1) + ft_words(q - 1); }
constexpr int kFtTotal = ft_off(4);

__constant__ double cMat64[kMatTotal];
__constant__ float cMat32[kMatTotal];
// Per order q, one byte per entry packed into 32-bit words: the volume node of
// face node k of face f ([f][k], 4 Nfp entries), then the volume node of the
// neighbour's face node that sits at face node k of this side, for every
// neighbour face nf and vertex permutation perm ([nf][perm][k], 24 Nfp).
__constant__ uint32_t cFaceTab[kFtTotal];

template <typename T> __device__ __forceinline__ const T* mats();
template <> __device__ __forceinline__ const double* mats<double>() { return cMat64; }
template <> __device__ __forceinline__ const float* mats<float>() { return cMat32; }

constexpr int EPW = 10;  // elements per 64-lane workgroup (60 active column lanes)

// Row access of NP contiguous values with the widest vector type the row
// alignment allows (rows start at multiples of NP * sizeof(T) bytes).
template <typename T, int NP> struct Row {
    static constexpr int BYTES = NP * (int)sizeof(T);
    static constexpr int VEC = (BYTES % 16 == 0) ? 16 : (BYTES % 8 == 0 ? 8 : (int)sizeof(T));
    static constexpr int PER = VEC / (int)sizeof(T);
    using V = typename std::conditional<VEC == 16, float4, typename std::conditional<VEC == 8, float2, T>::type>::type;
    __device__ __forceinline__ static void load(const T* __restrict__ p, T (&r)[NP]) {
        const V* q = reinterpret_cast<const V*>(p);
#pragma unroll
        for (int c = 0; c < NP / PER; ++c) {
            V v = q[c];
            const T* t = reinterpret_cast<const T*>(&v);
#pragma unroll
            for (int u = 0; u < PER; ++u) r[c * PER + u] = t[u];
        }
    }
    __device__ __forceinline__ static void store(T* __restrict__ p, const T (&r)[NP]) {
        V* q = reinterpret_cast<V*>(p);
#pragma unroll
        for (int c = 0; c < NP / PER; ++c) {
            V v;
            T* t = reinterpret_cast<T*>(&v);
#pragma unroll
            for (int u = 0; u < PER; ++u) t[u] = r[c * PER + u];
            q[c] = v;
        }
    }
};

// Low parts of a compensated FP32 state, stored as bfloat16 (8 more significant
// bits than the FP32 high part; round to nearest even).
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint32_t h) { return __uint_as_float(h << 16); }

// s + e == a + b exactly (Knuth's branch-free two-sum, any magnitudes).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// NP bfloat16 low parts of one row (rows start at multiples of 2 NP bytes;
// NP is even for every order, so 4-byte words always line up).
template <int NP> struct RowH {
    static_assert(NP % 2 == 0, "bfloat16 rows need an even node count");
    static constexpr int PER = (2 * NP) % 8 == 0 ? 4 : 2;
    using V = typename std::conditional<PER == 4, uint2, uint32_t>::type;
    __device__ __forceinline__ static void load(const uint16_t* __restrict__ p, float (&r)[NP]) {
        const V* q = reinterpret_cast<const V*>(p);
#pragma unroll
        for (int c = 0; c < NP / PER; ++c) {
            V v = q[c];
            const uint32_t* w = reinterpret_cast<const uint32_t*>(&v);
#pragma unroll
            for (int u = 0; u < PER / 2; ++u) {
                r[c * PER + 2 * u] = from_bf16(w[u] & 0xffffu);
                r[c * PER + 2 * u + 1] = from_bf16(w[u] >> 16);
            }
        }
    }
    __device__ __forceinline__ static void store(uint16_t* __restrict__ p, const float (&r)[NP]) {
        V* q = reinterpret_cast<V*>(p);
#pragma unroll
        for (int c = 0; c < NP / PER; ++c) {
            V v;
            uint32_t* w = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
            for (int u = 0; u < PER / 2; ++u)
                w[u] = (uint32_t)to_bf16(r[c * PER + 2 * u]) | ((uint32_t)to_bf16(r[c * PER + 2 * u + 1]) << 16);
            q[c] = v;
        }
    }
};

// Logical workgroup index with consecutive indices on one XCD: the hardware
// hands workgroup b to XCD b % 8, so b -> (b % 8) * per + b / 8 keeps each
// XCD on a contiguous element range (its face neighbours stay in that XCD's
// L2).  The grid is a multiple of 8; indices past the element range exit.
__device__ __forceinline__ int64_t xcd_block(int64_t per) {
    const int64_t b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

// Arguments of this workgroup's member in a batched launch (grid.y = member):
// field, source and filter pointers move by whole members, the stage scalars
// come from the member table; returns false when the member is idle (CG
// converged, or all of its steps in this period already taken).
template <typename T>
__device__ __forceinline__ bool member_args(const StageArgs& in, StageArgs& a) {
    a = in;
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
    if (in.smask) a.smask = in.smask + (int64_t)b * ((in.K + EPW - 1) / EPW);
    return true;
}

// One chunk's stage input and geometry (16-byte coalesced loads, all issued
// before the first is consumed) and its connectivity codes; put() stores them
// in LDS with the stage-input rows padded to NP + 1.  NTH threads share the
// work (thread index `lane` < NTH).
template <typename T, int Q, int NTH = 64> struct ChunkIn {
    static constexpr int NP = Dim<Q>::NP;
    static constexpr int PV = 16 / (int)sizeof(T);  // values per load
    static constexpr int NY = (EPW * 6 * NP / PV + NTH - 1) / NTH, NG = (EPW * kGeo / PV + NTH - 1) / NTH;
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    static_assert((6 * NP) % PV == 0 && kGeo % PV == 0, "rows must split into 16-byte groups");
    static constexpr int NT = (ft_words(Q) + NTH - 1) / NTH;  // face-table words per thread
    V y[NY], g[NG];
    int cd;
    uint32_t tw[NT];
    __device__ __forceinline__ void fetch(const T* __restrict__ Y, const T* __restrict__ geo,
                                          const int* __restrict__ conn, int64_t e0, int ne, int lane) {
        const V* Y4 = reinterpret_cast<const V*>(Y + e0 * 6 * NP);
        const V* G4 = reinterpret_cast<const V*>(geo + e0 * kGeo);
#pragma unroll
        for (int i = 0; i < NT; ++i)
            if (lane + NTH * i < ft_words(Q)) tw[i] = cFaceTab[ft_off(Q) + lane + NTH * i];
#pragma unroll
        for (int i = 0; i < NY; ++i)
            if (lane + NTH * i < ne * 6 * NP / PV) y[i] = Y4[lane + NTH * i];
#pragma unroll
        for (int i = 0; i < NG; ++i)
            if (lane + NTH * i < ne * kGeo / PV) g[i] = G4[lane + NTH * i];
        cd = lane < ne * 4 ? conn[e0 * 4 + lane] : -3;
    }
    // keep: bit e clear stages element e's input as zero (an input mask, B P y)
    __device__ __forceinline__ void put(T* sY, T* sG, int* sC, uint8_t* sT, int ne, int lane,
                                        uint32_t keep = 0xffffffffu) const {
        uint32_t* sT4 = reinterpret_cast<uint32_t*>(sT);
#pragma unroll
        for (int i = 0; i < NT; ++i)
            if (lane + NTH * i < ft_words(Q)) sT4[lane + NTH * i] = tw[i];
#pragma unroll
        for (int i = 0; i < NY; ++i) {
            const int g4 = lane + NTH * i;
            if (g4 < ne * 6 * NP / PV) {
                const T* t = reinterpret_cast<const T*>(&y[i]);
#pragma unroll
                for (int u = 0; u < PV; ++u) {
                    const int v = PV * g4 + u;
                    sY[v + v / NP] = ((keep >> (v / (6 * NP))) & 1u) ? t[u] : T(0);
                }
            }
        }
        V* sG4 = reinterpret_cast<V*>(sG);
#pragma unroll
        for (int i = 0; i < NG; ++i)
            if (lane + NTH * i < ne * kGeo / PV) sG4[lane + NTH * i] = g[i];
        if (lane < ne * 4) sC[lane] = cd;
    }
};

// The face-node tables reach LDS with the chunk (ChunkIn): own face nodes
// [f][k], then the node of the neighbour's face seen from this side
// [nf][perm][k], one byte each.

// Flux items of a lane: item it = lane + 64 r is face node k = it / ne of
// element fe = it % ne (consecutive lanes on different elements); computed
// once per chunk (the divisor is the compile-time chunk size for full chunks).
template <int Q, int RF> struct FluxItems {
    int k[RF], fe[RF];
    bool on[RF];
    __device__ __forceinline__ void init(int ne, int lane) {
        constexpr int NFP = Dim<Q>::NFP;
#pragma unroll
        for (int r = 0; r < RF; ++r) {
            const int it = lane + 64 * r;
            on[r] = it < ne * NFP;
            const int kk = ne == EPW ? it / EPW : it / ne;
            k[r] = on[r] ? kk : 0;
            fe[r] = on[r] ? it - kk * ne : 0;
        }
    }
};

// Neighbour traces of one face for the flux items a lane owns: the
// connectivity code and the neighbour's node come from LDS.  A neighbour in
// the same chunk (about half of the interior faces of a cube-ordered mesh)
// is read from the staged tile later (loc = its LDS offset); the others are
// one round of global loads (cache-resident: neighbours are nearby in the
// element ordering).  Boundary items keep the code and build a ghost later.
template <typename T, int Q, int RF> struct TraceGather {
    static constexpr int RS = Dim<Q>::NP + 1;  // staged row stride
    T v[RF][6];
    int code[RF], loc[RF];
    // imask (nullable): input mask, one word per element block; a neighbour
    // whose bit (xor inv) is clear contributes a zero trace
    __device__ __forceinline__ void issue(const T* __restrict__ Y, const int* sC, const uint8_t* sT,
                                          const FluxItems<Q, RF>& itm, int f, int64_t e0, int ne,
                                          const uint32_t* __restrict__ imask = nullptr, int inv = 0) {
        constexpr int NP = Dim<Q>::NP, NFP = Dim<Q>::NFP;
#pragma unroll
        for (int r = 0; r < RF; ++r) {
            code[r] = -3;
            loc[r] = -1;
            if (itm.on[r]) {
                const int cd = sC[itm.fe[r] * 4 + f];
                code[r] = cd;
                if (cd >= 0) {
                    const int nn = sT[4 * NFP + (((cd >> 3) & 3) * 6 + (cd & 7)) * NFP + itm.k[r]];
                    const int64_t nb = cd >> 5;
                    const int64_t d = nb - e0;
                    if (d >= 0 && d < ne) {
                        loc[r] = (int)d * 6 * RS + nn;
                    } else if (imask && !(((imask[nb / EPW] >> (int)(nb % EPW)) & 1u) ^ (uint32_t)inv)) {
#pragma unroll
                        for (int cc = 0; cc < 6; ++cc) v[r][cc] = T(0);
                    } else {
                        const T* q = Y + nb * 6 * NP + nn;
#pragma unroll
                        for (int cc = 0; cc < 6; ++cc) v[r][cc] = q[cc * NP];
                    }
                }
            }
        }
    }
    // neighbour values of item r (after issue; sY = the staged chunk)
    __device__ __forceinline__ void values(const T* sY, int r, T (&Ep)[3], T (&Hp)[3]) const {
        if (loc[r] >= 0) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                Ep[cc] = sY[loc[r] + cc * RS];
                Hp[cc] = sY[loc[r] + (3 + cc) * RS];
            }
        } else {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                Ep[cc] = v[r][cc];
                Hp[cc] = v[r][3 + cc];
            }
        }
    }
};

// PIPE: request the next face's neighbour traces (and, before the last face,
// the update operands) one face ahead.  Without it every face gathers and
// consumes in turn, which needs fewer registers.
// MH: several-frequency problems (further source harmonics and filters);
// the single-frequency instantiation carries none of that code.
// LTSM: the local-time-stepping substep modes (LTS_FWD, LTS_ADJ) only.
template <typename T, int Q, bool PIPE, bool MH, bool LTSM = false>
__global__ __launch_bounds__(64) void k_stage(StageArgs args, int64_t per) {
    constexpr int NP = Dim<Q>::NP, NFP = Dim<Q>::NFP, NF4 = 4 * NFP;
    constexpr int RS = NP + 1;            // padded LDS row stride (bank spread)
    constexpr int MO = mat_off(Q);
    constexpr int LO = MO + 3 * NP * NP;  // LIFT [NP][NF4]
    constexpr int RF = (EPW * NFP + 63) / 64;  // flux items per lane and face
    constexpr int FS = 65;                     // flux tile row stride (bank spread)
    __shared__ T sY[EPW * 6 * RS];
    __shared__ T sF[NFP * FS];
    __shared__ T sG[EPW * kGeo];
    __shared__ int sC[EPW * 4];
    __shared__ __align__(4) uint8_t sT[4 * ft_words(Q)];

    StageArgs a;
    if (!member_args<T>(args, a)) return;  // uniform per workgroup
    int64_t blk = xcd_block(per);
    if (a.blist) {  // only the listed element blocks
        if (blk >= a.nblist) return;
        blk = a.blist[blk];
    }
    const int64_t e0 = blk * EPW;
    if (e0 >= a.K) return;
    const T* __restrict__ Y = (const T*)a.Y;
    const int lane = threadIdx.x;
    const int ne = (int)((a.K - e0) < EPW ? (a.K - e0) : EPW);
    const int64_t base = e0 * 6 * NP;

    // column ownership: lane = (element, component)
    const int el = lane / 6;
    const int c = lane - 6 * el;
    const bool act = el < ne;
    const int elc = act ? el : 0;
    const int row = elc * 6 + c;
    const int64_t grow = base + (int64_t)row * NP;
    const int mode = a.mode;
    constexpr bool COMP = std::is_same<T, float>::value;  // compensated state U + Ulo
    const bool needL = COMP && (mode == RK2_S2 || mode == RK4_S4);
    const bool needU =
        LTSM ? (mode == LTS_FWD || mode == LTS_ADJ) : (mode == RK2_S2 || mode == RK4_S2 || mode == RK4_S3 || needL);
    const bool needA = LTSM ? (mode == LTS_ADJ || (mode == LTS_FWD && a.Acc != nullptr))
                            : (mode == RK4_S2 || mode == RK4_S3 || mode == RK4_S4);

    const uint32_t keep = a.imask ? (a.imask[blk] ^ (a.imask_inv ? 0xffffffffu : 0u)) : 0xffffffffu;
    {
        ChunkIn<T, Q> in;
        in.fetch(Y, (const T*)a.geo, a.conn, e0, ne, lane);
        in.put(sY, sG, sC, sT, ne, lane, keep);
    }
    __syncthreads();
    // neighbour traces of face 0 in flight during the volume work
    FluxItems<Q, RF> itm;
    itm.init(ne, lane);
    TraceGather<T, Q, RF> cur, nxt;
    if (PIPE) cur.issue(Y, sC, sT, itm, 0, e0, ne, a.imask, a.imask_inv);

    // ---- volume term: D_a y per column, curl terms exchanged between lanes
    T y[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) y[j] = sY[row * RS + j];
    const T* gg = &sG[elc * kGeo];
    const int c3 = c < 3 ? c : c - 3;
    const int kp = c3 == 0 ? 2 : c3 - 1;  // (c3 + 2) % 3
    const int km = c3 == 2 ? 0 : c3 + 1;  // (c3 + 1) % 3
    const int sb = elc * 6 + (c < 3 ? 3 : 0);
    const int lane_p = sb + (c3 == 0 ? 2 : c3 - 1);  // sends +d_{m+1} V_{m+2} (m = c3)
    const int lane_m = sb + (c3 == 2 ? 0 : c3 + 1);  // sends -d_{m+2} V_{m+1}
    const T* Mt = mats<T>();
    // this column's contributions to the curl of its field:
    // pv = d_{c3+2} V_{c3} (to curl component c3+1), mv = -d_{c3+1} V_{c3} (to c3+2)
    T pv[NP], mv[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        pv[i] = T(0);
        mv[i] = T(0);
    }
#pragma unroll 1
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
    // E rows take -curl H, H rows +curl E
    const T sgn = c < 3 ? T(-1) : T(1);
    T acc[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = sgn * (__shfl(pv[i], lane_p) + __shfl(mv[i], lane_m));

    // ---- upwind flux and lift, one face at a time; the next face's
    // neighbour traces (and before the last face the update operands) are
    // requested before this face's work
    T up[NP], ap[NP];
    float lo[NP];
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
        if (PIPE) {
            if (f < 3) {
                nxt.issue(Y, sC, sT, itm, f + 1, e0, ne, a.imask, a.imask_inv);
            } else if (act) {
                if (needU) Row<T, NP>::load((const T*)a.U + grow, up);
                if (needA) Row<T, NP>::load((const T*)a.Acc + grow, ap);
                if constexpr (COMP)
                    if (needL) RowH<NP>::load((const uint16_t*)a.Ulo + grow, lo);
            }
        } else {
            cur.issue(Y, sC, sT, itm, f, e0, ne, a.imask, a.imask_inv);
        }
#pragma unroll
        for (int r = 0; r < RF; ++r) {
            if (!itm.on[r]) continue;
            const int k = itm.k[r];
            const int fe = itm.fe[r];
            const int own = sT[f * NFP + k];
            T Em[3], Hm[3], Ep[3], Hp[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                Em[cc] = sY[(fe * 6 + cc) * RS + own];
                Hm[cc] = sY[(fe * 6 + 3 + cc) * RS + own];
            }
            const int code = cur.code[r];
            if (code >= 0) {
                cur.values(sY, r, Ep, Hp);
            } else if (code == -1) {  // PEC ghost: E+ = -E-, H+ = H-
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    Ep[cc] = -Em[cc];
                    Hp[cc] = Hm[cc];
                }
            } else {  // impedance ghost (homogeneous part): zero exterior state
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    Ep[cc] = T(0);
                    Hp[cc] = T(0);
                }
            }
            const T* g = &sG[fe * kGeo + 9 + 7 * f];
            const T n0 = g[0], n1 = g[1], n2 = g[2];
            const T cE1 = g[3], cE2 = g[4], cH1 = g[5], cH2 = g[6];
            const T dE0 = Ep[0] - Em[0], dE1 = Ep[1] - Em[1], dE2 = Ep[2] - Em[2];
            const T dH0 = Hp[0] - Hm[0], dH1 = Hp[1] - Hm[1], dH2 = Hp[2] - Hm[2];
            const T ndE = n0 * dE0 + n1 * dE1 + n2 * dE2;
            const T ndH = n0 * dH0 + n1 * dH1 + n2 * dH2;
            const T xH0 = n1 * dH2 - n2 * dH1, xH1 = n2 * dH0 - n0 * dH2, xH2 = n0 * dH1 - n1 * dH0;
            const T xE0 = n1 * dE2 - n2 * dE1, xE1 = n2 * dE0 - n0 * dE2, xE2 = n0 * dE1 - n1 * dE0;
            T* o = &sF[k * FS + fe * 6];
            o[0] = cE1 * (dE0 - ndE * n0) - cE2 * xH0;
            o[1] = cE1 * (dE1 - ndE * n1) - cE2 * xH1;
            o[2] = cE1 * (dE2 - ndE * n2) - cE2 * xH2;
            o[3] = cH1 * (dH0 - ndH * n0) + cH2 * xE0;
            o[4] = cH1 * (dH1 - ndH * n1) + cH2 * xE1;
            o[5] = cH1 * (dH2 - ndH * n2) + cH2 * xE2;
        }
        __syncthreads();
        T fl[NFP];
#pragma unroll
        for (int k = 0; k < NFP; ++k) fl[k] = sF[k * FS + lane];
        __syncthreads();  // the tile is rewritten by the next face
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            T s = acc[i];
#pragma unroll
            for (int k = 0; k < NFP; ++k) s = fma(Mt[LO + i * NF4 + f * NFP + k], fl[k], s);
            acc[i] = s;
        }
        if (PIPE && f < 3) cur = nxt;
    }
    if (!act) return;
    if (!PIPE) {
        if (needU) Row<T, NP>::load((const T*)a.U + grow, up);
        if (needA) Row<T, NP>::load((const T*)a.Acc + grow, ap);
        if constexpr (COMP)
            if (needL) RowH<NP>::load((const uint16_t*)a.Ulo + grow, lo);
    }

    // ---- stage update on the lane's row
    const T inv = c < 3 ? gg[37] : gg[38];
    const T sig = c < 3 ? gg[39] : T(0);
    T kv[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) kv[i] = fma(inv, acc[i], -sig * y[i]);
    if (c < a.src_rows && (!a.smask || ((a.smask[blk] >> elc) & 1u))) {
        T sr[NP], si[NP];
        Row<T, NP>::load((const T*)a.Sre + grow, sr);
        Row<T, NP>::load((const T*)a.Sim + grow, si);
        const T scos = (T)a.scos, ssin = (T)a.ssin;
#pragma unroll
        for (int i = 0; i < NP; ++i) kv[i] += scos * sr[i] - ssin * si[i];
#pragma unroll 1
        // further harmonics of a several-frequency source (single launches, so the
        // kernel arguments hold the tables; indexing the local copy put it in scratch)
        for (int h = 1; MH && h < a.nharm; ++h) {
            Row<T, NP>::load((const T*)args.Sre + h * args.hstride + grow, sr);
            Row<T, NP>::load((const T*)args.Sim + h * args.hstride + grow, si);
            const T hc = (T)args.hcos[h], hs = (T)args.hsin[h];
#pragma unroll
            for (int i = 0; i < NP; ++i) kv[i] += hc * sr[i] - hs * si[i];
        }
    }
    const T cy = (T)a.cy, ca = (T)a.ca, cu = (T)a.cu;
    T o1[NP], o2[NP];
    if constexpr (LTSM) {
        if (mode == LTS_CHAIN) {
            auto on = [&](const uint32_t* m, int inv) {
                return !m || ((((m[blk] >> elc) & 1u) ^ (uint32_t)inv) != 0);
            };
            const bool oa = on(a.lmask, a.linv), ob = on(a.lmaskB, a.linvB), oc = on(a.lmaskC, a.linvC);
#pragma unroll
            for (int i = 0; i < NP; ++i) o1[i] = oa ? kv[i] : T(0);
            T x[NP];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const bool use = j == 0 ? ob : j == 1 ? oc : true;
                if (!args.lw[j] || !use) continue;
                Row<T, NP>::load((const T*)args.lw[j] + grow, x);
#pragma unroll
                for (int i = 0; i < NP; ++i) o1[i] += x[i];
            }
            Row<T, NP>::store((T*)a.Uout + grow, o1);
        } else if (mode == LTS_FWD) {
            T w[NP];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j >= a.lnw) break;
                Row<T, NP>::load((const T*)args.lw[j] + grow, w);
                const T cj = (T)args.lcw[j];
#pragma unroll
                for (int i = 0; i < NP; ++i) kv[i] = fma(cj, w[i], kv[i]);
            }
            const T le = (T)a.le, lf = (T)a.lf;
            const bool hasA = a.Acc != nullptr;
            if (a.Ynext) {
#pragma unroll
                for (int i = 0; i < NP; ++i) o1[i] = fma(cy, kv[i], hasA ? fma(le, ap[i], up[i]) : up[i]);
                Row<T, NP>::store((T*)a.Ynext + grow, o1);
            }
            if (a.Uout) {
#pragma unroll
                for (int i = 0; i < NP; ++i) o2[i] = hasA ? fma(ca, kv[i], lf * ap[i]) : ca * kv[i];
                Row<T, NP>::store((T*)a.Uout + grow, o2);
            }
        } else {
            const bool on = ((a.lmask[blk] >> elc) & 1u) != 0;
            if (on) {
                T w[NP];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j >= a.lnw) break;
                    T* wj = (T*)args.lw[j] + grow;
                    if (a.linit) {
#pragma unroll
                        for (int i = 0; i < NP; ++i) w[i] = T(0);
                    } else {
                        Row<T, NP>::load(wj, w);
                    }
                    const T cj = (T)args.lcw[j];
#pragma unroll
                    for (int i = 0; i < NP; ++i) w[i] = fma(cj, y[i], w[i]);
                    Row<T, NP>::store(wj, w);
                }
            }
            const T le = (T)a.le, lf = (T)a.lf;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const T A = on ? kv[i] : T(0);
                o1[i] = up[i] + A;
                o2[i] = fma(lf, A, le * ap[i]);
            }
            Row<T, NP>::store((T*)a.Uout + grow, o1);
            if (a.Ynext) Row<T, NP>::store((T*)a.Ynext + grow, o2);
            if (a.lz) {  // the next substep's starting state and first stage vector
                Row<T, NP>::store((T*)a.lz + grow, o1);
                const T kc = (T)a.lkc;
#pragma unroll
                for (int i = 0; i < NP; ++i) o2[i] = kc * o1[i];
                Row<T, NP>::store((T*)a.lk + grow, o2);
            }
        }
    } else {
        switch (mode) {
            case RK2_S1:
#pragma unroll
                for (int i = 0; i < NP; ++i) o1[i] = fma(cy, kv[i], y[i]);
                Row<T, NP>::store((T*)a.Ynext + grow, o1);
                break;
            case RK2_S2:
                if constexpr (COMP) {
                    float e[NP];
#pragma unroll
                    for (int i = 0; i < NP; ++i) two_sum(up[i], fma(cu, kv[i], lo[i]), o1[i], e[i]);
                    Row<T, NP>::store((T*)a.Uout + grow, o1);
                    RowH<NP>::store((uint16_t*)a.Ulo + grow, e);
                } else {
#pragma unroll
                    for (int i = 0; i < NP; ++i) o1[i] = fma(cu, kv[i], up[i]);
                    Row<T, NP>::store((T*)a.Uout + grow, o1);
                }
                break;
            case RK4_S1:
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    o1[i] = fma(cy, kv[i], y[i]);
                    o2[i] = COMP ? ca * kv[i] : fma(ca, kv[i], y[i]);
                }
                Row<T, NP>::store((T*)a.Ynext + grow, o1);
                Row<T, NP>::store((T*)a.Acc + grow, o2);
                break;
            case RK4_S2:
            case RK4_S3:
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    o1[i] = fma(cy, kv[i], up[i]);
                    o2[i] = fma(ca, kv[i], ap[i]);
                }
                Row<T, NP>::store((T*)a.Ynext + grow, o1);
                Row<T, NP>::store((T*)a.Acc + grow, o2);
                break;
            case RK4_S4:
                if constexpr (COMP) {
                    float e[NP];
#pragma unroll
                    for (int i = 0; i < NP; ++i) two_sum(up[i], fma(cu, kv[i], ap[i]) + lo[i], o1[i], e[i]);
                    Row<T, NP>::store((T*)a.Uout + grow, o1);
                    RowH<NP>::store((uint16_t*)a.Ulo + grow, e);
                } else {
#pragma unroll
                    for (int i = 0; i < NP; ++i) o1[i] = fma(cu, kv[i], ap[i]);
                    Row<T, NP>::store((T*)a.Uout + grow, o1);
                }
                break;
            default:
                Row<T, NP>::store((T*)a.Kout + grow, kv);
                break;
        }
    }
    if (a.filter) {
        // F += fa * U + fb * k on the lane's row (U is the stage input here)
        double* fr = a.Fre + grow;
        double* fi = a.Fim + grow;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const double ud = (double)y[i], kd = (double)kv[i];
            fr[i] += a.fa_re * ud + a.fb_re * kd;
            fi[i] += a.fa_im * ud + a.fb_im * kd;
        }
#pragma unroll 1
        for (int h = 1; MH && h < a.nharm; ++h) {
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

// ---------------------------------------------------------------------------
// FP32 stage kernel on the matrix cores (q = 2, 3).
//
// Per 64-lane workgroup (10 elements, columns n = element * 6 + s):
//   volume:  C[i][n] = sum_{a,j} D_a[i][j] W_a[j][n],  W_a = sgn (grad xi_a x V)_m,
//            V = H for s < 3 (E rows, sgn = -1), V = E for s >= 3 (sgn = +1),
//            m = s mod 3 -- i.e. curl V = sum_a D_a (grad xi_a x V) for an affine
//            element, so the product already is the curl column;
//   lift:    C[i][n] += sum_{f,k} LIFT[i][f Nfp + k] flux_f[k][n], face by face;
// with v_mfma_f32_16x16x4f32: A = the reference matrices, held as register
// fragments (lane l holds A[l % 16][l / 16] of each 16x4 block, read once from a
// lane-ordered table), B = W or flux values from LDS, D rows per Mfma<T>::row.
// The volume's K steps are axis-major: step ks covers axis a = ks / NJ and
// nodes j = 4 (ks % NJ) + (0..3), so a lane meets the same nodes j = l/16 + 4 t
// on every axis and reads them once.  Rows i >= Np and nodes j >= Np carry
// zero A fragments.
template <int Q> struct MfmaDim {
    static constexpr int NP = Dim<Q>::NP, NFP = Dim<Q>::NFP;
    static constexpr int MT = (NP + 15) / 16;        // 16-row output tiles
    static constexpr int NJ = (NP + 3) / 4;          // K steps per axis of the volume product
    static constexpr int KSV = 3 * NJ;               // K steps of the volume product
    static constexpr int KSF = (NFP + 3) / 4;        // K steps per face of the lift
    static constexpr int NFRAG = MT * KSV + 4 * MT * KSF;
};
__host__ __device__ constexpr int frag_off(int q) {
    return q <= 2 ? 0 : frag_off(q - 1) + 64 * MfmaDim<2>::NFRAG;
}
constexpr int kFragTotal = 64 * (MfmaDim<2>::NFRAG + MfmaDim<3>::NFRAG);
__device__ float gFrag[kFragTotal];
__device__ double gFrag64[kFragTotal];
template <typename T> __device__ __forceinline__ const T* frags();
template <> __device__ __forceinline__ const float* frags<float>() { return gFrag; }
template <> __device__ __forceinline__ const double* frags<double>() { return gFrag64; }

// One 16x16x4 matrix-core product D = A B + C in the field precision:
// v_mfma_f32_16x16x4f32 or v_mfma_f64_16x16x4f64.  Both take A[l % 16][l / 16]
// and B[l / 16][l % 16] from lane l; their accumulators differ: register r of
// lane l holds D[row(l / 16, r)][l % 16] with row = 4 (l / 16) + r for FP32
// and 4 r + l / 16 for FP64 (measured with one-hot operands; checked against
// numpy through cmcg_debug_mfma).
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q4, int r) { return 4 * q4 + r; }
};
template <> struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q4, int r) { return 4 * r + q4; }
};

template <typename T, int Q, int NB = 1>
struct MfmaShared {
    static constexpr int NP = Dim<Q>::NP, NFP = Dim<Q>::NFP;
    static constexpr int RS = NP + 1;
    static constexpr int KF = 4 * MfmaDim<Q>::KSF;
    static constexpr int FS = 65;  // flux tile row stride: the face nodes of one column fall in different banks
    T sY[EPW * 6 * RS];       // stage input, rows (element, component) padded to NP + 1
    T sF[NB * KF * FS];       // NB flux tiles [face node][column], rows >= NFP stay zero
    T sG[EPW * kGeo];         // geometry of the chunk
    int sC[EPW * 4];          // connectivity codes of the chunk
    uint8_t sT[4 * ft_words(Q)];  // own face nodes [f][k], then neighbour face nodes [nf][perm][k]
};

// Operands of the coalesced update pass (16-byte groups v = lane + NTH t of
// the chunk: 4 FP32 or 2 FP64 values), all requested before the pass
// computes: r0 = U (modes that combine with the state) or the stage input
// (stage-1 modes, filter), r1 = Acc, r2 = the bfloat16 low parts (FP32).
template <typename T, int Q, int NTH = 64, bool LTSM = false> struct MfmaUpdateIn {
    static constexpr int PV = 16 / (int)sizeof(T);
    static constexpr bool COMP = std::is_same<T, float>::value;  // compensated state U + Ulo
    using V = typename std::conditional<COMP, float4, double2>::type;
    static constexpr int NIT = (EPW * 6 * Dim<Q>::NP / PV + NTH - 1) / NTH;
    V r0[NIT], r1[NIT];
    uint2 r2[COMP ? NIT : 1];
    __device__ __forceinline__ void fetch(const StageArgs& a, int64_t base, int nvv, int lane) {
        const int mode = a.mode;
        // LTS_FWD reads U (and Acc when given), LTS_ADJ the stage input and Acc
        const bool s1 = LTSM ? mode == LTS_ADJ : mode == RK2_S1 || mode == RK4_S1 || (mode == RHS && a.filter);
        // FP64 stage 4 forms U = Acc + cu k without the state
        const bool needU =
            LTSM ? mode == LTS_FWD : mode == RK2_S2 || mode == RK4_S2 || mode == RK4_S3 || (COMP && mode == RK4_S4);
        const bool needA = LTSM ? (mode == LTS_ADJ || (mode == LTS_FWD && a.Acc != nullptr))
                                : (mode == RK4_S2 || mode == RK4_S3 || mode == RK4_S4);
        const bool needL = !LTSM && COMP && (mode == RK2_S2 || mode == RK4_S4);
        const T* src0 = needU ? (const T*)a.U : (const T*)a.Y;
#pragma unroll
        for (int t = 0; t < NIT; ++t) {
            const int vv = lane + NTH * t;
            if (vv >= nvv) continue;
            const int64_t gi = base + PV * vv;
            if (s1 || needU) r0[t] = *reinterpret_cast<const V*>(src0 + gi);
            if (needA) r1[t] = *reinterpret_cast<const V*>((const T*)a.Acc + gi);
            if constexpr (COMP)
                if (needL) r2[t] = *reinterpret_cast<const uint2*>((const uint16_t*)a.Ulo + gi);
        }
    }
};

// PIPE: the next face's neighbour traces are requested before this face's
// flux (more registers, the gather latency hides behind the lift).
// W: waves per workgroup.  W = 2 gives each wave half the output tiles: P3
// one of its two 16-row tiles (both waves build the same B operands), P2 two
// of the four 16-column tiles (each wave builds only its own); each runs half
// the MFMAs, the flux items and the update pass are shared by 128 threads.  A
// block's dependent chain gets shorter at 6 waves per SIMD (76 registers),
// which pays where the launch ends in a partial round of workgroups.  Register
// allocation is held to 4 waves per SIMD (128 registers; the FP32 LDS tiles
// of MfmaShared<float, 3> stay under 10 KB so 16 workgroups fit a compute
// unit).  Requesting the update operands earlier (with the staging loads, or
// before the last face) was measured slower: the registers cost occupancy
// (P2) or spill (P3).  T = double runs the same data flow on
// v_mfma_f64_16x16x4f64 with FP64 fields (no compensated state).
// EAGER: the neighbour traces of all four faces are requested right after
// the staging (four faces' loads in flight during the volume product instead
// of one), and faces alternate between two flux tiles, so a face needs one
// barrier instead of two.  CSPLIT (P3, two waves): the waves split the output
// by column tiles, each building only its own B operands and running both
// row tiles.  W = 4: each wave one row tile and two column tiles (P3) or one
// column tile (P2), a quarter of the MFMAs and fewer registers per wave.
template <typename T, int Q, bool PIPE, bool MH, int W, bool EAGER = false, bool CSPLIT = false, bool LTSM = false>
__global__ __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (W == 4 ? (EAGER ? 5 : Q == 3 ? 7 : 8) : W == 1 || (EAGER && Q == 3) ? 4 : (EAGER || CSPLIT ? 5 : 6))
                                                   : (W == 4 ? (EAGER ? 2 : 4) : W == 1 || EAGER || CSPLIT ? 2 : 3), 8)))
void k_stage_mfma(StageArgs args, int64_t per) {
    using MD = MfmaDim<Q>;
    using acc_t = typename Mfma<T>::acc_t;
    constexpr bool COMP = std::is_same<T, float>::value;  // compensated state U + Ulo
    constexpr int NP = MD::NP, NFP = MD::NFP, MT = MD::MT, KSV = MD::KSV, KSF = MD::KSF;
    constexpr int RS = NP + 1;
    constexpr int KF = 4 * KSF;
    constexpr int NTH = 64 * W;                      // threads of the workgroup
    constexpr int RF = (EPW * NFP + NTH - 1) / NTH;  // flux items per thread and face
    // two waves split the output tiles: by rows when there are two row tiles
    // (P3, unless CSPLIT), by the four 16-column tiles otherwise; four waves
    // split by rows (P3) and by columns
    static_assert(W == 1 || W == 2 || W == 4, "one, two or four waves per block");
    constexpr bool ROWS = (W == 2 && MT == 2 && !CSPLIT) || (W == 4 && MT == 2);
    constexpr bool COLS = (W == 2 && (MT == 1 || CSPLIT)) || W == 4;
    constexpr int NB = EAGER ? 2 : 1;  // flux tiles
    using Sh = MfmaShared<T, Q, NB>;
    constexpr int MW = ROWS ? 1 : MT;  // output row tiles of one wave
    constexpr int CWAVES = COLS ? (ROWS ? W / 2 : W) : 1;  // waves across the column tiles
    constexpr int NW = 4 / CWAVES;                          // output column tiles of one wave
    static_assert(W == 1 || ((ROWS || COLS) && RF == 1), "several waves per block need one flux item per thread");
    __shared__ Sh sh;

    StageArgs a;
    if (!member_args<T>(args, a)) return;  // uniform per workgroup
    int64_t blk = xcd_block(per);
    if (a.blist) {  // only the listed element blocks
        if (blk >= a.nblist) return;
        blk = a.blist[blk];
    }
    const int64_t e0 = blk * EPW;
    if (e0 >= a.K) return;  // uniform per workgroup
    const T* __restrict__ Y = (const T*)a.Y;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int mt0 = ROWS ? (wave & 1) : 0;                           // first output row tile of this wave
    const int nt0 = COLS ? NW * (ROWS ? wave >> 1 : wave) : 0;  // first output column tile of this wave
    const int ne = (int)((a.K - e0) < EPW ? (a.K - e0) : EPW);
    const int64_t base = e0 * 6 * NP;
    constexpr int PV = 16 / (int)sizeof(T);  // values per 16-byte group
    const int nvv = ne * 6 * NP / PV;        // 16-byte groups of the chunk (6 NP ne is a multiple of 4)

    // matrix fragments (coalesced: fragment-major, lane-minor); lift
    // fragments one face at a time, requested one face ahead
    const T* fr = frags<T>() + frag_off(Q);
    T afV[MW][KSV], afL[MW][KSF], afN[MW][KSF];
    auto lift_frags = [&](int f, T (&d)[MW][KSF]) {
#pragma unroll
        for (int mt = 0; mt < MW; ++mt)
#pragma unroll
            for (int ks = 0; ks < KSF; ++ks) d[mt][ks] = fr[(MT * KSV + (f * MT + mt + mt0) * KSF + ks) * 64 + lane];
    };

    // ---- staging: chunk fields, geometry, connectivity, face-node tables;
    // the volume and face-0 lift fragments are requested right behind the
    // chunk's loads, so their latency hides behind the staging wait
    const uint32_t keep = a.imask ? (a.imask[blk] ^ (a.imask_inv ? 0xffffffffu : 0u)) : 0xffffffffu;
    {
        ChunkIn<T, Q, NTH> in;
        in.fetch(Y, (const T*)a.geo, a.conn, e0, ne, tid);
#pragma unroll
        for (int mt = 0; mt < MW; ++mt)
#pragma unroll
            for (int ks = 0; ks < KSV; ++ks) afV[mt][ks] = fr[((mt + mt0) * KSV + ks) * 64 + lane];
        lift_frags(0, afL);
        for (int v = tid; v < NB * KF * Sh::FS; v += NTH) sh.sF[v] = T(0);
        in.put(sh.sY, sh.sG, sh.sC, sh.sT, ne, tid, keep);
    }
    __syncthreads();

    // face 0's neighbour traces (EAGER: every face's) in flight during the volume product
    FluxItems<Q, RF> itm;
    itm.init(ne, tid);
    TraceGather<T, Q, RF> cur, nxt;
    TraceGather<T, Q, RF> all[EAGER ? 4 : 1];
    if constexpr (EAGER) {
#pragma unroll
        for (int f = 0; f < 4; ++f) all[f].issue(Y, sh.sC, sh.sT, itm, f, e0, ne, a.imask, a.imask_inv);
    } else {
        cur.issue(Y, sh.sC, sh.sT, itm, 0, e0, ne, a.imask, a.imask_inv);
    }

    const int q4 = lane >> 4;   // K row within a 4-row block / output row group
    const int l16 = lane & 15;  // output column within a 16-column tile
    acc_t acc[MW][NW];
#pragma unroll
    for (int mt = 0; mt < MW; ++mt)
#pragma unroll
        for (int nt = 0; nt < NW; ++nt) acc[mt][nt] = acc_t{T(0), T(0), T(0), T(0)};

    // ---- volume product: B[(a, j)][n] = sgn (g_a[m1] V_m2(j) - g_a[m2] V_m1(j));
    // padded columns read element 0 (their results are never stored)
#pragma unroll
    for (int nt = 0; nt < NW; ++nt) {
        const int n = (nt + nt0) * 16 + l16;
        const int e = n < 6 * ne ? n / 6 : 0;
        const int s = n - 6 * (n / 6);
        const int m = s < 3 ? s : s - 3;
        const int m1 = m == 2 ? 0 : m + 1, m2 = m == 0 ? 2 : m - 1;  // (m+1)%3, (m+2)%3
        const int vb = e * 6 + (s < 3 ? 3 : 0);
        const T sgn = s < 3 ? T(-1) : T(1);
        const T* gE = &sh.sG[e * kGeo];
        T g1[3], g2[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            g1[ax] = sgn * gE[3 * ax + m1];
            g2[ax] = sgn * gE[3 * ax + m2];
        }
        const T* v1 = &sh.sY[(vb + m1) * RS];
        const T* v2 = &sh.sY[(vb + m2) * RS];
        constexpr int NJ = MD::NJ;
        T r1[NJ], r2[NJ];
#pragma unroll
        for (int t = 0; t < NJ; ++t) {
            const int j = q4 + 4 * t;
            const bool in = NP % 4 == 0 || j < NP;  // j >= Np: zero fragment, zero operand
            r1[t] = in ? v1[in ? j : 0] : T(0);
            r2[t] = in ? v2[in ? j : 0] : T(0);
        }
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
#pragma unroll
            for (int t = 0; t < NJ; ++t) {
                const T b = g1[ax] * r2[t] - g2[ax] * r1[t];
#pragma unroll
                for (int mt = 0; mt < MW; ++mt)
                    acc[mt][nt] = Mfma<T>::mma(afV[mt][ax * NJ + t], b, acc[mt][nt]);
            }
    }

    // ---- upwind flux and lift, one face at a time
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (!EAGER && PIPE && f < 3) nxt.issue(Y, sh.sC, sh.sT, itm, f + 1, e0, ne, a.imask, a.imask_inv);
        if (f < 3) lift_frags(f + 1, afN);
        T* tile = sh.sF + (EAGER ? (f & 1) * KF * Sh::FS : 0);
        const TraceGather<T, Q, RF>& gat = EAGER ? all[f] : cur;
#pragma unroll
        for (int r = 0; r < RF; ++r) {
            if (!itm.on[r]) continue;
            const int k = itm.k[r];
            const int fe = itm.fe[r];
            const int own = sh.sT[f * NFP + k];
            T Em[3], Hm[3], Ep[3], Hp[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                Em[cc] = sh.sY[(fe * 6 + cc) * RS + own];
                Hm[cc] = sh.sY[(fe * 6 + 3 + cc) * RS + own];
            }
            const int code = gat.code[r];
            if (code >= 0) {
                gat.values(sh.sY, r, Ep, Hp);
            } else if (code == -1) {  // PEC ghost: E+ = -E-, H+ = H-
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    Ep[cc] = -Em[cc];
                    Hp[cc] = Hm[cc];
                }
            } else {  // impedance ghost (homogeneous part): zero exterior state
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    Ep[cc] = T(0);
                    Hp[cc] = T(0);
                }
            }
            const T* g = &sh.sG[fe * kGeo + 9 + 7 * f];
            const T n0 = g[0], n1 = g[1], n2 = g[2];
            const T cE1 = g[3], cE2 = g[4], cH1 = g[5], cH2 = g[6];
            const T dE0 = Ep[0] - Em[0], dE1 = Ep[1] - Em[1], dE2 = Ep[2] - Em[2];
            const T dH0 = Hp[0] - Hm[0], dH1 = Hp[1] - Hm[1], dH2 = Hp[2] - Hm[2];
            const T ndE = n0 * dE0 + n1 * dE1 + n2 * dE2;
            const T ndH = n0 * dH0 + n1 * dH1 + n2 * dH2;
            const T xH0 = n1 * dH2 - n2 * dH1, xH1 = n2 * dH0 - n0 * dH2, xH2 = n0 * dH1 - n1 * dH0;
            const T xE0 = n1 * dE2 - n2 * dE1, xE1 = n2 * dE0 - n0 * dE2, xE2 = n0 * dE1 - n1 * dE0;
            T* o = &tile[k * Sh::FS + fe * 6];
            o[0] = cE1 * (dE0 - ndE * n0) - cE2 * xH0;
            o[1] = cE1 * (dE1 - ndE * n1) - cE2 * xH1;
            o[2] = cE1 * (dE2 - ndE * n2) - cE2 * xH2;
            o[3] = cH1 * (dH0 - ndH * n0) + cH2 * xE0;
            o[4] = cH1 * (dH1 - ndH * n1) + cH2 * xE1;
            o[5] = cH1 * (dH2 - ndH * n2) + cH2 * xE2;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KSF; ++ks) {
            T b[NW];
#pragma unroll
            for (int nt = 0; nt < NW; ++nt) b[nt] = tile[(ks * 4 + q4) * Sh::FS + (nt + nt0) * 16 + l16];
#pragma unroll
            for (int nt = 0; nt < NW; ++nt)
#pragma unroll
                for (int mt = 0; mt < MW; ++mt)
                    acc[mt][nt] = Mfma<T>::mma(afL[mt][ks], b[nt], acc[mt][nt]);
        }
        // one tile: it is rewritten by the next face; two tiles: the next face
        // writes the other one, and the face after it only once every thread
        // has passed the next face's barrier (so has finished this lift)
        if (!EAGER) __syncthreads();
        if (f < 3) {
            if (!EAGER) {
                if (!PIPE) nxt.issue(Y, sh.sC, sh.sT, itm, f + 1, e0, ne, a.imask, a.imask_inv);
                cur = nxt;
            }
#pragma unroll
            for (int mt = 0; mt < MW; ++mt)
#pragma unroll
                for (int ks = 0; ks < KSF; ++ks) afL[mt][ks] = afN[mt][ks];
        }
    }

    // ---- scaled right-hand side (1/eps or 1/mu, conductivity) into the
    // staging tile, in place: every value is read and written by one lane
#pragma unroll
    for (int nt = 0; nt < NW; ++nt) {
        const int n = (nt + nt0) * 16 + l16;
        if (n >= 6 * ne) continue;
        const int e = n / 6;
        const int s = n - 6 * e;
        const T inv = s < 3 ? sh.sG[e * kGeo + 37] : sh.sG[e * kGeo + 38];
        const T sig = s < 3 ? sh.sG[e * kGeo + 39] : T(0);
#pragma unroll
        for (int mt = 0; mt < MW; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = (mt + mt0) * 16 + Mfma<T>::row(q4, r);
                if (i < NP) {
                    T* p = &sh.sY[n * RS + i];
                    *p = fma(inv, acc[mt][nt][r], -sig * *p);
                }
            }
    }
    __syncthreads();

    // ---- stage update: one coalesced pass over the chunk's contiguous rows
    const int mode = a.mode;
    const T scos = (T)a.scos, ssin = (T)a.ssin;
    const T cy = (T)a.cy, ca = (T)a.ca, cu = (T)a.cu;
    // elements whose source is zero (and H rows of an interior source) read none
    const uint32_t sm = a.smask ? a.smask[blk] : 0xffffffffu;
    auto takes_src = [&](int row) { return row - 6 * (row / 6) < a.src_rows && ((sm >> (row / 6)) & 1u); };
    using UIn = MfmaUpdateIn<T, Q, NTH, LTSM>;
    using V = typename UIn::V;
    UIn upd;
    upd.fetch(a, base, nvv, tid);
    auto ldv = [](const void* p, int64_t o, T (&r)[PV]) {
        const V v = *reinterpret_cast<const V*>((const T*)p + o);
        const T* t = reinterpret_cast<const T*>(&v);
#pragma unroll
        for (int u = 0; u < PV; ++u) r[u] = t[u];
    };
#pragma unroll
    for (int t = 0; t < UIn::NIT; ++t) {
        const int vv = tid + NTH * t;
        if (vv >= nvv) continue;
        const int v = PV * vv;
        const int64_t gi = base + v;
        T kv[PV];
#pragma unroll
        for (int u = 0; u < PV; ++u) kv[u] = sh.sY[v + u + (v + u) / NP];
        if (a.src_rows > 0 && (takes_src(v / NP) || takes_src((v + PV - 1) / NP))) {
            T srv[PV], siv[PV];
            ldv(a.Sre, gi, srv);
            ldv(a.Sim, gi, siv);
#pragma unroll
            for (int u = 0; u < PV; ++u) {
                const int row = (v + u) / NP;
                if (takes_src(row)) kv[u] += scos * srv[u] - ssin * siv[u];
            }
#pragma unroll 1
            // further harmonics (tables read from the kernel arguments, as in k_stage)
            for (int h = 1; MH && h < a.nharm; ++h) {
                T hrv[PV], hiv[PV];
                ldv(args.Sre, h * args.hstride + gi, hrv);
                ldv(args.Sim, h * args.hstride + gi, hiv);
                const T hc = (T)args.hcos[h], hs = (T)args.hsin[h];
#pragma unroll
                for (int u = 0; u < PV; ++u) {
                    const int row = (v + u) / NP;
                    if (takes_src(row)) kv[u] += hc * hrv[u] - hs * hiv[u];
                }
            }
        }
        T x0[PV], x1[PV];  // U (or Y in stage-1 modes), Acc
        {
            const T* p0 = reinterpret_cast<const T*>(&upd.r0[t]);
            const T* p1 = reinterpret_cast<const T*>(&upd.r1[t]);
#pragma unroll
            for (int u = 0; u < PV; ++u) {
                x0[u] = p0[u];
                x1[u] = p1[u];
            }
        }
        T lo[PV];
        if constexpr (COMP) {
            if (mode == RK2_S2 || mode == RK4_S4) {
                lo[0] = from_bf16(upd.r2[t].x & 0xffffu);
                lo[1] = from_bf16(upd.r2[t].x >> 16);
                lo[2] = from_bf16(upd.r2[t].y & 0xffffu);
                lo[3] = from_bf16(upd.r2[t].y >> 16);
            }
        }
        auto stv = [&](void* p, const T (&o)[PV]) {
            V w;
            T* q = reinterpret_cast<T*>(&w);
#pragma unroll
            for (int u = 0; u < PV; ++u) q[u] = o[u];
            *reinterpret_cast<V*>((T*)p + gi) = w;
        };
        T o1[PV], o2[PV];
        if constexpr (LTSM) {
            if (mode == LTS_CHAIN) {
                const int el = v / NP / 6;  // a 16-byte group never straddles an element
                auto on = [&](const uint32_t* m, int inv) {
                    return !m || ((((m[blk] >> el) & 1u) ^ (uint32_t)inv) != 0);
                };
                const bool oa = on(a.lmask, a.linv), ob = on(a.lmaskB, a.linvB), oc = on(a.lmaskC, a.linvC);
#pragma unroll
                for (int u = 0; u < PV; ++u) o1[u] = oa ? kv[u] : T(0);
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const bool use = j == 0 ? ob : j == 1 ? oc : true;
                    if (!args.lw[j] || !use) continue;
                    T x[PV];
                    ldv(args.lw[j], gi, x);
#pragma unroll
                    for (int u = 0; u < PV; ++u) o1[u] += x[u];
                }
                stv(a.Uout, o1);
            } else if (mode == LTS_FWD) {  // x0 = U, x1 = Acc
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j >= a.lnw) break;
                    T w[PV];
                    ldv(args.lw[j], gi, w);
                    const T cj = (T)args.lcw[j];
#pragma unroll
                    for (int u = 0; u < PV; ++u) kv[u] = fma(cj, w[u], kv[u]);
                }
                const T le = (T)a.le, lf = (T)a.lf;
                const bool hasA = a.Acc != nullptr;
                if (a.Ynext) {
#pragma unroll
                    for (int u = 0; u < PV; ++u) o1[u] = fma(cy, kv[u], hasA ? fma(le, x1[u], x0[u]) : x0[u]);
                    stv(a.Ynext, o1);
                }
                if (a.Uout) {
#pragma unroll
                    for (int u = 0; u < PV; ++u) o2[u] = hasA ? fma(ca, kv[u], lf * x1[u]) : ca * kv[u];
                    stv(a.Uout, o2);
                }
            } else {  // x0 = the stage input kcur, x1 = Acc
                // a 16-byte group never straddles an element (6 NP is a multiple of 4)
                const bool on = ((a.lmask[blk] >> (v / NP / 6)) & 1u) != 0;
                if (on) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (j >= a.lnw) break;
                        T w[PV];
                        if (a.linit) {
#pragma unroll
                            for (int u = 0; u < PV; ++u) w[u] = T(0);
                        } else {
                            ldv(args.lw[j], gi, w);
                        }
                        const T cj = (T)args.lcw[j];
#pragma unroll
                        for (int u = 0; u < PV; ++u) w[u] = fma(cj, x0[u], w[u]);
                        stv(const_cast<void*>(args.lw[j]), w);
                    }
                }
                T z[PV];
                ldv(a.U, gi, z);
                const T le = (T)a.le, lf = (T)a.lf;
#pragma unroll
                for (int u = 0; u < PV; ++u) {
                    const T A = on ? kv[u] : T(0);
                    o1[u] = z[u] + A;
                    o2[u] = fma(lf, A, le * x1[u]);
                }
                stv(a.Uout, o1);
                if (a.Ynext) stv(a.Ynext, o2);
                if (a.lz) {  // the next substep's starting state and first stage vector
                    stv(a.lz, o1);
                    const T kc = (T)a.lkc;
#pragma unroll
                    for (int u = 0; u < PV; ++u) o2[u] = kc * o1[u];
                    stv(a.lk, o2);
                }
            }
        } else {
            switch (mode) {
                case RK2_S1:
#pragma unroll
                    for (int u = 0; u < PV; ++u) o1[u] = fma(cy, kv[u], x0[u]);
                    stv(a.Ynext, o1);
                    break;
                case RK2_S2:
                    if constexpr (COMP) {
#pragma unroll
                        for (int u = 0; u < PV; ++u) two_sum(x0[u], fma(cu, kv[u], lo[u]), o1[u], o2[u]);
                        stv(a.Uout, o1);
                        uint2 w;
                        w.x = (uint32_t)to_bf16(o2[0]) | ((uint32_t)to_bf16(o2[1]) << 16);
                        w.y = (uint32_t)to_bf16(o2[2]) | ((uint32_t)to_bf16(o2[3]) << 16);
                        *reinterpret_cast<uint2*>((uint16_t*)a.Ulo + gi) = w;
                    } else {
#pragma unroll
                        for (int u = 0; u < PV; ++u) o1[u] = fma(cu, kv[u], x0[u]);
                        stv(a.Uout, o1);
                    }
                    break;
                case RK4_S1:
#pragma unroll
                    for (int u = 0; u < PV; ++u) {
                        o1[u] = fma(cy, kv[u], x0[u]);
                        o2[u] = COMP ? ca * kv[u] : fma(ca, kv[u], x0[u]);
                    }
                    stv(a.Ynext, o1);
                    stv(a.Acc, o2);
                    break;
                case RK4_S2:
                case RK4_S3:
#pragma unroll
                    for (int u = 0; u < PV; ++u) {
                        o1[u] = fma(cy, kv[u], x0[u]);
                        o2[u] = fma(ca, kv[u], x1[u]);
                    }
                    stv(a.Ynext, o1);
                    stv(a.Acc, o2);
                    break;
                case RK4_S4:
                    if constexpr (COMP) {
#pragma unroll
                        for (int u = 0; u < PV; ++u) two_sum(x0[u], fma(cu, kv[u], x1[u]) + lo[u], o1[u], o2[u]);
                        stv(a.Uout, o1);
                        uint2 w;
                        w.x = (uint32_t)to_bf16(o2[0]) | ((uint32_t)to_bf16(o2[1]) << 16);
                        w.y = (uint32_t)to_bf16(o2[2]) | ((uint32_t)to_bf16(o2[3]) << 16);
                        *reinterpret_cast<uint2*>((uint16_t*)a.Ulo + gi) = w;
                    } else {
#pragma unroll
                        for (int u = 0; u < PV; ++u) o1[u] = fma(cu, kv[u], x1[u]);
                        stv(a.Uout, o1);
                    }
                    break;
                default:
                    stv(a.Kout, kv);
                    break;
            }
        }
        if (a.filter) {  // stage-1 and RHS modes: x0 is the stage input
#pragma unroll
            for (int u = 0; u < PV; ++u) {
                const double ud = (double)x0[u], kd = (double)kv[u];
                a.Fre[gi + u] += a.fa_re * ud + a.fb_re * kd;
                a.Fim[gi + u] += a.fa_im * ud + a.fb_im * kd;
            }
#pragma unroll 1
            for (int h = 1; MH && h < a.nharm; ++h)
#pragma unroll
                for (int u = 0; u < PV; ++u) {
                    const double ud = (double)x0[u], kd = (double)kv[u];
                    args.Fre[h * args.hstride + gi + u] += args.hfa_re[h] * ud + args.hfb_re[h] * kd;
                    args.Fim[h * args.hstride + gi + u] += args.hfa_im[h] * ud + args.hfb_im[h] * kd;
                }
        }
    }
}

// One 16x16x4 matrix-core product with the lane layout the stage kernels
// assume (a single 64-lane wave): lane l takes A[l % 16][l / 16] and
// B[l / 16][l % 16] and returns D[Mfma<T>::row(l / 16, r)][l % 16], r = 0..3.
template <typename T>
__global__ __launch_bounds__(64) void k_mfma_probe(const double* __restrict__ A, const double* __restrict__ B,
                                                   double* __restrict__ D) {
    const int l = threadIdx.x;
    const T a = (T)A[(l % 16) * 4 + l / 16];
    const T b = (T)B[(l / 16) * 16 + l % 16];
    typename Mfma<T>::acc_t c = {T(0), T(0), T(0), T(0)};
    c = Mfma<T>::mma(a, b, c);
#pragma unroll
    for (int r = 0; r < 4; ++r) D[Mfma<T>::row(l / 16, r) * 16 + l % 16] = (double)c[r];
}

template <typename T>
__global__ void k_to_field(const double* __restrict__ X, T* __restrict__ U, uint16_t* __restrict__ Ulo, int64_t n,
                           int Np, int flipH) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double x = X[i];
        if (flipH && ((i / Np) % 6) >= 3) x = -x;
        const T hi = (T)x;
        U[i] = hi;
        if constexpr (std::is_same<T, float>::value)
            if (Ulo) Ulo[i] = to_bf16((float)(x - (double)hi));
    }
}

template <typename T>
__global__ void k_from_field(const T* __restrict__ U, const uint16_t* __restrict__ Ulo, double* __restrict__ Yo,
                             const double* __restrict__ sub, int64_t n, int Np, int flipH) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double x = (double)U[i];
        if constexpr (std::is_same<T, float>::value)
            if (Ulo) x += (double)from_bf16(Ulo[i]);
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

// One 64-lane workgroup per element block: bit e of mask[block] is set when
// element e has a nonzero source value (either part, any row or harmonic).
template <typename T>
__global__ __launch_bounds__(64) void k_source_mask(const T* Sre, const T* Sim, int nharm, int64_t hstride,
                                                    int64_t K, int np6, uint32_t* mask) {
    const int64_t blk = blockIdx.x;
    const int64_t e0 = blk * EPW;
    const int ne = (int)((K - e0) < EPW ? (K - e0) : EPW);
    const int n = ne * np6;
    uint32_t bits = 0;
    for (int h = 0; h < nharm; ++h)
        for (int v = threadIdx.x; v < n; v += 64) {
            const int64_t g = h * hstride + e0 * np6 + v;
            if ((Sre && Sre[g] != T(0)) || (Sim && Sim[g] != T(0))) bits |= 1u << (v / np6);
        }
    for (int o = 32; o > 0; o >>= 1) bits |= (uint32_t)__shfl_xor((int)bits, o, 64);
    if (threadIdx.x == 0) mask[blk] = bits;
}

// ---- local time stepping: elementwise combinations of field vectors (field
// precision T, coefficients in FP64).  Row masks use the per-block element
// words of the stage kernels' masks (bit e of word b: element b EPW + e).
__device__ __forceinline__ bool lts_row_on(const uint32_t* mask, int inv, int64_t i, int np6) {
    const int64_t e = i / np6;
    return ((mask[e / EPW] >> (int)(e % EPW)) & 1u) ^ (uint32_t)inv;
}

// Values an elementwise LTS kernel visits: all n, or (blist non-null) the
// rows of the listed element blocks; returns the count and maps a visit
// index to the value index.
struct LtsRange {
    const int* blist;
    int64_t nb, n, per;  // per = EPW * 6 Np values of a block
    __device__ __forceinline__ int64_t count() const { return blist ? nb * per : n; }
    __device__ __forceinline__ int64_t at(int64_t f) const {
        if (!blist) return f;
        const int64_t b = f / per;
        return (int64_t)blist[b] * per + (f - b * per);
    }
};

// z = a y + b rows(x), rows(x) = x on the mask's rows (all rows when mask is
// null), 0 elsewhere; y nullable (= 0); z may alias y
template <typename T>
__global__ void k_lts_axpy(LtsRange rg, int np6, const uint32_t* mask, int inv, double a, const T* y, double b,
                           const T* x, T* z) {
    const int64_t cnt = rg.count();
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < cnt; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = rg.at(v);
        if (i >= rg.n) continue;
        const T xv = (!mask || lts_row_on(mask, inv, i, np6)) ? x[i] : T(0);
        z[i] = (y ? (T)a * y[i] : T(0)) + (T)b * xv;
    }
}

// Rows outside the mask (the coarse unknowns away from the fine region):
// z += sum_j al_j W_j + sc Sre - ss Sim (Sre nullable; source rows only where
// the source mask and the row's component allow)
template <typename T>
__global__ void k_lts_closed(int64_t n, int np6, int Np, const uint32_t* mask, const T* W0, const T* W1, const T* W2,
                             const T* W3, int nw, double a0, double a1, double a2, double a3, const T* Sre,
                             const T* Sim, int src_rows, double sc, double ss, T* z) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (lts_row_on(mask, 0, i, np6)) continue;
        T acc = z[i];
        if (nw > 0) acc += (T)a0 * W0[i];
        if (nw > 1) acc += (T)a1 * W1[i];
        if (nw > 2) acc += (T)a2 * W2[i];
        if (nw > 3) acc += (T)a3 * W3[i];
        if (Sre && ((i / Np) % 6) < src_rows) acc += (T)sc * Sre[i] - (T)ss * Sim[i];
        z[i] = acc;
    }
}

// Adjoint Taylor weights of the rows outside the mask (every coarse unknown):
// wb_j = al_j zbar there; the mask's rows keep what the substeps accumulated.
template <typename T>
__global__ void k_lts_wbar_close(int64_t n, int np6, const uint32_t* mask, const T* zbar, T* wb0, T* wb1, T* wb2,
                                 T* wb3, int nw, double a0, double a1, double a2, double a3) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (lts_row_on(mask, 0, i, np6)) continue;
        const T z = zbar[i];
        if (nw > 0) wb0[i] = (T)a0 * z;
        if (nw > 1) wb1[i] = (T)a1 * z;
        if (nw > 2) wb2[i] = (T)a2 * z;
        if (nw > 3) wb3[i] = (T)a3 * z;
    }
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

// F += wa field(U) + wb field(D) (two levels of the filter sum in one pass)
template <typename T>
__global__ void k_filter_add2(const T* __restrict__ U, double ar, double ai, const T* __restrict__ D, double br,
                              double bi, double* Fre, double* Fim, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double u = (double)U[i], d = (double)D[i];
        Fre[i] += ar * u + br * d;
        Fim[i] += ai * u + bi * d;
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

// Batched dot: member b = blockIdx.y; per member the same block decomposition
// and summation order as k_dot / k_dot_final (results equal the single dots).
template <int Q>
__global__ __launch_bounds__(kDotThreads) void k_dot_batch(const double* __restrict__ U, const double* __restrict__ V,
                                                           const double* __restrict__ wE,
                                                           const double* __restrict__ wH, int64_t wstride,
                                                           int64_t K, double* __restrict__ partial) {
    constexpr int NP = Dim<Q>::NP;
    constexpr int MMO = mat_off(Q) + 3 * NP * NP + NP * 4 * Dim<Q>::NFP;
    __shared__ double sm[kDotThreads];
    const int64_t b = blockIdx.y;
    const int64_t n = 6 * K * NP;
    U += b * n;
    V += b * n;
    wE += b * wstride;
    wH += b * wstride;
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
    if (threadIdx.x == 0) partial[b * kDotBlocks + blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kDotThreads) void k_dot_final_batch(const double* __restrict__ partial, int n,
                                                                 double* __restrict__ out) {
    __shared__ double sm[kDotThreads];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kDotThreads) acc += partial[(int64_t)b * kDotBlocks + i];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = sm[0];
}

__global__ void k_axpby_batch(const double* __restrict__ a, const double* x, const double* __restrict__ c,
                              const double* y, double* z, int64_t n, int B) {
    const int64_t tot = n * B;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / n;
        z[i] = a[b] * x[i] + c[b] * y[i];
    }
}

template <typename T>
__global__ void k_filter_add_batch(const T* __restrict__ U, const double* __restrict__ wr,
                                   const double* __restrict__ wi, double* Fre, double* Fim, int64_t n, int B) {
    const int64_t tot = n * B;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / n;
        const double u = (double)U[i];
        Fre[i] += wr[b] * u;
        Fim[i] += wi[b] * u;
    }
}

__global__ void k_nonfinite(const double* X, int64_t n, int* flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = X[i];
        if (!(x == x) || x - x != 0.0) flag[0] = 1;
    }
}

// Stage-kernel variant per (q, precision): 0 = gather per face, 1 = gathers
// pipelined one face ahead, 2 / 3 = matrix cores (q >= 2) without /
// with the one-face-ahead gathers, 4 = 3 with two waves per block, 5-7 the
// eager-gather and column-split forms of 4, 8 = four waves per block, 9 = 8
// with every face's gathers at once; -1 = chosen per launch from its size.
// Overridable through cmcg_tune_stage() and the autotuner.  Defaults:
// per-face gathers for P1; for P2 and P3 the form the autotuner's timings
// favour at the launch's size (workgroups over all members).  FP32 P3 (us per
// launch, forms 4 / 6 / 8 / 9): 3072 tets 12.2 / 10.9 / 8.9 / 8.8, 10368 tets
// 15.6 / 14.3 / 13.8 / 13.5, 24576 tets 25.2 / 21.8 / 22.7 / 23.6, 48000 tets
// 38.7 / 37.1 / 36.8 / 39.6, 82944 tets 57.6 / 56.9 / 57.9 / -, 196608 tets
// 131.0 / 137.4 / 139.1 / -.  FP32 P2 (forms 3 / 4 / 5 / 8 / 9): 3072 tets
// 9.0 / 7.6 / 7.3 / 6.5 / 6.1, 10368 tets 10.7 / 8.9 / 8.7 / 8.4 / 8.0, 24576
// tets 14.2 / 13.1 / 12.2 / 13.8 / 13.6, 82944 tets 30.3 / 28.3 / 30.4 / 31.2
// / -, the 1,572,864-tet mesh 473 / 487 / 525 / - / -, 64 members of 10368
// tets 188 / 199 / 222 / - / -.  FP64 (forms 4 / 8 / 9): P2 3072 tets 9.4 /
// 8.1 / 7.8, 10368 tets 12.3 / 11.7 / 13.6, 48000 tets 33.3 / 35.6 / 37.2;
// P3 3072 tets 17.5 / 12.9 / 12.5, 48000 tets 69.6 / 68.9 / 75.3 (the VALU
// form: 112.7).
int g_variant[kMaxQ + 1][2] = {{0, 0}, {0, 0}, {-1, -1}, {-1, -1}};
inline int variant_by_size(int q, int precision, int64_t blocks) {
    if (precision == CMCG_FP64) {
        if (blocks <= 400) return 9;
        return blocks <= 1100 || (q == 3 && blocks <= 9000) ? 8 : 4;
    }
    if (q == 3) return blocks <= 1100 ? 9 : blocks <= 9000 ? 6 : 4;
    if (q == 2) return blocks <= 1100 ? 9 : blocks <= 3000 ? 5 : blocks <= 12000 ? 4 : 3;
    return 0;
}
inline int stage_variant(int q, int precision, int64_t blocks) {
    const int v = g_variant[q][precision];
    return v >= 0 ? v : variant_by_size(q, precision, blocks);
}

inline int grid_for(int64_t n, int threads = 256) {
    int64_t g = (n + threads - 1) / threads;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

template <typename T, int Q, bool MH>
void stage_launch_mh(const StageArgs& a, hipStream_t s) {
    const int64_t blocks = a.blist ? a.nblist : (a.K + EPW - 1) / EPW;
    const int64_t per = (blocks + 7) / 8;
    const int v = stage_variant(Q, sizeof(T) == 8 ? CMCG_FP64 : CMCG_FP32, blocks * (a.nmembers > 1 ? a.nmembers : 1));
    const dim3 grid((unsigned)(8 * per), (unsigned)(a.nmembers > 1 ? a.nmembers : 1));
    if constexpr (Q >= 2) {
        if (v == 2) {
            hipLaunchKernelGGL((k_stage_mfma<T, Q, false, MH, 1>), grid, dim3(64), 0, s, a, per);
            return;
        }
        if (v == 3) {
            hipLaunchKernelGGL((k_stage_mfma<T, Q, true, MH, 1>), grid, dim3(64), 0, s, a, per);
            return;
        }
        if (v == 4) {
            hipLaunchKernelGGL((k_stage_mfma<T, Q, true, MH, 2>), grid, dim3(128), 0, s, a, per);
            return;
        }
        if (v == 5) {
            hipLaunchKernelGGL((k_stage_mfma<T, Q, true, MH, 2, true>), grid, dim3(128), 0, s, a, per);
            return;
        }
        if (v == 8) {
            hipLaunchKernelGGL((k_stage_mfma<T, Q, true, MH, 4>), grid, dim3(256), 0, s, a, per);
            return;
        }
        if (v == 9) {
            hipLaunchKernelGGL((k_stage_mfma<T, Q, true, MH, 4, true>), grid, dim3(256), 0, s, a, per);
            return;
        }
        if constexpr (Q == 3) {
            if (v == 6) {
                hipLaunchKernelGGL((k_stage_mfma<T, Q, true, MH, 2, false, true>), grid, dim3(128), 0, s, a, per);
                return;
            }
            if (v == 7) {
                hipLaunchKernelGGL((k_stage_mfma<T, Q, true, MH, 2, true, true>), grid, dim3(128), 0, s, a, per);
                return;
            }
        }
    }
    if (v == 1)
        hipLaunchKernelGGL((k_stage<T, Q, true, MH>), grid, dim3(64), 0, s, a, per);
    else
        hipLaunchKernelGGL((k_stage<T, Q, false, MH>), grid, dim3(64), 0, s, a, per);
}

template <typename T, int Q>
void stage_launch(const StageArgs& a, hipStream_t s) {
    if (a.mode == LTS_FWD || a.mode == LTS_ADJ || a.mode == LTS_CHAIN) {  // one instantiation per order
        const int64_t blocks = a.blist ? a.nblist : (a.K + EPW - 1) / EPW;
        const int64_t per = (blocks + 7) / 8;
        const dim3 grid((unsigned)(8 * per));
        // four waves per block on the launches restricted to a block list
        // (the substep stages: a partial round of workgroups, whose time is
        // one block's chain) and where the chosen form has four (8, 9); two
        // otherwise
        if constexpr (Q >= 2) {
            if (a.blist || stage_variant(Q, sizeof(T) == 8 ? CMCG_FP64 : CMCG_FP32, blocks) >= 8)
                hipLaunchKernelGGL((k_stage_mfma<T, Q, true, false, 4, false, false, true>), grid, dim3(256), 0, s,
                                   a, per);
            else
                hipLaunchKernelGGL((k_stage_mfma<T, Q, true, false, 2, false, false, true>), grid, dim3(128), 0, s,
                                   a, per);
        } else
            hipLaunchKernelGGL((k_stage<T, Q, false, false, true>), grid, dim3(64), 0, s, a, per);
        return;
    }
    if (a.nharm > 1)
        stage_launch_mh<T, Q, true>(a, s);
    else
        stage_launch_mh<T, Q, false>(a, s);
}

void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(CMCG_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

// Fixed device array for the partial sums of the allocation-free inner
// product (one copy per GPU, held until the process ends).  Host code never
// passes its name to a kernel: the name is a host-side stand-in, and the
// device address comes from hipGetSymbolAddress, resolved once per device.
constexpr int kNoallocDoubles = 1024;
static_assert(kNoallocDoubles >= kDotBlocks, "the scratch array must hold every partial of a dot");
__device__ __align__(256) double scratch[kNoallocDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};

}  // namespace

size_t noalloc_scratch_doubles() { return kNoallocDoubles; }

double* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= 64) fail(CMCG_ERR_DEVICE, "device index out of range");
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        CMCG_HIP(hipGetDevice(&cur));
        if (cur != device) fail(CMCG_ERR_STATE, "scratch address requested for a device that is not current");
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            fail(CMCG_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[device] = (double*)ptr;
    }
    return g_scratch_ptr[device];
}

int dot_blocks(int64_t K) {
    const int64_t rows = 6 * K;
    int64_t blocks = (rows + kDotThreads - 1) / kDotThreads;
    if (blocks > kDotBlocks) blocks = kDotBlocks;
    return (int)(blocks < 1 ? 1 : blocks);
}

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
    {
        std::vector<int> nn(24 * NFP);
        for (int nf = 0; nf < 4; ++nf)
            for (int pm = 0; pm < 6; ++pm)
                for (int k = 0; k < NFP; ++k) nn[(nf * 6 + pm) * NFP + k] = fnode[nf * NFP + fperm[pm * NFP + k]];
        std::vector<uint32_t> words(ft_words(q), 0u);
        for (int i = 0; i < 28 * NFP; ++i) {
            const int v = i < 4 * NFP ? fnode[i] : nn[i - 4 * NFP];
            if (v < 0 || v > 255) fail(CMCG_ERR_ARG, "face-node table entry out of byte range");
            words[i / 4] |= (uint32_t)v << (8 * (i % 4));
        }
        CMCG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(cFaceTab), words.data(), words.size() * sizeof(uint32_t),
                                   ft_off(q) * sizeof(uint32_t), hipMemcpyHostToDevice));
    }
    if (q >= 2) {
        // lane-ordered A fragments of the matrix-core kernel: entry (frag, lane)
        // = A[16 mt + lane % 16][4 ks + lane / 16] of the block the fragment names
        const int MT = (NP + 15) / 16, NJ = (NP + 3) / 4, KSV = 3 * NJ, KSF = (NFP + 3) / 4;
        const int nfrag = MT * KSV + 4 * MT * KSF;
        std::vector<double> fr(64 * nfrag, 0.0);
        for (int l = 0; l < 64; ++l) {
            const int i_in = l % 16, k_in = l / 16;
            for (int mt = 0; mt < MT; ++mt) {
                const int i = 16 * mt + i_in;
                for (int ks = 0; ks < KSV; ++ks) {
                    const int a = ks / NJ, j = 4 * (ks % NJ) + k_in;  // axis-major K order
                    double v = 0.0;
                    if (i < NP && j < NP) v = D[(a * NP + i) * NP + j];
                    fr[(mt * KSV + ks) * 64 + l] = v;
                }
                for (int f = 0; f < 4; ++f)
                    for (int ks = 0; ks < KSF; ++ks) {
                        const int k = 4 * ks + k_in;
                        double v = 0.0;
                        if (i < NP && k < NFP) v = LIFT[i * 4 * NFP + f * NFP + k];
                        fr[(MT * KSV + (f * MT + mt) * KSF + ks) * 64 + l] = v;
                    }
            }
        }
        // FP32 fragments are the rounded FP64 ones
        std::vector<float> fr32(fr.begin(), fr.end());
        CMCG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(gFrag), fr32.data(), fr32.size() * sizeof(float),
                                   frag_off(q) * sizeof(float), hipMemcpyHostToDevice));
        CMCG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(gFrag64), fr.data(), fr.size() * sizeof(double),
                                   frag_off(q) * sizeof(double), hipMemcpyHostToDevice));
    }
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

void launch_to_field(int precision, int Np, const double* X, void* U, void* Ulo, int64_t n, int flipH,
                     hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_to_field<double>, dim3(grid_for(n)), dim3(256), 0, s, X, (double*)U, nullptr, n, Np,
                           flipH);
    else
        hipLaunchKernelGGL(k_to_field<float>, dim3(grid_for(n)), dim3(256), 0, s, X, (float*)U, (uint16_t*)Ulo, n,
                           Np, flipH);
    check_launch();
}

void launch_from_field(int precision, int Np, const void* U, const void* Ulo, double* Y, const double* sub,
                       int64_t n, int flipH, hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_from_field<double>, dim3(grid_for(n)), dim3(256), 0, s, (const double*)U, nullptr, Y,
                           sub, n, Np, flipH);
    else
        hipLaunchKernelGGL(k_from_field<float>, dim3(grid_for(n)), dim3(256), 0, s, (const float*)U,
                           (const uint16_t*)Ulo, Y, sub, n, Np, flipH);
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

int64_t source_mask_words(int64_t K) { return (K + EPW - 1) / EPW; }

void launch_source_mask(int precision, int Np, const void* Sre, const void* Sim, int nharm, int64_t hstride,
                        int64_t K, uint32_t* mask, hipStream_t s) {
    const int64_t nb = source_mask_words(K);
    if (nb == 0) return;
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_source_mask<double>, dim3((unsigned)nb), dim3(64), 0, s, (const double*)Sre,
                           (const double*)Sim, nharm, hstride, K, 6 * Np, mask);
    else
        hipLaunchKernelGGL(k_source_mask<float>, dim3((unsigned)nb), dim3(64), 0, s, (const float*)Sre,
                           (const float*)Sim, nharm, hstride, K, 6 * Np, mask);
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

void launch_filter_add2(int precision, const void* U, double ar, double ai, const void* D, double br, double bi,
                        double* Fre, double* Fim, int64_t n, hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_filter_add2<double>, dim3(grid_for(n)), dim3(256), 0, s, (const double*)U, ar, ai,
                           (const double*)D, br, bi, Fre, Fim, n);
    else
        hipLaunchKernelGGL(k_filter_add2<float>, dim3(grid_for(n)), dim3(256), 0, s, (const float*)U, ar, ai,
                           (const float*)D, br, bi, Fre, Fim, n);
    check_launch();
}

int dot_partials() { return kDotBlocks; }

namespace {
LtsRange lts_range(int64_t n, int np6, const int* blist, int64_t nb) {
    LtsRange r;
    r.blist = blist;
    r.nb = nb;
    r.n = n;
    r.per = (int64_t)EPW * np6;
    return r;
}
int64_t lts_count(const LtsRange& r) { return r.blist ? r.nb * r.per : r.n; }
}  // namespace

void launch_lts_axpy(int precision, int64_t n, int np6, const int* blist, int64_t nb, const uint32_t* mask, int inv,
                     double a, const void* y, double b, const void* x, void* z, hipStream_t s) {
    const LtsRange rg = lts_range(n, np6, blist, nb);
    const int g = grid_for(lts_count(rg));
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_lts_axpy<double>, dim3(g), dim3(256), 0, s, rg, np6, mask, inv, a, (const double*)y,
                           b, (const double*)x, (double*)z);
    else
        hipLaunchKernelGGL(k_lts_axpy<float>, dim3(g), dim3(256), 0, s, rg, np6, mask, inv, a, (const float*)y, b,
                           (const float*)x, (float*)z);
    check_launch();
}

void launch_lts_closed(int precision, int64_t n, int np6, int Np, const uint32_t* mask, const void* const* W,
                       const double* al, int nw, const void* Sre, const void* Sim, int src_rows, double sc, double ss,
                       void* z, hipStream_t s) {
    const void* Wp[4] = {nullptr, nullptr, nullptr, nullptr};
    double c[4] = {0, 0, 0, 0};
    for (int j = 0; j < nw && j < 4; ++j) {
        Wp[j] = W[j];
        c[j] = al[j];
    }
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_lts_closed<double>, dim3(grid_for(n)), dim3(256), 0, s, n, np6, Np, mask,
                           (const double*)Wp[0], (const double*)Wp[1], (const double*)Wp[2], (const double*)Wp[3], nw,
                           c[0], c[1], c[2], c[3], (const double*)Sre, (const double*)Sim, src_rows, sc, ss,
                           (double*)z);
    else
        hipLaunchKernelGGL(k_lts_closed<float>, dim3(grid_for(n)), dim3(256), 0, s, n, np6, Np, mask,
                           (const float*)Wp[0], (const float*)Wp[1], (const float*)Wp[2], (const float*)Wp[3], nw,
                           c[0], c[1], c[2], c[3], (const float*)Sre, (const float*)Sim, src_rows, sc, ss,
                           (float*)z);
    check_launch();
}

void launch_lts_wbar_close(int precision, int64_t n, int np6, const uint32_t* mask, const void* zbar,
                           void* const* wb, const double* al, int nw, hipStream_t s) {
    void* W[4] = {nullptr, nullptr, nullptr, nullptr};
    double c[4] = {0, 0, 0, 0};
    for (int j = 0; j < nw && j < 4; ++j) {
        W[j] = wb[j];
        c[j] = al[j];
    }
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_lts_wbar_close<double>, dim3(grid_for(n)), dim3(256), 0, s, n, np6, mask,
                           (const double*)zbar, (double*)W[0], (double*)W[1], (double*)W[2], (double*)W[3], nw, c[0],
                           c[1], c[2], c[3]);
    else
        hipLaunchKernelGGL(k_lts_wbar_close<float>, dim3(grid_for(n)), dim3(256), 0, s, n, np6, mask,
                           (const float*)zbar, (float*)W[0], (float*)W[1], (float*)W[2], (float*)W[3], nw, c[0], c[1],
                           c[2], c[3]);
    check_launch();
}

void launch_mfma_probe(int precision, const double* A, const double* B, double* D, hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_mfma_probe<double>, dim3(1), dim3(64), 0, s, A, B, D);
    else
        hipLaunchKernelGGL(k_mfma_probe<float>, dim3(1), dim3(64), 0, s, A, B, D);
    check_launch();
}

void set_stage_variant(int q, int precision, int variant) { g_variant[q][precision] = variant; }
int get_stage_variant(int q, int precision) { return g_variant[q][precision]; }
int resolve_stage_variant(int q, int precision, int64_t K, int members) {
    if (q < 1 || q > kMaxQ) return 0;
    return stage_variant(q, precision, (K + EPW - 1) / EPW * (members > 1 ? members : 1));
}

void launch_dot(int q, const double* U, const double* V, const double* wE, const double* wH, int64_t K,
                double* partial, double* out_dev, hipStream_t s) {
    const int blocks = dot_blocks(K);
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

void launch_dot_batch(int q, const double* U, const double* V, const double* wE, const double* wH, int64_t wstride,
                      int64_t K, int B, double* partial, double* out_dev, hipStream_t s) {
    int64_t rows = 6 * K;
    int blocks = (int)((rows + kDotThreads - 1) / kDotThreads);
    if (blocks > kDotBlocks) blocks = kDotBlocks;
    const dim3 grid(blocks, B);
    if (q == 1)
        hipLaunchKernelGGL(k_dot_batch<1>, grid, dim3(kDotThreads), 0, s, U, V, wE, wH, wstride, K, partial);
    else if (q == 2)
        hipLaunchKernelGGL(k_dot_batch<2>, grid, dim3(kDotThreads), 0, s, U, V, wE, wH, wstride, K, partial);
    else
        hipLaunchKernelGGL(k_dot_batch<3>, grid, dim3(kDotThreads), 0, s, U, V, wE, wH, wstride, K, partial);
    check_launch();
    hipLaunchKernelGGL(k_dot_final_batch, dim3(B), dim3(kDotThreads), 0, s, partial, blocks, out_dev);
    check_launch();
}

void launch_axpby_batch(const double* a, const double* x, const double* c, const double* y, double* z, int64_t n,
                        int B, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby_batch, dim3(grid_for(n * B)), dim3(256), 0, s, a, x, c, y, z, n, B);
    check_launch();
}

void launch_filter_add_batch(int precision, const void* U, const double* w_re, const double* w_im, double* Fre,
                             double* Fim, int64_t n, int B, hipStream_t s) {
    if (precision == CMCG_FP64)
        hipLaunchKernelGGL(k_filter_add_batch<double>, dim3(grid_for(n * B)), dim3(256), 0, s, (const double*)U,
                           w_re, w_im, Fre, Fim, n, B);
    else
        hipLaunchKernelGGL(k_filter_add_batch<float>, dim3(grid_for(n * B)), dim3(256), 0, s, (const float*)U,
                           w_re, w_im, Fre, Fim, n, B);
    check_launch();
}

void launch_nonfinite(const double* X, int64_t n, int* out_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n)), dim3(256), 0, s, X, n, out_dev);
    check_launch();
}

}  // namespace cmcg
