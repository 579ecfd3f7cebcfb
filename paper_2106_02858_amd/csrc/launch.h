// Kernel launch interface (kernels.hip) used by the host solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cmcg {

// Stage kernel update modes (one Runge-Kutta stage of Section 5.3, fused with
// the right-hand side Phi(t, Y) of Section 5.2):
//   k = Phi(t_s, Y)
//   RK2_S1: Ynext = U + cy k                      (U == Y)
//   RK2_S2: U     = U + cu k
//   RK4_S1: Ynext = U + cy k ; Acc = U + ca k     (U == Y)
//   RK4_S2/S3: Ynext = U + cy k ; Acc += ca k
//   RK4_S4: U     = Acc + cu k
//   RHS:    Kout  = k
//   LTS_FWD (local time stepping, substep stage): k += sum_j lcw_j lw_j;
//           Ynext = U + le Acc + cy k; Uout = lf Acc + ca k (Acc, Ynext, Uout
//           nullable; no compensated state)
//   LTS_ADJ (adjoint substep stage; Y = the adjoint stage vector kcur): on the
//           rows of the elements set in lmask A = k and lw_j += lcw_j kcur
//           (lw_j = lcw_j kcur when linit), elsewhere A = 0; Uout = U + A;
//           Ynext = le Acc + lf A (nullable); when lz is set (the last stage
//           of a substep), also lz = Uout and lk = lkc Uout (the next
//           substep's starting state and first stage vector)
//   LTS_CHAIN (adjoint Taylor chain): Uout = [A] k + [B] lw[0] + [C] lw[1] + lw[2],
//           [m] x = x on the rows of the elements whose bit of the mask (lmask,
//           lmaskB, lmaskC) xor its inv flag is set, 0 elsewhere (null mask:
//           every row); null lw[i]: no term
// Optional filter accumulation (FP64): F += fa * U + fb * k (complex).
//
// FP32 fields carry the state as an unevaluated sum U + Ulo (Ulo in bfloat16,
// |Ulo| <= half an FP32 ulp of U): Acc holds the increment only (RK4_S1:
// Acc = ca k; RK4_S4: U + Ulo += Acc + cu k) and the last update of a step adds
// its increment to U + Ulo with an exact two-sum, so rounding the state to
// FP32 once per step does not accumulate over the period.
enum StageMode { RK2_S1 = 0, RK2_S2, RK4_S1, RK4_S2, RK4_S3, RK4_S4, RHS, LTS_FWD, LTS_ADJ, LTS_CHAIN };

struct StageArgs {
    const void* Y;      // stage input (Phi argument), [K][6][Np]
    const void* U;      // base state
    void* Ynext;
    void* Acc;
    void* Uout;
    void* Kout;
    void* Ulo;          // FP32 fields: bfloat16 low parts of U (RK2_S2, RK4_S4 read and write it)
    const void* geo;    // [K][kGeo]
    const int* conn;    // [K][4]: >= 0: nbr<<5 | nbr_face<<3 | perm; -1 PEC; -2 impedance
    const void* Sre;    // source [K][6][Np] (nullable)
    const void* Sim;
    const uint32_t* smask;  // per element block of the stage kernels: bit e set when element e of the
                            // block has a nonzero source value (nullable: every element has)
    double* Fre;        // filter accumulators (nullable)
    double* Fim;
    int64_t K;
    double cy, ca, cu;
    double scos, ssin;  // Re(S e^{i w t}) = scos * Sre - ssin * Sim
    int src_rows;       // 0 none, 3 E rows, 6 all rows
    int mode;
    double fa_re, fa_im, fb_re, fb_im;
    int filter;
    // batched launches (grid.y = member); mtab == nullptr for a single problem
    int nmembers;           // members in the launch (>= 1)
    const double* mtab;     // per-member stage scalars [member][kMemberParams]
    const int* active;      // member still iterating (0: its workgroups exit)
    const int* msteps;      // steps per period of each member
    int step;               // time step of this launch; -1 skips the step check
    int64_t bstride;        // field elements between consecutive members
    int64_t gstride;        // geometry elements between members (0: shared)
    int64_t sstride;        // source elements between members
    // further harmonics h = 1 .. nharm - 1 of a several-frequency problem
    // (single launches): source Re(S_h e^{i k_h w0 t}) = hcos[h] Sre_h -
    // hsin[h] Sim_h, filter F_h += hfa[h] U + hfb[h] k; S_h and F_h sit
    // hstride elements after S_(h-1) and F_(h-1)
    int nharm;              // 1 for a single frequency
    int64_t hstride;
    double hcos[8], hsin[8], hfa_re[8], hfa_im[8], hfb_re[8], hfb_im[8];
    // input mask of a single 3-D launch (nullable): one word per element block
    // (layout of smask); Phi is evaluated on the input with every element whose
    // bit xor imask_inv is clear set to zero (B P y for local time stepping)
    const uint32_t* imask;
    int imask_inv;
    // single 3-D launches (nullable): run only the element blocks listed
    const int* blist;
    int64_t nblist;
    // LTS_FWD / LTS_ADJ operands (single 3-D launches)
    const void* lw[4];
    double lcw[4];
    int lnw;
    double le, lf;
    void* lz;     // LTS_ADJ: copy of Uout (nullable) ...
    void* lk;     // ... and lkc Uout
    double lkc;
    int linit;    // LTS_ADJ: lw_j = lcw_j kcur instead of lw_j += lcw_j kcur
    const uint32_t* lmask;  // LTS_ADJ: output rows (one word per element block, layout of smask)
    const uint32_t* lmaskB;
    const uint32_t* lmaskC;
    int linv, linvB, linvC;  // LTS_CHAIN: inversions of lmask, lmaskB, lmaskC
};
constexpr int kMaxHarm = 8;
// per-member scalars of a batched stage: cy, ca, cu, scos, ssin, fa_re, fa_im, fb_re, fb_im
constexpr int kMemberParams = 9;

// Source element mask (StageArgs::smask) of a [nharm][K][6][Np] source: one
// 32-bit word per element block; only exact zeros clear a bit, so skipping the
// source of a cleared element changes no value.
int64_t source_mask_words(int64_t K);
void launch_source_mask(int precision, int Np, const void* Sre, const void* Sim, int nharm, int64_t hstride,
                        int64_t K, uint32_t* mask, hipStream_t s);

void upload_constants(int q, int precision, const double* D, const double* LIFT, const double* M,
                      const int* fnode, const int* fperm);
void launch_stage(int q, int precision, const StageArgs& a, hipStream_t s);
// Local time stepping (field precision, n values, np6 = 6 Np values per
// element; masks: one word per element block, bit xor inv selects a row;
// blist / nb (nullable): visit only the rows of the listed element blocks):
//   axpy:    z = a y + b rows(x)   (mask null: all rows; y null: 0)
//   closed:  rows off the mask: z += sum_j al_j W_j + sc Sre - ss Sim (source rows)
void launch_lts_axpy(int precision, int64_t n, int np6, const int* blist, int64_t nb, const uint32_t* mask, int inv,
                     double a, const void* y, double b, const void* x, void* z, hipStream_t s);
void launch_lts_closed(int precision, int64_t n, int np6, int Np, const uint32_t* mask, const void* const* W,
                       const double* al, int nw, const void* Sre, const void* Sim, int src_rows, double sc, double ss,
                       void* z, hipStream_t s);
//   wbar_close: rows off the mask: wb_j = al_j zbar
void launch_lts_wbar_close(int precision, int64_t n, int np6, const uint32_t* mask, const void* zbar,
                           void* const* wb, const double* al, int nw, hipStream_t s);
// D[16][16] = A[16][4] B[4][16] on one matrix-core instruction of the field
// precision, through the lane layout the stage kernels use (FP64 in and out).
void launch_mfma_probe(int precision, const double* A, const double* B, double* D, hipStream_t s);
void set_stage_variant(int q, int precision, int variant);
int get_stage_variant(int q, int precision);
// the variant a launch over K elements and `members` members runs
int resolve_stage_variant(int q, int precision, int64_t K, int members);
constexpr int kStageVariants = CMCG_STAGE_VARIANTS;  // 2, 3: matrix cores (q >= 2; 3 gathers one face
                                                     // ahead); 4: as 3 with two waves per block (q >= 2)

// FP64 <-> field precision; flipH negates the magnetic rows (the S of P* = S P S).
// FP32: Ulo (nullable) receives / contributes the bfloat16 low part.
void launch_to_field(int precision, int Np, const double* X, void* U, void* Ulo, int64_t n, int flipH,
                     hipStream_t s);
// Y = field(U [+ Ulo]) * (flipH ? S : I) - sub   (sub, Ulo nullable)
void launch_from_field(int precision, int Np, const void* U, const void* Ulo, double* Y, const double* sub,
                       int64_t n, int flipH, hipStream_t s);
void launch_copy_field(int precision, const void* src, void* dst, int64_t n, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);
// z = a x + b y (FP64); y may alias z
void launch_axpby(double a, const double* x, double b, const double* y, double* z, int64_t n,
                  hipStream_t s);
// F += w * field(U) (FP64 complex accumulation of a real field)
void launch_filter_add(int precision, const void* U, double w_re, double w_im, double* Fre,
                       double* Fim, int64_t n, hipStream_t s);
// F += w_a * field(U) + w_b * field(D)
void launch_filter_add2(int precision, const void* U, double ar, double ai, const void* D, double br, double bi,
                        double* Fre, double* Fim, int64_t n, hipStream_t s);
// Deterministic M-weighted inner product (U, V)_{eps,mu}; result written to
// out_dev[0] (device).  partial: scratch of dot_partials() doubles.
int dot_partials();
// Partials (blocks) a 3-D dot over K elements writes; <= dot_partials().
int dot_blocks(int64_t K);
// Allocation-free inner product: device address of this GPU's fixed scratch
// array (resolved with hipGetSymbolAddress on the first request, with
// `device` current) and its capacity in doubles.  The 2-D dot writes
// dot2d_partials() partials.
double* noalloc_scratch(int device);
size_t noalloc_scratch_doubles();
int dot2d_partials();
void launch_dot(int q, const double* U, const double* V, const double* wE, const double* wH,
                int64_t K, double* partial, double* out_dev, hipStream_t s);
// Batched forms: members are consecutive blocks of n entries (K elements).
void launch_dot_batch(int q, const double* U, const double* V, const double* wE, const double* wH,
                      int64_t wstride, int64_t K, int B, double* partial, double* out_dev, hipStream_t s);
// z_b = a_b x_b + c_b y_b with coefficient arrays a[B], c[B] in device memory
void launch_axpby_batch(const double* a, const double* x, const double* c, const double* y, double* z,
                        int64_t n, int B, hipStream_t s);
// F_b += w_b field(U_b)
void launch_filter_add_batch(int precision, const void* U, const double* w_re, const double* w_im,
                             double* Fre, double* Fim, int64_t n, int B, hipStream_t s);
// non-finite check: out_dev[0] = 1 if any entry of X is not finite
void launch_nonfinite(const double* X, int64_t n, int* out_dev, hipStream_t s);

// 2-D transverse-magnetic path (kernels2d.hip): fields (e, h1, h2), dof layout
// [K][3][Np], geometry [K][kGeo2], connectivity [K][3] (perm bit: the
// neighbour runs the edge the other way); the same stage modes and
// compensated FP32 state as the 3-D kernels; batched launches (grid.y =
// member, StageArgs::mtab non-null) as in 3-D, without the source mask.
void upload_constants2d(int q, const double* D, const double* LIFT, const double* M, const int* fnode);
void launch_stage2d(int q, int precision, const StageArgs& a, hipStream_t s);
void launch_to_field2d(int precision, int Np, const double* X, void* U, void* Ulo, int64_t n, int flipH,
                       hipStream_t s);
void launch_from_field2d(int precision, int Np, const void* U, const void* Ulo, double* Y, const double* sub,
                         int64_t n, int flipH, hipStream_t s);
void launch_dot2d(int q, const double* U, const double* V, const double* wE, const double* wH, int64_t K,
                  double* partial, double* out_dev, hipStream_t s);
void launch_dot_batch2d(int q, const double* U, const double* V, const double* wE, const double* wH,
                        int64_t wstride, int64_t K, int B, double* partial, double* out_dev, hipStream_t s);

}  // namespace cmcg
