// Local time stepping (the paper's concluding remarks: locally refined meshes
// without the global CFL restriction of their smallest elements).
//
// One coarse step of size H from t, m fine substeps of size h = H / m
// (Runge-Kutta-based local time stepping with Taylor-frozen coarse unknowns;
// P = the unknowns of the fine elements, those whose own CFL step is shorter
// than H):
//   D_0 = y, D_{k+1} = B D_k + F^(k)(t)           (k + 1 < p; p = 2 RK2, 4 RK4)
//   W_k = B (I - P) D_k
//   z' = B P z + sum_k tau^k / k! W_k + F(t + tau), z(0) = y, m base-RK steps
//   y(t + H) = z(H)
// Every application of B is one stage-kernel launch (an input mask zeroes
// the unknowns outside P or I - P, including neighbour traces).  The backward
// periods of Algorithm 2 need the exact adjoint of this propagator: the
// step's operations in reverse order, transposed, in S-flipped variables
// (where B* = S B S becomes B and the masks move to the outputs).  Fields
// stay in the space's precision without the compensated FP32 state.
//
// Only the fine region pays for the substeps: B P z vanishes outside the
// fine elements and their face neighbours (the halo), so the substeps run
// on the element blocks that hold halo elements (one stage launch per
// substep stage, the polynomial W terms and the Runge-Kutta combination
// fused into its update pass), and every other unknown advances in closed
// form, z = y + sum_k al_k W_k + (RK quadrature of F) with al_k = sum over
// the substeps' stages of b_s h tau_s^k / k!.  Away from the halo blocks
// B (I - P) D_k = D_{k+1} - F^(k), so only W_{p-1} needs a full launch: a
// coarse step costs p full right-hand sides, p - 1 on the halo blocks and
// p m on the halo blocks for the substeps (RK4: 4 + 3 h + 16 h launches of
// B for m = 4 against 16 full ones of global stepping).  The adjoint runs
// its substeps on the halo blocks as well (outputs on the fine rows), the
// coarse rows' adjoint Taylor weights being al_k times the step's end
// value.
#include <cmath>

#include "objects.h"

namespace cmcg {

namespace {

// fine-element mask (one word per element block) for the coarse step of c,
// the mask of the element blocks that hold halo elements (fine ones or their
// face neighbours), the rows near the halo outside the fine elements, and the
// lists of halo blocks and of halo blocks with their face neighbours' blocks
void ensure_lts_mask(cmcg_problem* p, const StepCfg& c) {
    const SpaceData& s = *p->sp;
    // the fine set depends on the coarse step and the CFL constant
    if (p->lts_H == c.dt && p->lts_cq == c.cq && p->lts_mask.p) return;
    const MeshData& m = *s.mesh;
    const int64_t nw = source_mask_words(s.K);
    std::vector<uint32_t> w(nw, 0u), hb(nw, 0u);
    std::vector<char> halo(s.K, 0);
    p->lts_fine = 0;
    for (int64_t e = 0; e < s.K; ++e) {
        const double dte = c.cq * std::sqrt(p->mu[e] * p->eps[e]) * m.rho[e];
        if (dte < c.dt) {
            w[e / 10] |= 1u << (e % 10);
            ++p->lts_fine;
            halo[e] = 1;
            for (int f = 0; f < 4; ++f)
                if (m.nbr[4 * e + f] >= 0) halo[m.nbr[4 * e + f]] = 1;
        }
    }
    std::vector<int> hbl, h2l;
    std::vector<char> near(s.K, 0);  // elements of halo blocks and their face neighbours
    for (int64_t b = 0; b < nw; ++b) {
        bool any_h = false;
        for (int64_t e = 10 * b; e < std::min<int64_t>(10 * b + 10, s.K); ++e) any_h = any_h || halo[e];
        if (any_h) {
            hbl.push_back((int)b);
            hb[b] = 0x3ffu;  // every element of the block
            for (int64_t e = 10 * b; e < std::min<int64_t>(10 * b + 10, s.K); ++e) {
                near[e] = 1;
                for (int f = 0; f < 4; ++f)
                    if (m.nbr[4 * e + f] >= 0) near[m.nbr[4 * e + f]] = 1;
            }
        }
    }
    std::vector<uint32_t> h2nf(nw, 0u);  // rows of those blocks outside the fine elements
    for (int64_t b = 0; b < nw; ++b) {
        bool any = false;
        for (int64_t e = 10 * b; e < std::min<int64_t>(10 * b + 10, s.K); ++e) any = any || near[e];
        if (any) {
            h2l.push_back((int)b);
            h2nf[b] = ~w[b] & 0x3ffu;
        }
    }
    p->lts_mask.alloc(nw * 4);
    p->lts_hbmask.alloc(nw * 4);
    p->lts_h2nf.alloc(nw * 4);
    CMCG_HIP(hipMemcpy(p->lts_h2nf.p, h2nf.data(), nw * 4, hipMemcpyHostToDevice));
    CMCG_HIP(hipMemcpy(p->lts_mask.p, w.data(), nw * 4, hipMemcpyHostToDevice));
    CMCG_HIP(hipMemcpy(p->lts_hbmask.p, hb.data(), nw * 4, hipMemcpyHostToDevice));
    p->lts_nhb = (int64_t)hbl.size();
    p->lts_nh2b = (int64_t)h2l.size();
    p->lts_hblocks.alloc(std::max<size_t>(1, hbl.size()) * 4);
    p->lts_h2blocks.alloc(std::max<size_t>(1, h2l.size()) * 4);
    if (!hbl.empty()) CMCG_HIP(hipMemcpy(p->lts_hblocks.p, hbl.data(), hbl.size() * 4, hipMemcpyHostToDevice));
    if (!h2l.empty()) CMCG_HIP(hipMemcpy(p->lts_h2blocks.p, h2l.data(), h2l.size() * 4, hipMemcpyHostToDevice));
    // captured periods hold the old lists' addresses and the old step's coefficients
    for (auto& kv : p->lts_graphs) (void)hipGraphExecDestroy(kv.second);
    p->lts_graphs.clear();
    p->lts_H = c.dt;
    p->lts_cq = c.cq;
}

double inv_fact(int k) { return k == 0 ? 1.0 : k == 1 ? 1.0 : k == 2 ? 0.5 : 1.0 / 6.0; }

}  // namespace

void ensure_lts(cmcg_problem* p, const StepCfg& c) {
    const SpaceData& s = *p->sp;
    if (s.dim != 3) fail(CMCG_ERR_ARG, "local time stepping: tetrahedral spaces only");
    if (p->nharm != 1) fail(CMCG_ERR_ARG, "local time stepping: single-frequency problems only");
    ensure_lts_mask(p, c);
    const size_t fb = s.ndof * s.esize();
    for (auto& b : p->lD) b.alloc(fb);
    for (auto& b : p->lW) b.alloc(fb);
    for (auto& b : p->lWB) b.alloc(fb);
    p->lZ0.alloc(fb);
    p->Kbuf.alloc(fb);
}

void lts_period(cmcg_problem* p, const StepCfg& c, int direction, bool src, bool filt, hipStream_t st) {
    const SpaceData& s = *p->sp;
    const int prec = s.precision;
    const int64_t n = s.ndof;
    const int np6 = 6 * s.Np;
    const int order = c.scheme == 2 ? 2 : 4;
    const int m = c.lts;
    const int M = c.M;
    const double H = c.dt, h = H / m, w = p->omega;
    const uint32_t* fine = p->lts_mask.as<uint32_t>();
    void* U = p->U.p;
    void* Zs = p->Y1.p;
    void* Zs2 = p->Y2.p;
    void* Acc = p->Acc.p;
    void* Kb = p->Kbuf.p;
    void* D[4] = {U, p->lD[0].p, p->lD[1].p, p->lD[2].p};
    void* W[4] = {p->lW[0].p, p->lW[1].p, p->lW[2].p, p->lW[3].p};
    void* WB[4] = {p->lWB[0].p, p->lWB[1].p, p->lWB[2].p, p->lWB[3].p};
    const bool with_src = src && direction > 0 && p->src_rows;

    StageArgs a{};
    {
        // base arguments of the RHS launches
        a.geo = p->geo.p;
        a.conn = s.conn.as<int>();
        a.K = s.K;
        a.Sre = p->Sre.p;
        a.Sim = p->Sim.p;
        a.smask = p->smask.as<uint32_t>();
        a.nharm = 1;
        a.hstride = n;
        a.nmembers = 1;
        a.mode = RHS;
    }
    // Kout = B (mask y) [+ F^(deriv)(tt)]: F^(k)(t) = w^k Re(S e^{i(w t + k pi/2)})
    auto rhs = [&](const void* Y, void* Kout, bool f, double tt, int deriv, const uint32_t* imask, int inv) {
        a.Y = Y;
        a.U = Y;
        a.Kout = Kout;
        a.imask = imask;
        a.imask_inv = inv;
        a.src_rows = f ? p->src_rows : 0;
        const double ph = w * tt + deriv * 0.5 * M_PI, amp = std::pow(w, deriv);
        a.scos = amp * std::cos(ph);
        a.ssin = amp * std::sin(ph);
        stage_dim(s, a, st);
    };
    // sum_k tau^k / k! W_k coefficients
    auto poly = [&](double tau, double* cw) {
        double tk = 1.0;
        for (int k = 0; k < order; ++k) {
            cw[k] = tk * inv_fact(k);
            tk *= tau;
        }
    };
    // the base scheme's stages per substep: (offset in the substep, weight b_s)
    const int ns = c.scheme == 2 ? 1 : 4;
    const double st_off[4] = {c.scheme == 2 ? 0.5 : 0.0, 0.5, 0.5, 1.0};
    const double st_b[4] = {c.scheme == 2 ? 1.0 : 1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    // closed-form weights of the unknowns away from the fine region:
    // al_k = sum_{l,s} b_s h (tau_l + off_s h)^k / k!
    double al[4] = {0, 0, 0, 0};
    for (int l = 0; l < m; ++l)
        for (int si = 0; si < ns; ++si) {
            double cw[4];
            poly(l * h + st_off[si] * h, cw);
            for (int k = 0; k < order; ++k) al[k] += st_b[si] * h * cw[k];
        }
    const int* hbl = p->lts_hblocks.as<int>();
    const int64_t nhb = p->lts_nhb;
    const uint32_t* hbmask = p->lts_hbmask.as<uint32_t>();
    auto rhs_on = [&](const int* bl, int64_t nb) {
        a.blist = bl;
        a.nblist = nb;
    };
    // one substep stage on the halo blocks, fused with the combination:
    // k = B P Y [+ F(tt)] + sum_j cw_j W_j; out1 = base + e acc + c1 k;
    // out2 = f acc + c2 k (acc, out1, out2 nullable)
    auto fwd_stage = [&](const void* Yin, bool fsrc, double tt, const double* cw, const void* base, void* acc,
                         double e, double c1, void* out1, double f, double c2, void* out2) {
        a.Y = Yin;
        a.U = base;
        a.Acc = acc;
        a.Ynext = out1;
        a.Uout = out2;
        a.Kout = nullptr;
        a.imask = fine;
        a.imask_inv = 0;
        a.src_rows = fsrc ? p->src_rows : 0;
        a.scos = std::cos(w * tt);
        a.ssin = std::sin(w * tt);
        a.mode = LTS_FWD;
        a.cy = c1;
        a.ca = c2;
        a.le = e;
        a.lf = f;
        a.lnw = order;
        for (int j = 0; j < order; ++j) {
            a.lw[j] = W[j];
            a.lcw[j] = cw[j];
        }
        a.blist = hbl;
        a.nblist = nhb;
        stage_dim(s, a, st);
        a.mode = RHS;
        a.Acc = a.Ynext = a.Uout = nullptr;
        a.lnw = 0;
        a.blist = nullptr;
        a.nblist = 0;
    };

    if (direction > 0) {
        // filter weights (Section 5.4) at the coarse time levels t_nn = nn H
        std::complex<double> xi[4];
        if (filt && c.scheme == 4) hermite_weights(w, H, xi);
        const double twoT = 2.0 / c.T;
        auto ph = [&](double mm) {
            const double x = 2.0 * M_PI * mm / M;
            return std::complex<double>(std::cos(x), -std::sin(x));
        };
        if (filt) {
            launch_zero(p->Fre.p, p->Fre.bytes, st);
            launch_zero(p->Fim.p, p->Fim.bytes, st);
        }
        for (int nn = 0; nn < M; ++nn) {
            const double t = nn * H;
            // Taylor coefficients of the solution at t; D_1 = y'(t) is also the
            // derivative the Hermite filter takes at t_nn
            rhs_on(nullptr, 0);
            for (int k = 1; k < order; ++k) rhs(D[k - 1], D[k], with_src, t, k - 1, nullptr, 0);
            if (filt) {
                if (c.scheme == 2) {
                    const std::complex<double> wa = ph(nn) * ((nn == 0 ? 1.0 : 2.0) / M);
                    launch_filter_add(prec, U, wa.real(), wa.imag(), p->Fre.as<double>(), p->Fim.as<double>(), n, st);
                } else {
                    std::complex<double> wa = twoT * ph(nn) * xi[0], wb = twoT * ph(nn) * xi[2];
                    if (nn >= 1) {
                        wa += twoT * ph(nn - 1) * xi[1];
                        wb += twoT * ph(nn - 1) * xi[3];
                    }
                    launch_filter_add2(prec, U, wa.real(), wa.imag(), D[1], wb.real(), wb.imag(), p->Fre.as<double>(),
                                       p->Fim.as<double>(), n, st);
                }
            }
            // the coarse unknowns' contribution, frozen as a polynomial in tau:
            // W_{p-1} everywhere; W_k (k < p - 1) on the halo blocks only, since
            // away from the fine region B (I - P) D_k = B D_k = D_{k+1} - F^(k)
            rhs(D[order - 1], W[order - 1], false, 0.0, 0, fine, 1);
            // fine substeps on z (in place on U = D_0), only on the halo blocks
            if (nhb > 0) {
                rhs_on(hbl, nhb);
                for (int k = 0; k + 1 < order; ++k) rhs(D[k], W[k], false, 0.0, 0, fine, 1);
                double cw[4];
                for (int l = 0; l < m; ++l) {
                    const double tau = l * h;
                    if (c.scheme == 2) {
                        poly(tau, cw);
                        fwd_stage(U, with_src, t + tau, cw, U, nullptr, 0.0, 0.5 * h, Zs, 0.0, 0.0, nullptr);
                        poly(tau + 0.5 * h, cw);
                        fwd_stage(Zs, with_src, t + tau + 0.5 * h, cw, U, nullptr, 0.0, h, U, 0.0, 0.0, nullptr);
                    } else {
                        poly(tau, cw);
                        fwd_stage(U, with_src, t + tau, cw, U, nullptr, 0.0, 0.5 * h, Zs, 0.0, h / 6.0, Acc);
                        poly(tau + 0.5 * h, cw);
                        fwd_stage(Zs, with_src, t + tau + 0.5 * h, cw, U, Acc, 0.0, 0.5 * h, Zs2, 1.0, h / 3.0, Acc);
                        fwd_stage(Zs2, with_src, t + tau + 0.5 * h, cw, U, Acc, 0.0, h, Zs, 1.0, h / 3.0, Acc);
                        poly(tau + h, cw);
                        fwd_stage(Zs, with_src, t + tau + h, cw, U, Acc, 1.0, h / 6.0, U, 0.0, 0.0, nullptr);
                    }
                }
            }
            // every other unknown: z = y + sum_k al_k W_k + the quadrature of F,
            // with W_k = D_{k+1} - F^(k)(t) for k < p - 1
            double sc = 0, ss = 0;
            if (with_src) {
                for (int l = 0; l < m; ++l)
                    for (int si = 0; si < ns; ++si) {
                        const double x = w * (t + l * h + st_off[si] * h);
                        sc += st_b[si] * h * std::cos(x);
                        ss += st_b[si] * h * std::sin(x);
                    }
                for (int k = 0; k + 1 < order; ++k) {
                    const double phk = w * t + k * 0.5 * M_PI, amp = std::pow(w, k);
                    sc -= al[k] * amp * std::cos(phk);
                    ss -= al[k] * amp * std::sin(phk);
                }
            }
            const void* Wc[4] = {D[1], order > 2 ? D[2] : W[1], order > 2 ? D[3] : nullptr,
                                 order > 2 ? W[3] : nullptr};
            launch_lts_closed(prec, n, np6, s.Np, hbmask, Wc, al, order, with_src ? p->Sre.p : nullptr, p->Sim.p,
                              p->src_rows, sc, ss, U, st);
        }
        rhs_on(nullptr, 0);
        if (filt) {
            if (c.scheme == 2) {
                launch_filter_add(prec, U, 1.0 / M, 0.0, p->Fre.as<double>(), p->Fim.as<double>(), n, st);
            } else {
                rhs(U, D[1], with_src, M * H, 0, nullptr, 0);
                const std::complex<double> wa = twoT * ph(M - 1) * xi[1], wb = twoT * ph(M - 1) * xi[3];
                launch_filter_add2(prec, U, wa.real(), wa.imag(), D[1], wb.real(), wb.imag(), p->Fre.as<double>(),
                                   p->Fim.as<double>(), n, st);
            }
        }
        return;
    }

    // adjoint of the homogeneous step, M times (S-flipped variables: zbar = U);
    // the substeps' vectors live on the halo blocks, B runs on the fine blocks
    // (only its fine rows are used), the coarse rows' wbar_k = al_k zbar_end.
    // The forward's Taylor part, written with the halo-block mask h,
    //   D_{k+1} = B D_k,  W_k = h B (I - P) D_k + (1 - h) D_{k+1} (k < p - 1),
    //   W_{p-1} = B (I - P) D_{p-1},
    // transposes to A_{p-1} = (I - P) B wbar_{p-1} + (1 - h) wbar_{p-2},
    //   A_{j-1} = B A_j + (I - P) B (h wbar_{j-1}) [+ (1 - h) wbar_{j-2}],
    //   ybar = zbar + A_0,
    // where B (h x) is needed on the blocks of the halo blocks' elements and
    // their face neighbours only.
    void* KA = Zs;
    void* KB = Zs2;
    void* Z0 = p->lZ0.p;
    // one adjoint substep stage on the halo blocks, fused with its
    // combination: A = B kcur on the fine rows (0 elsewhere); zbar += A;
    // knext = a0 Z0 + b0 A; wbar_j += cw_j kcur on the fine rows (= when
    // init: the coarse step's first stage); the substep's last stage also
    // starts the next substep: Z0 = zbar, KA = kc zbar (z0next, knext2)
    auto adj_stage = [&](const void* kcur, const double* cw, double a0, double b0, void* knext, bool init = false,
                         void* z0next = nullptr, void* knext2 = nullptr, double kc = 0.0) {
        a.Y = kcur;
        a.U = U;
        a.Uout = U;
        a.Acc = Z0;
        a.Ynext = knext;
        a.Kout = nullptr;
        a.imask = nullptr;
        a.src_rows = 0;
        a.mode = LTS_ADJ;
        a.le = a0;
        a.lf = b0;
        a.lmask = fine;
        a.lnw = order;
        for (int j = 0; j < order; ++j) {
            a.lw[j] = WB[j];
            a.lcw[j] = cw[j];
        }
        a.linit = init ? 1 : 0;
        a.lz = z0next;
        a.lk = knext2;
        a.lkc = kc;
        a.blist = hbl;
        a.nblist = nhb;
        stage_dim(s, a, st);
        a.mode = RHS;
        a.Acc = a.Ynext = a.Uout = nullptr;
        a.lnw = 0;
        a.lmask = nullptr;
        a.linit = 0;
        a.lz = a.lk = nullptr;
        a.lkc = 0.0;
        a.blist = nullptr;
        a.nblist = 0;
    };
    // out = [rows of maskA ^ invA] B x + [outside the halo blocks] X
    //       + [near the halo, outside the fine elements] Z + Y  (full launch)
    const uint32_t* h2nf = p->lts_h2nf.as<uint32_t>();
    auto chain = [&](const void* x, const uint32_t* maskA, int invA, const void* X, const void* Z, const void* Yadd,
                     void* out) {
        a.Y = x;
        a.U = nullptr;
        a.Uout = out;
        a.Acc = a.Ynext = a.Kout = nullptr;
        a.imask = nullptr;
        a.src_rows = 0;
        a.mode = LTS_CHAIN;
        a.lmask = maskA;
        a.linv = invA;
        a.lmaskB = hbmask;
        a.linvB = 1;
        a.lmaskC = h2nf;
        a.linvC = 0;
        a.lw[0] = X;
        a.lw[1] = Z;
        a.lw[2] = Yadd;
        a.lnw = 0;
        a.blist = nullptr;
        a.nblist = 0;
        stage_dim(s, a, st);
        a.mode = RHS;
        a.Uout = nullptr;
        a.lmask = a.lmaskB = a.lmaskC = nullptr;
        a.lw[0] = a.lw[1] = a.lw[2] = nullptr;
    };
    const int* h2l = p->lts_h2blocks.as<int>();
    const int64_t nh2b = p->lts_nh2b;
    for (int nn = 0; nn < M; ++nn) {
        if (nhb > 0) {
            // the substeps accumulate wbar on the fine rows (the first stage
            // sets it); each substep starts from Z0 = zbar and its first
            // stage vector kc zbar, formed here for the first substep and by
            // the previous substep's last stage for the others
            double cw[4];
            const double kc = c.scheme == 2 ? h : h / 6.0;  // kbar2 = h zbar, kbar4 = h/6 zbar
            for (int l = m - 1; l >= 0; --l) {
                const double tau = l * h;
                const bool first = l == m - 1;
                if (first) {
                    launch_lts_axpy(prec, n, np6, hbl, nhb, nullptr, 0, 0.0, nullptr, 1.0, U, Z0, st);  // Z0 = zbar
                    launch_lts_axpy(prec, n, np6, hbl, nhb, nullptr, 0, 0.0, nullptr, kc, Z0, KA, st);
                }
                void* zn = l > 0 ? Z0 : nullptr;
                void* kn = l > 0 ? KA : nullptr;
                if (c.scheme == 2) {
                    poly(tau + 0.5 * h, cw);
                    adj_stage(KA, cw, 0.0, 0.5 * h, KB, first);
                    poly(tau, cw);
                    adj_stage(KB, cw, 0.0, 0.0, nullptr, false, zn, kn, kc);
                } else {
                    poly(tau + h, cw);
                    adj_stage(KA, cw, h / 3.0, h, KB, first);
                    poly(tau + 0.5 * h, cw);
                    adj_stage(KB, cw, h / 3.0, 0.5 * h, KA);
                    adj_stage(KA, cw, h / 6.0, 0.5 * h, KB);
                    poly(tau, cw);
                    adj_stage(KB, cw, 0.0, 0.0, nullptr, false, zn, kn, kc);
                }
            }
        }
        // coarse rows: wbar_k = al_k zbar (zbar there is the step's end value)
        launch_lts_wbar_close(prec, n, np6, fine, U, WB, al, order, st);
        // A_{p-1} = (I - P) B wbar_{p-1} + (1 - h) wbar_{p-2}, then the chain;
        // each step one right-hand side near the halo and one full launch whose
        // update pass forms the sum (outputs alternate between Kb and the
        // consumed wbar vector: a launch never writes its own input)
        chain(WB[order - 1], fine, 1, WB[order - 2], nullptr, nullptr, Kb);
        void* Ain = Kb;
        for (int j = order - 1; j >= 1; --j) {
            if (nh2b > 0) {  // B (h wbar_{j-1}) near the halo
                rhs_on(h2l, nh2b);
                rhs(WB[j - 1], KA, false, 0.0, 0, hbmask, 0);
                rhs_on(nullptr, 0);
            }
            void* out = j == 1 ? U : (Ain == Kb ? WB[j] : Kb);
            // A_{j-1} = B A_j + (1 - h) wbar_{j-2} + (I - P) B (h wbar_{j-1});
            // ybar = zbar + A_0
            chain(Ain, nullptr, 0, j >= 2 ? WB[j - 2] : nullptr, nh2b > 0 ? KA : nullptr, j == 1 ? U : nullptr,
                  out);
            Ain = out;
        }
    }
}

}  // namespace cmcg
