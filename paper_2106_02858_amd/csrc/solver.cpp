// Host side of the CMCG Maxwell library: object lifetimes, the period driver
// (Section 5.3 RK2 / RK4 over one period, hipGraph replay), the on-the-fly
// filter weights (Section 5.4), the CMCG controller (Section 2.2, Algorithms
// 1-3) and the extern "C" entry points declared in include/cmcg.h.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>

#include <array>
#include <tuple>

#include "objects.h"

namespace cmcg {

namespace {
thread_local std::string g_last_error;
}

void fail(int code, const std::string& msg) { throw Error{code, msg}; }
void set_last_error(const std::string& msg) { g_last_error = msg; }

std::shared_ptr<MeshData> build_mesh(int64_t nv, const double* xyz, int64_t K, const int64_t* tet,
                                     const int8_t* face_tag);
std::shared_ptr<MeshData> build_mesh2d(int64_t nv, const double* xy, int64_t K, const int64_t* tri,
                                       const int8_t* edge_tag);
void locality_order(int64_t nv, const double* xyz, int64_t K, const int64_t* tet, int64_t* order);

// ----------------------------------------------------------- device constants
namespace {
std::mutex g_const_mu;
bool g_const_done[64][kMaxQ + 1];
bool g_const2_done[64][kMaxQ + 1];
}

void ensure_constants(int device, int q, int dim) {
    std::lock_guard<std::mutex> lk(g_const_mu);
    if (device < 0 || device >= 64) fail(CMCG_ERR_DEVICE, "device index out of range");
    if (dim == 2) {
        if (g_const2_done[device][q]) return;
        const RefElem2D& r = ref_elem2d(q);
        upload_constants2d(q, r.D.data(), r.LIFT.data(), r.M.data(), r.fnode.data());
        g_const2_done[device][q] = true;
        return;
    }
    if (g_const_done[device][q]) return;
    const RefElem& r = ref_elem(q);
    upload_constants(q, 0, r.D.data(), r.LIFT.data(), r.M.data(), r.fnode.data(), r.fperm.data());
    g_const_done[device][q] = true;
}

int current_device() {
    int d = 0;
    CMCG_HIP(hipGetDevice(&d));
    return d;
}

// Hermite weights xi_ij = int_0^dt h_ij(s) e^{-i w s} ds by the power series
// of the exponential (long double), h_ij the cubic Hermite basis on [0, dt].
void hermite_weights(double omega, double dt, std::complex<double> xi[4]) {
    using LD = long double;
    const LD th = (LD)omega * (LD)dt;
    std::complex<LD> mu[4];
    for (int k = 0; k < 4; ++k) {
        std::complex<LD> s = 0, term = 1;  // (-i th)^n / n!
        for (int n = 0; n < 60; ++n) {
            s += term / (LD)(n + k + 1);
            term *= std::complex<LD>(0, -th) / (LD)(n + 1);
            if (std::abs(term) < 1e-40L) break;
        }
        mu[k] = s;
    }
    const LD h = dt;
    xi[0] = std::complex<double>(h * (mu[0] - (LD)3 * mu[2] + (LD)2 * mu[3]));
    xi[1] = std::complex<double>(h * ((LD)3 * mu[2] - (LD)2 * mu[3]));
    xi[2] = std::complex<double>(h * h * (mu[1] - (LD)2 * mu[2] + mu[3]));
    xi[3] = std::complex<double>(h * h * (mu[3] - mu[2]));
}

}  // namespace cmcg

namespace cmcg {

// ------------------------------------------------------------- problem setup
// 2-D: G[4] | per edge n[2], cE1, cE2, cH1, cH2 | 1/eps, 1/mu, sigma/eps
static void build_geo2d(cmcg_problem* p, double alpha, std::vector<double>& g) {
    const SpaceData& s = *p->sp;
    const MeshData& m = *s.mesh;
    const int64_t K = s.K;
    g.assign(kGeo2 * K, 0.0);
    for (int64_t e = 0; e < K; ++e) {
        double* o = &g[kGeo2 * e];
        for (int i = 0; i < 4; ++i) o[i] = m.G[4 * e + i];
        const double Zm = std::sqrt(p->mu[e] / p->eps[e]);
        for (int f = 0; f < 3; ++f) {
            double* q = o + 4 + 6 * f;
            q[0] = m.normal[6 * e + 2 * f];
            q[1] = m.normal[6 * e + 2 * f + 1];
            const int64_t nb = m.nbr[3 * e + f];
            const double Zp = nb >= 0 ? std::sqrt(p->mu[nb] / p->eps[nb]) : Zm;
            const double Ym = 1.0 / Zm, Yp = 1.0 / Zp;
            const double al = (nb < 0 && m.tag[3 * e + f] == CMCG_TAG_IMPEDANCE) ? 1.0 : alpha;
            const double fs = m.area[3 * e + f] / m.vol[e];
            q[2] = fs * al / (Zm + Zp);
            q[3] = fs * Zp / (Zm + Zp);
            q[4] = fs * al / (Ym + Yp);
            q[5] = fs * Yp / (Ym + Yp);
        }
        o[22] = 1.0 / p->eps[e];
        o[23] = 1.0 / p->mu[e];
        o[24] = p->sigma[e] / p->eps[e];
    }
}

void build_geo(cmcg_problem* p, double alpha) {
    const SpaceData& s = *p->sp;
    const MeshData& m = *s.mesh;
    const int64_t K = s.K;
    std::vector<double> g;
    if (s.dim == 2) {
        build_geo2d(p, alpha, g);
    } else {
    g.assign(kGeo * K, 0.0);
    for (int64_t e = 0; e < K; ++e) {
        double* o = &g[kGeo * e];
        for (int i = 0; i < 9; ++i) o[i] = m.G[9 * e + i];
        const double Zm = std::sqrt(p->mu[e] / p->eps[e]);
        for (int f = 0; f < 4; ++f) {
            double* q = o + 9 + 7 * f;
            for (int k = 0; k < 3; ++k) q[k] = m.normal[12 * e + 3 * f + k];
            const int64_t nb = m.nbr[4 * e + f];
            const double Zp = nb >= 0 ? std::sqrt(p->mu[nb] / p->eps[nb]) : Zm;
            const double Ym = 1.0 / Zm, Yp = 1.0 / Zp;
            const double al = (nb < 0 && m.tag[4 * e + f] == CMCG_TAG_IMPEDANCE) ? 1.0 : alpha;
            const double fs = m.area[4 * e + f] / m.vol[e];
            q[3] = fs * al / (Zm + Zp);
            q[4] = fs * Zp / (Zm + Zp);
            q[5] = fs * al / (Ym + Yp);
            q[6] = fs * Yp / (Ym + Yp);
        }
        o[37] = 1.0 / p->eps[e];
        o[38] = 1.0 / p->mu[e];
        o[39] = p->sigma[e] / p->eps[e];
    }
    }
    p->geo.alloc(g.size() * s.esize());
    if (s.precision == CMCG_FP64) {
        CMCG_HIP(hipMemcpy(p->geo.p, g.data(), g.size() * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> gf(g.begin(), g.end());
        CMCG_HIP(hipMemcpy(p->geo.p, gf.data(), gf.size() * 4, hipMemcpyHostToDevice));
    }
    p->geo_alpha = alpha;
}

static void upload_field(const SpaceData& s, DevBuf& b, const std::vector<double>& v) {
    b.alloc(v.size() * s.esize());
    if (s.precision == CMCG_FP64) {
        CMCG_HIP(hipMemcpy(b.p, v.data(), v.size() * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(v.begin(), v.end());
        CMCG_HIP(hipMemcpy(b.p, f.data(), f.size() * 4, hipMemcpyHostToDevice));
    }
}

// 2-D source: j [nh][K][Np] on the e row (harmonic h at hstride = ndof);
// impedance data G [K][3][Nfp] (one frequency) through the ghost e+ = G, h+ = 0
// of the wall edges: flux_e = G / (2 Z), flux_h = (n2 G, -n1 G) / 2, lifted
// with the edge scaling.
static void build_source2d(cmcg_problem* p, const double* j_re, const double* j_im, const double* g_re,
                           const double* g_im, int nh) {
    const SpaceData& s = *p->sp;
    const MeshData& m = *s.mesh;
    const int64_t K = s.K;
    const int Np = s.Np, Nfp = s.Nfp;
    const int64_t nj = nh * K * Np, ng = K * 3 * (int64_t)Nfp;
    for (const double* a : {j_re, j_im})
        if (a)
            for (int64_t i = 0; i < nj; ++i)
                if (!std::isfinite(a[i])) fail(CMCG_ERR_ARG, "problem: non-finite current density");
    for (const double* a : {g_re, g_im})
        if (a)
            for (int64_t i = 0; i < ng; ++i)
                if (!std::isfinite(a[i])) fail(CMCG_ERR_ARG, "problem: non-finite boundary data");
    p->has_j = j_re || j_im;
    p->has_g = g_re || g_im;
    if (!p->has_j && !p->has_g) return;
    std::vector<double> sr(s.ndof * nh, 0.0), si(s.ndof * nh, 0.0);
    for (int h = 0; h < nh; ++h)
        for (int64_t e = 0; e < K; ++e)
            for (int i = 0; i < Np; ++i) {
                const int64_t src = (h * K + e) * Np + i, dst = h * s.ndof + e * 3 * Np + i;
                if (j_re) sr[dst] = j_re[src] / p->eps[e];
                if (j_im) si[dst] = j_im[src] / p->eps[e];
            }
    if (p->has_g) {
        const RefElem2D& r = ref_elem2d(s.q);
        for (int64_t e = 0; e < K; ++e) {
            const double Z = std::sqrt(p->mu[e] / p->eps[e]);
            for (int f = 0; f < 3; ++f) {
                if (m.nbr[3 * e + f] >= 0 || m.tag[3 * e + f] != CMCG_TAG_IMPEDANCE) continue;
                const double n1 = m.normal[6 * e + 2 * f], n2 = m.normal[6 * e + 2 * f + 1];
                const double fs = m.area[3 * e + f] / m.vol[e];
                for (int part = 0; part < 2; ++part) {
                    const double* gsrc = part == 0 ? g_re : g_im;
                    if (!gsrc) continue;
                    std::vector<double>& S = part == 0 ? sr : si;
                    for (int k = 0; k < Nfp; ++k) {
                        const double G = gsrc[(e * 3 + f) * Nfp + k];
                        for (int i = 0; i < Np; ++i) {
                            const double L = r.LIFT[i * 3 * Nfp + f * Nfp + k] * fs;
                            S[(e * 3) * Np + i] += L * G / (2 * Z) / p->eps[e];
                            S[(e * 3 + 1) * Np + i] += L * (n2 * G) / 2 / p->mu[e];
                            S[(e * 3 + 2) * Np + i] += L * (-n1 * G) / 2 / p->mu[e];
                        }
                    }
                }
            }
        }
    }
    upload_field(s, p->Sre, sr);
    upload_field(s, p->Sim, si);
    p->src_rows = p->has_g ? 3 : 1;
}

// j_re / j_im: [nh][K][Np][3] (harmonic h with frequency ks[h] omega; nh = 1,
// ks = NULL for a single frequency); g only for a single frequency.  2-D
// spaces: j [K][Np], g [K][3][Nfp], a single frequency.
static cmcg_problem* make_problem(const cmcg_space* sh, const double* eps, const double* mu, const double* sigma,
                                  double omega, const double* j_re, const double* j_im, const double* g_re,
                                  const double* g_im, int nh = 1, const int* ks = nullptr) {
    if (!sh || !sh->d) fail(CMCG_ERR_ARG, "problem: NULL space");
    if (!eps || !mu) fail(CMCG_ERR_ARG, "problem: NULL eps or mu");
    if (!(omega > 0) || !std::isfinite(omega)) fail(CMCG_ERR_ARG, "problem: omega must be positive");
    auto sp = sh->d;
    if (current_device() != sp->device) fail(CMCG_ERR_STATE, "problem: wrong current device");
    const int64_t K = sp->K;
    const int Np = sp->Np, Nfp = sp->Nfp;
    if (nh < 1 || nh > kMaxHarm) fail(CMCG_ERR_ARG, "problem: 1 to 8 harmonics");
    std::unique_ptr<cmcg_problem> p(new cmcg_problem());
    p->sp = sp;
    p->omega = omega;
    p->nharm = nh;
    p->kharm.assign(nh, 1);
    if (ks) {
        for (int h = 0; h < nh; ++h) {
            if (ks[h] < 1) fail(CMCG_ERR_ARG, "problem: harmonic numbers must be positive");
            for (int h2 = 0; h2 < h; ++h2)
                if (ks[h2] == ks[h]) fail(CMCG_ERR_ARG, "problem: harmonic numbers must be distinct");
            p->kharm[h] = ks[h];
        }
    }
    if (nh > 1 && (g_re || g_im)) fail(CMCG_ERR_ARG, "problem: boundary data only for a single frequency");
    p->eps.assign(eps, eps + K);
    p->mu.assign(mu, mu + K);
    p->sigma.assign(K, 0.0);
    if (sigma) p->sigma.assign(sigma, sigma + K);
    for (int64_t e = 0; e < K; ++e) {
        if (!(p->eps[e] > 0) || !(p->mu[e] > 0) || !std::isfinite(p->eps[e]) || !std::isfinite(p->mu[e]))
            fail(CMCG_ERR_ARG, "problem: eps and mu must be positive and finite");
        if (!(p->sigma[e] >= 0) || !std::isfinite(p->sigma[e]))
            fail(CMCG_ERR_ARG, "problem: sigma must be non-negative and finite");
    }
    const MeshData& m = *sp->mesh;
    // mass weights of the eps,mu inner product
    std::vector<double> we(K), wh(K);
    for (int64_t e = 0; e < K; ++e) {
        we[e] = m.vol[e] * p->eps[e];
        wh[e] = m.vol[e] * p->mu[e];
    }
    p->wE.alloc(K * 8);
    p->wH.alloc(K * 8);
    CMCG_HIP(hipMemcpy(p->wE.p, we.data(), K * 8, hipMemcpyHostToDevice));
    CMCG_HIP(hipMemcpy(p->wH.p, wh.data(), K * 8, hipMemcpyHostToDevice));
    // per-device set-up that the allocation-free entry point relies on: the
    // reference matrices of this order and the address of the scratch array
    ensure_constants(sp->device, sp->q, sp->dim);
    (void)noalloc_scratch(sp->device);
    if (sp->dim == 2) {
        build_source2d(p.get(), j_re, j_im, g_re, g_im, nh);
        build_geo(p.get(), 1.0);
        p->pinned.reset(new HostPinned());
        return p.release();
    }
    // source vector S with Re(S e^{i w t}) = the forcing of Phi
    const int64_t nj = (int64_t)nh * K * Np * 3;
    for (const double* a : {j_re, j_im})
        if (a)
            for (int64_t i = 0; i < nj; ++i)
                if (!std::isfinite(a[i])) fail(CMCG_ERR_ARG, "problem: non-finite current density");
    const int64_t ng = K * 4 * (int64_t)Nfp * 3;
    for (const double* a : {g_re, g_im})
        if (a)
            for (int64_t i = 0; i < ng; ++i)
                if (!std::isfinite(a[i])) fail(CMCG_ERR_ARG, "problem: non-finite boundary data");
    p->has_j = j_re || j_im;
    p->has_g = g_re || g_im;
    if (p->has_j || p->has_g) {
        std::vector<double> sr(sp->ndof * nh, 0.0), si(sp->ndof * nh, 0.0);
        for (int h = 0; h < nh; ++h)
            for (int64_t e = 0; e < K; ++e)
                for (int c = 0; c < 3; ++c)
                    for (int i = 0; i < Np; ++i) {
                        const int64_t src = ((h * K + e) * Np + i) * 3 + c;
                        const int64_t dst = h * sp->ndof + (e * 6 + c) * Np + i;
                        if (j_re) sr[dst] = j_re[src] / p->eps[e];
                        if (j_im) si[dst] = j_im[src] / p->eps[e];
                    }
        if (p->has_g) {
            // ghost E+ = n x G on impedance faces: flux_E = (n x G)/(2Z),
            // flux_H = n x (n x G) / 2, lifted with the face scaling
            const RefElem& r = ref_elem(sp->q);
            for (int64_t e = 0; e < K; ++e) {
                const double Z = std::sqrt(p->mu[e] / p->eps[e]);
                for (int f = 0; f < 4; ++f) {
                    if (m.nbr[4 * e + f] >= 0 || m.tag[4 * e + f] != CMCG_TAG_IMPEDANCE) continue;
                    const double* n = &m.normal[12 * e + 3 * f];
                    const double fs = m.area[4 * e + f] / m.vol[e];
                    for (int k = 0; k < Nfp; ++k) {
                        for (int part = 0; part < 2; ++part) {
                            const double* gsrc = part == 0 ? g_re : g_im;
                            if (!gsrc) continue;
                            const double* G = &gsrc[((e * 4 + f) * Nfp + k) * 3];
                            const double nG[3] = {n[1] * G[2] - n[2] * G[1], n[2] * G[0] - n[0] * G[2],
                                                  n[0] * G[1] - n[1] * G[0]};
                            const double nnG[3] = {n[1] * nG[2] - n[2] * nG[1], n[2] * nG[0] - n[0] * nG[2],
                                                   n[0] * nG[1] - n[1] * nG[0]};
                            std::vector<double>& S = part == 0 ? sr : si;
                            for (int i = 0; i < Np; ++i) {
                                const double L = r.LIFT[i * 4 * Nfp + f * Nfp + k] * fs;
                                for (int c = 0; c < 3; ++c) {
                                    S[(e * 6 + c) * Np + i] += L * nG[c] / (2 * Z) / p->eps[e];
                                    S[(e * 6 + 3 + c) * Np + i] += L * nnG[c] / 2 / p->mu[e];
                                }
                            }
                        }
                    }
                }
            }
        }
        upload_field(*sp, p->Sre, sr);
        upload_field(*sp, p->Sim, si);
        p->src_rows = p->has_g ? 6 : 3;
        p->smask.alloc(source_mask_words(K) * 4);
        launch_source_mask(sp->precision, Np, p->Sre.p, p->Sim.p, nh, sp->ndof, K, p->smask.as<uint32_t>(), nullptr);
        CMCG_HIP(hipStreamSynchronize(nullptr));
    }
    build_geo(p.get(), 1.0);
    p->pinned.reset(new HostPinned());
    return p.release();
}

// -------------------------------------------------------------- time stepping
StepCfg step_config(const cmcg_problem* p, const cmcg_options* o) {
    const SpaceData& s = *p->sp;
    StepCfg c;
    c.scheme = o->scheme == CMCG_SCHEME_AUTO ? (s.q == 1 ? 2 : 4) : o->scheme;
    if (c.scheme != 2 && c.scheme != 4) fail(CMCG_ERR_ARG, "options: scheme must be AUTO, RK2 or RK4");
    if (o->flux != CMCG_FLUX_UPWIND && o->flux != CMCG_FLUX_CENTRED) fail(CMCG_ERR_ARG, "options: bad flux");
    c.alpha = o->flux == CMCG_FLUX_UPWIND ? 1.0 : 0.0;
    c.T = 2.0 * M_PI / p->omega;
    // 3-D: c_1 = 0.20 (readings for tetrahedra); 2-D: the paper's c_1 = 0.24, c_3 = 0.12
    const double c1 = s.dim == 2 ? 0.24 : 0.20;
    c.cq = o->cfl > 0 ? o->cfl : (s.q == 1 ? c1 : s.q == 2 ? 0.16 : 0.12);
    if (o->lts_ratio < 0 || o->lts_ratio > 64) fail(CMCG_ERR_ARG, "options: lts_ratio must be 0..64");
    c.lts = o->lts_ratio > 1 ? o->lts_ratio : 1;
    if (c.lts > 1 && (s.dim != 3 || p->nharm != 1))
        fail(CMCG_ERR_ARG, "options: local time stepping needs a tetrahedral space and one frequency");
    if (o->steps > 0) {
        c.M = o->steps;
    } else {
        const double cq = c.cq;
        const MeshData& m = *s.mesh;
        double mn = HUGE_VAL;
        for (int64_t e = 0; e < s.K; ++e) mn = std::fmin(mn, std::sqrt(p->mu[e] * p->eps[e]) * m.rho[e]);
        // local time stepping: the coarse step may be lts times the smallest
        // element's step (its m substeps then meet that element's CFL rule)
        const double dtmax = cq * mn * c.lts;
        long long M = (long long)std::ceil(c.T / dtmax);
        if (M < 1) M = 1;
        while (c.T / (double)M > dtmax) ++M;
        while (M > 1 && c.T / (double)(M - 1) <= dtmax) --M;
        if (M > 100000000LL) fail(CMCG_ERR_ARG, "options: more than 1e8 steps per period");
        c.M = (int)M;
    }
    if (c.M < 3) fail(CMCG_ERR_ARG, "options: at least 3 steps per period are required");
    c.dt = c.T / c.M;
    return c;
}

static void ensure_work(cmcg_problem* p) {
    const SpaceData& s = *p->sp;
    const size_t fb = s.ndof * s.esize(), db = s.ndof * 8;
    p->U.alloc(fb);
    p->Y1.alloc(fb);
    p->Y2.alloc(fb);
    p->Acc.alloc(fb);
    if (s.precision == CMCG_FP32) p->Ulo.alloc(s.ndof * 2);
    p->Fre.alloc(db * p->nharm);
    p->Fim.alloc(db * p->nharm);
    p->partial.alloc(dot_partials() * 8);
    p->scal.alloc(64);
}

// Inner product dispatch by dimension (stage and field conversions: objects.h).
static void dot_for(cmcg_problem* p, const double* U, const double* V, double* out_dev, hipStream_t st) {
    const SpaceData& s = *p->sp;
    if (s.dim == 2)
        launch_dot2d(s.q, U, V, p->wE.as<double>(), p->wH.as<double>(), s.K, p->partial.as<double>(), out_dev, st);
    else
        launch_dot(s.q, U, V, p->wE.as<double>(), p->wH.as<double>(), s.K, p->partial.as<double>(), out_dev, st);
}

static StageArgs base_args(cmcg_problem* p) {
    const SpaceData& s = *p->sp;
    StageArgs a{};
    a.geo = p->geo.p;
    a.conn = s.conn.as<int>();
    a.K = s.K;
    a.Sre = p->Sre.p;
    a.Sim = p->Sim.p;
    a.smask = p->smask.as<uint32_t>();
    a.Fre = p->Fre.as<double>();
    a.Fim = p->Fim.as<double>();
    a.Ulo = p->Ulo.p;
    a.nharm = p->nharm;
    a.hstride = s.ndof;
    return a;
}

// Steps m0 .. m1-1 of a period in place on p->U (field precision).  With
// `filt` (whole periods only), F = (2/T) int U e^{-i w t} is accumulated into
// Fre / Fim (zeroed here).
static void enqueue_steps(cmcg_problem* p, const StepCfg& c, bool src, bool filt, int m0, int m1,
                          hipStream_t st) {
    const SpaceData& s = *p->sp;
    const int prec = s.precision;
    const int M = c.M;
    const double dt = c.dt;
    const double two_pi = 2.0 * M_PI;
    StageArgs a = base_args(p);
    a.src_rows = (src && p->src_rows) ? p->src_rows : 0;
    if (filt) {
        launch_zero(p->Fre.p, p->Fre.bytes, st);
        launch_zero(p->Fim.p, p->Fim.bytes, st);
    }
    // harmonic h has frequency k_h omega (k = 1 for a single-frequency problem)
    const int H = p->nharm;
    std::vector<std::array<std::complex<double>, 4>> xi(H);
    if (filt && c.scheme == 4)
        for (int h = 0; h < H; ++h) hermite_weights(p->kharm[h] * p->omega, dt, xi[h].data());
    const double twoT = 2.0 / c.T;
    // e^{-i k_h omega t_m}
    auto ph = [&](int h, double m) {
        const double x = two_pi * p->kharm[h] * m / M;
        return std::complex<double>(std::cos(x), -std::sin(x));
    };
    auto set_src = [&](double mm) {
        for (int h = 0; h < H; ++h) {
            const double phase = two_pi * p->kharm[h] * mm / M;
            (h == 0 ? a.scos : a.hcos[h]) = std::cos(phase);
            (h == 0 ? a.ssin : a.hsin[h]) = std::sin(phase);
        }
    };
    auto set_filter = [&](int h, std::complex<double> wa, std::complex<double> wb) {
        (h == 0 ? a.fa_re : a.hfa_re[h]) = wa.real();
        (h == 0 ? a.fa_im : a.hfa_im[h]) = wa.imag();
        (h == 0 ? a.fb_re : a.hfb_re[h]) = wb.real();
        (h == 0 ? a.fb_im : a.hfb_im[h]) = wb.imag();
    };
    for (int m = m0; m < m1; ++m) {
        a.filter = 0;
        if (c.scheme == 2) {
            // stage 1: k1 = Phi(t_m, U); Y1 = U + dt/2 k1
            a.mode = RK2_S1;
            a.Y = p->U.p;
            a.U = p->U.p;
            a.Ynext = p->Y1.p;
            a.cy = 0.5 * dt;
            set_src(m);
            if (filt) {
                // trapezoid: weight (1/M) e^{-i w t_m}, doubled for interior levels
                a.filter = 1;
                for (int h = 0; h < H; ++h) set_filter(h, ph(h, m) * ((m == 0 ? 1.0 : 2.0) / M), 0.0);
            }
            stage_dim(s, a, st);
            a.filter = 0;
            // stage 2: k2 = Phi(t_m + dt/2, Y1); U += dt k2
            a.mode = RK2_S2;
            a.Y = p->Y1.p;
            a.U = p->U.p;
            a.Uout = p->U.p;
            a.cu = dt;
            set_src(m + 0.5);
            stage_dim(s, a, st);
        } else {
            a.mode = RK4_S1;
            a.Y = p->U.p;
            a.U = p->U.p;
            a.Ynext = p->Y1.p;
            a.Acc = p->Acc.p;
            a.cy = 0.5 * dt;
            a.ca = dt / 6.0;
            set_src(m);
            if (filt) {
                // Hermite: U_m and Phi_m weights of the intervals [t_{m-1}, t_m], [t_m, t_{m+1}]
                a.filter = 1;
                for (int h = 0; h < H; ++h) {
                    std::complex<double> wa = twoT * ph(h, m) * xi[h][0], wb = twoT * ph(h, m) * xi[h][2];
                    if (m >= 1) {
                        wa += twoT * ph(h, m - 1) * xi[h][1];
                        wb += twoT * ph(h, m - 1) * xi[h][3];
                    }
                    set_filter(h, wa, wb);
                }
            }
            stage_dim(s, a, st);
            a.filter = 0;
            a.mode = RK4_S2;
            a.Y = p->Y1.p;
            a.Ynext = p->Y2.p;
            a.cy = 0.5 * dt;
            a.ca = dt / 3.0;
            set_src(m + 0.5);
            stage_dim(s, a, st);
            a.mode = RK4_S3;
            a.Y = p->Y2.p;
            a.Ynext = p->Y1.p;
            a.cy = dt;
            a.ca = dt / 3.0;
            stage_dim(s, a, st);
            a.mode = RK4_S4;
            a.Y = p->Y1.p;
            a.Uout = p->U.p;
            a.cu = dt / 6.0;
            set_src(m + 1.0);
            stage_dim(s, a, st);
        }
    }
    if (filt && m1 == M) {
        if (c.scheme == 2) {
            // last level t_M = T: e^{-i k_h w T} = 1
            for (int h = 0; h < H; ++h)
                launch_filter_add(prec, p->U.p, 1.0 / M, 0.0, p->Fre.as<double>() + h * s.ndof,
                                  p->Fim.as<double>() + h * s.ndof, s.ndof, st);
        } else {
            // last level: Phi(t_M, U_M) and the weights of [t_{M-1}, t_M]
            p->Kbuf.alloc(s.ndof * s.esize());
            a.mode = RHS;
            a.Y = p->U.p;
            a.U = p->U.p;
            a.Kout = p->Kbuf.p;
            set_src(M);
            a.filter = 1;
            for (int h = 0; h < H; ++h)
                set_filter(h, twoT * ph(h, M - 1) * xi[h][1], twoT * ph(h, M - 1) * xi[h][3]);
            stage_dim(s, a, st);
        }
    }
}

// One period of M steps in place on p->U.
static void enqueue_period(cmcg_problem* p, const StepCfg& c, bool src, bool filt, hipStream_t st) {
    enqueue_steps(p, c, src, filt, 0, c.M, st);
}

static void run_period(cmcg_problem* p, const StepCfg& c, bool src, bool filt, bool use_graph, hipStream_t st) {
    if (!use_graph) {
        enqueue_period(p, c, src, filt, st);
        return;
    }
    // the stage variant is read when the launches are enqueued, so a graph
    // captured under one variant must not be replayed after another is chosen
    // (variant + 1: the size-based default is -1, which must not spill into the step count's bits)
    const int variant = p->sp->dim == 3 ? get_stage_variant(p->sp->q, p->sp->precision) : 0;
    const int64_t key = ((int64_t)c.M << 12) | ((int64_t)(variant + 1) << 8) | (c.scheme << 4) | (src ? 2 : 0) |
                        (filt ? 1 : 0);
    auto it = p->graphs.find(key);
    if (it == p->graphs.end()) {
        if (!p->cap_stream) CMCG_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        if (filt && c.scheme == 4) p->Kbuf.alloc(p->sp->ndof * p->sp->esize());
        CMCG_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_period(p, c, src, filt, p->cap_stream);
        } catch (...) {
            hipGraph_t g;
            (void)hipStreamEndCapture(p->cap_stream, &g);
            throw;
        }
        hipGraph_t g;
        CMCG_HIP(hipStreamEndCapture(p->cap_stream, &g));
        hipGraphExec_t ge;
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) fail(CMCG_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        it = p->graphs.emplace(key, ge).first;
    }
    CMCG_HIP(hipGraphLaunch(it->second, st));
}

// One LTS period (forward with or without source and filter, or the adjoint).
// A forward period is replayed from a captured graph when use_graph (one
// host call for its thousands of launches; as fast as the eager launches on
// the GPU).  The adjoint period always runs eager: replaying its graph was
// measured 19% slower than launching it (216 against 182 ms per period on a
// 55200-tet P2 FP64 mesh, 4 substeps).
static void run_lts_period(cmcg_problem* p, const StepCfg& c, int direction, bool src, bool filt, bool use_graph,
                           hipStream_t st) {
    if (!use_graph || direction < 0) {
        lts_period(p, c, direction, src, filt, st);
        return;
    }
    const int variant = get_stage_variant(p->sp->q, p->sp->precision);
    const int64_t key = ((int64_t)c.M << 24) | ((int64_t)c.lts << 16) | ((int64_t)(variant + 1) << 8) |
                        (direction < 0 ? 0x80 : 0) | (c.scheme << 4) | (src ? 2 : 0) | (filt ? 1 : 0);
    auto it = p->lts_graphs.find(key);
    if (it == p->lts_graphs.end()) {
        if (!p->cap_stream) CMCG_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        CMCG_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        try {
            lts_period(p, c, direction, src, filt, p->cap_stream);
        } catch (...) {
            hipGraph_t g;
            (void)hipStreamEndCapture(p->cap_stream, &g);
            throw;
        }
        hipGraph_t g;
        CMCG_HIP(hipStreamEndCapture(p->cap_stream, &g));
        hipGraphExec_t ge;
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) fail(CMCG_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        it = p->lts_graphs.emplace(key, ge).first;
    }
    CMCG_HIP(hipGraphLaunch(it->second, st));
}

// X (FP64 dof vector) -> propagate one period -> Y = S^d P S^d X - sub
void apply_period(cmcg_problem* p, const StepCfg& c, const cmcg_options* o, const double* X, double* Yo,
                         const double* sub, int direction, bool src, bool filt, hipStream_t st) {
    const SpaceData& s = *p->sp;
    const int flip = direction < 0 ? 1 : 0;
    if (c.lts > 1) {
        // local time stepping: plain field-precision state (no FP32 low part)
        ensure_lts(p, c);
        if (X)
            to_field_dim(s, X, p->U.p, nullptr, s.ndof, flip, st);
        else
            launch_zero(p->U.p, p->U.bytes, st);
        run_lts_period(p, c, direction, src && direction > 0, filt, o->use_graph != 0, st);
        if (Yo) from_field_dim(s, p->U.p, nullptr, Yo, sub, s.ndof, flip, st);
        return;
    }
    if (X) {
        to_field_dim(s, X, p->U.p, p->Ulo.p, s.ndof, flip, st);
    } else {
        launch_zero(p->U.p, p->U.bytes, st);
        if (p->Ulo.p) launch_zero(p->Ulo.p, p->Ulo.bytes, st);
    }
    run_period(p, c, src && direction > 0, filt, o->use_graph != 0, st);
    if (Yo) from_field_dim(s, p->U.p, p->Ulo.p, Yo, sub, s.ndof, flip, st);
}

double dot(cmcg_problem* p, const double* U, const double* V, hipStream_t st) {
    dot_for(p, U, V, p->scal.as<double>(), st);
    CMCG_HIP(hipMemcpyAsync(p->pinned->p, p->scal.p, 8, hipMemcpyDeviceToHost, st));
    CMCG_HIP(hipStreamSynchronize(st));
    return p->pinned->p[0];
}

void prepare(cmcg_problem* p, const StepCfg& c) {
    if (current_device() != p->sp->device) fail(CMCG_ERR_STATE, "wrong current device");
    ensure_constants(p->sp->device, p->sp->q, p->sp->dim);
    if (p->geo_alpha != c.alpha) {
        build_geo(p, c.alpha);
        for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
        p->graphs.clear();
        for (auto& kv : p->lts_graphs) (void)hipGraphExecDestroy(kv.second);
        p->lts_graphs.clear();
    }
    ensure_work(p);
}

// Inner product (U, V)_{eps,mu} into pinned slot k, ordered on the stream
// (read after the stream has been synchronised).
static void dot_async(cmcg_problem* p, const double* U, const double* V, int k, hipStream_t st) {
    dot_for(p, U, V, p->scal.as<double>() + k, st);
    CMCG_HIP(hipMemcpyAsync(p->pinned->p + k, p->scal.as<double>() + k, 8, hipMemcpyDeviceToHost, st));
}

// ----------------------------------------------------------------- autotuner
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int64_t, int>, int> g_tuned;

bool variant_applies(int q, int precision, int v) {
    (void)precision;  // the matrix-core variants exist in both field precisions
    return v <= 1 || (v <= 5 && q >= 2) || (v >= 8 && q >= 2) || q == 3;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        CMCG_HIP(hipEventCreate(&a));
        CMCG_HIP(hipEventCreate(&b));
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};
}  // namespace

int time_stage_variants(int q, int precision, hipStream_t st, const std::function<void()>& run, int nlaunch,
                        double* us) {
    EventPair ev;
    const int old = get_stage_variant(q, precision);
    int best = old;
    double best_us = HUGE_VAL;
    try {
        for (int v = 0; v < kStageVariants; ++v) {
            us[v] = 0.0;
            if (!variant_applies(q, precision, v)) continue;
            set_stage_variant(q, precision, v);
            run();  // warm-up (first launches, caches)
            float tmin = HUGE_VALF;
            for (int rep = 0; rep < 2; ++rep) {
                CMCG_HIP(hipEventRecord(ev.a, st));
                run();
                CMCG_HIP(hipEventRecord(ev.b, st));
                CMCG_HIP(hipEventSynchronize(ev.b));
                float ms = 0.f;
                CMCG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                tmin = std::fmin(tmin, ms);
            }
            us[v] = 1e3 * tmin / nlaunch;
            if (us[v] < best_us) {
                best_us = us[v];
                best = v;
            }
        }
    } catch (...) {
        set_stage_variant(q, precision, old);
        throw;
    }
    set_stage_variant(q, precision, best);
    return best;
}

bool apply_tuned_variant(int device, int q, int precision, int64_t K, int members) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(device, q, precision, K, members));
    if (it == g_tuned.end()) return false;
    set_stage_variant(q, precision, it->second);
    return true;
}

void remember_tuned_variant(int device, int q, int precision, int64_t K, int members, int variant) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(device, q, precision, K, members)] = variant;
}

// Times the variants on up to 8 homogeneous steps of p's own mesh (its work
// buffers, zeroed first).
static int autotune_problem(cmcg_problem* p, const StepCfg& c, hipStream_t st, double* us) {
    const SpaceData& s = *p->sp;
    StepCfg ct = c;
    ct.M = std::min(c.M, 8);
    launch_zero(p->U.p, p->U.bytes, st);
    if (p->Ulo.p) launch_zero(p->Ulo.p, p->Ulo.bytes, st);
    const int nlaunch = ct.M * (c.scheme == 4 ? 4 : 2);
    const int v = time_stage_variants(s.q, s.precision, st, [&] { enqueue_period(p, ct, false, false, st); },
                                      nlaunch, us);
    remember_tuned_variant(s.device, s.q, s.precision, s.K, 1, v);
    return v;
}

static void maybe_autotune(cmcg_problem* p, const cmcg_options* o, const StepCfg& c, hipStream_t st) {
    if (!o->autotune) return;
    const SpaceData& s = *p->sp;
    if (s.dim == 2) return;  // one 2-D stage kernel
    if (apply_tuned_variant(s.device, s.q, s.precision, s.K, 1)) return;
    double us[kStageVariants];
    autotune_problem(p, c, st, us);
}

// --------------------------------------------------------- CMCG state machine
// Algorithm 3 as a sequence of asynchronous chunks: start() enqueues
// Algorithm 1 and the first inner products; every complete() (called once the
// stream has drained) consumes the scalars of the last chunk and enqueues the
// next one.  Chunks: [A] the two periods of (I-P*)(I-P) D and (D, A);
// [B] the U, R updates (+ residual refresh) and (R, R); [F] the filter period.
void CgRun::start(cmcg_problem* pr, const cmcg_options* opt, const double* u0_, hipStream_t s_) {
    p = pr;
    o = *opt;
    st = s_;
    u0 = u0_;
    if (o.runup < 0) fail(CMCG_ERR_ARG, "options: runup must be >= 0");
    c = step_config(p, &o);
    prepare(p, c);
    maybe_autotune(p, &o, c, st);
    const SpaceData& s = *p->sp;
    n = s.ndof;
    const size_t db = n * 8;
    p->v_u.alloc(db);
    p->v_r.alloc(db);
    p->v_d.alloc(db);
    p->v_a.alloc(db);
    p->v_w.alloc(db);
    p->v_gs.alloc(db);
    res.reset(new cmcg_result());
    res->sp = p->sp;
    res->nharm = p->nharm;
    res->Fre.alloc(db * p->nharm);
    res->Fim.alloc(db * p->nharm);
    res->U0.alloc(db);
    fixed = o.fixed_iters > 0;
    refresh = o.residual_refresh > 0 ? o.residual_refresh : 0;
    limit = fixed ? o.fixed_iters : o.max_iter;
    CMCG_HIP(hipStreamSynchronize(st));
    t0 = std::chrono::steady_clock::now();
    double *U = p->v_u.as<double>(), *R = p->v_r.as<double>(), *D = p->v_d.as<double>(), *W = p->v_w.as<double>(),
           *Gs = p->v_gs.as<double>();
    // Algorithm 1: G = P_psi 0 (into W), G_T = P* G, G* = G - G_T
    apply_period(p, c, &o, nullptr, W, nullptr, +1, true, false, st);
    apply_period(p, c, &o, W, Gs, W, -1, false, false, st);  // Gs = P* G - G = -G*
    launch_axpby(-1.0, Gs, 0.0, Gs, Gs, n, st);              // G* = G - P* G
    periods += 2;
    dot_async(p, W, W, 0, st);
    if (u0)
        CMCG_HIP(hipMemcpyAsync(U, u0, db, hipMemcpyDeviceToDevice, st));
    else
        launch_zero(U, db, st);
    // run-up: limiting-amplitude periods U <- P_psi U from the initial guess
    for (int l = 0; l < o.runup; ++l) apply_period(p, c, &o, U, U, nullptr, +1, true, false, st);
    periods += o.runup;
    if (u0 || o.runup > 0) {
        gradient(R);
    } else {
        launch_axpby(-1.0, Gs, 0.0, Gs, R, n, st);  // R0 = -G*
    }
    CMCG_HIP(hipMemcpyAsync(D, R, db, hipMemcpyDeviceToDevice, st));
    if (!fixed) {
        p->v_best.alloc(db);
        CMCG_HIP(hipMemcpyAsync(p->v_best.p, U, db, hipMemcpyDeviceToDevice, st));
    }
    dot_async(p, R, R, 1, st);
    phase = kStart;
}

double CgRun::secs() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void CgRun::gradient(double* out) {
    // Algorithm 2: W_T = P U - U, W_0 = P* W_T, J' = W_0 - W_T - G*
    double *U = p->v_u.as<double>(), *W = p->v_w.as<double>(), *Gs = p->v_gs.as<double>();
    apply_period(p, c, &o, U, W, U, +1, false, false, st);
    apply_period(p, c, &o, W, out, W, -1, false, false, st);
    launch_axpby(1.0, out, -1.0, Gs, out, n, st);
    periods += 2;
}

// convergence test, then the next chunk: [A] or [F]
void CgRun::decide() {
    rel = rr0 > 0 ? std::sqrt(rr / rr0) : 0.0;
    if (t6 < 0 && rel <= 1e-6) t6 = secs();
    const bool conv = !fixed && rel <= o.tol;
    if (conv || rr0 == 0.0 || it >= limit || stopped || diverged) {
        // final period with source and filter
        double* U = p->v_u.as<double>();
        if (diverged) {
            CMCG_HIP(hipMemcpyAsync(U, p->v_best.p, n * 8, hipMemcpyDeviceToDevice, st));
            rel = best;
        }
        apply_period(p, c, &o, U, nullptr, nullptr, +1, true, true, st);
        periods += 1;
        const size_t db = n * 8;
        CMCG_HIP(hipMemcpyAsync(res->Fre.p, p->Fre.p, db * p->nharm, hipMemcpyDeviceToDevice, st));
        CMCG_HIP(hipMemcpyAsync(res->Fim.p, p->Fim.p, db * p->nharm, hipMemcpyDeviceToDevice, st));
        CMCG_HIP(hipMemcpyAsync(res->U0.p, U, db, hipMemcpyDeviceToDevice, st));
        phase = kFinal;
        return;
    }
    // A = (I - P*)(I - P) D = W_0 - W_T
    double *D = p->v_d.as<double>(), *W = p->v_w.as<double>(), *A = p->v_a.as<double>();
    apply_period(p, c, &o, D, W, D, +1, false, false, st);
    apply_period(p, c, &o, W, A, W, -1, false, false, st);
    periods += 2;
    dot_async(p, D, A, 2, st);
    phase = kAwaitDA;
}

void CgRun::complete() {
    const double* pin = p->pinned->p;
    double *U = p->v_u.as<double>(), *R = p->v_r.as<double>(), *D = p->v_d.as<double>(), *A = p->v_a.as<double>();
    switch (phase) {
        case kStart:
            J0 = 0.5 * pin[0];
            if (!std::isfinite(J0)) fail(CMCG_ERR_UNSTABLE, "solve: non-finite field after the first period");
            rr = rr0 = pin[1];
            if (!std::isfinite(rr)) fail(CMCG_ERR_UNSTABLE, "solve: non-finite initial residual");
            res->history.push_back(1.0);
            if (rr0 == 0.0) rel = 0.0;
            best = rel;
            decide();
            break;
        case kAwaitDA: {
            const double dA = pin[2];
            if (!std::isfinite(dA)) fail(CMCG_ERR_UNSTABLE, "solve: non-finite values (time step too large?)");
            if (!(dA > 0)) fail(CMCG_ERR_BREAKDOWN, "solve: CG breakdown, (D, A) <= 0");
            const double alpha = rr / dA;
            launch_axpby(-alpha, D, 1.0, U, U, n, st);
            launch_axpby(-alpha, A, 1.0, R, R, n, st);
            ++it;
            if (refresh > 0 && it % refresh == 0) gradient(R);
            dot_async(p, R, R, 3, st);
            phase = kAwaitRR;
            break;
        }
        case kAwaitRR: {
            const double rn = pin[3];
            if (!std::isfinite(rn)) fail(CMCG_ERR_UNSTABLE, "solve: non-finite residual");
            const double beta = rn / rr;
            launch_axpby(1.0, R, beta, D, D, n, st);
            rr = rn;
            rel = rr0 > 0 ? std::sqrt(rr / rr0) : 0.0;
            res->history.push_back(rel);
            if (!fixed) {
                if (rel < best) {
                    best = rel;
                    CMCG_HIP(hipMemcpyAsync(p->v_best.p, U, n * 8, hipMemcpyDeviceToDevice, st));
                } else if (rel > kDivergence * best) {
                    diverged = true;
                }
            }
            if (o.progress && o.progress(o.progress_ctx, it, rel) != 0) stopped = true;
            decide();
            break;
        }
        case kFinal: {
            if (t6 < 0 && rel <= 1e-6) t6 = secs();
            cmcg_stats& S = res->st;
            S.iters = it;
            S.periods = periods;
            S.steps = c.M;
            S.dt = c.dt;
            S.rel_res = rel;
            S.J0 = J0;
            S.res0 = std::sqrt(rr0);
            S.seconds = secs();
            S.seconds_to_1e6 = t6;
            S.dof_updates = (double)n * c.M * periods;
            S.status = (stopped || diverged || (!fixed && rel > o.tol)) ? CMCG_NOT_CONVERGED : CMCG_OK;
            phase = kDone;
            break;
        }
        default:
            fail(CMCG_ERR_STATE, "solve: no work pending");
    }
}

// Limiting-amplitude ("full wave") iteration of Section 6: plain periods with
// the source from u0 (or zero), stopping on the relative change of the state
// at the period starts; the approximation F_psi U_0^(l) comes from one final
// period with the filter, so the filter's FP64 accumulation is paid once.
cmcg_result* fw_solve(cmcg_problem* p, const cmcg_options* o, const double* u0, hipStream_t st) {
    const StepCfg c = step_config(p, o);
    prepare(p, c);
    maybe_autotune(p, o, c, st);
    const SpaceData& s = *p->sp;
    const int64_t n = s.ndof;
    const size_t db = n * 8;
    p->v_u.alloc(db);
    p->v_w.alloc(db);
    p->v_r.alloc(db);
    std::unique_ptr<cmcg_result> res(new cmcg_result());
    res->sp = p->sp;
    res->nharm = p->nharm;
    res->Fre.alloc(db * p->nharm);
    res->Fim.alloc(db * p->nharm);
    res->U0.alloc(db);
    double *U = p->v_u.as<double>(), *W = p->v_w.as<double>(), *D = p->v_r.as<double>();
    CMCG_HIP(hipStreamSynchronize(st));
    const auto t0 = std::chrono::steady_clock::now();
    if (u0)
        CMCG_HIP(hipMemcpyAsync(U, u0, db, hipMemcpyDeviceToDevice, st));
    else
        launch_zero(U, db, st);
    const bool fixed = o->fixed_iters > 0;
    const int limit = fixed ? o->fixed_iters : o->max_iter;
    double rel = 1.0;
    int plain = 0;
    bool stopped = false, converged = false;
    while (plain < limit - 1) {
        apply_period(p, c, o, U, W, nullptr, +1, true, false, st);
        launch_axpby(1.0, W, -1.0, U, D, n, st);
        const double dd = dot(p, D, D, st), ww = dot(p, W, W, st);
        if (!std::isfinite(dd) || !std::isfinite(ww)) fail(CMCG_ERR_UNSTABLE, "fw_solve: non-finite field");
        rel = ww > 0 ? std::sqrt(dd / ww) : 0.0;
        res->history.push_back(rel);
        std::swap(U, W);
        ++plain;
        if (o->progress && o->progress(o->progress_ctx, plain, rel) != 0) {
            stopped = true;
            break;
        }
        if (!fixed && rel <= o->tol) {
            converged = true;
            break;
        }
    }
    // the iterate U_0^(plain) and its filtered field
    CMCG_HIP(hipMemcpyAsync(res->U0.p, U, db, hipMemcpyDeviceToDevice, st));
    apply_period(p, c, o, U, nullptr, nullptr, +1, true, true, st);
    CMCG_HIP(hipMemcpyAsync(res->Fre.p, p->Fre.p, db * p->nharm, hipMemcpyDeviceToDevice, st));
    CMCG_HIP(hipMemcpyAsync(res->Fim.p, p->Fim.p, db * p->nharm, hipMemcpyDeviceToDevice, st));
    CMCG_HIP(hipStreamSynchronize(st));
    cmcg_stats& S = res->st;
    S.iters = plain;
    S.periods = plain + 1;
    S.steps = c.M;
    S.dt = c.dt;
    S.rel_res = rel;
    S.J0 = 0.0;
    S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    S.seconds_to_1e6 = -1.0;
    S.dof_updates = (double)n * c.M * (plain + 1);
    S.status = (stopped || (!fixed && !converged)) ? CMCG_NOT_CONVERGED : CMCG_OK;
    return res.release();
}

cmcg_result* solve(cmcg_problem* p, const cmcg_options* o, const double* u0, hipStream_t st) {
    CgRun run;
    run.start(p, o, u0, st);
    while (!run.done()) {
        CMCG_HIP(hipStreamSynchronize(st));
        run.complete();
    }
    return run.res.release();
}

}  // namespace cmcg

// ======================================================================= ABI
using namespace cmcg;

#define CMCG_GUARD_BEGIN try {
#define CMCG_GUARD_END                          \
    }                                           \
    catch (const Error& e) {                    \
        set_last_error(e.msg);                  \
        return e.code;                          \
    }                                           \
    catch (const std::bad_alloc&) {             \
        set_last_error("host allocation failed"); \
        return CMCG_ERR_NOMEM;                  \
    }                                           \
    catch (const std::exception& e) {           \
        set_last_error(e.what());               \
        return CMCG_ERR_ARG;                    \
    }

extern "C" {

const char* cmcg_last_error(void) { return g_last_error.c_str(); }
const char* cmcg_version(void) { return "cmcg-mi355x 0.1"; }

void cmcg_options_default(cmcg_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->max_iter = 1000;
    o->scheme = CMCG_SCHEME_AUTO;
    o->flux = CMCG_FLUX_UPWIND;
    o->use_graph = 1;
}

int cmcg_mesh_create(int64_t nv, const double* xyz, int64_t K, const int64_t* tet, const int8_t* face_tag,
                     cmcg_mesh** out) {
    CMCG_GUARD_BEGIN
    if (!out) fail(CMCG_ERR_ARG, "mesh: NULL output");
    *out = nullptr;
    auto d = build_mesh(nv, xyz, K, tet, face_tag);
    *out = new cmcg_mesh{d};
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_mesh2d_create(int64_t nv, const double* xy, int64_t K, const int64_t* tri, const int8_t* edge_tag,
                       cmcg_mesh** out) {
    CMCG_GUARD_BEGIN
    if (!out) fail(CMCG_ERR_ARG, "mesh2d: NULL output");
    *out = nullptr;
    auto d = build_mesh2d(nv, xy, K, tri, edge_tag);
    *out = new cmcg_mesh{d};
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_mesh_dim(const cmcg_mesh* m, int* dim) {
    CMCG_GUARD_BEGIN
    if (!m || !m->d || !dim) fail(CMCG_ERR_ARG, "mesh_dim: NULL argument");
    *dim = m->d->dim;
    return CMCG_OK;
    CMCG_GUARD_END
}

void cmcg_mesh_destroy(cmcg_mesh* m) { delete m; }

int cmcg_mesh_locality_order(int64_t nv, const double* xyz, int64_t K, const int64_t* tet, int64_t* order) {
    CMCG_GUARD_BEGIN
    locality_order(nv, xyz, K, tet, order);
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_mesh_info(const cmcg_mesh* m, int64_t* K, int64_t* nb, double* min_rho) {
    CMCG_GUARD_BEGIN
    if (!m || !m->d) fail(CMCG_ERR_ARG, "mesh_info: NULL mesh");
    if (K) *K = m->d->K;
    if (nb) *nb = m->d->n_boundary;
    if (min_rho) {
        double r = HUGE_VAL;
        for (double x : m->d->rho) r = std::fmin(r, x);
        *min_rho = r;
    }
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_space_create(const cmcg_mesh* m, int q, int precision, cmcg_space** out) {
    CMCG_GUARD_BEGIN
    if (!out) fail(CMCG_ERR_ARG, "space: NULL output");
    *out = nullptr;
    if (!m || !m->d) fail(CMCG_ERR_ARG, "space: NULL mesh");
    if (q < 1 || q > kMaxQ) fail(CMCG_ERR_ARG, "space: q must be 1, 2 or 3");
    if (precision != CMCG_FP64 && precision != CMCG_FP32) fail(CMCG_ERR_ARG, "space: bad precision");
    auto s = std::make_shared<SpaceData>();
    s->mesh = m->d;
    s->dim = m->d->dim;
    const int nf = s->dim == 2 ? 3 : 4;
    s->q = q;
    s->Np = s->dim == 2 ? np2_of(q) : np_of(q);
    s->Nfp = s->dim == 2 ? nfp2_of(q) : nfp_of(q);
    s->precision = precision;
    s->device = current_device();
    s->K = m->d->K;
    s->ndof = s->K * (s->dim == 2 ? 3 : 6) * s->Np;
    const MeshData& md = *m->d;
    s->conn_h.resize(nf * s->K);
    for (int64_t i = 0; i < nf * s->K; ++i) {
        if (md.nbr[i] >= 0)
            s->conn_h[i] = (int32_t)((md.nbr[i] << 5) | (md.nbr_face[i] << 3) | md.perm[i]);
        else
            s->conn_h[i] = md.tag[i] == CMCG_TAG_PEC ? -1 : -2;
    }
    ensure_constants(s->device, q, s->dim);
    s->conn.alloc(nf * s->K * sizeof(int32_t));
    CMCG_HIP(hipMemcpy(s->conn.p, s->conn_h.data(), nf * s->K * sizeof(int32_t), hipMemcpyHostToDevice));
    *out = new cmcg_space{s};
    return CMCG_OK;
    CMCG_GUARD_END
}

void cmcg_space_destroy(cmcg_space* s) { delete s; }

int cmcg_space_info(const cmcg_space* s, int* q, int* Np, int* Nfp, int64_t* K, int64_t* ndof) {
    CMCG_GUARD_BEGIN
    if (!s || !s->d) fail(CMCG_ERR_ARG, "space_info: NULL space");
    if (q) *q = s->d->q;
    if (Np) *Np = s->d->Np;
    if (Nfp) *Nfp = s->d->Nfp;
    if (K) *K = s->d->K;
    if (ndof) *ndof = s->d->ndof;
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_space_nodes(const cmcg_space* s, double* xyz) {
    CMCG_GUARD_BEGIN
    if (!s || !s->d || !xyz) fail(CMCG_ERR_ARG, "space_nodes: NULL argument");
    const SpaceData& sp = *s->d;
    const MeshData& m = *sp.mesh;
    if (sp.dim == 2) {
        const RefElem2D& r2 = ref_elem2d(sp.q);
        for (int64_t e = 0; e < sp.K; ++e) {
            const double* v0 = &m.xyz[2 * m.tet[3 * e]];
            for (int i = 0; i < sp.Np; ++i)
                for (int d = 0; d < 2; ++d) {
                    double x = v0[d];
                    for (int a = 0; a < 2; ++a)
                        x += r2.xi[2 * i + a] * (m.xyz[2 * m.tet[3 * e + a + 1] + d] - v0[d]);
                    xyz[(e * sp.Np + i) * 2 + d] = x;
                }
        }
        return CMCG_OK;
    }
    const RefElem& r = ref_elem(sp.q);
    for (int64_t e = 0; e < sp.K; ++e) {
        const double* v0 = &m.xyz[3 * m.tet[4 * e]];
        for (int i = 0; i < sp.Np; ++i)
            for (int d = 0; d < 3; ++d) {
                double x = v0[d];
                for (int a = 0; a < 3; ++a) x += r.xi[3 * i + a] * (m.xyz[3 * m.tet[4 * e + a + 1] + d] - v0[d]);
                xyz[(e * sp.Np + i) * 3 + d] = x;
            }
    }
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_problem_create(const cmcg_space* s, const double* eps, const double* mu, const double* sigma,
                        double omega, const double* j_re, const double* j_im, const double* g_re,
                        const double* g_im, cmcg_problem** out) {
    CMCG_GUARD_BEGIN
    if (!out) fail(CMCG_ERR_ARG, "problem: NULL output");
    *out = nullptr;
    *out = make_problem(s, eps, mu, sigma, omega, j_re, j_im, g_re, g_im);
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_problem_create_harmonics(const cmcg_space* s, const double* eps, const double* mu, const double* sigma,
                                  double omega0, int nh, const int* k, const double* j_re, const double* j_im,
                                  cmcg_problem** out) {
    CMCG_GUARD_BEGIN
    if (!out) fail(CMCG_ERR_ARG, "problem_harmonics: NULL output");
    *out = nullptr;
    if (!k) fail(CMCG_ERR_ARG, "problem_harmonics: NULL harmonic numbers");
    *out = make_problem(s, eps, mu, sigma, omega0, j_re, j_im, nullptr, nullptr, nh, k);
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_problem_create_device(const cmcg_space* s, const double* eps, const double* mu, const double* sigma,
                               double omega, const double* j_re_dev, const double* j_im_dev, const double* g_re_dev,
                               const double* g_im_dev, hipStream_t stream, cmcg_problem** out) {
    CMCG_GUARD_BEGIN
    if (!out) fail(CMCG_ERR_ARG, "problem: NULL output");
    *out = nullptr;
    if (!s || !s->d) fail(CMCG_ERR_ARG, "problem: NULL space");
    const SpaceData& sd = *s->d;
    const int comps = sd.dim == 2 ? 1 : 3;
    const size_t nj = (size_t)sd.K * sd.Np * comps, ng = (size_t)sd.K * (sd.dim + 1) * sd.Nfp * comps;
    // the device arrays are staged through host memory: the source and the
    // lifted boundary data are assembled on the host as for host inputs
    std::vector<double> bufs[4];
    const double* dev[4] = {j_re_dev, j_im_dev, g_re_dev, g_im_dev};
    const size_t len[4] = {nj, nj, ng, ng};
    for (int i = 0; i < 4; ++i)
        if (dev[i]) {
            bufs[i].resize(len[i]);
            CMCG_HIP(hipMemcpyAsync(bufs[i].data(), dev[i], len[i] * 8, hipMemcpyDeviceToHost, stream));
        }
    CMCG_HIP(hipStreamSynchronize(stream));
    auto host = [&](int i) { return dev[i] ? (const double*)bufs[i].data() : nullptr; };
    *out = make_problem(s, eps, mu, sigma, omega, host(0), host(1), host(2), host(3));
    return CMCG_OK;
    CMCG_GUARD_END
}

void cmcg_problem_destroy(cmcg_problem* p) { delete p; }

int cmcg_problem_steps(const cmcg_problem* p, const cmcg_options* o, int* M, double* dt) {
    CMCG_GUARD_BEGIN
    if (!p || !o) fail(CMCG_ERR_ARG, "problem_steps: NULL argument");
    StepCfg c = step_config(p, o);
    if (M) *M = c.M;
    if (dt) *dt = c.dt;
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_problem_lts_fine(const cmcg_problem* p, const cmcg_options* o, int8_t* fine, int64_t* n_fine) {
    CMCG_GUARD_BEGIN
    if (!p || !o) fail(CMCG_ERR_ARG, "problem_lts_fine: NULL argument");
    StepCfg c = step_config(p, o);
    if (c.lts <= 1) fail(CMCG_ERR_ARG, "problem_lts_fine: the options ask for no local time stepping");
    const SpaceData& s = *p->sp;
    const MeshData& m = *s.mesh;
    int64_t cnt = 0;
    for (int64_t e = 0; e < s.K; ++e) {
        const bool f = c.cq * std::sqrt(p->mu[e] * p->eps[e]) * m.rho[e] < c.dt;
        if (fine) fine[e] = f ? 1 : 0;
        cnt += f;
    }
    if (n_fine) *n_fine = cnt;
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_solve(cmcg_problem* p, const cmcg_options* o, const double* u0_dev, hipStream_t stream,
               cmcg_result** out) {
    CMCG_GUARD_BEGIN
    if (!out) fail(CMCG_ERR_ARG, "solve: NULL output");
    *out = nullptr;
    if (!p) fail(CMCG_ERR_ARG, "solve: NULL problem");
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    if (o->max_iter < 0 || o->fixed_iters < 0) fail(CMCG_ERR_ARG, "solve: negative iteration count");
    cmcg_result* r = solve(p, o, u0_dev, stream);
    *out = r;
    return r->st.status;
    CMCG_GUARD_END
}

int cmcg_fw_solve(cmcg_problem* p, const cmcg_options* o, const double* u0_dev, hipStream_t stream,
                  cmcg_result** out) {
    CMCG_GUARD_BEGIN
    if (!out) fail(CMCG_ERR_ARG, "fw_solve: NULL output");
    *out = nullptr;
    if (!p) fail(CMCG_ERR_ARG, "fw_solve: NULL problem");
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    if (o->max_iter < 0 || o->fixed_iters < 0) fail(CMCG_ERR_ARG, "fw_solve: negative period count");
    cmcg_result* r = fw_solve(p, o, u0_dev, stream);
    *out = r;
    return r->st.status;
    CMCG_GUARD_END
}

int cmcg_solve_batch(cmcg_problem* const* problems, int n, const cmcg_options* o, hipStream_t stream,
                     cmcg_result** results) {
    CMCG_GUARD_BEGIN
    if (!results || !problems || n < 1) fail(CMCG_ERR_ARG, "solve_batch: NULL argument or empty batch");
    if (n > 65535) fail(CMCG_ERR_ARG, "solve_batch: at most 65535 problems per batch");
    for (int b = 0; b < n; ++b) results[b] = nullptr;
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    if (o->max_iter < 0 || o->fixed_iters < 0) fail(CMCG_ERR_ARG, "solve_batch: negative iteration count");
    try {
        solve_batch(problems, n, o, stream, results);
    } catch (...) {
        for (int b = 0; b < n; ++b) {
            delete results[b];
            results[b] = nullptr;
        }
        throw;
    }
    int status = CMCG_OK;
    for (int b = 0; b < n; ++b)
        if (results[b]->st.status != CMCG_OK) status = CMCG_NOT_CONVERGED;
    return status;
    CMCG_GUARD_END
}

int cmcg_result_fields(const cmcg_result* r, double* e_re, double* e_im, double* h_re, double* h_im) {
    CMCG_GUARD_BEGIN
    if (!r || !r->sp) fail(CMCG_ERR_ARG, "result_fields: NULL result");
    const SpaceData& s = *r->sp;
    std::vector<double> fr(s.ndof), fi(s.ndof);
    CMCG_HIP(hipMemcpy(fr.data(), r->Fre.p, s.ndof * 8, hipMemcpyDeviceToHost));
    CMCG_HIP(hipMemcpy(fi.data(), r->Fim.p, s.ndof * 8, hipMemcpyDeviceToHost));
    const int Np = s.Np;
    if (s.dim == 2) {  // e [K][Np], h [K][Np][2]
        for (int64_t e = 0; e < s.K; ++e)
            for (int i = 0; i < Np; ++i) {
                if (e_re) e_re[e * Np + i] = fr[(e * 3) * Np + i];
                if (e_im) e_im[e * Np + i] = fi[(e * 3) * Np + i];
                for (int c = 0; c < 2; ++c) {
                    if (h_re) h_re[(e * Np + i) * 2 + c] = fr[(e * 3 + 1 + c) * Np + i];
                    if (h_im) h_im[(e * Np + i) * 2 + c] = fi[(e * 3 + 1 + c) * Np + i];
                }
            }
        return CMCG_OK;
    }
    for (int64_t e = 0; e < s.K; ++e)
        for (int i = 0; i < Np; ++i)
            for (int c = 0; c < 3; ++c) {
                const int64_t o = (e * Np + i) * 3 + c;
                if (e_re) e_re[o] = fr[(e * 6 + c) * Np + i];
                if (e_im) e_im[o] = fi[(e * 6 + c) * Np + i];
                if (h_re) h_re[o] = fr[(e * 6 + 3 + c) * Np + i];
                if (h_im) h_im[o] = fi[(e * 6 + 3 + c) * Np + i];
            }
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_result_filtered_device(const cmcg_result* r, double* f_re, double* f_im, hipStream_t stream) {
    CMCG_GUARD_BEGIN
    if (!r || !r->sp) fail(CMCG_ERR_ARG, "result: NULL result");
    const size_t b = r->sp->ndof * 8;
    if (f_re) CMCG_HIP(hipMemcpyAsync(f_re, r->Fre.p, b, hipMemcpyDeviceToDevice, stream));
    if (f_im) CMCG_HIP(hipMemcpyAsync(f_im, r->Fim.p, b, hipMemcpyDeviceToDevice, stream));
    CMCG_HIP(hipStreamSynchronize(stream));
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_result_harmonics(const cmcg_result* r, int* nh) {
    CMCG_GUARD_BEGIN
    if (!r || !nh) fail(CMCG_ERR_ARG, "result_harmonics: NULL argument");
    *nh = r->nharm;
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_result_filtered_harmonic_device(const cmcg_result* r, int h, double* f_re, double* f_im,
                                         hipStream_t stream) {
    CMCG_GUARD_BEGIN
    if (!r || !r->sp) fail(CMCG_ERR_ARG, "result: NULL result");
    if (h < 0 || h >= r->nharm) fail(CMCG_ERR_ARG, "result: harmonic index out of range");
    const size_t n = r->sp->ndof, b = n * 8;
    if (f_re) CMCG_HIP(hipMemcpyAsync(f_re, r->Fre.as<double>() + h * n, b, hipMemcpyDeviceToDevice, stream));
    if (f_im) CMCG_HIP(hipMemcpyAsync(f_im, r->Fim.as<double>() + h * n, b, hipMemcpyDeviceToDevice, stream));
    CMCG_HIP(hipStreamSynchronize(stream));
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_result_initial_device(const cmcg_result* r, double* u0, hipStream_t stream) {
    CMCG_GUARD_BEGIN
    if (!r || !r->sp || !u0) fail(CMCG_ERR_ARG, "result: NULL argument");
    CMCG_HIP(hipMemcpyAsync(u0, r->U0.p, r->sp->ndof * 8, hipMemcpyDeviceToDevice, stream));
    CMCG_HIP(hipStreamSynchronize(stream));
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_result_stats(const cmcg_result* r, cmcg_stats* st) {
    CMCG_GUARD_BEGIN
    if (!r || !st) fail(CMCG_ERR_ARG, "result_stats: NULL argument");
    *st = r->st;
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_result_history(const cmcg_result* r, double* rel, int cap, int* n) {
    CMCG_GUARD_BEGIN
    if (!r) fail(CMCG_ERR_ARG, "result_history: NULL result");
    const int m = (int)r->history.size();
    if (n) *n = m;
    if (rel)
        for (int i = 0; i < m && i < cap; ++i) rel[i] = r->history[i];
    return CMCG_OK;
    CMCG_GUARD_END
}

void cmcg_result_destroy(cmcg_result* r) { delete r; }

int cmcg_debug_rhs(cmcg_problem* p, const cmcg_options* o, double t, int with_source, const double* u,
                   double* out, hipStream_t stream) {
    CMCG_GUARD_BEGIN
    if (!p || !u || !out) fail(CMCG_ERR_ARG, "debug_rhs: NULL argument");
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    StepCfg c = step_config(p, o);
    prepare(p, c);
    const SpaceData& s = *p->sp;
    p->Kbuf.alloc(s.ndof * s.esize());
    to_field_dim(s, u, p->U.p, p->Ulo.p, s.ndof, 0, stream);
    StageArgs a = base_args(p);
    a.mode = RHS;
    a.Y = p->U.p;
    a.U = p->U.p;
    a.Kout = p->Kbuf.p;
    a.src_rows = (with_source && p->src_rows) ? p->src_rows : 0;
    a.scos = std::cos(p->omega * t);
    a.ssin = std::sin(p->omega * t);
    stage_dim(s, a, stream);
    from_field_dim(s, p->Kbuf.p, nullptr, out, nullptr, s.ndof, 0, stream);
    CMCG_HIP(hipStreamSynchronize(stream));
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_debug_period(cmcg_problem* p, const cmcg_options* o, int direction, int with_source, const double* u0,
                      double* ut, double* f_re, double* f_im, hipStream_t stream) {
    CMCG_GUARD_BEGIN
    if (!p || !u0 || !ut) fail(CMCG_ERR_ARG, "debug_period: NULL argument");
    if (direction != 1 && direction != -1) fail(CMCG_ERR_ARG, "debug_period: direction must be +1 or -1");
    if (direction < 0 && with_source) fail(CMCG_ERR_ARG, "debug_period: the adjoint period has no source");
    if (direction < 0 && (f_re || f_im)) fail(CMCG_ERR_ARG, "debug_period: filter only on forward periods");
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    StepCfg c = step_config(p, o);
    prepare(p, c);
    const bool filt = f_re || f_im;
    apply_period(p, c, o, u0, ut, nullptr, direction, with_source != 0, filt, stream);
    const size_t b = p->sp->ndof * 8;
    if (f_re) CMCG_HIP(hipMemcpyAsync(f_re, p->Fre.p, b, hipMemcpyDeviceToDevice, stream));
    if (f_im) CMCG_HIP(hipMemcpyAsync(f_im, p->Fim.p, b, hipMemcpyDeviceToDevice, stream));
    CMCG_HIP(hipStreamSynchronize(stream));
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_debug_step(cmcg_problem* p, const cmcg_options* o, int m, int direction, int with_source, const double* u,
                    double* out, hipStream_t stream) {
    CMCG_GUARD_BEGIN
    if (!p || !u || !out) fail(CMCG_ERR_ARG, "debug_step: NULL argument");
    if (direction != 1 && direction != -1) fail(CMCG_ERR_ARG, "debug_step: direction must be +1 or -1");
    if (direction < 0 && with_source) fail(CMCG_ERR_ARG, "debug_step: the adjoint step has no source");
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    StepCfg c = step_config(p, o);
    if (m < 0 || m >= c.M) fail(CMCG_ERR_ARG, "debug_step: step index outside 0 .. M-1");
    prepare(p, c);
    const SpaceData& s = *p->sp;
    const int flip = direction < 0 ? 1 : 0;
    to_field_dim(s, u, p->U.p, p->Ulo.p, s.ndof, flip, stream);
    enqueue_steps(p, c, with_source != 0 && direction > 0, false, m, m + 1, stream);
    from_field_dim(s, p->U.p, p->Ulo.p, out, nullptr, s.ndof, flip, stream);
    CMCG_HIP(hipStreamSynchronize(stream));
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_debug_dot(cmcg_problem* p, const double* u, const double* v, double* out, hipStream_t stream) {
    CMCG_GUARD_BEGIN
    if (!p || !u || !v || !out) fail(CMCG_ERR_ARG, "debug_dot: NULL argument");
    ensure_constants(p->sp->device, p->sp->q, p->sp->dim);
    ensure_work(p);
    *out = dot(p, u, v, stream);
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_debug_dot_noalloc(const cmcg_problem* p, const double* u, const double* v, double* out_dev,
                           hipStream_t stream) {
    CMCG_GUARD_BEGIN
    if (!p || !u || !v || !out_dev) fail(CMCG_ERR_ARG, "debug_dot_noalloc: NULL argument");
    const SpaceData& s = *p->sp;
    if (current_device() != s.device) fail(CMCG_ERR_STATE, "debug_dot_noalloc: wrong current device");
    // the partials the reduction writes must fit the fixed scratch array
    const size_t need = s.dim == 2 ? (size_t)dot2d_partials() : (size_t)dot_blocks(s.K);
    if (need > noalloc_scratch_doubles())
        fail(CMCG_ERR_ARG, "debug_dot_noalloc: " + std::to_string(need) + " partial sums exceed the scratch array of " +
                               std::to_string(noalloc_scratch_doubles()));
    // constants and the scratch address were set up when the problem was created
    double* partial = noalloc_scratch(s.device);
    if (s.dim == 2)
        launch_dot2d(s.q, u, v, p->wE.as<double>(), p->wH.as<double>(), s.K, partial, out_dev, stream);
    else
        launch_dot(s.q, u, v, p->wE.as<double>(), p->wH.as<double>(), s.K, partial, out_dev, stream);
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_debug_mfma(int precision, const double* a, const double* b, double* d, hipStream_t stream) {
    CMCG_GUARD_BEGIN
    if (!a || !b || !d) fail(CMCG_ERR_ARG, "debug_mfma: NULL argument");
    if (precision != CMCG_FP64 && precision != CMCG_FP32) fail(CMCG_ERR_ARG, "debug_mfma: unknown precision");
    launch_mfma_probe(precision, a, b, d, stream);
    CMCG_HIP(hipStreamSynchronize(stream));
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_tune_stage(int q, int precision, int variant) {
    CMCG_GUARD_BEGIN
    if (q < 1 || q > kMaxQ || (precision != CMCG_FP64 && precision != CMCG_FP32) || variant < -1 ||
        variant >= kStageVariants)
        fail(CMCG_ERR_ARG, "tune_stage: bad q, precision or variant");
    set_stage_variant(q, precision, variant);
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_autotune_stage(cmcg_problem* p, const cmcg_options* o, hipStream_t stream, int* variant,
                        double* us_per_launch) {
    CMCG_GUARD_BEGIN
    if (!p || !variant) fail(CMCG_ERR_ARG, "autotune_stage: NULL argument");
    if (p->sp->dim == 2) fail(CMCG_ERR_ARG, "autotune_stage: 2-D spaces have one stage kernel");
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    const StepCfg c = step_config(p, o);
    prepare(p, c);
    double us[kStageVariants];
    *variant = autotune_problem(p, c, stream, us);
    if (us_per_launch)
        for (int v = 0; v < kStageVariants; ++v) us_per_launch[v] = us[v];
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_autotune_batch(cmcg_problem* const* problems, int n, const cmcg_options* o, hipStream_t stream,
                        int* variant, double* us_per_launch) {
    CMCG_GUARD_BEGIN
    if (!problems || n < 1 || !variant) fail(CMCG_ERR_ARG, "autotune_batch: NULL argument or empty batch");
    if (n > 65535) fail(CMCG_ERR_ARG, "autotune_batch: at most 65535 problems per batch");
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    double us[kStageVariants] = {};
    *variant = autotune_batch(problems, n, o, stream, us);
    if (us_per_launch)
        for (int v = 0; v < kStageVariants; ++v) us_per_launch[v] = us[v];
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_tune_get_stage(int q, int precision, int* variant) {
    CMCG_GUARD_BEGIN
    if (q < 1 || q > kMaxQ || (precision != CMCG_FP64 && precision != CMCG_FP32) || !variant)
        fail(CMCG_ERR_ARG, "tune_get_stage: bad argument");
    *variant = get_stage_variant(q, precision);
    return CMCG_OK;
    CMCG_GUARD_END
}

int cmcg_tune_resolve_stage(int q, int precision, int64_t K, int members, int* variant) {
    CMCG_GUARD_BEGIN
    if (q < 1 || q > kMaxQ || (precision != CMCG_FP64 && precision != CMCG_FP32) || K < 1 || members < 1 ||
        !variant)
        fail(CMCG_ERR_ARG, "tune_resolve_stage: bad argument");
    *variant = resolve_stage_variant(q, precision, K, members);
    return CMCG_OK;
    CMCG_GUARD_END
}

}  // extern "C"
