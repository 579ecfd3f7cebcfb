// Batched CMCG: many independent problems on one space (same mesh, order and
// field precision; each with its own omega, current density and materials)
// advanced together.  Every RK stage is one launch over all members (grid.y =
// member), so a period costs max_b M_b x stages launches whatever the batch
// size; members whose period is shorter, or whose CG has converged, idle.  The
// CG recurrences of Algorithm 3 run per member in FP64 on the host; the
// member-wise inner products and vector updates use the same per-member
// arithmetic and reduction order as the single-problem path, so a member's
// result does not depend on the batch it runs in.
#include <chrono>
#include <cmath>
#include <cstring>

#include "objects.h"

namespace cmcg {

namespace {

struct Batch {
    int B = 0;
    std::shared_ptr<SpaceData> sp;
    int scheme = 2, S = 2, Mmax = 0;
    std::vector<StepCfg> cfg;
    std::vector<cmcg_problem*> P;
    bool shared_geo = true;
    int src_rows = 0;
    // device
    DevBuf geo, wE, wH, Sre, Sim, smask;
    DevBuf U, Y1, Y2, Acc, Fre, Fim, Kbuf;
    DevBuf Ulo;  // FP32 fields: bfloat16 low parts of U
    DevBuf vu, vr, vd, va, vw, vgs, vbest;
    DevBuf partial, dots, coefA, coefC, active, msteps, mtab, fw_re, fw_im;
    std::unique_ptr<HostPinned> pin;
    hipStream_t cap = nullptr;
    std::map<int, hipGraphExec_t> graphs;
    bool no_capture = false;  // periods without a captured graph run eagerly
    ~Batch() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        if (cap) (void)hipStreamDestroy(cap);
    }
    int64_t n() const { return sp->ndof; }
    size_t fb() const { return (size_t)n() * B * sp->esize(); }
    size_t db() const { return (size_t)n() * B * 8; }
};

// Stage scalars of every member for every (step, stage), plus one row (step
// Mmax, stage 0) with the last filter level t = T_b of each member.
void build_table(Batch& bt, hipStream_t st) {
    const int B = bt.B, S = bt.S;
    std::vector<double> tab((size_t)(bt.Mmax + 1) * S * B * kMemberParams, 0.0);
    std::vector<double> fwr(B), fwi(B);
    const double two_pi = 2.0 * M_PI;
    for (int b = 0; b < B; ++b) {
        const StepCfg& c = bt.cfg[b];
        const int M = c.M;
        const double dt = c.dt;
        const double twoT = 2.0 / c.T;
        std::complex<double> xi[4];
        if (bt.scheme == 4) hermite_weights(bt.P[b]->omega, dt, xi);
        auto ph = [&](double m) { return std::complex<double>(std::cos(two_pi * m / M), -std::sin(two_pi * m / M)); };
        for (int m = 0; m <= bt.Mmax; ++m) {
            for (int s = 0; s < S; ++s) {
                double* p = &tab[(((size_t)m * S + s) * B + b) * kMemberParams];
                double cs = 0;  // stage time offset in steps
                if (bt.scheme == 2) {
                    if (s == 0) {
                        p[0] = 0.5 * dt;
                    } else {
                        p[2] = dt;
                        cs = 0.5;
                    }
                } else {
                    if (s == 0) {
                        p[0] = 0.5 * dt;
                        p[1] = dt / 6.0;
                    } else if (s == 1) {
                        p[0] = 0.5 * dt;
                        p[1] = dt / 3.0;
                        cs = 0.5;
                    } else if (s == 2) {
                        p[0] = dt;
                        p[1] = dt / 3.0;
                        cs = 0.5;
                    } else {
                        p[2] = dt / 6.0;
                        cs = 1.0;
                    }
                }
                const int mm = m < M ? m : M;  // the extra row holds level M_b
                const double phase = two_pi * (mm + cs) / M;
                p[3] = std::cos(phase);
                p[4] = std::sin(phase);
                if (s == 0) {
                    std::complex<double> wa, wb;
                    if (m < M) {
                        if (bt.scheme == 2) {
                            wa = ph(m) * ((m == 0 ? 1.0 : 2.0) / M);
                        } else {
                            wa = twoT * ph(m) * xi[0];
                            wb = twoT * ph(m) * xi[2];
                            if (m >= 1) {
                                wa += twoT * ph(m - 1) * xi[1];
                                wb += twoT * ph(m - 1) * xi[3];
                            }
                        }
                    } else if (bt.scheme == 4) {  // level M_b: interval [t_{M-1}, t_M] only
                        wa = twoT * ph(M - 1) * xi[1];
                        wb = twoT * ph(M - 1) * xi[3];
                    }
                    p[5] = wa.real();
                    p[6] = wa.imag();
                    p[7] = wb.real();
                    p[8] = wb.imag();
                }
            }
        }
        fwr[b] = 1.0 / M;  // trapezoid weight of U_M (e^{-i w T} = 1)
        fwi[b] = 0.0;
    }
    bt.mtab.alloc(tab.size() * 8);
    bt.fw_re.alloc(B * 8);
    bt.fw_im.alloc(B * 8);
    // stream-ordered copies (no legacy-stream work: a batch may run on a
    // worker thread while another thread captures a graph)
    CMCG_HIP(hipMemcpyAsync(bt.mtab.p, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, st));
    CMCG_HIP(hipMemcpyAsync(bt.fw_re.p, fwr.data(), B * 8, hipMemcpyHostToDevice, st));
    CMCG_HIP(hipMemcpyAsync(bt.fw_im.p, fwi.data(), B * 8, hipMemcpyHostToDevice, st));
    CMCG_HIP(hipStreamSynchronize(st));
}

StageArgs batch_args(Batch& bt) {
    StageArgs a{};
    a.geo = bt.geo.p;
    a.conn = bt.sp->conn.as<int>();
    a.K = bt.sp->K;
    a.Sre = bt.Sre.p;
    a.Sim = bt.Sim.p;
    a.smask = bt.smask.as<uint32_t>();
    a.Fre = bt.Fre.as<double>();
    a.Fim = bt.Fim.as<double>();
    a.Ulo = bt.Ulo.p;
    a.nharm = 1;
    a.nmembers = bt.B;
    a.active = bt.active.as<int>();
    a.msteps = bt.msteps.as<int>();
    a.bstride = bt.n();
    a.gstride = bt.shared_geo ? 0 : (int64_t)geo_values(*bt.sp) * bt.sp->K;
    a.sstride = bt.n();
    return a;
}

void enqueue_batch_period(Batch& bt, bool src, bool filt, hipStream_t st) {
    const int prec = bt.sp->precision, S = bt.S, B = bt.B;
    StageArgs a = batch_args(bt);
    a.src_rows = src ? bt.src_rows : 0;
    if (filt) {
        launch_zero(bt.Fre.p, bt.Fre.bytes, st);
        launch_zero(bt.Fim.p, bt.Fim.bytes, st);
    }
    const double* tab = bt.mtab.as<double>();
    auto row = [&](int m, int s) { return tab + ((size_t)m * S + s) * B * kMemberParams; };
    for (int m = 0; m < bt.Mmax; ++m) {
        a.step = m;
        if (bt.scheme == 2) {
            a.mode = RK2_S1;
            a.Y = bt.U.p;
            a.U = bt.U.p;
            a.Ynext = bt.Y1.p;
            a.mtab = row(m, 0);
            a.filter = filt ? 1 : 0;
            stage_dim(*bt.sp, a, st);
            a.filter = 0;
            a.mode = RK2_S2;
            a.Y = bt.Y1.p;
            a.U = bt.U.p;
            a.Uout = bt.U.p;
            a.mtab = row(m, 1);
            stage_dim(*bt.sp, a, st);
        } else {
            a.mode = RK4_S1;
            a.Y = bt.U.p;
            a.U = bt.U.p;
            a.Ynext = bt.Y1.p;
            a.Acc = bt.Acc.p;
            a.mtab = row(m, 0);
            a.filter = filt ? 1 : 0;
            stage_dim(*bt.sp, a, st);
            a.filter = 0;
            a.mode = RK4_S2;
            a.Y = bt.Y1.p;
            a.Ynext = bt.Y2.p;
            a.mtab = row(m, 1);
            stage_dim(*bt.sp, a, st);
            a.mode = RK4_S3;
            a.Y = bt.Y2.p;
            a.Ynext = bt.Y1.p;
            a.mtab = row(m, 2);
            stage_dim(*bt.sp, a, st);
            a.mode = RK4_S4;
            a.Y = bt.Y1.p;
            a.Uout = bt.U.p;
            a.mtab = row(m, 3);
            stage_dim(*bt.sp, a, st);
        }
    }
    if (filt) {
        if (bt.scheme == 2) {
            launch_filter_add_batch(prec, bt.U.p, bt.fw_re.as<double>(), bt.fw_im.as<double>(), bt.Fre.as<double>(),
                                    bt.Fim.as<double>(), bt.n(), B, st);
        } else {
            a.mode = RHS;
            a.step = -1;
            a.Y = bt.U.p;
            a.U = bt.U.p;
            a.Kout = bt.Kbuf.p;
            a.mtab = row(bt.Mmax, 0);
            a.filter = 1;
            stage_dim(*bt.sp, a, st);
        }
    }
}

int batch_graph_key(const Batch& bt, bool src, bool filt) {
    // keyed by the stage variant as well: it is read when the launches are enqueued
    const int variant = bt.sp->dim == 3 ? get_stage_variant(bt.sp->q, bt.sp->precision) : 0;
    return (variant << 4) | (src ? 2 : 0) | (filt ? 1 : 0);
}

// the captured period for (src, filt), captured now if missing
hipGraphExec_t batch_graph(Batch& bt, bool src, bool filt) {
    const int key = batch_graph_key(bt, src, filt);
    auto it = bt.graphs.find(key);
    if (it == bt.graphs.end()) {
        if (!bt.cap) CMCG_HIP(hipStreamCreateWithFlags(&bt.cap, hipStreamNonBlocking));
        CMCG_HIP(hipStreamBeginCapture(bt.cap, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_batch_period(bt, src, filt, bt.cap);
        } catch (...) {
            hipGraph_t g;
            (void)hipStreamEndCapture(bt.cap, &g);
            throw;
        }
        hipGraph_t g;
        CMCG_HIP(hipStreamEndCapture(bt.cap, &g));
        hipGraphExec_t ge;
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) fail(CMCG_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        it = bt.graphs.emplace(key, ge).first;
    }
    return it->second;
}

void run_batch_period(Batch& bt, bool src, bool filt, bool use_graph, hipStream_t st) {
    if (!use_graph || (bt.no_capture && !bt.graphs.count(batch_graph_key(bt, src, filt)))) {
        enqueue_batch_period(bt, src, filt, st);
        return;
    }
    CMCG_HIP(hipGraphLaunch(batch_graph(bt, src, filt), st));
}

// Y_b = S^d P_b S^d X_b - sub_b for every member (X == nullptr: zero state)
void batch_apply(Batch& bt, const cmcg_options* o, const double* X, double* Yo, const double* sub, int direction,
                 bool src, bool filt, hipStream_t st) {
    const SpaceData& s = *bt.sp;
    const int flip = direction < 0 ? 1 : 0;
    const int64_t N = bt.n() * bt.B;
    if (X) {
        to_field_dim(s, X, bt.U.p, bt.Ulo.p, N, flip, st);
    } else {
        launch_zero(bt.U.p, bt.U.bytes, st);
        if (bt.Ulo.p) launch_zero(bt.Ulo.p, bt.Ulo.bytes, st);
    }
    run_batch_period(bt, src && direction > 0, filt, o->use_graph != 0, st);
    if (Yo) from_field_dim(s, bt.U.p, bt.Ulo.p, Yo, sub, N, flip, st);
}

void batch_dots(Batch& bt, const double* U, const double* V, std::vector<double>& out, hipStream_t st) {
    const SpaceData& s = *bt.sp;
    if (s.dim == 2)
        launch_dot_batch2d(s.q, U, V, bt.wE.as<double>(), bt.wH.as<double>(), bt.shared_geo ? 0 : s.K, s.K, bt.B,
                           bt.partial.as<double>(), bt.dots.as<double>(), st);
    else
        launch_dot_batch(s.q, U, V, bt.wE.as<double>(), bt.wH.as<double>(), bt.shared_geo ? 0 : s.K, s.K, bt.B,
                         bt.partial.as<double>(), bt.dots.as<double>(), st);
    CMCG_HIP(hipMemcpyAsync(bt.pin->p, bt.dots.p, bt.B * 8, hipMemcpyDeviceToHost, st));
    CMCG_HIP(hipStreamSynchronize(st));
    out.assign(bt.pin->p, bt.pin->p + bt.B);
}

void batch_axpby(Batch& bt, const std::vector<double>& a, const double* x, const std::vector<double>& c,
                 const double* y, double* z, hipStream_t st) {
    // coefficients staged through pinned memory (ordered on the stream)
    double* h = bt.pin->p + bt.B;  // second half of the staging area
    for (int b = 0; b < bt.B; ++b) {
        h[b] = a[b];
        h[bt.B + b] = c[b];
    }
    CMCG_HIP(hipMemcpyAsync(bt.coefA.p, h, bt.B * 8, hipMemcpyHostToDevice, st));
    CMCG_HIP(hipMemcpyAsync(bt.coefC.p, h + bt.B, bt.B * 8, hipMemcpyHostToDevice, st));
    launch_axpby_batch(bt.coefA.as<double>(), x, bt.coefC.as<double>(), y, z, bt.n(), bt.B, st);
    // the staging area is reused by the next call: wait for the copies
    CMCG_HIP(hipStreamSynchronize(st));
}

void set_active(Batch& bt, const std::vector<int>& act, hipStream_t st) {
    CMCG_HIP(hipMemcpyAsync(bt.active.p, act.data(), bt.B * sizeof(int), hipMemcpyHostToDevice, st));
    CMCG_HIP(hipStreamSynchronize(st));
}

// Validates the members and builds the batch's device state: shared or
// per-member geometry, sources, field / filter / CG vectors, the member
// scalar table and step counts; every member active.
void setup_batch(Batch& bt, cmcg_problem* const* probs, int B, const cmcg_options* o, hipStream_t st) {
    bt.B = B;
    bt.sp = probs[0] ? probs[0]->sp : nullptr;
    if (!bt.sp) fail(CMCG_ERR_ARG, "solve_batch: NULL problem");
    if (o->runup < 0) fail(CMCG_ERR_ARG, "options: runup must be >= 0");
    if (o->lts_ratio > 1) fail(CMCG_ERR_ARG, "solve_batch: local time stepping is for single solves");
    for (int b = 0; b < B; ++b) {
        if (!probs[b]) fail(CMCG_ERR_ARG, "solve_batch: NULL problem");
        if (probs[b]->sp != bt.sp) fail(CMCG_ERR_ARG, "solve_batch: all problems must share one space");
        if (probs[b]->nharm != 1) fail(CMCG_ERR_ARG, "solve_batch: several-frequency problems are solved singly");
        bt.P.push_back(probs[b]);
        bt.cfg.push_back(step_config(probs[b], o));
        if (bt.cfg[b].scheme != bt.cfg[0].scheme || bt.cfg[b].alpha != bt.cfg[0].alpha)
            fail(CMCG_ERR_ARG, "solve_batch: members must use one time scheme and flux");
        prepare(probs[b], bt.cfg[b]);
        bt.Mmax = std::max(bt.Mmax, bt.cfg[b].M);
        if (probs[b]->eps != probs[0]->eps || probs[b]->mu != probs[0]->mu || probs[b]->sigma != probs[0]->sigma)
            bt.shared_geo = false;
        bt.src_rows = std::max(bt.src_rows, probs[b]->src_rows);
    }
    bt.scheme = bt.cfg[0].scheme;
    bt.S = bt.scheme == 2 ? 2 : 4;
    const SpaceData& s = *bt.sp;
    const int64_t n = s.ndof, K = s.K;
    const size_t esz = s.esize();
    const int kG = geo_values(s);
    // shared or per-member geometry and mass weights
    if (bt.shared_geo) {
        bt.geo.alloc(kG * K * esz);
        bt.wE.alloc(K * 8);
        bt.wH.alloc(K * 8);
        CMCG_HIP(hipMemcpyAsync(bt.geo.p, probs[0]->geo.p, kG * K * esz, hipMemcpyDeviceToDevice, st));
        CMCG_HIP(hipMemcpyAsync(bt.wE.p, probs[0]->wE.p, K * 8, hipMemcpyDeviceToDevice, st));
        CMCG_HIP(hipMemcpyAsync(bt.wH.p, probs[0]->wH.p, K * 8, hipMemcpyDeviceToDevice, st));
    } else {
        bt.geo.alloc(kG * K * esz * B);
        bt.wE.alloc(K * 8 * B);
        bt.wH.alloc(K * 8 * B);
        for (int b = 0; b < B; ++b) {
            CMCG_HIP(hipMemcpyAsync((char*)bt.geo.p + b * kG * K * esz, probs[b]->geo.p, kG * K * esz,
                                    hipMemcpyDeviceToDevice, st));
            CMCG_HIP(hipMemcpyAsync(bt.wE.as<double>() + b * K, probs[b]->wE.p, K * 8, hipMemcpyDeviceToDevice, st));
            CMCG_HIP(hipMemcpyAsync(bt.wH.as<double>() + b * K, probs[b]->wH.p, K * 8, hipMemcpyDeviceToDevice, st));
        }
    }
    bt.U.alloc(bt.fb());
    bt.Y1.alloc(bt.fb());
    bt.Y2.alloc(bt.fb());
    bt.Acc.alloc(bt.fb());
    if (s.precision == CMCG_FP32) bt.Ulo.alloc((size_t)bt.n() * B * 2);
    bt.Kbuf.alloc(bt.fb());
    bt.Fre.alloc(bt.db());
    bt.Fim.alloc(bt.db());
    if (bt.src_rows) {
        bt.Sre.alloc(bt.fb());
        bt.Sim.alloc(bt.fb());
        launch_zero(bt.Sre.p, bt.Sre.bytes, st);
        launch_zero(bt.Sim.p, bt.Sim.bytes, st);
        const int64_t mw = s.dim == 2 ? 0 : source_mask_words(K);  // 2-D stages read every source row
        if (mw) {
            bt.smask.alloc((size_t)mw * 4 * B);
            launch_zero(bt.smask.p, bt.smask.bytes, st);
        }
        for (int b = 0; b < B; ++b) {
            if (!probs[b]->src_rows) continue;
            if (mw)
                CMCG_HIP(hipMemcpyAsync(bt.smask.as<uint32_t>() + b * mw, probs[b]->smask.p, mw * 4,
                                        hipMemcpyDeviceToDevice, st));
            CMCG_HIP(hipMemcpyAsync((char*)bt.Sre.p + b * n * esz, probs[b]->Sre.p, n * esz, hipMemcpyDeviceToDevice,
                                    st));
            CMCG_HIP(hipMemcpyAsync((char*)bt.Sim.p + b * n * esz, probs[b]->Sim.p, n * esz, hipMemcpyDeviceToDevice,
                                    st));
        }
    }
    bt.vu.alloc(bt.db());
    bt.vr.alloc(bt.db());
    bt.vd.alloc(bt.db());
    bt.va.alloc(bt.db());
    bt.vw.alloc(bt.db());
    bt.vgs.alloc(bt.db());
    if (o->fixed_iters <= 0) bt.vbest.alloc(bt.db());
    bt.partial.alloc((size_t)dot_partials() * B * 8);
    bt.dots.alloc(B * 8);
    bt.coefA.alloc(B * 8);
    bt.coefC.alloc(B * 8);
    bt.active.alloc(B * sizeof(int));
    bt.msteps.alloc(B * sizeof(int));
    bt.pin.reset(new HostPinned(3 * (size_t)B + 16));
    {
        std::vector<int> ms(B);
        for (int b = 0; b < B; ++b) ms[b] = bt.cfg[b].M;
        CMCG_HIP(hipMemcpyAsync(bt.msteps.p, ms.data(), B * sizeof(int), hipMemcpyHostToDevice, st));
        CMCG_HIP(hipStreamSynchronize(st));
    }
    build_table(bt, st);
    std::vector<int> act(B, 1);
    set_active(bt, act, st);
}

// Times the stage variants on up to 8 homogeneous steps of the batched launch
// (every member active), keeps the fastest as the process-wide choice and
// remembers it for this shape.
int tune_batch(Batch& bt, hipStream_t st, double* us) {
    const SpaceData& s = *bt.sp;
    const int save = bt.Mmax, Mt = std::min(save, 8);
    launch_zero(bt.U.p, bt.U.bytes, st);
    if (bt.Ulo.p) launch_zero(bt.Ulo.p, bt.Ulo.bytes, st);
    int v;
    try {
        v = time_stage_variants(s.q, s.precision, st, [&] {
            bt.Mmax = Mt;
            enqueue_batch_period(bt, false, false, st);
            bt.Mmax = save;
        }, Mt * bt.S, us);
    } catch (...) {
        bt.Mmax = save;
        throw;
    }
    remember_tuned_variant(s.device, s.q, s.precision, s.K, bt.B, v);
    return v;
}

}  // namespace

int autotune_batch(cmcg_problem* const* probs, int B, const cmcg_options* o, hipStream_t st, double* us) {
    if (!probs || B < 1) fail(CMCG_ERR_ARG, "autotune_batch: NULL argument or empty batch");
    Batch bt;
    setup_batch(bt, probs, B, o, st);
    if (bt.sp->dim != 3) fail(CMCG_ERR_ARG, "autotune_batch: the stage variants exist for tetrahedral spaces");
    double tmp[kStageVariants];
    const int v = tune_batch(bt, st, us ? us : tmp);
    CMCG_HIP(hipStreamSynchronize(st));
    return v;
}

namespace {

void solve_prepared(Batch& bt, const cmcg_options* o, hipStream_t st, cmcg_result** out) {
    const int B = bt.B;
    const SpaceData& s = *bt.sp;
    const int64_t n = s.ndof, K = s.K;
    std::vector<int> act(B, 1);
    if (o->autotune && s.dim == 3 && !apply_tuned_variant(s.device, s.q, s.precision, K, B)) {
        double us[kStageVariants];
        tune_batch(bt, st, us);
    }

    double *U = bt.vu.as<double>(), *R = bt.vr.as<double>(), *D = bt.vd.as<double>(), *A = bt.va.as<double>(),
           *W = bt.vw.as<double>(), *Gs = bt.vgs.as<double>();
    CMCG_HIP(hipStreamSynchronize(st));
    const auto t0 = std::chrono::steady_clock::now();
    auto secs = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    const std::vector<double> one(B, 1.0), zero(B, 0.0), mone(B, -1.0);
    std::vector<int> periods(B, 0), iters(B, 0);
    std::vector<double> t6(B, -1.0), rel(B, 1.0), J0(B), best(B, 1.0);
    std::vector<int> diverged(B, 0);
    std::vector<std::vector<double>> hist(B, std::vector<double>{1.0});
    auto count_periods = [&](int k) {
        for (int b = 0; b < B; ++b)
            if (act[b]) periods[b] += k;
    };
    // Algorithm 1 for every member
    batch_apply(bt, o, nullptr, W, nullptr, +1, true, false, st);
    batch_apply(bt, o, W, Gs, W, -1, false, false, st);
    batch_axpby(bt, mone, Gs, zero, Gs, Gs, st);
    count_periods(2);
    std::vector<double> d;
    batch_dots(bt, W, W, d, st);
    for (int b = 0; b < B; ++b) {
        J0[b] = 0.5 * d[b];
        if (!std::isfinite(J0[b]))
            fail(CMCG_ERR_UNSTABLE, "solve_batch: member " + std::to_string(b) + " non-finite after the first period");
    }
    const bool fixed = o->fixed_iters > 0;
    const int limit = fixed ? o->fixed_iters : o->max_iter;
    const int refresh = o->residual_refresh > 0 ? o->residual_refresh : 0;
    auto gradient = [&](double* outv) {
        batch_apply(bt, o, U, W, U, +1, false, false, st);
        batch_apply(bt, o, W, outv, W, -1, false, false, st);
        batch_axpby(bt, one, outv, mone, Gs, outv, st);
        count_periods(2);
    };
    launch_zero(U, bt.db(), st);
    if (o->runup > 0) {
        // run-up: limiting-amplitude periods U <- P_psi U from zero
        for (int l = 0; l < o->runup; ++l) batch_apply(bt, o, U, U, nullptr, +1, true, false, st);
        count_periods(o->runup);
    }
    if (!fixed) CMCG_HIP(hipMemcpyAsync(bt.vbest.p, U, bt.db(), hipMemcpyDeviceToDevice, st));
    if (o->runup > 0)
        gradient(R);
    else
        batch_axpby(bt, mone, Gs, zero, Gs, R, st);  // R0 = -G*
    CMCG_HIP(hipMemcpyAsync(D, R, bt.db(), hipMemcpyDeviceToDevice, st));
    std::vector<double> rr, rr0;
    batch_dots(bt, R, R, rr, st);
    rr0 = rr;
    for (int b = 0; b < B; ++b) {
        if (!std::isfinite(rr[b])) fail(CMCG_ERR_UNSTABLE, "solve_batch: non-finite initial residual");
        if (rr0[b] == 0.0) {
            rel[b] = 0.0;
            act[b] = 0;
        }
    }
    int it = 0;
    while (it < limit) {
        bool any = false;
        for (int b = 0; b < B; ++b) {
            if (!act[b]) continue;
            rel[b] = std::sqrt(rr[b] / rr0[b]);
            if (t6[b] < 0 && rel[b] <= 1e-6) t6[b] = secs();
            if (!fixed && rel[b] <= o->tol) {
                act[b] = 0;
                continue;
            }
            any = true;
        }
        if (!any) break;
        set_active(bt, act, st);
        batch_apply(bt, o, D, W, D, +1, false, false, st);
        batch_apply(bt, o, W, A, W, -1, false, false, st);
        count_periods(2);
        std::vector<double> dA;
        batch_dots(bt, D, A, dA, st);
        std::vector<double> na(B, 0.0);
        for (int b = 0; b < B; ++b) {
            if (!act[b]) continue;
            if (!std::isfinite(dA[b]))
                fail(CMCG_ERR_UNSTABLE, "solve_batch: member " + std::to_string(b) + " non-finite values");
            if (!(dA[b] > 0)) fail(CMCG_ERR_BREAKDOWN, "solve_batch: member " + std::to_string(b) + " CG breakdown");
            na[b] = -(rr[b] / dA[b]);
        }
        batch_axpby(bt, na, D, one, U, U, st);
        batch_axpby(bt, na, A, one, R, R, st);
        ++it;
        for (int b = 0; b < B; ++b)
            if (act[b]) ++iters[b];
        if (refresh > 0 && it % refresh == 0) gradient(R);
        std::vector<double> rn;
        batch_dots(bt, R, R, rn, st);
        std::vector<double> beta(B, 0.0), keep_new(B, 0.0), keep_old(B, 1.0);
        bool improved = false;
        for (int b = 0; b < B; ++b) {
            if (!act[b]) continue;
            if (!std::isfinite(rn[b])) fail(CMCG_ERR_UNSTABLE, "solve_batch: non-finite residual");
            beta[b] = rn[b] / rr[b];
            rr[b] = rn[b];
            rel[b] = std::sqrt(rr[b] / rr0[b]);
            hist[b].push_back(rel[b]);
            if (t6[b] < 0 && rel[b] <= 1e-6) t6[b] = secs();
            if (fixed) continue;
            if (rel[b] < best[b]) {  // the best iterate so far is kept (cf. kDivergence)
                best[b] = rel[b];
                keep_new[b] = 1.0;
                keep_old[b] = 0.0;
                improved = true;
            } else if (rel[b] > kDivergence * best[b]) {
                diverged[b] = 1;
                act[b] = 0;
            }
        }
        if (improved) batch_axpby(bt, keep_new, U, keep_old, bt.vbest.as<double>(), bt.vbest.as<double>(), st);
        batch_axpby(bt, one, R, beta, D, D, st);
        if (o->progress) {
            double worst = 0;
            for (int b = 0; b < B; ++b)
                if (act[b]) worst = std::max(worst, rel[b]);
            if (o->progress(o->progress_ctx, it, worst) != 0) break;
        }
    }
    // diverged members return to their best iterate
    {
        std::vector<double> take_best(B, 0.0), keep(B, 1.0);
        bool anyd = false;
        for (int b = 0; b < B; ++b)
            if (diverged[b]) {
                take_best[b] = 1.0;
                keep[b] = 0.0;
                rel[b] = best[b];
                anyd = true;
            }
        if (anyd) batch_axpby(bt, take_best, bt.vbest.as<double>(), keep, U, U, st);
    }
    // filter period for every member
    std::fill(act.begin(), act.end(), 1);
    set_active(bt, act, st);
    batch_apply(bt, o, U, nullptr, nullptr, +1, true, true, st);
    for (int b = 0; b < B; ++b) periods[b] += 1;
    CMCG_HIP(hipStreamSynchronize(st));
    const double total = secs();
    for (int b = 0; b < B; ++b) {
        std::unique_ptr<cmcg_result> r(new cmcg_result());
        r->sp = bt.sp;
        r->Fre.alloc(n * 8);
        r->Fim.alloc(n * 8);
        r->U0.alloc(n * 8);
        CMCG_HIP(hipMemcpyAsync(r->Fre.p, bt.Fre.as<double>() + b * n, n * 8, hipMemcpyDeviceToDevice, st));
        CMCG_HIP(hipMemcpyAsync(r->Fim.p, bt.Fim.as<double>() + b * n, n * 8, hipMemcpyDeviceToDevice, st));
        CMCG_HIP(hipMemcpyAsync(r->U0.p, U + b * n, n * 8, hipMemcpyDeviceToDevice, st));
        cmcg_stats& S = r->st;
        S.iters = iters[b];
        S.periods = periods[b];
        S.steps = bt.cfg[b].M;
        S.dt = bt.cfg[b].dt;
        S.rel_res = rel[b];
        S.J0 = J0[b];
        S.res0 = std::sqrt(rr0[b]);
        S.seconds = total;
        S.seconds_to_1e6 = t6[b];
        S.dof_updates = (double)n * bt.cfg[b].M * periods[b];
        S.status = (diverged[b] || (!fixed && rel[b] > o->tol)) ? CMCG_NOT_CONVERGED : CMCG_OK;
        r->history = hist[b];
        out[b] = r.release();
    }
    CMCG_HIP(hipStreamSynchronize(st));
}

}  // namespace

void solve_batch(cmcg_problem* const* probs, int B, const cmcg_options* o, hipStream_t st, cmcg_result** out) {
    if (!probs || B < 1 || !out) fail(CMCG_ERR_ARG, "solve_batch: NULL argument or empty batch");
    Batch bt;
    setup_batch(bt, probs, B, o, st);
    solve_prepared(bt, o, st, out);
}

struct BatchState {
    Batch bt;
};

BatchState* batch_prepare(cmcg_problem* const* probs, int B, const cmcg_options* o, hipStream_t st) {
    if (!probs || B < 1) fail(CMCG_ERR_ARG, "batch_prepare: NULL argument or empty batch");
    std::unique_ptr<BatchState> bs(new BatchState());
    setup_batch(bs->bt, probs, B, o, st);
    if (o->use_graph) {
        // every period the solve runs: with source (Algorithm 1, run-up), the
        // homogeneous forward / backward periods, the filter period
        batch_graph(bs->bt, true, false);
        batch_graph(bs->bt, false, false);
        batch_graph(bs->bt, true, true);
    }
    bs->bt.no_capture = true;
    CMCG_HIP(hipStreamSynchronize(st));
    return bs.release();
}

void batch_run(BatchState* bs, cmcg_problem* const* probs, int B, const cmcg_options* o, hipStream_t st,
               cmcg_result** out) {
    if (!bs || !probs || B != bs->bt.B || !out) fail(CMCG_ERR_ARG, "batch_run: arguments do not match the batch");
    for (int b = 0; b < B; ++b)
        if (probs[b] != bs->bt.P[b]) fail(CMCG_ERR_ARG, "batch_run: problems differ from the prepared batch");
    solve_prepared(bs->bt, o, st, out);
}

void batch_free(BatchState* bs) { delete bs; }

}  // namespace cmcg
