// Host-side object definitions shared by the single-problem and batched
// drivers (not part of the ABI).
#pragma once

#include <chrono>
#include <complex>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"
#include "launch.h"

namespace cmcg {

// Device buffer owned by a host object (hipMalloc / hipFree).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t b) {
        if (p && bytes == b) return;
        release();
        if (b == 0) return;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(CMCG_ERR_NOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
        }
        bytes = b;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T* as() const { return (T*)p; }
};

// Small pinned host staging area for scalar read-backs.
struct HostPinned {
    double* p = nullptr;
    explicit HostPinned(size_t n = 16) {
        if (hipHostMalloc((void**)&p, n * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(CMCG_ERR_NOMEM, "hipHostMalloc failed");
        }
    }
    ~HostPinned() {
        if (p) (void)hipHostFree(p);
    }
};

struct SpaceData {
    std::shared_ptr<MeshData> mesh;
    int dim = 3;  // 3: tetrahedra, fields [K][6][Np]; 2: triangles (TM), fields [K][3][Np]
    int q = 1, Np = 4, Nfp = 3, precision = CMCG_FP64, device = 0;
    int64_t K = 0, ndof = 0;
    std::vector<int32_t> conn_h;
    DevBuf conn;
    size_t esize() const { return precision == CMCG_FP64 ? 8 : 4; }
};

// Dimension dispatch (SpaceData::dim) of the stage and field-conversion
// kernels, and the per-element geometry size.
inline int geo_values(const SpaceData& s) { return s.dim == 2 ? kGeo2 : kGeo; }
inline void stage_dim(const SpaceData& s, const StageArgs& a, hipStream_t st) {
    if (s.dim == 2)
        launch_stage2d(s.q, s.precision, a, st);
    else
        launch_stage(s.q, s.precision, a, st);
}
inline void to_field_dim(const SpaceData& s, const double* X, void* U, void* Ulo, int64_t n, int flip,
                         hipStream_t st) {
    if (s.dim == 2)
        launch_to_field2d(s.precision, s.Np, X, U, Ulo, n, flip, st);
    else
        launch_to_field(s.precision, s.Np, X, U, Ulo, n, flip, st);
}
inline void from_field_dim(const SpaceData& s, const void* U, const void* Ulo, double* Y, const double* sub,
                           int64_t n, int flip, hipStream_t st) {
    if (s.dim == 2)
        launch_from_field2d(s.precision, s.Np, U, Ulo, Y, sub, n, flip, st);
    else
        launch_from_field(s.precision, s.Np, U, Ulo, Y, sub, n, flip, st);
}

// time-stepping configuration of one solve
struct StepCfg {
    int M = 0;           // (coarse) steps per period
    int scheme = 2;
    double dt = 0, T = 0;
    double alpha = 1.0;  // flux parameter
    double cq = 0;       // CFL constant of the step rule
    int lts = 1;         // > 1: local time stepping with lts fine substeps (lts.cpp)
};

}  // namespace cmcg

struct cmcg_space {
    std::shared_ptr<cmcg::SpaceData> d;
};

struct cmcg_problem {
    std::shared_ptr<cmcg::SpaceData> sp;
    double omega = 0;  // the (base) frequency: the period is 2 pi / omega
    int nharm = 1;                 // harmonics of the source (several-frequency problems)
    std::vector<int> kharm{1};     // harmonic h has frequency kharm[h] * omega
    std::vector<double> eps, mu, sigma;
    bool has_j = false, has_g = false;
    // device data
    cmcg::DevBuf geo, wE, wH, Sre, Sim;
    cmcg::DevBuf smask;  // source element mask (StageArgs::smask)
    double geo_alpha = -1;
    int src_rows = 0;
    // work buffers
    cmcg::DevBuf U, Y1, Y2, Acc, Fre, Fim, Kbuf;
    cmcg::DevBuf Ulo;  // FP32 fields: bfloat16 low parts of U
    cmcg::DevBuf v_u, v_r, v_d, v_a, v_w, v_gs, v_t, v_best;
    cmcg::DevBuf partial, scal;
    // local time stepping: fine-element mask (per element block) for the coarse
    // step lts_H, Taylor coefficients, frozen coarse terms, adjoint work vectors
    cmcg::DevBuf lts_mask, lts_hbmask, lts_h2nf, lts_hblocks, lts_h2blocks, lD[3], lW[4], lWB[4], lZ0;
    double lts_H = -1, lts_cq = -1;
    int64_t lts_fine = 0, lts_nhb = 0, lts_nh2b = 0;
    std::map<int64_t, hipGraphExec_t> lts_graphs;  // captured LTS periods
    std::unique_ptr<cmcg::HostPinned> pinned;
    hipStream_t cap_stream = nullptr;
    std::map<int64_t, hipGraphExec_t> graphs;
    ~cmcg_problem() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        for (auto& kv : lts_graphs) (void)hipGraphExecDestroy(kv.second);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

struct cmcg_result {
    std::shared_ptr<cmcg::SpaceData> sp;
    int nharm = 1;                 // filtered fields stacked per harmonic in Fre, Fim
    cmcg::DevBuf Fre, Fim, U0;
    cmcg_stats st{};
    std::vector<double> history;
};

namespace cmcg {

// One CMCG solve as a resumable sequence of asynchronous chunks (see
// solver.cpp); cmcg_solve drives it to the end, the serving engine
// interleaves many of them on separate streams.
struct CgRun {
    enum { kStart = 0, kAwaitDA, kAwaitRR, kFinal, kDone };
    cmcg_problem* p = nullptr;
    cmcg_options o{};
    StepCfg c;
    hipStream_t st = nullptr;
    const double* u0 = nullptr;
    std::unique_ptr<cmcg_result> res;
    int phase = kDone;
    int64_t n = 0;
    int it = 0, periods = 0, refresh = 0, limit = 0;
    bool fixed = false, stopped = false, diverged = false;
    double rr = 0, rr0 = 0, rel = 1, t6 = -1, J0 = 0, best = 0;
    std::chrono::steady_clock::time_point t0;
    void start(cmcg_problem* pr, const cmcg_options* opt, const double* u0_, hipStream_t s_);
    void complete();
    bool done() const { return phase == kDone; }
    double secs() const;

  private:
    void decide();
    void gradient(double* out);
};

// A solve whose recursive residual grows past this factor times the smallest
// one seen has left the range its arithmetic resolves: it stops, returns the
// best iterate and reports CMCG_NOT_CONVERGED.
constexpr double kDivergence = 100.0;

// Stage-variant autotuner (solver.cpp): runs `run` (which enqueues
// `nlaunch` stage launches, the same ones each call) under every variant that
// applies to (q, precision), keeps the fastest as the process-wide choice and
// returns it; us[v] = average microseconds per launch, 0 where v does not apply.
int time_stage_variants(int q, int precision, hipStream_t st, const std::function<void()>& run, int nlaunch,
                        double* us);
// Cached choice for (device, q, precision, K, members): applies it and returns
// true, or returns false when that shape has not been tuned in this process.
bool apply_tuned_variant(int device, int q, int precision, int64_t K, int members);
void remember_tuned_variant(int device, int q, int precision, int64_t K, int members, int variant);

// helpers defined in solver.cpp
void ensure_constants(int device, int q, int dim = 3);
int current_device();
StepCfg step_config(const cmcg_problem* p, const cmcg_options* o);
void hermite_weights(double omega, double dt, std::complex<double> xi[4]);
void build_geo(cmcg_problem* p, double alpha);
// local time stepping (lts.cpp): work buffers and fine mask for c, and one
// period on p->U (direction +1: forward, with source / filter as asked;
// -1: the adjoint of the homogeneous period, in S-flipped variables)
void ensure_lts(cmcg_problem* p, const StepCfg& c);
void lts_period(cmcg_problem* p, const StepCfg& c, int direction, bool src, bool filt, hipStream_t st);
void prepare(cmcg_problem* p, const StepCfg& c);
cmcg_result* solve(cmcg_problem* p, const cmcg_options* o, const double* u0, hipStream_t st);
cmcg_result* fw_solve(cmcg_problem* p, const cmcg_options* o, const double* u0, hipStream_t st);
void solve_batch(cmcg_problem* const* probs, int B, const cmcg_options* o, hipStream_t st, cmcg_result** out);
// The same in two parts, for a solve run on another thread than the one that
// prepares it: batch_prepare sets the batch up on st and, when o->use_graph,
// captures the graphs of its periods (a capture refuses legacy-stream work on
// every other thread, so it is done here, on the caller's thread); batch_run
// then only replays graphs (a period without a captured graph runs eagerly).
struct BatchState;
BatchState* batch_prepare(cmcg_problem* const* probs, int B, const cmcg_options* o, hipStream_t st);
void batch_run(BatchState* bs, cmcg_problem* const* probs, int B, const cmcg_options* o, hipStream_t st,
               cmcg_result** out);
void batch_free(BatchState* bs);
// Batched stage autotuner: every variant on up to 8 homogeneous steps of the
// batched launch with all members active; returns the fastest (kept as the
// process-wide choice), us[v] = microseconds per launch.
int autotune_batch(cmcg_problem* const* probs, int B, const cmcg_options* o, hipStream_t st, double* us);
}  // namespace cmcg
