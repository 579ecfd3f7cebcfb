// Serving engine: continuous batching of independent CMCG solves.
//
// Requests (problems of any mesh, order and frequency) are admitted into
// slots while their device working set fits the memory budget; each slot
// owns a HIP stream and a CMCG state machine (CgRun).  cmcg_engine_step
// visits the running slots in turn: it waits for the slot's in-flight chunk,
// consumes its scalars and enqueues the next chunk, so while the host waits
// for one slot the others' periods run on the device.  Finished solves stay
// resident until collected, which frees the slot and its budget.  A slot runs
// exactly the launch sequence of cmcg_solve, so a served result equals the
// same problem solved alone.
//
// cmcg_engine_step polls the slots' streams and advances every slot whose
// chunk has completed, so a short solve is never held back by a long one on
// another slot; it blocks (polling) only until at least one slot has
// advanced.
#include <atomic>
#include <thread>

#include "objects.h"

// A co-batched slot: requests on one space solved together by the batched
// path (cmcg_solve_batch's launches, one per Runge-Kutta stage for every
// member) on a worker thread that owns the slot's stream.  The batch is set
// up and its periods captured on the admitting thread; the worker replays.
struct BatchJob {
    std::vector<cmcg_problem*> probs;
    cmcg_options o{};
    cmcg::BatchState* bs = nullptr;
    std::vector<cmcg_result*> res;
    std::atomic<bool> done{false};
    std::atomic<bool> stop{false};  // set by a cancel: the solve stops at its next CG iteration
    int code = 0;
    std::string msg;
    std::thread th;
    static int progress(void* ctx, int, double) { return static_cast<BatchJob*>(ctx)->stop.load() ? 1 : 0; }
    ~BatchJob() {
        stop.store(true);
        if (th.joinable()) th.join();
        for (auto* r : res) delete r;
        cmcg::batch_free(bs);
    }
};

struct cmcg_engine {
    struct Slot {
        int state = 0;  // 0 free, 1 running, 2 finished, 3 failed
        cmcg_problem* p = nullptr;
        size_t bytes = 0;
        hipStream_t st = nullptr;
        std::unique_ptr<cmcg::CgRun> run;
        std::unique_ptr<cmcg_result> result;
        std::unique_ptr<BatchJob> job;  // co-batched slot
        int err = 0;
        std::string msg;
        bool holds(const cmcg_problem* q) const {
            if (p == q) return true;
            if (job)
                for (auto* b : job->probs)
                    if (b == q) return true;
            return false;
        }
    };
    int device = 0;
    size_t budget = 0, used = 0;
    std::vector<Slot> slots;
    ~cmcg_engine() {
        for (auto& s : slots) {
            s.job.reset();  // joins a running worker
            if (s.st) {
                (void)hipStreamSynchronize(s.st);
                (void)hipStreamDestroy(s.st);
            }
        }
    }
};

namespace cmcg {

// Device bytes a solve of p keeps resident: the problem's own data
// (geometry, source, mass weights) plus the solve's field, filter and CG
// vectors and its result.
size_t footprint(const cmcg_problem* p) {
    const SpaceData& s = *p->sp;
    const size_t n = s.ndof, es = s.esize(), K = s.K;
    const size_t H = p->nharm;
    size_t b = K * geo_values(s) * es + 2 * K * 8;  // geometry, mass weights
    if (p->src_rows) b += 2 * n * es * H + p->smask.bytes;  // source (per harmonic) and its element mask
    b += 5 * n * es;                       // U, Y1, Y2, Acc, RHS buffer
    if (s.precision == CMCG_FP32) b += 2 * n;  // bfloat16 low parts of U
    b += 2 * n * 8 * H;                    // filter accumulators (per harmonic)
    b += 7 * n * 8;                        // CG vectors (with the best iterate)
    b += (2 * H + 1) * n * 8;              // result: filtered fields, U0
    return b + (size_t)dot_partials() * 8 + 4096;
}

// footprint with the work buffers local time stepping adds (Taylor
// coefficients, frozen coarse terms, adjoint vectors; masks and block lists)
size_t footprint(const cmcg_problem* p, const cmcg_options* o) {
    size_t b = footprint(p);
    if (o && o->lts_ratio > 1) {
        const SpaceData& s = *p->sp;
        b += 12 * s.ndof * s.esize() + 5 * (size_t)source_mask_words(s.K) * 4;
    }
    return b;
}

namespace {

// footprint of a co-batched slot: the members' own footprints plus what the
// batch copies -- every member's source and source mask (when any member has
// a source) and the geometry and mass weights (once when the members share
// their media)
size_t batch_footprint(cmcg_problem* const* probs, int n) {
    const SpaceData& s = *probs[0]->sp;
    const size_t nd = s.ndof, es = s.esize(), K = s.K;
    size_t b = 0;
    bool shared = true, src = false;
    for (int i = 0; i < n; ++i) {
        b += footprint(probs[i]);
        shared = shared && probs[i]->eps == probs[0]->eps && probs[i]->mu == probs[0]->mu &&
                 probs[i]->sigma == probs[0]->sigma;
        src = src || probs[i]->src_rows != 0;
    }
    if (src) b += (size_t)n * (2 * nd * es + (size_t)source_mask_words(s.K) * 4);
    b += (shared ? 1 : (size_t)n) * (K * geo_values(s) * es + 2 * K * 8);
    return b;
}

}  // namespace

}  // namespace cmcg

using namespace cmcg;

#define ENGINE_GUARD_BEGIN try {
#define ENGINE_GUARD_END          \
    }                             \
    catch (const Error& e) {      \
        set_last_error(e.msg);    \
        return e.code;            \
    }                             \
    catch (const std::exception& e) { \
        set_last_error(e.what()); \
        return CMCG_ERR_ARG;      \
    }

extern "C" {

int cmcg_problem_footprint(const cmcg_problem* p, size_t* bytes) {
    ENGINE_GUARD_BEGIN
    if (!p || !bytes) fail(CMCG_ERR_ARG, "problem_footprint: NULL argument");
    *bytes = footprint(p);
    return CMCG_OK;
    ENGINE_GUARD_END
}

int cmcg_engine_create(size_t hbm_budget, int max_slots, cmcg_engine** out) {
    ENGINE_GUARD_BEGIN
    if (!out) fail(CMCG_ERR_ARG, "engine_create: NULL output");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 1024) fail(CMCG_ERR_ARG, "engine_create: max_slots must be 1..1024");
    std::unique_ptr<cmcg_engine> e(new cmcg_engine());
    e->device = current_device();
    e->budget = hbm_budget;
    e->slots.resize(max_slots);
    for (auto& s : e->slots) CMCG_HIP(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    *out = e.release();
    return CMCG_OK;
    ENGINE_GUARD_END
}

void cmcg_engine_destroy(cmcg_engine* e) { delete e; }

int cmcg_engine_admit(cmcg_engine* e, cmcg_problem* p, const cmcg_options* o, int* slot) {
    ENGINE_GUARD_BEGIN
    if (!e || !p || !slot) fail(CMCG_ERR_ARG, "engine_admit: NULL argument");
    *slot = -1;
    if (current_device() != e->device) fail(CMCG_ERR_STATE, "engine_admit: wrong current device");
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    int free_slot = -1;
    for (int i = 0; i < (int)e->slots.size(); ++i) {
        const auto& s = e->slots[i];
        if (s.state != 0 && s.holds(p)) fail(CMCG_ERR_STATE, "engine_admit: problem already held by a slot");
        if (s.state == 0 && free_slot < 0) free_slot = i;
    }
    const size_t need = footprint(p, o);
    // a request larger than the whole budget can never be admitted: tell the
    // caller so, instead of "not now"
    if (need > e->budget)
        fail(CMCG_ERR_TOO_LARGE, "engine_admit: footprint " + std::to_string(need) + " B exceeds the budget " +
                                     std::to_string(e->budget) + " B");
    if (free_slot < 0) fail(CMCG_ERR_NOMEM, "engine_admit: no free slot");
    if (e->used + need > e->budget) fail(CMCG_ERR_NOMEM, "engine_admit: over the memory budget");
    auto& s = e->slots[free_slot];
    cmcg_options oe = *o;
    oe.autotune = 0;  // the stage variant is process-wide and slots run concurrently
    s.run.reset(new CgRun());
    s.run->start(p, &oe, nullptr, s.st);
    s.state = 1;
    s.p = p;
    s.bytes = need;
    s.err = 0;
    s.msg.clear();
    e->used += need;
    *slot = free_slot;
    return CMCG_OK;
    ENGINE_GUARD_END
}

int cmcg_engine_admit_batch(cmcg_engine* e, cmcg_problem* const* problems, int n, const cmcg_options* o,
                            int* slot) {
    ENGINE_GUARD_BEGIN
    if (!e || !problems || !slot || n < 1) fail(CMCG_ERR_ARG, "engine_admit_batch: NULL argument or empty batch");
    *slot = -1;
    if (n > 65535) fail(CMCG_ERR_ARG, "engine_admit_batch: at most 65535 problems per batch");
    if (current_device() != e->device) fail(CMCG_ERR_STATE, "engine_admit_batch: wrong current device");
    cmcg_options def;
    cmcg_options_default(&def);
    if (!o) o = &def;
    if (o->lts_ratio > 1) fail(CMCG_ERR_ARG, "engine_admit_batch: local time stepping is for single solves");
    for (int b = 0; b < n; ++b) {
        if (!problems[b]) fail(CMCG_ERR_ARG, "engine_admit_batch: NULL problem");
        if (problems[b]->sp != problems[0]->sp) fail(CMCG_ERR_ARG, "engine_admit_batch: members must share a space");
        if (problems[b]->nharm != 1) fail(CMCG_ERR_ARG, "engine_admit_batch: several-frequency problems are single");
        for (int c = 0; c < b; ++c)
            if (problems[c] == problems[b]) fail(CMCG_ERR_ARG, "engine_admit_batch: a problem appears twice");
    }
    const size_t need = batch_footprint(problems, n);
    if (need > e->budget)
        fail(CMCG_ERR_TOO_LARGE, "engine_admit_batch: footprint " + std::to_string(need) + " B exceeds the budget " +
                                     std::to_string(e->budget) + " B");
    int free_slot = -1;
    for (int i = 0; i < (int)e->slots.size(); ++i) {
        const auto& s = e->slots[i];
        for (int b = 0; b < n; ++b)
            if (s.state != 0 && s.holds(problems[b]))
                fail(CMCG_ERR_STATE, "engine_admit_batch: a problem is already held by a slot");
        if (s.state == 0 && free_slot < 0) free_slot = i;
    }
    if (free_slot < 0) fail(CMCG_ERR_NOMEM, "engine_admit_batch: no free slot");
    if (e->used + need > e->budget) fail(CMCG_ERR_NOMEM, "engine_admit_batch: over the memory budget");
    auto& s = e->slots[free_slot];
    std::unique_ptr<BatchJob> job(new BatchJob());
    job->probs.assign(problems, problems + n);
    job->o = *o;
    job->o.autotune = 0;           // the stage variant is process-wide and slots run concurrently
    // no callbacks into the caller from the worker thread; the job's own one
    // lets a cancel stop the solve at its next iteration
    job->o.progress = &BatchJob::progress;
    job->o.progress_ctx = job.get();
    // set up and capture here: while a stream captures, the runtime refuses
    // legacy-stream work (synchronous copies, a caller's default-stream
    // kernels) from every other thread, so the worker thread never captures
    job->bs = batch_prepare(job->probs.data(), n, &job->o, s.st);
    job->res.assign(n, nullptr);
    BatchJob* jp = job.get();
    const int dev = e->device;
    hipStream_t st = s.st;
    job->th = std::thread([jp, dev, st] {
        try {
            CMCG_HIP(hipSetDevice(dev));
            batch_run(jp->bs, jp->probs.data(), (int)jp->probs.size(), &jp->o, st, jp->res.data());
        } catch (const Error& err) {
            jp->code = err.code;
            jp->msg = err.msg;
        } catch (const std::exception& err) {
            jp->code = CMCG_ERR_ARG;
            jp->msg = err.what();
        }
        jp->done.store(true, std::memory_order_release);
    });
    s.job = std::move(job);
    s.state = 1;
    s.p = nullptr;
    s.bytes = need;
    s.err = 0;
    s.msg.clear();
    e->used += need;
    *slot = free_slot;
    return CMCG_OK;
    ENGINE_GUARD_END
}

int cmcg_engine_slot_members(const cmcg_engine* e, int slot, int* n) {
    ENGINE_GUARD_BEGIN
    if (!e || !n || slot < 0 || slot >= (int)e->slots.size()) fail(CMCG_ERR_ARG, "engine_slot_members: bad argument");
    const auto& s = e->slots[slot];
    *n = s.state == 0 ? 0 : (s.job ? (int)s.job->probs.size() : 1);
    return CMCG_OK;
    ENGINE_GUARD_END
}

int cmcg_engine_collect_batch(cmcg_engine* e, int slot, cmcg_result** out, int n) {
    ENGINE_GUARD_BEGIN
    if (!e || !out || slot < 0 || slot >= (int)e->slots.size()) fail(CMCG_ERR_ARG, "engine_collect_batch: bad argument");
    auto& s = e->slots[slot];
    if (!s.job) fail(CMCG_ERR_STATE, "engine_collect_batch: not a co-batched slot");
    if (s.state != 2 && s.state != 3) fail(CMCG_ERR_STATE, "engine_collect_batch: slot has no finished solve");
    if (n != (int)s.job->probs.size()) fail(CMCG_ERR_ARG, "engine_collect_batch: wrong member count");
    const int code = s.state == 3 ? s.err : CMCG_OK;
    const std::string msg = s.msg;
    int status = CMCG_OK;
    for (int b = 0; b < n; ++b) {
        out[b] = s.job->res[b];
        if (out[b] && out[b]->st.status != CMCG_OK) status = CMCG_NOT_CONVERGED;
        s.job->res[b] = nullptr;
    }
    e->used -= s.bytes;
    s.job.reset();
    s.state = 0;
    s.bytes = 0;
    if (code != CMCG_OK) {
        for (int b = 0; b < n; ++b) {
            delete out[b];
            out[b] = nullptr;
        }
        fail(code, "engine_collect_batch: the batched solve failed: " + msg);
    }
    return status;
    ENGINE_GUARD_END
}

int cmcg_engine_step(cmcg_engine* e, int* n_running, int* n_finished) {
    ENGINE_GUARD_BEGIN
    if (!e) fail(CMCG_ERR_ARG, "engine_step: NULL engine");
    int running = 0, finished = 0;
    for (int spins = 0;; ++spins) {
        bool any = false, advanced = false;
        for (auto& s : e->slots) {
            if (s.state != 1) continue;
            any = true;
            if (s.job) {  // co-batched slot: its worker thread runs the whole solve
                if (s.job->done.load(std::memory_order_acquire)) {
                    s.job->th.join();
                    s.state = s.job->code == 0 ? 2 : 3;
                    s.err = s.job->code;
                    s.msg = s.job->msg;
                    advanced = true;
                }
                continue;
            }
            try {
                const hipError_t q = hipStreamQuery(s.st);
                if (q == hipErrorNotReady) {
                    (void)hipGetLastError();  // not an error: keep launch checks clean
                    continue;
                }
                CMCG_HIP(q);
                s.run->complete();
                advanced = true;
                if (s.run->done()) {
                    s.result = std::move(s.run->res);
                    s.run.reset();
                    s.state = 2;
                }
            } catch (const Error& err) {
                (void)hipGetLastError();
                (void)hipStreamSynchronize(s.st);
                s.run.reset();
                s.state = 3;
                s.err = err.code;
                s.msg = err.msg;
                advanced = true;
            }
        }
        if (!any || advanced) break;
        // nothing completed yet: poll again shortly
        if (spins > 64) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (auto& s : e->slots) {
        running += s.state == 1;
        finished += s.state >= 2;
    }
    if (n_running) *n_running = running;
    if (n_finished) *n_finished = finished;
    return CMCG_OK;
    ENGINE_GUARD_END
}

int cmcg_engine_poll(const cmcg_engine* e, int slot, int* state) {
    ENGINE_GUARD_BEGIN
    if (!e || !state || slot < 0 || slot >= (int)e->slots.size()) fail(CMCG_ERR_ARG, "engine_poll: bad argument");
    *state = e->slots[slot].state;
    return CMCG_OK;
    ENGINE_GUARD_END
}

int cmcg_engine_collect(cmcg_engine* e, int slot, cmcg_result** out) {
    ENGINE_GUARD_BEGIN
    if (!e || !out || slot < 0 || slot >= (int)e->slots.size()) fail(CMCG_ERR_ARG, "engine_collect: bad argument");
    *out = nullptr;
    auto& s = e->slots[slot];
    if (s.job) fail(CMCG_ERR_STATE, "engine_collect: a co-batched slot is collected with engine_collect_batch");
    if (s.state != 2 && s.state != 3) fail(CMCG_ERR_STATE, "engine_collect: slot has no finished solve");
    const int code = s.state == 3 ? s.err : CMCG_OK;
    const std::string msg = s.msg;
    cmcg_result* r = s.result.release();
    e->used -= s.bytes;
    s.state = 0;
    s.p = nullptr;
    s.bytes = 0;
    s.result.reset();
    s.run.reset();
    if (code != CMCG_OK) fail(code, "engine_collect: the solve failed: " + msg);
    *out = r;
    return r->st.status;
    ENGINE_GUARD_END
}

int cmcg_engine_cancel(cmcg_engine* e, int slot) {
    ENGINE_GUARD_BEGIN
    if (!e || slot < 0 || slot >= (int)e->slots.size()) fail(CMCG_ERR_ARG, "engine_cancel: bad argument");
    auto& s = e->slots[slot];
    if (s.state == 0) fail(CMCG_ERR_STATE, "engine_cancel: slot is free");
    s.job.reset();  // a co-batched solve stops at its next iteration (joins its worker)
    CMCG_HIP(hipStreamSynchronize(s.st));
    e->used -= s.bytes;
    s.run.reset();
    s.result.reset();
    s.state = 0;
    s.p = nullptr;
    s.bytes = 0;
    return CMCG_OK;
    ENGINE_GUARD_END
}

int cmcg_engine_info(const cmcg_engine* e, size_t* used, int* running, int* finished) {
    ENGINE_GUARD_BEGIN
    if (!e) fail(CMCG_ERR_ARG, "engine_info: NULL engine");
    int r = 0, f = 0;
    for (const auto& s : e->slots) {
        r += s.state == 1;
        f += s.state >= 2;
    }
    if (used) *used = e->used;
    if (running) *running = r;
    if (finished) *finished = f;
    return CMCG_OK;
    ENGINE_GUARD_END
}

}  // extern "C"
