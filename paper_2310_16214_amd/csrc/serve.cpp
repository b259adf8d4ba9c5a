// Continuous-batching request loop (include/ppx_serve.h): FIFO admission by
// HBM budget, one mixed persistent launch per progress step over everything
// admitted since the last launch, several launches in flight on separate
// streams, completion by events.  The per-request mode is the baseline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ppx_serve.h"
#include "../../include/ppx_tune.h"
#include "mixed.h"

namespace ppx {
namespace {

// Admission caps of one mixed launch.
constexpr int64_t kMixLaunchTiles = kMixMaxTiles;
constexpr int kMixLaunchJobs = kMixMaxJobs;

int64_t elem_bytes(int dtype) { return dtype == PPX_C64 || dtype == PPX_F64 ? 8 : 4; }

int64_t job_in_bytes(const ppx_job &j) {
    return (j.op == PPX_OP_TRIDIAG ? 4 : 1) * j.n * j.batch * elem_bytes(j.dtype);
}
int64_t job_out_bytes(const ppx_job &j) { return j.n * j.batch * elem_bytes(j.dtype); }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
  public:
    void reset(int64_t size) {
        free_.clear();
        if (size > 0) free_[0] = size;
    }
    int64_t alloc(int64_t bytes) {
        bytes = (bytes + 255) & ~int64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                const int64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest > 0) free_[off + bytes] = rest;
                return off;
            }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = (bytes + 255) & ~int64_t(255);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<int64_t, int64_t> free_;
};

struct Job {
    int64_t id;
    ppx_job job;
    double arrival_us = 0, admit_us = 0, complete_us = 0;
    int64_t footprint = 0, arena_off = -1;
    bool completed = false;
};

struct Launch {
    std::vector<int64_t> ids;
    hipEvent_t done = nullptr;
    int stream = 0;
    // a fused launch retires its jobs by stage: stage k's jobs are complete
    // once stage_ev[k] has fired (stages finish in order on the stream)
    std::vector<hipEvent_t> stage_ev;
    std::vector<std::vector<int64_t>> stage_ids;
    size_t stages_done = 0;
    // an online-tuning evaluation: timed by start -> done (both with timing)
    ppx_online *session = nullptr;
    hipEvent_t start = nullptr;
    double elems = 0;
};

// Jobs smaller than this (elements) are not timed for online tuning: below
// it a launch does not fill the GPU and its time is mostly fixed overhead.
constexpr double kOnlineMinElems = double(1 << 20);

}  // namespace
}  // namespace ppx

struct ppx_server {
    int flags = 0, max_inflight = 1;
    int64_t budget = 0, used = 0, peak = 0;
    char *arena_base = nullptr;
    ppx::Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> free_events;
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, ppx::Job> jobs;
    std::deque<ppx::Launch> inflight;
    std::deque<int64_t> completed;
    int64_t next_id = 1, submitted = 0, admitted = 0, ncompleted = 0, released = 0, launches = 0;
    int max_inflight_seen = 0, rr = 0;
    int64_t online_evals = 0;
    // online tuning sessions by (op, dtype, n, tridiagonal family or -1)
    std::map<std::tuple<int, int, int64_t, int>, ppx_online *> sessions;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    bool null_device() const { return flags & PPX_SERVE_NULL_DEVICE; }
    bool per_request() const { return flags & PPX_SERVE_PER_REQUEST; }
    bool online() const { return flags & PPX_SERVE_ONLINE_TUNE; }
    double now_us() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace ppx {
namespace {

hipEvent_t take_event(ppx_server *s) {
    if (s->null_device()) return nullptr;
    if (!s->free_events.empty()) {
        hipEvent_t e = s->free_events.back();
        s->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

int launch_single(const ppx_job &j, hipStream_t st, const ppx_config *cfg) {
    if (j.op == PPX_OP_SCAN && j.algo == PPX_JOB_SCAN_EXCLUSIVE)
        return scan_exclusive_batched(j.in, j.out, j.n, j.batch, j.dtype, cfg, st);
    if (cfg) {
        switch (j.op) {
            case PPX_OP_FFT: return fft_batched(j.in, j.out, j.n, j.batch, j.direction, cfg, st);
            case PPX_OP_SCAN: return scan_batched(j.in, j.out, j.n, j.batch, j.dtype, cfg, st);
            default: return tridiag_batched(j.in, j.b, j.c, j.d, j.out, j.n, j.batch, j.dtype, cfg, st);
        }
    }
    switch (j.op) {
        case PPX_OP_FFT: return fft_batched(j.in, j.out, j.n, j.batch, j.direction, nullptr, st);
        case PPX_OP_SCAN: return scan_batched(j.in, j.out, j.n, j.batch, j.dtype, nullptr, st);
        default: {
            // the job's family: its tuned entry, else the analytical choice
            // within it (the configuration the mixed launch's tiles follow)
            ppx_config c{};
            if (int rc = job_config(j, c)) return rc;
            return tridiag_batched(j.in, j.b, j.c, j.d, j.out, j.n, j.batch, j.dtype, &c, st);
        }
    }
}

void complete_job(ppx_server *s, int64_t id, double t) {
    Job &j = s->jobs[id];
    j.completed = true;
    j.complete_us = t;
    s->completed.push_back(id);
    ++s->ncompleted;
}

// Retires launches whose completion event has fired (all of them, in the
// null-device mode), and the finished stages of fused launches still
// running.
void retire(ppx_server *s) {
    const double t = s->now_us();
    for (auto it = s->inflight.begin(); it != s->inflight.end();) {
        while (!s->null_device() && it->stages_done < it->stage_ev.size() &&
               hipEventQuery(it->stage_ev[it->stages_done]) == hipSuccess) {
            for (int64_t id : it->stage_ids[it->stages_done]) complete_job(s, id, t);
            s->free_events.push_back(it->stage_ev[it->stages_done]);
            ++it->stages_done;
        }
        bool done = s->null_device() || hipEventQuery(it->done) == hipSuccess;
        if (!done) {
            ++it;
            continue;
        }
        if (it->session) {  // an online-tuning evaluation: report its cost
            float ms = -1.0f;
            const bool timed = hipEventElapsedTime(&ms, it->start, it->done) == hipSuccess;
            (void)ppx_online_report(it->session, timed ? ms * 1e6 / it->elems : -1.0);  // ns per element
            (void)hipEventDestroy(it->start);
            (void)hipEventDestroy(it->done);
            it->done = nullptr;
        }
        if (it->stage_ev.empty()) {
            for (int64_t id : it->ids) complete_job(s, id, t);
        } else {  // the stages not seen yet (all fired with the final event)
            for (; it->stages_done < it->stage_ev.size(); ++it->stages_done) {
                for (int64_t id : it->stage_ids[it->stages_done]) complete_job(s, id, t);
                s->free_events.push_back(it->stage_ev[it->stages_done]);
            }
        }
        if (it->done) s->free_events.push_back(it->done);
        it = s->inflight.erase(it);
    }
}

// Admits pending jobs in arrival order while they fit; stops at the first
// that does not (no overtaking), so a large job is delayed, never starved.
// One launch takes at most budget / max_inflight bytes of footprint (a job
// larger than that goes alone): with every job pending at once, one launch
// would otherwise take the whole budget, the next could be admitted only
// after it completed, and the GPU would idle while the host retires,
// admits and launches; with the cap a launch is always queued behind the
// running one.
std::vector<int64_t> admit(ppx_server *s, int64_t tile_cap, int job_cap) {
    std::vector<int64_t> out;
    int64_t tiles = 0, bytes = 0;
    const int64_t launch_cap = s->budget / std::max(1, s->max_inflight);
    const double t = s->now_us();
    while (!s->pending.empty() && (int)out.size() < job_cap) {
        Job &j = s->jobs[s->pending.front()];
        if (s->used + j.footprint > s->budget) break;
        if (!out.empty() && bytes + j.footprint > launch_cap) break;
        const int64_t jt = mixed_tile_count(&j.job, 1);  // planned at submit: >= 1
        if (!out.empty() && tiles + jt > tile_cap) break;
        if (!j.job.out) {
            const int64_t off = s->arena.alloc(job_out_bytes(j.job));
            if (off < 0) break;  // fragmented: wait for releases
            j.arena_off = off;
            j.job.out = s->null_device() ? reinterpret_cast<void *>(0x100000 + off)
                                         : static_cast<void *>(s->arena_base + off);
        }
        s->used += j.footprint;
        bytes += j.footprint;
        s->peak = std::max(s->peak, s->used);
        j.admit_us = t;
        tiles += jt;
        out.push_back(j.id);
        s->pending.pop_front();
        ++s->admitted;
    }
    return out;
}

// The online session of a job's class, created on first use (typical batch
// for its analytical fallback: the job's own).
int online_session(ppx_server *s, const ppx_job &j, ppx_online **out) {
    const int fam = j.op == PPX_OP_TRIDIAG ? tri_family(j.algo) : -1;
    const auto key = std::make_tuple(j.op, j.dtype, j.n, fam);
    auto it = s->sessions.find(key);
    if (it == s->sessions.end()) {
        ppx_online *o = nullptr;
        if (int rc = ppx_online_create(j.op, j.dtype, j.n, j.batch, fam, 0, &o)) return rc;
        it = s->sessions.emplace(key, o).first;
    }
    *out = it->second;
    return PPX_OK;
}

// Undoes the admission of jobs whose launch failed: they go back to the
// front of the queue in their order, their budget and arena space are
// returned, and so are the launch's events.
void unadmit(ppx_server *s, const std::vector<int64_t> &ids, Launch &l) {
    for (auto it = ids.rbegin(); it != ids.rend(); ++it) {
        Job &j = s->jobs[*it];
        s->used -= j.footprint;
        if (j.arena_off >= 0) {
            s->arena.release(j.arena_off, job_out_bytes(j.job));
            j.arena_off = -1;
            j.job.out = nullptr;
        }
        j.admit_us = 0;
        s->pending.push_front(*it);
        --s->admitted;
    }
    for (hipEvent_t e : l.stage_ev) s->free_events.push_back(e);
    l.stage_ev.clear();
    l.stage_ids.clear();
    if (l.start) (void)hipEventDestroy(l.start);
    if (l.session) {  // a timed evaluation: its events were its own
        if (l.done) (void)hipEventDestroy(l.done);
        (void)ppx_online_report(l.session, -1.0);  // the candidate counts as failed
        --s->online_evals;
    } else if (l.done) {
        s->free_events.push_back(l.done);
    }
    l.done = l.start = nullptr;
    l.session = nullptr;
}

// Records the completion event of a fused launch's next stage.
struct StageArg {
    ppx_server *s;
    Launch *l;
};
int record_stage(void *arg, hipStream_t st) {
    auto *a = static_cast<StageArg *>(arg);
    hipEvent_t e = take_event(a->s);
    if (!e) return fail(PPX_EHIP, "event creation failed");
    a->l->stage_ev.push_back(e);
    return fail_hip(hipEventRecord(e, st), "event record");
}

// Launches the admitted jobs `ids` as l (one job alone in the per-request
// mode, as a candidate of its online session when that mode tunes online; a
// mixed launch otherwise).  On failure nothing of l is in flight.
int launch_admitted(ppx_server *s, const std::vector<int64_t> &ids, Launch &l) {
    l.done = take_event(s);
    if (!l.done) return fail(PPX_EHIP, "event creation failed");
    hipStream_t st = s->streams[l.stream];
    const bool single = s->per_request();
    int rc;
    if (single && s->online()) {
        const ppx_job &j = s->jobs[ids[0]].job;
        ppx_online *sess = nullptr;
        if ((rc = online_session(s, j, &sess))) return rc;
        const double elems = double(j.n) * double(j.batch);
        ppx_config cfg{};
        const int r = ppx_online_next(sess, elems >= kOnlineMinElems, &cfg);
        if (r < 0) return r;
        if (r == 1) {  // time this launch: swap in events that record time
            s->free_events.push_back(l.done);
            l.done = nullptr;
            l.session = sess;  // from here on a failure reports the candidate as failed
            l.elems = elems;
            ++s->online_evals;
            if (hipEventCreate(&l.start) != hipSuccess || hipEventCreate(&l.done) != hipSuccess)
                return fail(PPX_EHIP, "event creation failed");
            if ((rc = fail_hip(hipEventRecord(l.start, st), "event record"))) return rc;
        }
        rc = launch_single(j, st, &cfg);
        if (rc == PPX_OK) rc = fail_hip(hipEventRecord(l.done, st), "event record");
    } else if (single) {
        rc = launch_single(s->jobs[ids[0]].job, st, nullptr);
        if (rc == PPX_OK) rc = fail_hip(hipEventRecord(l.done, st), "event record");
    } else {
        std::vector<ppx_job> batch;
        batch.reserve(ids.size());
        for (int64_t id : ids) batch.push_back(s->jobs[id].job);
        std::vector<int> job_stage(ids.size(), -1);
        StageArg sa{s, &l};
        const MixStageHook hook{record_stage, &sa, job_stage.data()};
        rc = launch_mixed_impl(batch.data(), (int)batch.size(), st, l.done, &hook);
        if (rc == PPX_OK) {
            l.stage_ids.resize(l.stage_ev.size());
            for (size_t k = 0; k < ids.size(); ++k) {
                if (job_stage[k] < 0 || job_stage[k] >= (int)l.stage_ids.size())
                    return fail(PPX_EHIP, "mixed launch: a job without a completion stage");
                l.stage_ids[job_stage[k]].push_back(ids[k]);
            }
        }
    }
    return rc;
}

// Retires what has completed, then fills the free launch slots.  In the
// fused mode the pending jobs are spread over the free slots (each launch
// takes its share of them, at least one): at light load, when jobs arrive
// one by one, each goes out alone at once as it would per request, and it
// takes a backlog for launches to batch.
int progress(ppx_server *s, int *launched) {
    if (launched) *launched = 0;
    retire(s);
    while ((int)s->inflight.size() < s->max_inflight && !s->pending.empty()) {
        const bool single = s->per_request();
        const int64_t free_slots = s->max_inflight - (int64_t)s->inflight.size();
        const int64_t share = ((int64_t)s->pending.size() + free_slots - 1) / free_slots;
        const int job_cap = single ? 1 : (int)std::min<int64_t>(kMixLaunchJobs, share);
        std::vector<int64_t> ids = admit(s, kMixLaunchTiles, job_cap);
        if (ids.empty()) break;
        Launch l;
        l.ids = ids;
        l.stream = s->rr++ % (int)std::max<size_t>(1, s->streams.size());
        if (!s->null_device()) {
            if (int rc = launch_admitted(s, ids, l)) {
                unadmit(s, ids, l);
                return rc;
            }
        }
        s->inflight.push_back(l);
        ++s->launches;
        s->max_inflight_seen = std::max(s->max_inflight_seen, (int)s->inflight.size());
        if (launched) *launched += (int)ids.size();
    }
    return PPX_OK;
}

}  // namespace
}  // namespace ppx

using namespace ppx;

extern "C" {

int ppx_server_create(int64_t budget, int max_inflight, int flags, ppx_server **out) {
    if (!out) return fail(PPX_EINVAL, "null output");
    *out = nullptr;
    if (budget < 1) return fail(PPX_EINVAL, "budget must be positive");
    if (max_inflight < 1 || max_inflight > 4) return fail(PPX_EINVAL, "max_inflight must be in 1..4");
    if ((flags & PPX_SERVE_ONLINE_TUNE) && !(flags & PPX_SERVE_PER_REQUEST))
        return fail(PPX_EINVAL, "online tuning applies to the per-request mode (the fused tiles have fixed shapes)");
    auto *s = new ppx_server();
    s->flags = flags;
    s->max_inflight = max_inflight;
    s->budget = budget;
    s->arena.reset(budget);
    if (!s->null_device()) {
        if (!device_info()) {
            delete s;
            return PPX_EDEVICE;
        }
        if (hipMalloc(reinterpret_cast<void **>(&s->arena_base), budget) != hipSuccess) {
            delete s;
            return fail(PPX_ENOMEM, "could not allocate the server's HBM arena");
        }
        s->streams.resize(max_inflight);
        for (auto &st : s->streams)
            if (hipStreamCreate(&st) != hipSuccess) {
                ppx_server_destroy(s);
                return fail(PPX_EHIP, "stream creation failed");
            }
    }
    *out = s;
    return PPX_OK;
}

int ppx_server_destroy(ppx_server *s) {
    if (!s) return PPX_OK;
    if (!s->null_device()) {
        for (auto st : s->streams)
            if (st) (void)hipStreamSynchronize(st);
        for (auto &l : s->inflight) {
            if (l.done) (void)hipEventDestroy(l.done);
            if (l.start) (void)hipEventDestroy(l.start);
        }
        for (auto e : s->free_events) (void)hipEventDestroy(e);
        for (auto st : s->streams)
            if (st) (void)hipStreamDestroy(st);
        if (s->arena_base) (void)hipFree(s->arena_base);
    }
    for (auto &kv : s->sessions) ppx_online_destroy(kv.second);
    delete s;
    return PPX_OK;
}

int ppx_server_submit(ppx_server *s, const ppx_job *job, int64_t *id) {
    if (!s || !job) return fail(PPX_EINVAL, "null argument");
    ppx_job j = *job;
    // validate as the mixed launch would, with a placeholder output if the
    // server is to allocate it
    ppx_job probe = j;
    if (!probe.out) probe.out = reinterpret_cast<void *>(256);
    if (int rc = check_job(probe)) return rc;
    const int64_t fp = job_in_bytes(j) + job_out_bytes(j);
    if (fp > s->budget) return fail(PPX_ENOMEM, "job footprint exceeds the server's HBM budget");
    Job rec;
    rec.id = s->next_id++;
    rec.job = j;
    rec.footprint = fp;
    rec.arrival_us = s->now_us();
    s->jobs[rec.id] = rec;
    s->pending.push_back(rec.id);
    ++s->submitted;
    if (id) *id = rec.id;
    return PPX_OK;
}

int ppx_server_progress(ppx_server *s, int *launched) {
    if (!s) return fail(PPX_EINVAL, "null server");
    return progress(s, launched);
}

int ppx_server_poll(ppx_server *s, ppx_completion *out, int cap, int *count) {
    if (!s) return fail(PPX_EINVAL, "null server");
    int k = 0;
    while (!s->completed.empty() && k < cap && out) {
        const Job &j = s->jobs[s->completed.front()];
        out[k++] = ppx_completion{j.id, j.job.out, j.arrival_us, j.admit_us, j.complete_us};
        s->completed.pop_front();
    }
    if (count) *count = k;
    return PPX_OK;
}

int ppx_server_release(ppx_server *s, int64_t id) {
    if (!s) return fail(PPX_EINVAL, "null server");
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return fail(PPX_EINVAL, "unknown job id");
    if (!it->second.completed) return fail(PPX_EINVAL, "job has not completed");
    s->used -= it->second.footprint;
    if (it->second.arena_off >= 0) s->arena.release(it->second.arena_off, job_out_bytes(it->second.job));
    s->jobs.erase(it);
    ++s->released;
    return PPX_OK;
}

int ppx_server_read(ppx_server *s, int64_t id, void *host_dst, int64_t bytes) {
    if (!s || !host_dst) return fail(PPX_EINVAL, "null argument");
    auto it = s->jobs.find(id);
    if (it == s->jobs.end() || !it->second.completed) return fail(PPX_EINVAL, "no completed job with that id");
    if (bytes < 0 || bytes > job_out_bytes(it->second.job)) return fail(PPX_EINVAL, "bad byte count");
    if (s->null_device()) return fail(PPX_EDEVICE, "null-device server holds no data");
    return fail_hip(hipMemcpy(host_dst, it->second.job.out, bytes, hipMemcpyDeviceToHost), "read");
}

int ppx_server_stats_get(ppx_server *s, ppx_server_stats *o) {
    if (!s || !o) return fail(PPX_EINVAL, "null argument");
    *o = ppx_server_stats{s->submitted, s->admitted, s->ncompleted, s->released, s->launches,
                          s->budget, s->used, s->peak, s->max_inflight_seen, (int32_t)s->pending.size()};
    return PPX_OK;
}

int ppx_server_online_stats(ppx_server *s, int *sessions, int64_t *evaluations, int *converged) {
    if (!s) return fail(PPX_EINVAL, "null server");
    int conv = 0;
    for (auto &kv : s->sessions) {
        int c = 0;
        ppx_online_status(kv.second, nullptr, &c, nullptr, nullptr);
        conv += c;
    }
    if (sessions) *sessions = (int)s->sessions.size();
    if (evaluations) *evaluations = s->online_evals;
    if (converged) *converged = conv;
    return PPX_OK;
}

int ppx_serve_replay(ppx_server *s, const ppx_request *reqs, int n, int auto_release,
                     ppx_completion *out) {
    if (!s || (!reqs && n > 0) || !out) return fail(PPX_EINVAL, "null argument");
    for (int i = 0; i + 1 < n; ++i)
        if (reqs[i + 1].arrival_us < reqs[i].arrival_us) return fail(PPX_EINVAL, "arrivals must be sorted");
    std::unordered_map<int64_t, int> slot;
    const double start = s->now_us();
    int next = 0, done = 0;
    std::vector<ppx_completion> buf(256);
    while (done < n) {
        bool busy = false;
        const double t = s->now_us() - start;
        while (next < n && reqs[next].arrival_us <= t) {
            int64_t id;
            if (int rc = ppx_server_submit(s, &reqs[next].job, &id)) return rc;
            s->jobs[id].arrival_us = start + reqs[next].arrival_us;  // queueing counts
            slot[id] = next++;
            busy = true;
        }
        int launched = 0;
        if (int rc = progress(s, &launched)) return rc;
        int got = 0;
        ppx_server_poll(s, buf.data(), (int)buf.size(), &got);
        for (int k = 0; k < got; ++k) {
            out[slot[buf[k].id]] = buf[k];
            ++done;
            if (auto_release) ppx_server_release(s, buf[k].id);
        }
        if (!busy && launched == 0 && got == 0) std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
    return PPX_OK;
}

}  // extern "C"
