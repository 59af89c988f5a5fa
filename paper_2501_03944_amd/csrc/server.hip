// Serving loop: continuous batching of MGFWA jobs (declarations in include/mgfwa.h).
//
// Every job is an ordinary context (its own workspace, stream, graph) carved
// from one caller-owned device arena.  A tick
//   1. collects generations whose end event has fired (latency = device time
//      between the generation's start and end events on its stream),
//   2. retires jobs that reached their budget or raised the stop flag (the
//      best is copied to the host, the context destroyed, the memory freed),
//   3. admits queued jobs in arrival order wherever they fit (first fit,
//      later small jobs may pass a large one that does not fit yet),
//   4. enqueues one more generation of every running job that has fewer than
//      two generations in flight.
// Jobs on different streams overlap on the device; the kernels of a job do not
// depend on anything outside its workspace, so its state is the same alone and
// in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "../../include/mgfwa.h"
#include "internal.h"

using mgfwa::fail;

namespace {

constexpr int MAX_INFLIGHT = 2;
constexpr size_t ARENA_ALIGN = 256;

struct Inflight {
    hipEvent_t start, end;
    int32_t *ctrl_host;   // pinned copy of the job's control words after this generation
};

struct Job {
    int64_t id = 0;
    mgfwa_config cfg{};
    mgfwa_problem prob{};
    size_t bytes = 0, off = 0;
    int state = MGFWA_JOB_QUEUED;
    mgfwa_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    int D = 0, C = 0, budget = 0;
    int enqueued = 0, completed = 0;
    bool stopping = false;
    hipEvent_t inputs_read = nullptr;   // recorded after the initialisation (input packing)
    bool released = false;              // the caller's problem buffers are no longer read
    float best = 0.0f;
    std::vector<float> best_x;
    double t_submit = 0, t_admit = 0, t_finish = 0;
    std::deque<Inflight> inflight;
};

}  // namespace

struct mgfwa_server {
    char *arena = nullptr;
    size_t arena_bytes = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_blocks;       // offset -> size
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    std::vector<Job *> jobs;                    // by id
    std::deque<int64_t> queue;
    std::vector<double> lat;
    long generations = 0;
    double evals = 0.0;
    std::chrono::steady_clock::time_point t0;
    std::vector<hipEvent_t> event_pool;
    std::vector<int32_t *> pinned_pool;

    double now_ms() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

bool arena_alloc(mgfwa_server *s, size_t bytes, size_t *off)
{
    for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t roff = it->first + bytes;
            s->free_blocks.erase(it);
            if (rest) s->free_blocks[roff] = rest;
            s->used += bytes;
            s->peak = std::max(s->peak, s->used);
            return true;
        }
    }
    return false;
}

void arena_free(mgfwa_server *s, size_t off, size_t bytes)
{
    auto it = s->free_blocks.emplace(off, bytes).first;
    // merge with the next and the previous block
    auto nx = std::next(it);
    if (nx != s->free_blocks.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        s->free_blocks.erase(nx);
    }
    if (it != s->free_blocks.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            s->free_blocks.erase(it);
        }
    }
    s->used -= bytes;
}

hipError_t take_event(mgfwa_server *s, hipEvent_t *e)
{
    if (!s->event_pool.empty()) {
        *e = s->event_pool.back();
        s->event_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

hipError_t take_pinned(mgfwa_server *s, int32_t **p)
{
    if (!s->pinned_pool.empty()) {
        *p = s->pinned_pool.back();
        s->pinned_pool.pop_back();
        return hipSuccess;
    }
    return hipHostMalloc(reinterpret_cast<void **>(p), 4 * sizeof(int32_t), hipHostMallocDefault);
}

void give_back(mgfwa_server *s, Inflight &f)
{
    s->event_pool.push_back(f.start);
    s->event_pool.push_back(f.end);
    s->pinned_pool.push_back(f.ctrl_host);
}

// Collect the finished generations of a running job (non-blocking).
mgfwa_status collect(mgfwa_server *s, Job *j)
{
    while (!j->inflight.empty()) {
        Inflight &f = j->inflight.front();
        const hipError_t q = hipEventQuery(f.end);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return fail(MGFWA_EHIP, "job %lld: %s", (long long)j->id, hipGetErrorString(q));
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, f.start, f.end) == hipSuccess) s->lat.push_back(ms);
        const bool done_flag = f.ctrl_host[1] != 0;
        if (!done_flag || !j->stopping) {
            j->completed += 1;
            s->generations += 1;
            s->evals += j->C;
        }
        if (done_flag) j->stopping = true;
        give_back(s, f);
        j->inflight.pop_front();
    }
    if (j->completed >= j->budget) j->stopping = true;
    return MGFWA_OK;
}

mgfwa_status retire(mgfwa_server *s, Job *j)
{
    std::vector<float> bx((size_t)j->cfg.n_populations * j->D), bf(j->cfg.n_populations);
    mgfwa_status r = mgfwa_best_all(j->ctx, bx.data(), bf.data(), nullptr);
    if (r == MGFWA_OK) {
        int pb = 0;
        for (int b = 1; b < j->cfg.n_populations; ++b)
            if (bf[b] < bf[pb]) pb = b;
        j->best = bf[pb];
        j->best_x.assign(bx.begin() + (size_t)pb * j->D, bx.begin() + (size_t)(pb + 1) * j->D);
    }
    mgfwa_destroy(j->ctx);
    j->ctx = nullptr;
    if (j->inputs_read) {
        s->event_pool.push_back(j->inputs_read);
        j->inputs_read = nullptr;
    }
    j->released = true;
    arena_free(s, j->off, j->bytes);
    j->state = r == MGFWA_OK ? MGFWA_JOB_DONE : MGFWA_JOB_FAILED;
    j->t_finish = s->now_ms();
    return MGFWA_OK;
}

mgfwa_status admit(mgfwa_server *s, Job *j)
{
    size_t off = 0;
    if (!arena_alloc(s, j->bytes, &off)) return MGFWA_ENOMEM;
    j->off = off;
    j->stream = s->streams[s->next_stream];
    s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
    mgfwa_status r = mgfwa_init(&j->ctx, &j->cfg, &j->prob, s->arena + off, j->bytes, j->stream);
    j->t_admit = s->now_ms();
    if (r != MGFWA_OK) {
        arena_free(s, off, j->bytes);
        j->state = MGFWA_JOB_FAILED;
        j->t_finish = j->t_admit;
        return MGFWA_OK;   // the job failed; the server carries on
    }
    // the caller may release the problem buffers once the initialisation, which
    // packs them into the workspace, has run on the device
    hipError_t e = take_event(s, &j->inputs_read);
    if (e == hipSuccess) e = hipEventRecord(j->inputs_read, j->stream);
    if (e != hipSuccess) return fail(MGFWA_EHIP, "admit: %s", hipGetErrorString(e));
    mgfwa_state_info info;
    mgfwa_state(j->ctx, &info);
    j->D = info.D;
    j->C = j->cfg.n_populations * j->cfg.n_fireworks * info.n_candidates;
    j->state = MGFWA_JOB_RUNNING;
    return MGFWA_OK;
}

// Whether the job no longer reads the caller's problem buffers (non-blocking).
bool inputs_released(const Job *j)
{
    if (j->released) return true;
    if (j->state != MGFWA_JOB_RUNNING) return false;   // queued: not read yet
    return hipEventQuery(j->inputs_read) == hipSuccess;
}

mgfwa_status enqueue(mgfwa_server *s, Job *j)
{
    Inflight f{};
    hipError_t e = take_event(s, &f.start);
    if (e == hipSuccess) e = take_event(s, &f.end);
    if (e == hipSuccess) e = take_pinned(s, &f.ctrl_host);
    if (e != hipSuccess) return fail(MGFWA_EHIP, "server resources: %s", hipGetErrorString(e));
    mgfwa_state_info info;
    mgfwa_state(j->ctx, &info);
    e = hipEventRecord(f.start, j->stream);
    if (e != hipSuccess) return fail(MGFWA_EHIP, "event: %s", hipGetErrorString(e));
    mgfwa_status r = mgfwa_step(j->ctx, 1);
    if (r != MGFWA_OK) return r;
    // the control words follow the generation so the host can see the stop flag
    const char *base = reinterpret_cast<const char *>(s->arena + j->off);
    e = hipMemcpyAsync(f.ctrl_host, base + info.gen, 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                       j->stream);
    if (e == hipSuccess) e = hipEventRecord(f.end, j->stream);
    if (e != hipSuccess) return fail(MGFWA_EHIP, "enqueue: %s", hipGetErrorString(e));
    j->inflight.push_back(f);
    j->enqueued += 1;
    return MGFWA_OK;
}

}  // namespace

extern "C" {

mgfwa_status mgfwa_server_create(mgfwa_server **out, void *arena_dev, size_t arena_bytes,
                                 int n_streams)
{
    if (!out) return fail(MGFWA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!arena_dev || arena_bytes < ARENA_ALIGN) return fail(MGFWA_ENOMEM, "empty arena");
    if (reinterpret_cast<uintptr_t>(arena_dev) % ARENA_ALIGN)
        return fail(MGFWA_ENOMEM, "arena must be %zu-byte aligned", ARENA_ALIGN);
    if (n_streams < 1 || n_streams > 64) return fail(MGFWA_EINVAL, "n_streams must be in [1, 64]");
    mgfwa_server *s = new mgfwa_server();
    s->arena = static_cast<char *>(arena_dev);
    s->arena_bytes = arena_bytes / ARENA_ALIGN * ARENA_ALIGN;
    s->free_blocks[0] = s->arena_bytes;
    s->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < n_streams; ++i) {
        hipStream_t st = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            mgfwa_server_destroy(s);
            return fail(MGFWA_EHIP, "stream: %s", hipGetErrorString(e));
        }
        s->streams.push_back(st);
    }
    *out = s;
    return MGFWA_OK;
}

mgfwa_status mgfwa_server_submit(mgfwa_server *s, const mgfwa_config *config,
                                 const mgfwa_problem *problem, int64_t *job_id)
{
    if (!s || !config || !problem || !job_id) return fail(MGFWA_EINVAL, "NULL argument");
    if (config->external_fitness) return fail(MGFWA_EINVAL, "served jobs use the built-in fitness");
    const size_t need = mgfwa_workspace_bytes(config, problem);
    if (need == 0) return fail(MGFWA_EINVAL, "invalid job: %s", mgfwa_last_error());
    const size_t bytes = (need + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
    if (bytes > s->arena_bytes)
        return fail(MGFWA_ENOMEM, "job needs %zu bytes, arena has %zu", bytes, s->arena_bytes);
    Job *j = new Job();
    j->id = (int64_t)s->jobs.size();
    j->cfg = *config;
    j->prob = *problem;
    j->bytes = bytes;
    j->budget = config->max_generations;
    j->t_submit = s->now_ms();
    s->jobs.push_back(j);
    s->queue.push_back(j->id);
    *job_id = j->id;
    return MGFWA_OK;
}

mgfwa_status mgfwa_server_tick(mgfwa_server *s)
{
    if (!s) return fail(MGFWA_EINVAL, "NULL server");
    // 1-2: collect finished generations, retire finished jobs
    for (Job *j : s->jobs) {
        if (j->state != MGFWA_JOB_RUNNING) continue;
        if (!j->released) j->released = inputs_released(j);
        mgfwa_status r = collect(s, j);
        if (r) return r;
        if (j->stopping && j->inflight.empty()) {
            r = retire(s, j);
            if (r) return r;
        }
    }
    // 3: admit in arrival order wherever the workspace fits
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Job *j = s->jobs[*it];
        if (admit(s, j) == MGFWA_ENOMEM) {
            ++it;
            continue;
        }
        it = s->queue.erase(it);
    }
    // 4: one more generation of every running job with room in its pipeline
    for (Job *j : s->jobs) {
        if (j->state != MGFWA_JOB_RUNNING || j->stopping) continue;
        if ((int)j->inflight.size() >= MAX_INFLIGHT || j->enqueued >= j->budget) continue;
        mgfwa_status r = enqueue(s, j);
        if (r) return r;
    }
    return MGFWA_OK;
}

mgfwa_status mgfwa_server_drain(mgfwa_server *s)
{
    if (!s) return fail(MGFWA_EINVAL, "NULL server");
    for (;;) {
        mgfwa_status r = mgfwa_server_tick(s);
        if (r) return r;
        bool busy = !s->queue.empty();
        Job *oldest = nullptr;
        for (Job *j : s->jobs) {
            if (j->state == MGFWA_JOB_RUNNING) {
                busy = true;
                if (!j->inflight.empty() && !oldest) oldest = j;
            }
        }
        if (!busy) return MGFWA_OK;
        if (oldest) {
            hipError_t e = hipEventSynchronize(oldest->inflight.front().end);
            if (e != hipSuccess) return fail(MGFWA_EHIP, "drain: %s", hipGetErrorString(e));
        } else if (!s->queue.empty()) {
            bool any_running = false;
            for (Job *j : s->jobs) any_running |= j->state == MGFWA_JOB_RUNNING;
            if (!any_running)   // nothing running and nothing admissible: cannot progress
                return fail(MGFWA_ENOMEM, "queued jobs do not fit the free arena");
        }
    }
}

mgfwa_status mgfwa_server_job(mgfwa_server *s, int64_t id, mgfwa_job_info *info, float *x_host)
{
    if (!s || id < 0 || id >= (int64_t)s->jobs.size()) return fail(MGFWA_EINVAL, "unknown job");
    Job *j = s->jobs[id];
    if (j->state == MGFWA_JOB_RUNNING && !j->released) j->released = inputs_released(j);
    if (info) {
        // a running job whose initialisation has not yet read the caller's
        // problem buffers still reports QUEUED
        info->state = j->state == MGFWA_JOB_RUNNING && !j->released ? MGFWA_JOB_QUEUED : j->state;
        info->generations = j->completed;
        info->best_fitness = j->best;
        info->workspace_bytes = j->bytes;
        info->submit_ms = j->t_submit;
        info->admit_ms = j->t_admit;
        info->finish_ms = j->t_finish;
    }
    if (x_host && j->state == MGFWA_JOB_DONE && !j->best_x.empty())
        std::memcpy(x_host, j->best_x.data(), j->best_x.size() * sizeof(float));
    return MGFWA_OK;
}

mgfwa_status mgfwa_server_stats_get(mgfwa_server *s, mgfwa_server_stats *st)
{
    if (!s || !st) return fail(MGFWA_EINVAL, "NULL argument");
    std::memset(st, 0, sizeof *st);
    for (const Job *j : s->jobs) {
        st->queued += j->state == MGFWA_JOB_QUEUED;
        st->running += j->state == MGFWA_JOB_RUNNING;
        st->done += j->state == MGFWA_JOB_DONE;
        st->failed += j->state == MGFWA_JOB_FAILED;
    }
    st->generations = s->generations;
    if (!s->lat.empty()) {
        std::vector<double> v = s->lat;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            size_t i = (size_t)(q * v.size());
            return v[std::min(i, v.size() - 1)];
        };
        st->gen_ms_p50 = pct(0.50);
        st->gen_ms_p99 = pct(0.99);
    }
    st->wall_ms = s->now_ms();
    st->spark_evals_per_s = st->wall_ms > 0 ? s->evals / (st->wall_ms / 1e3) : 0.0;
    st->arena_bytes = s->arena_bytes;
    st->arena_used = s->used;
    st->arena_peak = s->peak;
    return MGFWA_OK;
}

void mgfwa_server_destroy(mgfwa_server *s)
{
    if (!s) return;
    for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
    for (Job *j : s->jobs) {
        for (Inflight &f : j->inflight) give_back(s, f);
        if (j->inputs_read) s->event_pool.push_back(j->inputs_read);
        if (j->ctx) mgfwa_destroy(j->ctx);
        delete j;
    }
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (int32_t *p : s->pinned_pool) (void)hipHostFree(p);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
}

}  // extern "C"
