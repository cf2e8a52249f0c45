// Extraction request server: continuous batching of independent volumes on
// one GPU.
//
// Requests arrive one at a time (sift3d_server_submit). A scheduler thread
// admits them in arrival order as soon as two resources allow it:
//   - an in-flight slot (at most max_inflight requests on the device), and
//   - device memory: each request needs a slot of its shape, i.e. the
//     workspace of its pyramid plus its keypoint and descriptor buffers.
//     Slots are cached per shape; a new one is allocated while the total
//     stays within hbm_budget, after evicting idle slots of other shapes if
//     needed.
// Admitted requests are spread over n_streams streams, so the kernels of
// different requests run side by side: the small late octaves and the
// descriptor gathers of one request fill the device while another request
// streams its first octave. Completion is detected by polling an event per
// request; the keypoint count travels back with the event in pinned host
// memory. A slot stays with its request (its outputs live there) until the
// client releases the ticket.
//
// Every request runs exactly the kernels of sift3d_extract on its own
// workspace, so its result does not depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sift3d.h"

namespace {

using Shape = std::array<int, 3>;

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Slot {
    Shape shape;
    sift3d_plan *plan;      // shared per shape, owned by the server
    char *mem;              // one device allocation
    size_t bytes;
    void *ws;
    size_t ws_bytes;
    sift3d_keypoint *kp;
    int *count;
    uint8_t *sr;
    uint64_t *br;
    uint8_t *rr;
    int *h_count;           // pinned host copy of *count
    double last_use;
};

struct Request {
    int64_t id;
    const float *vol;
    Shape shape;
    sift3d_plan *plan;
    size_t footprint;
    int state;              // 0 pending, 1 on the device, 2 done, 3 failed
    int rc;
    int hip_error;
    Slot *slot;
    int stream;
    hipEvent_t ev;
    int count;
    double t_submit, t_start, t_done;
};

enum { kPending = 0, kRunning = 1, kDone = 2, kFailed = 3 };

}  // namespace

struct sift3d_server {
    sift3d_ctx *ctx;
    sift3d_server_config cfg;
    int device;
    int brief_n;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;

    // shared with client threads (guarded by mu)
    std::mutex mu;
    std::condition_variable cv_work;   // scheduler: new request or stop
    std::condition_variable cv_done;   // clients: a request finished
    std::deque<Request *> pending;
    std::unordered_map<int64_t, Request *> reqs;
    std::vector<Slot *> to_release;    // released by clients, returned to the pool by the scheduler
    std::map<Shape, sift3d_plan *> plans;
    int64_t next_id = 1;
    bool stop = false;
    sift3d_server_counters stats{};

    // scheduler-only state
    std::vector<Request *> running;
    std::map<Shape, std::vector<Slot *>> idle;
    std::vector<hipEvent_t> free_events;
    size_t allocated = 0;

    std::thread thread;
};

namespace {

size_t outputs_bytes(int cap, int brief_n)
{
    return align256((size_t)cap * sizeof(sift3d_keypoint)) + align256(sizeof(int)) + align256((size_t)cap * 64) +
           align256((size_t)cap * (brief_n / 8)) + align256((size_t)cap * brief_n);
}

// Device bytes of a slot for `plan`.
size_t slot_bytes(const sift3d_server *sv, const sift3d_plan *plan)
{
    size_t ws = 0;
    sift3d_plan_info(plan, &ws, nullptr, nullptr);
    return align256(ws) + outputs_bytes(sv->cfg.kp_capacity, sv->brief_n);
}

void free_slot(sift3d_server *sv, Slot *s)
{
    (void)hipFree(s->mem);
    (void)hipHostFree(s->h_count);
    sv->allocated -= s->bytes;
    delete s;
}

Slot *new_slot(sift3d_server *sv, const Shape &shape, sift3d_plan *plan, size_t bytes)
{
    Slot *s = new (std::nothrow) Slot();
    if (s == nullptr) return nullptr;
    s->shape = shape;
    s->plan = plan;
    s->bytes = bytes;
    if (hipMalloc((void **)&s->mem, bytes) != hipSuccess) {
        delete s;
        return nullptr;
    }
    if (hipHostMalloc((void **)&s->h_count, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(s->mem);
        delete s;
        return nullptr;
    }
    const int cap = sv->cfg.kp_capacity, n = sv->brief_n;
    sift3d_plan_info(plan, &s->ws_bytes, nullptr, nullptr);
    char *p = s->mem;
    s->ws = p;
    p += align256(s->ws_bytes);
    s->kp = reinterpret_cast<sift3d_keypoint *>(p);
    p += align256((size_t)cap * sizeof(sift3d_keypoint));
    s->count = reinterpret_cast<int *>(p);
    p += align256(sizeof(int));
    s->sr = reinterpret_cast<uint8_t *>(p);
    p += align256((size_t)cap * 64);
    s->br = n > 0 ? reinterpret_cast<uint64_t *>(p) : nullptr;
    p += align256((size_t)cap * (n / 8));
    s->rr = n > 0 ? reinterpret_cast<uint8_t *>(p) : nullptr;
    sv->allocated += bytes;
    ++sv->stats.slot_allocations;
    if (sv->allocated > sv->stats.peak_allocated) sv->stats.peak_allocated = sv->allocated;
    return s;
}

// A slot for request r: an idle one of its shape, a new one within the
// budget, or a new one after evicting idle slots of other shapes (oldest
// first). nullptr: wait for a running request to be released.
Slot *acquire_slot(sift3d_server *sv, Request *r)
{
    auto it = sv->idle.find(r->shape);
    if (it != sv->idle.end() && !it->second.empty()) {
        Slot *s = it->second.back();
        it->second.pop_back();
        return s;
    }
    const size_t budget = sv->cfg.hbm_budget;
    while (sv->allocated + r->footprint > budget) {
        Slot *oldest = nullptr;
        std::vector<Slot *> *from = nullptr;
        for (auto &kv : sv->idle)
            for (Slot *s : kv.second)
                if (oldest == nullptr || s->last_use < oldest->last_use) oldest = s, from = &kv.second;
        if (oldest == nullptr) return nullptr;
        for (size_t i = 0; i < from->size(); ++i)
            if ((*from)[i] == oldest) {
                from->erase(from->begin() + (long)i);
                break;
            }
        free_slot(sv, oldest);
        ++sv->stats.slot_evictions;
    }
    return new_slot(sv, r->shape, r->plan, r->footprint);
}

void start_request(sift3d_server *sv, Request *r, Slot *s)
{
    int best = 0;
    for (int i = 1; i < (int)sv->streams.size(); ++i)
        if (sv->stream_load[i] < sv->stream_load[best]) best = i;
    hipStream_t st = sv->streams[best];
    r->slot = s;
    r->stream = best;
    r->t_start = now_s();
    if (sv->free_events.empty()) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            r->rc = SIFT3D_E_HIP;
            r->hip_error = (int)hipGetLastError();
            r->state = kFailed;
            return;
        }
        sv->free_events.push_back(ev);
    }
    r->ev = sv->free_events.back();
    sv->free_events.pop_back();
    int rc = sift3d_extract(r->plan, r->vol, s->ws, s->ws_bytes, s->kp, sv->cfg.kp_capacity, s->count, s->sr,
                            s->br, s->rr, st);
    hipError_t e = hipSuccess;
    if (rc == SIFT3D_OK) {
        e = hipMemcpyAsync(s->h_count, s->count, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(r->ev, st);
        if (e != hipSuccess) rc = SIFT3D_E_HIP;
    } else {
        e = (hipError_t)sift3d_last_hip_error();
    }
    if (rc != SIFT3D_OK) {
        r->rc = rc;
        r->hip_error = (int)e;
        r->state = kFailed;
        sv->free_events.push_back(r->ev);
        r->ev = nullptr;
        return;
    }
    r->state = kRunning;
    ++sv->stream_load[best];
}

void scheduler(sift3d_server *sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        // released slots go back to the idle pool
        for (Slot *s : sv->to_release) {
            s->last_use = now_s();
            sv->idle[s->shape].push_back(s);
        }
        sv->to_release.clear();

        // completions
        bool finished = false;
        for (size_t i = 0; i < sv->running.size();) {
            Request *r = sv->running[i];
            const hipError_t q = hipEventQuery(r->ev);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            r->t_done = now_s();
            if (q == hipSuccess) {
                r->count = *r->slot->h_count;
                r->state = kDone;
                ++sv->stats.completed;
            } else {
                r->rc = SIFT3D_E_HIP;
                r->hip_error = (int)q;
                r->state = kFailed;
                ++sv->stats.failed;
            }
            --sv->stream_load[r->stream];
            sv->free_events.push_back(r->ev);
            r->ev = nullptr;
            sv->running[i] = sv->running.back();
            sv->running.pop_back();
            finished = true;
        }

        // admissions, in arrival order
        while (!sv->pending.empty() && (int)sv->running.size() < sv->cfg.max_inflight) {
            Request *r = sv->pending.front();
            Slot *s = acquire_slot(sv, r);
            if (s == nullptr) break;  // memory frees up when a held slot is released
            sv->pending.pop_front();
            start_request(sv, r, s);
            if (r->state == kRunning) {
                sv->running.push_back(r);
            } else {
                // launch failure: the slot goes back to the pool
                s->last_use = now_s();
                sv->idle[s->shape].push_back(s);
                r->slot = nullptr;
                r->t_done = now_s();
                ++sv->stats.failed;
                finished = true;
            }
        }
        sv->stats.in_flight = (int)sv->running.size();
        sv->stats.pending = (int)sv->pending.size();
        sv->stats.allocated = sv->allocated;
        if (finished) sv->cv_done.notify_all();

        if (sv->stop) {
            // requests not yet admitted are cancelled; those on the device finish
            for (Request *r : sv->pending) {
                r->rc = SIFT3D_E_ARG;
                r->state = kFailed;
                r->t_done = now_s();
                ++sv->stats.failed;
            }
            if (!sv->pending.empty()) sv->cv_done.notify_all();
            sv->pending.clear();
            if (sv->running.empty()) break;
        }
        if (sv->running.empty()) {
            sv->cv_work.wait(lk);
        } else {
            // poll the device; new submissions and releases wake us early
            sv->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

extern "C" {

int sift3d_server_create(sift3d_ctx *ctx, const sift3d_server_config *cfg, sift3d_server **out)
{
    if (out == nullptr) return SIFT3D_E_ARG;
    *out = nullptr;
    if (ctx == nullptr || cfg == nullptr) return SIFT3D_E_ARG;
    if (cfg->n_streams < 1 || cfg->n_streams > 8 || cfg->max_inflight < 1 || cfg->max_inflight > 256 ||
        cfg->kp_capacity < 1 || cfg->hbm_budget == 0)
        return SIFT3D_E_ARG;
    sift3d_params p;
    sift3d_ctx_params(ctx, &p);
    sift3d_server *sv = new (std::nothrow) sift3d_server();
    if (sv == nullptr) return SIFT3D_E_ARG;
    sv->ctx = ctx;
    sv->cfg = *cfg;
    sv->brief_n = p.brief_n;
    if (hipGetDevice(&sv->device) != hipSuccess) {
        delete sv;
        return SIFT3D_E_HIP;
    }
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
            delete sv;
            return SIFT3D_E_HIP;
        }
        sv->streams.push_back(st);
        sv->stream_load.push_back(0);
    }
    sv->stats.hbm_budget = cfg->hbm_budget;
    sv->thread = std::thread(scheduler, sv);
    *out = sv;
    return SIFT3D_OK;
}

int sift3d_server_footprint(sift3d_server *sv, int nx, int ny, int nz, size_t *bytes)
{
    if (sv == nullptr || bytes == nullptr) return SIFT3D_E_ARG;
    if (nx < 1 || ny < 1 || nz < 1) return SIFT3D_E_ARG;
    int rc = SIFT3D_OK;
    std::lock_guard<std::mutex> lk(sv->mu);
    const Shape shape{nx, ny, nz};
    auto it = sv->plans.find(shape);
    sift3d_plan *plan = nullptr;
    if (it == sv->plans.end()) {
        rc = sift3d_plan_create(sv->ctx, nx, ny, nz, sv->cfg.kp_capacity, &plan);
        if (rc != SIFT3D_OK) return rc;
        sv->plans[shape] = plan;
    } else {
        plan = it->second;
    }
    *bytes = slot_bytes(sv, plan);
    return SIFT3D_OK;
}

int sift3d_server_submit(sift3d_server *sv, const float *d_vol, int nx, int ny, int nz, int64_t *ticket)
{
    if (sv == nullptr || d_vol == nullptr || ticket == nullptr) return SIFT3D_E_ARG;
    size_t fp = 0;
    int rc = sift3d_server_footprint(sv, nx, ny, nz, &fp);
    if (rc != SIFT3D_OK) return rc;
    if (fp > sv->cfg.hbm_budget) return SIFT3D_E_WORKSPACE;
    Request *r = new (std::nothrow) Request();
    if (r == nullptr) return SIFT3D_E_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) {
            delete r;
            return SIFT3D_E_ARG;
        }
        r->id = sv->next_id++;
        r->vol = d_vol;
        r->shape = Shape{nx, ny, nz};
        r->plan = sv->plans[r->shape];
        r->footprint = fp;
        r->state = kPending;
        r->rc = SIFT3D_OK;
        r->t_submit = now_s();
        sv->reqs[r->id] = r;
        sv->pending.push_back(r);
        ++sv->stats.submitted;
        *ticket = r->id;
    }
    sv->cv_work.notify_one();
    return SIFT3D_OK;
}

int sift3d_server_result(sift3d_server *sv, int64_t ticket, int wait, sift3d_result *out)
{
    if (sv == nullptr || out == nullptr) return SIFT3D_E_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return SIFT3D_E_ARG;
    Request *r = it->second;
    if (wait)
        sv->cv_done.wait(lk, [r] { return r->state == kDone || r->state == kFailed; });
    else if (r->state != kDone && r->state != kFailed)
        return SIFT3D_PENDING;
    out->status = r->state == kDone ? SIFT3D_OK : r->rc;
    out->hip_error = r->hip_error;
    out->count = r->count;
    out->capacity = sv->cfg.kp_capacity;
    const Slot *s = r->state == kDone ? r->slot : nullptr;
    out->d_kp = s ? s->kp : nullptr;
    out->d_siftrank = s ? s->sr : nullptr;
    out->d_brief = s ? s->br : nullptr;
    out->d_rrief = s ? s->rr : nullptr;
    out->stream = r->stream;
    out->t_submit = r->t_submit;
    out->t_start = r->t_start;
    out->t_done = r->t_done;
    return SIFT3D_OK;
}

int sift3d_server_fetch(sift3d_server *sv, int64_t ticket, sift3d_keypoint *h_kp, uint8_t *h_siftrank,
                        uint64_t *h_brief, uint8_t *h_rrief)
{
    if (sv == nullptr) return SIFT3D_E_ARG;
    Slot *s = nullptr;
    int rows = 0, stream = 0;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end() || it->second->state != kDone) return SIFT3D_E_ARG;
        s = it->second->slot;
        rows = std::min(it->second->count, sv->cfg.kp_capacity);
        stream = it->second->stream;
    }
    // the slot cannot be reused before the client releases this ticket
    hipStream_t st = sv->streams[stream];
    const size_t n = (size_t)rows, bn = (size_t)sv->brief_n;
    hipError_t e = hipSuccess;
    if (h_kp && n) e = hipMemcpyAsync(h_kp, s->kp, n * sizeof(sift3d_keypoint), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && h_siftrank && n) e = hipMemcpyAsync(h_siftrank, s->sr, n * 64, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && h_brief && n && bn) e = hipMemcpyAsync(h_brief, s->br, n * bn / 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && h_rrief && n && bn) e = hipMemcpyAsync(h_rrief, s->rr, n * bn, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? SIFT3D_OK : SIFT3D_E_HIP;
}

int sift3d_server_release(sift3d_server *sv, int64_t ticket)
{
    if (sv == nullptr) return SIFT3D_E_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end()) return SIFT3D_E_ARG;
        Request *r = it->second;
        if (r->state != kDone && r->state != kFailed) return SIFT3D_E_ARG;
        if (r->slot != nullptr) sv->to_release.push_back(r->slot);
        sv->reqs.erase(it);
        delete r;
    }
    sv->cv_work.notify_one();
    return SIFT3D_OK;
}

int sift3d_server_stats(sift3d_server *sv, sift3d_server_counters *out)
{
    if (sv == nullptr || out == nullptr) return SIFT3D_E_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    return SIFT3D_OK;
}

double sift3d_server_clock(void) { return now_s(); }

int sift3d_server_destroy(sift3d_server *sv)
{
    if (sv == nullptr) return SIFT3D_E_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_one();
    sv->thread.join();
    for (hipStream_t st : sv->streams) (void)hipStreamSynchronize(st);
    for (auto &kv : sv->reqs) {
        if (kv.second->slot != nullptr) free_slot(sv, kv.second->slot);
        delete kv.second;
    }
    for (Slot *s : sv->to_release) free_slot(sv, s);
    for (auto &kv : sv->idle)
        for (Slot *s : kv.second) free_slot(sv, s);
    for (hipEvent_t ev : sv->free_events) (void)hipEventDestroy(ev);
    for (hipStream_t st : sv->streams) (void)hipStreamDestroy(st);
    for (auto &kv : sv->plans) sift3d_plan_destroy(kv.second);
    delete sv;
    return SIFT3D_OK;
}

}  // extern "C"
