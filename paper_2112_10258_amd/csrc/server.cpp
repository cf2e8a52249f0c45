// Extraction request server: continuous batching of independent volumes on
// one GPU.
//
// Requests arrive one at a time (sift3d_server_submit). A scheduler thread
// admits them in arrival order. When the request at the head of the queue
// is admitted, up to max_batch - 1 later requests of the same shape that are
// already waiting join it (the group size is rounded down to a power of
// two); the group runs as one batch extraction, so each pyramid, detection
// and descriptor launch covers all of its volumes. A group is admitted as
// soon as two resources allow it:
//   - an in-flight slot (at most max_inflight groups on the device), and
//   - device memory: the group needs a batch slot of its (shape, size), i.e.
//     the packed input, the workspace of the batch plan and the keypoint and
//     descriptor buffers of its requests. Batch slots are cached per (shape,
//     size); a new one is allocated while the total stays within hbm_budget,
//     after evicting idle slots of other kinds if needed, and a group that
//     does not fit is shrunk before it waits.
// Groups are spread over n_streams streams, so the kernels of different
// groups run side by side. Completion is detected by polling an event per
// group; the keypoint counts travel back with it in pinned host memory. A
// batch slot stays with its group (the results live there) until the client
// has released every ticket of the group.
//
// A batch plan gives each volume exactly the results of a one-volume plan
// (same kernels, same arithmetic), so a request's result does not depend on
// what it was grouped with or what else is in flight.
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
#include <utility>
#include <vector>

#include "sift3d.h"

namespace {

using Shape = std::array<int, 3>;
using Kind = std::pair<Shape, int>;   // (shape, volumes per batch)

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// A device allocation for one group of n requests of one shape.
struct Slot {
    Kind kind;
    sift3d_plan *plan;      // the (shape, n) batch plan, owned by the server's plan cache
    char *mem;              // one device allocation
    size_t bytes;
    float *in;              // packed input: volume i at in_off[i]
    std::vector<size_t> in_off;
    size_t vol_bytes;
    void *ws;
    size_t ws_bytes;
    sift3d_keypoint *kp;    // [n][cap]
    int *count;             // [n]
    uint8_t *sr;            // [n][cap][64]
    uint64_t *br;           // [n][cap][brief_n/64]
    uint8_t *rr;            // [n][cap][brief_n]
    int *h_count;           // pinned host copy of count
    int holders;            // requests of the group not yet released
    double last_use;
};

struct Request {
    int64_t id;
    const float *vol;
    Shape shape;
    size_t footprint;       // bytes of a lone slot of its shape
    int state;              // 0 pending, 1 on the device, 2 done, 3 failed
    int rc;
    int hip_error;
    Slot *slot;
    int index;              // volume index within the slot
    int stream;
    int count;
    double t_submit, t_start, t_done;
};

// A group on the device.
struct Group {
    Slot *slot;
    std::vector<Request *> reqs;
    int stream;
    hipEvent_t ev;
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
    std::condition_variable cv_work;   // scheduler: new request, release or stop
    std::condition_variable cv_done;   // clients: a request finished
    std::deque<Request *> pending;
    std::unordered_map<int64_t, Request *> reqs;
    std::vector<Slot *> to_release;    // slots whose group is fully released
    std::map<Kind, sift3d_plan *> plans;
    int64_t next_id = 1;
    bool stop = false;
    sift3d_server_counters stats{};

    // scheduler-only state
    std::vector<Group> running;
    std::map<Kind, std::vector<Slot *>> idle;
    std::vector<hipEvent_t> free_events;
    size_t allocated = 0;
    size_t idle_bytes = 0;             // part of `allocated` in idle (evictable) slots

    std::thread thread;
};

namespace {

size_t outputs_bytes(int cap, int brief_n)
{
    return align256((size_t)cap * sizeof(sift3d_keypoint)) + align256((size_t)cap * 64) +
           align256((size_t)cap * (brief_n / 8)) + align256((size_t)cap * brief_n);
}

// The (shape, n) batch plan, created on first use. Caller holds mu.
int get_plan(sift3d_server *sv, const Kind &k, sift3d_plan **out)
{
    auto it = sv->plans.find(k);
    if (it != sv->plans.end()) {
        *out = it->second;
        return SIFT3D_OK;
    }
    std::vector<int> dims;
    for (int i = 0; i < k.second; ++i) dims.insert(dims.end(), k.first.begin(), k.first.end());
    sift3d_plan *p = nullptr;
    const int rc = sift3d_plan_create_batch(sv->ctx, k.second, dims.data(), sv->cfg.kp_capacity, &p);
    if (rc != SIFT3D_OK) return rc;
    sv->plans[k] = p;
    *out = p;
    return SIFT3D_OK;
}

// Device bytes of a slot for `plan` (n volumes).
size_t slot_bytes(const sift3d_server *sv, const sift3d_plan *plan, int n)
{
    size_t ws = 0, in_elems = 0;
    sift3d_plan_info(plan, &ws, nullptr, &in_elems);
    return align256(ws) + align256(in_elems * sizeof(float)) + align256((size_t)n * sizeof(int)) +
           (size_t)n * outputs_bytes(sv->cfg.kp_capacity, sv->brief_n);
}

void free_slot(sift3d_server *sv, Slot *s)
{
    (void)hipFree(s->mem);
    (void)hipHostFree(s->h_count);
    sv->allocated -= s->bytes;
    delete s;
}

Slot *new_slot(sift3d_server *sv, const Kind &k, sift3d_plan *plan, size_t bytes)
{
    const int n = k.second;
    Slot *s = new (std::nothrow) Slot();
    if (s == nullptr) return nullptr;
    s->kind = k;
    s->plan = plan;
    s->bytes = bytes;
    if (hipMalloc((void **)&s->mem, bytes) != hipSuccess) {
        delete s;
        return nullptr;
    }
    if (hipHostMalloc((void **)&s->h_count, (size_t)n * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(s->mem);
        delete s;
        return nullptr;
    }
    const int cap = sv->cfg.kp_capacity, nb = sv->brief_n;
    size_t in_elems = 0;
    sift3d_plan_info(plan, &s->ws_bytes, nullptr, &in_elems);
    s->in_off.resize(n);
    for (int i = 0; i < n; ++i) sift3d_plan_volume(plan, i, nullptr, &s->in_off[i], nullptr);
    s->vol_bytes = (size_t)k.first[0] * k.first[1] * k.first[2] * sizeof(float);
    // workspace, packed input, counts, then [n] blocks of each output, laid
    // out as the batch plan's calls address them (block i at i * capacity)
    char *p = s->mem;
    s->ws = p;
    p += align256(s->ws_bytes);
    s->in = reinterpret_cast<float *>(p);
    p += align256(in_elems * sizeof(float));
    s->count = reinterpret_cast<int *>(p);
    p += align256((size_t)n * sizeof(int));
    s->kp = reinterpret_cast<sift3d_keypoint *>(p);
    p += align256((size_t)n * cap * sizeof(sift3d_keypoint));
    s->sr = reinterpret_cast<uint8_t *>(p);
    p += align256((size_t)n * cap * 64);
    s->br = nb > 0 ? reinterpret_cast<uint64_t *>(p) : nullptr;
    p += align256((size_t)n * cap * (nb / 8));
    s->rr = nb > 0 ? reinterpret_cast<uint8_t *>(p) : nullptr;
    sv->allocated += bytes;
    ++sv->stats.slot_allocations;
    if (sv->allocated > sv->stats.peak_allocated) sv->stats.peak_allocated = sv->allocated;
    return s;
}

// A slot of kind k: an idle one, a new one within the budget, or a new one
// after evicting idle slots of other kinds (least recently used first).
// nullptr: not now (wait for a release), or the plan could not be made.
Slot *acquire_slot(sift3d_server *sv, const Kind &k)
{
    auto it = sv->idle.find(k);
    if (it != sv->idle.end() && !it->second.empty()) {
        Slot *s = it->second.back();
        it->second.pop_back();
        sv->idle_bytes -= s->bytes;
        return s;
    }
    sift3d_plan *plan = nullptr;
    if (get_plan(sv, k, &plan) != SIFT3D_OK) return nullptr;
    const size_t need = slot_bytes(sv, plan, k.second);
    const size_t budget = sv->cfg.hbm_budget;
    if (need > budget) return nullptr;
    while (sv->allocated + need > budget) {
        Slot *oldest = nullptr;
        std::vector<Slot *> *from = nullptr;
        for (auto &kv : sv->idle)
            for (Slot *s : kv.second)
                if (oldest == nullptr || s->last_use < oldest->last_use) oldest = s, from = &kv.second;
        if (oldest == nullptr) return nullptr;
        from->erase(std::find(from->begin(), from->end(), oldest));
        sv->idle_bytes -= oldest->bytes;
        free_slot(sv, oldest);
        ++sv->stats.slot_evictions;
    }
    return new_slot(sv, k, plan, need);
}

int pick_stream(const sift3d_server *sv)
{
    int best = 0;
    for (int i = 1; i < (int)sv->streams.size(); ++i)
        if (sv->stream_load[i] < sv->stream_load[best]) best = i;
    return best;
}

// Launch a group on its slot: copy the volumes into the packed input, run
// the batch extraction, bring the counts back. false: launch failed (the
// requests are marked failed, the slot goes back to the pool).
bool start_group(sift3d_server *sv, Group &g)
{
    Slot *s = g.slot;
    g.stream = pick_stream(sv);
    hipStream_t st = sv->streams[g.stream];
    const double t = now_s();
    for (size_t i = 0; i < g.reqs.size(); ++i) {
        Request *r = g.reqs[i];
        r->slot = s;
        r->index = (int)i;
        r->stream = g.stream;
        r->t_start = t;
    }
    if (sv->free_events.empty()) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) sv->free_events.push_back(ev);
    }
    int rc = SIFT3D_OK;
    hipError_t e = hipSuccess;
    if (sv->free_events.empty()) {
        rc = SIFT3D_E_HIP;
        e = hipErrorOutOfMemory;
    } else {
        g.ev = sv->free_events.back();
        sv->free_events.pop_back();
    }
    for (size_t i = 0; rc == SIFT3D_OK && i < g.reqs.size(); ++i) {
        e = hipMemcpyAsync(s->in + s->in_off[i], g.reqs[i]->vol, s->vol_bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) rc = SIFT3D_E_HIP;
    }
    if (rc == SIFT3D_OK) {
        rc = sift3d_extract(s->plan, s->in, s->ws, s->ws_bytes, s->kp, sv->cfg.kp_capacity, s->count, s->sr, s->br,
                            s->rr, st);
        if (rc != SIFT3D_OK) e = (hipError_t)sift3d_last_hip_error();
    }
    if (rc == SIFT3D_OK) {
        e = hipMemcpyAsync(s->h_count, s->count, g.reqs.size() * sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(g.ev, st);
        if (e != hipSuccess) rc = SIFT3D_E_HIP;
    }
    if (rc != SIFT3D_OK) {
        for (Request *r : g.reqs) {
            r->rc = rc;
            r->hip_error = (int)e;
            r->state = kFailed;
            r->slot = nullptr;
            r->t_done = now_s();
            ++sv->stats.failed;
        }
        if (g.ev != nullptr) sv->free_events.push_back(g.ev);
        s->last_use = now_s();
        sv->idle[s->kind].push_back(s);
        sv->idle_bytes += s->bytes;
        return false;
    }
    for (Request *r : g.reqs) r->state = kRunning;
    s->holders = (int)g.reqs.size();
    ++sv->stream_load[g.stream];
    return true;
}

// The head request and up to max_batch - 1 later pending requests of its
// shape, size rounded down to a power of two. A group that passes over
// waiting requests of other shapes must leave room for a lone slot for each
// of them next to the memory already held and its own slot: a client that
// consumes results in submission order may keep the group's slot until it
// has received those requests' results, so they must never wait for it.
std::vector<Request *> form_group(sift3d_server *sv)
{
    std::vector<Request *> grp;
    const Shape shape = sv->pending.front()->shape;
    for (Request *r : sv->pending) {
        if (r->shape == shape) grp.push_back(r);
        if ((int)grp.size() == sv->cfg.max_batch) break;
    }
    size_t n = 1;
    while (n * 2 <= grp.size()) n *= 2;
    const size_t held = sv->allocated - sv->idle_bytes;
    for (; n > 1; n /= 2) {
        // lone slots of the requests passed over, up to the group's last member
        size_t skipped = 0;
        for (Request *r : sv->pending) {
            if (r == grp[n - 1]) break;
            if (r->shape != shape) skipped += r->footprint;
        }
        sift3d_plan *plan = nullptr;
        if (get_plan(sv, Kind{shape, (int)n}, &plan) != SIFT3D_OK) continue;
        if (held + slot_bytes(sv, plan, (int)n) + skipped <= sv->cfg.hbm_budget) break;
    }
    grp.resize(n);
    return grp;
}

void scheduler(sift3d_server *sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        // slots of fully released groups go back to the pool
        for (Slot *s : sv->to_release) {
            s->last_use = now_s();
            sv->idle[s->kind].push_back(s);
            sv->idle_bytes += s->bytes;
        }
        sv->to_release.clear();

        // completions
        bool finished = false;
        for (size_t i = 0; i < sv->running.size();) {
            Group &g = sv->running[i];
            const hipError_t q = hipEventQuery(g.ev);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            const double t = now_s();
            for (size_t j = 0; j < g.reqs.size(); ++j) {
                Request *r = g.reqs[j];
                r->t_done = t;
                if (q == hipSuccess) {
                    r->count = g.slot->h_count[j];
                    r->state = kDone;
                    ++sv->stats.completed;
                } else {
                    r->rc = SIFT3D_E_HIP;
                    r->hip_error = (int)q;
                    r->state = kFailed;
                    ++sv->stats.failed;
                }
            }
            --sv->stream_load[g.stream];
            sv->free_events.push_back(g.ev);
            sv->running[i] = sv->running.back();
            sv->running.pop_back();
            finished = true;
        }

        // admissions, in arrival order; a group that does not fit is shrunk
        while (!sv->pending.empty() && (int)sv->running.size() < sv->cfg.max_inflight) {
            std::vector<Request *> grp = form_group(sv);
            Slot *s = nullptr;
            while (!grp.empty()) {
                s = acquire_slot(sv, Kind{grp[0]->shape, (int)grp.size()});
                if (s != nullptr) break;
                grp.resize(grp.size() / 2);
            }
            if (s == nullptr) break;  // memory frees up when a held slot is released
            for (Request *r : grp) sv->pending.erase(std::find(sv->pending.begin(), sv->pending.end(), r));
            Group g{s, grp, 0, nullptr};
            if (start_group(sv, g))
                sv->running.push_back(g);
            else
                finished = true;
            ++sv->stats.groups;
            sv->stats.grouped_requests += (int64_t)grp.size();
        }
        sv->stats.in_flight = 0;
        for (const Group &g : sv->running) sv->stats.in_flight += (int)g.reqs.size();
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
        cfg->kp_capacity < 1 || cfg->hbm_budget == 0 || cfg->max_batch < 1 || cfg->max_batch > 64)
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
    std::lock_guard<std::mutex> lk(sv->mu);
    sift3d_plan *plan = nullptr;
    const int rc = get_plan(sv, Kind{Shape{nx, ny, nz}, 1}, &plan);
    if (rc != SIFT3D_OK) return rc;
    *bytes = slot_bytes(sv, plan, 1);
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
    const size_t cap = (size_t)sv->cfg.kp_capacity, nb = (size_t)sv->brief_n;
    const Slot *s = r->state == kDone ? r->slot : nullptr;
    const size_t i = (size_t)r->index;
    out->status = r->state == kDone ? SIFT3D_OK : r->rc;
    out->hip_error = r->hip_error;
    out->count = r->count;
    out->capacity = (int)cap;
    out->d_kp = s ? s->kp + i * cap : nullptr;
    out->d_siftrank = s ? s->sr + i * cap * 64 : nullptr;
    out->d_brief = (s && s->br) ? s->br + i * cap * (nb / 64) : nullptr;
    out->d_rrief = (s && s->rr) ? s->rr + i * cap * nb : nullptr;
    out->stream = r->stream;
    out->t_submit = r->t_submit;
    out->t_start = r->t_start;
    out->t_done = r->t_done;
    return SIFT3D_OK;
}

int sift3d_server_fetch(sift3d_server *sv, int64_t ticket, sift3d_keypoint *h_kp, uint8_t *h_siftrank,
                        uint64_t *h_brief, uint8_t *h_rrief)
{
    sift3d_result res;
    const int rc = sift3d_server_result(sv, ticket, 1, &res);
    if (rc != SIFT3D_OK) return rc;
    if (res.status != SIFT3D_OK) return res.status;
    // the slot cannot be reused before the client releases this ticket
    hipStream_t st = sv->streams[res.stream];
    const size_t n = (size_t)std::min(res.count, res.capacity), bn = (size_t)sv->brief_n;
    hipError_t e = hipSuccess;
    if (h_kp && n) e = hipMemcpyAsync(h_kp, res.d_kp, n * sizeof(sift3d_keypoint), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && h_siftrank && n)
        e = hipMemcpyAsync(h_siftrank, res.d_siftrank, n * 64, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && h_brief && n && bn)
        e = hipMemcpyAsync(h_brief, res.d_brief, n * bn / 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && h_rrief && n && bn)
        e = hipMemcpyAsync(h_rrief, res.d_rrief, n * bn, hipMemcpyDeviceToHost, st);
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
        if (r->slot != nullptr && --r->slot->holders == 0) sv->to_release.push_back(r->slot);
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
    // slots still held by unreleased requests, then the pool
    std::vector<Slot *> held;
    for (auto &kv : sv->reqs) {
        Slot *s = kv.second->slot;
        if (s != nullptr && std::find(held.begin(), held.end(), s) == held.end()) held.push_back(s);
        delete kv.second;
    }
    for (Slot *s : held) free_slot(sv, s);
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
