// Extraction request server: continuous batching of independent volumes on
// one GPU.
//
// Requests arrive one at a time (sift3d_server_submit). A scheduler thread
// admits them in arrival order under the policy of server_policy.h: the
// head of the queue runs together with up to max_batch - 1 later requests of
// its shape (a power-of-two group), as one batch extraction, so each
// pyramid, detection and descriptor launch covers every volume of the group.
// A group runs on a slot: one device allocation holding the packed input,
// the batch plan's workspace and the keypoint and descriptor buffers of its
// requests, cached per (shape, group size) and kept by the group until the
// client has released every ticket of it. At most max_inflight groups are on
// the device, spread over n_streams streams so their kernels overlap.
//
// The scheduler holds the server mutex only while it applies releases,
// decides admissions and publishes results. Frees, allocations, launches
// and completion polls run outside it, so clients' submit, result and
// release calls never wait behind device work. Plans are created by
// submit (the first request of a shape plans every group size) under a
// mutex of their own.
//
// Groups launch their extraction directly on their stream. (With a HIP
// graph captured per slot by the scheduler thread while client threads used
// the device, later work on the process's legacy stream failed with a
// capture-in-progress error; a captured config-2 extraction also replays no
// faster than its launches. Slots hold no graph.)
// Clients' result copies run on a stream of their own.
//
// A batch plan gives each volume exactly the results of a one-volume plan
// (same kernels, same arithmetic), so a request's result does not depend on
// what it was grouped with or what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "server_policy.h"
#include "sift3d.h"

namespace {

using s3d::serve::Kind;
using s3d::serve::Shape;

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// A device allocation for one group of n requests of one shape.
struct Slot {
    Kind kind;
    size_t bytes;
    double last_use;
    sift3d_plan *plan;      // the (shape, n) batch plan, owned by the server's plan cache
    char *mem;              // one device allocation
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
};

struct Request {
    int64_t id;
    const float *vol;
    Shape shape;
    int state;              // 0 pending, 1 on the device, 2 done, 3 failed
    int rc;
    int hip_error;
    Slot *slot;
    int index;              // volume index within the slot
    int stream;
    int count;
    double t_submit, t_start, t_done;
};

enum { kPending = 0, kRunning = 1, kDone = 2, kFailed = 3 };

// A group on the device (scheduler-only).
struct Group {
    Slot *slot;
    std::vector<Request *> reqs;
    int stream;
    hipEvent_t ev;
    double t_start;
};

// A group decided under the lock, started outside it.
struct Start {
    s3d::serve::Admission<Slot> adm;
    std::vector<Request *> reqs;
    Group g{};
    int rc = SIFT3D_OK;
    int hip_error = 0;
};

}  // namespace

struct sift3d_server {
    sift3d_ctx *ctx;
    sift3d_server_config cfg;
    int device;
    int brief_n;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;       // scheduler-only
    hipStream_t fetch_stream = nullptr;     // result copies of sift3d_server_fetch (client threads)

    // plans and slot sizes per kind (plan_mu); never held together with mu
    std::mutex plan_mu;
    std::map<Kind, sift3d_plan *> plans;

    // shared with client threads (guarded by mu)
    std::mutex mu;
    std::condition_variable cv_work;   // scheduler: new request, release or stop
    std::condition_variable cv_done;   // clients: a request finished
    std::unordered_map<int64_t, Request *> reqs;
    std::vector<Slot *> to_release;    // slots whose group is fully released
    std::map<Kind, size_t> kind_bytes; // slot bytes per kind (0: cannot be planned)
    s3d::serve::Policy<Slot> *policy = nullptr;
    int64_t next_id = 1;
    int64_t work_gen = 0;              // bumped by every submission, release and stop
    bool stop = false;
    sift3d_server_counters stats{};

    // scheduler-only state
    std::vector<Group> running;
    std::vector<hipEvent_t> free_events;

    std::thread thread;
};

namespace {

size_t outputs_bytes(int cap, int brief_n)
{
    return align256((size_t)cap * sizeof(sift3d_keypoint)) + align256((size_t)cap * 64) +
           align256((size_t)cap * (brief_n / 8)) + align256((size_t)cap * brief_n);
}

// Device bytes of a slot for `plan` (n volumes).
size_t slot_bytes(const sift3d_server *sv, const sift3d_plan *plan, int n)
{
    size_t ws = 0, in_elems = 0;
    sift3d_plan_info(plan, &ws, nullptr, &in_elems);
    return align256(ws) + align256(in_elems * sizeof(float)) + align256((size_t)n * sizeof(int)) +
           (size_t)n * outputs_bytes(sv->cfg.kp_capacity, sv->brief_n);
}

// Plans of every group size (powers of two up to max_batch) of a shape, and
// their slot sizes; returns the rc of the lone plan. Takes plan_mu only.
int ensure_plans(sift3d_server *sv, const Shape &shape, std::vector<std::pair<Kind, size_t>> &sizes)
{
    std::lock_guard<std::mutex> lk(sv->plan_mu);
    int rc_lone = SIFT3D_OK;
    for (int n = 1; n <= sv->cfg.max_batch; n *= 2) {
        const Kind k{shape, n};
        auto it = sv->plans.find(k);
        sift3d_plan *p = it == sv->plans.end() ? nullptr : it->second;
        if (p == nullptr) {
            std::vector<int> dims;
            for (int i = 0; i < n; ++i) dims.insert(dims.end(), shape.begin(), shape.end());
            const int rc = sift3d_plan_create_batch(sv->ctx, n, dims.data(), sv->cfg.kp_capacity, &p);
            if (rc != SIFT3D_OK) {
                p = nullptr;
                if (n == 1) rc_lone = rc;
            } else {
                sv->plans[k] = p;
            }
        }
        sizes.emplace_back(k, p ? slot_bytes(sv, p, n) : 0);
        if (n == 1 && p == nullptr) break;
    }
    return rc_lone;
}

sift3d_plan *find_plan(sift3d_server *sv, const Kind &k)
{
    std::lock_guard<std::mutex> lk(sv->plan_mu);
    auto it = sv->plans.find(k);
    return it == sv->plans.end() ? nullptr : it->second;
}

void free_slot(Slot *s)
{
    (void)hipFree(s->mem);
    (void)hipHostFree(s->h_count);
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
    return s;
}

int pick_stream(const sift3d_server *sv)
{
    int best = 0;
    for (int i = 1; i < (int)sv->streams.size(); ++i)
        if (sv->stream_load[i] < sv->stream_load[best]) best = i;
    return best;
}

// Outside the lock: free the evicted slots, get the group's slot and launch
// the input copies, the extraction and the copy of the counts, then an
// event. On failure the slot is kept out of the pool until its stream has
// drained (st.rc != OK; the slot is returned in st.g.slot, or null).
void start_group(sift3d_server *sv, Start &st)
{
    for (Slot *s : st.adm.evict) free_slot(s);
    Group &g = st.g;
    g.stream = pick_stream(sv);
    hipStream_t hs = sv->streams[g.stream];
    Slot *s = st.adm.reuse;
    if (s == nullptr) {
        sift3d_plan *plan = find_plan(sv, st.adm.kind);
        s = plan ? new_slot(sv, st.adm.kind, plan, st.adm.new_bytes) : nullptr;
        if (s == nullptr) {
            st.rc = SIFT3D_E_HIP;
            st.hip_error = (int)hipErrorOutOfMemory;
            g.slot = nullptr;
            return;
        }
    }
    g.slot = s;
    g.reqs = st.reqs;
    g.t_start = now_s();
    if (sv->free_events.empty()) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) sv->free_events.push_back(ev);
    }
    hipError_t e = hipSuccess;
    int rc = SIFT3D_OK;
    if (sv->free_events.empty()) {
        rc = SIFT3D_E_HIP;
        e = hipErrorOutOfMemory;
    } else {
        g.ev = sv->free_events.back();
        sv->free_events.pop_back();
    }
    for (size_t i = 0; rc == SIFT3D_OK && i < g.reqs.size(); ++i) {
        e = hipMemcpyAsync(s->in + s->in_off[i], g.reqs[i]->vol, s->vol_bytes, hipMemcpyDeviceToDevice, hs);
        if (e != hipSuccess) rc = SIFT3D_E_HIP;
    }
    if (rc == SIFT3D_OK) {
        rc = sift3d_extract(s->plan, s->in, s->ws, s->ws_bytes, s->kp, sv->cfg.kp_capacity, s->count, s->sr, s->br,
                            s->rr, hs);
        if (rc != SIFT3D_OK) e = (hipError_t)sift3d_last_hip_error();
    }
    if (rc == SIFT3D_OK) {
        e = hipMemcpyAsync(s->h_count, s->count, g.reqs.size() * sizeof(int), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipEventRecord(g.ev, hs);
        if (e != hipSuccess) rc = SIFT3D_E_HIP;
    }
    if (rc != SIFT3D_OK) {
        // work already enqueued may still use the slot: drain the stream
        // before the slot can go back to the pool
        (void)hipStreamSynchronize(hs);
        if (g.ev != nullptr) sv->free_events.push_back(g.ev);
        g.ev = nullptr;
        st.rc = rc;
        st.hip_error = (int)e;
        return;
    }
    ++sv->stream_load[g.stream];
}

void fail_request(sift3d_server *sv, Request *r, int rc, int hip_error)
{
    r->rc = rc;
    r->hip_error = hip_error;
    r->state = kFailed;
    r->slot = nullptr;
    r->t_done = now_s();
    ++sv->stats.failed;
}

void scheduler(sift3d_server *sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        const int64_t gen = sv->work_gen;
        // under the lock: released slots back to the pool, then admissions
        for (Slot *s : sv->to_release) sv->policy->add_idle(s, now_s());
        sv->to_release.clear();
        bool expired_any = false;
        {
            // requests past their admission deadline end before admissions
            std::vector<int64_t> expired;
            sv->policy->expire(now_s(), expired);
            for (int64_t id : expired) fail_request(sv, sv->reqs.at(id), SIFT3D_E_TIMEOUT, 0);
            expired_any = !expired.empty();
        }
        std::vector<Start> starts;
        while ((int)(sv->running.size() + starts.size()) < sv->cfg.max_inflight) {
            Start st;
            if (!sv->policy->admit(st.adm)) break;
            for (int64_t id : st.adm.reqs) st.reqs.push_back(sv->reqs.at(id));
            starts.push_back(std::move(st));
        }
        if (sv->stop) {
            // requests not yet admitted are cancelled; those on the device finish
            bool any = false;
            for (const s3d::serve::Waiting &w : sv->policy->pending) {
                fail_request(sv, sv->reqs.at(w.id), SIFT3D_E_ARG, 0);
                any = true;
            }
            sv->policy->pending.clear();
            if (any) sv->cv_done.notify_all();
        }
        const bool stopping = sv->stop;
        lk.unlock();

        // outside the lock: launches and completion polls
        for (Start &st : starts) start_group(sv, st);
        std::vector<std::pair<Group, hipError_t>> finished;
        for (size_t i = 0; i < sv->running.size();) {
            const hipError_t q = hipEventQuery(sv->running[i].ev);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            finished.emplace_back(sv->running[i], q);
            sv->running[i] = sv->running.back();
            sv->running.pop_back();
        }
        for (auto &f : finished) {
            --sv->stream_load[f.first.stream];
            sv->free_events.push_back(f.first.ev);
        }

        lk.lock();
        // publish
        bool notify = expired_any;
        for (Start &st : starts) {
            if (st.rc != SIFT3D_OK) {
                for (Request *r : st.reqs) fail_request(sv, r, st.rc, st.hip_error);
                if (st.g.slot != nullptr)
                    sv->policy->add_idle(st.g.slot, now_s());
                else if (st.adm.reuse == nullptr)
                    sv->policy->drop(st.adm.new_bytes);   // the reservation was not allocated
                notify = true;
            } else {
                for (size_t i = 0; i < st.reqs.size(); ++i) {
                    Request *r = st.reqs[i];
                    r->slot = st.g.slot;
                    r->index = (int)i;
                    r->stream = st.g.stream;
                    r->t_start = st.g.t_start;
                    r->state = kRunning;
                }
                st.g.slot->holders = (int)st.reqs.size();
                if (st.adm.reuse == nullptr) {
                    ++sv->stats.slot_allocations;
                    sv->stats.peak_allocated = std::max(sv->stats.peak_allocated, sv->policy->allocated());
                }
                sv->running.push_back(st.g);
            }
            sv->stats.slot_evictions += (int64_t)st.adm.evict.size();
            ++sv->stats.groups;
            sv->stats.grouped_requests += (int64_t)st.reqs.size();
        }
        for (auto &f : finished) {
            const double t = now_s();
            for (size_t j = 0; j < f.first.reqs.size(); ++j) {
                Request *r = f.first.reqs[j];
                r->t_done = t;
                if (f.second == hipSuccess) {
                    r->count = f.first.slot->h_count[j];
                    r->state = kDone;
                    ++sv->stats.completed;
                } else {
                    r->rc = SIFT3D_E_HIP;
                    r->hip_error = (int)f.second;
                    r->state = kFailed;
                    ++sv->stats.failed;
                }
            }
            notify = true;
        }
        sv->stats.in_flight = 0;
        for (const Group &g : sv->running) sv->stats.in_flight += (int)g.reqs.size();
        sv->stats.pending = (int)sv->policy->pending.size();
        sv->stats.allocated = sv->policy->allocated();
        if (notify) sv->cv_done.notify_all();
        if (stopping && sv->running.empty()) break;
        if (sv->work_gen != gen || !starts.empty() || !finished.empty()) continue;   // new work arrived meanwhile
        if (sv->running.empty()) {
            // idle until a submission, a release or stop (nothing pending can
            // start before one), or until the next admission deadline
            const double dl = sv->policy->next_deadline();
            if (dl > 0.0) {
                const double wait_s = std::max(0.0, dl - now_s());
                sv->cv_work.wait_for(lk, std::chrono::duration<double>(wait_s),
                                     [&] { return sv->work_gen != gen; });
            } else {
                sv->cv_work.wait(lk, [&] { return sv->work_gen != gen; });
            }
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
        cfg->kp_capacity < 1 || cfg->hbm_budget == 0 || cfg->max_batch < 1 || cfg->max_batch > 64 ||
        !(cfg->admit_timeout_s >= 0.0) || !std::isfinite(cfg->admit_timeout_s))
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
    for (int i = 0; i < cfg->n_streams + 1; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
            delete sv;
            return SIFT3D_E_HIP;
        }
        if (i == cfg->n_streams) {
            sv->fetch_stream = st;
        } else {
            sv->streams.push_back(st);
            sv->stream_load.push_back(0);
        }
    }
    // the policy reads slot sizes that submit recorded (under mu)
    sv->policy = new s3d::serve::Policy<Slot>(cfg->hbm_budget, cfg->max_batch, [sv](const Kind &k) {
        auto it = sv->kind_bytes.find(k);
        return it == sv->kind_bytes.end() ? (size_t)0 : it->second;
    });
    sv->stats.hbm_budget = cfg->hbm_budget;
    sv->thread = std::thread(scheduler, sv);
    *out = sv;
    return SIFT3D_OK;
}

int sift3d_server_footprint(sift3d_server *sv, int nx, int ny, int nz, size_t *bytes)
{
    if (sv == nullptr || bytes == nullptr) return SIFT3D_E_ARG;
    if (nx < 1 || ny < 1 || nz < 1) return SIFT3D_E_ARG;
    std::vector<std::pair<Kind, size_t>> sizes;
    const int rc = ensure_plans(sv, Shape{nx, ny, nz}, sizes);
    if (rc != SIFT3D_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto &ks : sizes) sv->kind_bytes.insert(ks);
    }
    *bytes = sizes[0].second;
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
        r->state = kPending;
        r->rc = SIFT3D_OK;
        r->t_submit = now_s();
        sv->reqs[r->id] = r;
        const double deadline = sv->cfg.admit_timeout_s > 0.0 ? r->t_submit + sv->cfg.admit_timeout_s : 0.0;
        sv->policy->pending.push_back(s3d::serve::Waiting{r->id, r->shape, fp, deadline});
        ++sv->work_gen;
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
    // the request's group has completed (the scheduler saw its event) and
    // the slot cannot be reused before the client releases this ticket; the
    // copies go on the server's fetch stream, and an event after them is
    // the only thing waited for
    hipStream_t st = sv->fetch_stream;
    const size_t n = (size_t)std::min(res.count, res.capacity), bn = (size_t)sv->brief_n;
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess && h_kp && n)
        e = hipMemcpyAsync(h_kp, res.d_kp, n * sizeof(sift3d_keypoint), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && h_siftrank && n)
        e = hipMemcpyAsync(h_siftrank, res.d_siftrank, n * 64, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && h_brief && n && bn)
        e = hipMemcpyAsync(h_brief, res.d_brief, n * bn / 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && h_rrief && n && bn)
        e = hipMemcpyAsync(h_rrief, res.d_rrief, n * bn, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    if (e == hipSuccess) e = hipEventSynchronize(ev);
    if (ev != nullptr) (void)hipEventDestroy(ev);
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
        ++sv->work_gen;
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
        ++sv->work_gen;
    }
    sv->cv_work.notify_one();
    sv->thread.join();
    for (hipStream_t st : sv->streams) (void)hipStreamSynchronize(st);
    (void)hipStreamSynchronize(sv->fetch_stream);
    // slots still held by unreleased requests, then the pool
    std::vector<Slot *> held;
    for (auto &kv : sv->reqs) {
        Slot *s = kv.second->slot;
        if (s != nullptr && std::find(held.begin(), held.end(), s) == held.end()) held.push_back(s);
        delete kv.second;
    }
    for (Slot *s : held) free_slot(s);
    for (Slot *s : sv->to_release) free_slot(s);
    for (auto &kv : sv->policy->idle())
        for (Slot *s : kv.second) free_slot(s);
    delete sv->policy;
    for (hipEvent_t ev : sv->free_events) (void)hipEventDestroy(ev);
    for (hipStream_t st : sv->streams) (void)hipStreamDestroy(st);
    (void)hipStreamDestroy(sv->fetch_stream);
    for (auto &kv : sv->plans) sift3d_plan_destroy(kv.second);
    delete sv;
    return SIFT3D_OK;
}

}  // extern "C"
