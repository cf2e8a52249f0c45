// Discrete-event simulation of the request server's admission policy
// (paper_2112_10258_amd/csrc/server_policy.h, the code the server runs)
// with a stand-in executor: slots are byte counts, a group finishes after a
// modelled duration, and a client consumes results in submission order and
// releases each ticket as soon as it has read it. Host only, no device.
//
// Usage: server_policy_sim SEED BUDGET_MB MAX_BATCH MAX_INFLIGHT N_REQ SATURATED
// Prints one JSON line with the outcome and the invariants checked:
//   - the bytes of all live slots never exceed the budget;
//   - every request completes (no state in which nothing runs, nothing
//     arrives and requests still wait);
//   - a group holds requests of one shape, its size a power of two at most
//     MAX_BATCH, its first request the head of the queue at admission;
//   - at most MAX_INFLIGHT groups run at once.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "server_policy.h"

using s3d::serve::Admission;
using s3d::serve::Kind;
using s3d::serve::Policy;
using s3d::serve::Shape;

namespace {

struct FakeSlot {
    Kind kind;
    size_t bytes;
    double last_use;
    int holders;
    long id;
};

// A slot's bytes: a pyramid workspace of about 80 bytes per voxel per
// volume, plus 1 MiB of fixed buffers (a stand-in for the real sizes).
size_t fake_bytes(const Kind &k)
{
    const double vox = (double)k.first[0] * k.first[1] * k.first[2];
    return (size_t)(k.second * vox * 80.0) + (1u << 20);
}

double fake_duration(const Kind &k)
{
    const double vox = (double)k.first[0] * k.first[1] * k.first[2];
    return 50e-6 + 20e-6 * k.second + k.second * vox / 20e9;   // seconds
}

struct Req {
    Shape shape;
    double arrival;
    int state = 0;          // 0 waiting to arrive, 1 pending, 2 running, 3 done, 4 timed out
    FakeSlot *slot = nullptr;
};

struct Running {
    FakeSlot *slot;
    std::vector<long> reqs;
    double t_end;
};

}  // namespace

int main(int argc, char **argv)
{
    if (argc != 7 && argc != 8) {
        std::fprintf(stderr, "usage: %s SEED BUDGET_MB MAX_BATCH MAX_INFLIGHT N_REQ SATURATED [TIMEOUT_S]\n", argv[0]);
        return 2;
    }
    const double timeout = argc == 8 ? std::atof(argv[7]) : 0.0;
    const unsigned seed = (unsigned)std::atoi(argv[1]);
    const size_t budget = (size_t)(std::atof(argv[2]) * (1 << 20));
    const int max_batch = std::atoi(argv[3]), max_inflight = std::atoi(argv[4]), n_req = std::atoi(argv[5]);
    const bool saturated = std::atoi(argv[6]) != 0;

    std::mt19937_64 rng(seed);
    const std::vector<Shape> shapes = {{64, 64, 64}, {145, 174, 145}, {192, 224, 192}, {256, 256, 256}};
    const std::vector<double> probs = {0.2, 0.5, 0.2, 0.1};
    std::discrete_distribution<int> pick(probs.begin(), probs.end());
    std::exponential_distribution<double> gap(200.0);
    std::vector<Req> reqs;
    double t = 0.0;
    int rejected = 0;
    for (int i = 0; i < n_req; ++i) {
        Req r;
        r.shape = shapes[pick(rng)];
        if (!saturated) t += gap(rng);
        r.arrival = t;
        if (fake_bytes(Kind{r.shape, 1}) > budget) {   // submit refuses it
            ++rejected;
            continue;
        }
        reqs.push_back(r);
    }

    Policy<FakeSlot> pol(budget, max_batch, fake_bytes);
    std::vector<Running> running;
    std::set<FakeSlot *> live;
    size_t live_bytes = 0, peak = 0;
    long next_slot = 0, groups = 0, evictions = 0, allocations = 0, max_group = 0, max_running = 0;
    bool ok_budget = true, ok_shape = true, ok_pow2 = true, ok_head = true, deadlock = false, ok_deadline = true;
    long expired = 0;
    size_t next_arrival = 0, consumer = 0, done = 0;
    double now = 0.0;
    std::vector<FakeSlot *> released;

    while (done < reqs.size()) {
        // arrivals up to now
        while (next_arrival < reqs.size() && reqs[next_arrival].arrival <= now) {
            Req &r = reqs[next_arrival];
            r.state = 1;
            pol.pending.push_back(s3d::serve::Waiting{(int64_t)next_arrival, r.shape, fake_bytes(Kind{r.shape, 1}),
                                                      timeout > 0.0 ? r.arrival + timeout : 0.0});
            ++next_arrival;
        }
        // the client: results in submission order, released once read
        while (consumer < reqs.size() && (reqs[consumer].state == 3 || reqs[consumer].state == 4)) {
            FakeSlot *s = reqs[consumer].slot;
            if (s != nullptr && --s->holders == 0) released.push_back(s);
            ++consumer;
        }
        for (FakeSlot *s : released) pol.add_idle(s, now);
        released.clear();
        // requests past their admission deadline end first
        {
            std::vector<int64_t> exp;
            pol.expire(now, exp);
            for (int64_t id : exp) {
                if (now - reqs[id].arrival < timeout) ok_deadline = false;
                reqs[id].state = 4;
                reqs[id].slot = nullptr;
                ++expired;
                ++done;
            }
        }
        // admissions
        while ((int)running.size() < max_inflight) {
            const int64_t head = pol.pending.empty() ? -1 : pol.pending.front().id;
            Admission<FakeSlot> a;
            if (!pol.admit(a)) break;
            ++groups;
            max_group = std::max<long>(max_group, (long)a.reqs.size());
            if (a.reqs.front() != head) ok_head = false;
            const size_t n = a.reqs.size();
            if ((n & (n - 1)) != 0 || (int)n > max_batch) ok_pow2 = false;
            for (int64_t id : a.reqs)
                if (reqs[id].shape != a.kind.first) ok_shape = false;
            for (FakeSlot *e : a.evict) {
                live.erase(e);
                live_bytes -= e->bytes;
                delete e;
                ++evictions;
            }
            FakeSlot *s = a.reuse;
            if (s == nullptr) {
                s = new FakeSlot{a.kind, a.new_bytes, now, 0, next_slot++};
                live.insert(s);
                live_bytes += s->bytes;
                ++allocations;
            }
            if (live_bytes > budget || pol.allocated() != live_bytes) ok_budget = false;
            peak = std::max(peak, live_bytes);
            s->holders = (int)n;
            Running g{s, {}, now + fake_duration(a.kind)};
            for (int64_t id : a.reqs) {
                if (timeout > 0.0 && now > reqs[id].arrival + timeout) ok_deadline = false;
                reqs[id].state = 2;
                reqs[id].slot = s;
                g.reqs.push_back(id);
            }
            running.push_back(g);
            max_running = std::max<long>(max_running, (long)running.size());
        }
        // next event: a completion or an arrival
        double t_next = 1e300;
        for (const Running &g : running) t_next = std::min(t_next, g.t_end);
        if (next_arrival < reqs.size()) t_next = std::min(t_next, reqs[next_arrival].arrival);
        if (pol.next_deadline() > 0.0) t_next = std::min(t_next, pol.next_deadline());
        const bool client_can_move =
            consumer < reqs.size() && (reqs[consumer].state == 3 || reqs[consumer].state == 4);
        if (t_next == 1e300 && !client_can_move && released.empty()) {
            deadlock = true;
            break;
        }
        if (t_next != 1e300 && !client_can_move) now = std::max(now, t_next);
        for (size_t i = 0; i < running.size();) {
            if (running[i].t_end <= now) {
                for (long id : running[i].reqs) {
                    reqs[id].state = 3;
                    ++done;
                }
                running[i] = running.back();
                running.pop_back();
            } else {
                ++i;
            }
        }
    }
    for (FakeSlot *s : live) delete s;
    std::printf("{\"requests\": %zu, \"rejected\": %d, \"completed\": %zu, \"deadlock\": %s, \"budget\": %zu, "
                "\"peak_bytes\": %zu, \"groups\": %ld, \"max_group\": %ld, \"allocations\": %ld, "
                "\"evictions\": %ld, \"max_running\": %ld, \"ok_budget\": %s, \"ok_shape\": %s, \"ok_pow2\": %s, "
                "\"ok_head\": %s, \"expired\": %ld, \"ok_deadline\": %s, \"sim_seconds\": %.6f}\n",
                reqs.size(), rejected, done, deadlock ? "true" : "false", budget, peak, groups, max_group, allocations,
                evictions, max_running, ok_budget ? "true" : "false", ok_shape ? "true" : "false",
                ok_pow2 ? "true" : "false", ok_head ? "true" : "false", expired, ok_deadline ? "true" : "false", now);
    return 0;
}
