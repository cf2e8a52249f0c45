// Admission policy of the request server: which waiting requests run
// together, and on which device memory. Pure host logic with no device
// calls, so the scheduler runs it under its lock for microseconds and does
// all device work (allocation, frees, launches) outside; the same code is
// driven on the CPU by a stand-in executor in the tests.
//
// Rules (all in bytes of device memory):
//   - Requests are admitted in arrival order. The head of the queue takes
//     up to max_batch - 1 later waiting requests of its shape with it; the
//     group size is rounded down to a power of two.
//   - A group runs on a slot of its kind (shape, size): an idle slot of that
//     kind if there is one, else a new one. A new slot is taken only if the
//     bytes of all slots stay within the budget, after freeing idle slots of
//     other kinds least recently used first (and only when freeing every
//     idle slot would make enough room). A group that gets no slot is
//     halved before the head waits.
//   - A group may pass over waiting requests of other shapes only if the
//     bytes held by groups, its own slot and a lone slot for every request
//     it passes over all fit in the budget. A client that consumes results in
//     submission order may keep a group's slot until it has received the
//     results of the requests that group passed over; those must therefore
//     never wait for that memory.
#pragma once

#include <algorithm>
#include <array>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <utility>
#include <vector>

namespace s3d {
namespace serve {

using Shape = std::array<int, 3>;
using Kind = std::pair<Shape, int>;   // (shape, volumes per group)

struct Waiting {
    int64_t id;
    Shape shape;
    size_t footprint;                 // bytes of a lone slot of its shape
    double deadline = 0.0;            // admission deadline (clock seconds); 0 = none
};

// What the executor must do to start one admitted group.
template <class Slot>
struct Admission {
    std::vector<int64_t> reqs;        // request ids, in arrival order
    Kind kind;
    Slot *reuse = nullptr;            // an idle slot of the kind, or
    size_t new_bytes = 0;             // the size of a new slot (reuse == nullptr)
    std::vector<Slot *> evict;        // idle slots to free before allocating
};

// Slot must have the fields `Kind kind; size_t bytes; double last_use;`.
template <class Slot>
class Policy {
public:
    // slot_bytes(kind): bytes of a slot of that kind, 0 if the kind cannot be planned.
    Policy(size_t budget, int max_batch, std::function<size_t(const Kind &)> slot_bytes)
        : budget_(budget), max_batch_(max_batch), slot_bytes_(std::move(slot_bytes))
    {
    }

    std::deque<Waiting> pending;

    size_t allocated() const { return allocated_; }   // all slots, idle or held, and reservations
    size_t idle_bytes() const { return idle_bytes_; }
    const std::map<Kind, std::vector<Slot *>> &idle() const { return idle_; }

    // Requests whose admission deadline has passed leave the queue; their
    // ids are appended to `out` in arrival order.
    void expire(double now, std::vector<int64_t> &out)
    {
        for (size_t i = 0; i < pending.size();) {
            if (pending[i].deadline > 0.0 && pending[i].deadline <= now) {
                out.push_back(pending[i].id);
                pending.erase(pending.begin() + (long)i);
            } else {
                ++i;
            }
        }
    }

    // Earliest admission deadline of the queue, or 0 if none.
    double next_deadline() const
    {
        double t = 0.0;
        for (const Waiting &w : pending)
            if (w.deadline > 0.0 && (t == 0.0 || w.deadline < t)) t = w.deadline;
        return t;
    }

    // A slot whose group has been released (or never ran) becomes idle.
    void add_idle(Slot *s, double now)
    {
        s->last_use = now;
        idle_[s->kind].push_back(s);
        idle_bytes_ += s->bytes;
    }

    // A reservation that was not turned into a slot, or a slot that was freed
    // outside the policy (shutdown).
    void drop(size_t bytes) { allocated_ -= bytes; }

    // Decide the next group: pops its requests from `pending`. false if
    // nothing is pending or the head has to wait for memory.
    bool admit(Admission<Slot> &a)
    {
        if (pending.empty()) return false;
        std::vector<size_t> grp = form_group();
        while (!grp.empty()) {
            a = Admission<Slot>{};
            a.kind = Kind{pending[grp[0]].shape, (int)grp.size()};
            if (take_slot(a)) break;
            grp.resize(grp.size() / 2);
        }
        if (grp.empty()) return false;
        for (size_t i : grp) a.reqs.push_back(pending[i].id);
        for (size_t k = grp.size(); k-- > 0;) pending.erase(pending.begin() + (long)grp[k]);
        return true;
    }

private:
    // Indexes into `pending` of the head group (head first), already sized
    // by the pass-over rule.
    std::vector<size_t> form_group() const
    {
        std::vector<size_t> grp;
        const Shape shape = pending.front().shape;
        for (size_t i = 0; i < pending.size() && (int)grp.size() < max_batch_; ++i)
            if (pending[i].shape == shape) grp.push_back(i);
        size_t n = 1;
        while (n * 2 <= grp.size()) n *= 2;
        const size_t held = allocated_ - idle_bytes_;
        for (; n > 1; n /= 2) {
            size_t skipped = 0;   // lone slots of the requests passed over, up to the group's last member
            for (size_t i = 0; i < grp[n - 1]; ++i)
                if (pending[i].shape != shape) skipped += pending[i].footprint;
            const size_t need = slot_bytes_(Kind{shape, (int)n});
            if (need != 0 && held + need + skipped <= budget_) break;
        }
        grp.resize(n);
        return grp;
    }

    bool take_slot(Admission<Slot> &a)
    {
        auto it = idle_.find(a.kind);
        if (it != idle_.end() && !it->second.empty()) {
            a.reuse = it->second.back();
            it->second.pop_back();
            idle_bytes_ -= a.reuse->bytes;
            return true;
        }
        const size_t need = slot_bytes_(a.kind);
        if (need == 0 || need > budget_) return false;
        if (allocated_ - idle_bytes_ + need > budget_) return false;   // freeing every idle slot would not do
        while (allocated_ + need > budget_) {
            Slot *oldest = nullptr;
            std::vector<Slot *> *from = nullptr;
            for (auto &kv : idle_)
                for (Slot *s : kv.second)
                    if (oldest == nullptr || s->last_use < oldest->last_use) oldest = s, from = &kv.second;
            from->erase(std::find(from->begin(), from->end(), oldest));
            idle_bytes_ -= oldest->bytes;
            allocated_ -= oldest->bytes;
            a.evict.push_back(oldest);
        }
        allocated_ += need;
        a.new_bytes = need;
        return true;
    }

    size_t budget_;
    int max_batch_;
    std::function<size_t(const Kind &)> slot_bytes_;
    std::map<Kind, std::vector<Slot *>> idle_;
    size_t allocated_ = 0;
    size_t idle_bytes_ = 0;
};

}  // namespace serve
}  // namespace s3d
