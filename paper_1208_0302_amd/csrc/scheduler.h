// Admission and bookkeeping of the continuous-batching service, host code
// only (no HIP), so that it runs unchanged against the device allocator in
// serving.hip and against a mock allocator in a CPU test.
//
// A request (a tile of pixels) waits in arrival order until its resident
// population fits in the memory budget (and, with a pixel cap, until the
// resident pixels plus its own stay within the cap; a request is always
// admitted into an empty session).  Each step advances every resident request
// by up to gens_per_step generations; a request that reaches its own
// generation count leaves at once and returns its memory.  A cancelled
// request leaves the queue at once, or the resident set at the next step.
// A finished or cancelled request stays known (for polling) until released.
#ifndef GENESIS_SCHEDULER_H
#define GENESIS_SCHEDULER_H

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <memory>
#include <unordered_map>
#include <vector>

namespace genesis {

enum SchedState { kQueued = 0, kResident = 1, kDone = 2, kCancelled = 3 };

// Payload: what the caller keeps per request (device descriptors, events).
template <class Payload>
struct SchedReq {
    uint64_t id = 0;
    int64_t npix = 0;
    int32_t generations = 0;  // G of the request
    int32_t gen_done = -1;    // generations completed, -1 = generation 0 not created
    int32_t gen_to = 0;       // generation to reach in the launch being planned
    size_t bytes = 0;         // session-owned memory while resident
    int state = kQueued;
    bool cancel = false;
    Payload p{};
};

template <class Payload>
class Scheduler {
public:
    using Req = SchedReq<Payload>;
    using Ptr = std::shared_ptr<Req>;

    Scheduler(size_t budget, int gens_per_step) : budget_(budget), gens_(gens_per_step) {}

    size_t budget() const { return budget_; }
    size_t in_use() const { return in_use_; }
    int64_t resident_pixels() const { return pixels_; }
    size_t queued() const { return queue_.size(); }
    size_t resident() const { return resident_.size(); }
    size_t tracked() const { return all_.size(); }
    void set_max_pixels(int64_t n) { max_pixels_ = n; }

    // Queue a request; false when it can never fit (larger than the budget).
    bool submit(const Ptr &r)
    {
        if (r->bytes > budget_)
            return false;
        r->id = next_id_++;
        r->state = kQueued;
        queue_.push_back(r);
        all_[r->id] = r;
        return true;
    }

    Req *find(uint64_t id)
    {
        auto it = all_.find(id);
        return it == all_.end() ? nullptr : it->second.get();
    }

    // false for an unknown id
    bool cancel(uint64_t id)
    {
        Req *r = find(id);
        if (!r)
            return false;
        if (r->state == kQueued) {
            for (auto q = queue_.begin(); q != queue_.end(); ++q)
                if ((*q)->id == id) {
                    queue_.erase(q);
                    break;
                }
            r->state = kCancelled;
        } else if (r->state == kResident) {
            r->cancel = true;
        }
        return true;
    }

    // Forget a finished or cancelled request; false if it is still queued or
    // resident (or unknown).  `drop(req)` frees what the caller kept for it.
    template <class Drop>
    bool release(uint64_t id, Drop &&drop)
    {
        auto it = all_.find(id);
        if (it == all_.end())
            return false;
        Req &r = *it->second;
        if (r.state != kDone && r.state != kCancelled)
            return false;
        drop(r);
        all_.erase(it);
        return true;
    }

    // First half of a step: cancelled residents leave (free), queued requests
    // are admitted in arrival order while the budget and the cap allow
    // (alloc(req) -> false stops admission and makes plan return false, the
    // request staying first in the queue), and every resident request gets the
    // generation it reaches in this launch.  `out` lists the residents.
    template <class Alloc, class Free>
    bool plan(Alloc &&alloc, Free &&free, std::vector<Req *> &out)
    {
        for (auto it = resident_.begin(); it != resident_.end();) {
            if ((*it)->cancel) {
                leave(**it, free);
                (*it)->state = kCancelled;
                it = resident_.erase(it);
            } else {
                ++it;
            }
        }
        bool ok = true;
        while (!queue_.empty()) {
            Req &r = *queue_.front();
            if (in_use_ + r.bytes > budget_)
                break;
            if (max_pixels_ > 0 && !resident_.empty() && pixels_ + r.npix > max_pixels_)
                break;
            if (!alloc(r)) {
                ok = false;
                break;
            }
            in_use_ += r.bytes;
            pixels_ += r.npix;
            r.state = kResident;
            resident_.push_back(queue_.front());
            queue_.pop_front();
        }
        out.clear();
        for (auto &rp : resident_) {
            Req &r = *rp;
            const int from = r.gen_done < 0 ? 0 : r.gen_done;
            r.gen_to = std::min(from + gens_, r.generations);
            out.push_back(&r);
        }
        return ok;
    }

    // Second half, once the launch of the planned residents is enqueued:
    // each reaches gen_to; those at their generation count finish
    // (done(req), then free) and leave.
    template <class Done, class Free>
    void commit(Done &&done, Free &&free)
    {
        for (auto it = resident_.begin(); it != resident_.end();) {
            Req &r = **it;
            r.gen_done = r.gen_to;
            if (r.gen_done == r.generations) {
                done(r);
                leave(r, free);
                r.state = kDone;
                it = resident_.erase(it);
            } else {
                ++it;
            }
        }
    }

    // Every request still known, for teardown.
    template <class F>
    void for_each(F &&f)
    {
        for (auto &kv : all_)
            f(*kv.second);
    }
    template <class F>
    void for_each_resident(F &&f)
    {
        for (auto &r : resident_)
            f(*r);
    }

private:
    template <class Free>
    void leave(Req &r, Free &&free)
    {
        free(r);
        in_use_ -= r.bytes;
        pixels_ -= r.npix;
    }

    size_t budget_ = 0, in_use_ = 0;
    int64_t max_pixels_ = 0, pixels_ = 0;
    int gens_ = 1;
    uint64_t next_id_ = 1;
    std::deque<Ptr> queue_;
    std::vector<Ptr> resident_;
    std::unordered_map<uint64_t, Ptr> all_;
};

}  // namespace genesis

#endif  // GENESIS_SCHEDULER_H
