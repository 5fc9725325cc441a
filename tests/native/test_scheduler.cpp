// CPU test of the service's admission and bookkeeping (scheduler.h) against a
// mock device allocator and a mock launch: the memory budget is never
// exceeded, admission is first come first served, the resident-pixel cap is
// respected, every resident request advances by the step's generations,
// cancelled and finished requests return their memory, a failed allocation
// leaves the request first in the queue, and nothing leaks.  Built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_native_host.py.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <vector>

#include "../../paper_1208_0302_amd/csrc/scheduler.h"

using namespace genesis;

namespace {

int failures = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            std::fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

// What a request carries in the mock: its allocation handle and a record of
// the generations it was advanced through.
struct Mock {
    int handle = -1;
    std::vector<int> launches;  // gen_to of each launch it took part in
    bool done_called = false;
};
using Req = SchedReq<Mock>;

struct Device {
    size_t capacity = 0;
    size_t used = 0;
    int next = 0;
    std::map<int, size_t> live;
    bool fail_next = false;
    bool alloc(Req &r)
    {
        if (fail_next || used + r.bytes > capacity) {
            fail_next = false;
            return false;
        }
        r.p.handle = next++;
        live[r.p.handle] = r.bytes;
        used += r.bytes;
        return true;
    }
    void free(Req &r)
    {
        auto it = live.find(r.p.handle);
        CHECK(it != live.end());
        if (it != live.end()) {
            used -= it->second;
            live.erase(it);
        }
        r.p.handle = -1;
    }
};

uint64_t lcg(uint64_t &s)
{
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return s >> 33;
}

std::shared_ptr<Req> make(int64_t npix, int gens, size_t bytes_per_px)
{
    auto r = std::make_shared<Req>();
    r->npix = npix;
    r->generations = gens;
    r->bytes = (size_t)npix * bytes_per_px;
    return r;
}

// One step: plan, "launch" (record gen_to), commit.
bool step(Scheduler<Mock> &s, Device &dev, int gens, std::vector<uint64_t> *admitted = nullptr)
{
    std::vector<Req *> res;
    std::set<uint64_t> before;
    s.for_each_resident([&](Req &r) { before.insert(r.id); });
    const bool ok = s.plan([&](Req &r) { return dev.alloc(r); }, [&](Req &r) { dev.free(r); },
                           res);
    CHECK(s.in_use() <= s.budget());
    CHECK(s.in_use() == dev.used);
    for (Req *r : res) {
        const int from = r->gen_done < 0 ? 0 : r->gen_done;
        CHECK(r->gen_to == std::min(from + gens, r->generations));
        r->p.launches.push_back(r->gen_to);
        if (admitted && !before.count(r->id))
            admitted->push_back(r->id);
    }
    s.commit([](Req &r) { r.p.done_called = true; }, [&](Req &r) { dev.free(r); });
    CHECK(s.in_use() == dev.used);
    return ok;
}

void test_random_stream()
{
    const size_t per_px = 100;
    const size_t budget = 5000 * per_px;
    Scheduler<Mock> s(budget, 3);
    const int64_t cap = 6000;
    s.set_max_pixels(cap);
    Device dev;
    dev.capacity = budget;
    uint64_t seed = 12345;
    std::vector<std::shared_ptr<Req>> reqs;
    std::vector<uint64_t> order, admitted;
    std::set<uint64_t> cancelled;
    for (int t = 0; t < 400; ++t) {
        const int arrivals = (int)(lcg(seed) % 3);
        for (int a = 0; a < arrivals && reqs.size() < 300; ++a) {
            auto r = make(1 + (int64_t)(lcg(seed) % 3000), (int)(lcg(seed) % 12), per_px);
            CHECK(s.submit(r));
            reqs.push_back(r);
            order.push_back(r->id);
        }
        if (!reqs.empty() && lcg(seed) % 10 == 0) {
            auto &r = reqs[lcg(seed) % reqs.size()];
            if (r->state == kQueued || r->state == kResident) {
                CHECK(s.cancel(r->id));
                cancelled.insert(r->id);
            }
        }
        CHECK(step(s, dev, 3, &admitted));
        int64_t px = 0;
        size_t nres = 0;
        s.for_each_resident([&](Req &r) {
            px += r.npix;
            ++nres;
        });
        CHECK(px == s.resident_pixels());
        CHECK(nres <= 1 || px <= cap);
    }
    for (int t = 0; t < 200 && (s.queued() || s.resident()); ++t)
        CHECK(step(s, dev, 3, &admitted));
    CHECK(s.queued() == 0 && s.resident() == 0);
    CHECK(dev.live.empty() && dev.used == 0 && s.in_use() == 0);
    // first come, first served: the admission order is the arrival order
    std::vector<uint64_t> expect;
    for (uint64_t id : order) {
        bool was_admitted = false;
        for (uint64_t a : admitted)
            was_admitted |= a == id;
        if (was_admitted)
            expect.push_back(id);
    }
    CHECK(expect == admitted);
    for (auto &r : reqs) {
        if (r->state == kDone) {
            // advanced 3 generations per launch up to its count, then finished
            CHECK(r->p.done_called);
            CHECK(!cancelled.count(r->id));
            int g = 0;
            for (int to : r->p.launches) {
                CHECK(to == std::min(g + 3, r->generations));
                g = to;
            }
            CHECK(g == r->generations);
        } else {
            CHECK(r->state == kCancelled && cancelled.count(r->id));
            CHECK(!r->p.done_called);
        }
        CHECK(r->p.handle == -1);
        CHECK(s.release(r->id, [](Req &) {}));
    }
    CHECK(s.tracked() == 0);
}

void test_cancel_release_and_errors()
{
    Scheduler<Mock> s(1000, 2);
    Device dev;
    dev.capacity = 1000;
    auto a = make(6, 4, 100), b = make(5, 4, 100), c = make(3, 4, 100);
    CHECK(s.submit(a) && s.submit(b) && s.submit(c));
    CHECK(!s.submit(make(11, 1, 100)));  // larger than the budget
    CHECK(step(s, dev, 2));
    // b does not fit beside a; c would, but waits behind b (arrival order)
    CHECK(a->state == kResident && b->state == kQueued && c->state == kQueued);
    CHECK(!s.release(a->id, [](Req &) {}));  // resident
    CHECK(!s.release(b->id, [](Req &) {}));  // queued
    CHECK(!s.release(999, [](Req &) {}));    // unknown
    CHECK(!s.cancel(999));
    CHECK(s.cancel(b->id) && b->state == kCancelled && s.queued() == 1);
    CHECK(s.cancel(a->id) && a->state == kResident);  // leaves at the next step
    CHECK(step(s, dev, 2));
    CHECK(a->state == kCancelled && a->p.handle == -1 && c->state == kResident);
    int released = 0;
    CHECK(s.release(b->id, [&](Req &) { ++released; }) && released == 1);
    CHECK(s.find(b->id) == nullptr);
}

void test_alloc_failure_keeps_queue_order()
{
    Scheduler<Mock> s(10000, 5);
    Device dev;
    dev.capacity = 10000;
    auto a = make(10, 5, 100), b = make(10, 5, 100);
    CHECK(s.submit(a) && s.submit(b));
    dev.fail_next = true;
    CHECK(!step(s, dev, 5));  // the first allocation fails: nothing admitted
    CHECK(a->state == kQueued && b->state == kQueued && s.in_use() == 0 && dev.live.empty());
    CHECK(step(s, dev, 5));   // then both fit, in order
    CHECK(a->state == kDone && b->state == kDone && dev.live.empty());
}

void test_fcfs_blocks_behind_large_request()
{
    // strict arrival order: a small request does not overtake a large one
    // that waits for memory
    Scheduler<Mock> s(1000, 1);
    Device dev;
    dev.capacity = 1000;
    auto a = make(7, 3, 100), b = make(6, 3, 100), c = make(1, 3, 100);
    CHECK(s.submit(a) && s.submit(b) && s.submit(c));
    CHECK(step(s, dev, 1));
    CHECK(a->state == kResident && b->state == kQueued && c->state == kQueued);
    CHECK(step(s, dev, 1) && step(s, dev, 1));
    CHECK(a->state == kDone);
    CHECK(step(s, dev, 1));
    CHECK(b->state == kResident && c->state == kResident);
}

void test_cap_admits_into_empty_session()
{
    Scheduler<Mock> s(1 << 20, 1);
    s.set_max_pixels(100);
    Device dev;
    dev.capacity = 1 << 20;
    auto big = make(500, 2, 1), small = make(50, 2, 1);
    CHECK(s.submit(big) && s.submit(small));
    CHECK(step(s, dev, 1));
    CHECK(big->state == kResident && small->state == kQueued);  // above the cap, but alone
    CHECK(step(s, dev, 1));
    CHECK(big->state == kDone);
    CHECK(step(s, dev, 1));
    CHECK(small->state == kResident);
}

void test_zero_generations()
{
    // G = 0: generation 0 is created and evaluated in one launch, then done
    Scheduler<Mock> s(1000, 4);
    Device dev;
    dev.capacity = 1000;
    auto r = make(3, 0, 10);
    CHECK(s.submit(r));
    CHECK(step(s, dev, 4));
    CHECK(r->state == kDone && r->p.launches.size() == 1 && r->p.launches[0] == 0);
}

}  // namespace

int main()
{
    test_random_stream();
    test_cancel_release_and_errors();
    test_alloc_failure_keeps_queue_order();
    test_fcfs_blocks_behind_large_request();
    test_cap_admits_into_empty_session();
    test_zero_generations();
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("scheduler: all checks passed\n");
    return 0;
}
