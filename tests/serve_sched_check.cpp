// CPU check of the serving scheduler with a fake executor: random arrivals,
// sizes, slice limits, slices that stay in flight for a while, and
// cancellations in every state; every step checks the invariants the device
// side relies on.  Built and run by test_serve_sched.py (host compiler only).
#include "serve_sched.hpp"

#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <set>

using namespace mb::serve;

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);       \
            std::exit(1);                                          \
        }                                                          \
    } while (0)

int main(int argc, char **argv) {
    const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1;
    std::mt19937_64 g(seed);
    const int64_t budget = 1000;
    const int slots = 1 + (int)(g() % 6);
    Scheduler s(budget, slots, 1 + (int64_t)(g() % 40));
    struct Rec {
        int64_t reserve, keep, units;
        std::vector<char> seen;  // each unit issued once
        bool admitted = false, started = false, finished = false, released = false;
        bool cancel_marked = false, cancelled = false;
    };
    std::vector<Rec> recs;
    std::set<int> used_slots;
    std::vector<int64_t> admit_order, finish_order;
    int64_t next_id = 0, ticks = 0, degenerate = 0, cancelled = 0;
    const int n_req = 300;
    std::vector<int64_t> admitted_not_started;
    std::deque<Slice> inflight;
    // the executor releases a request exactly once
    auto release = [&](int64_t id) {
        Rec &r = recs[id];
        CHECK(!r.released);
        used_slots.erase(s.slot_of(id));
        s.release(id);
        r.released = true;
    };
    while ((int64_t)finish_order.size() + degenerate + cancelled < n_req || next_id < n_req) {
        CHECK(++ticks < 1000000);
        // arrivals
        const int arrive = (int)(g() % 3);
        for (int a = 0; a < arrive && next_id < n_req; ++a) {
            Rec r;
            r.reserve = 1 + (int64_t)(g() % 400);
            r.keep = 1 + (int64_t)(g() % r.reserve);
            r.units = (g() % 10 == 0) ? 0 : 1 + (int64_t)(g() % 200);
            r.seen.assign(r.units, 0);
            CHECK(s.can_ever_fit(r.reserve));
            s.enqueue(next_id, r.reserve);
            recs.push_back(r);
            ++next_id;
        }
        if (g() % 7 == 0) s.set_slice_units(1 + (int64_t)(g() % 60));
        // admission: arrival order, budget and slots respected
        for (int64_t id : s.admit()) {
            CHECK(!recs[id].admitted);
            recs[id].admitted = true;
            // arrival order: the requests skipped left the queue by cancellation
            for (int64_t q = admit_order.empty() ? 0 : admit_order.back() + 1; q < id; ++q)
                CHECK(recs[q].cancelled && !recs[q].admitted);
            CHECK(admit_order.empty() || id > admit_order.back());
            admit_order.push_back(id);
            const int slot = s.slot_of(id);
            CHECK(slot >= 0 && slot < slots);
            CHECK(used_slots.insert(slot).second);
            admitted_not_started.push_back(id);
        }
        CHECK(s.reserved() <= budget);
        CHECK(s.active() <= slots);
        // staging finishes for some admitted requests; units == 0 stands for a
        // request rejected on the device (degenerate points)
        std::vector<int64_t> still;
        for (int64_t id : admitted_not_started) {
            if (g() % 2) {
                still.push_back(id);
                continue;
            }
            Rec &r = recs[id];
            if (r.cancel_marked) {  // cancelled while staging: dropped
                release(id);
                r.cancelled = true;
                ++cancelled;
            } else if (r.units == 0) {
                s.finish_now(id);
                release(id);
                ++degenerate;
            } else {
                s.start(id, r.units, r.keep);
                r.started = true;
            }
        }
        admitted_not_started.swap(still);
        CHECK(s.reserved() <= budget);
        // one slice
        Slice sl = s.next_slice();
        CHECK(sl.units <= s.slice_units());
        int64_t prev_left = -1;
        std::vector<int64_t> ids_in_slice;
        for (const Range &rg : sl.ranges) {
            // a request appears at most once per slice
            for (int64_t other : ids_in_slice) CHECK(other != rg.id);
            ids_in_slice.push_back(rg.id);
            Rec &r = recs[rg.id];
            CHECK(r.started && !r.finished && !r.cancel_marked);
            CHECK(rg.slot == s.slot_of(rg.id));
            CHECK(rg.u0 < rg.u1 && rg.u1 <= r.units);
            for (int64_t u = rg.u0; u < rg.u1; ++u) {
                CHECK(!r.seen[u]);
                r.seen[u] = 1;
            }
            (void)prev_left;
        }
        if (!sl.empty()) inflight.push_back(sl);
        // slices finish in order, up to three in flight
        while (!inflight.empty() && (inflight.size() > 3 || g() % 2)) {
            for (int64_t id : s.slice_done(inflight.front())) {
                Rec &r = recs[id];
                CHECK(!r.finished);
                r.finished = true;
                if (r.cancel_marked) {  // its handed-out units have run
                    r.cancelled = true;
                    ++cancelled;
                } else {
                    for (char c : r.seen) CHECK(c);
                    finish_order.push_back(id);
                }
                release(id);
            }
            inflight.pop_front();
        }
        // a cancellation of a random request, in whatever state it is
        if (next_id > 0 && g() % 6 == 0) {
            const int64_t id = (int64_t)(g() % (uint64_t)next_id);
            Rec &r = recs[id];
            const Cancel c = s.cancel(id);
            switch (c) {
            case Cancel::Removed:
                CHECK(!r.admitted && !r.released);
                CHECK(!s.known(id));
                r.released = r.cancelled = true;
                ++cancelled;
                break;
            case Cancel::Finished:
                CHECK(r.started && !r.finished && !r.cancel_marked);
                for (const Slice &q : inflight)
                    for (const Range &rg : q.ranges) CHECK(rg.id != id);
                r.finished = r.cancelled = true;
                ++cancelled;
                release(id);
                break;
            case Cancel::Later:
                CHECK(r.admitted && !r.released);
                r.cancel_marked = true;
                break;
            case Cancel::Ignored:
                CHECK(r.released);
                break;
            }
        }
    }
    CHECK(inflight.empty());
    for (const Rec &r : recs) {
        CHECK(r.released);
        if (!r.cancelled)
            for (char c : r.seen) CHECK(c);
    }
    CHECK(s.idle());
    CHECK(s.reserved() == 0);
    CHECK(s.peak_reserved() <= budget);
    CHECK(cancelled > 0);
    std::printf("OK seed=%u slots=%d finished=%zu degenerate=%lld cancelled=%lld ticks=%lld peak=%lld\n",
                seed, slots, finish_order.size(), (long long)degenerate, (long long)cancelled,
                (long long)ticks, (long long)s.peak_reserved());
    return 0;
}
