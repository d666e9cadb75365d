// CPU check of the serving scheduler with a fake executor: random arrivals,
// sizes and slice limits; every step checks the invariants the device side
// relies on.  Built and run by test_serve_sched.py (host compiler only).
#include "serve_sched.hpp"

#include <cstdio>
#include <cstdlib>
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
    };
    std::vector<Rec> recs;
    std::set<int> used_slots;
    std::vector<int64_t> admit_order, finish_order;
    int64_t next_id = 0, ticks = 0, degenerate = 0;
    const int n_req = 300;
    std::vector<int64_t> admitted_not_started;
    while ((int64_t)finish_order.size() + degenerate < n_req || next_id < n_req) {
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
            CHECK(admit_order.empty() || id == admit_order.back() + 1);
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
            if (r.units == 0) {
                s.finish_now(id);
                used_slots.erase(s.slot_of(id));
                s.release(id);
                r.released = true;
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
            CHECK(r.started && !r.finished);
            CHECK(rg.slot == s.slot_of(rg.id));
            CHECK(rg.u0 < rg.u1 && rg.u1 <= r.units);
            for (int64_t u = rg.u0; u < rg.u1; ++u) {
                CHECK(!r.seen[u]);
                r.seen[u] = 1;
            }
            (void)prev_left;
        }
        for (int64_t id : s.slice_done(sl)) {
            Rec &r = recs[id];
            for (char c : r.seen) CHECK(c);
            CHECK(!r.finished);
            r.finished = true;
            finish_order.push_back(id);
            used_slots.erase(s.slot_of(id));
            s.release(id);
            r.released = true;
        }
    }
    for (const Rec &r : recs) {
        CHECK(r.released);
        for (char c : r.seen) CHECK(c);
    }
    CHECK(s.idle());
    CHECK(s.reserved() == 0);
    CHECK(s.peak_reserved() <= budget);
    std::printf("OK seed=%u slots=%d finished=%zu degenerate=%lld ticks=%lld peak=%lld\n", seed, slots,
                finish_order.size(), (long long)degenerate, (long long)ticks,
                (long long)s.peak_reserved());
    return 0;
}
