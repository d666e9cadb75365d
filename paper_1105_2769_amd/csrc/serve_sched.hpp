// Host-side scheduling of the serving loop (an extension: the paper has no
// serving mode).  Admission under an HBM budget and a slot limit, continuous
// batching of work units across the admitted requests, and completion
// bookkeeping.  This class makes no device calls: the executor does the
// copies and launches, and a CPU test drives it with a fake executor.
//
// Life of a request:
//   Pending   submitted, waiting in arrival (FIFO) order;
//   Admitted  holds a slot and `reserve` bytes of the budget; its points are
//             being staged and validated;
//   Running   has `units` work units, some not yet handed to a slice;
//   Draining  every unit has been handed out, some slices not yet finished;
//   Finished  every unit's slice has finished: the executor copies the result
//             back and calls release(), which frees the slot and the bytes.
//
// Cancellation (cancel()) takes a Pending request out of the queue, and makes
// a Running one Draining with the units handed out so far as its whole work,
// so it reaches Finished once those have run; the executor then releases it
// without a result.
//
// Slices.  A slice is one launch of the drain kernel over at most
// `slice_units` units.  Requests fill it in order of least remaining work
// (fewest units left to hand out), so a short request that arrives while a
// long one runs is not held behind it; ties go to the earlier arrival.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace mb {
namespace serve {

enum class State { Pending, Admitted, Running, Draining, Finished };

// What cancel() did: Removed - a Pending request left the queue and the
// scheduler (it holds nothing); Finished - a Running request has no unit left
// on the device: release it now; Later - it finishes (Admitted: the executor
// drops it when its staging lands; Running or Draining: slice_done reports it
// once its handed-out units have run); Ignored - unknown, or already Finished.
enum class Cancel { Removed, Finished, Later, Ignored };

struct Range {
    int64_t id;
    int slot;
    int64_t u0, u1;  // units [u0, u1) of the request
};

struct Slice {
    int64_t seq = -1;
    int64_t units = 0;
    std::vector<Range> ranges;
    bool empty() const { return ranges.empty(); }
};

class Scheduler {
public:
    Scheduler(int64_t budget_bytes, int max_slots, int64_t slice_units)
        : budget_(budget_bytes), max_slots_(max_slots), slice_units_(slice_units) {
        for (int s = max_slots - 1; s >= 0; --s) free_slots_.push_back(s);
    }

    int64_t budget() const { return budget_; }
    int64_t reserved() const { return reserved_; }
    int64_t peak_reserved() const { return peak_reserved_; }
    int active() const { return max_slots_ - (int)free_slots_.size(); }
    int peak_active() const { return peak_active_; }
    size_t pending() const { return fifo_.size(); }
    int64_t slice_units() const { return slice_units_; }
    void set_slice_units(int64_t u) { slice_units_ = u < 1 ? 1 : u; }
    bool idle() const { return reqs_.empty(); }
    bool has_runnable() const {
        for (const auto &kv : reqs_)
            if (kv.second.state == State::Running) return true;
        return false;
    }
    int slot_of(int64_t id) const { return reqs_.at(id).slot; }
    State state_of(int64_t id) const { return reqs_.at(id).state; }
    bool known(int64_t id) const { return reqs_.count(id) != 0; }

    // A request that needs more than the whole budget can never be admitted.
    bool can_ever_fit(int64_t reserve) const { return reserve <= budget_ && max_slots_ > 0; }

    void enqueue(int64_t id, int64_t reserve) {
        Req r;
        r.reserve = reserve;
        reqs_[id] = r;
        fifo_.push_back(id);
    }

    // Admit from the head of the queue while a slot and the bytes are free.
    // Arrival order is kept: a request that does not fit blocks the ones
    // behind it, so a large request cannot be starved by small ones.
    std::vector<int64_t> admit() {
        std::vector<int64_t> out;
        while (!fifo_.empty() && !free_slots_.empty()) {
            Req &r = reqs_.at(fifo_.front());
            if (reserved_ + r.reserve > budget_) break;
            r.slot = free_slots_.back();
            free_slots_.pop_back();
            r.state = State::Admitted;
            reserved_ += r.reserve;
            peak_reserved_ = std::max(peak_reserved_, reserved_);
            peak_active_ = std::max(peak_active_, active());
            out.push_back(fifo_.front());
            fifo_.pop_front();
        }
        return out;
    }

    // Staging done: the request has `units` units (>= 1) and keeps `reserve`
    // bytes (<= what admission reserved).
    void start(int64_t id, int64_t units, int64_t reserve) {
        Req &r = reqs_.at(id);
        if (reserve < r.reserve) {
            reserved_ -= r.reserve - reserve;
            r.reserve = reserve;
        }
        r.units = units;
        r.state = units > 0 ? State::Running : State::Finished;
    }

    // The request needs no device work (an error, or n < 3).
    void finish_now(int64_t id) { reqs_.at(id).state = State::Finished; }

    Cancel cancel(int64_t id) {
        auto it = reqs_.find(id);
        if (it == reqs_.end()) return Cancel::Ignored;
        Req &r = it->second;
        switch (r.state) {
        case State::Pending:
            fifo_.erase(std::find(fifo_.begin(), fifo_.end(), id));
            reqs_.erase(it);
            return Cancel::Removed;
        case State::Running:
            r.units = r.issued;
            if (r.in_flight == 0) {  // every handed-out unit has run
                r.state = State::Finished;
                return Cancel::Finished;
            }
            r.state = State::Draining;
            return Cancel::Later;
        case State::Admitted:
        case State::Draining:
            return Cancel::Later;
        case State::Finished:
            break;
        }
        return Cancel::Ignored;
    }

    Slice next_slice() {
        Slice sl;
        std::vector<std::pair<int64_t, int64_t>> order;  // (units left to hand out, id)
        for (const auto &kv : reqs_)
            if (kv.second.state == State::Running)
                order.emplace_back(kv.second.units - kv.second.issued, kv.first);
        std::sort(order.begin(), order.end());
        int64_t room = slice_units_;
        for (const auto &o : order) {
            if (room <= 0) break;
            Req &r = reqs_.at(o.second);
            const int64_t take = std::min(room, r.units - r.issued);
            sl.ranges.push_back(Range{o.second, r.slot, r.issued, r.issued + take});
            r.issued += take;
            room -= take;
            sl.units += take;
            r.in_flight += 1;
            if (r.issued == r.units) r.state = State::Draining;
        }
        if (!sl.empty()) sl.seq = next_seq_++;
        return sl;
    }

    // The slice's kernels have finished.  Returns the requests that are
    // now Finished.
    std::vector<int64_t> slice_done(const Slice &sl) {
        std::vector<int64_t> out;
        for (const auto &rg : sl.ranges) {
            Req &r = reqs_.at(rg.id);
            r.done += rg.u1 - rg.u0;
            r.in_flight -= 1;
            if (r.state == State::Draining && r.in_flight == 0 && r.done == r.units) {
                r.state = State::Finished;
                out.push_back(rg.id);
            }
        }
        return out;
    }

    // Result copied back: the slot and the bytes return to the pool.
    void release(int64_t id) {
        auto it = reqs_.find(id);
        if (it == reqs_.end()) return;
        if (it->second.slot >= 0) {
            free_slots_.push_back(it->second.slot);
            reserved_ -= it->second.reserve;
        }
        reqs_.erase(it);
    }

    // Units handed out and finished for one request (for checks).
    int64_t units_of(int64_t id) const { return reqs_.at(id).units; }
    int64_t done_of(int64_t id) const { return reqs_.at(id).done; }

private:
    struct Req {
        State state = State::Pending;
        int slot = -1;
        int64_t reserve = 0;
        int64_t units = 0, issued = 0, done = 0;
        int in_flight = 0;
    };
    int64_t budget_;
    int max_slots_;
    int64_t slice_units_;
    int64_t reserved_ = 0, peak_reserved_ = 0;
    int peak_active_ = 0;
    int64_t next_seq_ = 0;
    std::vector<int> free_slots_;
    std::deque<int64_t> fifo_;
    std::map<int64_t, Req> reqs_;
};

}  // namespace serve
}  // namespace mb
