// Host bookkeeping of the serving drain ring (an extension: the paper has no
// serving mode).  Host arithmetic only, so that a CPU test can drive it
// against a simulated drain kernel.
//
// Protocol.  Work items are numbered 0, 1, 2, ... in the order the host
// publishes them; item k lives in ring entry k mod cap.  The host writes
// the entry, then advances `tail` (release).  Each workgroup of the drain
// kernel takes a ticket k from a device counter `head` (atomic add), waits
// until k < tail, runs item k and sets done[k mod cap] (release).  A
// workgroup that finds nothing to do for a bounded time, or sees the stop
// flag, exits while holding its ticket; the kernel ends when all have.
//
// The host consumes finished items in any order, and reuses an entry only
// after its item is consumed.  After the kernel has ended, the device
// counter says which tickets were taken: a published item with a ticket
// below it that never finished was abandoned by an exiting workgroup and is
// published again under a new number; numbers that were taken but never
// published are skipped.  The next kernel continues from the device counter.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace mb {
namespace serve {

template <typename P>
class RingBook {
public:
    // guard: how many entries past the tail collect() checks for stray done
    // flags (default: all free entries)
    explicit RingBook(int64_t cap, int64_t guard = -1)
        : cap_(cap), guard_(guard < 0 ? cap : guard), ent_(cap), state_(cap, kFree) {}

    int64_t cap() const { return cap_; }
    int64_t tail() const { return tail_; }
    int64_t oldest() const { return oldest_; }
    // entries free for new items
    int64_t room() const { return cap_ - (tail_ - oldest_); }
    // published items not yet consumed
    int64_t outstanding() const { return outstanding_; }

    // Place an item at the tail; returns its number.  room() must be > 0.
    // The caller writes the payload to ring entry (number mod cap) before it
    // publishes the new tail.
    int64_t push(const P &p) {
        const int64_t k = tail_++;
        ent_[k % cap_] = p;
        state_[k % cap_] = kPublished;
        ++outstanding_;
        return k;
    }
    const P &payload(int64_t k) const { return ent_[k % cap_]; }

    // Consume every published item whose done flag is set: on_done(payload)
    // for each; done(e) returns entry e's flag and clears it for the entry's
    // next use.  Returns false if a flag is set on a free entry within the
    // guard window past the tail (the kernel ran something it was not given).
    template <typename Flags, typename F>
    bool collect(Flags &&done, F &&on_done) {
        for (int64_t k = oldest_; k < tail_; ++k) {
            const int64_t e = k % cap_;
            if (state_[e] == kPublished && done(e)) {
                state_[e] = kConsumed;
                --outstanding_;
                on_done(ent_[e]);
            }
        }
        for (int64_t k = tail_; k < std::min(oldest_ + cap_, tail_ + guard_); ++k)
            if (done(k % cap_)) return false;
        advance();
        return true;
    }

    // The kernel has ended with its ticket counter at `head`.  Call after a
    // final collect().  Abandoned items are published again (their new
    // numbers come from push); taken but unpublished numbers are skipped.
    // Needs room for the items republished: at most one per workgroup.
    // Returns how many were republished.
    int64_t after_exit(int64_t head) {
        std::vector<P> again;
        const int64_t hi = std::min(tail_, head);
        for (int64_t k = oldest_; k < hi; ++k) {
            const int64_t e = k % cap_;
            if (state_[e] == kPublished) {
                again.push_back(ent_[e]);
                state_[e] = kVoid;
                --outstanding_;
            }
        }
        while (tail_ < head) state_[tail_++ % cap_] = kVoid;
        advance();
        for (const P &p : again) push(p);
        return (int64_t)again.size();
    }

private:
    enum : uint8_t { kFree, kPublished, kConsumed, kVoid };
    void advance() {
        while (oldest_ < tail_ &&
               (state_[oldest_ % cap_] == kConsumed || state_[oldest_ % cap_] == kVoid))
            state_[oldest_++ % cap_] = kFree;
    }
    int64_t cap_, guard_;
    int64_t oldest_ = 0, tail_ = 0, outstanding_ = 0;
    std::vector<P> ent_;
    std::vector<uint8_t> state_;
};

}  // namespace serve
}  // namespace mb
