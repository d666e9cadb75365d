// CPU model of the serving drain ring (serve_ring.hpp): host threads stand
// in for the drain kernel's workgroups and follow its protocol - take a
// ticket from a shared counter, wait until the ticket is published or the
// idle rule ends the kernel, run the item, set its done flag - while the
// main thread publishes the units of many requests in slices, consumes done
// flags, and after each "kernel" ends republishes abandoned items and
// launches the next one.  Requests hold one of a few slots while they run;
// a slot's descriptor is rewritten, and its generation bumped, for each
// request it takes, and a workgroup re-reads a descriptor only when an
// item's slot word (slot and generation) differs from the last one it read.
// Checks: every unit runs exactly once and with its own request's
// descriptor, no flag appears on an unpublished entry, and the book is empty
// at the end.
// Built and run by test_serve_ring.py under ThreadSanitizer and under
// AddressSanitizer + UndefinedBehaviorSanitizer.
#include "serve_ring.hpp"

#include <atomic>
#include <chrono>
#include <cstdio>
#include <memory>
#include <random>
#include <thread>
#include <vector>

using namespace mb::serve;

struct Item {
    int req, unit;
    int64_t slice;
    int32_t slot_word;  // slot | generation << kSlotBits
};

constexpr int kSlotBits = 12;
constexpr int kMaxSlots = 5;

struct Shared {
    // host-written, kernel-read
    std::atomic<int64_t> tail{0};
    std::atomic<int> stop{0};
    std::vector<Item> ring;
    // kernel-written
    std::unique_ptr<std::atomic<uint32_t>[]> done;
    std::atomic<int64_t> head{0};
    std::atomic<int> idle{0}, closing{0};
    // what ran
    std::vector<std::unique_ptr<std::atomic<int>[]>> runs;
    // per slot: the descriptor (here the request it holds), written by the
    // host before the request's first item is published
    int desc[kMaxSlots] = {};
    std::atomic<int> wrong_desc{0};
};

// One workgroup of the drain kernel.
static void workgroup(Shared &sh, int grid, int64_t cap, int idle_spins, int hard_spins,
                      unsigned seed) {
    std::mt19937 rng(seed);
    int32_t dkey = -1;  // slot word of the cached descriptor
    int dcache = -1;
    for (;;) {
        const int64_t t = sh.head.fetch_add(1);
        int spins = 0;
        bool counted = false, run = false;
        for (;;) {
            if (t < sh.tail.load(std::memory_order_acquire)) {
                if (counted) sh.idle.fetch_sub(1);
                run = true;
                break;
            }
            if (sh.stop.load() || sh.closing.load()) break;
            ++spins;
            if (!counted && spins > idle_spins) {
                counted = true;
                if (sh.idle.fetch_add(1) + 1 == grid) sh.closing.store(1);
            }
            if (spins > hard_spins) break;
            std::this_thread::yield();
        }
        if (!run) return;  // exits holding ticket t
        const Item it = sh.ring[t % cap];
        if (it.slot_word != dkey) {
            dcache = sh.desc[it.slot_word & ((1 << kSlotBits) - 1)];
            dkey = it.slot_word;
        }
        if (dcache != it.req) sh.wrong_desc.fetch_add(1);
        sh.runs[it.req][it.unit].fetch_add(1);
        if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
        sh.done[t % cap].store(1, std::memory_order_release);
    }
}

// One run of the model with n_slots slots (1: consecutive requests share the
// slot, so only the generation tells their descriptors apart).
static int run(int n_slots) {
    const int64_t cap = 4096;
    const int grid = 6;
    std::mt19937 rng(12345);
    const int n_req = 300;
    std::vector<int> units(n_req);
    for (int r = 0; r < n_req; ++r) units[r] = 1 + (int)(rng() % 200);

    Shared sh;
    sh.ring.resize(cap);
    sh.done.reset(new std::atomic<uint32_t>[cap]);
    for (int64_t e = 0; e < cap; ++e) sh.done[e].store(0);
    for (int r = 0; r < n_req; ++r) {
        sh.runs.emplace_back(new std::atomic<int>[units[r]]);
        for (int u = 0; u < units[r]; ++u) sh.runs[r][u].store(0);
    }

    RingBook<Item> book(cap);
    std::vector<int> issued(n_req, 0), finished_units(n_req, 0), slot_of(n_req, -1);
    std::vector<int> free_slots;
    for (int q = n_slots - 1; q >= 0; --q) free_slots.push_back(q);
    uint32_t gen[kMaxSlots] = {};
    int next_req = 0, launches = 0;
    int64_t republished = 0;
    int64_t slice_seq = 0;
    std::vector<std::thread> kernel;
    auto kernel_running = [&] { return !kernel.empty(); };
    std::atomic<int> exited{0};
    auto launch = [&] {
        sh.idle.store(0);
        sh.closing.store(0);
        exited.store(0);
        ++launches;
        for (int w = 0; w < grid; ++w)
            kernel.emplace_back([&, w] {
                workgroup(sh, grid, cap, 20 + (int)(w * 37 % 60), 200000, 77u * launches + w);
                exited.fetch_add(1);
            });
    };
    auto publish_tail = [&] { sh.tail.store(book.tail(), std::memory_order_release); };
    auto flags = [&](int64_t e) {
        if (sh.done[e].load(std::memory_order_acquire)) {
            sh.done[e].store(0, std::memory_order_relaxed);
            return true;
        }
        return false;
    };
    auto on_done = [&](const Item &it) {
        if (++finished_units[it.req] == units[it.req]) free_slots.push_back(slot_of[it.req]);
    };
    int active_from = 0;
    for (int step = 0;; ++step) {
        // publish a slice of up to 64 units from the admitted requests
        if (step % 3 == 0 && next_req < n_req) ++next_req;  // arrivals
        const int64_t before = book.tail();
        int64_t room = std::min<int64_t>(64, book.room() - 2 * grid);
        for (int r = active_from; r < next_req && room > 0; ++r) {
            if (slot_of[r] < 0) {  // admit into a free slot: new generation, new descriptor
                if (free_slots.empty()) continue;
                const int q = free_slots.back();
                free_slots.pop_back();
                gen[q] = (gen[q] + 1) & 0x7FFFF;
                sh.desc[q] = r;
                slot_of[r] = q;
            }
            const int32_t word = slot_of[r] | (int32_t)(gen[slot_of[r]] << kSlotBits);
            while (issued[r] < units[r] && room > 0) {
                const int64_t k = book.push(Item{r, issued[r]++, slice_seq, word});
                sh.ring[k % cap] = book.payload(k);
                --room;
            }
        }
        if (book.tail() != before) {
            ++slice_seq;
            publish_tail();
        }
        while (active_from < next_req && issued[active_from] == units[active_from]) ++active_from;
        if (!book.collect(flags, on_done)) {
            std::printf("FAIL: done flag on an unpublished entry\n");
            return 1;
        }
        // kernel ended (all workgroups exited): republish and relaunch
        if (kernel_running() && exited.load() == grid) {
            for (auto &t : kernel) t.join();
            kernel.clear();
            if (!book.collect(flags, on_done)) {
                std::printf("FAIL: done flag on an unpublished entry\n");
                return 1;
            }
            const int64_t again = book.after_exit(sh.head.load());
            republished += again;
            for (int64_t k = book.tail() - again; k < book.tail(); ++k)
                sh.ring[k % cap] = book.payload(k);
            publish_tail();
        }
        const bool all_issued = next_req == n_req && active_from == n_req;
        if (!kernel_running() && (book.outstanding() > 0 || (!all_issued && step % 50 == 0)))
            launch();
        if (all_issued && book.outstanding() == 0) break;
        if (step % 7 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
        if (step % 40 == 0) std::this_thread::sleep_for(std::chrono::microseconds(2000));
    }
    sh.stop.store(1);
    for (auto &t : kernel) t.join();
    kernel.clear();
    long checked = 0;
    for (int r = 0; r < n_req; ++r)
        for (int u = 0; u < units[r]; ++u) {
            if (sh.runs[r][u].load() != 1) {
                std::printf("FAIL: request %d unit %d ran %d times\n", r, u, sh.runs[r][u].load());
                return 1;
            }
            ++checked;
        }
    for (int r = 0; r < n_req; ++r)
        if (finished_units[r] != units[r]) {
            std::printf("FAIL: request %d finished %d of %d units\n", r, finished_units[r], units[r]);
            return 1;
        }
    if (book.outstanding() != 0 || book.oldest() != book.tail()) {
        std::printf("FAIL: book not empty\n");
        return 1;
    }
    if (sh.wrong_desc.load() != 0) {
        std::printf("FAIL: %d units ran with another request's descriptor\n", sh.wrong_desc.load());
        return 1;
    }
    if (launches < 5) {
        std::printf("FAIL: only %d kernel launches: the relaunch path was not exercised\n", launches);
        return 1;
    }
    std::printf("OK %d slots: %ld units, %d launches, %ld items republished\n", n_slots, checked,
                launches, (long)republished);
    return 0;
}

int main() {
    for (int n_slots : {1, kMaxSlots})
        if (run(n_slots) != 0) return 1;
    return 0;
}
