// Serving loop (an extension: the paper has no serving mode).  Requests of
// different N arrive on the host; a scheduler thread admits them under an
// HBM budget and a slot limit, stages and validates their points on the
// device while earlier requests compute, and drains the work units of all
// admitted requests together through one persistent drain kernel: its
// workgroups take (request, block triple) items from a ring in device
// memory that the scheduler thread keeps filled by copies from pinned host
// memory, run the exhaustive-sum tile code on them and flag each item done
// in pinned host memory (serve_ring.hpp gives the protocol).  A request finishes when every one of its units has run; its
// Phi is then copied back to the host.
//
// The drain kernel stays resident while there is work and for a bounded
// idle time after it; it exits when all its workgroups have been idle that
// long at once (or at shutdown), and the scheduler launches it again when
// work arrives.  It leaves a few CUs free, so that staging (copy in,
// validation, tables) and finishing (binary64 repairs, copy out) of
// requests, which run on a second stream, are never held behind it.  The
// scheduler thread enqueues those and polls per-slot events, so it never
// blocks on the device.
#include "direct_tile.hpp"
#include "lock_check.hpp"
#include "mb_internal.hpp"
#include "serve_ring.hpp"
#include "serve_sched.hpp"
#include "serve_sizes.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <queue>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace mb {
namespace {

struct ServeDesc {
    const double *x;
    double *phi;
    const void *tab;
    int32_t n, na;
    double scale, out_scale;
    int32_t f64, pad;  // tile type: binary64 if nonzero
};

// A work item: the slot word (slot in the low kSlotBits bits, the slot's
// generation above them, bumped for each request the slot holds) and the
// unit's I block, J block and K tile.
struct ServeItem {
    int32_t slot, a, b, t;
};
static_assert(sizeof(ServeItem) == 16 && sizeof(ServeDesc) == 56, "8-byte words for system_load");
constexpr int kSlotBits = 12;  // max_slots <= 4096
constexpr int32_t kSlotMask = (1 << kSlotBits) - 1;
constexpr uint32_t kGenMask = (1u << (31 - kSlotBits)) - 1;  // slot words stay >= 0

// Load a small struct at a wave-uniform address and mark every word uniform,
// so that pointers and sizes read from it live in SGPRs (the loop's atomics
// keep the compiler from proving the loads scalar by itself).
template <typename S>
__device__ __forceinline__ S uniform_load(const S *p) {
    static_assert(sizeof(S) % 4 == 0, "word-sized struct");
    constexpr int W = sizeof(S) / 4;
    const unsigned *w = reinterpret_cast<const unsigned *>(p);
    unsigned v[W];
#pragma unroll
    for (int e = 0; e < W; ++e) v[e] = __builtin_amdgcn_readfirstlane(w[e]);
    S out;
    __builtin_memcpy(&out, v, sizeof(S));
    return out;
}

// Control words of the drain ring.  They, the ring entries and the request
// descriptors live in fine-grained (coherent) pinned host memory: the host
// writes them with plain stores (the tail last, with release order), and the
// kernel reads them at system scope over the host link while it runs.  Device
// memory from hipMalloc is coarse-grained: a running kernel is guaranteed to
// see what a copy wrote there only at a dispatch boundary, and a polled line
// can keep being served stale from a cache.
struct DrainCtl {
    unsigned long long tail;  // items [0, tail) are published
    unsigned int stop;        // set at shutdown
    unsigned int pad[13];
};

// The drain ring's device side: the ticket counter and the idle count,
// device-scope atomics among the workgroups; the host reads head after the
// kernel has ended.
struct DrainDev {
    unsigned long long head;  // next ticket; continues across launches
    unsigned int idle;        // workgroups waiting past the idle limit
    unsigned int closing;     // they all were at once: every workgroup exits
};

struct DrainArgs {
    const DrainCtl *ctl;
    const ServeItem *ring;  // coherent host memory, cap entries
    const ServeDesc *desc;  // coherent host memory, one per slot
    unsigned int *done;     // host memory, cap flags
    DrainDev *dev;
    unsigned int cap, grid;
    int n_slots, pad;
    unsigned long long idle_ticks, hard_ticks;  // wall-clock ticks
};

#ifndef MB_DRAIN_POLL_ACQUIRE
#define MB_DRAIN_POLL_ACQUIRE 1
#endif
#ifndef MB_DRAIN_DONE_RELEASE
#define MB_DRAIN_DONE_RELEASE 1
#endif
constexpr int kPollOrder = MB_DRAIN_POLL_ACQUIRE ? __ATOMIC_ACQUIRE : __ATOMIC_RELAXED;
constexpr int kDoneOrder = MB_DRAIN_DONE_RELEASE ? __ATOMIC_RELEASE : __ATOMIC_RELAXED;

// Done flag values: the unit ran, or the item was refused as out of range.
constexpr unsigned kDoneRan = 1, kDoneRefused = 2;

// Whether an item names a unit of its request (bounds of the tile code).
template <typename T>
__device__ __forceinline__ bool item_in_range(const ServeItem &it, const ServeDesc &d) {
    return d.x != nullptr && d.n >= 3 && it.a >= 0 && it.a < d.na && it.b >= 0 &&
           (int64_t)it.b * kB < d.n && it.t >= 0 && (int64_t)it.t * DirectLds<T>::KT < d.n &&
           (int64_t)d.na * DirectLds<T>::IB >= d.n;
}

__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// A struct of 8-byte words from host memory at system scope, made
// wave-uniform: lane l of the wave loads word l, so the whole struct is one
// vector load and one round trip over the host link.
template <typename S>
__device__ __forceinline__ S system_load(const S *p, int lane) {
    static_assert(sizeof(S) % 8 == 0 && sizeof(S) / 8 <= 64, "8-byte words, one per lane");
    constexpr int W = sizeof(S) / 8;
    const unsigned long long *w = reinterpret_cast<const unsigned long long *>(p);
    unsigned long long v = 0;
    if (lane < W) v = __hip_atomic_load(w + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    unsigned u[2 * W];
#pragma unroll
    for (int e = 0; e < W; ++e) {
        u[2 * e] = __builtin_amdgcn_readlane((unsigned)v, e);
        u[2 * e + 1] = __builtin_amdgcn_readlane((unsigned)(v >> 32), e);
    }
    S out;
    __builtin_memcpy(&out, u, sizeof(S));
    return out;
}

// vmcnt(0), the other counters left alone: this wave's stores and atomics
// have been performed.
__device__ __forceinline__ void wait_vm_all() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_sched_barrier(0);
}

template <typename T, typename L>
__device__ __forceinline__ void drain_unit(L &s, const ServeItem &it, const ServeDesc &d) {
    constexpr int IB = DirectLds<T>::IB;
    // the tables are written before their items are published and only read
    using CT = __attribute__((address_space(4))) const T;
    CT *blk = (CT *)static_cast<const T *>(d.tab) +
              ((int64_t)it.b * d.na + it.a) * (IB * kB * kPairVals);
    direct_unit<T, CT *>(s, d.x, d.n, it.a, it.b, it.t, blk, d.scale, d.out_scale, d.phi);
}

// The persistent drain.  Wave 0 of a workgroup takes a ticket and waits for
// it to be published, for the stop flag, or until every workgroup has
// waited longer than idle_ticks at once (then all exit); hard_ticks bounds
// any single wait.  Every condition it branches on is wave-uniform, and all
// 64 lanes of wave 0 take part in the ticket and flag updates (lane 0 adds
// 1, the others 0), so no lane-divergent region meets the loop's back edge.
// After a unit each wave waits for its own atomics, the workgroup meets at a
// barrier, and wave 0 sets the item's done flag with a system-scope release
// store, which writes the L2 back first: the host sees the flag only after
// the unit's sums have reached memory.
__global__ __launch_bounds__(512, 1) void drain_kernel(DrainArgs a) {
    static_assert(DirectLds<float>::TPB == 512 && DirectLds<double>::TPB == 512,
                  "one block size for both tile types");
    __shared__ union {
        DirectLds<float> f;
        DirectLds<double> d;
    } s;
    __shared__ ServeItem s_it;
    __shared__ ServeDesc s_d;
    __shared__ unsigned long long s_tk;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr unsigned long long kExit = ~0ull;
    // wave 0: the largest tail read so far (the tail only grows), so that the
    // host word is read over the link only when the ticket is past it; and
    // the descriptor of the last item's slot word
    unsigned long long seen = 0;
    int32_t dkey = -1;
    ServeDesc dcache{};
    for (;;) {
        if (wave == 0) {
            const unsigned long long tk =
                uniform64(atomicAdd(&a.dev->head, lane == 0 ? 1ull : 0ull));  // lane 0's
            unsigned long long res = tk;
            const unsigned long long t0 = wall_clock64();
            bool counted = false;
            int polls = 0;
            for (;;) {
                if (tk >= seen)
                    seen = uniform64(
                        __hip_atomic_load(&a.ctl->tail, kPollOrder, __HIP_MEMORY_SCOPE_SYSTEM));
                if (tk < seen) {
                    if (counted) atomicSub(&a.dev->idle, lane == 0 ? 1u : 0u);
                    break;
                }
                const unsigned closing = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                    &a.dev->closing, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                const unsigned stop = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(&a.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
                if (stop || closing) {
                    res = kExit;
                    break;
                }
                const unsigned long long dt = (unsigned long long)wall_clock64() - t0;
                if (!counted && dt > a.idle_ticks) {
                    counted = true;
                    const unsigned prev = __builtin_amdgcn_readfirstlane(
                        atomicAdd(&a.dev->idle, lane == 0 ? 1u : 0u));
                    if (prev + 1 == a.grid)
                        __hip_atomic_store(&a.dev->closing, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
                if (dt > a.hard_ticks) {
                    res = kExit;
                    break;
                }
                // short pauses first, then about 25 us between reads of the
                // host word, so that idle workgroups load the link little
                if (polls < 16) {
                    ++polls;
                    __builtin_amdgcn_s_sleep(63);
                } else {
#pragma unroll
                    for (int z = 0; z < 8; ++z) __builtin_amdgcn_s_sleep(127);
                }
            }
            if (res != kExit) {
                ServeItem it = system_load(a.ring + res % a.cap, lane);
                // the descriptor is read again only when the slot or its
                // generation changes (a slot's next request has a new one)
                const int slot = it.slot & kSlotMask;
                if (it.slot >= 0 && slot < a.n_slots && it.slot != dkey) {
                    dcache = system_load(a.desc + slot, lane);
                    dkey = it.slot;
                }
                s_it = it;  // every lane of the wave writes the same value
                s_d = it.slot == dkey ? dcache : ServeDesc{};
            }
            s_tk = res;
        }
        __syncthreads();
        const unsigned long long tk = uniform64(s_tk);
        if (tk == kExit) break;
        const ServeItem it = uniform_load(&s_it);
        const ServeDesc d = uniform_load(&s_d);
        // an item outside its request's units is refused, not run
        const bool ok = it.slot >= 0 && (it.slot & kSlotMask) < a.n_slots &&
                        (d.f64 ? item_in_range<double>(it, d) : item_in_range<float>(it, d));
        if (ok) {
            if (d.f64)
                drain_unit<double>(s.d, it, d);
            else
                drain_unit<float>(s.f, it, d);
        }
        wait_vm_all();
        __syncthreads();
        if (wave == 0)
            __hip_atomic_store(a.done + tk % a.cap, ok ? kDoneRan : kDoneRefused,
                               kDoneOrder, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}


// Unit enumeration of the exhaustive sum for one request and tile type.
struct UnitMap {
    int ib = 0, kr = 1, na = 0, nb = 0, nt = 0;
    std::vector<int64_t> off;  // units of J blocks < b
    template <typename T>
    void build(int64_t n) {
        ib = DirectLds<T>::IB;
        kr = DirectLds<T>::KR;
        na = (int)((n + ib - 1) / ib);
        nb = (int)((n + kB - 1) / kB);
        nt = (int)((n + DirectLds<T>::KT - 1) / DirectLds<T>::KT);
        off.assign(nb + 1, 0);
        for (int b = 0; b < nb; ++b) off[b + 1] = off[b] + (int64_t)units_a(b, ib, na) * (nt - b / kr);
    }
    int64_t units() const { return off.empty() ? 0 : off.back(); }
    void decode(int64_t u, int &a, int &b, int &t) const {
        b = (int)(std::upper_bound(off.begin(), off.end(), u) - off.begin()) - 1;
        const int64_t rem = u - off[b];
        const int tc = nt - b / kr;
        a = (int)(rem / tc);
        t = b / kr + (int)(rem % tc);
    }
};

// The exhaustive sum's table shapes of the two tile types.
const serve::TableShape kTab32{DirectLds<float>::IB, kB, 4, kPairVals};
const serve::TableShape kTab64{DirectLds<double>::IB, kB, 8, kPairVals};

// Device bytes a request holds while admitted: its whole chunk (points, Phi,
// near-field magnitudes and a table region that fits either tile type).
int64_t footprint(int64_t n) { return serve::chunk_layout(n, kTab32, kTab64).total; }

// Pinned host memory for requests' points and results.  Allocating pinned
// memory waits for the whole device, which here means for the resident
// drain kernel, so it is carved from blocks that are kept: one free list
// per power-of-two size, refilled a block of at least 1 MiB at a time.
class PinnedPool {
public:
    PinnedPool() = default;
    PinnedPool(const PinnedPool &) = delete;
    PinnedPool &operator=(const PinnedPool &) = delete;
    ~PinnedPool() {
        for (void *b : blocks_) (void)hipHostFree(b);
    }
    // A buffer of at least `bytes` bytes (null on failure).
    void *get(size_t bytes) {
        const int c = size_class(bytes);
        std::vector<void *> &fl = free_[c];
        if (fl.empty()) {
            const size_t sz = (size_t)1 << c;
            const size_t per = std::max<size_t>(1, ((size_t)1 << 20) / sz);
            void *b = nullptr;
            if (hipHostMalloc(&b, sz * per, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            blocks_.push_back(b);
            for (size_t e = per; e-- > 0;) fl.push_back(static_cast<char *>(b) + e * sz);
        }
        void *p = fl.back();
        fl.pop_back();
        size_of_[p] = c;
        return p;
    }
    size_t blocks() const { return blocks_.size(); }
    void put(void *p) {
        if (!p) return;
        auto it = size_of_.find(p);
        if (it == size_of_.end()) return;
        free_[it->second].push_back(p);
        size_of_.erase(it);
    }

private:
    static int size_class(size_t bytes) {
        int c = 12;  // 4 KiB at least
        while (((size_t)1 << c) < bytes) ++c;
        return c;
    }
    std::map<int, std::vector<void *>> free_;
    std::map<void *, int> size_of_;
    std::vector<void *> blocks_;
};

struct Request {
    int64_t id = 0, n = 0;
    int prec_req = MB_FP32C, prec = MB_FP32C;
    std::vector<double> x, phi;
    mb_status status = MB_OK;
    std::string msg;
    double t_submit = 0.0, t_done = 0.0;
    int32_t timeout_ms = 0;  // the server's time limit when it was submitted (0: none)
    bool done = false, fetched = false;
    // device side, owned by the scheduler thread
    void *chunk = nullptr;
    double *dx = nullptr, *dphi = nullptr, *dmag = nullptr;
    void *dtab = nullptr;
    int64_t tab_bytes = 0;  // size of the table region at dtab
    double scale = 1.0, out_scale = 1.0;
    UnitMap um;
    int64_t units = 0, keep = 0;  // from staging, applied once the tables are built
    double *pin_x = nullptr, *pin_phi = nullptr;  // pinned copies of the points and Phi
    bool cancel = false;     // cancelled; dropped when its device work has landed
    std::string cancel_msg;
};

class Server {
public:
    Server(int64_t budget, int max_slots, hipStream_t user)
        : sched_(budget, max_slots, 1), max_slots_(max_slots), user_stream_(user) {}

    mb_status init() {
        MB_HIP(hipGetDevice(&dev_));
        device_pool_setup();
        int cus = 0;
        MB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_));
        int occ = 0;
        MB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, drain_kernel, 512, 0));
        // every workgroup must be resident at once (the idle rule counts all
        // of them; the cooperative launch checks it); kReserveCus CUs stay
        // free for staging and finishing
        grid_ = std::max(1, std::max(1, occ) * (cus - std::min(cus / 2, kReserveCus)));
        sched_.set_slice_units(std::min<int64_t>(8 * (int64_t)grid_, kMaxSliceUnits));
        int rate_khz = 0;
        MB_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev_));
        if (rate_khz <= 0) return fail(MB_ERR_DEVICE, "no device wall clock rate");
        idle_ticks_ = (unsigned long long)rate_khz * kIdleMs;
        hard_ticks_ = (unsigned long long)rate_khz * kHardMs;
        if (user_stream_) {
            cs_ = user_stream_;
        } else {
            MB_HIP(hipStreamCreateWithFlags(&own_cs_, hipStreamNonBlocking));
            cs_ = own_cs_;
        }
        MB_HIP(hipStreamCreateWithFlags(&as_, hipStreamNonBlocking));
        MB_HIP(hipEventCreateWithFlags(&ev_k0_, hipEventDefault));
        MB_HIP(hipEventCreateWithFlags(&ev_k1_, hipEventDefault));
        // control words, ring entries, descriptors and done flags:
        // fine-grained pinned host memory, written and read while the kernel
        // runs (see DrainCtl)
        MB_HIP(hipHostMalloc((void **)&ctl_, sizeof(DrainCtl), hipHostMallocCoherent));
        MB_HIP(hipHostMalloc((void **)&done_, sizeof(unsigned) * kRingCap, hipHostMallocCoherent));
        MB_HIP(hipHostMalloc((void **)&ring_, sizeof(ServeItem) * kRingCap, hipHostMallocCoherent));
        MB_HIP(hipHostMalloc((void **)&hdesc_, sizeof(ServeDesc) * max_slots_,
                             hipHostMallocCoherent));
        std::memset((void *)ctl_, 0, sizeof(DrainCtl));
        std::memset((void *)done_, 0, sizeof(unsigned) * kRingCap);
        std::memset((void *)hdesc_, 0, sizeof(ServeDesc) * max_slots_);
        MB_HIP(hipMalloc((void **)&ddev_, sizeof(DrainDev)));
        MB_HIP(hipMemset(ddev_, 0, sizeof(DrainDev)));
        MB_HIP(hipDeviceSynchronize());
        desc_host_.assign(max_slots_, ServeDesc{});
        gen_.assign(max_slots_, 0);
        MB_HIP(hipHostMalloc(&slot_host_, sizeof(SlotHost) * max_slots_, hipHostMallocDefault));
        std::memset(slot_host_, 0, sizeof(SlotHost) * max_slots_);
        slot_ev_.assign(max_slots_, nullptr);
        for (hipEvent_t &e : slot_ev_) MB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        thread_ = std::thread([this] { loop(); });
        return MB_OK;
    }

    ~Server() {
        {
            Lock g(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
        if (thread_.joinable()) thread_.join();
        if (ctl_) {  // the kernel, if resident, exits at its next wait
            __atomic_store_n(&ctl_->stop, 1u, __ATOMIC_RELEASE);
            if (running_) (void)hipEventSynchronize(ev_k1_);
        }
        if (ev_k0_) (void)hipEventDestroy(ev_k0_);
        if (ev_k1_) (void)hipEventDestroy(ev_k1_);
        if (ddev_) (void)hipFree(ddev_);
        if (ctl_) (void)hipHostFree((void *)ctl_);
        if (ring_) (void)hipHostFree((void *)ring_);
        if (done_) (void)hipHostFree((void *)done_);
        if (hdesc_) (void)hipHostFree((void *)hdesc_);
        for (hipEvent_t e : slot_ev_)
            if (e) (void)hipEventDestroy(e);
        if (slot_host_) (void)hipHostFree(slot_host_);
        if (as_) (void)hipStreamDestroy(as_);
        if (own_cs_) (void)hipStreamDestroy(own_cs_);
    }

    mb_status submit(const double *hx, int64_t n, int prec, int64_t *id) {
        if (!id || n < 0 || (n > 0 && !hx)) return fail(MB_ERR_INVALID, "bad request");
        if (prec != MB_FP64 && prec != MB_FP32C) return fail(MB_ERR_INVALID, "unknown precision");
        if (n > (int64_t)65535 * kB) return fail(MB_ERR_UNSUPPORTED, "n must be <= 65535 * 64");
        for (int64_t e = 0; e < 3 * n; ++e)
            if (!std::isfinite(hx[e])) return fail(MB_ERR_INVALID, "non-finite coordinate");
        const int64_t need = footprint(n);
        if (n >= 3 && !sched_.can_ever_fit(need))
            return fail(MB_ERR_OOM, "request needs " + std::to_string(need) +
                                        " device bytes, more than the server's budget");
        auto r = std::make_unique<Request>();
        r->n = n;
        r->prec_req = r->prec = prec;
        r->t_submit = now_s();
        Lock g(mu_);
        if (broken_) return fail(MB_ERR_DEVICE, "server stopped after a device error: " + broken_msg_);
        r->id = next_id_++;
        r->timeout_ms = timeout_ms_;
        *id = r->id;
        stats_.submitted += 1;
        if (n < 3) {  // the empty sum
            r->phi.assign(n, 0.0);
            r->t_done = r->t_submit;
            r->done = true;
            stats_.completed += 1;
            reqs_[r->id] = std::move(r);
            cv_done_.notify_all();
            return MB_OK;
        }
        r->x.assign(hx, hx + 3 * n);
        inbox_.push_back(r->id);
        reqs_[r->id] = std::move(r);
        cv_work_.notify_all();
        return MB_OK;
    }

    mb_status poll(int64_t id, double *out, int32_t *done) {
        Lock g(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end()) return fail(MB_ERR_INVALID, "unknown request id");
        Request &r = *it->second;
        if (done) *done = r.done ? 1 : 0;
        if (!r.done) return MB_OK;
        if (r.status != MB_OK) return fail(r.status, r.msg);
        if (out) {
            if (r.fetched) return fail(MB_ERR_INVALID, "result already fetched");
            std::copy(r.phi.begin(), r.phi.end(), out);
            r.fetched = true;
            std::vector<double>().swap(r.phi);
        }
        return MB_OK;
    }

    mb_status wait(int64_t id, int32_t timeout_ms, int32_t *done) {
        Lock g(mu_);
        auto ready = [&]() MB_REQUIRES(mu_) {
            if (id < 0) return stats_.completed + stats_.failed == stats_.submitted;
            auto it = reqs_.find(id);
            return it == reqs_.end() || it->second->done;
        };
        if (id >= 0 && reqs_.find(id) == reqs_.end()) return fail(MB_ERR_INVALID, "unknown request id");
        bool ok;
        if (timeout_ms < 0) {
            cv_done_.wait(g.native(), ready);
            ok = true;
        } else {
            ok = cv_done_.wait_for(g.native(), std::chrono::milliseconds(timeout_ms), ready);
        }
        if (done) *done = ok ? 1 : 0;
        return MB_OK;
    }

    mb_status latency(int64_t id, double *sec) {
        Lock g(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end()) return fail(MB_ERR_INVALID, "unknown request id");
        if (!it->second->done) return fail(MB_ERR_INVALID, "request not finished");
        *sec = it->second->t_done - it->second->t_submit;
        return MB_OK;
    }

    void get_stats(mb_server_stats *out) {
        Lock g(mu_);
        *out = stats_;
    }

    // The scheduler thread carries the cancellation out (cancel_one).
    mb_status cancel(int64_t id) {
        Lock g(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end()) return fail(MB_ERR_INVALID, "unknown request id");
        if (!it->second->done) {
            cancels_.emplace_back(id, "cancelled");
            cv_work_.notify_all();
        }
        return MB_OK;
    }

    mb_status set_timeout(int32_t ms) {
        Lock g(mu_);
        timeout_ms_ = ms > 0 ? ms : 0;
        return MB_OK;
    }

    mb_status set_slice_units(int64_t u) {
        if (u < 1) return fail(MB_ERR_INVALID, "slice_units < 1");
        Lock g(mu_);
        slice_request_ = std::min<int64_t>(u, kMaxSliceUnits);
        return MB_OK;
    }

private:
    static constexpr int64_t kMaxSliceUnits = 1 << 16;
    static constexpr int64_t kRingCap = 1 << 18;  // ring entries (4 MiB of items)
#ifndef MB_RESERVE_CUS
#define MB_RESERVE_CUS 32
#endif
    static constexpr int kReserveCus = MB_RESERVE_CUS;  // CUs the drain kernel leaves free
    static constexpr unsigned long long kIdleMs = 20;   // idle time before the kernel exits
    static constexpr unsigned long long kHardMs = 500;  // longest single wait
    static constexpr int kMaxStalled = 50;             // launches in a row that ran nothing

    // A slice published to the ring: its ranges and how many of its units
    // have not finished.
    struct Live {
        serve::Slice sl;
        int64_t left;
    };
    struct Entry {
        int64_t seq;  // slice
        ServeItem item;
    };

    Request &req(int64_t id) {
        Lock g(mu_);
        return *reqs_.at(id);
    }

    // Mark a request finished (result or error) and wake waiters.
    void complete(Request &r, mb_status st, const std::string &msg) {
        Lock g(mu_);
        r.status = st;
        r.msg = msg;
        r.t_done = now_s();
        r.done = true;
        if (st == MB_OK) {
            stats_.completed += 1;
            const double n = (double)r.n;
            stats_.triples += n * (n - 1) * (n - 2) / 6.0;
        } else {
            stats_.failed += 1;
            if (st == MB_ERR_CANCELLED) stats_.cancelled += 1;
        }
        std::vector<double>().swap(r.x);
        cv_done_.notify_all();
    }

    // Staging, first half: allocate, copy the points in, zero Phi and enqueue
    // the validation whose result lands in the slot's pinned record.  No wait.
    mb_status stage_begin(Request &r, int slot) {
        const int64_t n = r.n;
        const serve::ChunkLayout lay = serve::chunk_layout(n, kTab32, kTab64);
        const double tm0 = now_s();
        const hipError_t me = hipMallocAsync(&r.chunk, lay.total, as_);
        tr_.malloc_ms += (now_s() - tm0) * 1e3;
        if (me != hipSuccess) {
            r.chunk = nullptr;
            (void)hipGetLastError();
            return fail(MB_ERR_OOM,
                        "device allocation of " + std::to_string(lay.total) + " bytes failed");
        }
        char *base = static_cast<char *>(r.chunk);
        r.dx = reinterpret_cast<double *>(base);
        r.dphi = reinterpret_cast<double *>(base + lay.phi);
        r.dmag = reinterpret_cast<double *>(base + lay.mag);
        r.dtab = base + lay.tab;
        r.tab_bytes = lay.tab_bytes;
        const double tp0 = now_s();
        r.pin_x = static_cast<double *>(pinned_.get(sizeof(double) * 3 * n));
        tr_.pin_ms += (now_s() - tp0) * 1e3;
        if (!r.pin_x) return fail(MB_ERR_OOM, "pinned host allocation failed");
        std::memcpy(r.pin_x, r.x.data(), sizeof(double) * 3 * n);
        MB_HIP(hipMemcpyAsync(r.dx, r.pin_x, sizeof(double) * 3 * n, hipMemcpyHostToDevice, as_));
        mb_status st = zero_doubles(r.dphi, n, as_);
        if (st != MB_OK) return st;
        // the magnitude region (>= 256 bytes) holds the device record until the
        // near-field refinement, enqueued after the record is read, zeroes it
        st = validate_enqueue(r.dx, n, as_, reinterpret_cast<ValidateOut *>(r.dmag),
                              &slot_host_[slot].v);
        if (st != MB_OK) return st;
        MB_HIP(hipEventRecord(slot_ev_[slot], as_));
        return MB_OK;
    }

    // Staging, second half (the validation record has landed): choose the tile
    // type, build the (i, j) table and the binary32 refinement.
    mb_status stage_end(Request &r, int slot, int64_t &units, int64_t &keep, std::string &why) {
        const int64_t n = r.n;
        ValidateOut v = slot_host_[slot].v;
        validate_decode(&v, n);
        double md2;
        std::memcpy(&md2, &v.min_d2_bits, sizeof md2);
        if (v.nonfinite) {
            why = "non-finite coordinate";
            return MB_ERR_INVALID;
        }
        if (!(md2 > 0.0)) {
            why = "two points coincide";
            return MB_ERR_DEGENERATE;
        }
        r.prec = r.prec_req;
        r.scale = 1.0;
        if (r.prec == MB_FP32C) {
            if (!fp32c_suitable(v, n)) {
                r.prec = MB_FP64;
                Lock g(mu_);
                stats_.fp64_fallbacks += 1;
            } else {
                r.scale = unit_scale(md2);
            }
        }
        const double s2 = r.scale * r.scale;
        r.out_scale = s2 * s2 * s2 * s2 * r.scale;
        const bool f64 = r.prec == MB_FP64;
        // the table kernel must stay inside the chunk's table region
        if (serve::table_extent(n, f64 ? kTab64 : kTab32) > r.tab_bytes) {
            why = "pair-term table larger than its region";
            return MB_ERR_DEVICE;
        }
        if (f64) r.um.build<double>(n); else r.um.build<float>(n);
        dim3 g((unsigned)r.um.na, (unsigned)r.um.nb);
        if (f64)
            pair_table_kernel<double><<<g, 256, 0, as_>>>(r.dx, (int)n, r.um.na, 0, r.scale,
                                                          static_cast<double *>(r.dtab));
        else
            pair_table_kernel<float><<<g, 256, 0, as_>>>(r.dx, (int)n, r.um.na, 0, r.scale,
                                                         static_cast<float *>(r.dtab));
        MB_HIP(hipGetLastError());
        if (!f64) {
            const mb_status fx =
                near_refine_launch(r.dx, n, r.scale, kNearFixFactor * std::sqrt(md2), r.dphi,
                                   r.dmag, as_);
            if (fx != MB_OK) return fx;
        }
        units = r.um.units();
        keep = footprint(n);  // the chunk keeps its size whichever tile type runs
        ServeDesc &d = desc_host_[slot];
        d.x = r.dx;
        d.phi = r.dphi;
        d.tab = r.dtab;
        d.n = (int32_t)n;
        d.na = r.um.na;
        d.scale = r.scale;
        d.out_scale = r.out_scale;
        d.f64 = f64 ? 1 : 0;
        d.pad = 0;
        return MB_OK;
    }

    // Publish slices while fewer than two slices' worth of units are
    // outstanding and the ring has room (with a margin for the items an
    // ending kernel leaves to republish and the tickets it skips).
    mb_status publish() {
        bool any = false;
        while (sched_.has_runnable() && book_.outstanding() < 2 * sched_.slice_units() &&
               book_.room() >= sched_.slice_units() + 4 * (int64_t)grid_) {
            serve::Slice sl = sched_.next_slice();
            if (sl.empty()) break;
            for (const auto &rg : sl.ranges) {
                Request &r = req(rg.id);
                for (int64_t u = rg.u0; u < rg.u1; ++u) {
                    ServeItem it;
                    it.slot = rg.slot | (int32_t)(gen_[rg.slot] << kSlotBits);
                    r.um.decode(u, it.a, it.b, it.t);
                    const int64_t k = book_.push(Entry{sl.seq, it});
                    ring_[k % kRingCap] = it;
                }
            }
            {
                Lock g(mu_);
                stats_.slices += 1;
                if (sl.ranges.size() > 1) stats_.mixed_slices += 1;
            }
            const int64_t seq = sl.seq, units = sl.units;
            live_[seq] = Live{std::move(sl), units};
            any = true;
        }
        if (any) publish_tail();
        return MB_OK;
    }

    // Release the ring entries written so far to the kernel: a release store
    // of the tail, after the entries (and the descriptors of their requests)
    // in program order.
    void publish_tail() {
        __atomic_store_n(&ctl_->tail, (unsigned long long)book_.tail(), __ATOMIC_RELEASE);
    }

    // Consume the done flags the kernel has set; slices whose units have all
    // run finish their requests.
    mb_status collect(std::vector<int64_t> &finished) {
        int64_t n_done = 0;
        bool refused = false;
        auto flags = [&](int64_t e) {
            const unsigned f = __atomic_load_n(&done_[e], __ATOMIC_ACQUIRE);
            if (f == 0) return false;
            refused = refused || f != kDoneRan;
            __atomic_store_n(&done_[e], 0u, __ATOMIC_RELAXED);
            return true;
        };
        auto on_done = [&](const Entry &en) {
            ++n_done;
            auto it = live_.find(en.seq);
            if (it == live_.end()) return;
            if (--it->second.left == 0) {
                for (int64_t id : sched_.slice_done(it->second.sl)) finished.push_back(id);
                live_.erase(it);
            }
        };
        if (!book_.collect(flags, on_done))
            return fail(MB_ERR_DEVICE, "the drain kernel flagged an item it was not given");
        if (refused) return fail(MB_ERR_DEVICE, "the drain kernel refused an item out of range");
        if (n_done) {
            units_done_ += n_done;
            Lock g(mu_);
            stats_.units += n_done;
        }
        return MB_OK;
    }

    // An ended kernel: republish what its exiting workgroups abandoned.
    // Outstanding work and no kernel: launch one.
    mb_status drain_lifecycle(std::vector<int64_t> &finished) {
        mb_status st;
        if (running_) {
            const hipError_t q = hipEventQuery(ev_k1_);
            if (q == hipErrorNotReady) return MB_OK;
            MB_HIP(q);
            running_ = false;
            unsigned long long head = 0;
            MB_HIP(hipMemcpyAsync(&head, &ddev_->head, sizeof head, hipMemcpyDeviceToHost, cs_));
            const double ts0 = now_s();
            MB_HIP(hipStreamSynchronize(cs_));
            tr_.sync_ms += (now_s() - ts0) * 1e3;
            if ((st = collect(finished)) != MB_OK) return st;
            // a kernel that ended with work published before its launch and
            // ran none of it saw no items: after a run of such launches the
            // server gives up rather than relaunch for ever
            stalled_ = units_at_launch_ == units_done_ && out_at_launch_ > 0 ? stalled_ + 1 : 0;
            if (stalled_ > kMaxStalled)
                return fail(MB_ERR_DEVICE, "the drain kernel ran no published item in " +
                                               std::to_string(stalled_) + " launches");
            const int64_t again = book_.after_exit((int64_t)head);
            for (int64_t k = book_.tail() - again; k < book_.tail(); ++k)
                ring_[k % kRingCap] = book_.payload(k).item;
            publish_tail();
        }
        if (!running_ && book_.outstanding() > 0) {
            // the ticket counter continues; the idle count and latch restart
            MB_HIP(hipMemsetAsync(&ddev_->idle, 0, 2 * sizeof(unsigned), cs_));
            DrainArgs a;
            a.ctl = ctl_;
            a.ring = ring_;
            a.desc = hdesc_;
            a.done = done_;
            a.dev = ddev_;
            a.cap = (unsigned)kRingCap;
            a.grid = (unsigned)grid_;
            a.n_slots = max_slots_;
            a.pad = 0;
            a.idle_ticks = idle_ticks_;
            a.hard_ticks = hard_ticks_;
            units_at_launch_ = units_done_;
            out_at_launch_ = book_.outstanding();
            MB_HIP(hipEventRecord(ev_k0_, cs_));
            // A cooperative launch: every workgroup is resident at once (the
            // idle rule counts all of them), and the kernel runs from a
            // hardware queue of its own.  Streams share hardware queues, and
            // work on a stream whose queue a plain launch of the resident
            // kernel held would wait until the kernel went idle.
            void *args[] = {(void *)&a};
            MB_HIP(hipLaunchCooperativeKernel((const void *)drain_kernel, dim3((unsigned)grid_),
                                              dim3(512), args, 0, cs_));
            MB_HIP(hipEventRecord(ev_k1_, cs_));
            running_ = true;
            Lock g(mu_);
            stats_.drain_launches += 1;
        }
        return MB_OK;
    }

    // Finishing, first half: binary64 repairs of a binary32 result, copy of
    // Phi into the slot's pinned buffer.  No wait.
    mb_status finish_begin(Request &r, int slot) {
        SlotHost &h = slot_host_[slot];
        const double tp0 = now_s();
        r.pin_phi = static_cast<double *>(pinned_.get(sizeof(double) * (size_t)r.n));
        tr_.pin_ms += (now_s() - tp0) * 1e3;
        if (!r.pin_phi) return fail(MB_ERR_OOM, "pinned host allocation failed");
        h.flagged = 0;
        if (r.prec == MB_FP32C) {
            const mb_status st = point_fp64_enqueue(r.dx, r.n, r.dmag, r.dphi, as_, &h.flagged);
            if (st != MB_OK) return st;
        }
        MB_HIP(hipMemcpyAsync(r.pin_phi, r.dphi, sizeof(double) * r.n, hipMemcpyDeviceToHost, as_));
        MB_HIP(hipEventRecord(slot_ev_[slot], as_));
        return MB_OK;
    }

    // Finishing, second half (the copy has landed).
    mb_status finish_end(int64_t id, int slot) {
        Request &r = req(id);
        SlotHost &h = slot_host_[slot];
        int64_t flagged = h.flagged;
        if (flagged > point_fix_cap(r.n)) {  // rare: redo the request in binary64
            mb_status st = point_fp64_redo_all(r.dx, r.n, r.dphi, as_);
            if (st != MB_OK) return st;
            MB_HIP(hipMemcpyAsync(r.pin_phi, r.dphi, sizeof(double) * r.n, hipMemcpyDeviceToHost, as_));
            MB_HIP(hipStreamSynchronize(as_));
            flagged = r.n;
        }
        r.phi.assign(r.pin_phi, r.pin_phi + r.n);
        pinned_.put(r.pin_phi);
        r.pin_phi = nullptr;
        pinned_.put(r.pin_x);  // the points' copy has long landed
        r.pin_x = nullptr;
        if (flagged) {
            Lock g(mu_);
            stats_.points_fp64 += flagged;
        }
        MB_HIP(hipFreeAsync(r.chunk, as_));
        r.chunk = nullptr;
        sched_.release(id);
        complete(r, MB_OK, "");
        return MB_OK;
    }

    // A cancellation or time-out, in whatever state the request is.
    void cancel_one(int64_t id, const std::string &msg) {
        Request &r = req(id);
        if (r.done || r.cancel) return;
        switch (sched_.cancel(id)) {
        case serve::Cancel::Removed:  // still queued: holds nothing
            complete(r, MB_ERR_CANCELLED, msg);
            break;
        case serve::Cancel::Finished:  // none of its units is on the device
            drop(id, MB_ERR_CANCELLED, msg);
            break;
        case serve::Cancel::Later:  // staging, or units still to run
            r.cancel = true;
            r.cancel_msg = msg;
            break;
        case serve::Cancel::Ignored:  // its result is being copied back
            break;
        }
    }

    void drop(int64_t id, mb_status st, const std::string &msg) {
        Request &r = req(id);
        if (r.chunk) (void)hipFreeAsync(r.chunk, as_);
        r.chunk = nullptr;
        pinned_.put(r.pin_x);  // dropped before its copy was issued or after it landed
        r.pin_x = nullptr;
        sched_.release(id);
        complete(r, st, msg);
    }

    mb_status step(std::vector<int64_t> &finished, bool &idle) {
        {
            Lock g(mu_);
            if (slice_request_ > 0) {
                sched_.set_slice_units(slice_request_);
                slice_request_ = 0;
            }
            for (int64_t id : inbox_) {
                const Request &r = *reqs_.at(id);
                sched_.enqueue(id, footprint(r.n));
                if (r.timeout_ms > 0)
                    deadlines_.push(Deadline{r.t_submit + 1e-3 * r.timeout_ms, id, r.timeout_ms});
            }
            inbox_.clear();
            cancel_work_.swap(cancels_);
        }
        // time-outs (earliest deadline first; requests submitted under
        // different limits reach theirs out of submission order), then
        // cancellations
        for (const double t = now_s(); !deadlines_.empty() && deadlines_.top().t <= t;) {
            cancel_work_.emplace_back(deadlines_.top().id, "timed out after " +
                                                              std::to_string(deadlines_.top().ms) +
                                                              " ms");
            deadlines_.pop();
        }
        for (const auto &c : cancel_work_) cancel_one(c.first, c.second);
        cancel_work_.clear();
        {  // wall time with units outstanding on the device
            const double t = now_s();
            if (book_.outstanding() > 0 && t_last_ > 0.0) {
                Lock g(mu_);
                stats_.busy_ms += (t - t_last_) * 1e3;
            }
            t_last_ = t;
        }
        mb_status st;
        // 1. units that have run; the kernel's end and (re)launch
        if ((st = collect(finished)) != MB_OK) return st;
        if ((st = drain_lifecycle(finished)) != MB_OK) return st;
        // 2. finished requests: enqueue their repairs and copies
        const double t0 = now_s();
        for (int64_t id : finished) {
            Request &r = req(id);
            if (r.cancel) {  // its handed-out units have run
                drop(id, MB_ERR_CANCELLED, r.cancel_msg);
                continue;
            }
            const int slot = sched_.slot_of(id);
            if ((st = finish_begin(r, slot)) != MB_OK) return st;
            finishing_.push_back(id);
        }
        finished.clear();
        // 3. copies that have landed complete their requests
        for (size_t q = 0; q < finishing_.size();) {
            const int64_t id = finishing_[q];
            const int slot = sched_.slot_of(id);
            const hipError_t e = hipEventQuery(slot_ev_[slot]);
            if (e == hipErrorNotReady) {
                ++q;
                continue;
            }
            MB_HIP(e);
            if ((st = finish_end(id, slot)) != MB_OK) return st;
            finishing_.erase(finishing_.begin() + (long)q);
        }
        const double t1 = now_s();
        // 4. admit new requests and enqueue their staging
        for (int64_t id : sched_.admit()) {
            Request &r = req(id);
            st = stage_begin(r, sched_.slot_of(id));
            if (st == MB_ERR_OOM) {  // this request only; the server goes on
                drop(id, st, last_error_cstr());
                continue;
            }
            if (st != MB_OK) return st;
            validating_.push_back(id);
        }
        // 5. validations that have landed: enqueue the tables
        for (size_t q = 0; q < validating_.size();) {
            const int64_t id = validating_[q];
            const int slot = sched_.slot_of(id);
            const hipError_t e = hipEventQuery(slot_ev_[slot]);
            if (e == hipErrorNotReady) {
                ++q;
                continue;
            }
            MB_HIP(e);
            validating_.erase(validating_.begin() + (long)q);
            Request &r = req(id);
            if (r.cancel) {
                drop(id, MB_ERR_CANCELLED, r.cancel_msg);
                continue;
            }
            std::string why;
            st = stage_end(r, slot, r.units, r.keep, why);
            if (st == MB_ERR_OOM) {
                (void)hipGetLastError();
                why = last_error_cstr();
            }
            if (st == MB_ERR_DEGENERATE || st == MB_ERR_INVALID || st == MB_ERR_OOM) {
                drop(id, st, why);
                continue;
            }
            if (st != MB_OK) return st;
            MB_HIP(hipEventRecord(slot_ev_[slot], as_));
            staging_.push_back(id);
        }
        // 6. tables built: the request's units may be published
        for (size_t q = 0; q < staging_.size();) {
            const int64_t id = staging_[q];
            const int slot = sched_.slot_of(id);
            const hipError_t e = hipEventQuery(slot_ev_[slot]);
            if (e == hipErrorNotReady) {
                ++q;
                continue;
            }
            MB_HIP(e);
            staging_.erase(staging_.begin() + (long)q);
            Request &r = req(id);
            if (r.cancel) {
                drop(id, MB_ERR_CANCELLED, r.cancel_msg);
                continue;
            }
            gen_[slot] = (gen_[slot] + 1) & kGenMask;  // items carry the slot's new word
            hdesc_[slot] = desc_host_[slot];          // written before the request's items
            sched_.start(id, r.units, r.keep);
        }
        {
            Lock g(mu_);
            stats_.finalize_ms += (t1 - t0) * 1e3;
            stats_.stage_ms += (now_s() - t1) * 1e3;
        }
        // 7. publish, and launch a kernel if none is resident
        if ((st = publish()) != MB_OK) return st;
        if ((st = drain_lifecycle(finished)) != MB_OK) return st;
        idle = book_.outstanding() == 0 && !sched_.has_runnable() && finishing_.empty() &&
               validating_.empty() && staging_.empty() && finished.empty();
        if (tr_.on) trace_line(idle);
        if (!idle) std::this_thread::sleep_for(std::chrono::microseconds(10));
        {
            Lock g(mu_);
            stats_.peak_reserved = sched_.peak_reserved();
            stats_.peak_active = sched_.peak_active();
        }
        return MB_OK;
    }

    // MB_SERVE_TRACE set: a line every 2 s on stderr with the queue depths and
    // the host time spent in the calls that can wait for the device.
    struct Trace {
        bool on = std::getenv("MB_SERVE_TRACE") != nullptr;
        double t0 = 0.0, last = 0.0;
        double malloc_ms = 0.0, pin_ms = 0.0, sync_ms = 0.0;
    } tr_;
    void trace_line(bool idle) {
        const double t = now_s();
        if (tr_.t0 == 0.0) tr_.t0 = tr_.last = t;
        if (t - tr_.last < 2.0) return;
        tr_.last = t;
        mb_server_stats st;
        get_stats(&st);
        std::fprintf(stderr,
                     "[mb serve] %.1f s: submitted %lld done %lld failed %lld units %lld "
                     "outstanding %lld launches %d running %d idle %d | validating %zu staging %zu "
                     "finishing %zu slices %zu pinned blocks %zu | ms in malloc %.0f pinned %.0f "
                     "kernel-end sync %.0f\n",
                     t - tr_.t0, (long long)st.submitted, (long long)st.completed,
                     (long long)st.failed, (long long)st.units, (long long)book_.outstanding(),
                     st.drain_launches, (int)running_, (int)idle, validating_.size(),
                     staging_.size(), finishing_.size(), live_.size(), pinned_.blocks(),
                     tr_.malloc_ms, tr_.pin_ms, tr_.sync_ms);
    }

    void loop() {
        if (hipSetDevice(dev_) != hipSuccess) {
            break_all("hipSetDevice failed in the serving thread");
            return;
        }
        std::vector<int64_t> finished;
        for (;;) {
            bool idle = false;
            mb_status st = step(finished, idle);
            if (st != MB_OK) {
                break_all(last_error_cstr());
                return;
            }
            if (idle) {
                Lock g(mu_);
                if (inbox_.empty()) {
                    if (stop_ && sched_.idle()) return;
                    cv_work_.wait_for(g.native(), std::chrono::milliseconds(2));
                }
            }
        }
    }

    // A device error ends the server: every unfinished request fails.
    void break_all(const std::string &msg) {
        Lock g(mu_);
        broken_ = true;
        broken_msg_ = msg;
        for (auto &kv : reqs_) {
            Request &r = *kv.second;
            if (r.done) continue;
            r.status = MB_ERR_DEVICE;
            r.msg = msg;
            r.t_done = now_s();
            r.done = true;
            stats_.failed += 1;
        }
        cv_done_.notify_all();
    }

    serve::Scheduler sched_;  // scheduler thread only
    int max_slots_;
    hipStream_t user_stream_ = nullptr, own_cs_ = nullptr, cs_ = nullptr, as_ = nullptr;
    int dev_ = 0, grid_ = 1;
    // the drain ring (host memory shared with the kernel) and the kernel's state
    DrainCtl *ctl_ = nullptr;
    ServeItem *ring_ = nullptr;
    unsigned *done_ = nullptr;
    ServeDesc *hdesc_ = nullptr;
    DrainDev *ddev_ = nullptr;
    int64_t units_done_ = 0, units_at_launch_ = 0, out_at_launch_ = 0;
    int stalled_ = 0;
    serve::RingBook<Entry> book_{kRingCap, 4096};
    std::map<int64_t, Live> live_;  // published slices by sequence number
    bool running_ = false;
    hipEvent_t ev_k0_ = nullptr, ev_k1_ = nullptr;
    unsigned long long idle_ticks_ = 0, hard_ticks_ = 0;
    double t_last_ = 0.0;
    // per slot: pinned validation record and repair count, and
    // an event marking when the staging or finishing work has landed
    struct SlotHost {
        ValidateOut v;
        int32_t flagged;
    };
    SlotHost *slot_host_ = nullptr;
    std::vector<hipEvent_t> slot_ev_;
    std::vector<int64_t> validating_, staging_, finishing_;
    struct Deadline {
        double t;
        int64_t id;
        int32_t ms;
    };
    struct LaterDeadline {
        bool operator()(const Deadline &a, const Deadline &b) const { return a.t > b.t; }
    };
    // earliest deadline on top; scheduler thread only
    std::priority_queue<Deadline, std::vector<Deadline>, LaterDeadline> deadlines_;
    std::vector<std::pair<int64_t, std::string>> cancel_work_;  // scheduler thread only
    std::vector<ServeDesc> desc_host_;  // per slot, written at staging
    std::vector<uint32_t> gen_;         // per slot: generation of its current request
    PinnedPool pinned_;                 // scheduler thread only
    std::thread thread_;

    // Shared between the callers' threads and the scheduler thread: only
    // with mu_ held (checked by the compiler's thread-safety analysis).
    Mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::map<int64_t, std::unique_ptr<Request>> reqs_ MB_GUARDED_BY(mu_);
    std::vector<int64_t> inbox_ MB_GUARDED_BY(mu_);
    std::vector<std::pair<int64_t, std::string>> cancels_ MB_GUARDED_BY(mu_);
    int32_t timeout_ms_ MB_GUARDED_BY(mu_) = 0;
    int64_t next_id_ MB_GUARDED_BY(mu_) = 0;
    int64_t slice_request_ MB_GUARDED_BY(mu_) = 0;
    bool stop_ MB_GUARDED_BY(mu_) = false;
    bool broken_ MB_GUARDED_BY(mu_) = false;
    std::string broken_msg_ MB_GUARDED_BY(mu_);
    mb_server_stats stats_ MB_GUARDED_BY(mu_){};
};

}  // namespace
}  // namespace mb

using namespace mb;

extern "C" {

mb_status mb_server_create(int64_t hbm_budget_bytes, int32_t max_slots, void *stream, void **srv) {
    clear_error();
    if (!srv) return fail(MB_ERR_INVALID, "null output");
    *srv = nullptr;
    if (hbm_budget_bytes <= 0 || max_slots < 1 || max_slots > 4096)
        return fail(MB_ERR_INVALID, "budget must be > 0 and 1 <= max_slots <= 4096");
    auto s = std::make_unique<Server>(hbm_budget_bytes, max_slots, (hipStream_t)stream);
    mb_status st = s->init();
    if (st != MB_OK) return st;
    *srv = s.release();
    return MB_OK;
}

mb_status mb_server_submit(void *srv, const double *host_x, int64_t n, int32_t prec,
                           int64_t *req_id) {
    clear_error();
    if (!srv) return fail(MB_ERR_INVALID, "null server");
    return static_cast<Server *>(srv)->submit(host_x, n, prec, req_id);
}

mb_status mb_server_poll(void *srv, int64_t req_id, double *host_phi, int32_t *done) {
    clear_error();
    if (!srv || !done) return fail(MB_ERR_INVALID, "null argument");
    return static_cast<Server *>(srv)->poll(req_id, host_phi, done);
}

mb_status mb_server_wait(void *srv, int64_t req_id, int32_t timeout_ms, int32_t *done) {
    clear_error();
    if (!srv) return fail(MB_ERR_INVALID, "null server");
    return static_cast<Server *>(srv)->wait(req_id, timeout_ms, done);
}

mb_status mb_server_latency(void *srv, int64_t req_id, double *seconds) {
    clear_error();
    if (!srv || !seconds) return fail(MB_ERR_INVALID, "null argument");
    return static_cast<Server *>(srv)->latency(req_id, seconds);
}

mb_status mb_server_stats_get(void *srv, mb_server_stats *out) {
    clear_error();
    if (!srv || !out) return fail(MB_ERR_INVALID, "null argument");
    static_cast<Server *>(srv)->get_stats(out);
    return MB_OK;
}

mb_status mb_server_cancel(void *srv, int64_t req_id) {
    clear_error();
    if (!srv) return fail(MB_ERR_INVALID, "null server");
    return static_cast<Server *>(srv)->cancel(req_id);
}

mb_status mb_server_set_timeout(void *srv, int32_t timeout_ms) {
    clear_error();
    if (!srv) return fail(MB_ERR_INVALID, "null server");
    return static_cast<Server *>(srv)->set_timeout(timeout_ms);
}

mb_status mb_server_set_slice_units(void *srv, int64_t units) {
    clear_error();
    if (!srv) return fail(MB_ERR_INVALID, "null server");
    return static_cast<Server *>(srv)->set_slice_units(units);
}

mb_status mb_server_destroy(void *srv) {
    clear_error();
    delete static_cast<Server *>(srv);
    return MB_OK;
}

}  // extern "C"
