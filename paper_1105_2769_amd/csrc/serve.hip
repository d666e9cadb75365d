// Serving loop (an extension: the paper has no serving mode).  Requests of
// different N arrive on the host; a scheduler thread admits them under an
// HBM budget and a slot limit, stages and validates their points on the
// device while earlier requests compute, and drains the work units of all
// admitted requests together: each slice is one launch of a drain kernel
// whose resident workgroups pop (request, block triple) items from a list
// and run the exhaustive-sum tile code on them.  A request finishes when
// every one of its units has run; its Phi is then copied back to the host.
//
// Up to two slices are queued on the compute stream.  Staging (copy in,
// validation, tables) and finishing (binary64 repairs, copy out) of
// requests run on a second stream and never block the scheduler thread: it
// enqueues them and polls per-slot events between slices, so the compute
// stream sees back-to-back slices.  Every slice ends with a count check:
// each slot's items run == items issued.
#include "direct_tile.hpp"
#include "mb_internal.hpp"
#include "serve_sched.hpp"
#include "serve_sizes.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
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
};

struct ServeItem {
    int32_t slot, a, b, t;
};

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

constexpr int kHeaderWords = 16;  // next-item counters (two used), padded to 64 B

// Resident workgroups pop items until the list is exhausted.  Every
// workgroup reaches the exit: the counter only grows.
//
// The item fetch and the count update are done by all 64 lanes of wave 0
// under a wave-uniform branch (lane 0 adds 1, the others 0), never under a
// per-lane condition: a lane-divergent region at the loop boundary can be
// merged across the back edge by the compiler so that the other lanes of
// the wave re-enter the barrier without the fetching lane, and the item
// index is then never refreshed.
template <typename T>
__global__ __launch_bounds__(DirectLds<T>::TPB, 1) void serve_kernel(const ServeDesc *__restrict__ desc,
                                                            const ServeItem *__restrict__ items,
                                                            int n_items, unsigned *__restrict__ next,
                                                            unsigned *__restrict__ counts) {
    constexpr int IB = DirectLds<T>::IB;
    __shared__ DirectLds<T> s;
    __shared__ int cur;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (;;) {
        if (wave == 0) {
            const unsigned got = atomicAdd(next, lane == 0 ? 1u : 0u);
            cur = (int)__builtin_amdgcn_readfirstlane(got);  // lane 0's old value
        }
        __syncthreads();
        // read before the unit's first barrier, so wave 0 cannot overwrite it
        // first; uniform, so the item and its descriptor sit in SGPRs
        const int idx = __builtin_amdgcn_readfirstlane(cur);
        if (idx >= n_items) break;
        const ServeItem it = uniform_load(items + idx);
        const ServeDesc d = uniform_load(desc + it.slot);
        // the tables are written before the launch and only read by it
        using CT = __attribute__((address_space(4))) const T;
        CT *blk = (CT *)static_cast<const T *>(d.tab) + ((int64_t)it.b * d.na + it.a) * (IB * kB * kPairVals);
        direct_unit<T, CT *>(s, d.x, d.n, it.a, it.b, it.t, blk, d.scale, d.out_scale, d.phi);
        if (wave == 0) atomicAdd(&counts[it.slot], lane == 0 ? 1u : 0u);
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

struct Request {
    int64_t id = 0, n = 0;
    int prec_req = MB_FP32C, prec = MB_FP32C;
    std::vector<double> x, phi;
    mb_status status = MB_OK;
    std::string msg;
    double t_submit = 0.0, t_done = 0.0;
    bool done = false, fetched = false;
    // device side, owned by the scheduler thread
    void *chunk = nullptr;
    double *dx = nullptr, *dphi = nullptr, *dmag = nullptr;
    void *dtab = nullptr;
    int64_t tab_bytes = 0;  // size of the table region at dtab
    double scale = 1.0, out_scale = 1.0;
    UnitMap um;
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
        int occ_f = 0, occ_d = 0;
        MB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_f, serve_kernel<float>, DirectLds<float>::TPB, 0));
        MB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_d, serve_kernel<double>, DirectLds<double>::TPB, 0));
        grid_f_ = std::max(1, occ_f) * cus;
        grid_d_ = std::max(1, occ_d) * cus;
        sched_.set_slice_units(std::min<int64_t>(8 * (int64_t)grid_f_, kMaxSliceUnits));
        if (user_stream_) {
            cs_ = user_stream_;
        } else {
            MB_HIP(hipStreamCreateWithFlags(&own_cs_, hipStreamNonBlocking));
            cs_ = own_cs_;
        }
        MB_HIP(hipStreamCreateWithFlags(&as_, hipStreamNonBlocking));
        MB_HIP(hipEventCreateWithFlags(&ev_adm_, hipEventDisableTiming));
        desc_table_.assign(max_slots_, ServeDesc{});
        ring_bytes_ = sizeof(unsigned) * (kHeaderWords + align_slots()) +
                      sizeof(ServeItem) * (size_t)kMaxSliceUnits;
        for (SliceBuf &b : buf_) {
            MB_HIP(hipEventCreateWithFlags(&b.ev_end, hipEventDefault));
            MB_HIP(hipEventCreateWithFlags(&b.ev_start, hipEventDefault));
            MB_HIP(hipMalloc(&b.d_desc, sizeof(ServeDesc) * max_slots_));
            MB_HIP(hipHostMalloc(&b.h_desc, sizeof(ServeDesc) * max_slots_, hipHostMallocDefault));
            MB_HIP(hipMalloc(&b.d_ring, ring_bytes_));
            MB_HIP(hipHostMalloc(&b.h_ring, ring_bytes_, hipHostMallocDefault));
            MB_HIP(hipHostMalloc(&b.h_counts, sizeof(unsigned) * max_slots_, hipHostMallocDefault));
        }
        MB_HIP(hipHostMalloc(&slot_host_, sizeof(SlotHost) * max_slots_, hipHostMallocDefault));
        std::memset(slot_host_, 0, sizeof(SlotHost) * max_slots_);
        slot_ev_.assign(max_slots_, nullptr);
        for (hipEvent_t &e : slot_ev_) MB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        thread_ = std::thread([this] { loop(); });
        return MB_OK;
    }

    ~Server() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
        if (thread_.joinable()) thread_.join();
        for (SliceBuf &b : buf_) {
            if (b.d_desc) (void)hipFree(b.d_desc);
            if (b.d_ring) (void)hipFree(b.d_ring);
            if (b.h_desc) (void)hipHostFree(b.h_desc);
            if (b.h_ring) (void)hipHostFree(b.h_ring);
            if (b.h_counts) (void)hipHostFree(b.h_counts);
            if (b.ev_end) (void)hipEventDestroy(b.ev_end);
            if (b.ev_start) (void)hipEventDestroy(b.ev_start);
        }
        if (ev_adm_) (void)hipEventDestroy(ev_adm_);
        for (hipEvent_t e : slot_ev_)
            if (e) (void)hipEventDestroy(e);
        if (slot_host_) {
            for (int q = 0; q < max_slots_; ++q)
                if (slot_host_[q].phi) (void)hipHostFree(slot_host_[q].phi);
            (void)hipHostFree(slot_host_);
        }
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
        std::lock_guard<std::mutex> g(mu_);
        if (broken_) return fail(MB_ERR_DEVICE, "server stopped after a device error: " + broken_msg_);
        r->id = next_id_++;
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
        std::lock_guard<std::mutex> g(mu_);
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
        std::unique_lock<std::mutex> g(mu_);
        auto ready = [&] {
            if (id < 0) return stats_.completed + stats_.failed == stats_.submitted;
            auto it = reqs_.find(id);
            return it == reqs_.end() || it->second->done;
        };
        if (id >= 0 && reqs_.find(id) == reqs_.end()) return fail(MB_ERR_INVALID, "unknown request id");
        bool ok;
        if (timeout_ms < 0) {
            cv_done_.wait(g, ready);
            ok = true;
        } else {
            ok = cv_done_.wait_for(g, std::chrono::milliseconds(timeout_ms), ready);
        }
        if (done) *done = ok ? 1 : 0;
        return MB_OK;
    }

    mb_status latency(int64_t id, double *sec) {
        std::lock_guard<std::mutex> g(mu_);
        auto it = reqs_.find(id);
        if (it == reqs_.end()) return fail(MB_ERR_INVALID, "unknown request id");
        if (!it->second->done) return fail(MB_ERR_INVALID, "request not finished");
        *sec = it->second->t_done - it->second->t_submit;
        return MB_OK;
    }

    void get_stats(mb_server_stats *out) {
        std::lock_guard<std::mutex> g(mu_);
        *out = stats_;
    }

    mb_status set_slice_units(int64_t u) {
        if (u < 1) return fail(MB_ERR_INVALID, "slice_units < 1");
        std::lock_guard<std::mutex> g(mu_);
        slice_request_ = std::min<int64_t>(u, kMaxSliceUnits);
        return MB_OK;
    }

private:
    static constexpr int64_t kMaxSliceUnits = 1 << 16;

    // Buffers of one slice in flight; two alternate, so that the host can
    // queue slice s + 1 while slice s runs.
    struct SliceBuf {
        ServeDesc *d_desc = nullptr, *h_desc = nullptr;
        void *d_ring = nullptr, *h_ring = nullptr;
        unsigned *h_counts = nullptr;
        hipEvent_t ev_start = nullptr, ev_end = nullptr;
    };

    size_t align_slots() const { return (size_t)((max_slots_ + 15) / 16) * 16; }
    static unsigned *d_header(const SliceBuf &b) { return static_cast<unsigned *>(b.d_ring); }
    static unsigned *d_counts(const SliceBuf &b) { return d_header(b) + kHeaderWords; }
    ServeItem *d_items(const SliceBuf &b) const {
        return reinterpret_cast<ServeItem *>(d_counts(b) + align_slots());
    }
    ServeItem *h_items(const SliceBuf &b) const {
        return reinterpret_cast<ServeItem *>(static_cast<unsigned *>(b.h_ring) + kHeaderWords +
                                             align_slots());
    }

    Request &req(int64_t id) {
        std::lock_guard<std::mutex> g(mu_);
        return *reqs_.at(id);
    }

    // Mark a request finished (result or error) and wake waiters.
    void complete(Request &r, mb_status st, const std::string &msg) {
        std::lock_guard<std::mutex> g(mu_);
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
        }
        std::vector<double>().swap(r.x);
        cv_done_.notify_all();
    }

    // Staging, first half: allocate, copy the points in, zero Phi and enqueue
    // the validation whose result lands in the slot's pinned record.  No wait.
    mb_status stage_begin(Request &r, int slot) {
        const int64_t n = r.n;
        const serve::ChunkLayout lay = serve::chunk_layout(n, kTab32, kTab64);
        if (hipMallocAsync(&r.chunk, lay.total, as_) != hipSuccess) {
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
        MB_HIP(hipMemcpyAsync(r.dx, r.x.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, as_));
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
                std::lock_guard<std::mutex> g(mu_);
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
        return MB_OK;
    }

    mb_status launch(const serve::Slice &sl, SliceBuf &b) {
        // items of binary32 requests first, then binary64
        std::vector<ServeItem> fi, di;
        for (const auto &rg : sl.ranges) {
            Request &r = req(rg.id);
            auto &dst = r.prec == MB_FP64 ? di : fi;
            for (int64_t u = rg.u0; u < rg.u1; ++u) {
                ServeItem it;
                it.slot = rg.slot;
                r.um.decode(u, it.a, it.b, it.t);
                dst.push_back(it);
            }
            ServeDesc &d = desc_table_[rg.slot];
            d.x = r.dx;
            d.phi = r.dphi;
            d.tab = r.dtab;
            d.n = (int32_t)r.n;
            d.na = r.um.na;
            d.scale = r.scale;
            d.out_scale = r.out_scale;
        }
        const int nf = (int)fi.size();
        const int nd = (int)di.size();
        // the pinned copies of b were last read by slice seq - 2, which has finished
        std::memcpy(b.h_desc, desc_table_.data(), sizeof(ServeDesc) * max_slots_);
        std::memset(b.h_ring, 0, sizeof(unsigned) * (kHeaderWords + align_slots()));
        std::copy(fi.begin(), fi.end(), h_items(b));
        std::copy(di.begin(), di.end(), h_items(b) + nf);
        const size_t bytes = sizeof(unsigned) * (kHeaderWords + align_slots()) +
                             sizeof(ServeItem) * (size_t)(nf + nd);
        MB_HIP(hipEventRecord(b.ev_start, cs_));
        MB_HIP(hipMemcpyAsync(b.d_desc, b.h_desc, sizeof(ServeDesc) * max_slots_,
                              hipMemcpyHostToDevice, cs_));
        MB_HIP(hipMemcpyAsync(b.d_ring, b.h_ring, bytes, hipMemcpyHostToDevice, cs_));
        if (nf)
            serve_kernel<float><<<(unsigned)std::min(nf, grid_f_), DirectLds<float>::TPB, 0, cs_>>>(
                b.d_desc, d_items(b), nf, d_header(b) + 0, d_counts(b));
        if (nd)
            serve_kernel<double><<<(unsigned)std::min(nd, grid_d_), DirectLds<double>::TPB, 0, cs_>>>(
                b.d_desc, d_items(b) + nf, nd, d_header(b) + 1, d_counts(b));
        MB_HIP(hipGetLastError());
        MB_HIP(hipMemcpyAsync(b.h_counts, d_counts(b), sizeof(unsigned) * max_slots_,
                              hipMemcpyDeviceToHost, cs_));
        MB_HIP(hipEventRecord(b.ev_end, cs_));
        return MB_OK;
    }

    mb_status finish_slice(const serve::Slice &sl, const SliceBuf &b,
                           std::vector<int64_t> &finished) {
        MB_HIP(hipEventSynchronize(b.ev_end));
        float ms = 0.f;
        MB_HIP(hipEventElapsedTime(&ms, b.ev_start, b.ev_end));
        std::vector<int64_t> expect(max_slots_, 0);
        for (const auto &rg : sl.ranges) expect[rg.slot] += rg.u1 - rg.u0;
        for (int s = 0; s < max_slots_; ++s)
            if ((int64_t)b.h_counts[s] != expect[s])
                return fail(MB_ERR_DEVICE, "drain kernel ran " + std::to_string(b.h_counts[s]) +
                                               " items of slot " + std::to_string(s) + ", issued " +
                                               std::to_string(expect[s]));
        {
            std::lock_guard<std::mutex> g(mu_);
            stats_.slices += 1;
            stats_.units += sl.units;
            if (sl.ranges.size() > 1) stats_.mixed_slices += 1;
            stats_.busy_ms += ms;
        }
        for (int64_t id : sched_.slice_done(sl)) finished.push_back(id);
        return MB_OK;
    }

    // Finishing, first half: binary64 repairs of a binary32 result, copy of
    // Phi into the slot's pinned buffer.  No wait.
    mb_status finish_begin(Request &r, int slot) {
        SlotHost &h = slot_host_[slot];
        if (h.phi_cap < r.n) {
            if (h.phi) (void)hipHostFree(h.phi);
            h.phi = nullptr;
            h.phi_cap = 0;
            MB_HIP(hipHostMalloc(&h.phi, sizeof(double) * (size_t)r.n, hipHostMallocDefault));
            h.phi_cap = r.n;
        }
        h.flagged = 0;
        if (r.prec == MB_FP32C) {
            const mb_status st = point_fp64_enqueue(r.dx, r.n, r.dmag, r.dphi, as_, &h.flagged);
            if (st != MB_OK) return st;
        }
        MB_HIP(hipMemcpyAsync(h.phi, r.dphi, sizeof(double) * r.n, hipMemcpyDeviceToHost, as_));
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
            MB_HIP(hipMemcpyAsync(h.phi, r.dphi, sizeof(double) * r.n, hipMemcpyDeviceToHost, as_));
            MB_HIP(hipStreamSynchronize(as_));
            flagged = r.n;
        }
        r.phi.assign(h.phi, h.phi + r.n);
        if (flagged) {
            std::lock_guard<std::mutex> g(mu_);
            stats_.points_fp64 += flagged;
        }
        MB_HIP(hipFreeAsync(r.chunk, as_));
        r.chunk = nullptr;
        sched_.release(id);
        complete(r, MB_OK, "");
        return MB_OK;
    }

    void drop(int64_t id, mb_status st, const std::string &msg) {
        Request &r = req(id);
        if (r.chunk) (void)hipFreeAsync(r.chunk, as_);
        r.chunk = nullptr;
        sched_.release(id);
        complete(r, st, msg);
    }

    mb_status step(std::vector<int64_t> &finished, bool &idle) {
        {
            std::lock_guard<std::mutex> g(mu_);
            if (slice_request_ > 0) {
                sched_.set_slice_units(slice_request_);
                slice_request_ = 0;
            }
            for (int64_t id : inbox_) sched_.enqueue(id, footprint(reqs_.at(id)->n));
            inbox_.clear();
        }
        mb_status st;
        // 1. keep up to two slices queued on the compute stream
        if (inflight_.size() < 2) {
            serve::Slice sl = sched_.next_slice();
            if (!sl.empty()) {
                if ((st = launch(sl, buf_[sl.seq & 1])) != MB_OK) return st;
                inflight_.push_back(std::move(sl));
            }
        }
        // 2. finished requests: enqueue their repairs and copies
        const double t0 = now_s();
        for (int64_t id : finished) {
            const int slot = sched_.slot_of(id);
            if ((st = finish_begin(req(id), slot)) != MB_OK) return st;
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
        // 5. validations that have landed: finish staging, then the request runs
        bool staged = false;
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
            int64_t units = 0, keep = 0;
            std::string why;
            st = stage_end(r, slot, units, keep, why);
            if (st == MB_ERR_OOM) {
                (void)hipGetLastError();
                why = last_error_cstr();
            }
            if (st == MB_ERR_DEGENERATE || st == MB_ERR_INVALID || st == MB_ERR_OOM) {
                drop(id, st, why);
                continue;
            }
            if (st != MB_OK) return st;
            sched_.start(id, units, keep);
            staged = true;
        }
        if (staged) {
            MB_HIP(hipEventRecord(ev_adm_, as_));
            MB_HIP(hipStreamWaitEvent(cs_, ev_adm_, 0));
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            stats_.finalize_ms += (t1 - t0) * 1e3;
            stats_.stage_ms += (now_s() - t1) * 1e3;
        }
        // 6. collect the oldest slice when two are queued or nothing else can
        // be queued, once its end event has passed (polled, so that arrivals
        // keep being staged meanwhile); with no slice in flight, report
        // whether anything is pending
        idle = false;
        if (!inflight_.empty() && (inflight_.size() == 2 || !sched_.has_runnable())) {
            const serve::Slice &old = inflight_.front();
            const hipError_t q = hipEventQuery(buf_[old.seq & 1].ev_end);
            if (q == hipSuccess) {
                if ((st = finish_slice(old, buf_[old.seq & 1], finished)) != MB_OK) return st;
                inflight_.pop_front();
            } else if (q == hipErrorNotReady) {
                std::this_thread::sleep_for(std::chrono::microseconds(10));
            } else {
                return fail(MB_ERR_DEVICE, std::string("hipEventQuery: ") + hipGetErrorString(q));
            }
        } else if (inflight_.empty() && !sched_.has_runnable()) {
            if (finishing_.empty() && validating_.empty() && finished.empty()) {
                idle = true;
            } else {
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            stats_.peak_reserved = sched_.peak_reserved();
            stats_.peak_active = sched_.peak_active();
        }
        return MB_OK;
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
                std::unique_lock<std::mutex> g(mu_);
                if (inbox_.empty()) {
                    if (stop_ && sched_.idle()) return;
                    cv_work_.wait_for(g, std::chrono::milliseconds(2));
                }
            }
        }
    }

    // A device error ends the server: every unfinished request fails.
    void break_all(const std::string &msg) {
        std::lock_guard<std::mutex> g(mu_);
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
    hipEvent_t ev_adm_ = nullptr;
    int dev_ = 0, grid_f_ = 1, grid_d_ = 1;
    SliceBuf buf_[2];
    // per slot: pinned validation record, repair count and result buffer, and
    // an event marking when the staging or finishing copies have landed
    struct SlotHost {
        ValidateOut v;
        int32_t flagged;
        double *phi;
        int64_t phi_cap;
    };
    SlotHost *slot_host_ = nullptr;
    std::vector<hipEvent_t> slot_ev_;
    std::vector<int64_t> validating_, finishing_;
    std::vector<ServeDesc> desc_table_;   // per slot, host master copy
    std::deque<serve::Slice> inflight_;   // slices queued on the compute stream
    size_t ring_bytes_ = 0;
    std::thread thread_;

    std::mutex mu_;  // guards everything below
    std::condition_variable cv_work_, cv_done_;
    std::map<int64_t, std::unique_ptr<Request>> reqs_;
    std::vector<int64_t> inbox_;
    int64_t next_id_ = 0;
    int64_t slice_request_ = 0;
    bool stop_ = false, broken_ = false;
    std::string broken_msg_;
    mb_server_stats stats_{};
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
