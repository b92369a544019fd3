// Trace-driven serving on the persistent progress kernel: producer threads
// replay arrivals, admission reserves destination memory under a heap
// budget, and a completion thread frees reservations as requests finish so
// new ones are admitted while others are still on the device.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include <sys/prctl.h>

#include "serving.hpp"

using namespace vshmem;
using Clock = std::chrono::steady_clock;

namespace {

struct Slot {
    std::atomic<int> state{0};          // 0 waiting, 1 submitted, 2 done
    uint64_t ticket = 0;
    Clock::time_point arrival, submitted;
    uint64_t dst = 0, ctr = 0, bytes = 0;
    int dst_pe = 0;
};

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// How admitted requests reach the device and how their completion is seen.
struct Backend {
    virtual ~Backend() = default;
    // Issue request `index` from producer `lane`; on success *ticket names it.
    virtual int submit(const shmemx_desc_t &d, size_t index, int lane, uint64_t *ticket) = 0;
    std::atomic<uint64_t> busy_retries{0};
    // 1 and *out filled when finished, 0 when not yet, < 0 on error.
    virtual int poll(uint64_t ticket, shmemx_completion_t *out) = 0;
    // Called by the completion thread after a pass that freed ring slots.
    virtual void slots_freed() {}
};

// The persistent progress kernel: requests go through its host ring.
// A producer that finds the ring full sleeps until the completion thread
// has freed slots (a generation count) instead of spinning on the ring's
// cache lines, which starved the completion thread itself.
struct ProgressBackend final : Backend {
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<uint64_t> gen{0};

    int submit(const shmemx_desc_t &d, size_t, int lane, uint64_t *ticket) override
    {
        const Clock::time_point t0 = Clock::now();
        for (;;) {
            const uint64_t seen = gen.load(std::memory_order_acquire);
            const int rc = shmemx_progress_submit(lane % SHMEMX_PROGRESS_LANES, &d, ticket);
            if (rc != SHMEMX_ERR_BUSY) return rc;
            busy_retries.fetch_add(1, std::memory_order_relaxed);
            if (Clock::now() - t0 > std::chrono::seconds(30)) return rc;
            std::unique_lock<std::mutex> lk(mu);
            cv.wait_for(lk, std::chrono::milliseconds(1), [&] { return gen.load(std::memory_order_acquire) != seen; });
        }
    }
    int poll(uint64_t ticket, shmemx_completion_t *out) override { return shmemx_progress_poll(ticket, out); }
    void slots_freed() override
    {
        gen.fetch_add(1, std::memory_order_release);
        { std::lock_guard<std::mutex> lk(mu); }
        cv.notify_all();
    }
};

// One kernel launch per request on the producer lane's own stream; an event
// recorded after the launch marks completion.  Events come from a pool that
// grows to the peak number of requests in flight.
struct PerOpBackend final : Backend {
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> by_request;
    std::vector<hipEvent_t> pool, all;
    std::mutex mu;
    uint64_t chunk;
    int wg;

    PerOpBackend(size_t n, uint64_t chunk_bytes, int wg_size) : by_request(n, nullptr), chunk(chunk_bytes), wg(wg_size) {}
    ~PerOpBackend() override
    {
        for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
        for (hipEvent_t e : all) (void)hipEventDestroy(e);
        for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    }
    int init(int lanes)
    {
        for (int l = 0; l < lanes; ++l) {
            hipStream_t s = nullptr;
            if (VSHMEM_HIP_FAILED(hipStreamCreateWithFlags(&s, hipStreamNonBlocking))) return SHMEMX_ERR_HIP;
            streams.push_back(s);
        }
        return SHMEMX_OK;
    }
    int submit(const shmemx_desc_t &d, size_t index, int lane, uint64_t *ticket) override
    {
        hipEvent_t e = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (!pool.empty()) {
                e = pool.back();
                pool.pop_back();
            } else {
                if (VSHMEM_HIP_FAILED(hipEventCreateWithFlags(&e, hipEventDisableTiming))) return SHMEMX_ERR_HIP;
                all.push_back(e);
            }
        }
        if (int rc = shmemx_launch_request(&d, chunk, wg, streams[lane])) return rc;
        if (VSHMEM_HIP_FAILED(hipEventRecord(e, streams[lane]))) return SHMEMX_ERR_HIP;
        by_request[index] = e;
        *ticket = index;
        return SHMEMX_OK;
    }
    int poll(uint64_t ticket, shmemx_completion_t *out) override
    {
        const hipError_t q = hipEventQuery(by_request[ticket]);
        if (q == hipErrorNotReady) return 0;
        if (q != hipSuccess) {
            set_hip_error(q, "serve per-op: hipEventQuery");
            return SHMEMX_ERR_HIP;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            pool.push_back(by_request[ticket]);
        }
        *out = shmemx_completion_t{};
        out->ticket = ticket;
        return 1;
    }
};

// Windowed batches: submit() queues the request; a dispatcher thread takes
// everything queued once the oldest request has waited `window` (or a full
// batch is queued) and launches it as one batch from a free slot (the slot's
// previous batch must have completed).  A request completes when its
// batch's event does.
struct WindowBackend final : Backend {
    WindowBatcher *wb = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    struct Pending {
        shmemx_desc_t d;
        size_t index;
        Clock::time_point enqueued;
    };
    std::vector<Pending> pending;
    Clock::time_point oldest;   // enqueue time of pending.front()
    std::vector<std::atomic<int64_t>> batch_of;   // request -> batch, -1 before launch
    std::vector<hipEvent_t> batch_done;           // batch -> event (grows; guarded by events_mu)
    std::mutex events_mu;
    std::chrono::nanoseconds window;
    std::atomic<bool> stop{false};
    std::atomic<int> error{0};
    std::thread dispatcher;
    size_t batches = 0;

    WindowBackend(size_t n, uint64_t window_ns) : batch_of(n), window(window_ns)
    {
        for (auto &b : batch_of) b.store(-1);
    }
    int init(bool graph, uint64_t chunk, int nwg, int wg, hipStream_t stream)
    {
        int rc = SHMEMX_OK;
        wb = window_batcher_create(graph, chunk, nwg, wg, stream, &rc);
        if (rc) return rc;
        dispatcher = std::thread([this] { run(); });
        return SHMEMX_OK;
    }
    ~WindowBackend() override
    {
        stop.store(true);
        cv.notify_all();
        if (dispatcher.joinable()) dispatcher.join();
        window_batcher_destroy(wb);
        for (hipEvent_t e : batch_done) (void)hipEventDestroy(e);
    }
    void run()
    {
        // A 20 us window must not wait out the default 50 us timer slack.
        (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0, 0, 0);
        std::vector<shmemx_desc_t> d;
        std::vector<size_t> idx;
        hipEvent_t slot_event[kWindowSlots] = {};
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop.load() || !pending.empty(); });
                if (pending.empty()) return;   // stopped
                // Wait out the window of the oldest request unless a batch is full.
                while (!stop.load() && pending.size() < kWindowBatchMax && Clock::now() < oldest + window)
                    cv.wait_until(lk, oldest + window);
                const size_t take = std::min(pending.size(), kWindowBatchMax);
                d.clear();
                idx.clear();
                for (size_t i = 0; i < take; ++i) {
                    d.push_back(pending[i].d);
                    idx.push_back(pending[i].index);
                }
                pending.erase(pending.begin(), pending.begin() + (ptrdiff_t)take);
                // The window of what is left runs from its own oldest arrival,
                // not from this dispatch.
                if (!pending.empty()) oldest = pending.front().enqueued;
            }
            const int slot = (int)(batches % kWindowSlots);
            if (slot_event[slot] && VSHMEM_HIP_FAILED(hipEventSynchronize(slot_event[slot]))) {
                error.store(SHMEMX_ERR_HIP);
                return;
            }
            hipEvent_t e = nullptr;
            if (VSHMEM_HIP_FAILED(hipEventCreateWithFlags(&e, hipEventDisableTiming))) {
                error.store(SHMEMX_ERR_HIP);
                return;
            }
            if (int rc = window_batcher_launch(wb, slot, d.data(), d.size(), e)) {
                (void)hipEventDestroy(e);
                error.store(rc);
                return;
            }
            slot_event[slot] = e;
            {
                std::lock_guard<std::mutex> lk(events_mu);
                batch_done.push_back(e);
            }
            for (size_t i : idx) batch_of[i].store((int64_t)batches, std::memory_order_release);
            ++batches;
        }
    }
    int submit(const shmemx_desc_t &d, size_t index, int, uint64_t *ticket) override
    {
        if (int rc = error.load()) return rc;
        {
            std::lock_guard<std::mutex> lk(mu);
            const Clock::time_point now = Clock::now();
            if (pending.empty()) oldest = now;
            pending.push_back(Pending{d, index, now});
        }
        cv.notify_all();
        *ticket = index;
        return SHMEMX_OK;
    }
    int poll(uint64_t ticket, shmemx_completion_t *out) override
    {
        if (int rc = error.load()) return rc;
        const int64_t b = batch_of[ticket].load(std::memory_order_acquire);
        if (b < 0) return 0;
        hipEvent_t e;
        {
            std::lock_guard<std::mutex> lk(events_mu);
            e = batch_done[(size_t)b];
        }
        const hipError_t q = hipEventQuery(e);
        if (q == hipErrorNotReady) return 0;
        if (q != hipSuccess) {
            set_hip_error(q, "serve windowed: hipEventQuery");
            return SHMEMX_ERR_HIP;
        }
        *out = shmemx_completion_t{};
        out->ticket = ticket;
        return 1;
    }
};

int serve_common(Backend &be, const shmemx_request_t *reqs, size_t n, int lanes, uint64_t region_off,
                 uint64_t region_bytes, uint64_t budget_bytes, uint64_t *dst_off_out, uint64_t *latency_ns,
                 shmemx_completion_t *completions, shmemx_serve_stats_t *stats)
{
    const State &s = st();
    if ((!reqs && n) || lanes < 1 || lanes > 64 || !in_user_heap(region_off, region_bytes) || region_bytes < 4096 ||
        budget_bytes == 0)
        return SHMEMX_ERR_ARG;
    for (size_t i = 0; i < n; ++i) {
        const shmemx_request_t &r = reqs[i];
        bool ok = r.issuer_pe >= 0 && r.issuer_pe < s.npes && r.target_pe >= 0 && r.target_pe < s.npes && r.lane >= 0 &&
                  r.lane < lanes && r.arrival_s >= 0 && r.nbytes > 0 &&
                  (r.op == SHMEMX_OP_PUT || r.op == SHMEMX_OP_GET || r.op == SHMEMX_OP_AMO_FETCH_ADD);
        if (ok && r.op != SHMEMX_OP_AMO_FETCH_ADD) ok = in_user_heap(r.src_off, r.nbytes);
        if (ok && r.op == SHMEMX_OP_AMO_FETCH_ADD) ok = (r.nbytes & 7) == 0;
        if (!ok) return SHMEMX_ERR_ARG;
    }
    // Destinations: the lower three quarters of the region, first fit with
    // reuse.  Counters of fetch_add requests: the top quarter, bump
    // allocated so every request starts from zeroed counters.
    Admission adm;
    const uint64_t dst_bytes = (region_bytes / 4 * 3) & ~255ull;
    adm.pe.resize(s.npes);
    for (auto &a : adm.pe) {
        a = std::make_unique<PeRegion>();
        a->dst.reset(dst_bytes);
    }
    adm.ctr_base = region_off + dst_bytes;
    adm.ctr_bytes = (region_bytes - dst_bytes) & ~255ull;
    adm.budget = budget_bytes;
    std::vector<Slot> slots(n);
    std::atomic<int> failed{0};
    // One past the largest request index submitted so far: the completion
    // thread's passes stop there instead of walking the whole trace.
    std::atomic<size_t> submitted_end{0};
    std::atomic<size_t> ndone{0};
    // Arrival times count from `start`, a short lead after this point that
    // lets the producer and completion threads start first.
    const Clock::time_point start = Clock::now() + std::chrono::microseconds(200);

    // Arrivals are replayed on time: a sleeping thread wakes up to the
    // timer slack late (50 us by default), which the latency would count,
    // so producers take a 1 us slack and spin through the last 50 us.
    auto wait_until = [](Clock::time_point due) {
        const auto spin = std::chrono::microseconds(50);
        if (Clock::now() + spin < due) std::this_thread::sleep_until(due - spin);
        while (Clock::now() < due) std::this_thread::yield();
    };
    auto producer = [&](int lane) {
        (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0, 0, 0);
        for (size_t i = 0; i < n && !failed.load(); ++i) {
            const shmemx_request_t &r = reqs[i];
            if (r.lane != lane) continue;
            const Clock::time_point due = start + std::chrono::duration_cast<Clock::duration>(
                                                      std::chrono::duration<double>(r.arrival_s));
            wait_until(due);
            Slot &sl = slots[i];
            sl.arrival = due;
            const uint64_t need = round_up(r.nbytes, 256);
            const int dpe = r.op == SHMEMX_OP_PUT ? r.target_pe : r.issuer_pe;   // GET and AMO results land on the issuer
            {
                const bool amo = r.op == SHMEMX_OP_AMO_FETCH_ADD;
                const uint64_t extra = need + (amo ? need : 0);
                if (extra > adm.budget || need > dst_bytes) {   // could never be admitted
                    failed.store(SHMEMX_ERR_NOMEM);
                    adm.released();
                    return;
                }
                bool waited = false;
                for (;;) {
                    if (failed.load()) return;
                    const uint64_t seen = adm.gen.load(std::memory_order_acquire);
                    if (adm.reserve(extra)) {
                        const uint64_t off = adm.pe[dpe]->alloc(need, 256);
                        if (off != UINT64_MAX) {
                            sl.dst = region_off + off;
                            sl.dst_pe = dpe;
                            sl.bytes = extra;
                            if (amo) {
                                const uint64_t c = adm.pe[r.target_pe]->ctr_next.fetch_add(need);
                                if (c + need > adm.ctr_bytes) {
                                    failed.store(SHMEMX_ERR_NOMEM);
                                    adm.released();
                                    return;
                                }
                                sl.ctr = adm.ctr_base + c;
                            }
                            break;
                        }
                        adm.reserved.fetch_sub(extra, std::memory_order_relaxed);   // no space on the PE yet
                    }
                    if (!waited) {
                        adm.waits.fetch_add(1, std::memory_order_relaxed);
                        waited = true;
                    }
                    adm.wait_after(seen);
                }
            }
            shmemx_desc_t d{};
            d.op = (uint8_t)r.op;
            d.scope = SHMEMX_SCOPE_AUTO;
            d.issuer_pe = r.issuer_pe;
            d.target_pe = r.target_pe;
            d.result_idx = SHMEMX_NO_RESULT;
            d.nbytes = r.nbytes;
            if (r.op == SHMEMX_OP_AMO_FETCH_ADD) {
                d.src = sl.ctr;
                d.dst = sl.dst;
                d.value = 1;
            } else {
                d.src = r.src_off;
                d.dst = sl.dst;
            }
            uint64_t t = 0;
            const int rc = be.submit(d, i, lane, &t);
            if (rc != SHMEMX_OK) {
                failed.store(rc);
                return;
            }
            sl.ticket = t;
            sl.submitted = Clock::now();
            sl.state.store(1, std::memory_order_release);
            size_t e = submitted_end.load(std::memory_order_relaxed);
            while (e < i + 1 && !submitted_end.compare_exchange_weak(e, i + 1, std::memory_order_release)) {
            }
        }
    };

    auto completer = [&]() {
        size_t lo = 0;
        Clock::time_point last_progress = Clock::now();
        while (ndone.load() < n && !failed.load()) {
            bool any = false;
            const size_t scan_end = submitted_end.load(std::memory_order_acquire);
            for (size_t i = lo; i < scan_end; ++i) {
                Slot &sl = slots[i];
                const int stt = sl.state.load(std::memory_order_acquire);
                if (stt != 1) continue;
                shmemx_completion_t c;
                const int pr = be.poll(sl.ticket, &c);
                if (pr < 0) {
                    failed.store(pr);
                    break;
                }
                if (pr == 1) {
                    const Clock::time_point now = Clock::now();
                    if (latency_ns) latency_ns[i] = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(now - sl.arrival).count();
                    c.submit_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(sl.submitted - sl.arrival).count();
                    if (completions) completions[i] = c;
                    if (dst_off_out) dst_off_out[i] = sl.dst;
                    adm.pe[sl.dst_pe]->release_later(sl.dst - region_off);
                    adm.reserved.fetch_sub(sl.bytes, std::memory_order_relaxed);
                    adm.released();
                    sl.state.store(2, std::memory_order_release);
                    ndone.fetch_add(1);
                    any = true;
                    if (c.status != 0) failed.store(SHMEMX_ERR_DEVICE);
                }
            }
            while (lo < n && slots[lo].state.load(std::memory_order_acquire) == 2) ++lo;
            if (any) be.slots_freed();
            if (any) last_progress = Clock::now();
            else if (Clock::now() - last_progress > std::chrono::seconds(60)) failed.store(SHMEMX_ERR_TIMEOUT);
            else std::this_thread::yield();
        }
    };

    std::vector<std::thread> th;
    for (int l = 0; l < lanes; ++l) th.emplace_back(producer, l);
    std::thread ct(completer);
    for (auto &t : th) t.join();
    ct.join();
    const double wall = std::chrono::duration<double>(Clock::now() - start).count();
    if (stats) {
        stats->wall_s = wall;
        stats->bytes = 0;
        stats->amo_ops = 0;
        for (size_t i = 0; i < n; ++i) {
            if (reqs[i].op == SHMEMX_OP_AMO_FETCH_ADD) stats->amo_ops += reqs[i].nbytes / 8;
            else stats->bytes += reqs[i].nbytes;
        }
        stats->max_reserved_bytes = adm.max_reserved.load();
        stats->admission_waits = adm.waits.load();
        stats->ring_full_retries = be.busy_retries.load();
    }
    return failed.load();
}

}  // namespace

extern "C" int shmemx_serve_run(const shmemx_request_t *reqs, size_t n, int lanes, uint64_t region_off,
                                uint64_t region_bytes, uint64_t budget_bytes, uint64_t *dst_off_out, uint64_t *latency_ns,
                                shmemx_completion_t *completions, shmemx_serve_stats_t *stats)
{
    if (int rc = check_ready()) return rc;
    if (!progress_running()) return SHMEMX_ERR_STATE;
    ProgressBackend be;
    return serve_common(be, reqs, n, lanes, region_off, region_bytes, budget_bytes, dst_off_out, latency_ns,
                        completions, stats);
}

extern "C" int shmemx_serve_run_per_op(const shmemx_request_t *reqs, size_t n, int lanes, uint64_t region_off,
                                       uint64_t region_bytes, uint64_t budget_bytes, uint64_t chunk_bytes, int wg_size,
                                       uint64_t *dst_off_out, uint64_t *latency_ns, shmemx_completion_t *completions,
                                       shmemx_serve_stats_t *stats)
{
    if (int rc = check_ready()) return rc;
    if (progress_running()) return SHMEMX_ERR_STATE;
    if (lanes < 1 || lanes > 64 || chunk_bytes == 0 || (chunk_bytes & 15) || !valid_wg_size(wg_size))
        return SHMEMX_ERR_ARG;
    PerOpBackend be(n, chunk_bytes, wg_size);
    if (int rc = be.init(lanes)) return rc;
    return serve_common(be, reqs, n, lanes, region_off, region_bytes, budget_bytes, dst_off_out, latency_ns,
                        completions, stats);
}

extern "C" int shmemx_serve_run_batched(const shmemx_request_t *reqs, size_t n, int lanes, uint64_t region_off,
                                        uint64_t region_bytes, uint64_t budget_bytes, uint64_t window_ns, int use_graph,
                                        uint64_t chunk_bytes, int wg_size, uint64_t *dst_off_out, uint64_t *latency_ns,
                                        shmemx_completion_t *completions, shmemx_serve_stats_t *stats)
{
    if (int rc = check_ready()) return rc;
    if (progress_running()) return SHMEMX_ERR_STATE;
    if (lanes < 1 || lanes > 64 || chunk_bytes == 0 || (chunk_bytes & 15) || !valid_wg_size(wg_size) ||
        window_ns > 1000000000ull)
        return SHMEMX_ERR_ARG;
    hipStream_t stream = nullptr;
    if (VSHMEM_HIP_FAILED(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking))) return SHMEMX_ERR_HIP;
    int rc;
    {
        WindowBackend be(n, window_ns);
        rc = be.init(use_graph != 0, chunk_bytes, st().num_cus, wg_size, stream);
        if (!rc)
            rc = serve_common(be, reqs, n, lanes, region_off, region_bytes, budget_bytes, dst_off_out, latency_ns,
                              completions, stats);
    }
    (void)hipStreamSynchronize(stream);
    (void)hipStreamDestroy(stream);
    return rc;
}
