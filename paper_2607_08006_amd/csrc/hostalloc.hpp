// Host-side bookkeeping with no device code: the symmetric-heap allocator
// and the serving admission budget.  Kept free of HIP so that it also
// builds with a plain C++ compiler (the sanitizer tests do that).
#pragma once
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

namespace vshmem {

constexpr uint64_t kMinAlign = 256;               // default allocation alignment

// First-fit allocator over [0, capacity) with a coalescing free list.  The
// same call sequence always yields the same offsets: allocation is
// symmetric by construction because one offset names the object on every PE.
class SymAllocator {
  public:
    void reset(uint64_t capacity);
    // Returns the offset or UINT64_MAX.
    uint64_t alloc(uint64_t size, uint64_t align);
    bool free(uint64_t off);
    uint64_t used() const { return used_; }
    uint64_t capacity() const { return cap_; }

  private:
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    std::map<uint64_t, uint64_t> live_;   // offset -> length
    uint64_t cap_ = 0, used_ = 0;
};

// Admission is sharded so that producers for different PEs do not
// serialise: the budget is one atomic counter, each PE's destination
// allocator has its own lock, and counter pools are atomic bump pointers.
// Producers that cannot be admitted sleep on a generation count that every
// completion advances.  (One global lock here capped a burst at about
// 0.7 M requests/s.)
//
// The completion thread does not free a finished request's range itself:
// it queues the offset (release_later) and the next producer that
// allocates on the PE, which holds the PE's lock anyway, frees everything
// queued first (alloc).  Freeing on the single completion thread, under
// locks the producers were holding, cost 230-370 ns per request and capped
// serving at about 2 M requests/s.
struct PeRegion {
    std::mutex mu;
    SymAllocator dst;                  // offsets relative to the region
    std::atomic<uint64_t> ctr_next{0}; // bump pointer of the PE's counter pool
    std::mutex pend_mu;
    std::vector<uint64_t> pending;     // finished ranges not yet returned to dst (pend_mu)
    std::vector<uint64_t> draining;    // their storage while they are freed (mu)

    void release_later(uint64_t off)
    {
        std::lock_guard<std::mutex> lk(pend_mu);
        pending.push_back(off);
    }
    // Return the queued ranges, then allocate.  UINT64_MAX when it does not fit.
    uint64_t alloc(uint64_t size, uint64_t align)
    {
        std::lock_guard<std::mutex> lk(mu);
        draining.clear();
        {
            std::lock_guard<std::mutex> lp(pend_mu);
            draining.swap(pending);   // both keep their capacity: no allocation in steady state
        }
        for (uint64_t off : draining) dst.free(off);
        return dst.alloc(size, align);
    }
};

struct Admission {
    std::vector<std::unique_ptr<PeRegion>> pe;
    uint64_t ctr_base = 0, ctr_bytes = 0, budget = 0;
    std::atomic<uint64_t> reserved{0}, max_reserved{0}, waits{0}, gen{0};
    std::atomic<int> waiting{0};
    std::mutex wait_mu;
    std::condition_variable cv;

    // Reserve `bytes` of the budget; false when it does not fit now.
    bool reserve(uint64_t bytes)
    {
        uint64_t cur = reserved.load(std::memory_order_relaxed);
        do {
            if (cur + bytes > budget) return false;
        } while (!reserved.compare_exchange_weak(cur, cur + bytes, std::memory_order_relaxed));
        uint64_t m = max_reserved.load(std::memory_order_relaxed);
        while (cur + bytes > m && !max_reserved.compare_exchange_weak(m, cur + bytes, std::memory_order_relaxed)) {
        }
        return true;
    }
    // Wake producers waiting for budget or space (after a release).
    void released()
    {
        {
            std::lock_guard<std::mutex> lk(wait_mu);
            gen.fetch_add(1, std::memory_order_release);
        }
        if (waiting.load(std::memory_order_acquire) > 0) cv.notify_all();
    }
    // Sleep until a completion after generation `seen` (bounded).
    void wait_after(uint64_t seen)
    {
        std::unique_lock<std::mutex> lk(wait_mu);
        waiting.fetch_add(1, std::memory_order_acq_rel);
        cv.wait_for(lk, std::chrono::milliseconds(5), [&] { return gen.load(std::memory_order_acquire) != seen; });
        waiting.fetch_sub(1, std::memory_order_acq_rel);
    }
};

}  // namespace vshmem
