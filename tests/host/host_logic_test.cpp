// Host-logic checks built with the sanitizers: the symmetric-heap allocator
// against a brute-force byte map, and the serving admission budget under
// concurrent producers.  Prints "ok" and exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "hostalloc.hpp"

using vshmem::SymAllocator;

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static uint64_t rng(uint64_t &s)
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void allocator_basics()
{
    SymAllocator a;
    a.reset(1 << 20);
    CHECK(a.alloc(0, 256) == UINT64_MAX);                     // zero bytes: no object
    const uint64_t x = a.alloc(1000, 256), y = a.alloc(3 << 18, 256), z = a.alloc(1, 4096);
    CHECK(x == 0 && y == 1024);                               // first fit, sizes rounded to 256
    CHECK(z % 4096 == 0 && z >= y + (3 << 18));
    CHECK(a.alloc(1 << 20, 256) == UINT64_MAX);               // exhaustion
    CHECK(!a.free(12345) && a.free(y) && !a.free(y));         // unknown and double frees refused
    CHECK(a.alloc(3 << 18, 256) == y);                        // the hole is reused
    CHECK(a.free(x) && a.free(y) && a.free(z) && a.used() == 0);
    CHECK(a.alloc(1 << 20, 256) == 0);                        // everything coalesced back
    // Same call sequence, same offsets (symmetry by construction).
    SymAllocator b, c;
    b.reset(8 << 20);
    c.reset(8 << 20);
    uint64_t s1 = 7, s2 = 7;
    for (int i = 0; i < 2000; ++i) {
        const uint64_t n1 = 1 + rng(s1) % 40000, n2 = 1 + rng(s2) % 40000;
        CHECK(b.alloc(n1, 256) == c.alloc(n2, 256));
    }
}

// Random alloc/free against a byte map: live objects never overlap, are
// aligned and inside the capacity; used() equals the live bytes.
static void allocator_against_byte_map()
{
    const uint64_t cap = 1 << 20;
    SymAllocator a;
    a.reset(cap);
    std::vector<int> owner(cap, -1);
    std::vector<std::pair<uint64_t, uint64_t>> live;   // (offset, rounded size)
    uint64_t s = 99, bytes = 0;
    for (int step = 0; step < 20000; ++step) {
        if (!live.empty() && rng(s) % 3 == 0) {
            const size_t k = rng(s) % live.size();
            CHECK(a.free(live[k].first));
            for (uint64_t i = live[k].first; i < live[k].first + live[k].second; ++i) owner[i] = -1;
            bytes -= live[k].second;
            live[k] = live.back();
            live.pop_back();
        } else {
            const uint64_t n = 1 + rng(s) % 20000;
            const uint64_t al = 256ull << (rng(s) % 4);
            const uint64_t off = a.alloc(n, al);
            if (off == UINT64_MAX) continue;
            const uint64_t r = (n + 255) & ~255ull;
            CHECK(off % al == 0 && off + r <= cap);
            for (uint64_t i = off; i < off + r; ++i) {
                CHECK(owner[i] == -1);
                owner[i] = step;
            }
            live.push_back({off, r});
            bytes += r;
        }
        CHECK(a.used() == bytes);
    }
}

static void admission_budget()
{
    vshmem::Admission adm;
    adm.budget = 1000;
    CHECK(adm.reserve(600) && !adm.reserve(500) && adm.reserve(400) && !adm.reserve(1));
    adm.reserved.fetch_sub(1000);
    CHECK(adm.max_reserved.load() == 1000);
    // Concurrent producers: never more than the budget at once.
    adm.max_reserved = 0;
    adm.budget = 64;
    std::vector<std::thread> th;
    std::atomic<int> over{0};
    for (int t = 0; t < 8; ++t) {
        th.emplace_back([&adm, &over, t] {
            uint64_t s = (uint64_t)t + 1;
            for (int i = 0; i < 20000; ++i) {
                const uint64_t b = 1 + rng(s) % 16;
                const uint64_t seen = adm.gen.load();
                if (!adm.reserve(b)) {
                    adm.wait_after(seen);
                    continue;
                }
                if (adm.reserved.load() > adm.budget) over.fetch_add(1);
                adm.reserved.fetch_sub(b);
                adm.released();
            }
        });
    }
    for (auto &x : th) x.join();
    CHECK(over.load() == 0 && adm.reserved.load() == 0 && adm.max_reserved.load() <= 64);
}

// Deferred frees of a PE's destination region: a range queued by the
// completion side comes back at the next allocation, a producer and a
// completion thread running together never hand out a range twice, and
// everything is returned in the end.
static void region_deferred_frees()
{
    vshmem::PeRegion pr;
    pr.dst.reset(1 << 20);
    const uint64_t a = pr.alloc(1 << 19, 256), b = pr.alloc(1 << 19, 256);
    CHECK(a == 0 && b == (1u << 19) && pr.alloc(256, 256) == UINT64_MAX);   // full
    pr.release_later(a);
    CHECK(pr.dst.used() == (1u << 20));                                     // not yet returned
    CHECK(pr.alloc(1 << 18, 256) == 0);                                     // returned, then reused
    pr.release_later(0);
    pr.release_later(b);
    CHECK(pr.alloc(1 << 20, 256) == 0);                                     // both returned and coalesced
    pr.release_later(0);
    // One producer and one completion thread: live ranges never overlap.
    pr.dst.reset(1 << 16);
    std::atomic<bool> stop{false};
    std::vector<std::atomic<int>> owner(256);
    for (auto &o : owner) o.store(0);
    std::atomic<int> overlaps{0};
    std::vector<std::pair<uint64_t, uint64_t>> handoff;
    std::mutex hm;
    std::thread completer([&] {
        for (;;) {
            const bool last = stop.load();
            std::pair<uint64_t, uint64_t> r{UINT64_MAX, 0};
            {
                std::lock_guard<std::mutex> lk(hm);
                if (!handoff.empty()) {
                    r = handoff.back();
                    handoff.pop_back();
                }
            }
            if (r.first == UINT64_MAX) {
                if (last) break;   // the producer had stopped before this empty look
                continue;
            }
            for (uint64_t k = r.first / 256; k < (r.first + r.second) / 256; ++k) owner[k].fetch_sub(1);
            pr.release_later(r.first);
        }
    });
    uint64_t s = 99;
    for (int i = 0; i < 20000; ++i) {
        const uint64_t len = 256 * (1 + rng(s) % 8);
        const uint64_t off = pr.alloc(len, 256);
        if (off == UINT64_MAX) continue;
        for (uint64_t k = off / 256; k < (off + len) / 256; ++k)
            if (owner[k].fetch_add(1) != 0) overlaps.fetch_add(1);
        std::lock_guard<std::mutex> lk(hm);
        handoff.emplace_back(off, len);
    }
    stop.store(true);
    completer.join();
    CHECK(overlaps.load() == 0);
    CHECK(pr.alloc(1 << 16, 256) == 0);   // every range came back
}

int main()
{
    allocator_basics();
    allocator_against_byte_map();
    admission_budget();
    region_deferred_frees();
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
