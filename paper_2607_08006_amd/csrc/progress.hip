// Persistent progress kernel (GPU-driven progress for requests that arrive
// while the kernel runs) and the host side of its request ring.
//
// Host producers publish 64-byte descriptors into a ring in pinned, coherent
// host memory, one sequence word per slot (a bounded multi-producer queue:
// slot s is free for ticket t when seq[s] == t and published when t + 1).
// The device reports completion in a separate word (done[s] = t + 1, after
// the completion record); the host's poll consumes the record and only then
// frees the slot for ticket t + slots, so a record is never overwritten
// before it was read.  On the device one front-end wavefront (the first of
// work-group 0) reads published descriptors in ticket order and expands
// each into work items of chunk_bytes times the queued items per worker
// (at least 1, at most 8) in a device-memory queue;
// every other work-group claims items from that queue one at a time and
// executes each with all its threads, and the work-group that finishes a
// request's last item writes its completion record to host memory and then
// releases the slot with a system-scope store.  The kernel ends when the
// host raises the stop flag or after idle_timeout_ms without a request;
// either way every wavefront reaches its exit.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>

#include "serving.hpp"

using namespace vshmem;

namespace {

constexpr uint64_t kItemPoison = ~0ull;

struct Item {              // 64 bytes, device memory
    uint64_t seq;
    uint64_t parent;       // ring slot of the request, or kItemPoison
    uint64_t ticket;       // ticket of the request (consistency check)
    uint64_t lo, hi;       // byte range of the request's payload
    uint64_t pad[3];
};

struct alignas(128) Parent {   // device memory, one per ring slot, own cache line
    shmemx_desc_t d;
    uint64_t ticket;
    uint64_t remaining;    // items not yet finished
    uint64_t t_start;
    uint64_t hash;
    uint64_t t_queued;     // front-end pickup
    int32_t status;
    int32_t pad;
};

struct ProgArgs {
    shmemx_dctx_pub_t c;
    shmemx_desc_t *ring;          // host memory (device-mapped)
    uint64_t *ring_seq;           // host memory (device-mapped)
    uint64_t *ring_done;          // host memory (device-mapped)
    shmemx_completion_t *comp;    // host memory (device-mapped)
    uint64_t *stop;               // host memory (device-mapped)
    Item *items;
    Parent *parents;
    uint64_t *claim;              // device: next item ticket for workers
    uint64_t slots, qsize;
    uint64_t chunk;               // item size while workers keep up
    uint64_t idle_ticks;
    uint64_t hold_ticks;          // longest a finished item waits for its work-group's release
    int verify;
};

__device__ __forceinline__ uint64_t ld_sys(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t ld_dev(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// Relaxed coherent loads: records written by another work-group (or by the
// host) are read through atomic loads, which are served at the coherence
// point rather than from a possibly stale cached line.
__device__ __forceinline__ uint64_t ldr_dev(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ldr_sys(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void load_desc(shmemx_desc_t &d, const shmemx_desc_t *src, bool system)
{
    uint64_t w[8];
    const uint64_t *q = (const uint64_t *)src;
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = system ? ldr_sys(q + i) : ldr_dev(q + i);
    memcpy(&d, w, sizeof(d));
}

// Output checksum: XOR over the output's 8-byte words w_i (last one zero
// padded) of mix(w_i ^ ((i + 1) * golden)), i counted from the start of the
// request's output, so it does not depend on where the output was placed.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// This thread's share of the hash of words [lo/8, (hi+7)/8), reduced over its
// wavefront (lane 0 holds the wavefront's share).
__device__ uint64_t hash_range(const uint8_t *out, uint64_t lo, uint64_t hi, uint64_t total)
{
    // lo is a multiple of 8 (chunks are multiples of 16); words are indexed from 0.
    uint64_t h = 0;
    const uint64_t w0 = lo / 8, w1 = (hi + 7) / 8;
    const bool aligned = ((uintptr_t)out & 7) == 0;
    for (uint64_t w = w0 + threadIdx.x; w < w1; w += blockDim.x) {
        uint64_t x = 0;
        const uint64_t b = w * 8;
        if (aligned && b + 8 <= total) {
            x = *(const uint64_t *)(out + b);
        } else {
            for (int k = 0; k < 8; ++k)
                if (b + k < total) x |= (uint64_t)out[b + k] << (8 * k);
        }
        h ^= mix64(x ^ ((w + 1) * 0x9E3779B97F4A7C15ull));
    }
    for (int off = 32; off > 0; off >>= 1) h ^= __shfl_xor(h, off, 64);
    return h;
}


// Execute bytes [lo, hi) of a request with all threads of the work-group.
__device__ void exec_item(const ProgArgs &a, const shmemx_desc_t &d, uint64_t lo, uint64_t hi, uint64_t *hash_acc)
{
    uint8_t *out = exec_request_range(a.c, d, lo, hi, threadIdx.x, blockDim.x);
    if (a.verify) {
        // Every thread's stores complete before any thread reads the output.
        vshmem_detail::release_agent();
        __syncthreads();
        vshmem_detail::acquire_agent();
        const uint64_t h = hash_range(out, lo, hi, d.nbytes);
        if (__lane_id() == 0 && h) __hip_atomic_fetch_xor(hash_acc, h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ bool valid_request(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d)
{
    if (d.issuer_pe < 0 || d.issuer_pe >= c.npes || d.target_pe < 0 || d.target_pe >= c.npes) return false;
    auto in = [&](uint64_t off, uint64_t n) { return off <= c.user_bytes && n <= c.user_bytes - off; };
    if (d.op == SHMEMX_OP_PUT || d.op == SHMEMX_OP_GET) return in(d.src, d.nbytes) && in(d.dst, d.nbytes);
    if (d.op == SHMEMX_OP_AMO_FETCH_ADD)
        return (d.nbytes & 7) == 0 && (d.src & 7) == 0 && (d.dst & 7) == 0 && in(d.src, d.nbytes) && in(d.dst, d.nbytes);
    return false;
}

__device__ void post_completion(const ProgArgs &a, uint32_t slot, Parent &P, int32_t status)
{
    shmemx_completion_t *cp = a.comp + slot;
    cp->ticket = ldr_dev(&P.ticket);
    cp->t_start = __hip_atomic_load(&P.t_start, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    cp->t_end = wall_clock64();
    cp->hash = __hip_atomic_load(&P.hash, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    cp->t_queued = ldr_dev(&P.t_queued);
    cp->submit_ns = 0;
    cp->status = status;
    cp->lane = (int32_t)P.d.reserved;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");   // system scope: the record before the done word
    st_sys(a.ring_done + slot, cp->ticket + 1);
}

// Front-end: wavefront 0 of work-group 0.  Each round its 64 lanes look at
// up to the next 256 tickets and take the published prefix at once, under
// one acquire and one release: descriptors are read in parallel, item
// positions come from wavefront prefix sums, the items are written by all
// lanes evenly, and the release publishes the round's records before the
// items' sequence words are stored.
__device__ bool wait_item_free(const ProgArgs &a, Item *it, uint64_t pos)
{
    const uint64_t t0 = wall_clock64();
    while (ldr_dev(&it->seq) != pos) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > a.idle_ticks) return false;
    }
    return true;
}

constexpr int kFrontBatches = 4;   // a round takes up to 4 x 64 published tickets
// Largest item size under backlog, in units of chunk_bytes.  On a burst of
// 10^4 log-uniform requests (64 B - 16 MiB) with 256 KiB chunks, items in
// proportion to the backlog capped at 4, 8 and 16 gave 1.35, 1.59 and 1.47
// TB/s of payload: larger items cut per-item costs until too few remain to
// balance the tail.
constexpr uint64_t kBacklogSplit = 8;

__device__ void front_end(const ProgArgs &a, uint64_t nworkers)
{
    const uint64_t qmask = a.qsize - 1, smask = a.slots - 1;
    const uint32_t lane = __lane_id();
    const uint64_t window = a.slots < 64ull * kFrontBatches ? a.slots : 64ull * kFrontBatches;
    uint64_t next = 0, pub = 0;
    uint64_t idle0 = wall_clock64();
    bool ok = true;
    for (;;) {
        // The published prefix of the next `window` tickets, 64 at a time.
        uint64_t c_total = 0;
        for (int r = 0; r < kFrontBatches; ++r) {
            const uint64_t idx = (uint64_t)r * 64 + lane;
            const uint64_t t = next + idx;
            const bool published = idx < window && ldr_sys(a.ring_seq + (t & smask)) == t + 1;
            const uint64_t mask = __ballot(published);
            const uint32_t c = ~mask == 0 ? 64u : (uint32_t)__builtin_ctzll(~mask);
            c_total += c;
            if (c < 64) break;
        }
        if (c_total == 0) {
            bool stop = false;
            if (lane == 0) stop = ldr_sys(a.stop) != 0;
            if (__shfl((int)stop, 0, 64)) break;
            if (wall_clock64() - idle0 > a.idle_ticks) {
                if (lane == 0) vshmem_detail::latch_error(a.c, 0x4u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");   // system scope: descriptors after their sequence words
        // Backlog-adaptive split: the item size is chunk_bytes times the
        // number of queued items per worker (published, not yet claimed),
        // at least 1 and at most kBacklogSplit.  A short queue keeps small
        // items that spread a request over many work-groups (latency); a
        // deep one gets large items that cut the per-item claim, drain and
        // release costs (throughput).  One decision per round, uniform over
        // the lanes.
        const uint64_t claimed = __shfl(lane == 0 ? ldr_dev(a.claim) : 0ull, 0, 64);
        const uint64_t per_worker = pub > claimed ? (pub - claimed) / nworkers : 0;
        const uint64_t chunk = per_worker <= 1 ? a.chunk : a.chunk * min<uint64_t>(per_worker, kBacklogSplit);
        uint64_t pos0 = pub;                            // next free item position
        uint64_t invalid = 0;                           // bit r: this lane's request of batch r is invalid
        for (int r = 0; r * 64ull < c_total; ++r) {
            const uint64_t t = next + (uint64_t)r * 64 + lane;
            const bool mine = (uint64_t)r * 64 + lane < c_total;
            const uint32_t slot = (uint32_t)(t & smask);
            shmemx_desc_t d{};
            bool valid = false;
            uint64_t nitems = 0;
            if (mine) {
                // After the acquire, plain 16-byte loads: the four loads of a
                // lane share one host cache line, fetched over PCIe once.
                const vshmem_detail::v4u *q = (const vshmem_detail::v4u *)(a.ring + slot);
                vshmem_detail::v4u w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] = q[i];
                memcpy(&d, w, sizeof(d));
                valid = valid_request(a.c, d);
                nitems = valid ? (d.nbytes == 0 ? 1 : (d.nbytes + chunk - 1) / chunk) : 0;
                if (!valid) invalid |= 1ull << r;
            }
            uint64_t incl = nitems;
            for (int off = 1; off < 64; off <<= 1) {
                const uint64_t y = __shfl_up(incl, off, 64);
                if ((int)lane >= off) incl += y;
            }
            const uint64_t first = incl - nitems;      // this lane's first item, relative to pos0
            const uint64_t total = __shfl(incl, 63, 64);
            if (mine) {
                Parent &P = a.parents[slot];
                P.d = d;
                P.ticket = t;
                P.t_start = 0;
                P.hash = 0;
                P.t_queued = wall_clock64();
                P.remaining = nitems;
                P.status = 0;
            }
            // The batch's items are spread over all lanes: item j belongs to
            // the last lane whose first item is <= j (lanes without items
            // share the next lane's first, so the last such lane owns it).
            for (uint64_t j0 = 0; j0 < total; j0 += 64) {
                if (pos0 + j0 + 64 - pub > a.qsize) {
                    // The queue holds qsize items: publish the ones written so
                    // far so that workers can free slots for the rest.
                    if (__ballot(!ok)) break;
                    vshmem_detail::release_agent();
                    for (uint64_t pos = pub + lane; pos < pos0 + j0; pos += 64)
                        __hip_atomic_store(&a.items[pos & qmask].seq, pos + 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    pub = pos0 + j0;
                }
                const uint64_t j = j0 + lane;
                uint32_t lo = 0, hi = 63;
#pragma unroll
                for (int step = 0; step < 6; ++step) {
                    const uint32_t mid = (lo + hi + 1) / 2;
                    const uint64_t f = __shfl(first, (int)mid, 64);
                    if (f <= j) lo = mid;
                    else hi = mid - 1;
                }
                const uint64_t o_first = __shfl(first, (int)lo, 64);
                const uint64_t o_ticket = __shfl(t, (int)lo, 64);
                const uint64_t o_bytes = __shfl(d.nbytes, (int)lo, 64);
                const uint32_t o_slot = (uint32_t)__shfl((int)slot, (int)lo, 64);
                if (j < total && ok) {
                    const uint64_t k = j - o_first;
                    const uint64_t pos = pos0 + j;
                    Item *it = a.items + (pos & qmask);
                    ok = wait_item_free(a, it, pos);
                    if (ok) {
                        it->parent = o_slot;
                        it->ticket = o_ticket;
                        it->lo = k * chunk;
                        it->hi = min(o_bytes, (k + 1) * chunk);
                    }
                }
            }
            pos0 += total;
        }
        if (__ballot(!ok)) break;            // an item slot never came free: shut down
        vshmem_detail::release_agent();   // records and items before their sequence words
        for (uint64_t pos = pub + lane; pos < pos0; pos += 64)
            __hip_atomic_store(&a.items[pos & qmask].seq, pos + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int r = 0; invalid >> r; ++r) {
            if ((invalid >> r) & 1) {
                const uint32_t slot = (uint32_t)((next + (uint64_t)r * 64 + lane) & smask);
                a.parents[slot].t_start = wall_clock64();
                vshmem_detail::latch_error(a.c, 0x2u);
                post_completion(a, slot, a.parents[slot], -1);
            }
        }
        next += c_total;
        pub = pos0;
        idle0 = wall_clock64();
    }
    // One poison item per worker work-group, lanes in parallel.
    for (uint64_t w0 = 0; w0 < nworkers; w0 += 64) {
        const uint64_t w = w0 + lane;
        bool freed = false;
        if (w < nworkers) {
            Item *it = a.items + ((pub + w - w0) & qmask);
            freed = wait_item_free(a, it, pub + w - w0);
            if (freed) it->parent = kItemPoison;
        }
        vshmem_detail::release_agent();
        if (freed)
            __hip_atomic_store(&a.items[(pub + w - w0) & qmask].seq, pub + w - w0 + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        pub += min<uint64_t>(64, nworkers - w0);
    }
}

// A worker work-group: thread 0 claims the next item ticket, waits for the
// item, and shares it through LDS; the whole work-group executes it (wide,
// contiguous streams keep HBM busy); the last item of a request posts its
// completion.
struct ClaimedItem {
    shmemx_desc_t d;
    uint64_t parent, lo, hi;
    int state;   // 0 run, 1 stop, 2 skip
};

// Finished items whose completion waits for the work-group's next release.
// One agent release covers every item the work-group finished before it, so
// a worker that goes straight on to the next ready item defers the release
// and the request counts it owes (at most kMaxHold items, at most
// hold_ticks old), and settles them before any wait and before an item of
// more than kHoldSpanBytes, whose copy would hold them back for longer than
// the release saves.  Thread 0 owns it.
constexpr uint32_t kMaxHold = 4;
constexpr uint64_t kHoldSpanBytes = 64u << 10;
struct Held {
    uint64_t parent[kMaxHold];
    uint64_t t_first;
    uint32_t n;
};

// Thread 0: one release for all held items, then their request counts; the
// last item of a request posts its completion.
__device__ void settle(const ProgArgs &a, Held &h)
{
    if (h.n == 0) return;
    vshmem_detail::release_agent();   // the work-group's stores of every held item, device-wide
    for (uint32_t k = 0; k < h.n; ++k) {
        Parent &P = a.parents[h.parent[k]];
        const uint64_t left = __hip_atomic_fetch_sub(&P.remaining, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (left == 1) {
            vshmem_detail::acquire_agent();
            post_completion(a, (uint32_t)h.parent[k], P, 0);
        }
    }
    h.n = 0;
}

// Thread 0 of the work-group: claim the next item and fill `ci`.  Held
// items are settled first unless the next item is already published, and
// whenever the claimed item has to be waited for.
__device__ void claim_item(const ProgArgs &a, ClaimedItem &ci, Held &h)
{
    const uint64_t qmask = a.qsize - 1;
    if (h.n) {
        const uint64_t c = __hip_atomic_load(a.claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ldr_dev(&a.items[c & qmask].seq) != c + 1 || wall_clock64() - h.t_first > a.hold_ticks) settle(a, h);
    }
    const uint64_t t = __hip_atomic_fetch_add(a.claim, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    Item *it = a.items + (t & qmask);
    const uint64_t t0 = wall_clock64();
    bool ready = true;
    while (ldr_dev(&it->seq) != t + 1) {
        settle(a, h);   // no-op once nothing is held
        __builtin_amdgcn_s_sleep(2);
        if (wall_clock64() - t0 > 2 * a.idle_ticks) {
            ready = false;
            break;
        }
    }
    ci.state = 1;
    if (!ready) return;
    vshmem_detail::acquire_agent();
    const uint64_t parent = ldr_dev(&it->parent);
    const uint64_t ticket = ldr_dev(&it->ticket);
    ci.lo = ldr_dev(&it->lo);
    ci.hi = ldr_dev(&it->hi);
    st_dev(&it->seq, t + a.qsize);   // the slot is free again
    if (parent == kItemPoison || ci.hi - ci.lo > kHoldSpanBytes) settle(a, h);
    if (parent == kItemPoison) return;
    Parent &P = a.parents[parent];
    load_desc(ci.d, &P.d, false);
    ci.parent = parent;
    if (ldr_dev(&P.ticket) != ticket) {
        // A record that does not belong to this item: report it, skip it.
        vshmem_detail::latch_error(a.c, 0x8u);
        ci.state = 2;
        return;
    }
    uint64_t zero = 0;
    __hip_atomic_compare_exchange_strong(&P.t_start, &zero, (uint64_t)wall_clock64(), __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ci.state = 0;
}

// Values every thread reads from LDS, made visibly uniform (scalar registers).
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ void uniform_copy(void *dst, const void *src, size_t bytes)
{
    uint32_t *d = (uint32_t *)dst;
    const uint32_t *q = (const uint32_t *)src;
    for (size_t i = 0; i < bytes / 4; ++i) d[i] = __builtin_amdgcn_readfirstlane(q[i]);
}

// Every branch around a barrier below is uniform across the work-group and
// visibly so to the compiler (wavefront index and item state go through
// readfirstlane): a loop whose exit the compiler must treat as divergent
// can be restructured so that some lanes cycle through the barriers while
// thread 0, which claims the next item, stays masked off.
__device__ void worker(const ProgArgs &a)
{
    __shared__ ClaimedItem ci;
    __shared__ Held held;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    if (threadIdx.x == 0) held.n = 0;
    for (;;) {
        if (wave == 0) {
            if (__lane_id() == 0) claim_item(a, ci, held);
        }
        __syncthreads();
        const int state = __builtin_amdgcn_readfirstlane(ci.state);
        if (state == 1) break;
        if (state == 0) {
            shmemx_desc_t d;
            uniform_copy(&d, &ci.d, sizeof(d));
            const uint64_t parent = uniform_u64(ci.parent), lo = uniform_u64(ci.lo), hi = uniform_u64(ci.hi);
            Parent &P = a.parents[parent];
            exec_item(a, d, lo, hi, &P.hash);
            vshmem_detail::wait_vm_complete();   // this thread's stores of the item reached L2
            __syncthreads();
            if (threadIdx.x == 0) {
                // Held until thread 0's next release (see Held).
                if (held.n == 0) held.t_first = wall_clock64();
                held.parent[held.n++] = parent;
                if (held.n == kMaxHold) settle(a, held);
            }
        }
        __syncthreads();   // every thread is done with `ci` before the next claim
    }
}

__global__ void __launch_bounds__(1024) k_progress(ProgArgs a)
{
    // Work-group 0: its first wavefront is the front-end, its other
    // wavefronts idle.  Every other work-group is one worker.
    if (blockIdx.x == 0) {
        if (threadIdx.x < 64) front_end(a, (uint64_t)gridDim.x - 1);
        return;
    }
    worker(a);
}

// Start-up state of a run: item k free for ticket k (seq = k, the rest
// zero), every request record and the claim counter zero.  Grid-stride.
static_assert(sizeof(Parent) % 8 == 0, "request records are whole words");
__global__ void __launch_bounds__(256) k_progress_init(Item *items, uint64_t qsize, uint64_t *parent_words,
                                                        uint64_t nwords, uint64_t *claim)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = g; k < qsize; k += stride) items[k] = Item{k, 0, 0, 0, 0, {0, 0, 0}};
    for (uint64_t k = g; k < nwords; k += stride) parent_words[k] = 0;
    if (g < 256 / 8) claim[g] = 0;
}

// One request executed by a launch of its own (the per-op serving form):
// work-group b handles bytes [b*chunk, (b+1)*chunk) of the request.
__global__ void __launch_bounds__(1024) k_request(shmemx_dctx_pub_t c, shmemx_desc_t d, uint64_t chunk)
{
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint64_t hi = min(d.nbytes, lo + chunk);
    if (lo < hi) exec_request_range(c, d, lo, hi, threadIdx.x, blockDim.x);
    vshmem_detail::release_wg_at_exit();   // quiet
}

}  // namespace

namespace vshmem {
bool valid_request_host(const shmemx_desc_t &d)
{
    const State &s = st();
    if (d.issuer_pe < 0 || d.issuer_pe >= s.npes || d.target_pe < 0 || d.target_pe >= s.npes) return false;
    if (d.op == SHMEMX_OP_PUT || d.op == SHMEMX_OP_GET) return in_user_heap(d.src, d.nbytes) && in_user_heap(d.dst, d.nbytes);
    if (d.op == SHMEMX_OP_AMO_FETCH_ADD)
        return (d.nbytes & 7) == 0 && (d.src & 7) == 0 && (d.dst & 7) == 0 && in_user_heap(d.src, d.nbytes) &&
               in_user_heap(d.dst, d.nbytes);
    return false;
}
}  // namespace vshmem

namespace {

// ------------------------------------------------------------------ host
struct Progress {
    bool running = false;
    uint64_t qsize = 0;
    hipStream_t stream = nullptr;
    shmemx_desc_t *ring = nullptr;     // pinned host
    uint64_t *ring_seq = nullptr;      // pinned host
    uint64_t *ring_done = nullptr;     // pinned host
    shmemx_completion_t *comp = nullptr;
    uint64_t *stop = nullptr;
    Item *items = nullptr;             // device
    Parent *parents = nullptr;         // device
    uint64_t *claim = nullptr;         // device
    uint64_t slots = 0;
    std::atomic<uint64_t> head{0};
    int reserved_cus = 0;   // CUs its work-groups hold while it runs
};

Progress g_prog;

void release_progress()
{
    Progress &p = g_prog;
    if (p.ring) (void)hipHostFree(p.ring);
    if (p.ring_seq) (void)hipHostFree(p.ring_seq);
    if (p.ring_done) (void)hipHostFree(p.ring_done);
    if (p.comp) (void)hipHostFree(p.comp);
    if (p.stop) (void)hipHostFree(p.stop);
    if (p.items) (void)hipFree(p.items);
    if (p.parents) (void)hipFree(p.parents);
    if (p.claim) (void)hipFree(p.claim);
    p.ring = nullptr;
    p.ring_seq = nullptr;
    p.ring_done = nullptr;
    p.comp = nullptr;
    p.stop = nullptr;
    p.items = nullptr;
    p.parents = nullptr;
    p.claim = nullptr;
    p.running = false;
}

template <typename T>
int host_alloc(T **p, size_t bytes)
{
    if (VSHMEM_HIP_FAILED(hipHostMalloc((void **)p, bytes, hipHostMallocMapped | hipHostMallocCoherent))) return SHMEMX_ERR_HIP;
    memset(*p, 0, bytes);
    return SHMEMX_OK;
}

template <typename T>
T *dev_view(T *host)
{
    void *d = nullptr;
    if (VSHMEM_HIP_FAILED(hipHostGetDevicePointer(&d, host, 0))) return nullptr;
    return (T *)d;
}

}  // namespace

namespace vshmem {
bool progress_running() { return g_prog.running; }
void progress_release() { release_progress(); }
int progress_reserved_cus() { return g_prog.running ? g_prog.reserved_cus : 0; }
}  // namespace vshmem

extern "C" {

int shmemx_progress_start(const shmemx_progress_cfg_t *cfg_in, void *stream)
{
    if (int rc = check_ready()) return rc;
    Progress &p = g_prog;
    if (p.running) return SHMEMX_ERR_BUSY;
    shmemx_progress_cfg_t cfg{};
    if (cfg_in) cfg = *cfg_in;
    if (cfg.wg_size == 0) cfg.wg_size = 1024;
    if (cfg.ring_slots == 0) cfg.ring_slots = 4096;
    if (cfg.chunk_bytes == 0) cfg.chunk_bytes = 256ull << 10;
    if (cfg.idle_timeout_ms == 0) cfg.idle_timeout_ms = 30000;
    const State &s = st();
    if (cfg.nwg == 0) cfg.nwg = s.num_cus;
    if (!valid_wg_size(cfg.wg_size) || cfg.nwg < 2 || cfg.nwg > 8 * s.num_cus || cfg.ring_slots < 2 ||
        (cfg.ring_slots & (cfg.ring_slots - 1)) || (cfg.chunk_bytes & 15) || cfg.chunk_bytes > (1ull << 40))
        return SHMEMX_ERR_ARG;
    const uint64_t slots = (uint64_t)cfg.ring_slots;
    const uint64_t qsize = 1ull << 16;
    if (p.ring && p.slots != slots) release_progress();
    int rc = SHMEMX_OK;
    if (!p.ring) {
        rc = host_alloc(&p.ring, slots * sizeof(shmemx_desc_t));
        if (!rc) rc = host_alloc(&p.ring_seq, slots * sizeof(uint64_t));
        if (!rc) rc = host_alloc(&p.ring_done, slots * sizeof(uint64_t));
        if (!rc) rc = host_alloc(&p.comp, slots * sizeof(shmemx_completion_t));
        if (!rc) rc = host_alloc(&p.stop, 64);
        if (!rc && VSHMEM_HIP_FAILED(hipMalloc((void **)&p.items, qsize * sizeof(Item)))) rc = SHMEMX_ERR_HIP;
        if (!rc && VSHMEM_HIP_FAILED(hipMalloc((void **)&p.parents, slots * sizeof(Parent)))) rc = SHMEMX_ERR_HIP;
        if (!rc && VSHMEM_HIP_FAILED(hipMalloc((void **)&p.claim, 256))) rc = SHMEMX_ERR_HIP;
    }
    if (rc || !p.ring_seq || !p.ring_done || !p.comp || !p.stop || !p.items || !p.parents || !p.claim) {
        if (!rc) rc = SHMEMX_ERR_HIP;
        release_progress();
        return rc;
    }
    for (uint64_t i = 0; i < slots; ++i) {
        p.ring_seq[i] = i;
        p.ring_done[i] = 0;
    }
    memset(p.comp, 0, slots * sizeof(shmemx_completion_t));
    *p.stop = 0;
    hipStream_t hs = (hipStream_t)stream;
    // Device-side reset, ordered before the kernel on the same stream.
    hipLaunchKernelGGL(k_progress_init, dim3(256), dim3(256), 0, hs, p.items, qsize, (uint64_t *)p.parents,
                       slots * sizeof(Parent) / 8, p.claim);
    if (VSHMEM_HIP_FAILED(hipGetLastError())) {
        release_progress();
        return SHMEMX_ERR_HIP;
    }
    ProgArgs a{};
    a.c = pub();
    a.ring = dev_view(p.ring);
    a.ring_seq = dev_view(p.ring_seq);
    a.ring_done = dev_view(p.ring_done);
    a.comp = dev_view(p.comp);
    a.stop = dev_view(p.stop);
    if (!a.ring || !a.ring_seq || !a.ring_done || !a.comp || !a.stop) {
        release_progress();
        return SHMEMX_ERR_HIP;
    }
    a.items = p.items;
    a.parents = p.parents;
    a.claim = p.claim;
    a.slots = slots;
    a.qsize = qsize;
    a.chunk = cfg.chunk_bytes;
    a.idle_ticks = cfg.idle_timeout_ms * (s.wallclock_hz / 1000);
    a.hold_ticks = s.wallclock_hz / 50000;   // 20 us
    a.verify = cfg.verify;
    p.slots = slots;
    p.head.store(0);
    p.stream = hs;
    // The CUs its work-groups occupy (per_cu of them fit a CU; a CU that
    // holds any is taken as full by the co-residency checks).
    int per_cu = 0;
    if (int rc2 = blocks_per_cu(k_progress, cfg.wg_size, &per_cu)) {
        release_progress();
        return rc2;
    }
    p.reserved_cus = per_cu > 0 ? std::min(s.num_cus, (cfg.nwg + per_cu - 1) / per_cu) : s.num_cus;
    hipLaunchKernelGGL(k_progress, dim3(cfg.nwg), dim3(cfg.wg_size), 0, hs, a);
    if (VSHMEM_HIP_FAILED(hipGetLastError())) {
        release_progress();
        return SHMEMX_ERR_HIP;
    }
    p.running = true;
    return SHMEMX_OK;
}

int shmemx_launch_request(const shmemx_desc_t *desc, uint64_t chunk_bytes, int wg_size, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!desc || !valid_request_host(*desc) || chunk_bytes == 0 || (chunk_bytes & 15) || !valid_wg_size(wg_size))
        return SHMEMX_ERR_ARG;
    const uint64_t nb = desc->nbytes ? (desc->nbytes + chunk_bytes - 1) / chunk_bytes : 1;
    if (nb > (1u << 30)) return SHMEMX_ERR_ARG;
    hipLaunchKernelGGL(k_request, dim3((unsigned)nb), dim3(wg_size), 0, (hipStream_t)stream, pub(), *desc, chunk_bytes);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_progress_submit(int lane, const shmemx_desc_t *desc, uint64_t *ticket)
{
    Progress &p = g_prog;
    if (!p.running) return SHMEMX_ERR_STATE;
    if (!desc || !ticket || lane < 0 || lane >= SHMEMX_PROGRESS_LANES) return SHMEMX_ERR_ARG;
    const uint64_t mask = p.slots - 1;
    uint64_t t = p.head.load(std::memory_order_relaxed);
    for (;;) {
        const uint64_t s = __atomic_load_n(p.ring_seq + (t & mask), __ATOMIC_ACQUIRE);
        if (s == t) {
            if (p.head.compare_exchange_weak(t, t + 1, std::memory_order_relaxed)) break;
        } else if (s < t) {
            return SHMEMX_ERR_BUSY;   // the slot still holds a request in flight: the ring is full
        } else {
            t = p.head.load(std::memory_order_relaxed);
        }
    }
    shmemx_desc_t *slot = p.ring + (t & mask);
    *slot = *desc;
    slot->reserved = (uint64_t)lane;     // carried to the completion record
    __atomic_store_n(p.ring_seq + (t & mask), t + 1, __ATOMIC_RELEASE);
    *ticket = t;
    return SHMEMX_OK;
}

int shmemx_progress_poll(uint64_t ticket, shmemx_completion_t *out)
{
    Progress &p = g_prog;
    if (!p.ring_seq) return SHMEMX_ERR_STATE;
    const uint64_t slot = ticket & (p.slots - 1);
    uint64_t s = __atomic_load_n(p.ring_seq + slot, __ATOMIC_ACQUIRE);
    if (s > ticket + 1) {               // consumed by an earlier poll: the record is gone
        if (out) {
            memset(out, 0, sizeof(*out));
            out->ticket = ticket;
        }
        return 1;
    }
    if (s != ticket + 1) return 0;      // not submitted
    if (__atomic_load_n(p.ring_done + slot, __ATOMIC_ACQUIRE) != ticket + 1) return 0;
    shmemx_completion_t c = p.comp[slot];
    // Consume: free the slot for ticket + slots (only one poller wins).
    if (!__atomic_compare_exchange_n(p.ring_seq + slot, &s, ticket + p.slots, false, __ATOMIC_ACQ_REL,
                                     __ATOMIC_ACQUIRE)) {
        memset(&c, 0, sizeof(c));
        c.ticket = ticket;
    }
    if (out) *out = c;
    return 1;
}

int shmemx_progress_stop(int timeout_ms)
{
    Progress &p = g_prog;
    if (!p.running) return SHMEMX_ERR_STATE;
    __atomic_store_n(p.stop, 1ull, __ATOMIC_RELEASE);
    auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        hipError_t e = hipStreamQuery(p.stream);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) {
            release_progress();
            return SHMEMX_ERR_HIP;
        }
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms)) return SHMEMX_ERR_TIMEOUT;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    p.running = false;     // buffers stay allocated for the next start
    return SHMEMX_OK;
}

}  // extern "C"
