// Batches over a descriptor table that lives in DEVICE memory.  The table is
// read on the device at every launch, so a kernel (or a copy) may rewrite it
// between launches; the host never sees its contents.
//
// The fused form runs three kernels on the caller's stream and together they
// derive what the host plan builder derives.  The classify kernel (one
// thread per descriptor) validates each operation and resolves its scope and
// chunking from the tune table; the index kernel (one work-group) finds each
// operation's phase from its issuer's ordering points (barriers seen, fences
// and quiets since the last barrier) and counting-sorts the operations by
// (phase, kind).  The executor then runs the phases in order; inside a
// phase the tasks (work-group byte ranges first, then wavefront packs, then
// single-lane packs) are dealt to its work-groups round robin, and a grid
// barrier separates the phases.
// Long-lived kernels that consume descriptor tables are the paper's Section 3
// case for device-side batching; the stream-ordered forms of Section 4.3 are
// what the caller's stream gives.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "exec.hpp"
#include "runtime.hpp"

using namespace vshmem;
using namespace vshmem_exec;

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kIndexThreads = 1024;
constexpr int kIndexWaves = kIndexThreads / 64;
constexpr int kClassifyThreads = 256;
constexpr int kIndexMaxPes = 4096;          // per-issuer ordering state held in LDS
constexpr int kIndexItems = 8;              // descriptors per index thread per tile
constexpr uint32_t kLdsEpochs = 4096;       // epochs whose counters the index kernel keeps in LDS
constexpr uint32_t kLdsBuckets = 8192;      // buckets whose counters the index kernel keeps in LDS
constexpr uint32_t kExecLdsPhases = 512;    // phases whose bounds the executor keeps in LDS
constexpr uint32_t kIndexTile = kIndexThreads * kIndexItems;
static_assert(kIndexThreads <= (1 << 19) && kIndexMaxPes <= (1 << 12), "sync_entry packs 19 + 1 + 12 bits");
constexpr uint64_t kMaxTable = 1ull << 26;  // descriptors per table

// Control words of one workspace (written by the index kernel).
struct Ctl {
    uint32_t nphases;
    uint32_t active;   // executor work-groups that take part (the rest leave at once)
    uint32_t last;     // 1 + the last phase that has tasks (0: nothing to run)
    uint32_t nvalid;   // operations that execute
    uint32_t pad[12];
};

// Sections of a workspace for tables of up to `cap` descriptors.  The
// barrier words come first: count at 0 and generation VSHMEM_SYNC_GEN_OFF
// further, the layout counter_barrier expects.
struct Ws {
    uint64_t *bar;
    Ctl *ctl;
    uint32_t *eb;      // per op: barrier epoch (kNone: not executed)
    uint32_t *ef;      // per op: fences since the epoch began
    uint32_t *key;     // per op: class word, then bucket = 3 * phase + kind (kNone: not executed)
    uint32_t *nch;     // per op: work-group tasks (0 for packed kinds)
    uint32_t *sorted;  // op indices by bucket
    uint32_t *maxf;    // per epoch: largest fence count of an op in it
    uint32_t *base;    // per epoch: its first phase
    uint32_t *cnt;     // per bucket: count, then scatter cursor
    uint32_t *off;     // per bucket: first sorted position (one extra entry: the end)
    uint64_t *cs;      // per sorted position: first work-group task (one extra entry)
};

constexpr uint64_t kHeaderBytes = VSHMEM_SYNC_GEN_OFF + 256;

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }
uint64_t phase_cap(uint64_t cap) { return 2 * cap + 1; }
uint64_t bucket_cap(uint64_t cap) { return 3 * phase_cap(cap) + 1; }

// Byte size of each section, in carve order.
void sections(uint64_t cap, uint64_t out[12])
{
    const uint64_t c4 = cap * 4;
    out[0] = c4;                              // eb
    out[1] = c4;                              // ef
    out[2] = c4;                              // key
    out[3] = c4;                              // nch
    out[4] = c4;                              // sorted
    out[5] = (cap + 1) * 4;                   // maxf
    out[6] = (cap + 1) * 4;                   // base
    out[7] = bucket_cap(cap) * 4;             // cnt
    out[8] = bucket_cap(cap) * 4;             // off
    out[9] = (cap + 1) * 8;                   // cs
    out[10] = 0;
}

uint64_t ws_bytes(uint64_t cap)
{
    uint64_t s[12], total = kHeaderBytes;
    sections(cap, s);
    for (int i = 0; i < 10; ++i) total += align256(s[i]);
    return total;
}

// Largest table a workspace of `bytes` holds.
uint64_t ws_capacity(uint64_t bytes)
{
    uint64_t lo = 0, hi = kMaxTable;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) / 2;
        if (ws_bytes(mid) <= bytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

Ws ws_carve(uint8_t *w, uint64_t cap)
{
    Ws r;
    r.bar = (uint64_t *)w;
    r.ctl = (Ctl *)(w + 128);
    uint64_t s[12];
    sections(cap, s);
    uint8_t *p = w + kHeaderBytes;
    void **dst[10] = {(void **)&r.eb,     (void **)&r.ef,   (void **)&r.key,  (void **)&r.nch,
                      (void **)&r.sorted, (void **)&r.maxf, (void **)&r.base, (void **)&r.cnt,
                      (void **)&r.off,    (void **)&r.cs};
    for (int i = 0; i < 10; ++i) {
        *dst[i] = p;
        p += align256(s[i]);
    }
    return r;
}

struct BatchArgs {
    shmemx_dctx_pub_t c;
    const shmemx_desc_t *D;
    uint32_t n;
    uint32_t exec_wg;    // executor work-group size
    uint32_t exec_grid;  // executor grid
    uint32_t pad;
    const shmemx_tune_t *tune;
    uint64_t *results;
    Ws w;
};

// ---------------------------------------------------------------- device
__device__ __forceinline__ bool dev_in_heap(const shmemx_dctx_pub_t &c, uint64_t off, uint64_t n)
{
    return off <= c.user_bytes && n <= c.user_bytes - off;
}

// A data operation (put, get, signal-put, atomic) the batch can execute:
// PEs, ranges inside the user heap, aligned words, a known scope, and a
// result index inside the n-entry result array.
__device__ __forceinline__ bool dev_valid(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d, uint32_t n,
                                          const uint64_t *results)
{
    if (d.target_pe < 0 || d.target_pe >= c.npes) return false;
    if (d.scope > SHMEMX_SCOPE_GRID && d.scope != SHMEMX_SCOPE_AUTO) return false;
    if (is_amo_op(d.op)) {
        const bool fetching = d.op != SHMEMX_OP_AMO_ADD && d.op != SHMEMX_OP_AMO_XOR && d.op != SHMEMX_OP_AMO_SET;
        if (fetching && results && d.result_idx != SHMEMX_NO_RESULT && d.result_idx >= n) return false;
        return (d.src & 7) == 0 && dev_in_heap(c, d.src, 8);
    }
    if (!dev_in_heap(c, d.src, d.nbytes) || !dev_in_heap(c, d.dst, d.nbytes)) return false;
    if (d.op == SHMEMX_OP_PUT_SIGNAL && ((d.cond & 7) || !dev_in_heap(c, d.cond, 8))) return false;
    return true;
}

__device__ __forceinline__ bool is_data_op(uint8_t op)
{
    return op == SHMEMX_OP_PUT || op == SHMEMX_OP_GET || op == SHMEMX_OP_PUT_SIGNAL || is_amo_op(op);
}

// Exclusive prefix sum over a work-group of NW wavefronts; *total receives
// the sum.  Every thread calls it.  The wavefront totals are read back all
// at once (one LDS latency, not NW).
template <int NW, typename T>
__device__ __forceinline__ T block_scan(T x, T *total)
{
    __shared__ __align__(16) T wsum[NW];
    const uint32_t lane = __lane_id(), w = threadIdx.x / 64;
    T incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T y = __shfl_up(incl, off, 64);
        if ((int)lane >= off) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    T v[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) v[k] = wsum[k];
    T before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        before += (uint32_t)k < w ? v[k] : 0;
        all += v[k];
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

__device__ __forceinline__ shmemx_desc_t load_desc(const shmemx_desc_t *p)
{
    shmemx_desc_t d;
    const vshmem_detail::v4u *q = (const vshmem_detail::v4u *)p;
    vshmem_detail::v4u w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = q[i];
    memcpy(&d, w, sizeof(d));
    return d;
}

// The fields the classify kernel reads: all but value and reserved (zero in
// the copy).
__device__ __forceinline__ shmemx_desc_t load_desc_head(const shmemx_desc_t *p)
{
    const vshmem_detail::v4u *q = (const vshmem_detail::v4u *)p;
    const vshmem_detail::v4u w0 = q[0], w1 = q[1];
    const uint64_t *u = (const uint64_t *)p;
    shmemx_desc_t d;
    memcpy(&d, &w0, 16);
    memcpy((uint8_t *)&d + 16, &w1, 16);
    d.nbytes = u[4];
    d.value = 0;
    d.cond = u[6];
    d.reserved = 0;
    return d;
}

__device__ __forceinline__ uint32_t ld_l2(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront-aggregated counters over R items per lane.  Consecutive
// descriptors mostly share their (phase, kind) and their epoch, so one atomic
// per distinct key per wavefront replaces one per descriptor: a single
// counter hit by every descriptor of a table serialises in L2.

// Picks the next key still to do: the key of the first (item, lane) in
// `todo` order.  Every lane returns the same key.
template <int R>
__device__ __forceinline__ uint32_t agg_next(const uint32_t (&key)[R], const uint64_t (&todo)[R])
{
    uint32_t k = 0;
    bool found = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!found && todo[r]) {
            k = __builtin_amdgcn_readlane(key[r], __builtin_ctzll(todo[r]));
            found = true;
        }
    }
    return k;
}

// counter[key[r]] += 1 for each item with valid[r].  With RET, pos[r]
// receives the item's slot: the counter's value before the item's own
// increment.  When every valid item of the wavefront has one key (runs of
// operations of one phase and kind), one atomic serves them all; otherwise
// an LDS counter takes one atomic per item (the LDS resolves equal
// addresses itself) and a counter in memory one per distinct key.
template <int R, bool RET, bool LDS>
__device__ __forceinline__ void agg_inc(uint32_t *counter, const uint32_t (&key)[R], const bool (&valid)[R],
                                        uint32_t (&pos)[R])
{
    const uint32_t lane = __lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t todo[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        todo[r] = __ballot(valid[r]);
        any |= todo[r] != 0;
    }
    if (!any) return;
    uint32_t k = agg_next<R>(key, todo);
    bool one = true;
#pragma unroll
    for (int r = 0; r < R; ++r) one &= __ballot(valid[r] && key[r] != k) == 0;
    if (LDS && !one) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (valid[r]) {
                if (RET) pos[r] = atomicAdd(counter + key[r], 1u);
                else (void)atomicAdd(counter + key[r], 1u);
            }
        }
        return;
    }
    for (;;) {
        uint64_t same[R];
        uint32_t total = 0;
        int leader = 64;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            same[r] = __ballot(valid[r] && key[r] == k) & todo[r];
            total += (uint32_t)__builtin_popcountll(same[r]);
            if (leader == 64 && same[r]) leader = __builtin_ctzll(same[r]);
        }
        uint32_t base = 0;
        if ((int)lane == leader) {
            if (RET) base = atomicAdd(counter + k, total);
            else (void)atomicAdd(counter + k, total);
        }
        if (RET) {
            base = __builtin_amdgcn_readlane(base, leader);
            uint32_t before = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if ((same[r] >> lane) & 1ull) pos[r] = base + before + (uint32_t)__builtin_popcountll(same[r] & below);
                before += (uint32_t)__builtin_popcountll(same[r]);
            }
        }
        any = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            todo[r] &= ~same[r];
            any |= todo[r] != 0;
        }
        if (!any) break;
        k = agg_next<R>(key, todo);
    }
}

// Class word of a descriptor, written by the classify kernel: issuer in
// bits 0-11, type in bits 12-13, kind in bits 14-15.
constexpr uint32_t kTypeSkip = 0;      // NOP or invalid: not executed
constexpr uint32_t kTypeFence = 1;     // fence or quiet
constexpr uint32_t kTypeBarrier = 2;   // barrier_all
constexpr uint32_t kTypeData = 3;      // executes
__device__ __forceinline__ uint32_t class_word(uint32_t iss, uint32_t type, uint32_t kind)
{
    return iss | (type << 12) | (kind << 14);
}
__device__ __forceinline__ uint32_t class_type(uint32_t cw) { return (cw >> 12) & 3u; }
__device__ __forceinline__ uint32_t class_kind(uint32_t cw) { return cw >> 14; }
__device__ __forceinline__ uint32_t class_issuer(uint32_t cw) { return cw & 0xFFFu; }

// One entry of a tile's list of ordering points: tile position, barrier
// flag, issuer.
__device__ __forceinline__ uint32_t sync_entry(uint32_t pos, bool barrier, uint32_t iss)
{
    return (pos << 13) | ((uint32_t)barrier << 12) | iss;
}

// v[r] = p[i0 + r] for i0 + r < n, else `fill`.  A whole run is read as
// 16-byte vectors (i0 is a multiple of R and the sections are 256-byte
// aligned).
template <int R>
__device__ __forceinline__ void load_run(const uint32_t *p, uint32_t i0, uint32_t n, uint32_t fill, uint32_t (&v)[R])
{
    if (i0 + R <= n) {
#pragma unroll
        for (int q = 0; q < R / 4; ++q) {
            const vshmem_detail::v4u x = *(const vshmem_detail::v4u *)(p + i0 + 4 * q);
            v[4 * q] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = i0 + r < n ? p[i0 + r] : fill;
    }
}

// p[i0 + r] = v[r] for i0 + r < n.
template <int R>
__device__ __forceinline__ void store_run(uint32_t *p, uint32_t i0, uint32_t n, const uint32_t (&v)[R])
{
    if (i0 + R <= n) {
#pragma unroll
        for (int q = 0; q < R / 4; ++q)
            *(vshmem_detail::v4u *)(p + i0 + 4 * q) = vshmem_detail::v4u{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (i0 + r < n) p[i0 + r] = v[r];
    }
}

// Classify kernel: one thread per descriptor, over the whole GPU.  It
// validates the descriptor, resolves its scope and chunking, and writes its
// class word (to the key section) and its work-group task count.  Invalid
// descriptors latch SHMEMX_DEVERR_BAD_DESC and are skipped.
__global__ void __launch_bounds__(kClassifyThreads) k_batch_classify(BatchArgs a)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const shmemx_desc_t d = load_desc_head(a.D + i);
    const uint32_t iss = (uint32_t)d.issuer_pe;
    const bool iss_ok = iss < (uint32_t)a.c.npes;
    uint32_t type = kTypeSkip, kind = 0, nch = 0;
    if (iss_ok && is_sync_op(d.op)) {
        type = d.op == SHMEMX_OP_BARRIER_ALL ? kTypeBarrier : kTypeFence;
    } else if (iss_ok && is_data_op(d.op) && dev_valid(a.c, d, a.n, a.results)) {
        const shmemx_tune_t &tune = *a.tune;
        const int sc = resolve_scope(d, tune);
        kind = sc == SHMEMX_SCOPE_THREAD ? 2u : (sc == SHMEMX_SCOPE_WAVE ? 1u : 0u);
        if (kind == 0) {
            const uint64_t ch = resolve_chunk(d, sc, tune);
            const uint64_t k = d.nbytes ? (d.nbytes + ch - 1) / ch : 1;
            nch = k < 0xFFFFFFFFull ? (uint32_t)k : 0xFFFFFFFFu;
        }
        type = kTypeData;
    } else if (d.op != SHMEMX_OP_NOP) {
        // A bad code, WAIT_UNTIL, a bad issuer or an invalid operation.
        vshmem_detail::latch_error(a.c, SHMEMX_DEVERR_BAD_DESC);
    }
    a.w.key[i] = class_word(iss_ok ? iss : 0, type, kind);
    a.w.nch[i] = nch;
}

// Index kernel: one work-group of kIndexThreads threads, after the classify
// kernel.  It walks the table in tiles of kIndexTile positions and loads a
// tile's words before it uses them, so one work-group pays one memory
// latency per tile and pass.  Past pass 1, thread t takes the run of
// kIndexItems consecutive positions starting at t * kIndexItems: it reads
// and writes its per-descriptor words as 16-byte vectors, and a tile needs
// one work-group scan of per-thread sums.  The per-epoch and per-bucket
// counters live in LDS while they fit (the usual case), so the counting
// sort runs on LDS atomics.
__global__ void __launch_bounds__(kIndexThreads) k_batch_index(BatchArgs a)
{
    constexpr int R = kIndexItems;
    __shared__ uint32_t nbar[kIndexMaxPes], nfen[kIndexMaxPes];
    __shared__ uint32_t lsync[kIndexThreads];
    __shared__ __align__(16) uint32_t wcount[2][kIndexWaves];
    __shared__ uint32_t s_tmask[3];
    __shared__ uint32_t lepoch[kLdsEpochs];    // per epoch: largest fence count, then first phase
    __shared__ uint32_t lcnt[kLdsBuckets];     // per bucket: count, then scatter cursor
    __shared__ uint32_t s_max, s_last, s_bad, s_wg;
    const uint32_t tid = threadIdx.x, nt = blockDim.x, n = a.n;
    const int npes = a.c.npes;
    const Ws &w = a.w;

    for (int p = tid; p < npes; p += nt) nbar[p] = nfen[p] = 0;
    for (uint32_t b = tid; b < kLdsEpochs; b += nt) lepoch[b] = 0;
    for (uint32_t b = kLdsEpochs + tid; b <= n; b += nt) w.maxf[b] = 0;   // epochs past the LDS ones
    if (tid == 0) {
        s_max = 0;
        s_wg = 0;
        s_last = 0;
        s_bad = 0;
        s_tmask[0] = 0;
    }
    __syncthreads();

    // Pass 1: each operation's (barrier epoch, fences since) from its issuer's
    // ordering points.  A tile's class words are loaded at once (position
    // r * kIndexThreads + t of the tile in item r of thread t), then walked
    // one sub-tile of kIndexThreads positions at a time: an operation starts
    // from its issuer's state at the sub-tile's start and applies the
    // sub-tile's points that precede it, so the walk costs the sub-tile's
    // points, not the tile's.
    const uint32_t lane = __lane_id(), wave = tid / 64;
    const uint64_t lanes_below = (1ull << lane) - 1ull;
    for (uint32_t t0 = 0; t0 < n; t0 += kIndexTile) {
        uint32_t cw[R], ebr[R], efr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t i = t0 + r * nt + tid;
            cw[r] = i < n ? w.key[i] : 0;
            ebr[r] = kNone;
            efr[r] = 0;
        }
        // The sub-tiles that hold ordering points (bit r), once per tile: the
        // others need no barrier at all.  Three masks in turn: thread 0 clears
        // the one the next tile fills, which every thread last read two tiles
        // ago, before the previous tile's mask barrier that thread 0 has
        // passed; the next tile fills it only after this tile's.
        uint32_t msk = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t ty = class_type(cw[r]);
            msk |= __ballot(ty == kTypeFence || ty == kTypeBarrier) ? 1u << r : 0u;
        }
        const uint32_t tix = (t0 / kIndexTile) % 3;
        if (tid == 0) s_tmask[(tix + 1) % 3] = 0;
        if (lane == 0 && msk) atomicOr(&s_tmask[tix], msk);
        __syncthreads();
        const uint32_t tmask = s_tmask[tix];
        // Results are stored once per tile: a work-group barrier waits for
        // every outstanding global access of the waves it joins.
#pragma unroll 1
        for (int r = 0; r < R && t0 + r * nt < n; ++r) {
            uint32_t c = cw[0];
#pragma unroll
            for (int q = 1; q < R; ++q) c = r == q ? cw[q] : c;
            const uint32_t ty = class_type(c), pe = class_issuer(c);
            const bool sync = ty == kTypeFence || ty == kTypeBarrier, live = ty == kTypeData;
            // The sub-tile's ordering points, in table order: a ballot per
            // wavefront and a prefix over the wavefront counts.
            uint32_t nsync = 0, nb = 0;
            if ((tmask >> r) & 1u) {
                const uint64_t m = __ballot(sync);
                uint32_t *wc = wcount[r & 1];   // alternate: a fast wave may already write the next sub-tile's
                if (lane == 0) wc[wave] = (uint32_t)__builtin_popcountll(m);
                __syncthreads();
                uint32_t wv[kIndexWaves], before = 0;
#pragma unroll
                for (int k = 0; k < kIndexWaves; ++k) wv[k] = wc[k];
#pragma unroll
                for (int k = 0; k < kIndexWaves; ++k) {
                    before += (uint32_t)k < wave ? wv[k] : 0;
                    nsync += wv[k];
                }
                nb = before + (uint32_t)__builtin_popcountll(m & lanes_below);   // points before me
            }
            if (nsync) {
                if (sync) lsync[nb] = sync_entry(tid, ty == kTypeBarrier, pe);
                __syncthreads();
            }
            // An operation's state, and an ordering point's state after it;
            // the last point of an issuer in the sub-tile carries the issuer's
            // state into the next.
            uint32_t eb = 0, ef = 0;
            bool last = false;
            if (live || sync) {
                eb = nbar[pe];
                ef = nfen[pe];
                for (uint32_t j = 0; j < nb; ++j) {
                    const uint32_t e = lsync[j];
                    if ((e & 0xFFFu) == pe) {
                        const bool bar = (e >> 12) & 1u;
                        eb = bar ? eb + 1 : eb;
                        ef = bar ? 0 : ef + 1;
                    }
                }
                if (sync) {
                    const bool bar = ty == kTypeBarrier;
                    eb = bar ? eb + 1 : eb;
                    ef = bar ? 0 : ef + 1;
                    last = true;
                    for (uint32_t j = nb + 1; j < nsync; ++j) {
                        if ((lsync[j] & 0xFFFu) == pe) {
                            last = false;
                            break;
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                ebr[q] = r == q ? (live ? eb : kNone) : ebr[q];
                efr[q] = r == q ? ef : efr[q];
            }
            // Epoch maxima: one atomic per wavefront when its operations share
            // (epoch, fences), as runs of operations between ordering points do.
            const uint64_t lm = __ballot(live);
            if (lm) {
                const int fl = __builtin_ctzll(lm);
                const uint32_t eb0 = __builtin_amdgcn_readlane(eb, fl), ef0 = __builtin_amdgcn_readlane(ef, fl);
                const bool one = __ballot(live && (eb != eb0 || ef != ef0)) == 0;
                if (one ? (int)lane == fl : live) {
                    if (eb < kLdsEpochs) atomicMax(&lepoch[eb], ef);
                    else atomicMax(&w.maxf[eb], ef);
                }
            }
            if (nsync) {
                __syncthreads();   // the walks' reads of nbar, nfen and lsync precede the update
                if (last) {
                    nbar[pe] = eb;
                    nfen[pe] = ef;
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t i = t0 + r * nt + tid;
            if (i < n) {
                w.eb[i] = ebr[r];
                w.ef[i] = efr[r];
            }
        }
    }
    // Every PE's program holds the same number of barriers.
    for (int p = tid; p < npes; p += nt)
        if (nbar[p] != nbar[0]) s_bad = 1;
    __syncthreads();
    if (s_bad) {
        if (tid == 0) {
            vshmem_detail::latch_error(a.c, SHMEMX_DEVERR_BAD_DESC);
            w.ctl->nphases = 0;
            w.ctl->active = 0;
            w.ctl->last = 0;
            w.ctl->nvalid = 0;
        }
        return;
    }
    const uint32_t nepochs = nbar[0] + 1;

    // Pass 2: first phase of each epoch (phases of epoch b: maxf[b] + 1).
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nepochs; b0 += nt) {
        const uint32_t b = b0 + tid;
        // Past the LDS epochs maxf was built with atomics (performed in L2):
        // read it the same way.
        const uint32_t v = b < nepochs ? (b < kLdsEpochs ? lepoch[b] : ld_l2(w.maxf + b)) + 1 : 0;
        uint32_t tot = 0;
        const uint32_t ex = block_scan<kIndexWaves, uint32_t>(v, &tot);
        if (b < nepochs) {
            if (b < kLdsEpochs) lepoch[b] = carry + ex;
            else w.base[b] = carry + ex;
        }
        carry += tot;
    }
    const uint32_t nphases = carry;
    const uint32_t nbk = 3 * nphases;
    const bool lds_cnt = nbk <= kLdsBuckets;
    if (lds_cnt) {
        for (uint32_t k = tid; k < nbk; k += nt) lcnt[k] = 0;
    } else {
        for (uint32_t k = tid; k <= nbk; k += nt) w.cnt[k] = 0;
    }
    __syncthreads();

    // Pass 3: bucket of each operation (3 * phase + kind; kinds in bucket
    // order: 0 work-group byte ranges, 1 wavefront, 2 single lane) and the
    // count per bucket.
    for (uint32_t t0 = 0; t0 < n; t0 += kIndexTile) {
        const uint32_t i0 = t0 + tid * R;
        uint32_t eb[R], ef[R], key[R], unused[R];
        bool live[R];
        load_run<R>(w.eb, i0, n, kNone, eb);
        load_run<R>(w.ef, i0, n, 0, ef);
        load_run<R>(w.key, i0, n, 0, key);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            live[r] = eb[r] != kNone;
            if (live[r]) {
                const uint32_t base = eb[r] < kLdsEpochs ? lepoch[eb[r]] : w.base[eb[r]];
                key[r] = 3 * (base + ef[r]) + class_kind(key[r]);
            } else {
                key[r] = kNone;
            }
        }
        if (lds_cnt) agg_inc<R, false, true>(lcnt, key, live, unused);
        else agg_inc<R, false, false>(w.cnt, key, live, unused);
        store_run<R>(w.key, i0, n, key);
    }
    __syncthreads();

    // Pass 4: bucket offsets; the counts become scatter cursors.
    carry = 0;
    for (uint32_t k0 = 0; k0 < nbk; k0 += nt) {
        const uint32_t k = k0 + tid;
        // Counters in memory were built with atomics (performed in L2).
        const uint32_t v = k < nbk ? (lds_cnt ? lcnt[k] : ld_l2(w.cnt + k)) : 0;
        uint32_t tot = 0;
        const uint32_t ex = block_scan<kIndexWaves, uint32_t>(v, &tot);
        if (k < nbk) {
            w.off[k] = carry + ex;
            if (lds_cnt) lcnt[k] = carry + ex;
            else w.cnt[k] = carry + ex;
        }
        carry += tot;
    }
    const uint32_t nvalid = carry;
    if (tid == 0) w.off[nbk] = nvalid;
    __syncthreads();

    // Pass 5: scatter.  The order inside a bucket is free: its operations run
    // concurrently anyway.
    for (uint32_t t0 = 0; t0 < n; t0 += kIndexTile) {
        const uint32_t i0 = t0 + tid * R;
        uint32_t key[R], nch[R], pos[R];
        bool live[R];
        load_run<R>(w.key, i0, n, kNone, key);
        load_run<R>(w.nch, i0, n, 0, nch);
#pragma unroll
        for (int r = 0; r < R; ++r) live[r] = key[r] != kNone;
        if (lds_cnt) agg_inc<R, true, true>(lcnt, key, live, pos);
        else agg_inc<R, true, false>(w.cnt, key, live, pos);
        bool wg = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (live[r]) {
                w.sorted[pos[r]] = i0 + r;
                w.cs[pos[r]] = nch[r];
                wg |= nch[r] != 0;
            }
        }
        if (wg) s_wg = 1;   // every writer stores the same value
    }
    __syncthreads();

    // Pass 6: work-group task offsets over the sorted order.  Each position
    // is read and rewritten by the same thread.  Only work-group operations
    // have tasks; without any, every position's count is 0 and so is its
    // prefix: pass 5 already wrote it.
    uint64_t carry64 = 0;
    const bool any_wg = s_wg != 0;
    for (uint32_t t0 = 0; any_wg && t0 < nvalid; t0 += kIndexTile) {
        const uint32_t s0 = t0 + tid * R;
        uint64_t v[R], mine = 0;
        if (s0 + R <= nvalid) {
#pragma unroll
            for (int q = 0; q < R / 2; ++q) {
                const vshmem_detail::v4u x = *(const vshmem_detail::v4u *)(w.cs + s0 + 2 * q);
                v[2 * q] = (uint64_t)x.x | ((uint64_t)x.y << 32);
                v[2 * q + 1] = (uint64_t)x.z | ((uint64_t)x.w << 32);
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = s0 + r < nvalid ? w.cs[s0 + r] : 0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) mine += v[r];
        uint64_t tot = 0;
        uint64_t run = carry64 + block_scan<kIndexWaves, uint64_t>(mine, &tot);
        carry64 += tot;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t x = v[r];
            v[r] = run;
            run += x;
        }
        if (s0 + R <= nvalid) {
#pragma unroll
            for (int q = 0; q < R / 2; ++q)
                *(vshmem_detail::v4u *)(w.cs + s0 + 2 * q) =
                    vshmem_detail::v4u{(uint32_t)v[2 * q], (uint32_t)(v[2 * q] >> 32), (uint32_t)v[2 * q + 1],
                                       (uint32_t)(v[2 * q + 1] >> 32)};
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (s0 + r < nvalid) w.cs[s0 + r] = v[r];
        }
    }
    if (tid == 0) w.cs[nvalid] = carry64;
    __syncthreads();

    // Pass 7: tasks per phase, the executor's active work-groups and the last
    // phase with tasks.
    const uint32_t bd = a.exec_wg, waves = bd / 64;
    for (uint32_t ph = tid; ph < nphases; ph += nt) {
        const uint32_t o0 = w.off[3 * ph], o1 = w.off[3 * ph + 1], o2 = w.off[3 * ph + 2], o3 = w.off[3 * ph + 3];
        const uint64_t nt_ph = (w.cs[o1] - w.cs[o0]) + (o2 - o1 + waves - 1) / waves + (o3 - o2 + bd - 1) / bd;
        if (nt_ph) {
            atomicMax(&s_max, nt_ph < 0xFFFFFFFFull ? (uint32_t)nt_ph : 0xFFFFFFFFu);
            atomicMax(&s_last, ph + 1);
        }
    }
    __syncthreads();
    if (tid == 0) {
        w.ctl->nphases = nphases;
        w.ctl->active = s_max == 0 ? 0 : (s_max < a.exec_grid ? s_max : a.exec_grid);
        w.ctl->last = s_last;
        w.ctl->nvalid = nvalid;
        w.bar[0] = 0;
        *(uint64_t *)((uint8_t *)w.bar + VSHMEM_SYNC_GEN_OFF) = 0;
    }
}

__device__ __forceinline__ uint32_t rfl(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t rfl64(uint64_t x) { return vshmem_detail::first_lane64(x); }

// Last sorted position s in [lo, hi) with cs[s] <= target (cs strictly
// increasing over work-group operations): a 64-way search by one wavefront.
__device__ __forceinline__ uint32_t wave_search(const uint64_t *cs, uint32_t lo, uint32_t hi, uint64_t target)
{
    const uint32_t lane = __lane_id();
    while (hi - lo > 1) {
        const uint32_t span = hi - lo;
        const uint32_t p = lo + (uint32_t)(((uint64_t)span * lane) / 64);
        const bool le = cs[p] <= target;
        const uint64_t m = __ballot(le);
        const uint32_t k = 63 - (uint32_t)__builtin_clzll(m);   // lane 0 always holds
        const uint32_t nlo = lo + (uint32_t)(((uint64_t)span * k) / 64);
        const uint32_t nhi = k == 63 ? hi : lo + (uint32_t)(((uint64_t)span * (k + 1)) / 64);
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// Executor: up to exec_grid work-groups; those past ctl->active leave.
__global__ void __launch_bounds__(1024) k_batch_exec(BatchArgs a)
{
    __shared__ shmemx_tune_t tune;
    // Every phase's bounds (its bucket offsets and first work-group tasks),
    // read from the workspace once for all phases: per phase they were two
    // dependent memory round trips in every work-group.
    __shared__ uint32_t s_off[3 * kExecLdsPhases + 1];
    __shared__ uint64_t s_c0[kExecLdsPhases], s_c1[kExecLdsPhases];
    const Ws &w = a.w;
    const uint32_t active = rfl(w.ctl->active), last = rfl(w.ctl->last);
    if (blockIdx.x >= active) return;
    if (threadIdx.x == 0) tune = *a.tune;
    const bool lds = last <= kExecLdsPhases;
    if (lds) {
        for (uint32_t k = threadIdx.x; k <= 3 * last; k += blockDim.x) s_off[k] = w.off[k];
        __syncthreads();
        for (uint32_t ph = threadIdx.x; ph < last; ph += blockDim.x) {
            s_c0[ph] = w.cs[s_off[3 * ph]];
            s_c1[ph] = w.cs[s_off[3 * ph + 1]];
        }
    }
    __syncthreads();
    const uint32_t bd = blockDim.x, waves = bd / 64;
    for (uint32_t ph = 0; ph < last; ++ph) {
        const uint32_t *off = lds ? s_off : w.off;
        const uint32_t o0 = rfl(off[3 * ph]), o1 = rfl(off[3 * ph + 1]);
        const uint32_t o2 = rfl(off[3 * ph + 2]), o3 = rfl(off[3 * ph + 3]);
        const uint64_t c0 = rfl64(lds ? s_c0[ph] : w.cs[o0]);
        const uint64_t nwg = rfl64(lds ? s_c1[ph] : w.cs[o1]) - c0;
        const uint64_t nwv = (o2 - o1 + waves - 1) / waves;
        const uint64_t ntask = nwg + nwv + (o3 - o2 + bd - 1) / bd;
        if (ntask == 0) continue;
        // Tasks are dealt round robin (no shared cursor: a pop would cost
        // a returning atomic and two work-group barriers per task).  Every
        // wavefront finds a task's operation itself.
        for (uint64_t t = blockIdx.x; t < ntask; t += active) {
            if (t < nwg) {
                const uint32_t s = wave_search(w.cs, o0, o1, c0 + t);
                const shmemx_desc_t d = load_desc(a.D + rfl(w.sorted[s]));
                const int sc = resolve_scope(d, tune);
                const uint64_t ch = resolve_chunk(d, sc, tune);
                const uint64_t k = c0 + t - rfl64(w.cs[s]);
                const uint64_t lo = k * ch;
                const uint64_t hi = lo + ch < d.nbytes ? lo + ch : d.nbytes;
                exec_wg(a.c, d, lo, hi, a.results);
            } else if (t < nwg + nwv) {
                const uint64_t first = o1 + (t - nwg) * waves + threadIdx.x / 64;
                if (first < o2) exec_wave(a.c, load_desc(a.D + w.sorted[first]), a.results);
            } else {
                const uint64_t idx = o2 + (t - nwg - nwv) * bd + threadIdx.x;
                if (idx < o3) exec_thread(a.c, load_desc(a.D + w.sorted[idx]), a.results);
            }
        }
        if (ph + 1 < last) {
            vshmem_detail::wait_vm_complete();
            __syncthreads();
            if (threadIdx.x == 0) vshmem_detail::counter_barrier(a.c, w.bar, active);
            __syncthreads();
        }
    }
    vshmem_detail::release_wg_at_exit();   // quiet
}

// Per-operation form: launch i executes descriptor i of the table.
__global__ void __launch_bounds__(1024) k_batch_one(shmemx_dctx_pub_t c, const shmemx_desc_t *D, uint32_t i,
                                                    uint32_t n, const shmemx_tune_t *tune, uint64_t *results)
{
    shmemx_desc_t d = load_desc(D + i);
    uint32_t *dw = (uint32_t *)&d;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(d) / 4); ++k) dw[k] = rfl(dw[k]);
    if (d.op == SHMEMX_OP_NOP || is_sync_op(d.op)) return;   // stream order is the ordering
    if (!is_data_op(d.op) || d.issuer_pe < 0 || d.issuer_pe >= c.npes || !dev_valid(c, d, n, results)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) vshmem_detail::latch_error(c, SHMEMX_DEVERR_BAD_DESC);
        return;
    }
    const int sc = resolve_scope(d, *tune);
    if (sc == SHMEMX_SCOPE_THREAD) {
        if (blockIdx.x == 0 && threadIdx.x == 0) exec_thread(c, d, results);
    } else if (sc == SHMEMX_SCOPE_WAVE) {
        if (blockIdx.x == 0 && threadIdx.x < 64) exec_wave(c, d, results);
    } else {
        const uint64_t ch = resolve_chunk(d, sc, *tune);
        const uint64_t nch = d.nbytes ? (d.nbytes + ch - 1) / ch : 1;
        for (uint64_t k = blockIdx.x; k < nch; k += gridDim.x) {
            const uint64_t lo = k * ch;
            exec_wg(c, d, lo, lo + ch < d.nbytes ? lo + ch : d.nbytes, results);
        }
    }
    vshmem_detail::release_wg_at_exit();   // quiet
}

// ------------------------------------------------------------------ host
struct StreamWs {
    uint8_t *buf = nullptr;
    uint64_t cap = 0;
};
std::mutex g_ws_mu;
std::map<hipStream_t, StreamWs> g_ws;      // fused-form workspaces, one per stream

// Launch shape of the executor and the per-op kernel from the library's tune.
int exec_shape(uint32_t *wg, uint32_t *grid)
{
    const shmemx_tune_t &t = st().tune;
    int64_t cap = 0;
    if (int rc = coresident_capacity(k_batch_exec, t.wg_size, &cap)) return rc;
    if (cap <= 0) {
        int per_cu = 0;
        (void)blocks_per_cu(k_batch_exec, t.wg_size, &per_cu);
        if (per_cu > 0) {
            set_error_detail(SHMEMX_ERR_BUSY, "k_batch_exec: no CU is free next to the progress kernel");
            return SHMEMX_ERR_BUSY;
        }
        set_error_detail(SHMEMX_ERR_UNSUPPORTED, "k_batch_exec: no work-group of %d threads can be resident",
                         t.wg_size);
        return SHMEMX_ERR_UNSUPPORTED;
    }
    if (t.grid_wgs > 0 && t.grid_wgs < cap) cap = t.grid_wgs;
    *wg = (uint32_t)t.wg_size;
    *grid = (uint32_t)cap;
    return SHMEMX_OK;
}

int check_table(const shmemx_desc_t *d_descs, size_t n)
{
    if (int rc = check_ready()) return rc;
    if ((!d_descs && n) || n > kMaxTable) return SHMEMX_ERR_ARG;
    if (st().npes > kIndexMaxPes) {
        set_error_detail(SHMEMX_ERR_UNSUPPORTED, "device descriptor tables support up to %d PEs", kIndexMaxPes);
        return SHMEMX_ERR_UNSUPPORTED;
    }
    return SHMEMX_OK;
}

// Index + executor on `stream` over a workspace of capacity >= n.
int launch_fused(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results, const shmemx_tune_t *d_tune,
                 uint8_t *ws, uint64_t cap, hipStream_t stream)
{
    uint32_t wg = 0, grid = 0;
    if (int rc = exec_shape(&wg, &grid)) return rc;
    BatchArgs a{};
    a.c = pub();
    a.D = d_descs;
    a.n = (uint32_t)n;
    a.exec_wg = wg;
    a.exec_grid = grid;
    a.tune = d_tune ? d_tune : st().d_tune;
    a.results = d_results;
    a.w = ws_carve(ws, cap);
    const uint32_t ncls = (uint32_t)((n + kClassifyThreads - 1) / kClassifyThreads);
    hipLaunchKernelGGL(k_batch_classify, dim3(ncls), dim3(kClassifyThreads), 0, stream, a);
    hipLaunchKernelGGL(k_batch_index, dim3(1), dim3(kIndexThreads), 0, stream, a);
    hipLaunchKernelGGL(k_batch_exec, dim3(grid), dim3(wg), 0, stream, a);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int launch_ops(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results, const shmemx_tune_t *d_tune,
               hipStream_t stream)
{
    const shmemx_tune_t &t = st().tune;
    const shmemx_tune_t *tp = d_tune ? d_tune : st().d_tune;
    const unsigned grid = t.grid_wgs > 0 ? (unsigned)t.grid_wgs : (unsigned)st().num_cus;
    const shmemx_dctx_pub_t c = pub();
    for (size_t i = 0; i < n; ++i)
        hipLaunchKernelGGL(k_batch_one, dim3(grid), dim3(t.wg_size), 0, stream, c, d_descs, (uint32_t)i, (uint32_t)n,
                           tp, d_results);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

constexpr uint64_t kNoAllocBytes = 4ull << 20;
std::mutex g_noalloc_mu;
std::map<int, uint8_t *> g_noalloc_ptr;     // device ordinal -> address of its copy of `scratch`

}  // namespace

// Workspace of shmemx_launch_batch_noalloc: a fixed array in device memory
// that every call on a device shares.  Its device address comes from
// hipGetSymbolAddress once per device; in host code the name is only a
// stand-in, never an address to hand to a kernel.
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

struct shmemx_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint8_t *ws = nullptr;
};

namespace vshmem {
int batch_noalloc_setup(int device)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr.count(device)) return SHMEMX_OK;
    void *ptr = nullptr;
    VSHMEM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_noalloc_ptr[device] = (uint8_t *)ptr;
    return SHMEMX_OK;
}

void batch_release_workspaces()
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto &kv : g_ws)
        if (kv.second.buf) (void)hipFree(kv.second.buf);
    g_ws.clear();
}
}  // namespace vshmem

extern "C" {

int shmemx_launch_batch(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results, const shmemx_tune_t *d_tune,
                        void *stream)
{
    if (int rc = check_table(d_descs, n)) return rc;
    if (n == 0) return SHMEMX_OK;
    hipStream_t hs = (hipStream_t)stream;
    uint8_t *buf = nullptr;
    uint64_t cap = 0;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        StreamWs &sw = g_ws[hs];
        if (sw.cap < n) {
            // The stream's earlier launches may still read the old workspace.
            VSHMEM_HIP(hipStreamSynchronize(hs));
            if (sw.buf) (void)hipFree(sw.buf);
            sw.buf = nullptr;
            sw.cap = 0;
            const uint64_t want = std::max<uint64_t>(n, 4096);
            VSHMEM_HIP(hipMalloc((void **)&sw.buf, ws_bytes(want)));
            sw.cap = want;
        }
        buf = sw.buf;
        cap = sw.cap;
    }
    return launch_fused(d_descs, n, d_results, d_tune, buf, cap, hs);
}

int shmemx_launch_batch_noalloc(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results,
                                const shmemx_tune_t *d_tune, void *stream)
{
    if (int rc = check_table(d_descs, n)) return rc;
    static const uint64_t cap = ws_capacity(kNoAllocBytes);
    if (n > cap) {
        set_error_detail(SHMEMX_ERR_ARG, "shmemx_launch_batch_noalloc: %zu descriptors, at most %llu fit its %llu-byte "
                         "workspace", n, (unsigned long long)cap, (unsigned long long)kNoAllocBytes);
        return SHMEMX_ERR_ARG;
    }
    if (n == 0) return SHMEMX_OK;
    uint8_t *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        auto it = g_noalloc_ptr.find(st().device);
        if (it != g_noalloc_ptr.end()) ws = it->second;
    }
    if (!ws) return SHMEMX_ERR_STATE;   // set up at initialisation
    return launch_fused(d_descs, n, d_results, d_tune, ws, cap, (hipStream_t)stream);
}

uint64_t shmemx_launch_batch_noalloc_max(void) { return ws_capacity(kNoAllocBytes); }

int shmemx_launch_per_op(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results, const shmemx_tune_t *d_tune,
                         void *stream)
{
    if (int rc = check_table(d_descs, n)) return rc;
    return launch_ops(d_descs, n, d_results, d_tune, (hipStream_t)stream);
}

int shmemx_graph_build(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results, const shmemx_tune_t *d_tune,
                       int form, shmemx_graph_t **out)
{
    if (int rc = check_table(d_descs, n)) return rc;
    if (!out || (form != 0 && form != 1)) return SHMEMX_ERR_ARG;
    *out = nullptr;
    auto *g = new shmemx_graph();
    int rc = SHMEMX_OK;
    const uint64_t cap = std::max<uint64_t>(n, 1);
    if (form == 1 && VSHMEM_HIP_FAILED(hipMalloc((void **)&g->ws, ws_bytes(cap)))) rc = SHMEMX_ERR_HIP;
    hipStream_t cs = nullptr;
    if (!rc && VSHMEM_HIP_FAILED(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking))) rc = SHMEMX_ERR_HIP;
    if (!rc && VSHMEM_HIP_FAILED(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal))) rc = SHMEMX_ERR_HIP;
    if (!rc) {
        int lrc = SHMEMX_OK;
        if (n) lrc = form == 1 ? launch_fused(d_descs, n, d_results, d_tune, g->ws, cap, cs)
                               : launch_ops(d_descs, n, d_results, d_tune, cs);
        hipGraph_t graph = nullptr;
        if (VSHMEM_HIP_FAILED(hipStreamEndCapture(cs, &graph)) && !lrc) lrc = SHMEMX_ERR_HIP;
        g->graph = graph;
        rc = lrc;
        if (!rc && VSHMEM_HIP_FAILED(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0))) rc = SHMEMX_ERR_HIP;
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (rc) {
        shmemx_graph_destroy(g);
        set_last_error(rc);
        return rc;
    }
    *out = g;
    return SHMEMX_OK;
}

int shmemx_graph_launch(shmemx_graph_t *g, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!g || !g->exec) return SHMEMX_ERR_ARG;
    VSHMEM_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return SHMEMX_OK;
}

void shmemx_graph_destroy(shmemx_graph_t *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ws) (void)hipFree(g->ws);
    delete g;
}

}  // extern "C"
