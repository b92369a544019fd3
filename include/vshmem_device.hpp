/*
 * vshmem device API: device-initiated OpenSHMEM operations on virtual PEs
 * for gfx950 (MI355X).  HIP only; include from .hip sources.
 *
 * A kernel obtains the default device context (SHMEM_DEVICE_CTX_DEFAULT of
 * the paper's Section 6.2: created on the host at initialisation, published
 * GPU-visible, used by kernels, destroyed at finalisation) as a kernel
 * argument and binds it to the virtual PE the calling work-group acts for:
 *
 *     shmem_dctx_t ctx = shmemx_dctx_bind(published, blockIdx.x / wgs_per_pe);
 *
 * All pointer arguments are canonical symmetric addresses (PE 0's copy, as
 * returned by shmem_malloc); the library translates them with
 * addr(pe) = sym + pe * stride, without classifying pointers (Section 6.3).
 *
 * Scopes (Section 4.1, Section 6.3): a plain name is issued by one thread;
 * _wave by all 64 lanes of a wavefront; _wg by every thread of the
 * work-group; _grid by every work-group acting for the PE.  Every
 * participant passes identical arguments.
 *
 * Completion and ordering (Section 6.3, Section 6.4): a blocking put/get
 * returns at local completion (the source may be reused); remote
 * visibility needs shmem_quiet or a barrier.  shmem_fence orders the
 * caller's later operations after its earlier ones; shmem_quiet completes
 * the caller's operations device-wide (agent scope), which on this part
 * writes back dirty L2 lines so other XCDs observe them.  Atomics are
 * relaxed at agent scope: atomicity does not imply ordering.
 */
#ifndef VSHMEM_DEVICE_HPP
#define VSHMEM_DEVICE_HPP

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "vshmem.h"

/* ------------------------------------------------------------- contexts */
/* The published device context (one per library instance). */
struct shmemx_dctx_pub_t {
    uint8_t *base;               /* canonical base: PE 0's slice */
    uint64_t stride;             /* bytes between PE slices */
    uint64_t user_bytes;         /* allocatable bytes per PE */
    uint64_t scratch_off;        /* offset of the library scratch in a slice */
    uint32_t *err;               /* device error word */
    uint64_t wait_timeout_ticks; /* spin limit in wall-clock ticks */
    int32_t npes;
    int32_t debug;
};

/* A context bound to the virtual PE a caller acts for.  PE arguments of
 * the operations are numbered in the context's team: argument p names
 * world PE tstart + p * tstride.  The default context's team is the world
 * (identity numbering); an explicit context's team is the team it was
 * created from. */
struct shmem_dctx_t {
    shmemx_dctx_pub_t c;
    int32_t me;      /* world PE the caller acts for */
    int32_t idx;     /* its number in the context's team: shmem_my_pe */
    int32_t tstart;
    int32_t tstride;
    int32_t tsize;   /* shmem_n_pes */
    int32_t tslot;   /* the team's barrier words */
    int64_t options; /* SHMEM_CTX_* bits it was created with */
};

/* Device teams are shmemx_dteam_t of vshmem.h. */

/* An explicit device context as shmemx_device_ctx_create publishes it in
 * device memory (the explicit contexts of Section 6.2: created on the host,
 * passed to kernels as device-visible handles).  Read-only for kernels. */
struct shmemx_dctx_rec_t {
    shmemx_dctx_pub_t pub;
    shmemx_dteam_t team;
    int64_t options;
};

#define VSHMEM_SCRATCH_BYTES (64u << 10)
#define VSHMEM_SYNC_SLOT_BYTES 128u
#define VSHMEM_MAX_TEAMS 256
/* A barrier's arrival count is at scratch + slot * VSHMEM_SYNC_SLOT_BYTES and
 * its generation word VSHMEM_SYNC_GEN_OFF bytes further, in a second array
 * of slots: waiters poll the generation while arrivals add to the count, and
 * on one cache line the polls queue with the atomics. */
#define VSHMEM_SYNC_GEN_OFF (32u << 10)
static_assert(VSHMEM_MAX_TEAMS * VSHMEM_SYNC_SLOT_BYTES <= VSHMEM_SYNC_GEN_OFF &&
                  VSHMEM_SYNC_GEN_OFF + VSHMEM_MAX_TEAMS * VSHMEM_SYNC_SLOT_BYTES <= VSHMEM_SCRATCH_BYTES,
              "barrier counts and generations fit the scratch tail");

/* The default context (SHMEM_DEVICE_CTX_DEFAULT) for world PE `me`. */
__device__ __forceinline__ shmem_dctx_t shmemx_dctx_bind(const shmemx_dctx_pub_t &pub, int me)
{
    shmem_dctx_t c;
    c.c = pub;
    c.me = me;
    c.idx = me;
    c.tstart = 0;
    c.tstride = 1;
    c.tsize = pub.npes;
    c.tslot = 0;
    c.options = 0;
    return c;
}

/* An explicit context for its team's member `idx` (0 <= idx < team size). */
__device__ __forceinline__ shmem_dctx_t shmemx_dctx_bind_explicit(const shmemx_dctx_rec_t &rec, int idx)
{
    shmem_dctx_t c;
    c.c = rec.pub;
    c.me = rec.team.start + idx * rec.team.stride;
    c.idx = idx;
    c.tstart = rec.team.start;
    c.tstride = rec.team.stride;
    c.tsize = rec.team.size;
    c.tslot = rec.team.slot;
    c.options = rec.options;
    return c;
}

__device__ __forceinline__ int shmem_my_pe(const shmem_dctx_t &ctx) { return ctx.idx; }
__device__ __forceinline__ int shmem_n_pes(const shmem_dctx_t &ctx) { return ctx.tsize; }

/* The context's team as a device team descriptor. */
__device__ __forceinline__ shmemx_dteam_t shmemx_ctx_team(const shmem_dctx_t &ctx)
{
    return shmemx_dteam_t{ctx.tstart, ctx.tstride, ctx.tsize, ctx.tslot};
}

/* PE `pe`'s copy of a symmetric object, pe numbered in the context's team:
 * the device-domain shmem_ptr. */
template <typename T>
__device__ __forceinline__ T *shmem_ptr(const shmem_dctx_t &ctx, const T *sym, int pe)
{
    return (T *)((uint8_t *)sym + (uint64_t)(ctx.tstart + pe * ctx.tstride) * ctx.c.stride);
}

/* The caller's own copy of a symmetric object. */
template <typename T>
__device__ __forceinline__ T *shmemx_local_ptr(const shmem_dctx_t &ctx, const T *sym)
{
    return (T *)((uint8_t *)sym + (uint64_t)ctx.me * ctx.c.stride);
}

__device__ __forceinline__ int shmemx_team_pe(const shmemx_dteam_t &t, int k) { return t.start + k * t.stride; }

/* --------------------------------------------------------------- details */
namespace vshmem_detail {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t now() { return wall_clock64(); }

__device__ __forceinline__ void latch_error(const shmemx_dctx_pub_t &c, uint32_t bits)
{
    __hip_atomic_fetch_or(c.err, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
/* Wait until this thread's earlier vector memory operations have completed
 * (stores acknowledged by L2): vmcnt(0), with the export and LDS counters
 * left alone.  Followed by a work-group barrier and one agent-scope release
 * by a single thread, it gives the whole work-group's stores agent-scope
 * visibility with one L2 write-back instead of one per wavefront. */
__device__ __forceinline__ void wait_vm_complete()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

/* Agent-scope release of everything the work-group stored, with one L2
 * write-back: every thread waits for its own operations, the work-group
 * synchronises, thread 0 releases.  Every thread of the work-group must
 * call it.  An agent release per wavefront costs one write-back each, and
 * those serialise in the L2s (thousands of wavefronts: hundreds of us). */
__device__ __forceinline__ void release_wg_at_exit()
{
    wait_vm_complete();
    __syncthreads();
    if (threadIdx.x == 0) release_agent();
}
/* As above, and no thread returns before the release is done. */
__device__ __forceinline__ void release_wg()
{
    release_wg_at_exit();
    __syncthreads();
}
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

template <bool NT, typename T>
__device__ __forceinline__ T ld(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st(T *p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

/* Vector body: lane handles elements lane, lane+nl, ...; U loads are issued
 * before their stores so each lane keeps U*sizeof(V) bytes in flight. */
template <typename V, int U, bool NT>
__device__ __forceinline__ void copy_body(V *__restrict__ d, const V *__restrict__ s, uint64_t nv,
                                          uint64_t lane, uint64_t nl)
{
    uint64_t i = lane;
    if constexpr (U > 1) {
        for (; i + (uint64_t)(U - 1) * nl < nv; i += (uint64_t)U * nl) {
            V r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) r[u] = ld<NT>(s + i + (uint64_t)u * nl);
#pragma unroll
            for (int u = 0; u < U; ++u) st<NT>(d + i + (uint64_t)u * nl, r[u]);
        }
    }
    for (; i < nv; i += nl) st<NT>(d + i, ld<NT>(s + i));
}

/* The n < A bytes before or after the vector body of a copy by one lane
 * whose source and destination agree modulo A, in the widest naturally
 * aligned pieces: an 8-byte message is one 8-byte move, not eight. */
template <uint64_t A>
__device__ __forceinline__ void copy_edge_lone(uint8_t *d, const uint8_t *s, uint64_t n)
{
    for (uint64_t o = 0; o < n;) {
        const uint64_t a = (uintptr_t)(d + o), r = n - o;
        if (A > 8 && (a & 7) == 0 && r >= 8) {
            *(uint64_t *)(d + o) = *(const uint64_t *)(s + o);
            o += 8;
        } else if (A > 4 && (a & 3) == 0 && r >= 4) {
            *(uint32_t *)(d + o) = *(const uint32_t *)(s + o);
            o += 4;
        } else if (A > 2 && (a & 1) == 0 && r >= 2) {
            *(uint16_t *)(d + o) = *(const uint16_t *)(s + o);
            o += 2;
        } else {
            d[o] = s[o];
            o += 1;
        }
    }
}

/* Copy n bytes whose source and destination agree modulo sizeof(V): byte
 * edges, then the vector body.  Cooperating lanes take one edge byte each
 * (one instruction); a lone lane (LONE: the caller passes lane 0 of 1)
 * takes wide pieces.  LONE is a template parameter rather than a test of
 * nl so that the cooperative copies compile exactly as without it. */
template <typename V, int U, bool NT, bool LONE = false>
__device__ __forceinline__ void copy_aligned(uint8_t *__restrict__ d, const uint8_t *__restrict__ s,
                                             uint64_t n, uint64_t lane, uint64_t nl)
{
    constexpr uint64_t A = sizeof(V);
    uint64_t head = (A - ((uintptr_t)d & (A - 1))) & (A - 1);
    if (head > n) head = n;
    if constexpr (LONE) copy_edge_lone<A>(d, s, head);
    else
        for (uint64_t i = lane; i < head; i += nl) d[i] = s[i];
    uint64_t nv = (n - head) / A;
    copy_body<V, U, NT>((V *)(d + head), (const V *)(s + head), nv, lane, nl);
    if constexpr (LONE) {
        const uint64_t t = head + nv * A;
        copy_edge_lone<A>(d + t, s + t, n - t);
    } else {
        for (uint64_t i = head + nv * A + lane; i < n; i += nl) d[i] = s[i];
    }
}

/* Body of a copy whose source is `sh` = 4*Q + r bytes (1 <= sh <= 15) past
 * a 16-byte boundary while the destination is 16-byte aligned: destination
 * vector i is bytes [16i + sh, 16i + sh + 16) of the aligned source stream
 * s_al, taken from the two aligned vectors that hold them with byte funnel
 * shifts (v_alignbyte_b32).  Both loaded vectors hold bytes of the source
 * range, so no load touches a page the range does not touch.  Neighbouring
 * lanes load each other's vectors, which the caches absorb: HBM still
 * reads each source byte once. */
template <int Q, int U, bool NT>
__device__ __forceinline__ void copy_shifted_body(v4u *__restrict__ d, const v4u *__restrict__ s_al, uint32_t r,
                                                  uint64_t nv, uint64_t lane, uint64_t nl)
{
    auto join = [r](const v4u &a, const v4u &b) {
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        v4u o;
        o.x = __builtin_amdgcn_alignbyte(w[Q + 1], w[Q + 0], r);
        o.y = __builtin_amdgcn_alignbyte(w[Q + 2], w[Q + 1], r);
        o.z = __builtin_amdgcn_alignbyte(w[Q + 3], w[Q + 2], r);
        o.w = __builtin_amdgcn_alignbyte(w[Q + 4], w[Q + 3], r);
        return o;
    };
    uint64_t i = lane;
    for (; i + (uint64_t)(U - 1) * nl < nv; i += (uint64_t)U * nl) {
        v4u a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = ld<NT>(s_al + i + (uint64_t)u * nl);
            b[u] = ld<NT>(s_al + i + (uint64_t)u * nl + 1);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) st<NT>(d + i + (uint64_t)u * nl, join(a[u], b[u]));
    }
    for (; i < nv; i += nl) st<NT>(d + i, join(ld<NT>(s_al + i), ld<NT>(s_al + i + 1)));
}

template <int U, bool NT>
__device__ __forceinline__ void copy_shifted(uint8_t *__restrict__ d, const uint8_t *__restrict__ s, uint64_t n,
                                             uint64_t lane, uint64_t nl)
{
    uint64_t head = (16 - ((uintptr_t)d & 15)) & 15;
    if (head > n) head = n;
    for (uint64_t i = lane; i < head; i += nl) d[i] = s[i];
    const uint8_t *sb = s + head;
    const uint64_t nv = (n - head) / 16;
    const uint32_t sh = (uint32_t)((uintptr_t)sb & 15);   // not 0: source and destination disagree mod 16
    const v4u *s_al = (const v4u *)(sb - sh);
    v4u *db = (v4u *)(d + head);
    // Two loads per stored vector: half the unroll keeps the same bytes in
    // flight without raising register pressure in the aligned path's kernels.
    constexpr int US = U > 2 ? U / 2 : 1;
    switch (sh >> 2) {
    case 0: copy_shifted_body<0, US, NT>(db, s_al, sh & 3, nv, lane, nl); break;
    case 1: copy_shifted_body<1, US, NT>(db, s_al, sh & 3, nv, lane, nl); break;
    case 2: copy_shifted_body<2, US, NT>(db, s_al, sh & 3, nv, lane, nl); break;
    default: copy_shifted_body<3, US, NT>(db, s_al, sh & 3, nv, lane, nl); break;
    }
    for (uint64_t i = head + nv * 16 + lane; i < n; i += nl) d[i] = s[i];
}

/* Copies shorter than this take the narrower vector paths below when source
 * and destination disagree modulo 16. */
constexpr uint64_t kShiftedMin = 256;

/* Copy n bytes with nl cooperating lanes (this one is `lane`): 16-byte
 * vectors when source and destination agree modulo 16; otherwise, with
 * SHIFT, 16-byte destination vectors assembled from the source by funnel
 * shifts (copies of kShiftedMin bytes or more), else 8-, 4- or 1-byte
 * elements.  SHIFT is for callers that see arbitrary offsets (the device
 * API, serving, plans, host-issued moves); the put/get pattern kernels keep
 * it off so that their aligned path's registers stay as they were (the
 * grid-scope kernel is already at the 128-register limit of its launch).
 * LONE marks a copy by one lane (lane 0 of 1), whose unaligned edges move
 * in wide pieces. */
template <int U, bool NT, bool SHIFT = false, bool LONE = false>
__device__ __forceinline__ void copy_bytes(uint8_t *d, const uint8_t *s, uint64_t n, uint64_t lane, uint64_t nl)
{
    uint64_t x = (uintptr_t)d ^ (uintptr_t)s;
    if ((x & 15) == 0) copy_aligned<v4u, U, NT, LONE>(d, s, n, lane, nl);
    else if (SHIFT && n >= kShiftedMin) copy_shifted<U, NT>(d, s, n, lane, nl);
    else if ((x & 7) == 0) copy_aligned<uint64_t, U, NT, LONE>(d, s, n, lane, nl);
    else if ((x & 3) == 0) copy_aligned<uint32_t, U, NT, LONE>(d, s, n, lane, nl);
    else
        for (uint64_t i = lane; i < n; i += nl) d[i] = s[i];
}

__device__ __forceinline__ bool cmp_holds_u(uint64_t x, int cmp, uint64_t v)
{
    switch (cmp) {
    case 0: return x == v;
    case 1: return x != v;
    case 2: return x > v;
    case 3: return x >= v;
    case 4: return x < v;
    default: return x <= v;
    }
}

__device__ __forceinline__ bool cmp_holds_s(int64_t x, int cmp, int64_t v)
{
    switch (cmp) {
    case 0: return x == v;
    case 1: return x != v;
    case 2: return x > v;
    case 3: return x >= v;
    case 4: return x < v;
    default: return x <= v;
    }
}

/* Spin until the 64-bit word satisfies cmp, with backoff and a spin limit;
 * returns the last value read.  Latches a device error on timeout. */
template <bool SIGNED>
__device__ __forceinline__ uint64_t spin_until(const shmemx_dctx_pub_t &c, uint64_t *w, int cmp, uint64_t v)
{
    uint64_t x = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool ok = SIGNED ? cmp_holds_s((int64_t)x, cmp, (int64_t)v) : cmp_holds_u(x, cmp, v);
    if (!ok) {
        uint64_t t0 = now();
        for (;;) {
            __builtin_amdgcn_s_sleep(1);
            x = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = SIGNED ? cmp_holds_s((int64_t)x, cmp, (int64_t)v) : cmp_holds_u(x, cmp, v);
            if (ok) break;
            if (now() - t0 > c.wait_timeout_ticks) {
                latch_error(c, 0x1u);
                break;
            }
        }
    }
    acquire_agent();
    return x;
}

__device__ __forceinline__ uint64_t *sync_slot(const shmemx_dctx_pub_t &c, int pe, int slot)
{
    return (uint64_t *)(c.base + (uint64_t)pe * c.stride + c.scratch_off + (uint64_t)slot * VSHMEM_SYNC_SLOT_BYTES);
}

/* Counter barrier among `units` arriving work-groups; one thread per
 * work-group calls it.  The arrival word holds the phase number (high 32
 * bits) and the arrivals of the phase so far (low 32 bits); the generation
 * word, VSHMEM_SYNC_GEN_OFF further on a line of its own, holds the number
 * of completed phases.  An arrival learns its phase from its own fetch_add
 * and waits until the generation reaches phase + 1; the last arrival
 * resets the count with the next phase number and then releases the
 * generation.  No separate read of the generation precedes the arrival: on
 * a line of its own such a read can complete after the arrival, see the
 * next generation, and wait for a phase that needs its own arrival.
 * Release before arriving, acquire after leaving (in both the last arrival
 * and the waiters), so it also completes (quiets) the arrivals' stores.
 * Called after the work-group's threads waited for their own operations
 * and synchronised, the release and acquire of this one thread cover the
 * whole work-group: they write back and invalidate the caches the
 * work-group's wavefronts share.  With the generation word on a line of
 * its own a 64-PE barrier took 3.2 us instead of 5.9, a 256-PE one 9.5
 * instead of 21.5 (waiters' polls no longer queue with the arrivals'
 * atomics). */
__device__ __forceinline__ void counter_barrier(const shmemx_dctx_pub_t &c, uint64_t *slot, uint64_t units)
{
    uint64_t *cnt = slot;
    uint64_t *gen = (uint64_t *)((uint8_t *)slot + VSHMEM_SYNC_GEN_OFF);
    release_agent();
    const uint64_t old = __hip_atomic_fetch_add(cnt, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t next = (uint64_t)((uint32_t)(old >> 32) + 1u);
    if ((old & 0xffffffffull) == units - 1) {
        acquire_agent();   // the other arrivals' releases
        __hip_atomic_store(cnt, next << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(gen, next, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        spin_until<false>(c, gen, 0 /*EQ*/, next);
    }
    acquire_agent();
}

} // namespace vshmem_detail

/* ---------------------------------------------------------- debug checks */
/* Contexts published with debug set (VSHMEM_DEBUG at init) check every
 * operation's arguments: operands inside PE 0's user heap (canonical
 * symmetric addresses), 8-byte words aligned, PE numbers inside the
 * context's team, and for _wave/_wg/_grid calls one argument set across the
 * participants.  A failed check latches SHMEMX_DEVERR_BAD_ADDRESS or
 * SHMEMX_DEVERR_NONUNIFORM and the operation does nothing (every
 * participant of a scoped call takes the same decision).  Without debug the
 * checks reduce to one uniform branch. */
namespace vshmem_detail {

__device__ __forceinline__ uint64_t first_lane64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ bool in_user_heap(const shmem_dctx_t &ctx, const void *p, uint64_t n)
{
    const uint8_t *q = (const uint8_t *)p;
    if (q < ctx.c.base) return false;
    const uint64_t off = (uint64_t)(q - ctx.c.base);
    return off <= ctx.c.user_bytes && n <= ctx.c.user_bytes - off;
}

__device__ __forceinline__ bool pe_in_team(const shmem_dctx_t &ctx, int pe) { return pe >= 0 && pe < ctx.tsize; }

__device__ __forceinline__ bool checked(const shmem_dctx_t &ctx, bool ok)
{
    if (!ok) latch_error(ctx.c, SHMEMX_DEVERR_BAD_ADDRESS);
    return ok;
}

/* A put or get of n bytes with PE pe (both operands symmetric). */
__device__ __forceinline__ bool rma_ok(const shmem_dctx_t &ctx, const void *dest, const void *src, uint64_t n, int pe)
{
    return !ctx.c.debug || checked(ctx, in_user_heap(ctx, dest, n) && in_user_heap(ctx, src, n) && pe_in_team(ctx, pe));
}

/* A naturally aligned symmetric 8-byte word on PE pe. */
__device__ __forceinline__ bool word_ok(const shmem_dctx_t &ctx, const void *w, int pe)
{
    return !ctx.c.debug || checked(ctx, ((uintptr_t)w & 7) == 0 && in_user_heap(ctx, w, 8) && pe_in_team(ctx, pe));
}

/* Wavefront scope: every lane passed lane 0's arguments and found them
 * valid.  All lanes return the same answer. */
__device__ __forceinline__ bool wave_agree(const shmem_dctx_t &ctx, bool ok, uint64_t a, uint64_t b, uint64_t c,
                                           uint64_t d)
{
    if (!ctx.c.debug) return true;
    const bool same = a == first_lane64(a) && b == first_lane64(b) && c == first_lane64(c) && d == first_lane64(d);
    if (__ballot(!same) != 0 && __lane_id() == 0) latch_error(ctx.c, SHMEMX_DEVERR_NONUNIFORM);
    return __ballot(!(ok && same)) == 0;
}

/* Work-group scope: the same through LDS.  Every thread must call it. */
__device__ __forceinline__ bool wg_agree(const shmem_dctx_t &ctx, bool ok, uint64_t a, uint64_t b, uint64_t c,
                                         uint64_t d)
{
    if (!ctx.c.debug) return true;
    __shared__ uint64_t ref[4];
    __shared__ uint32_t verdict;   // bit 0: a thread found its arguments invalid; bit 1: arguments differ
    if (threadIdx.x == 0) {
        ref[0] = a;
        ref[1] = b;
        ref[2] = c;
        ref[3] = d;
        verdict = 0;
    }
    __syncthreads();
    const bool same = a == ref[0] && b == ref[1] && c == ref[2] && d == ref[3];
    if (!ok || !same) atomicOr(&verdict, (ok ? 0u : 1u) | (same ? 0u : 2u));
    __syncthreads();
    const uint32_t v = __builtin_amdgcn_readfirstlane(verdict);
    __syncthreads();   // ref and verdict are free for the next call
    if ((v & 2u) && threadIdx.x == 0) latch_error(ctx.c, SHMEMX_DEVERR_NONUNIFORM);
    return v == 0;
}

} // namespace vshmem_detail

#define VSHMEM_U64(x) ((uint64_t)(uintptr_t)(x))

/* ------------------------------------------------------------ put / get */
#define VSHMEM_COPY_UNROLL 4

/* put: PE `pe`'s dest[0, n) <- my src[0, n) */
__device__ __forceinline__ void shmem_putmem(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    if (!vshmem_detail::rma_ok(ctx, dest, src, n, pe)) return;
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false, true, true>(shmem_ptr(ctx, (uint8_t *)dest, pe),
                                                               shmemx_local_ptr(ctx, (const uint8_t *)src), n, 0, 1);
}
__device__ __forceinline__ void shmem_putmem_nbi(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmem_putmem_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    if (!vshmem_detail::wave_agree(ctx, vshmem_detail::rma_ok(ctx, dest, src, n, pe), VSHMEM_U64(dest),
                                   VSHMEM_U64(src), n, (uint64_t)pe))
        return;
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false, true>(shmem_ptr(ctx, (uint8_t *)dest, pe),
                                                         shmemx_local_ptr(ctx, (const uint8_t *)src), n,
                                                         __lane_id(), 64);
}
__device__ __forceinline__ void shmem_putmem_nbi_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem_wave(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmem_putmem_nbi_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    if (!vshmem_detail::wg_agree(ctx, vshmem_detail::rma_ok(ctx, dest, src, n, pe), VSHMEM_U64(dest), VSHMEM_U64(src),
                                 n, (uint64_t)pe))
        return;
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false, true>(shmem_ptr(ctx, (uint8_t *)dest, pe),
                                                         shmemx_local_ptr(ctx, (const uint8_t *)src), n,
                                                         threadIdx.x, blockDim.x);
}
__device__ __forceinline__ void shmem_putmem_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem_nbi_wg(ctx, dest, src, n, pe);
    __syncthreads();
}
/* Grid scope: the nwgs work-groups acting for the PE (this one is `rank`)
 * share the message; each returns when its own share is locally complete.
 * Debug checks compare arguments within each work-group. */
__device__ __forceinline__ void shmemx_putmem_grid(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n,
                                                   int pe, int rank, int nwgs)
{
    if (!vshmem_detail::wg_agree(ctx, vshmem_detail::rma_ok(ctx, dest, src, n, pe), VSHMEM_U64(dest), VSHMEM_U64(src),
                                 n, ((uint64_t)(uint32_t)nwgs << 32) | (uint32_t)pe))
        return;
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false, true>(shmem_ptr(ctx, (uint8_t *)dest, pe),
                                                         shmemx_local_ptr(ctx, (const uint8_t *)src), n,
                                                         (uint64_t)rank * blockDim.x + threadIdx.x,
                                                         (uint64_t)nwgs * blockDim.x);
}

/* get: my dest[0, n) <- PE `pe`'s src[0, n) */
__device__ __forceinline__ void shmem_getmem(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    if (!vshmem_detail::rma_ok(ctx, dest, src, n, pe)) return;
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false, true, true>(shmemx_local_ptr(ctx, (uint8_t *)dest),
                                                               shmem_ptr(ctx, (const uint8_t *)src, pe), n, 0, 1);
}
__device__ __forceinline__ void shmem_getmem_nbi(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_getmem(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmem_getmem_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    if (!vshmem_detail::wave_agree(ctx, vshmem_detail::rma_ok(ctx, dest, src, n, pe), VSHMEM_U64(dest),
                                   VSHMEM_U64(src), n, (uint64_t)pe))
        return;
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false, true>(shmemx_local_ptr(ctx, (uint8_t *)dest),
                                                         shmem_ptr(ctx, (const uint8_t *)src, pe), n,
                                                         __lane_id(), 64);
}
__device__ __forceinline__ void shmem_getmem_nbi_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_getmem_wave(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmem_getmem_nbi_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    if (!vshmem_detail::wg_agree(ctx, vshmem_detail::rma_ok(ctx, dest, src, n, pe), VSHMEM_U64(dest), VSHMEM_U64(src),
                                 n, (uint64_t)pe))
        return;
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false, true>(shmemx_local_ptr(ctx, (uint8_t *)dest),
                                                         shmem_ptr(ctx, (const uint8_t *)src, pe), n,
                                                         threadIdx.x, blockDim.x);
}
__device__ __forceinline__ void shmem_getmem_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_getmem_nbi_wg(ctx, dest, src, n, pe);
    __syncthreads();
}
__device__ __forceinline__ void shmemx_getmem_grid(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n,
                                                   int pe, int rank, int nwgs)
{
    if (!vshmem_detail::wg_agree(ctx, vshmem_detail::rma_ok(ctx, dest, src, n, pe), VSHMEM_U64(dest), VSHMEM_U64(src),
                                 n, ((uint64_t)(uint32_t)nwgs << 32) | (uint32_t)pe))
        return;
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false, true>(shmemx_local_ptr(ctx, (uint8_t *)dest),
                                                         shmem_ptr(ctx, (const uint8_t *)src, pe), n,
                                                         (uint64_t)rank * blockDim.x + threadIdx.x,
                                                         (uint64_t)nwgs * blockDim.x);
}

/* GPU-space names.  The paper's GPU-space usage example (Section 6.1) writes
 * a device-initiated put to an object from shmemg_malloc as shmemg_put and
 * marks its names as illustrative.  Here the GPU space is the default heap,
 * so these are the put and get above under that prefix. */
__device__ __forceinline__ void shmemg_putmem(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmemg_putmem_nbi(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem_nbi(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmemg_putmem_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem_wave(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmemg_putmem_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem_wg(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmemg_getmem(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_getmem(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmemg_getmem_nbi(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_getmem_nbi(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmemg_getmem_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_getmem_wave(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmemg_getmem_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_getmem_wg(ctx, dest, src, n, pe);
}

/* -------------------------------------------------------- fence / quiet */
__device__ __forceinline__ void shmem_fence(const shmem_dctx_t &) { vshmem_detail::release_agent(); }
__device__ __forceinline__ void shmem_quiet(const shmem_dctx_t &) { vshmem_detail::release_agent(); }
__device__ __forceinline__ void shmem_quiet_wave(const shmem_dctx_t &) { vshmem_detail::release_agent(); }
__device__ __forceinline__ void shmem_fence_wave(const shmem_dctx_t &) { vshmem_detail::release_agent(); }
/* Every lane completes its own stores, then the work-group synchronises:
 * all of the work-group's earlier operations are complete on return. */
__device__ __forceinline__ void shmem_quiet_wg(const shmem_dctx_t &) { vshmem_detail::release_wg(); }
__device__ __forceinline__ void shmem_fence_wg(const shmem_dctx_t &ctx) { shmem_quiet_wg(ctx); }

/* --------------------------------------------------------------- atomics */
#define VSHMEM_AMO_PTR(T) ((T *)shmem_ptr(ctx, (uint8_t *)dest, pe))

__device__ __forceinline__ int64_t shmem_int64_atomic_fetch_add(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return 0;
    return (int64_t)__hip_atomic_fetch_add(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void shmem_int64_atomic_add(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return;
    __hip_atomic_fetch_add(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t shmem_uint64_atomic_fetch_xor(const shmem_dctx_t &ctx, uint64_t *dest, uint64_t v, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return 0;
    return __hip_atomic_fetch_xor(VSHMEM_AMO_PTR(uint64_t), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t shmem_int64_atomic_fetch_xor(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return 0;
    return (int64_t)__hip_atomic_fetch_xor(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void shmem_uint64_atomic_xor(const shmem_dctx_t &ctx, uint64_t *dest, uint64_t v, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return;
    __hip_atomic_fetch_xor(VSHMEM_AMO_PTR(uint64_t), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void shmem_int64_atomic_xor(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return;
    __hip_atomic_fetch_xor(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t shmem_int64_atomic_compare_swap(const shmem_dctx_t &ctx, int64_t *dest, int64_t cond,
                                                                   int64_t v, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return 0;
    uint64_t expected = (uint64_t)cond;
    __hip_atomic_compare_exchange_strong(VSHMEM_AMO_PTR(uint64_t), &expected, (uint64_t)v, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (int64_t)expected;
}
__device__ __forceinline__ int64_t shmem_int64_atomic_fetch(const shmem_dctx_t &ctx, const int64_t *dest, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return 0;
    return (int64_t)__hip_atomic_load((uint64_t *)shmem_ptr(ctx, (const uint8_t *)dest, pe), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void shmem_int64_atomic_set(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return;
    __hip_atomic_store(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t shmem_int64_atomic_swap(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    if (!vshmem_detail::word_ok(ctx, dest, pe)) return 0;
    return (int64_t)__hip_atomic_exchange(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
}

/* ------------------------------------------------- signals and waiting */
__device__ __forceinline__ void vshmemx_signal_update(const shmem_dctx_t &ctx, uint64_t *sig, uint64_t v, int sig_op, int pe)
{
    if (!vshmem_detail::word_ok(ctx, sig, pe)) return;
    uint64_t *s = shmem_ptr(ctx, sig, pe);
    if (sig_op == 1)
        __hip_atomic_fetch_add(s, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_store(s, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

/* put with signal: the data, a release, then the signal; the signal is
 * never observable before the data. */
__device__ __forceinline__ void shmem_putmem_signal(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n,
                                                    uint64_t *sig, uint64_t sigval, int sig_op, int pe)
{
    if (!vshmem_detail::word_ok(ctx, sig, pe) || !vshmem_detail::rma_ok(ctx, dest, src, n, pe)) return;
    shmem_putmem(ctx, dest, src, n, pe);
    vshmem_detail::release_agent();
    vshmemx_signal_update(ctx, sig, sigval, sig_op, pe);
}
__device__ __forceinline__ void shmem_putmem_signal_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n,
                                                         uint64_t *sig, uint64_t sigval, int sig_op, int pe)
{
    const bool data_ok = vshmem_detail::wave_agree(ctx, vshmem_detail::rma_ok(ctx, dest, src, n, pe), VSHMEM_U64(dest),
                                                   VSHMEM_U64(src), n, (uint64_t)pe);
    const bool sig_ok = vshmem_detail::wave_agree(ctx, vshmem_detail::word_ok(ctx, sig, pe), VSHMEM_U64(sig), sigval,
                                                  (uint64_t)sig_op, (uint64_t)pe);
    if (!data_ok || !sig_ok) return;
    shmem_putmem_wave(ctx, dest, src, n, pe);
    vshmem_detail::release_agent();
    if (__lane_id() == 0) vshmemx_signal_update(ctx, sig, sigval, sig_op, pe);
}
__device__ __forceinline__ void shmem_putmem_signal_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n,
                                                       uint64_t *sig, uint64_t sigval, int sig_op, int pe)
{
    const bool data_ok = vshmem_detail::wg_agree(ctx, vshmem_detail::rma_ok(ctx, dest, src, n, pe), VSHMEM_U64(dest),
                                                 VSHMEM_U64(src), n, (uint64_t)pe);
    const bool sig_ok = vshmem_detail::wg_agree(ctx, vshmem_detail::word_ok(ctx, sig, pe), VSHMEM_U64(sig), sigval,
                                                (uint64_t)sig_op, (uint64_t)pe);
    if (!data_ok || !sig_ok) return;
    shmem_putmem_nbi_wg(ctx, dest, src, n, pe);
    vshmem_detail::release_wg_at_exit();
    if (threadIdx.x == 0) vshmemx_signal_update(ctx, sig, sigval, sig_op, pe);
    __syncthreads();
}

/* Wait on my own copy of a symmetric uint64 signal. */
__device__ __forceinline__ uint64_t shmem_signal_wait_until(const shmem_dctx_t &ctx, uint64_t *sig, int cmp, uint64_t v)
{
    if (!vshmem_detail::word_ok(ctx, sig, ctx.idx)) return 0;
    return vshmem_detail::spin_until<false>(ctx.c, shmemx_local_ptr(ctx, sig), cmp, v);
}
__device__ __forceinline__ void shmem_int64_wait_until(const shmem_dctx_t &ctx, int64_t *ivar, int cmp, int64_t v)
{
    if (!vshmem_detail::word_ok(ctx, ivar, ctx.idx)) return;
    vshmem_detail::spin_until<true>(ctx.c, (uint64_t *)shmemx_local_ptr(ctx, ivar), cmp, (uint64_t)v);
}
__device__ __forceinline__ int shmem_int64_test(const shmem_dctx_t &ctx, int64_t *ivar, int cmp, int64_t v)
{
    if (!vshmem_detail::word_ok(ctx, ivar, ctx.idx)) return 0;
    int64_t x = (int64_t)__hip_atomic_load((uint64_t *)shmemx_local_ptr(ctx, ivar), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    bool ok = vshmem_detail::cmp_holds_s(x, cmp, v);
    if (ok) vshmem_detail::acquire_agent();
    return ok ? 1 : 0;
}
/* Work-group scope wait: thread 0 spins, everyone acquires. */
__device__ __forceinline__ uint64_t shmem_signal_wait_until_wg(const shmem_dctx_t &ctx, uint64_t *sig, int cmp, uint64_t v)
{
    __shared__ uint64_t seen;
    if (threadIdx.x == 0) seen = shmem_signal_wait_until(ctx, sig, cmp, v);
    __syncthreads();
    vshmem_detail::acquire_agent();
    return seen;
}

/* ------------------------------------------------------------- barriers */
/* Team barriers (Section 6.3: barriers among the device-initiated
 * collectives; the scope suffix names who calls, as in the _wave example
 * of Section 8).  No member leaves before every member arrived, and each
 * caller's earlier operations are complete and visible device-wide on
 * return (the barrier implies quiet).  The counter lives in the scratch
 * tail of the team's first member, at the team's slot.
 *
 *   plain  one thread acts for its PE (exactly one per member calls);
 *   _wave  all 64 lanes of one wavefront act for the PE;
 *   _wg    every thread of one work-group acts for the PE;
 *   units  every thread of `units_per_pe` work-groups per PE.
 *
 * All callers of one barrier must be resident together: a caller that is
 * waiting for a work-group slot never arrives. */
__device__ __forceinline__ void shmemx_team_sync_units(const shmem_dctx_t &ctx, const shmemx_dteam_t &team,
                                                       uint64_t units_per_pe)
{
    // Every thread's operations complete before the work-group arrives;
    // thread 0's release and acquire inside the barrier then cover them all.
    vshmem_detail::wait_vm_complete();
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t *slot = vshmem_detail::sync_slot(ctx.c, team.start, team.slot);
        vshmem_detail::counter_barrier(ctx.c, slot, (uint64_t)team.size * units_per_pe);
    }
    __syncthreads();
}

__device__ __forceinline__ int shmem_team_sync(const shmem_dctx_t &ctx, const shmemx_dteam_t &team)
{
    vshmem_detail::counter_barrier(ctx.c, vshmem_detail::sync_slot(ctx.c, team.start, team.slot),
                                   (uint64_t)team.size);
    return 0;
}
__device__ __forceinline__ int shmem_team_sync_wave(const shmem_dctx_t &ctx, const shmemx_dteam_t &team)
{
    // One wavefront: its memory counter covers all 64 lanes, so lane 0's
    // release after the wait covers the wave's stores; the acquire runs
    // with every lane active once lane 0 is back.
    vshmem_detail::wait_vm_complete();
    if (__lane_id() == 0)
        vshmem_detail::counter_barrier(ctx.c, vshmem_detail::sync_slot(ctx.c, team.start, team.slot),
                                       (uint64_t)team.size);
    vshmem_detail::acquire_agent();
    return 0;
}
__device__ __forceinline__ int shmem_team_sync_wg(const shmem_dctx_t &ctx, const shmemx_dteam_t &team)
{
    shmemx_team_sync_units(ctx, team, 1);
    return 0;
}

__device__ __forceinline__ shmemx_dteam_t shmemx_team_world(const shmem_dctx_t &ctx)
{
    return shmemx_dteam_t{0, 1, ctx.c.npes, 0};
}
__device__ __forceinline__ void shmem_barrier_all(const shmem_dctx_t &ctx) { shmem_team_sync(ctx, shmemx_team_world(ctx)); }
__device__ __forceinline__ void shmem_barrier_all_wave(const shmem_dctx_t &ctx)
{
    shmem_team_sync_wave(ctx, shmemx_team_world(ctx));
}
__device__ __forceinline__ void shmem_barrier_all_wg(const shmem_dctx_t &ctx)
{
    shmemx_team_sync_units(ctx, shmemx_team_world(ctx), 1);
}

/* ---------------------------------------------------------- collectives */
namespace vshmem_detail {

constexpr uint64_t kCollChunk = 256ull << 10;   // bytes per task: broadcast, fcollect, alltoall
constexpr uint64_t kRedChunk = 16ull << 10;     // bytes per task: reductions
constexpr int kMcastTile = 16;                  // 16-byte vectors per lane in a multicast tile
constexpr int kRedBatch = 8;                    // member loads in flight per lane before combining

// The work-groups of a collective, numbered across the team: member k's
// work-group `rank` (of nwgs) is worker k * nwgs + rank of size * nwgs.
// (32-bit: a grid has fewer than 2^32 work-groups, and 64-bit division and
// remainder would expand to long vector sequences.)
struct Workers {
    uint32_t w, n;
};
__device__ __forceinline__ Workers team_workers(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, int rank,
                                                int nwgs)
{
    const uint32_t k = (uint32_t)((ctx.me - team.start) / team.stride);
    return Workers{k * (uint32_t)nwgs + (uint32_t)rank, (uint32_t)team.size * (uint32_t)nwgs};
}

// Member 0's copy of a symmetric object, and the distance between members.
__device__ __forceinline__ uint8_t *member0(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, const void *sym)
{
    return (uint8_t *)sym + (uint64_t)team.start * ctx.c.stride;
}
__device__ __forceinline__ uint64_t member_stride(const shmem_dctx_t &ctx, const shmemx_dteam_t &team)
{
    return (uint64_t)team.stride * ctx.c.stride;
}

// Copy one source range to the same place on every team member (d0 is
// member 0's copy, members pstride apart).  Aligned ranges go through a
// register tile: each lane loads kMcastTile 16-byte vectors once, then the
// whole tile is written to one member after another, starting at a member
// that depends on the worker so that concurrent work-groups spread over
// the members.  Long contiguous writes per member page measured about 10%
// faster on MI355X than writing every vector to all members in turn.
template <bool NT>
__device__ __forceinline__ void multicast(uint8_t *d0, uint64_t pstride, int P, const uint8_t *src, uint64_t len,
                                          uint32_t worker)
{
    if ((((uintptr_t)src | (uintptr_t)d0 | len) & 15) == 0) {
        const v4u *s = (const v4u *)src;
        const uint64_t nv = len / 16, bd = blockDim.x;
        for (uint64_t i0 = threadIdx.x; i0 < nv; i0 += kMcastTile * bd) {
            v4u r[kMcastTile];
#pragma unroll
            for (int u = 0; u < kMcastTile; ++u)
                if (i0 + u * bd < nv) r[u] = ld<true>(s + i0 + u * bd);
            int p = (int)(worker % (uint32_t)P);
            for (int k = 0; k < P; ++k) {
                v4u *d = (v4u *)(d0 + (uint64_t)p * pstride);
#pragma unroll
                for (int u = 0; u < kMcastTile; ++u)
                    if (i0 + u * bd < nv) st<NT>(d + i0 + u * bd, r[u]);
                if (++p == P) p = 0;
            }
        }
    } else {
        for (int p = 0; p < P; ++p)
            copy_bytes<VSHMEM_COPY_UNROLL, NT>(d0 + p * pstride, src, len, threadIdx.x, blockDim.x);
    }
}

// Every member's dest[0, n) <- member root's src[0, n), root included.
template <bool NT>
__device__ __forceinline__ void broadcast(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, void *dest,
                                          const void *src, uint64_t n, int root, int rank, int nwgs, uint64_t chunk)
{
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
    const Workers W = team_workers(ctx, team, rank, nwgs);
    const uint8_t *S = (const uint8_t *)src + (uint64_t)shmemx_team_pe(team, root) * ctx.c.stride;
    uint8_t *D = member0(ctx, team, dest);
    const uint64_t ps = member_stride(ctx, team);
    const uint64_t ntask = (n + chunk - 1) / chunk;
    for (uint64_t t = W.w; t < ntask; t += W.n) {
        const uint64_t off = t * chunk;
        multicast<NT>(D + off, ps, team.size, S + off, min(chunk, n - off), W.w);
    }
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
}

// Every member's dest[q*n, (q+1)*n) <- member q's src[0, n).
template <bool NT>
__device__ __forceinline__ void fcollect(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, void *dest,
                                         const void *src, uint64_t n, int rank, int nwgs, uint64_t chunk)
{
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
    const Workers W = team_workers(ctx, team, rank, nwgs);
    const uint8_t *S0 = member0(ctx, team, src);
    uint8_t *D = member0(ctx, team, dest);
    const uint64_t ps = member_stride(ctx, team);
    const uint64_t nch = (n + chunk - 1) / chunk;
    const uint64_t ntask = nch * (uint64_t)team.size;
    for (uint64_t t = W.w; t < ntask; t += W.n) {
        const uint64_t q = t / nch;
        const uint64_t off = (t - q * nch) * chunk;
        multicast<NT>(D + q * n + off, ps, team.size, S0 + q * ps + off, min(chunk, n - off), W.w);
    }
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
}

// Member p's dest[q*n, (q+1)*n) <- member q's src[p*n, (p+1)*n).  A task is
// one chunk of one block.  A task shorter than half of one pass of the
// work-group (U 16-byte vectors per lane) goes to a group of g lanes: the
// smallest power of two, at most a wavefront, that covers it in one pass.
// A work-group then copies blockDim/g small blocks at once; one task per
// work-group would leave most lanes idle and pay a memory round trip per
// block.  Consecutive tasks go to different work-groups first, so a few
// tiny blocks per member still spread over every work-group.
template <bool NT, int U>
__device__ __forceinline__ void alltoall(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, void *dest,
                                         const void *src, uint64_t n, int rank, int nwgs, uint64_t chunk)
{
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
    const Workers W = team_workers(ctx, team, rank, nwgs);
    const uint8_t *S0 = member0(ctx, team, src);
    uint8_t *D0 = member0(ctx, team, dest);
    const uint64_t ps = member_stride(ctx, team);
    const uint64_t P = (uint64_t)team.size;
    const uint64_t nch = (n + chunk - 1) / chunk;
    const uint64_t ntask = nch * P * P;
    constexpr uint64_t kPass = 16ull * U;   // bytes per lane per pass
    const uint64_t task = min(chunk, n);
    uint32_t g = blockDim.x;
    if (task * 2 < kPass * blockDim.x) {
        const uint64_t need = (task + kPass - 1) / kPass;
        g = 1;
        while (g < 64 && g < need) g <<= 1;
    }
    const uint32_t groups = blockDim.x / g;   // threads past groups * g stay idle
    if (threadIdx.x < groups * g) {
        const uint64_t lane = threadIdx.x % g;
        for (uint64_t t = (uint64_t)(threadIdx.x / g) * W.n + W.w; t < ntask; t += (uint64_t)W.n * groups) {
            const uint64_t blk = t / nch;
            const uint64_t p = blk / P;   // destination member
            const uint64_t q = blk % P;   // source member
            const uint64_t off = (t - blk * nch) * chunk;
            copy_bytes<U, NT>(D0 + p * ps + q * n + off, S0 + q * ps + p * n + off, min(chunk, n - off), lane, g);
        }
    }
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
}

// TREE in streaming form.  Pushing x_0, x_1, ... keeps, for every set bit j
// of the count, the reduction of an aligned block of 2^j consecutive inputs
// (slot j).  Pushing merges equal-sized blocks left to right, which is
// exactly the pairing of one TREE level.  At the end the blocks, largest
// (leftmost) first, are combined right-nested: op(B_a, op(B_b, ... B_z)),
// which is how TREE's carried odd elements meet the full subtrees.
struct OpSum {
    template <typename T> __device__ __forceinline__ static T f(T a, T b) { return a + b; }
};
struct OpMax {
    template <typename T> __device__ __forceinline__ static T f(T a, T b) { return (b > a) ? b : a; }
};

constexpr int kTreeLevels = 9;   // teams of up to 2^9 - 1 members

template <typename A, int E, class OP, int LEVELS = kTreeLevels>
struct TreeAcc {
    A s[LEVELS][E];
    __device__ __forceinline__ void push(uint32_t count, const A (&x)[E])
    {
        // The new input merges with the tz occupied slots below the first
        // free one (tz = trailing ones of count) and lands in slot tz.
        const uint32_t tz = (uint32_t)__builtin_ctz(~count);
        A c[E];
#pragma unroll
        for (int e = 0; e < E; ++e) c[e] = x[e];
#pragma unroll
        for (int j = 0; j < LEVELS; ++j) {
            if ((uint32_t)j < tz) {
#pragma unroll
                for (int e = 0; e < E; ++e) c[e] = OP::f(s[j][e], c[e]);
            } else if ((uint32_t)j == tz) {
#pragma unroll
                for (int e = 0; e < E; ++e) s[j][e] = c[e];
            }
        }
    }
    // count >= 1 inputs pushed.
    __device__ __forceinline__ void result(uint32_t count, A (&r)[E]) const
    {
        bool have = false;
#pragma unroll
        for (int j = 0; j < LEVELS; ++j) {
            if ((count >> j) & 1u) {
                if (!have) {
#pragma unroll
                    for (int e = 0; e < E; ++e) r[e] = s[j][e];
                    have = true;
                } else {
#pragma unroll
                    for (int e = 0; e < E; ++e) r[e] = OP::f(s[j][e], r[e]);
                }
            }
        }
    }
};

// Element codecs: a 16-byte vector of the storage type <-> E accumulators.
struct CodecI64 {
    using A = int64_t;
    static constexpr int E = 2;
    static constexpr int ES = 8;
    __device__ __forceinline__ static void unpack(const v4u &v, A (&x)[E])
    {
        x[0] = (int64_t)(((uint64_t)v.y << 32) | v.x);
        x[1] = (int64_t)(((uint64_t)v.w << 32) | v.z);
    }
    __device__ __forceinline__ static v4u pack(const A (&x)[E])
    {
        v4u v;
        v.x = (uint32_t)x[0];
        v.y = (uint32_t)((uint64_t)x[0] >> 32);
        v.z = (uint32_t)x[1];
        v.w = (uint32_t)((uint64_t)x[1] >> 32);
        return v;
    }
    __device__ __forceinline__ static A load1(const uint8_t *p) { return *(const int64_t *)p; }
    __device__ __forceinline__ static void store1(uint8_t *p, A v) { *(int64_t *)p = v; }
};

struct CodecF32 {
    using A = float;
    static constexpr int E = 4;
    static constexpr int ES = 4;
    __device__ __forceinline__ static void unpack(const v4u &v, A (&x)[E])
    {
        x[0] = __uint_as_float(v.x);
        x[1] = __uint_as_float(v.y);
        x[2] = __uint_as_float(v.z);
        x[3] = __uint_as_float(v.w);
    }
    __device__ __forceinline__ static v4u pack(const A (&x)[E])
    {
        v4u v;
        v.x = __float_as_uint(x[0]);
        v.y = __float_as_uint(x[1]);
        v.z = __float_as_uint(x[2]);
        v.w = __float_as_uint(x[3]);
        return v;
    }
    __device__ __forceinline__ static A load1(const uint8_t *p) { return *(const float *)p; }
    __device__ __forceinline__ static void store1(uint8_t *p, A v) { *(float *)p = v; }
};

// bf16 -> fp32 is exact (the bf16 bits are the high half of the fp32).
// fp32 -> bf16 rounds to nearest, ties to even; NaN stays a quiet NaN.
__device__ __forceinline__ float bf16_up(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t bf16_down(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (u >> 16) | 0x40u;
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

struct CodecBF16 {
    using A = float;
    static constexpr int E = 8;
    static constexpr int ES = 2;
    __device__ __forceinline__ static void unpack(const v4u &v, A (&x)[E])
    {
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            x[2 * i] = bf16_up(w[i] & 0xFFFFu);
            x[2 * i + 1] = bf16_up(w[i] >> 16);
        }
    }
    __device__ __forceinline__ static v4u pack(const A (&x)[E])
    {
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = bf16_down(x[2 * i]) | (bf16_down(x[2 * i + 1]) << 16);
        v4u v;
        v.x = w[0];
        v.y = w[1];
        v.z = w[2];
        v.w = w[3];
        return v;
    }
    __device__ __forceinline__ static A load1(const uint8_t *p) { return bf16_up(*(const uint16_t *)p); }
    __device__ __forceinline__ static void store1(uint8_t *p, A v) { *(uint16_t *)p = (uint16_t)bf16_down(v); }
};

// Elements before the first 16-byte boundary of the source when source and
// destination lie at the same offset from a boundary (every member's copy
// does, the member stride being a multiple of 16) and that offset is a
// whole number of elements; ~0 when the vector path does not apply.
template <int ES>
__device__ __forceinline__ uint64_t vec_head(const uint8_t *s0, const uint8_t *d0, uint64_t pstride, uint64_t nelem)
{
    const uint64_t sm = (uintptr_t)s0 & 15, dm = (uintptr_t)d0 & 15;
    if (sm != dm || (pstride & 15) || (sm % ES)) return ~0ull;
    const uint64_t head = ((16 - sm) & 15) / ES;
    return head < nelem ? head : nelem;
}

// Single-element reduce-to-all of elements [0, lo) and [hi, nelem): one lane
// per element over every worker of the collective.
template <class CODEC, class OP>
__device__ __forceinline__ void reduce_singles(int P, uint64_t pstride, const uint8_t *s0, uint8_t *d0, uint64_t nelem,
                                               uint64_t lo, uint64_t hi, const Workers &W)
{
    using A = typename CODEC::A;
    const uint64_t nsingle = lo + (nelem - hi);
    for (uint64_t q = (uint64_t)W.w * blockDim.x + threadIdx.x; q < nsingle; q += (uint64_t)W.n * blockDim.x) {
        const uint64_t k = q < lo ? q : hi + (q - lo);
        TreeAcc<A, 1, OP> acc;
        for (int p = 0; p < P; ++p) {
            A x[1] = {CODEC::load1(s0 + (uint64_t)p * pstride + k * CODEC::ES)};
            acc.push((uint32_t)p, x);
        }
        A r[1];
        acc.result((uint32_t)P, r);
        for (int p = 0; p < P; ++p) CODEC::store1(d0 + (uint64_t)p * pstride + k * CODEC::ES, r[0]);
    }
}

// Every member's dest[k] <- TREE over members of src[k], for k < nelem.
// Each lane owns K 16-byte vectors of the range, blockDim.x vectors apart:
// it loads them from every member (kRedBatch loads in flight), folds each
// in member order and writes the results to every member.  With K > 1 a
// wavefront's consecutive loads and stores fall K times in a row into one
// member's page, so each address translation serves K KiB instead of 1
// KiB: the member walk visits 2P pages per vector, more than a CU's
// first-level translation cache holds.  LEVELS bounds the team size
// (2^LEVELS - 1 members).  Returns SHMEMX_ERR_UNSUPPORTED, without
// synchronising, for teams larger than that.
template <class CODEC, class OP, bool NT, int K = 1, int LEVELS = kTreeLevels>
__device__ __forceinline__ int reduce(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, void *dest,
                                      const void *src, uint64_t nelem, int rank, int nwgs, uint64_t chunk)
{
    using A = typename CODEC::A;
    constexpr int E = CODEC::E;
    constexpr int B = kRedBatch / K > 0 ? kRedBatch / K : 1;   // members per load batch
    if (team.size >= (1 << LEVELS)) return SHMEMX_ERR_UNSUPPORTED;
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
    const Workers W = team_workers(ctx, team, rank, nwgs);
    const int P = team.size;
    const uint64_t pstride = member_stride(ctx, team);
    const uint8_t *s0 = member0(ctx, team, src);
    uint8_t *d0 = member0(ctx, team, dest);
    // Vector part: from the first 16-byte boundary of the source when source
    // and destination share their offset from it (a head of single
    // elements before); otherwise everything is single elements.
    const uint64_t head = vec_head<CODEC::ES>(s0, d0, pstride, nelem);
    const bool vec = head != ~0ull;
    const uint64_t h = vec ? head : 0;
    const uint64_t nvec = vec ? (nelem - h) * CODEC::ES / 16 : 0;
    const uint8_t *sv = s0 + h * CODEC::ES;
    uint8_t *dv = d0 + h * CODEC::ES;
    // Vectors per task: the chunk, or an even share per worker when that is
    // smaller, so a small reduction still spreads over every work-group
    // (each element's order over the members does not depend on who runs it).
    const uint64_t share = (nvec + W.n - 1) / W.n;
    const uint64_t vpt = max<uint64_t>(1, min<uint64_t>(chunk / 16, share));
    const uint64_t ntask = (nvec + vpt - 1) / vpt;
    const uint64_t bd = blockDim.x;
    for (uint64_t t = W.w; t < ntask; t += W.n) {
        const uint64_t v1 = min(nvec, (t + 1) * vpt);
        for (uint64_t i = t * vpt + threadIdx.x; i < v1; i += K * bd) {
            TreeAcc<A, E, OP, LEVELS> acc[K];
            const uint8_t *sp = sv + i * 16;
            for (int p0 = 0; p0 < P; p0 += B) {
                v4u raw[B][K];
#pragma unroll
                for (int u = 0; u < B; ++u)
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (p0 + u < P && i + k * bd < v1)
                            raw[u][k] = ld<NT>((const v4u *)(sp + k * bd * 16 + (uint64_t)(p0 + u) * pstride));
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    if (p0 + u < P) {
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            A x[E];
                            CODEC::unpack(raw[u][k], x);
                            acc[k].push((uint32_t)(p0 + u), x);
                        }
                    }
                }
            }
            v4u out[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                A r[E];
                acc[k].result((uint32_t)P, r);
                out[k] = CODEC::pack(r);
            }
            uint8_t *dp = dv + i * 16;
            for (int p = 0; p < P; ++p, dp += pstride)
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (i + k * bd < v1) st<NT>((v4u *)(dp + k * bd * 16), out[k]);
        }
    }
    reduce_singles<CODEC, OP>(P, pstride, s0, d0, nelem, h, h + nvec * 16 / CODEC::ES, W);
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
    return 0;
}

// Reduce-to-all with the team's members split over the work-group's
// wavefronts.  Member block b is members [8b, 8b + 8) (the last may be
// shorter).  TREE over all members equals TREE over the blocks' TREE
// results: TREE's first three levels pair elements only inside aligned
// blocks of eight, and a block's last element is carried exactly when it
// is the list's last.  Per step, wavefront w folds block b of one tile of
// 64 vectors (one vector per lane, the block's up to 8 loads in flight),
// leaves the block result in LDS, and after one work-group barrier every
// wavefront of the tile folds the tile's block results in block order and
// stores the packed result to its own block's members.  A work-group of
// `waves` wavefronts serves teams of up to 8 * waves members and works on
// waves / m tiles per step (m = number of blocks); its tasks are `chunk`
// bytes of every member, walked tile by tile.  The LDS block results
// are double-buffered, so one barrier per step suffices.  Every thread of
// the work-group calls it; blockDim.x is a multiple of 64, at most
// 64 * kRedWaveMax.
constexpr int kRedWaveMax = 8;

template <class CODEC, class OP, bool NT>
__device__ __forceinline__ void reduce_waves(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, void *dest,
                                             const void *src, uint64_t nelem, int rank, int nwgs, uint64_t chunk)
{
    using A = typename CODEC::A;
    constexpr int E = CODEC::E;
    __shared__ A part[2][kRedWaveMax][E][64];
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
    const Workers W = team_workers(ctx, team, rank, nwgs);
    const int P = team.size;
    const uint32_t waves = blockDim.x / 64, w = threadIdx.x / 64, lane = __lane_id();
    const uint32_t m = (uint32_t)(P + 7) / 8;          // member blocks
    const uint32_t G = waves / m;                      // tiles per step
    const uint32_t j = w / m, b = w - j * m;           // this wavefront's tile slot and block
    const int p0 = 8 * (int)b, p1 = min(p0 + 8, P);
    const uint64_t pstride = member_stride(ctx, team);
    const uint8_t *s0 = member0(ctx, team, src);
    uint8_t *d0 = member0(ctx, team, dest);
    const uint64_t head = vec_head<CODEC::ES>(s0, d0, pstride, nelem);
    const bool vec = head != ~0ull;
    const uint64_t h = vec ? head : 0;
    const uint64_t nvec = vec ? (nelem - h) * CODEC::ES / 16 : 0;
    const uint8_t *sv = s0 + h * CODEC::ES;
    uint8_t *dv = d0 + h * CODEC::ES;
    // Tasks of `chunk` bytes per member (whole tiles of 64 vectors), dealt to
    // the workers round robin; a worker walks its task's tiles in order.
    const uint64_t ntile = (nvec + 63) / 64;
    const uint64_t tpt = chunk >= 1024 ? chunk / 1024 : 1;
    const uint64_t ntask = (ntile + tpt - 1) / tpt;
    int buf = 0;
    for (uint64_t task = W.w; task < ntask; task += W.n)
    for (uint64_t t0 = task * tpt; t0 < (task + 1) * tpt && t0 < ntile; t0 += G) {
        const uint64_t i = (t0 + j) * 64 + lane;
        const bool mine = j < G && t0 + j < (task + 1) * tpt && i < nvec;
        if (mine) {
            const uint8_t *sp = sv + i * 16 + (uint64_t)p0 * pstride;
            v4u raw[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (p0 + u < p1) raw[u] = ld<NT>((const v4u *)(sp + (uint64_t)u * pstride));
            TreeAcc<A, E, OP, 4> acc;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (p0 + u < p1) {
                    A x[E];
                    CODEC::unpack(raw[u], x);
                    acc.push((uint32_t)u, x);
                }
            }
            A r[E];
            acc.result((uint32_t)(p1 - p0), r);
#pragma unroll
            for (int e = 0; e < E; ++e) part[buf][w][e][lane] = r[e];
        }
        __syncthreads();
        if (mine) {
            TreeAcc<A, E, OP, 4> acc;
            for (uint32_t bb = 0; bb < m; ++bb) {
                A x[E];
#pragma unroll
                for (int e = 0; e < E; ++e) x[e] = part[buf][j * m + bb][e][lane];
                acc.push(bb, x);
            }
            A r[E];
            acc.result(m, r);
            const v4u out = CODEC::pack(r);
            uint8_t *dp = dv + i * 16 + (uint64_t)p0 * pstride;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (p0 + u < p1) st<NT>((v4u *)(dp + (uint64_t)u * pstride), out);
        }
        buf ^= 1;
    }
    reduce_singles<CODEC, OP>(P, pstride, s0, d0, nelem, h, h + nvec * 16 / CODEC::ES, W);
    shmemx_team_sync_units(ctx, team, (uint64_t)nwgs);
}

} // namespace vshmem_detail

namespace vshmem_detail {
/* Debug check of a collective call: the team lies inside the world and has
 * the caller as a member, both ranges are inside PE 0's user heap, `extra`
 * holds, and the work-group's threads agree on (dest, src, n, tag). */
__device__ __forceinline__ bool coll_ok(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, const void *dest,
                                        uint64_t dbytes, const void *src, uint64_t sbytes, bool extra, uint64_t n,
                                        uint64_t tag)
{
    if (!ctx.c.debug) return true;
    const bool team_ok = team.size >= 1 && team.stride >= 1 && team.start >= 0 &&
                         (int64_t)team.start + (int64_t)(team.size - 1) * team.stride < ctx.c.npes &&
                         ctx.me >= team.start && (ctx.me - team.start) % team.stride == 0 &&
                         (ctx.me - team.start) / team.stride < team.size;
    const bool ok = checked(ctx, team_ok && extra && in_user_heap(ctx, dest, dbytes) && in_user_heap(ctx, src, sbytes));
    return wg_agree(ctx, ok, VSHMEM_U64(dest), VSHMEM_U64(src), n, tag);
}
} // namespace vshmem_detail

/* Team collectives (Section 6.3 names broadcast and reductions among the
 * device-initiated operations; fcollect and alltoall follow OpenSHMEM).
 * Pointers are canonical symmetric addresses; n counts bytes for the
 * data-movement routines and elements for the reductions.
 *
 *   _wg    one work-group per member calls it;
 *   _grid  nwgs work-groups per member call it, this one being `rank`
 *          (0 <= rank < nwgs) among those acting for its PE; the work is
 *          spread over all team.size * nwgs of them.
 *
 * Every participant passes identical arguments (rank aside) and all of them
 * must be resident together.  Each routine starts and ends with a barrier
 * of the team (at its slot), so sources may be rewritten and destinations
 * read, on any member, as soon as it returns.  Destination and source must
 * not overlap (a reduction may run in place).  Reductions fold members in
 * the fixed TREE order (pairs of neighbours, level by level), so results
 * are reproducible bit for bit; bf16 accumulates in fp32 and rounds once to
 * nearest-even; teams of 512 or more members get SHMEMX_ERR_UNSUPPORTED
 * from the reductions, which then do nothing.  With debug checks on, a call
 * whose arguments fail them returns SHMEMX_ERR_ARG before any barrier.
 * Return 0 otherwise. */
__device__ __forceinline__ int shmemx_broadcastmem_grid(const shmem_dctx_t &ctx, const shmemx_dteam_t &team,
                                                        void *dest, const void *src, size_t n, int root, int rank,
                                                        int nwgs)
{
    if (!vshmem_detail::coll_ok(ctx, team, dest, n, src, n, root >= 0 && root < team.size && rank >= 0 && rank < nwgs,
                                n, ((uint64_t)(uint32_t)nwgs << 32) | (uint32_t)root))
        return SHMEMX_ERR_ARG;
    vshmem_detail::broadcast<false>(ctx, team, dest, src, n, root, rank, nwgs, vshmem_detail::kCollChunk);
    return 0;
}
__device__ __forceinline__ int shmem_broadcastmem_wg(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, void *dest,
                                                     const void *src, size_t n, int root)
{
    return shmemx_broadcastmem_grid(ctx, team, dest, src, n, root, 0, 1);
}
__device__ __forceinline__ int shmemx_fcollectmem_grid(const shmem_dctx_t &ctx, const shmemx_dteam_t &team,
                                                       void *dest, const void *src, size_t n, int rank, int nwgs)
{
    if (!vshmem_detail::coll_ok(ctx, team, dest, (uint64_t)n * team.size, src, n, rank >= 0 && rank < nwgs, n,
                                (uint64_t)nwgs))
        return SHMEMX_ERR_ARG;
    vshmem_detail::fcollect<false>(ctx, team, dest, src, n, rank, nwgs, vshmem_detail::kCollChunk);
    return 0;
}
__device__ __forceinline__ int shmem_fcollectmem_wg(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, void *dest,
                                                    const void *src, size_t n)
{
    return shmemx_fcollectmem_grid(ctx, team, dest, src, n, 0, 1);
}
__device__ __forceinline__ int shmemx_alltoallmem_grid(const shmem_dctx_t &ctx, const shmemx_dteam_t &team,
                                                       void *dest, const void *src, size_t n, int rank, int nwgs)
{
    if (!vshmem_detail::coll_ok(ctx, team, dest, (uint64_t)n * team.size, src, (uint64_t)n * team.size,
                                rank >= 0 && rank < nwgs, n, (uint64_t)nwgs))
        return SHMEMX_ERR_ARG;
    vshmem_detail::alltoall<true, 8>(ctx, team, dest, src, n, rank, nwgs, vshmem_detail::kCollChunk);
    return 0;
}
__device__ __forceinline__ int shmem_alltoallmem_wg(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, void *dest,
                                                    const void *src, size_t n)
{
    return shmemx_alltoallmem_grid(ctx, team, dest, src, n, 0, 1);
}

#define VSHMEM_DEVICE_REDUCE(PREFIX, NAME, T, CODEC, OP)                                                             \
    __device__ __forceinline__ int PREFIX##NAME##_reduce_grid(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, \
                                                              T *dest, const T *src, size_t nreduce, int rank,     \
                                                              int nwgs)                                            \
    {                                                                                                              \
        if (!vshmem_detail::coll_ok(ctx, team, dest, nreduce * sizeof(T), src, nreduce * sizeof(T),               \
                                    rank >= 0 && rank < nwgs, nreduce, (uint64_t)nwgs))                            \
            return SHMEMX_ERR_ARG;                                                                                 \
        return vshmem_detail::reduce<vshmem_detail::CODEC, vshmem_detail::OP, true>(                               \
            ctx, team, dest, src, nreduce, rank, nwgs, vshmem_detail::kRedChunk);                                  \
    }
/* The grid forms carry the shmemx_ prefix; the _wg forms are OpenSHMEM names. */
#define VSHMEM_DEVICE_REDUCE_WG(NAME, GRIDNAME, T)                                                                   \
    __device__ __forceinline__ int NAME##_reduce_wg(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, T *dest,  \
                                                    const T *src, size_t nreduce)                                  \
    {                                                                                                              \
        return GRIDNAME##_reduce_grid(ctx, team, dest, src, nreduce, 0, 1);                                        \
    }
VSHMEM_DEVICE_REDUCE(shmemx_, int64_sum, int64_t, CodecI64, OpSum)
VSHMEM_DEVICE_REDUCE(shmemx_, int64_max, int64_t, CodecI64, OpMax)
VSHMEM_DEVICE_REDUCE(shmemx_, float_sum, float, CodecF32, OpSum)
VSHMEM_DEVICE_REDUCE(shmemx_, float_max, float, CodecF32, OpMax)
VSHMEM_DEVICE_REDUCE(shmemx_, bfloat16_sum, uint16_t, CodecBF16, OpSum)   /* bf16 as its bits */
VSHMEM_DEVICE_REDUCE(shmemx_, bfloat16_max, uint16_t, CodecBF16, OpMax)
VSHMEM_DEVICE_REDUCE_WG(shmem_int64_sum, shmemx_int64_sum, int64_t)
VSHMEM_DEVICE_REDUCE_WG(shmem_int64_max, shmemx_int64_max, int64_t)
VSHMEM_DEVICE_REDUCE_WG(shmem_float_sum, shmemx_float_sum, float)
VSHMEM_DEVICE_REDUCE_WG(shmem_float_max, shmemx_float_max, float)
VSHMEM_DEVICE_REDUCE_WG(shmemx_bfloat16_sum, shmemx_bfloat16_sum, uint16_t)
VSHMEM_DEVICE_REDUCE_WG(shmemx_bfloat16_max, shmemx_bfloat16_max, uint16_t)
#undef VSHMEM_DEVICE_REDUCE
#undef VSHMEM_DEVICE_REDUCE_WG

#endif /* VSHMEM_DEVICE_HPP */
