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

/* The default context bound to one virtual PE. */
struct shmem_dctx_t {
    shmemx_dctx_pub_t c;
    int32_t me;
};

/* Device team: members start + k*stride, k < size; slot selects its
 * barrier words in the first member's scratch. */
struct shmemx_dteam_t {
    int32_t start;
    int32_t stride;
    int32_t size;
    int32_t slot;
};

#define VSHMEM_SCRATCH_BYTES (64u << 10)
#define VSHMEM_SYNC_SLOT_BYTES 128u
#define VSHMEM_MAX_TEAMS 256

__device__ __forceinline__ shmem_dctx_t shmemx_dctx_bind(const shmemx_dctx_pub_t &pub, int me)
{
    shmem_dctx_t c;
    c.c = pub;
    c.me = me;
    return c;
}

__device__ __forceinline__ int shmem_my_pe(const shmem_dctx_t &ctx) { return ctx.me; }
__device__ __forceinline__ int shmem_n_pes(const shmem_dctx_t &ctx) { return ctx.c.npes; }

/* PE `pe`'s copy of a symmetric object: the device-domain shmem_ptr. */
template <typename T>
__device__ __forceinline__ T *shmem_ptr(const shmem_dctx_t &ctx, const T *sym, int pe)
{
    return (T *)((uint8_t *)sym + (uint64_t)pe * ctx.c.stride);
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

template <typename V, int U, bool NT>
__device__ __forceinline__ void copy_aligned(uint8_t *__restrict__ d, const uint8_t *__restrict__ s,
                                             uint64_t n, uint64_t lane, uint64_t nl)
{
    constexpr uint64_t A = sizeof(V);
    uint64_t head = (A - ((uintptr_t)d & (A - 1))) & (A - 1);
    if (head > n) head = n;
    for (uint64_t i = lane; i < head; i += nl) d[i] = s[i];
    uint64_t nv = (n - head) / A;
    copy_body<V, U, NT>((V *)(d + head), (const V *)(s + head), nv, lane, nl);
    for (uint64_t i = head + nv * A + lane; i < n; i += nl) d[i] = s[i];
}

/* Copy n bytes with nl cooperating lanes (this one is `lane`): 16-byte
 * vectors when source and destination agree modulo 16, else 8, 4 or 1. */
template <int U, bool NT>
__device__ __forceinline__ void copy_bytes(uint8_t *d, const uint8_t *s, uint64_t n, uint64_t lane, uint64_t nl)
{
    uint64_t x = (uintptr_t)d ^ (uintptr_t)s;
    if ((x & 15) == 0) copy_aligned<v4u, U, NT>(d, s, n, lane, nl);
    else if ((x & 7) == 0) copy_aligned<uint64_t, U, NT>(d, s, n, lane, nl);
    else if ((x & 3) == 0) copy_aligned<uint32_t, U, NT>(d, s, n, lane, nl);
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

/* Sense-reversing counter barrier among `units` arriving work-groups; one
 * thread per work-group calls it.  Release before arriving, acquire after
 * leaving (in both the last arrival and the waiters), so it also completes
 * (quiets) the arrivals' stores.  Called after the work-group's threads
 * waited for their own operations and synchronised, the release and
 * acquire of this one thread cover the whole work-group: they write back
 * and invalidate the caches the work-group's wavefronts share. */
__device__ __forceinline__ void counter_barrier(const shmemx_dctx_pub_t &c, uint64_t *slot, uint64_t units)
{
    uint64_t *cnt = slot;
    uint64_t *gen = slot + 1;
    release_agent();
    uint64_t g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t old = __hip_atomic_fetch_add(cnt, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == units - 1) {
        acquire_agent();   // the other arrivals' releases
        __hip_atomic_store(cnt, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        spin_until<false>(c, gen, 1 /*NE*/, g);
    }
    acquire_agent();
}

} // namespace vshmem_detail

/* ------------------------------------------------------------ put / get */
#define VSHMEM_COPY_UNROLL 4

/* put: PE `pe`'s dest[0, n) <- my src[0, n) */
__device__ __forceinline__ void shmem_putmem(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false>(shmem_ptr(ctx, (uint8_t *)dest, pe),
                                                         shmem_ptr(ctx, (const uint8_t *)src, ctx.me), n, 0, 1);
}
__device__ __forceinline__ void shmem_putmem_nbi(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmem_putmem_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false>(shmem_ptr(ctx, (uint8_t *)dest, pe),
                                                         shmem_ptr(ctx, (const uint8_t *)src, ctx.me), n,
                                                         __lane_id(), 64);
}
__device__ __forceinline__ void shmem_putmem_nbi_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem_wave(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmem_putmem_nbi_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false>(shmem_ptr(ctx, (uint8_t *)dest, pe),
                                                         shmem_ptr(ctx, (const uint8_t *)src, ctx.me), n,
                                                         threadIdx.x, blockDim.x);
}
__device__ __forceinline__ void shmem_putmem_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_putmem_nbi_wg(ctx, dest, src, n, pe);
    __syncthreads();
}
/* Grid scope: the nwgs work-groups acting for the PE (this one is `rank`)
 * share the message; each returns when its own share is locally complete. */
__device__ __forceinline__ void shmemx_putmem_grid(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n,
                                                   int pe, int rank, int nwgs)
{
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false>(shmem_ptr(ctx, (uint8_t *)dest, pe),
                                                         shmem_ptr(ctx, (const uint8_t *)src, ctx.me), n,
                                                         (uint64_t)rank * blockDim.x + threadIdx.x,
                                                         (uint64_t)nwgs * blockDim.x);
}

/* get: my dest[0, n) <- PE `pe`'s src[0, n) */
__device__ __forceinline__ void shmem_getmem(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false>(shmem_ptr(ctx, (uint8_t *)dest, ctx.me),
                                                         shmem_ptr(ctx, (const uint8_t *)src, pe), n, 0, 1);
}
__device__ __forceinline__ void shmem_getmem_nbi(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_getmem(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmem_getmem_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false>(shmem_ptr(ctx, (uint8_t *)dest, ctx.me),
                                                         shmem_ptr(ctx, (const uint8_t *)src, pe), n,
                                                         __lane_id(), 64);
}
__device__ __forceinline__ void shmem_getmem_nbi_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    shmem_getmem_wave(ctx, dest, src, n, pe);
}
__device__ __forceinline__ void shmem_getmem_nbi_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n, int pe)
{
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false>(shmem_ptr(ctx, (uint8_t *)dest, ctx.me),
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
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false>(shmem_ptr(ctx, (uint8_t *)dest, ctx.me),
                                                         shmem_ptr(ctx, (const uint8_t *)src, pe), n,
                                                         (uint64_t)rank * blockDim.x + threadIdx.x,
                                                         (uint64_t)nwgs * blockDim.x);
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
    return (int64_t)__hip_atomic_fetch_add(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void shmem_int64_atomic_add(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    __hip_atomic_fetch_add(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t shmem_uint64_atomic_fetch_xor(const shmem_dctx_t &ctx, uint64_t *dest, uint64_t v, int pe)
{
    return __hip_atomic_fetch_xor(VSHMEM_AMO_PTR(uint64_t), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t shmem_int64_atomic_fetch_xor(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    return (int64_t)__hip_atomic_fetch_xor(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void shmem_uint64_atomic_xor(const shmem_dctx_t &ctx, uint64_t *dest, uint64_t v, int pe)
{
    __hip_atomic_fetch_xor(VSHMEM_AMO_PTR(uint64_t), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void shmem_int64_atomic_xor(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    __hip_atomic_fetch_xor(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t shmem_int64_atomic_compare_swap(const shmem_dctx_t &ctx, int64_t *dest, int64_t cond,
                                                                   int64_t v, int pe)
{
    uint64_t expected = (uint64_t)cond;
    __hip_atomic_compare_exchange_strong(VSHMEM_AMO_PTR(uint64_t), &expected, (uint64_t)v, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (int64_t)expected;
}
__device__ __forceinline__ int64_t shmem_int64_atomic_fetch(const shmem_dctx_t &ctx, const int64_t *dest, int pe)
{
    return (int64_t)__hip_atomic_load((uint64_t *)shmem_ptr(ctx, (const uint8_t *)dest, pe), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void shmem_int64_atomic_set(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    __hip_atomic_store(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t shmem_int64_atomic_swap(const shmem_dctx_t &ctx, int64_t *dest, int64_t v, int pe)
{
    return (int64_t)__hip_atomic_exchange(VSHMEM_AMO_PTR(uint64_t), (uint64_t)v, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
}

/* ------------------------------------------------- signals and waiting */
__device__ __forceinline__ void vshmemx_signal_update(const shmem_dctx_t &ctx, uint64_t *sig, uint64_t v, int sig_op, int pe)
{
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
    shmem_putmem(ctx, dest, src, n, pe);
    vshmem_detail::release_agent();
    vshmemx_signal_update(ctx, sig, sigval, sig_op, pe);
}
__device__ __forceinline__ void shmem_putmem_signal_wave(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n,
                                                         uint64_t *sig, uint64_t sigval, int sig_op, int pe)
{
    shmem_putmem_wave(ctx, dest, src, n, pe);
    vshmem_detail::release_agent();
    if (__lane_id() == 0) vshmemx_signal_update(ctx, sig, sigval, sig_op, pe);
}
__device__ __forceinline__ void shmem_putmem_signal_wg(const shmem_dctx_t &ctx, void *dest, const void *src, size_t n,
                                                       uint64_t *sig, uint64_t sigval, int sig_op, int pe)
{
    shmem_putmem_nbi_wg(ctx, dest, src, n, pe);
    vshmem_detail::release_wg_at_exit();
    if (threadIdx.x == 0) vshmemx_signal_update(ctx, sig, sigval, sig_op, pe);
    __syncthreads();
}

/* Wait on my own copy of a symmetric uint64 signal. */
__device__ __forceinline__ uint64_t shmem_signal_wait_until(const shmem_dctx_t &ctx, uint64_t *sig, int cmp, uint64_t v)
{
    return vshmem_detail::spin_until<false>(ctx.c, shmem_ptr(ctx, sig, ctx.me), cmp, v);
}
__device__ __forceinline__ void shmem_int64_wait_until(const shmem_dctx_t &ctx, int64_t *ivar, int cmp, int64_t v)
{
    vshmem_detail::spin_until<true>(ctx.c, (uint64_t *)shmem_ptr(ctx, ivar, ctx.me), cmp, (uint64_t)v);
}
__device__ __forceinline__ int shmem_int64_test(const shmem_dctx_t &ctx, int64_t *ivar, int cmp, int64_t v)
{
    int64_t x = (int64_t)__hip_atomic_load((uint64_t *)shmem_ptr(ctx, ivar, ctx.me), __ATOMIC_RELAXED,
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
/* Barrier of a team where `units_per_pe` work-groups act for each member
 * and every one of them calls this (work-group scope per caller).  Implies
 * quiet for every caller's earlier operations. */
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

/* barrier_all with one work-group per PE (rocSHMEM-style _wg routine). */
__device__ __forceinline__ void shmem_barrier_all_wg(const shmem_dctx_t &ctx)
{
    shmemx_dteam_t world{0, 1, ctx.c.npes, 0};
    shmemx_team_sync_units(ctx, world, 1);
}
__device__ __forceinline__ void shmem_team_sync_wg(const shmem_dctx_t &ctx, const shmemx_dteam_t &team)
{
    shmemx_team_sync_units(ctx, team, 1);
}

#endif /* VSHMEM_DEVICE_HPP */
