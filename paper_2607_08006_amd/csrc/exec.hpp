// Executors of single descriptor operations, shared by the batched forms
// (plans built on the host, descriptor tables in device memory) and their
// per-operation launches.  Internal to the library.
#pragma once
#include "runtime.hpp"

namespace vshmem_exec {

// Host and device: whether an op code is a fence, quiet or barrier, and
// whether it is an atomic.
__host__ __device__ __forceinline__ bool is_sync_op(uint8_t op)
{
    return op == SHMEMX_OP_FENCE || op == SHMEMX_OP_QUIET || op == SHMEMX_OP_BARRIER_ALL;
}
__host__ __device__ __forceinline__ bool is_amo_op(uint8_t op)
{
    return op >= SHMEMX_OP_AMO_FETCH_ADD && op <= SHMEMX_OP_AMO_SWAP;
}
// Size class of a message: floor(log2(n)), capped at the table's last class.
__host__ __device__ __forceinline__ int size_class(uint64_t n)
{
    int c = 0;
    while (c + 1 < SHMEMX_TUNE_CLASSES && (2ull << c) <= n) ++c;
    return c;
}
// Scope an operation executes at: an explicit scope, else the table's
// choice for its size class (atomics: one lane).
__host__ __device__ __forceinline__ int resolve_scope(const shmemx_desc_t &d, const shmemx_tune_t &tune)
{
    if (is_amo_op(d.op)) return d.scope == SHMEMX_SCOPE_AUTO ? SHMEMX_SCOPE_THREAD : d.scope;
    if (d.scope != SHMEMX_SCOPE_AUTO) return d.scope;
    return tune.scope[size_class(d.nbytes)];
}
// Bytes per work-group task of an operation at `scope`: the table's chunk
// for its class (grid scope: 256 KiB when the table has none), rounded up
// to 16; signal-puts and atomics are never split.
__host__ __device__ __forceinline__ uint64_t resolve_chunk(const shmemx_desc_t &d, int scope, const shmemx_tune_t &tune)
{
    if (d.op == SHMEMX_OP_PUT_SIGNAL || is_amo_op(d.op)) return d.nbytes ? d.nbytes : 1;
    uint64_t ch = tune.chunk[size_class(d.nbytes)];
    if (scope == SHMEMX_SCOPE_GRID && ch == 0) ch = 256ull << 10;
    if (ch == 0 || ch >= d.nbytes) return d.nbytes ? d.nbytes : 1;
    return (ch + 15) & ~15ull;
}

__device__ __forceinline__ uint64_t *amo_word(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d)
{
    return (uint64_t *)(c.base + (uint64_t)d.target_pe * c.stride + d.src);
}

// Atomics and signal-free single-lane work.
__device__ __forceinline__ void exec_amo(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d, uint64_t *results)
{
    uint64_t *w = amo_word(c, d);
    uint64_t old = 0;
    bool fetch = true;
    switch (d.op) {
    case SHMEMX_OP_AMO_FETCH_ADD: old = __hip_atomic_fetch_add(w, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    case SHMEMX_OP_AMO_FETCH_XOR: old = __hip_atomic_fetch_xor(w, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    case SHMEMX_OP_AMO_COMPARE_SWAP: {
        uint64_t e = d.cond;
        __hip_atomic_compare_exchange_strong(w, &e, d.value, __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        old = e;
        break;
    }
    case SHMEMX_OP_AMO_ADD:
        __hip_atomic_fetch_add(w, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        fetch = false;
        break;
    case SHMEMX_OP_AMO_XOR:
        __hip_atomic_fetch_xor(w, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        fetch = false;
        break;
    case SHMEMX_OP_AMO_SET:
        __hip_atomic_store(w, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        fetch = false;
        break;
    case SHMEMX_OP_AMO_FETCH: old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    case SHMEMX_OP_AMO_SWAP: old = __hip_atomic_exchange(w, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); break;
    default: fetch = false;
    }
    if (fetch && results && d.result_idx != SHMEMX_NO_RESULT) results[d.result_idx] = old;
}

// Byte range [lo, hi) of a put/get, copied by nl lanes (LONE: by one lane).
template <bool LONE = false>
__device__ __forceinline__ void exec_copy(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d, uint64_t lo, uint64_t hi,
                                          uint64_t lane, uint64_t nl)
{
    const bool get = d.op == SHMEMX_OP_GET;
    const int spe = get ? d.target_pe : d.issuer_pe;
    const int dpe = get ? d.issuer_pe : d.target_pe;
    const uint8_t *S = c.base + (uint64_t)spe * c.stride + d.src + lo;
    uint8_t *D = c.base + (uint64_t)dpe * c.stride + d.dst + lo;
    vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, false, true, LONE>(D, S, hi - lo, lane, nl);
}

__device__ __forceinline__ void signal_of(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d)
{
    uint64_t *s = (uint64_t *)(c.base + (uint64_t)d.target_pe * c.stride + d.cond);
    if (d.aux == SHMEM_SIGNAL_ADD)
        __hip_atomic_fetch_add(s, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_store(s, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One operation by a single lane.
__device__ __forceinline__ void exec_thread(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d, uint64_t *results)
{
    if (is_amo_op(d.op)) {
        exec_amo(c, d, results);
    } else if (d.op == SHMEMX_OP_PUT || d.op == SHMEMX_OP_GET || d.op == SHMEMX_OP_PUT_SIGNAL) {
        exec_copy<true>(c, d, 0, d.nbytes, 0, 1);
        if (d.op == SHMEMX_OP_PUT_SIGNAL) {
            vshmem_detail::release_agent();
            signal_of(c, d);
        }
    }
}

// One operation by a whole wavefront.
__device__ __forceinline__ void exec_wave(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d, uint64_t *results)
{
    if (is_amo_op(d.op)) {
        if (__lane_id() == 0) exec_amo(c, d, results);
    } else if (d.op == SHMEMX_OP_PUT || d.op == SHMEMX_OP_GET || d.op == SHMEMX_OP_PUT_SIGNAL) {
        exec_copy(c, d, 0, d.nbytes, __lane_id(), 64);
        if (d.op == SHMEMX_OP_PUT_SIGNAL) {
            vshmem_detail::release_agent();
            if (__lane_id() == 0) signal_of(c, d);
        }
    }
}

// A byte range of one operation by a whole work-group.
__device__ __forceinline__ void exec_wg(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d, uint64_t lo, uint64_t hi,
                                        uint64_t *results)
{
    if (is_amo_op(d.op)) {
        if (threadIdx.x == 0) exec_amo(c, d, results);
    } else if (d.op == SHMEMX_OP_PUT || d.op == SHMEMX_OP_GET || d.op == SHMEMX_OP_PUT_SIGNAL) {
        exec_copy(c, d, lo, hi, threadIdx.x, blockDim.x);
        if (__builtin_amdgcn_readfirstlane(d.op) == SHMEMX_OP_PUT_SIGNAL) {   // uniform: a barrier follows
            vshmem_detail::release_wg_at_exit();
            if (threadIdx.x == 0) signal_of(c, d);
        }
    }
}

}  // namespace vshmem_exec
