// Pieces shared by the serving forms: the persistent progress kernel, one
// launch per request, and windowed batches (fused or replayed from a graph).
#pragma once
#include "runtime.hpp"

namespace vshmem {

// A serving request is PUT, GET, or AMO_FETCH_ADD over nbytes/8 counters at
// src on the target PE with the fetched values to dst on the issuer; every
// range inside the user heap.
bool valid_request_host(const shmemx_desc_t &d);

__device__ __forceinline__ uint8_t *pe_slice(const shmemx_dctx_pub_t &c, int pe)
{
    return c.base + (uint64_t)pe * c.stride;
}

// Bytes [lo, hi) of a serving request, executed by nl cooperating lanes
// (this one is `lane`).  Returns the start of the request's output.
__device__ __forceinline__ uint8_t *exec_request_range(const shmemx_dctx_pub_t &c, const shmemx_desc_t &d,
                                                       uint64_t lo, uint64_t hi, uint64_t lane, uint64_t nl)
{
    if (d.op == SHMEMX_OP_AMO_FETCH_ADD) {
        uint64_t *ctr = (uint64_t *)(pe_slice(c, d.target_pe) + d.src);
        uint64_t *res = (uint64_t *)(pe_slice(c, d.issuer_pe) + d.dst);
        // kAmoBatch atomics in flight per lane, then their results: a result
        // store may alias a later counter, so one atomic per store would
        // cost a full round trip each.
        constexpr int kAmoBatch = 8;
        uint64_t k = lo / 8 + lane;
        const uint64_t end = hi / 8;
        for (; k + (kAmoBatch - 1) * nl < end; k += kAmoBatch * nl) {
            uint64_t old[kAmoBatch];
#pragma unroll
            for (int j = 0; j < kAmoBatch; ++j)
                old[j] = __hip_atomic_fetch_add(ctr + k + j * nl, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int j = 0; j < kAmoBatch; ++j) res[k + j * nl] = old[j];
        }
        for (; k < end; k += nl)
            res[k] = __hip_atomic_fetch_add(ctr + k, d.value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return (uint8_t *)res;
    }
    const bool get = d.op == SHMEMX_OP_GET;
    const int spe = get ? d.target_pe : d.issuer_pe;
    const int dpe = get ? d.issuer_pe : d.target_pe;
    uint8_t *out = pe_slice(c, dpe) + d.dst;
    if (lo < hi) vshmem_detail::copy_bytes<8, true, true>(out + lo, pe_slice(c, spe) + d.src + lo, hi - lo, lane, nl);
    return out;
}

// Windowed batches: up to kWindowBatchMax requests per batch, kWindowSlots
// batches in flight.  A batch is staged from pinned host memory into device
// memory by one kernel and executed by a second (fixed grid, so the pair can
// be captured once per slot in a graph and replayed).
constexpr size_t kWindowBatchMax = 4096;
constexpr int kWindowSlots = 4;
struct WindowBatcher;
WindowBatcher *window_batcher_create(bool graph, uint64_t chunk_bytes, int nwg, int wg_size, hipStream_t stream,
                                     int *rc);
// Launch requests d[0, n) from slot `slot` (whose previous batch must have
// completed) and record `done` after them.
int window_batcher_launch(WindowBatcher *b, int slot, const shmemx_desc_t *d, size_t n, hipEvent_t done);
void window_batcher_destroy(WindowBatcher *b);

}  // namespace vshmem
