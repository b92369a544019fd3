// Kernels written the way a library user writes them: they include only the
// public headers, receive the published device context and a team
// descriptor from the host, and call the device-side collectives and team
// barriers themselves.  Built into its own shared library, apart from
// libvshmem.so, so that the header-only device API is exercised on its own.
#include <algorithm>
#include <hip/hip_runtime.h>

#include "vshmem.h"
#include "vshmem_device.hpp"

namespace {

enum { KIND_BROADCAST = 0, KIND_FCOLLECT = 1, KIND_ALLTOALL = 2, KIND_REDUCE = 3 };

// One collective per launch; nwgs == 1 selects the _wg routines, more the
// _grid ones.  Work-group b acts for team member b / nwgs.  One kernel per
// routine keeps each one's registers its own.
template <int KIND, int DT, int OP>
__device__ int one_collective(const shmem_dctx_t &ctx, const shmemx_dteam_t &team, void *dest, const void *src,
                              size_t n, int root, int rank, int nwgs)
{
    const bool wg = nwgs == 1;
    if (KIND == KIND_BROADCAST)
        return wg ? shmem_broadcastmem_wg(ctx, team, dest, src, n, root)
                  : shmemx_broadcastmem_grid(ctx, team, dest, src, n, root, rank, nwgs);
    if (KIND == KIND_FCOLLECT)
        return wg ? shmem_fcollectmem_wg(ctx, team, dest, src, n)
                  : shmemx_fcollectmem_grid(ctx, team, dest, src, n, rank, nwgs);
    if (KIND == KIND_ALLTOALL)
        return wg ? shmem_alltoallmem_wg(ctx, team, dest, src, n)
                  : shmemx_alltoallmem_grid(ctx, team, dest, src, n, rank, nwgs);
#define USER_RED(T, WGF, GRIDF)                                                                              \
    return wg ? WGF(ctx, team, (T *)dest, (const T *)src, n) : GRIDF(ctx, team, (T *)dest, (const T *)src, n, \
                                                                      rank, nwgs)
    constexpr bool sum = OP == SHMEMX_RED_SUM;
    if (DT == SHMEMX_DT_INT64) {
        if (sum) USER_RED(int64_t, shmem_int64_sum_reduce_wg, shmemx_int64_sum_reduce_grid);
        USER_RED(int64_t, shmem_int64_max_reduce_wg, shmemx_int64_max_reduce_grid);
    }
    if (DT == SHMEMX_DT_FP32) {
        if (sum) USER_RED(float, shmem_float_sum_reduce_wg, shmemx_float_sum_reduce_grid);
        USER_RED(float, shmem_float_max_reduce_wg, shmemx_float_max_reduce_grid);
    }
    if (sum) USER_RED(uint16_t, shmemx_bfloat16_sum_reduce_wg, shmemx_bfloat16_sum_reduce_grid);
    USER_RED(uint16_t, shmemx_bfloat16_max_reduce_wg, shmemx_bfloat16_max_reduce_grid);
#undef USER_RED
}

template <int KIND, int DT, int OP>
__global__ void __launch_bounds__(256) k_user_collective(const shmemx_dctx_pub_t *pub, shmemx_dteam_t team, void *dest,
                                                         const void *src, size_t n, int root, int nwgs, int *status)
{
    const int k = (int)(blockIdx.x / (unsigned)nwgs);
    const shmem_dctx_t ctx = shmemx_dctx_bind(*pub, shmemx_team_pe(team, k));
    const int rc = one_collective<KIND, DT, OP>(ctx, team, dest, src, n, root, (int)blockIdx.x - k * nwgs, nwgs);
    if (threadIdx.x == 0) status[blockIdx.x] = rc;
}

// Three steps in one launch: every member scales its own int64 input by
// (its PE number + 1) into x, the team sums x into y, and fcollect gathers
// the first m elements of every member's y into z.
__global__ void __launch_bounds__(256) k_user_pipeline(const shmemx_dctx_pub_t *pub, shmemx_dteam_t team,
                                                       const int64_t *src, int64_t *x, int64_t *y, int64_t *z,
                                                       size_t n, size_t m, int nwgs)
{
    const int k = (int)(blockIdx.x / (unsigned)nwgs);
    const int rank = (int)blockIdx.x - k * nwgs;
    const shmem_dctx_t ctx = shmemx_dctx_bind(*pub, shmemx_team_pe(team, k));
    const int64_t *s = shmemx_local_ptr(ctx, src);
    int64_t *xm = shmemx_local_ptr(ctx, x);
    const int64_t f = ctx.me + 1;
    for (size_t i = (size_t)rank * blockDim.x + threadIdx.x; i < n; i += (size_t)nwgs * blockDim.x) xm[i] = s[i] * f;
    // The reduction opens with a team barrier, which completes these stores.
    shmemx_int64_sum_reduce_grid(ctx, team, y, x, n, rank, nwgs);
    shmemx_fcollectmem_grid(ctx, team, z, y, m * sizeof(int64_t), rank, nwgs);
}

// Token exchange through a barrier at one scope: in round r the caller of
// member k stores r + 1 into its own tok, synchronises, checks that member
// k + 1 (mod size) stored r + 1 too, and synchronises again before the next
// round may overwrite it.  One work-group per member.
__global__ void __launch_bounds__(256) k_user_barrier(const shmemx_dctx_pub_t *pub, shmemx_dteam_t team, int scope,
                                                      int world, int iters, int64_t *tok, unsigned long long *bad)
{
    const int k = (int)blockIdx.x;
    const shmem_dctx_t ctx = shmemx_dctx_bind(*pub, shmemx_team_pe(team, k));
    const int64_t *next = shmem_ptr(ctx, tok, shmemx_team_pe(team, (k + 1) % team.size));
    int64_t *mine = shmemx_local_ptr(ctx, tok);
    // Who calls: thread 0 (thread scope), wavefront 0 (wave scope) or all.
    const bool caller = scope == SHMEMX_SCOPE_THREAD ? threadIdx.x == 0
                        : scope == SHMEMX_SCOPE_WAVE ? threadIdx.x < 64
                                                     : true;
    const bool leader = threadIdx.x == 0;
    if (!caller) return;
    for (int r = 0; r < iters; ++r) {
        if (leader) __hip_atomic_store(mine, (int64_t)r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int half = 0; half < 2; ++half) {
            if (half == 1 && leader &&
                __hip_atomic_load(next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != (int64_t)r + 1)
                atomicAdd(bad, 1ull);
            if (scope == SHMEMX_SCOPE_THREAD) {
                if (world) shmem_barrier_all(ctx);
                else shmem_team_sync(ctx, team);
            } else if (scope == SHMEMX_SCOPE_WAVE) {
                if (world) shmem_barrier_all_wave(ctx);
                else shmem_team_sync_wave(ctx, team);
            } else {
                if (world) shmem_barrier_all_wg(ctx);
                else shmem_team_sync_wg(ctx, team);
            }
        }
    }
}

// An explicit context bound to a team, one work-group per member: record
// shmem_my_pe and shmem_n_pes, put the local block to member k + 1 (team
// numbering), synchronise the context's team, get member k - 1's block, and
// add one to member 0's counter, keeping the value fetched.
__global__ void __launch_bounds__(256) k_user_ctx(const shmemx_dctx_rec_t *rec, const uint8_t *src, uint8_t *dst,
                                                  uint8_t *back, size_t n, int64_t *ctr, int32_t *ids,
                                                  int64_t *fetched)
{
    const shmem_dctx_t ctx = shmemx_dctx_bind_explicit(*rec, (int)blockIdx.x);
    const int me = shmem_my_pe(ctx), np = shmem_n_pes(ctx);
    if (threadIdx.x == 0) {
        ids[2 * blockIdx.x] = me;
        ids[2 * blockIdx.x + 1] = np;
    }
    shmem_putmem_wg(ctx, dst, src, n, (me + 1) % np);
    shmem_team_sync_wg(ctx, shmemx_ctx_team(ctx));   // completes every member's put
    shmem_getmem_wg(ctx, back, dst, n, (me + np - 1) % np);
    if (threadIdx.x == 0) fetched[blockIdx.x] = shmem_int64_atomic_fetch_add(ctx, ctr, 1, 0);
    shmem_quiet_wg(ctx);
}

// The GPU-space usage example, one work-group per PE on objects from
// shmemg_malloc: put the local block to PE me + 1 at work-group scope, fence
// and quiet, barrier; then wave 0 gets the block back from PE me + 1 and
// thread 0 gets `tail` bytes of it at offset `at` with a thread-scope get.
__global__ void __launch_bounds__(256) k_user_gspace(const shmemx_dctx_pub_t *pub, const uint8_t *src, uint8_t *dst,
                                                     uint8_t *back, uint8_t *part, size_t n, size_t at, size_t tail)
{
    const shmem_dctx_t ctx = shmemx_dctx_bind(*pub, (int)blockIdx.x);
    const int me = shmem_my_pe(ctx), np = shmem_n_pes(ctx);
    shmemg_putmem_wg(ctx, dst, src, n, (me + 1) % np);
    shmem_fence_wg(ctx);
    shmem_quiet_wg(ctx);
    shmem_barrier_all_wg(ctx);
    if (threadIdx.x < 64) shmemg_getmem_wave(ctx, back, dst, n, (me + 1) % np);
    if (threadIdx.x == 0) shmemg_getmem(ctx, part, dst + at, tail, (me + 1) % np);
    shmem_quiet_wg(ctx);
}

// Ordering by fence: the producer (work-group 0, PE prod) fills its local
// block with the round number, puts it to the consumer, fences, and sets the
// consumer's flag to round + 1; the consumer (work-group 1, PE cons) waits
// for the flag, checks every word it received and acknowledges on the
// producer's flag before the next round may overwrite the block.
__global__ void __launch_bounds__(256) k_user_fence(const shmemx_dctx_pub_t *pub, int prod, int cons, int64_t *block,
                                                    size_t nwords, uint64_t *flag, int rounds,
                                                    unsigned long long *bad)
{
    const bool producer = blockIdx.x == 0;
    const shmem_dctx_t ctx = shmemx_dctx_bind(*pub, producer ? prod : cons);
    int64_t *mine = shmemx_local_ptr(ctx, block);
    for (int r = 0; r < rounds; ++r) {
        if (producer) {
            for (size_t i = threadIdx.x; i < nwords; i += blockDim.x) mine[i] = r;
            __syncthreads();
            shmem_putmem_nbi_wg(ctx, block, block, nwords * sizeof(int64_t), cons);
            shmem_fence_wg(ctx);
            if (threadIdx.x == 0) vshmemx_signal_update(ctx, flag, (uint64_t)r + 1, SHMEM_SIGNAL_SET, cons);
            shmem_signal_wait_until_wg(ctx, flag, SHMEM_CMP_GE, (uint64_t)r + 1);
        } else {
            shmem_signal_wait_until_wg(ctx, flag, SHMEM_CMP_GE, (uint64_t)r + 1);
            unsigned long long nb = 0;
            for (size_t i = threadIdx.x; i < nwords; i += blockDim.x) nb += mine[i] != r;
            if (nb) atomicAdd(bad, nb);
            __syncthreads();
            if (threadIdx.x == 0) vshmemx_signal_update(ctx, flag, (uint64_t)r + 1, SHMEM_SIGNAL_SET, prod);
        }
    }
}

// Debug-mode argument checks (the library initialised with VSHMEM_DEBUG
// set): each case makes calls that a check must refuse, except case 4,
// which is valid.  `outside` is device memory outside the heap and every
// refused PE number still names memory inside the heap, so a call that got
// past its check would write valid memory rather than fault.
__global__ void __launch_bounds__(256) k_user_debug(const shmemx_dctx_pub_t *pub, const shmemx_dctx_rec_t *rec,
                                                    shmemx_dteam_t pair, int which, uint8_t *sym, uint8_t *outside,
                                                    int64_t *out)
{
    const shmem_dctx_t ctx = shmemx_dctx_bind(*pub, (int)blockIdx.x);
    switch (which) {
    case 0:   // destination outside the heap
        if (threadIdx.x == 0) shmem_putmem(ctx, outside, sym, 64, 1);
        break;
    case 1:   // atomic on a word outside the heap
        if (threadIdx.x == 0) out[0] = shmem_int64_atomic_fetch_add(ctx, (int64_t *)outside, 1, 1);
        break;
    case 2:   // wavefront call where lane 5 passes another size
        if (threadIdx.x < 64) shmem_putmem_wave(ctx, sym + 4096, sym, threadIdx.x == 5 ? 32 : 64, 1);
        break;
    case 3:   // work-group call where thread 100 passes another PE
        shmem_putmem_wg(ctx, sym + 4096, sym, 64, threadIdx.x == 100 ? 2 : 1);
        break;
    case 4:   // valid
        if (threadIdx.x == 0) shmem_putmem(ctx, sym + 4096, sym, 64, 1);
        break;
    case 5: { // PE 2 of a two-member explicit context
        const shmem_dctx_t two = shmemx_dctx_bind_explicit(*rec, 0);
        if (threadIdx.x == 0) shmem_putmem(two, sym + 4096, sym, 64, 2);
        break;
    }
    default: { // broadcast from a root outside the two-member team: refused before any barrier
        const int rc = shmem_broadcastmem_wg(ctx, pair, sym + 4096, sym, 64, 2);
        if (threadIdx.x == 0) out[blockIdx.x] = rc;
        break;
    }
    }
}

// A kernel that writes a descriptor table: record i is assembled from
// column arrays (op, scope, aux and flags packed in one word per record).
__global__ void k_user_write_table(shmemx_desc_t *out, size_t n, const uint32_t *code, const int32_t *issuer,
                                   const int32_t *target, const uint32_t *ridx, const uint64_t *src,
                                   const uint64_t *dst, const uint64_t *nbytes, const uint64_t *value,
                                   const uint64_t *cond)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        shmemx_desc_t d;
        d.op = (uint8_t)(code[i] & 0xFF);
        d.scope = (uint8_t)((code[i] >> 8) & 0xFF);
        d.aux = (uint8_t)((code[i] >> 16) & 0xFF);
        d.flags = (uint8_t)(code[i] >> 24);
        d.issuer_pe = issuer[i];
        d.target_pe = target[i];
        d.result_idx = ridx[i];
        d.src = src[i];
        d.dst = dst[i];
        d.nbytes = nbytes[i];
        d.value = value[i];
        d.cond = cond[i];
        d.reserved = 0;
        out[i] = d;
    }
}

}  // namespace

extern "C" {

int usertest_write_table(void *out, size_t n, const void *code, const void *issuer, const void *target,
                         const void *ridx, const void *src, const void *dst, const void *nbytes, const void *value,
                         const void *cond, void *stream)
{
    if (!out || (n && (!code || !issuer || !target || !ridx || !src || !dst || !nbytes || !value || !cond))) return -1;
    if (n == 0) return 0;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_user_write_table, dim3(grid), dim3(256), 0, (hipStream_t)stream, (shmemx_desc_t *)out, n,
                       (const uint32_t *)code, (const int32_t *)issuer, (const int32_t *)target,
                       (const uint32_t *)ridx, (const uint64_t *)src, (const uint64_t *)dst, (const uint64_t *)nbytes,
                       (const uint64_t *)value, (const uint64_t *)cond);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Each launcher checks what it can on the host and returns 0, or -1 for an
// argument its kernel would not handle.
int usertest_collective(const void *dctx, const shmemx_dteam_t *team, int kind, int dtype, int op, void *dest,
                        const void *src, size_t n, int root, int nwgs, int wg, int *status, void *stream)
{
    if (!dctx || !team || kind < 0 || kind > KIND_REDUCE || nwgs < 1 || wg < 64 || wg > 256 || wg % 64 || !status)
        return -1;
    if (kind == KIND_REDUCE && (dtype < SHMEMX_DT_INT64 || dtype > SHMEMX_DT_BF16 || op < SHMEMX_RED_SUM ||
                                op > SHMEMX_RED_MAX))
        return -1;
    const dim3 grid(team->size * nwgs), block(wg);
    const auto *pub = (const shmemx_dctx_pub_t *)dctx;
    hipStream_t s = (hipStream_t)stream;
#define USER_LAUNCH(K, D, O) \
    hipLaunchKernelGGL((k_user_collective<K, D, O>), grid, block, 0, s, pub, *team, dest, src, n, root, nwgs, status)
    if (kind == KIND_BROADCAST) USER_LAUNCH(KIND_BROADCAST, 0, 0);
    else if (kind == KIND_FCOLLECT) USER_LAUNCH(KIND_FCOLLECT, 0, 0);
    else if (kind == KIND_ALLTOALL) USER_LAUNCH(KIND_ALLTOALL, 0, 0);
    else if (dtype == SHMEMX_DT_INT64 && op == SHMEMX_RED_SUM) USER_LAUNCH(KIND_REDUCE, SHMEMX_DT_INT64, SHMEMX_RED_SUM);
    else if (dtype == SHMEMX_DT_INT64) USER_LAUNCH(KIND_REDUCE, SHMEMX_DT_INT64, SHMEMX_RED_MAX);
    else if (dtype == SHMEMX_DT_FP32 && op == SHMEMX_RED_SUM) USER_LAUNCH(KIND_REDUCE, SHMEMX_DT_FP32, SHMEMX_RED_SUM);
    else if (dtype == SHMEMX_DT_FP32) USER_LAUNCH(KIND_REDUCE, SHMEMX_DT_FP32, SHMEMX_RED_MAX);
    else if (op == SHMEMX_RED_SUM) USER_LAUNCH(KIND_REDUCE, SHMEMX_DT_BF16, SHMEMX_RED_SUM);
    else USER_LAUNCH(KIND_REDUCE, SHMEMX_DT_BF16, SHMEMX_RED_MAX);
#undef USER_LAUNCH
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int usertest_pipeline(const void *dctx, const shmemx_dteam_t *team, const int64_t *src, int64_t *x, int64_t *y,
                      int64_t *z, size_t n, size_t m, int nwgs, int wg, void *stream)
{
    if (!dctx || !team || m > n || nwgs < 1 || wg < 64 || wg > 256 || wg % 64) return -1;
    hipLaunchKernelGGL(k_user_pipeline, dim3(team->size * nwgs), dim3(wg), 0, (hipStream_t)stream,
                       (const shmemx_dctx_pub_t *)dctx, *team, src, x, y, z, n, m, nwgs);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int usertest_barrier(const void *dctx, const shmemx_dteam_t *team, int scope, int world, int iters, int64_t *tok,
                     unsigned long long *bad, int wg, void *stream)
{
    if (!dctx || !team || scope < SHMEMX_SCOPE_THREAD || scope > SHMEMX_SCOPE_WG || iters < 0 || wg < 64 ||
        wg > 256 || wg % 64 || !bad)
        return -1;
    hipLaunchKernelGGL(k_user_barrier, dim3(team->size), dim3(wg), 0, (hipStream_t)stream,
                       (const shmemx_dctx_pub_t *)dctx, *team, scope, world, iters, tok, bad);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int usertest_gspace(const void *dctx, int npes, const void *src, void *dst, void *back, void *part, size_t n,
                    size_t at, size_t tail, void *stream)
{
    if (!dctx || npes < 1 || npes > 64 || at > n || tail > n - at) return -1;
    hipLaunchKernelGGL(k_user_gspace, dim3(npes), dim3(256), 0, (hipStream_t)stream, (const shmemx_dctx_pub_t *)dctx,
                       (const uint8_t *)src, (uint8_t *)dst, (uint8_t *)back, (uint8_t *)part, n, at, tail);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int usertest_ctx(const void *rec, int team_size, const void *src, void *dst, void *back, size_t n, int64_t *ctr,
                 int32_t *ids, int64_t *fetched, int wg, void *stream)
{
    if (!rec || team_size < 1 || wg < 64 || wg > 256 || wg % 64 || !ids || !fetched) return -1;
    hipLaunchKernelGGL(k_user_ctx, dim3(team_size), dim3(wg), 0, (hipStream_t)stream, (const shmemx_dctx_rec_t *)rec,
                       (const uint8_t *)src, (uint8_t *)dst, (uint8_t *)back, n, ctr, ids, fetched);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int usertest_fence(const void *dctx, int prod, int cons, int64_t *block, size_t nwords, uint64_t *flag, int rounds,
                   unsigned long long *bad, void *stream)
{
    if (!dctx || prod == cons || rounds < 0 || !bad) return -1;
    hipLaunchKernelGGL(k_user_fence, dim3(2), dim3(256), 0, (hipStream_t)stream, (const shmemx_dctx_pub_t *)dctx,
                       prod, cons, block, nwords, flag, rounds, bad);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int usertest_debug(const void *dctx, const void *rec, const shmemx_dteam_t *pair, int which, void *sym, void *outside,
                   int64_t *out, int grid, void *stream)
{
    if (!dctx || !rec || !pair || which < 0 || which > 6 || grid < 1 || grid > 2) return -1;
    hipLaunchKernelGGL(k_user_debug, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const shmemx_dctx_pub_t *)dctx,
                       (const shmemx_dctx_rec_t *)rec, *pair, which, (uint8_t *)sym, (uint8_t *)outside, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
