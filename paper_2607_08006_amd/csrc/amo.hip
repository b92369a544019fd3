// Atomics and point-to-point synchronisation: GUPS-style random-access
// atomics, put-with-signal ping-pong, and the team barrier kernel.
#include <atomic>

#include "runtime.hpp"

using namespace vshmem;

namespace {

__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Update u: index x_{3u} mod 2^log2_table, value x_{3u+1}, fetch_add when
// x_{3u+2} mod add_every == 0 else fetch_xor, on the word's home PE.
template <bool STORE>
__global__ void __launch_bounds__(256) k_gups(shmemx_dctx_pub_t c, uint64_t table_off, uint64_t gmask,
                                              int log2_per_pe, uint64_t nupd, uint64_t seed, uint64_t add_every,
                                              uint64_t *__restrict__ fetched, uint64_t *acc)
{
    const uint64_t lmask = (1ull << log2_per_pe) - 1;
    uint64_t x = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < nupd;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t g = splitmix_at(seed, 3 * u) & gmask;
        const uint64_t v = splitmix_at(seed, 3 * u + 1);
        const bool is_add = (splitmix_at(seed, 3 * u + 2) % add_every) == 0;
        uint64_t *w = (uint64_t *)(c.base + (g >> log2_per_pe) * c.stride + table_off + (g & lmask) * 8);
        const uint64_t old = is_add ? __hip_atomic_fetch_add(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                    : __hip_atomic_fetch_xor(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if constexpr (STORE) fetched[u] = old;
        x ^= old;
    }
    if (acc) {
        // Wavefront XOR-reduction, then one atomic per wavefront.
        for (int off = 32; off > 0; off >>= 1) x ^= __shfl_xor(x, off, 64);
        if (__lane_id() == 0 && x) __hip_atomic_fetch_xor(acc, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One wavefront per block; lane 0 of each block plays one side of a pair.
__global__ void __launch_bounds__(64) k_pingpong(shmemx_dctx_pub_t c, uint64_t data_off, uint64_t sig_off,
                                                 const int32_t *__restrict__ pairs, int npairs, int rounds,
                                                 uint64_t nbytes, int same_xcd, uint64_t tag,
                                                 uint64_t *__restrict__ rtt)
{
    int pair, role;
    if (same_xcd) {
        // Blocks b and b+8 share an XCD (blocks are dealt to XCDs round robin).
        int grp = blockIdx.x / 16, r = blockIdx.x % 16;
        pair = grp * 8 + (r % 8);
        role = r / 8;
    } else {
        pair = blockIdx.x / 2;
        role = blockIdx.x % 2;
    }
    if (pair >= npairs) return;
    const int a = pairs[2 * pair], b = pairs[2 * pair + 1];
    if (a < 0 || a >= c.npes || b < 0 || b >= c.npes) {
        if (__lane_id() == 0) vshmem_detail::latch_error(c, 0x2u);
        return;
    }
    const int me = role == 0 ? a : b, peer = role == 0 ? b : a;
    shmem_dctx_t ctx = shmemx_dctx_bind(c, me);
    uint8_t *data = c.base + data_off;
    uint64_t *sig = (uint64_t *)(c.base + sig_off);
    if (__lane_id() != 0) return;
    for (int r = 1; r <= rounds; ++r) {
        const uint64_t v = tag | (uint64_t)r;
        if (role == 0) {
            const uint64_t t0 = wall_clock64();
            shmem_putmem_signal(ctx, data, data, nbytes, sig, v, SHMEM_SIGNAL_SET, peer);
            shmem_signal_wait_until(ctx, sig, SHMEM_CMP_EQ, v);
            if (rtt) rtt[(uint64_t)pair * rounds + (r - 1)] = wall_clock64() - t0;
        } else {
            shmem_signal_wait_until(ctx, sig, SHMEM_CMP_EQ, v);
            shmem_putmem_signal(ctx, data, data, nbytes, sig, v, SHMEM_SIGNAL_SET, peer);
        }
    }
    shmem_quiet(ctx);
}

// One work-group per team member; `iters` barriers, optionally checking
// that every member's token of the iteration arrived before the barrier
// released anyone.
__global__ void __launch_bounds__(256) k_barrier(shmemx_dctx_pub_t c, shmemx_dteam_t team, int iters,
                                                 uint64_t tokens_off, uint64_t *bad, uint64_t *cycles)
{
    const int k = blockIdx.x;
    const int me = shmemx_team_pe(team, k);
    shmem_dctx_t ctx = shmemx_dctx_bind(c, me);
    const bool tokens = tokens_off != UINT64_MAX;
    uint64_t nbad = 0;
    const uint64_t t0 = wall_clock64();
    for (int it = 0; it < iters; ++it) {
        const uint64_t par = (uint64_t)(it & 1) * team.size;
        if (tokens) {
            // My token of this iteration into every member's slot k.
            for (int q = threadIdx.x; q < team.size; q += blockDim.x) {
                uint64_t *slot = (uint64_t *)(c.base + (uint64_t)shmemx_team_pe(team, q) * c.stride + tokens_off) + par + k;
                *slot = ((uint64_t)it << 32) | (uint64_t)me;
            }
        }
        shmemx_team_sync_units(ctx, team, 1);
        if (tokens) {
            const uint64_t *mine = (const uint64_t *)(c.base + (uint64_t)me * c.stride + tokens_off) + par;
            for (int q = threadIdx.x; q < team.size; q += blockDim.x)
                nbad += (mine[q] != (((uint64_t)it << 32) | (uint64_t)shmemx_team_pe(team, q)));
        }
    }
    if (cycles && k == 0 && threadIdx.x == 0) *cycles = wall_clock64() - t0;
    if (tokens && bad && nbad) __hip_atomic_fetch_add(bad, nbad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_wait_until(shmemx_dctx_pub_t c, int pe, uint64_t off, int cmp, uint64_t value, int is_unsigned,
                             uint64_t *out)
{
    if (threadIdx.x != 0) return;
    shmem_dctx_t ctx = shmemx_dctx_bind(c, pe);
    uint64_t *w = (uint64_t *)(c.base + off);
    uint64_t x = is_unsigned ? shmem_signal_wait_until(ctx, w, cmp, value)
                             : vshmem_detail::spin_until<true>(c, shmem_ptr(ctx, w, pe), cmp, value);
    if (out) *out = x;
}

std::atomic<uint64_t> g_pingpong_calls{1};

}  // namespace

extern "C" {

int shmemx_gups(uint64_t table_off, int log2_table, uint64_t nupdates, uint64_t seed, int add_every,
                uint64_t *fetched, uint64_t *acc, const shmemx_launch_t *launch, void *stream)
{
    if (int rc = check_ready()) return rc;
    const State &s = st();
    int log2_npes = 0;
    while ((1 << log2_npes) < s.npes) ++log2_npes;
    if ((1 << log2_npes) != s.npes || log2_table < log2_npes || log2_table > 40 || add_every <= 0 ||
        !in_user_heap(table_off, 8ull << (log2_table - log2_npes)) || (table_off & 7)) {
        set_last_error(SHMEMX_ERR_ARG);
        return SHMEMX_ERR_ARG;
    }
    if (nupdates == 0) return SHMEMX_OK;
    shmemx_launch_t tmp;
    const shmemx_launch_t &L = launch_or_default(launch, tmp, 0, 256, 0);
    uint64_t grid = L.wgs_per_pe > 0 && launch ? (uint64_t)L.wgs_per_pe * s.npes : (uint64_t)s.num_cus * 16;
    uint64_t need = (nupdates + 255) / 256;
    if (grid > need) grid = need;
    if (grid > (1u << 30)) grid = 1u << 30;
    const uint64_t gmask = (1ull << log2_table) - 1;
    const int log2_per_pe = log2_table - log2_npes;
    if (fetched)
        hipLaunchKernelGGL(k_gups<true>, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, pub(), table_off,
                           gmask, log2_per_pe, nupdates, seed, (uint64_t)add_every, fetched, acc);
    else
        hipLaunchKernelGGL(k_gups<false>, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, pub(), table_off,
                           gmask, log2_per_pe, nupdates, seed, (uint64_t)add_every, fetched, acc);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_pingpong(uint64_t data_off, uint64_t sig_off, const int32_t *pairs, int npairs, int rounds,
                    uint64_t payload_bytes, int same_xcd, uint64_t *rtt_cycles, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!pairs || npairs <= 0 || rounds <= 0 || (sig_off & 7) || !in_user_heap(sig_off, 8) ||
        !in_user_heap(data_off, payload_bytes) || (sig_off < data_off + payload_bytes && data_off < sig_off + 8) ||
        2ull * npairs > (uint64_t)st().npes) {
        set_last_error(SHMEMX_ERR_ARG);
        return SHMEMX_ERR_ARG;
    }
    // Signal values carry a per-call tag so stale values from earlier calls
    // never satisfy a wait.
    const uint64_t tag = (g_pingpong_calls.fetch_add(1) & 0xFFFFFFFFull) << 32;
    const unsigned grid = same_xcd ? (unsigned)(((npairs + 7) / 8) * 16) : (unsigned)(2 * npairs);
    if (int rc = check_coresident(k_pingpong, grid, 64, "pingpong")) {
        set_last_error(rc);
        return rc;
    }
    hipLaunchKernelGGL(k_pingpong, dim3(grid), dim3(64), 0, (hipStream_t)stream, pub(), data_off, sig_off, pairs,
                       npairs, rounds, payload_bytes, same_xcd, tag, rtt_cycles);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_wait_until_launch(int pe, uint64_t ivar_off, int cmp, uint64_t value, int is_unsigned, uint64_t *out,
                             void *stream)
{
    if (int rc = check_ready()) return rc;
    if (pe < 0 || pe >= st().npes || cmp < 0 || cmp > SHMEM_CMP_LE || (ivar_off & 7) || !in_user_heap(ivar_off, 8)) {
        set_last_error(SHMEMX_ERR_ARG);
        return SHMEMX_ERR_ARG;
    }
    hipLaunchKernelGGL(k_wait_until, dim3(1), dim3(64), 0, (hipStream_t)stream, pub(), pe, ivar_off, cmp, value,
                       is_unsigned, out);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_barrier_launch(shmem_team_t team, int iters, uint64_t tokens_off, uint64_t *bad, uint64_t *cycles,
                          void *stream)
{
    if (int rc = check_ready()) return rc;
    shmemx_dteam_t t;
    if (team_get(team, &t) != SHMEMX_OK || iters < 0 ||
        (tokens_off != UINT64_MAX && ((tokens_off & 7) || !in_user_heap(tokens_off, 16ull * t.size)))) {
        set_last_error(SHMEMX_ERR_ARG);
        return SHMEMX_ERR_ARG;
    }
    if (int rc = check_coresident(k_barrier, t.size, 256, "barrier")) return rc;
    hipLaunchKernelGGL(k_barrier, dim3(t.size), dim3(256), 0, (hipStream_t)stream, pub(), t, iters, tokens_off, bad,
                       cycles);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

}  // extern "C"
