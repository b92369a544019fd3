// Device-initiated put/get traffic patterns, the seeded payload fill, and the
// probes that supply measured ceilings (copy bandwidth, atomic rate, launch
// latency, XCD placement).
#include "runtime.hpp"

using namespace vshmem;

namespace {

// Thread-scope messages of m <= 2 elements of V each (addresses, size and
// steps all multiples of sizeof(V)), one lane per message: the lane loads
// four messages before it stores any of them, as a run of non-blocking puts
// may, so that their round trips overlap instead of following one another.
// (Messages of three or four vectors measured slower this way than one at a
// time.)  Returns the first message index it did not move.
template <typename V, bool NT>
__device__ __forceinline__ uint64_t copy_msgs4(uint8_t *D, const uint8_t *S, uint32_t m, uint64_t sstep,
                                               uint64_t dstep, uint64_t j, uint64_t nmsg, uint64_t nl)
{
    constexpr int G = 4;
    for (; j + (G - 1) * nl < nmsg; j += G * nl) {
        V r[G][2];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const V *s = (const V *)(S + (j + g * nl) * sstep);
            r[g][0] = vshmem_detail::ld<NT>(s);
            if (m > 1) r[g][1] = vshmem_detail::ld<NT>(s + 1);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            V *d = (V *)(D + (j + g * nl) * dstep);
            vshmem_detail::st<NT>(d, r[g][0]);
            if (m > 1) vshmem_detail::st<NT>(d + 1, r[g][1]);
        }
    }
    return j;
}

// Every virtual PE p issues nmsg messages to targets[p] at the given scope,
// then quiets.  Work-group w acts for PE w / wgs_per_pe.  MAXT is the
// largest work-group the instance accepts: launches of at most 256 threads
// take an instance compiled for that size, whose register budget (up to 512
// per lane) holds the 8-deep grid-scope body without spilling; under the
// 1024-thread bound the same body needs 60 bytes of scratch per lane.
template <int SCOPE, bool IS_PUT, bool NT, int U, int MAXT>
__global__ void __launch_bounds__(MAXT) k_rma_pattern(shmemx_dctx_pub_t c, const int32_t *__restrict__ targets,
                                                      uint64_t src_off, uint64_t dst_off, uint64_t msg, uint64_t nmsg,
                                                      uint64_t sstep, uint64_t dstep, int wgs_per_pe)
{
    const int pe = blockIdx.x / wgs_per_pe;
    const int rank = blockIdx.x - pe * wgs_per_pe;
    const int tgt = targets[pe];
    if (tgt < 0) return;
    // Source and destination PE of every message of this PE.
    const int spe = IS_PUT ? pe : tgt;
    const int dpe = IS_PUT ? tgt : pe;
    const uint8_t *S = c.base + (uint64_t)spe * c.stride + src_off;
    uint8_t *D = c.base + (uint64_t)dpe * c.stride + dst_off;
    if constexpr (SCOPE == SHMEMX_SCOPE_THREAD) {
        const uint64_t nl = (uint64_t)wgs_per_pe * blockDim.x;
        uint64_t j = (uint64_t)rank * blockDim.x + threadIdx.x;
        const uint64_t al = (uintptr_t)S | (uintptr_t)D | msg | sstep | dstep;
        if (msg <= 32 && (al & 15) == 0)
            j = copy_msgs4<vshmem_detail::v4u, NT>(D, S, (uint32_t)(msg / 16), sstep, dstep, j, nmsg, nl);
        else if (msg <= 16 && (al & 7) == 0)
            j = copy_msgs4<uint64_t, NT>(D, S, (uint32_t)(msg / 8), sstep, dstep, j, nmsg, nl);
        for (; j < nmsg; j += nl) vshmem_detail::copy_bytes<U, NT, false, true>(D + j * dstep, S + j * sstep, msg, 0, 1);
    } else if constexpr (SCOPE == SHMEMX_SCOPE_WAVE) {
        const uint64_t waves = blockDim.x / 64;
        const uint64_t nw = (uint64_t)wgs_per_pe * waves;
        for (uint64_t j = (uint64_t)rank * waves + threadIdx.x / 64; j < nmsg; j += nw)
            vshmem_detail::copy_bytes<U, NT>(D + j * dstep, S + j * sstep, msg, __lane_id(), 64);
    } else if constexpr (SCOPE == SHMEMX_SCOPE_WG) {
        for (uint64_t j = rank; j < nmsg; j += wgs_per_pe)
            vshmem_detail::copy_bytes<U, NT>(D + j * dstep, S + j * sstep, msg, threadIdx.x, blockDim.x);
    } else {
        const uint64_t lane = (uint64_t)rank * blockDim.x + threadIdx.x;
        const uint64_t nl = (uint64_t)wgs_per_pe * blockDim.x;
        for (uint64_t j = 0; j < nmsg; ++j)
            vshmem_detail::copy_bytes<U, NT>(D + j * dstep, S + j * sstep, msg, lane, nl);
    }
    vshmem_detail::release_wg_at_exit();   // quiet
}

template <int SCOPE, bool IS_PUT>
void launch_pattern(int flags, int grid, int wg, hipStream_t s, const shmemx_dctx_pub_t &c, const int32_t *targets,
                    uint64_t so, uint64_t d, uint64_t m, uint64_t n, uint64_t ss, uint64_t ds, int wgs)
{
    const bool nt = (flags & SHMEMX_LAUNCH_NONTEMPORAL) != 0, deep = (flags & SHMEMX_LAUNCH_DEEP) != 0;
#define VSHMEM_PAT_K(NT, U)                                                                                        \
    do {                                                                                                           \
        if (wg <= 256)                                                                                             \
            hipLaunchKernelGGL((k_rma_pattern<SCOPE, IS_PUT, NT, U, 256>), dim3(grid), dim3(wg), 0, s, c, targets, so, \
                               d, m, n, ss, ds, wgs);                                                              \
        else                                                                                                       \
            hipLaunchKernelGGL((k_rma_pattern<SCOPE, IS_PUT, NT, U, 1024>), dim3(grid), dim3(wg), 0, s, c, targets,    \
                               so, d, m, n, ss, ds, wgs);                                                          \
    } while (0)
    if (nt && deep) VSHMEM_PAT_K(true, 8);
    else if (nt) VSHMEM_PAT_K(true, 4);
    else if (deep) VSHMEM_PAT_K(false, 8);
    else VSHMEM_PAT_K(false, 4);
#undef VSHMEM_PAT_K
}

// ---------------------------------------------------------------- fill
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_fill_random(uint8_t *dst, uint64_t nbytes, uint64_t seed, uint64_t word0)
{
    const uint64_t nw = nbytes / 8;
    uint64_t *d = (uint64_t *)dst;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += (uint64_t)gridDim.x * blockDim.x)
        d[i] = splitmix_at(seed, word0 + i);
    if (blockIdx.x == 0 && threadIdx.x < (nbytes & 7)) {
        uint64_t w = splitmix_at(seed, word0 + nw);
        dst[nw * 8 + threadIdx.x] = (uint8_t)(w >> (8 * threadIdx.x));
    }
}

__global__ void k_fill_typed(uint8_t *dst, uint64_t count, int dtype, uint64_t seed, uint64_t index0)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = splitmix_at(seed, index0 + i);
        if (dtype == SHMEMX_DT_INT64) {
            ((uint64_t *)dst)[i] = x;
        } else {
            const float f = (float)((double)(x >> 40) * 0x1.0p-24 * 2.0 - 1.0);
            if (dtype == SHMEMX_DT_FP32) {
                ((float *)dst)[i] = f;
            } else {
                const uint32_t u = __float_as_uint(f);
                ((uint16_t *)dst)[i] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
            }
        }
    }
}

// --------------------------------------------------------------- probes
// Achievable-copy probe in the shape that measured fastest on MI355X: each
// work-group streams contiguous chunks of `cv` vectors (dealt round robin),
// nontemporal loads and stores, 8 vectors in flight per lane.
__global__ void __launch_bounds__(1024) k_probe_copy(vshmem_detail::v4u *__restrict__ d,
                                                     const vshmem_detail::v4u *__restrict__ s, uint64_t nv,
                                                     uint64_t cv)
{
    const uint64_t nch = (nv + cv - 1) / cv;
    for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const uint64_t b = c * cv;
        const uint64_t n = min(cv, nv - b);
        vshmem_detail::copy_body<vshmem_detail::v4u, 8, true>(d + b, s + b, n, threadIdx.x, blockDim.x);
    }
}

__global__ void k_probe_atomics(uint64_t *table, uint64_t mask, uint64_t nupd, uint64_t seed, uint64_t *acc)
{
    uint64_t x = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < nupd; u += (uint64_t)gridDim.x * blockDim.x)
        x ^= __hip_atomic_fetch_add(table + (splitmix_at(seed, u) & mask), 1ull, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    if (acc && x) __hip_atomic_fetch_xor(acc, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_probe_xcd(int32_t *out, int n)
{
    if (threadIdx.x == 0 && (int)blockIdx.x < n) {
        // XCC_ID hardware register (id 20), bits [3:0].
        uint32_t v = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
        out[blockIdx.x] = (int32_t)(v & 0xf);
    }
}

__global__ void k_probe_empty() {}

}  // namespace

extern "C" {

int shmemx_rma_pattern(int op, int scope, const int32_t *targets, uint64_t src_off, uint64_t dst_off,
                       uint64_t msg_bytes, uint64_t nmsg, uint64_t src_step, uint64_t dst_step,
                       const shmemx_launch_t *launch, void *stream)
{
    if (int rc = check_ready()) return rc;
    shmemx_launch_t tmp;
    const shmemx_launch_t &L = launch_or_default(launch, tmp, 4, 256, 0);
    const State &s = st();
    bool ok = (op == SHMEMX_OP_PUT || op == SHMEMX_OP_GET) && scope >= 0 && scope <= SHMEMX_SCOPE_GRID && targets &&
              valid_wg_size(L.wg_size) && L.wgs_per_pe > 0 && (uint64_t)L.wgs_per_pe * s.npes <= (1ull << 31);
    if (ok && nmsg > 0) {
        uint64_t last = nmsg - 1;
        ok = (src_step == 0 || last <= UINT64_MAX / src_step) && (dst_step == 0 || last <= UINT64_MAX / dst_step) &&
             in_user_heap(src_off, last * src_step) && in_user_heap(src_off + last * src_step, msg_bytes) &&
             in_user_heap(dst_off, last * dst_step) && in_user_heap(dst_off + last * dst_step, msg_bytes) &&
             (nmsg == 1 || dst_step >= msg_bytes);
    }
    if (!ok) {
        set_last_error(SHMEMX_ERR_ARG);
        return SHMEMX_ERR_ARG;
    }
    if (nmsg == 0 || msg_bytes == 0) return SHMEMX_OK;
    const int grid = L.wgs_per_pe * s.npes;
    hipStream_t hs = (hipStream_t)stream;
    shmemx_dctx_pub_t c = pub();
#define VSHMEM_PAT(SC)                                                                                        \
    if (op == SHMEMX_OP_PUT)                                                                                  \
        launch_pattern<SC, true>(L.flags, grid, L.wg_size, hs, c, targets, src_off, dst_off, msg_bytes, nmsg, src_step, \
                                 dst_step, L.wgs_per_pe);                                                     \
    else                                                                                                      \
        launch_pattern<SC, false>(L.flags, grid, L.wg_size, hs, c, targets, src_off, dst_off, msg_bytes, nmsg, src_step, \
                                  dst_step, L.wgs_per_pe);
    switch (scope) {
    case SHMEMX_SCOPE_THREAD: VSHMEM_PAT(SHMEMX_SCOPE_THREAD) break;
    case SHMEMX_SCOPE_WAVE: VSHMEM_PAT(SHMEMX_SCOPE_WAVE) break;
    case SHMEMX_SCOPE_WG: VSHMEM_PAT(SHMEMX_SCOPE_WG) break;
    default: VSHMEM_PAT(SHMEMX_SCOPE_GRID) break;
    }
#undef VSHMEM_PAT
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_fill_random(void *dst, uint64_t nbytes, uint64_t seed, uint64_t word_offset, void *stream)
{
    if (!dst && nbytes) return SHMEMX_ERR_ARG;
    if (nbytes == 0) return SHMEMX_OK;
    uint64_t nw = nbytes / 8 + 1;
    uint64_t grid = (nw + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_fill_random, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, (uint8_t *)dst, nbytes,
                       seed, word_offset);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_fill_typed(void *dst, uint64_t count, int dtype, uint64_t seed, uint64_t index0, void *stream)
{
    const uint64_t es = dtype == SHMEMX_DT_INT64 ? 8 : dtype == SHMEMX_DT_FP32 ? 4 : 2;
    if (dtype < SHMEMX_DT_INT64 || dtype > SHMEMX_DT_BF16 || (!dst && count) || ((uintptr_t)dst % es))
        return SHMEMX_ERR_ARG;
    if (count == 0) return SHMEMX_OK;
    uint64_t grid = (count + 255) / 256;
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL(k_fill_typed, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, (uint8_t *)dst, count,
                       dtype, seed, index0);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_probe_copy(void *dst, const void *src, uint64_t nbytes, int nwg, int wg_size, void *stream)
{
    if (!dst || !src || (nbytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15) || nwg <= 0 ||
        !valid_wg_size(wg_size))
        return SHMEMX_ERR_ARG;
    hipLaunchKernelGGL(k_probe_copy, dim3(nwg), dim3(wg_size), 0, (hipStream_t)stream, (vshmem_detail::v4u *)dst,
                       (const vshmem_detail::v4u *)src, nbytes / 16, (uint64_t)(16u << 20) / 16);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_probe_atomics(uint64_t *table, uint64_t nwords, uint64_t nupdates, uint64_t seed, uint64_t *acc, void *stream)
{
    if (!table || nwords == 0 || (nwords & (nwords - 1))) return SHMEMX_ERR_ARG;
    hipLaunchKernelGGL(k_probe_atomics, dim3(4096), dim3(256), 0, (hipStream_t)stream, table, nwords - 1, nupdates,
                       seed, acc);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_probe_xcd(int32_t *out, int nblocks, void *stream)
{
    if (!out || nblocks <= 0) return SHMEMX_ERR_ARG;
    hipLaunchKernelGGL(k_probe_xcd, dim3(nblocks), dim3(64), 0, (hipStream_t)stream, out, nblocks);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_probe_empty(void *stream)
{
    hipLaunchKernelGGL(k_probe_empty, dim3(1), dim3(64), 0, (hipStream_t)stream);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

}  // extern "C"
