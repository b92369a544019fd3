// HBM probes: the rates that bound the copy-shaped rows.  A copy moves each
// byte twice through HBM (read, then write); these kernels measure a copy
// under three work schedules, a read-only stream and a write-only stream,
// so that the copy's rate can be set against the read and write rates the
// memory itself reaches.
#include "runtime.hpp"

using namespace vshmem;
using vshmem_detail::v4u;

namespace {

constexpr int kU = 8;   // 16-byte vectors in flight per lane

// Grid-stride copy: the whole grid sweeps the buffer, lane l of the grid
// taking vectors l, l + nl, ...
__global__ void __launch_bounds__(1024) k_probe_copy_gridstride(v4u *__restrict__ d, const v4u *__restrict__ s,
                                                                uint64_t nv)
{
    const uint64_t nl = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kU - 1) * nl < nv; i += kU * nl) {
        v4u r[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) r[u] = __builtin_nontemporal_load(s + i + u * nl);
#pragma unroll
        for (int u = 0; u < kU; ++u) __builtin_nontemporal_store(r[u], d + i + u * nl);
    }
    for (; i < nv; i += nl) __builtin_nontemporal_store(__builtin_nontemporal_load(s + i), d + i);
}

// Tile copy: tiles of kU * blockDim vectors dealt to work-groups round
// robin (the grid moves through one window of tiles at a time).
__global__ void __launch_bounds__(1024) k_probe_copy_tiles(v4u *__restrict__ d, const v4u *__restrict__ s, uint64_t nv)
{
    const uint64_t nl = blockDim.x, T = kU * nl, nt = (nv + T - 1) / T;
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const uint64_t b = t * T + threadIdx.x;
        v4u r[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (b + u * nl < nv) r[u] = __builtin_nontemporal_load(s + b + u * nl);
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (b + u * nl < nv) __builtin_nontemporal_store(r[u], d + b + u * nl);
    }
}

// Read-only stream in 16 MiB chunks per work-group; the loaded words are
// folded into *acc so the loads stay.
__global__ void __launch_bounds__(1024) k_probe_read(const v4u *__restrict__ s, uint64_t nv, uint64_t cv, uint32_t *acc)
{
    const uint64_t nch = (nv + cv - 1) / cv, nl = blockDim.x;
    uint32_t x = 0;
    for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const uint64_t b = c * cv, n = min(cv, nv - b);
        uint64_t i = threadIdx.x;
        for (; i + (kU - 1) * nl < n; i += kU * nl) {
            v4u r[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) r[u] = __builtin_nontemporal_load(s + b + i + u * nl);
#pragma unroll
            for (int u = 0; u < kU; ++u) x ^= r[u].x ^ r[u].y ^ r[u].z ^ r[u].w;
        }
        for (; i < n; i += nl) {
            const v4u r = __builtin_nontemporal_load(s + b + i);
            x ^= r.x ^ r.y ^ r.z ^ r.w;
        }
    }
    if (x) __hip_atomic_fetch_xor(acc, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Write-only stream in 16 MiB chunks per work-group (temporal stores: the
// faster kind for pure writes on MI355X).
__global__ void __launch_bounds__(1024) k_probe_write(v4u *__restrict__ d, uint64_t nv, uint64_t cv)
{
    const uint64_t nch = (nv + cv - 1) / cv, nl = blockDim.x;
    for (uint64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const uint64_t b = c * cv, n = min(cv, nv - b);
        for (uint64_t i = threadIdx.x; i < n; i += nl) {
            const v4u v = {(uint32_t)(b + i), (uint32_t)c, 0x5A5A5A5Au, 0xA5A5A5A5u};
            d[b + i] = v;
        }
    }
}

}  // namespace

extern "C" {

int shmemx_probe_hbm(int kind, void *dst, const void *src, uint64_t nbytes, int nwg, int wg_size, uint32_t *acc,
                     void *stream)
{
    if (nbytes == 0 || (nbytes & 15) || nwg <= 0 || !valid_wg_size(wg_size)) return SHMEMX_ERR_ARG;
    const bool reads = kind != SHMEMX_PROBE_WRITE, writes = kind != SHMEMX_PROBE_READ;
    if ((reads && (!src || ((uintptr_t)src & 15))) || (writes && (!dst || ((uintptr_t)dst & 15))) ||
        (kind == SHMEMX_PROBE_READ && !acc))
        return SHMEMX_ERR_ARG;
    const uint64_t nv = nbytes / 16, cv = (16ull << 20) / 16;
    hipStream_t s = (hipStream_t)stream;
    switch (kind) {
    case SHMEMX_PROBE_COPY_CHUNKED: return shmemx_probe_copy(dst, src, nbytes, nwg, wg_size, stream);
    case SHMEMX_PROBE_COPY_GRIDSTRIDE:
        hipLaunchKernelGGL(k_probe_copy_gridstride, dim3(nwg), dim3(wg_size), 0, s, (v4u *)dst, (const v4u *)src, nv);
        break;
    case SHMEMX_PROBE_COPY_TILES:
        hipLaunchKernelGGL(k_probe_copy_tiles, dim3(nwg), dim3(wg_size), 0, s, (v4u *)dst, (const v4u *)src, nv);
        break;
    case SHMEMX_PROBE_READ:
        hipLaunchKernelGGL(k_probe_read, dim3(nwg), dim3(wg_size), 0, s, (const v4u *)src, nv, cv, acc);
        break;
    case SHMEMX_PROBE_WRITE:
        hipLaunchKernelGGL(k_probe_write, dim3(nwg), dim3(wg_size), 0, s, (v4u *)dst, nv, cv);
        break;
    default: return SHMEMX_ERR_ARG;
    }
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

}  // extern "C"
