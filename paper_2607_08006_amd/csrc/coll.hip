// Team collectives executed by the work-groups of every team member:
// broadcast, fcollect, alltoall and reductions to all (sum, max) over int64,
// fp32 and bf16 with fp32 accumulation, in the fixed TREE order.
#include <algorithm>
#include <cstdio>

#include "runtime.hpp"

using namespace vshmem;

namespace {

using vshmem_detail::v4u;

struct Geo {
    shmemx_dctx_pub_t c;
    shmemx_dteam_t team;
    uint64_t dst_off, src_off;
    uint64_t n;          // bytes per block (elements for reduce)
    uint64_t chunk;      // bytes per task
    int wgs_per_pe;
};

__device__ __forceinline__ uint8_t *pe_addr(const Geo &g, int k, uint64_t off)
{
    return g.c.base + (uint64_t)shmemx_team_pe(g.team, k) * g.c.stride + off;
}

__device__ __forceinline__ void enter(const Geo &g, shmem_dctx_t &ctx)
{
    ctx = shmemx_dctx_bind(g.c, shmemx_team_pe(g.team, blockIdx.x / g.wgs_per_pe));
    shmemx_team_sync_units(ctx, g.team, g.wgs_per_pe);
}

// Copy one source range to the same offset on every team member (member
// stride in bytes = pstride).  Aligned ranges go through a register tile:
// each lane loads kMcastTile 16-byte vectors once, then the whole tile is
// written to one member after another, starting at a member that depends on
// the work-group so that concurrent work-groups spread over the members.
// Long contiguous writes per member page measured about 10% faster on
// MI355X than writing every vector to all members in turn.
constexpr int kMcastTile = 16;

template <bool NT>
__device__ __forceinline__ void multicast(const Geo &g, const uint8_t *src, uint64_t dst_off, uint64_t len)
{
    const int P = g.team.size;
    const uint64_t pstride = (uint64_t)g.team.stride * g.c.stride;
    uint8_t *d0 = pe_addr(g, 0, dst_off);
    if ((((uintptr_t)src | (uintptr_t)d0 | len) & 15) == 0) {
        const v4u *s = (const v4u *)src;
        const uint64_t nv = len / 16, bd = blockDim.x;
        for (uint64_t i0 = threadIdx.x; i0 < nv; i0 += kMcastTile * bd) {
            v4u r[kMcastTile];
#pragma unroll
            for (int u = 0; u < kMcastTile; ++u)
                if (i0 + u * bd < nv) r[u] = vshmem_detail::ld<true>(s + i0 + u * bd);
            int p = (int)(blockIdx.x % (unsigned)P);
            for (int k = 0; k < P; ++k) {
                v4u *d = (v4u *)(d0 + (uint64_t)p * pstride);
#pragma unroll
                for (int u = 0; u < kMcastTile; ++u)
                    if (i0 + u * bd < nv) vshmem_detail::st<NT>(d + i0 + u * bd, r[u]);
                if (++p == P) p = 0;
            }
        }
    } else {
        for (int p = 0; p < P; ++p)
            vshmem_detail::copy_bytes<VSHMEM_COPY_UNROLL, NT>(d0 + p * pstride, src, len, threadIdx.x, blockDim.x);
    }
}

template <bool NT>
__global__ void __launch_bounds__(1024) k_broadcast(Geo g, int root)
{
    shmem_dctx_t ctx;
    enter(g, ctx);
    const uint8_t *S = pe_addr(g, root, g.src_off);
    const uint64_t ntask = (g.n + g.chunk - 1) / g.chunk;
    for (uint64_t t = blockIdx.x; t < ntask; t += gridDim.x) {
        const uint64_t off = t * g.chunk;
        const uint64_t len = min(g.chunk, g.n - off);
        multicast<NT>(g, S + off, g.dst_off + off, len);
    }
    shmemx_team_sync_units(ctx, g.team, g.wgs_per_pe);
}

template <bool NT>
__global__ void __launch_bounds__(1024) k_fcollect(Geo g)
{
    shmem_dctx_t ctx;
    enter(g, ctx);
    const uint64_t nch = (g.n + g.chunk - 1) / g.chunk;
    const uint64_t ntask = nch * g.team.size;
    for (uint64_t t = blockIdx.x; t < ntask; t += gridDim.x) {
        const int q = (int)(t / nch);
        const uint64_t off = (t - (uint64_t)q * nch) * g.chunk;
        const uint64_t len = min(g.chunk, g.n - off);
        multicast<NT>(g, pe_addr(g, q, g.src_off) + off, g.dst_off + (uint64_t)q * g.n + off, len);
    }
    shmemx_team_sync_units(ctx, g.team, g.wgs_per_pe);
}

template <bool NT, int U>
__global__ void __launch_bounds__(1024) k_alltoall(Geo g)
{
    shmem_dctx_t ctx;
    enter(g, ctx);
    const int P = g.team.size;
    const uint64_t nch = (g.n + g.chunk - 1) / g.chunk;
    const uint64_t ntask = nch * (uint64_t)P * P;
    for (uint64_t t = blockIdx.x; t < ntask; t += gridDim.x) {
        const uint64_t blk = t / nch;
        const int p = (int)(blk / P);   // destination member
        const int q = (int)(blk % P);   // source member
        const uint64_t off = (t - blk * nch) * g.chunk;
        const uint64_t len = min(g.chunk, g.n - off);
        vshmem_detail::copy_bytes<U, NT>(pe_addr(g, p, g.dst_off + (uint64_t)q * g.n + off),
                                                          pe_addr(g, q, g.src_off + (uint64_t)p * g.n + off), len,
                                                          threadIdx.x, blockDim.x);
    }
    shmemx_team_sync_units(ctx, g.team, g.wgs_per_pe);
}

// ------------------------------------------------------------ reductions
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

template <typename A, int E, class OP, int LEVELS = 9>
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

constexpr int kRedBatch = 8;   // loads in flight per lane before they are combined

template <class CODEC, class OP, bool NT>
__global__ void __launch_bounds__(256) k_reduce(Geo g)
{
    using A = typename CODEC::A;
    constexpr int E = CODEC::E;
    shmem_dctx_t ctx;
    enter(g, ctx);
    const int P = g.team.size;
    const uint64_t pstride = (uint64_t)g.team.stride * g.c.stride;
    const uint8_t *s0 = pe_addr(g, 0, g.src_off);
    uint8_t *d0 = pe_addr(g, 0, g.dst_off);
    const uint64_t nbytes = g.n * CODEC::ES;
    const bool vec = (((uintptr_t)s0 | (uintptr_t)d0 | pstride) & 15) == 0;
    const uint64_t nvec = vec ? nbytes / 16 : 0;
    const uint64_t vpt = g.chunk / 16;               // vectors per task
    const uint64_t ntask = (nvec + vpt - 1) / vpt;
    for (uint64_t t = blockIdx.x; t < ntask; t += gridDim.x) {
        const uint64_t v1 = min(nvec, (t + 1) * vpt);
        for (uint64_t i = t * vpt + threadIdx.x; i < v1; i += blockDim.x) {
            TreeAcc<A, E, OP> acc;
            const uint8_t *sp = s0 + i * 16;
            for (int p0 = 0; p0 < P; p0 += kRedBatch) {
                v4u raw[kRedBatch];
#pragma unroll
                for (int u = 0; u < kRedBatch; ++u)
                    if (p0 + u < P) raw[u] = vshmem_detail::ld<NT>((const v4u *)(sp + (uint64_t)(p0 + u) * pstride));
#pragma unroll
                for (int u = 0; u < kRedBatch; ++u) {
                    if (p0 + u < P) {
                        A x[E];
                        CODEC::unpack(raw[u], x);
                        acc.push((uint32_t)(p0 + u), x);
                    }
                }
            }
            A r[E];
            acc.result((uint32_t)P, r);
            const v4u out = CODEC::pack(r);
            uint8_t *dp = d0 + i * 16;
            for (int p = 0; p < P; ++p, dp += pstride) vshmem_detail::st<NT>((v4u *)dp, out);
        }
    }
    // Elements past the vector part (or all of them when unaligned).
    const uint64_t e0 = nvec * 16 / CODEC::ES;
    for (uint64_t k = e0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < g.n;
         k += (uint64_t)gridDim.x * blockDim.x) {
        TreeAcc<A, 1, OP> acc;
        for (int p = 0; p < P; ++p) {
            A x[1] = {CODEC::load1(s0 + (uint64_t)p * pstride + k * CODEC::ES)};
            acc.push((uint32_t)p, x);
        }
        A r[1];
        acc.result((uint32_t)P, r);
        for (int p = 0; p < P; ++p) CODEC::store1(d0 + (uint64_t)p * pstride + k * CODEC::ES, r[0]);
    }
    shmemx_team_sync_units(ctx, g.team, g.wgs_per_pe);
}

// ------------------------------------------------------------- launching
template <typename K>
int check_coresident(K kernel, int grid, int wg)
{
    int per_cu = 0;
    if (int rc = blocks_per_cu(kernel, wg, &per_cu)) return rc;
    if ((int64_t)per_cu * st().num_cus < grid) {
        set_error_detail(SHMEMX_ERR_ARG, "%d work-groups of %d threads cannot be co-resident (%d per CU x %d CUs)", grid,
                         wg, per_cu, st().num_cus);
        if (st().debug) fprintf(stderr, "vshmem: %s\n", "collective work-groups cannot be co-resident");
        return SHMEMX_ERR_ARG;
    }
    return SHMEMX_OK;
}

// Launch a kernel whose work-groups synchronise with each other.  When the
// caller left wgs_per_pe at 0, fill the device: as many work-groups per
// member as stay co-resident (at most 16).
template <typename K, typename... Args>
int launch_team_kernel(K kernel, Geo &g, int wg, hipStream_t s, bool auto_wgs, Args... args)
{
    if (auto_wgs) {
        // About one work-group per CU: in measurements on MI355X, streaming
        // kernels reached higher HBM bandwidth with one wide work-group per
        // CU than with the grid filled to its occupancy limit.
        int per_cu = 0;
        if (int rc = blocks_per_cu(kernel, wg, &per_cu)) return rc;
        const int64_t cap = (int64_t)per_cu * st().num_cus;
        const int64_t want = std::max<int64_t>(1, st().num_cus / g.team.size);
        g.wgs_per_pe = (int)std::max<int64_t>(1, std::min<int64_t>(want, cap / g.team.size));
    }
    const int grid = g.wgs_per_pe * g.team.size;
    if (int rc = check_coresident(kernel, grid, wg)) return rc;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(wg), 0, s, g, args...);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int make_geo(shmem_team_t team, const void *dest, const void *src, uint64_t dst_bytes, uint64_t src_bytes,
             const shmemx_launch_t *launch, int def_wg, Geo &g, shmemx_launch_t &L, uint64_t def_chunk = 256ull << 10,
             int def_flags = 0)
{
    if (int rc = check_ready()) return rc;
    if (team_get(team, &g.team) != SHMEMX_OK) return SHMEMX_ERR_ARG;
    launch_or_default(launch, L, 1, def_wg, def_chunk);
    if (!launch) L.flags = def_flags;
    if (launch && launch->wgs_per_pe < 0) return SHMEMX_ERR_ARG;
    if (!valid_wg_size(L.wg_size) || (L.chunk_bytes & 15) || (int64_t)L.wgs_per_pe * g.team.size > (1 << 24))
        return SHMEMX_ERR_ARG;
    g.dst_off = sym_offset(dest, dst_bytes);
    g.src_off = sym_offset(src, src_bytes);
    if (g.dst_off == UINT64_MAX || g.src_off == UINT64_MAX) return SHMEMX_ERR_ARG;
    g.c = pub();
    g.chunk = L.chunk_bytes;
    g.wgs_per_pe = L.wgs_per_pe;
    return SHMEMX_OK;
}

bool overlap(uint64_t a, uint64_t an, uint64_t b, uint64_t bn) { return a < b + bn && b < a + an; }

}  // namespace

extern "C" {

int shmemx_broadcastmem_launch(shmem_team_t team, void *dest, const void *src, size_t n, int root,
                               const shmemx_launch_t *launch, void *stream)
{
    Geo g{};
    shmemx_launch_t L;
    int rc = make_geo(team, dest, src, n, n, launch, 1024, g, L);
    if (!rc && (root < 0 || root >= g.team.size || overlap(g.dst_off, n, g.src_off, n))) rc = SHMEMX_ERR_ARG;
    if (rc) {
        set_last_error(rc);
        return rc;
    }
    g.n = n;
    const bool aw = !launch || launch->wgs_per_pe == 0;
    if (L.flags & SHMEMX_LAUNCH_NONTEMPORAL)
        return launch_team_kernel(k_broadcast<true>, g, L.wg_size, (hipStream_t)stream, aw, root);
    return launch_team_kernel(k_broadcast<false>, g, L.wg_size, (hipStream_t)stream, aw, root);
}

int shmemx_fcollectmem_launch(shmem_team_t team, void *dest, const void *src, size_t n, const shmemx_launch_t *launch,
                              void *stream)
{
    Geo g{};
    shmemx_launch_t L;
    int rc = SHMEMX_OK;
    if (int r0 = check_ready()) return r0;
    int tsize = shmem_team_n_pes(team);
    if (tsize <= 0) rc = SHMEMX_ERR_ARG;
    if (!rc) rc = make_geo(team, dest, src, (uint64_t)n * tsize, n, launch, 1024, g, L);
    if (!rc && overlap(g.dst_off, (uint64_t)n * tsize, g.src_off, n)) rc = SHMEMX_ERR_ARG;
    if (rc) {
        set_last_error(rc);
        return rc;
    }
    g.n = n;
    const bool aw = !launch || launch->wgs_per_pe == 0;
    if (L.flags & SHMEMX_LAUNCH_NONTEMPORAL)
        return launch_team_kernel(k_fcollect<true>, g, L.wg_size, (hipStream_t)stream, aw);
    return launch_team_kernel(k_fcollect<false>, g, L.wg_size, (hipStream_t)stream, aw);
}

int shmemx_alltoallmem_launch(shmem_team_t team, void *dest, const void *src, size_t n, const shmemx_launch_t *launch,
                              void *stream)
{
    Geo g{};
    shmemx_launch_t L;
    if (int r0 = check_ready()) return r0;
    int tsize = shmem_team_n_pes(team);
    int rc = tsize <= 0 ? SHMEMX_ERR_ARG : SHMEMX_OK;
    if (!rc)
        rc = make_geo(team, dest, src, (uint64_t)n * tsize, (uint64_t)n * tsize, launch, 1024, g, L, 256ull << 10,
                      SHMEMX_LAUNCH_NONTEMPORAL | SHMEMX_LAUNCH_DEEP);
    if (!rc && overlap(g.dst_off, (uint64_t)n * tsize, g.src_off, (uint64_t)n * tsize)) rc = SHMEMX_ERR_ARG;
    if (rc) {
        set_last_error(rc);
        return rc;
    }
    g.n = n;
    const bool aw = !launch || launch->wgs_per_pe == 0;
    const bool nt = (L.flags & SHMEMX_LAUNCH_NONTEMPORAL) != 0, deep = (L.flags & SHMEMX_LAUNCH_DEEP) != 0;
    hipStream_t hs = (hipStream_t)stream;
    if (nt && deep) return launch_team_kernel(k_alltoall<true, 8>, g, L.wg_size, hs, aw);
    if (nt) return launch_team_kernel(k_alltoall<true, 4>, g, L.wg_size, hs, aw);
    if (deep) return launch_team_kernel(k_alltoall<false, 8>, g, L.wg_size, hs, aw);
    return launch_team_kernel(k_alltoall<false, 4>, g, L.wg_size, hs, aw);
}

int shmemx_reduce_launch(shmem_team_t team, int dtype, int op, void *dest, const void *src, size_t nreduce,
                         const shmemx_launch_t *launch, void *stream)
{
    Geo g{};
    shmemx_launch_t L;
    const uint64_t es = dtype == SHMEMX_DT_INT64 ? 8 : dtype == SHMEMX_DT_FP32 ? 4 : 2;
    int rc = (dtype < SHMEMX_DT_INT64 || dtype > SHMEMX_DT_BF16 || op < SHMEMX_RED_SUM || op > SHMEMX_RED_MAX)
                 ? SHMEMX_ERR_ARG
                 : SHMEMX_OK;
    shmemx_launch_t L0 = launch ? *launch : shmemx_launch_t{0, 256, 16ull << 10, SHMEMX_LAUNCH_NONTEMPORAL, 0};
    if (L0.wg_size == 0) L0.wg_size = 256;
    if (!rc) rc = make_geo(team, dest, src, nreduce * es, nreduce * es, &L0, 256, g, L);
    // In place is allowed; partial overlap is not.
    if (!rc && g.dst_off != g.src_off && overlap(g.dst_off, nreduce * es, g.src_off, nreduce * es)) rc = SHMEMX_ERR_ARG;
    if (!rc && (L.wg_size > 256 || L.chunk_bytes == 0)) rc = SHMEMX_ERR_ARG;
    if (!rc && g.team.size > 511) rc = SHMEMX_ERR_UNSUPPORTED;   // TreeAcc holds 9 levels
    if (rc) {
        set_last_error(rc);
        return rc;
    }
    g.n = nreduce;
    const bool aw = !launch || launch->wgs_per_pe == 0;
    hipStream_t s = (hipStream_t)stream;
    const bool nt = (L.flags & SHMEMX_LAUNCH_NONTEMPORAL) != 0;
#define VSHMEM_RED(CODEC)                                                                                   \
    if (op == SHMEMX_RED_SUM)                                                                               \
        return nt ? launch_team_kernel(k_reduce<CODEC, OpSum, true>, g, L.wg_size, s, aw)                   \
                  : launch_team_kernel(k_reduce<CODEC, OpSum, false>, g, L.wg_size, s, aw);                 \
    return nt ? launch_team_kernel(k_reduce<CODEC, OpMax, true>, g, L.wg_size, s, aw)                       \
              : launch_team_kernel(k_reduce<CODEC, OpMax, false>, g, L.wg_size, s, aw);
    if (dtype == SHMEMX_DT_INT64) {
        VSHMEM_RED(CodecI64)
    } else if (dtype == SHMEMX_DT_FP32) {
        VSHMEM_RED(CodecF32)
    } else {
        VSHMEM_RED(CodecBF16)
    }
#undef VSHMEM_RED
}

}  // extern "C"
