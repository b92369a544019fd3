// Host launchers of the team collectives: broadcast, fcollect, alltoall and
// reductions to all (sum, max) over int64, fp32 and bf16 with fp32
// accumulation, in the fixed TREE order.  The kernels call the device
// collectives of vshmem_device.hpp with launch-chosen task sizes and
// store kinds.
#include <algorithm>
#include <cstdio>

#include "runtime.hpp"

using namespace vshmem;

namespace {

using vshmem_detail::CodecBF16;
using vshmem_detail::CodecF32;
using vshmem_detail::CodecI64;
using vshmem_detail::OpMax;
using vshmem_detail::OpSum;

struct Geo {
    shmemx_dctx_pub_t c;
    shmemx_dteam_t team;
    uint64_t dst_off, src_off;
    uint64_t n;          // bytes per block (elements for reduce)
    uint64_t chunk;      // bytes per task
    int wgs_per_pe;
};

// The library's launches are user kernels of the device collectives: work-
// group b acts for team member b / wgs_per_pe, as its rank b % wgs_per_pe.
struct Caller {
    shmem_dctx_t ctx;
    void *dst;
    const void *src;
    int rank;
};

__device__ __forceinline__ Caller caller(const Geo &g)
{
    const int k = (int)(blockIdx.x / (unsigned)g.wgs_per_pe);
    return Caller{shmemx_dctx_bind(g.c, shmemx_team_pe(g.team, k)), g.c.base + g.dst_off, g.c.base + g.src_off,
                  (int)(blockIdx.x - (unsigned)k * (unsigned)g.wgs_per_pe)};
}

template <bool NT>
__global__ void __launch_bounds__(1024) k_broadcast(Geo g, int root)
{
    const Caller a = caller(g);
    vshmem_detail::broadcast<NT>(a.ctx, g.team, a.dst, a.src, g.n, root, a.rank, g.wgs_per_pe, g.chunk);
}

template <bool NT>
__global__ void __launch_bounds__(1024) k_fcollect(Geo g)
{
    const Caller a = caller(g);
    vshmem_detail::fcollect<NT>(a.ctx, g.team, a.dst, a.src, g.n, a.rank, g.wgs_per_pe, g.chunk);
}

template <bool NT, int U>
__global__ void __launch_bounds__(1024) k_alltoall(Geo g)
{
    const Caller a = caller(g);
    vshmem_detail::alltoall<NT, U>(a.ctx, g.team, a.dst, a.src, g.n, a.rank, g.wgs_per_pe, g.chunk);
}

template <class CODEC, class OP, bool NT>
__global__ void __launch_bounds__(256) k_reduce(Geo g)
{
    const Caller a = caller(g);
    (void)vshmem_detail::reduce<CODEC, OP, NT>(a.ctx, g.team, a.dst, a.src, g.n, a.rank, g.wgs_per_pe, g.chunk);
}

// Two vectors per lane and a TREE stack for teams of up to 127 members.
template <class CODEC, class OP, bool NT>
__global__ void __launch_bounds__(256) k_reduce2(Geo g)
{
    const Caller a = caller(g);
    (void)vshmem_detail::reduce<CODEC, OP, NT, 2, 7>(a.ctx, g.team, a.dst, a.src, g.n, a.rank, g.wgs_per_pe,
                                                      g.chunk);
}

template <class CODEC, class OP, bool NT>
__global__ void __launch_bounds__(64 * vshmem_detail::kRedWaveMax) k_reduce_waves(Geo g)
{
    const Caller a = caller(g);
    vshmem_detail::reduce_waves<CODEC, OP, NT>(a.ctx, g.team, a.dst, a.src, g.n, a.rank, g.wgs_per_pe, g.chunk);
}

// ------------------------------------------------------------- launching
// Bytes a member writes per automatically added work-group: below this a
// second work-group per member costs more in barrier arrivals than it saves
// in copying (64 PEs: alltoall of 4 KiB blocks took 16 us with one
// work-group per member and 25 us with four; 16 KiB blocks 41 us with two,
// 47 with four and 56 with one).
constexpr uint64_t kAutoBytesPerWg = 512ull << 10;

// Launch a kernel whose work-groups synchronise with each other.  When the
// caller left wgs_per_pe at 0, about one work-group per CU over the team,
// fewer when each member writes little (bytes_per_member), and never more
// than stay co-resident.
template <typename K, typename... Args>
int launch_team_kernel(K kernel, Geo &g, int wg, hipStream_t s, bool auto_wgs, uint64_t bytes_per_member,
                       Args... args)
{
    if (auto_wgs) {
        // About one work-group per CU: in measurements on MI355X, streaming
        // kernels reached higher HBM bandwidth with one wide work-group per
        // CU than with the grid filled to its occupancy limit.
        // Only the CUs the progress kernel leaves free count.
        int64_t cap = 0;
        if (int rc = coresident_capacity(kernel, wg, &cap)) return rc;
        const int64_t free_cus = st().num_cus - progress_reserved_cus();
        const uint64_t by_bytes = (bytes_per_member + kAutoBytesPerWg - 1) / kAutoBytesPerWg;
        const int64_t want = std::max<int64_t>(
            1, std::min<int64_t>(free_cus / g.team.size, (int64_t)std::min<uint64_t>(by_bytes, 1u << 20)));
        g.wgs_per_pe = (int)std::max<int64_t>(1, std::min<int64_t>(want, cap / g.team.size));
    }
    const int grid = g.wgs_per_pe * g.team.size;
    if (int rc = check_coresident(kernel, grid, wg, "team collective")) return rc;
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
        return launch_team_kernel(k_broadcast<true>, g, L.wg_size, (hipStream_t)stream, aw, (uint64_t)n, root);
    return launch_team_kernel(k_broadcast<false>, g, L.wg_size, (hipStream_t)stream, aw, (uint64_t)n, root);
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
        return launch_team_kernel(k_fcollect<true>, g, L.wg_size, (hipStream_t)stream, aw, (uint64_t)n * tsize);
    return launch_team_kernel(k_fcollect<false>, g, L.wg_size, (hipStream_t)stream, aw, (uint64_t)n * tsize);
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
    const uint64_t wb = (uint64_t)n * tsize;
    if (nt && deep) return launch_team_kernel(k_alltoall<true, 8>, g, L.wg_size, hs, aw, wb);
    if (nt) return launch_team_kernel(k_alltoall<true, 4>, g, L.wg_size, hs, aw, wb);
    if (deep) return launch_team_kernel(k_alltoall<false, 8>, g, L.wg_size, hs, aw, wb);
    return launch_team_kernel(k_alltoall<false, 4>, g, L.wg_size, hs, aw, wb);
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
    // Work-groups of up to 256 threads: one lane folds every member
    // (k_reduce).  Larger ones (up to 512): the members are split over the
    // wavefronts (k_reduce_waves), for teams of at most 8 members per
    // wavefront.  On MI355X the two measured the same at their best shapes
    // (the split form needs two work-groups per CU to get there), so the
    // default stays with the first.
    shmemx_launch_t L0 = launch ? *launch : shmemx_launch_t{0, 256, 16ull << 10, SHMEMX_LAUNCH_NONTEMPORAL, 0};
    if (L0.wg_size == 0) L0.wg_size = 256;
    if (!rc) rc = make_geo(team, dest, src, nreduce * es, nreduce * es, &L0, 256, g, L);
    // In place is allowed; partial overlap is not.
    if (!rc && g.dst_off != g.src_off && overlap(g.dst_off, nreduce * es, g.src_off, nreduce * es)) rc = SHMEMX_ERR_ARG;
    const bool waves = L.wg_size > 256;
    // SHMEMX_LAUNCH_DEEP: two vectors per lane (teams of up to 127 members).
    const bool two = !waves && (L.flags & SHMEMX_LAUNCH_DEEP) && g.team.size < 128;
    if (!rc && (L.wg_size > 64 * vshmem_detail::kRedWaveMax || L.chunk_bytes == 0 ||
                (waves && g.team.size > 8 * (L.wg_size / 64))))
        rc = SHMEMX_ERR_ARG;
    if (!rc && g.team.size > 511) rc = SHMEMX_ERR_UNSUPPORTED;   // TreeAcc holds 9 levels
    if (rc) {
        set_last_error(rc);
        return rc;
    }
    g.n = nreduce;
    const bool aw = !launch || launch->wgs_per_pe == 0;
    hipStream_t s = (hipStream_t)stream;
    const bool nt = (L.flags & SHMEMX_LAUNCH_NONTEMPORAL) != 0;
    const uint64_t wb = nreduce * es;
#define VSHMEM_RED_K(K, CODEC)                                                                              \
    if (op == SHMEMX_RED_SUM)                                                                               \
        return nt ? launch_team_kernel(K<CODEC, OpSum, true>, g, L.wg_size, s, aw, wb)                      \
                  : launch_team_kernel(K<CODEC, OpSum, false>, g, L.wg_size, s, aw, wb);                    \
    return nt ? launch_team_kernel(K<CODEC, OpMax, true>, g, L.wg_size, s, aw, wb)                          \
              : launch_team_kernel(K<CODEC, OpMax, false>, g, L.wg_size, s, aw, wb);
#define VSHMEM_RED(CODEC)                                                                                   \
    if (waves) {                                                                                            \
        VSHMEM_RED_K(k_reduce_waves, CODEC)                                                                 \
    }                                                                                                       \
    if (two) {                                                                                              \
        VSHMEM_RED_K(k_reduce2, CODEC)                                                                      \
    }                                                                                                       \
    VSHMEM_RED_K(k_reduce, CODEC)
    if (dtype == SHMEMX_DT_INT64) {
        VSHMEM_RED(CodecI64)
    } else if (dtype == SHMEMX_DT_FP32) {
        VSHMEM_RED(CodecF32)
    } else {
        VSHMEM_RED(CodecBF16)
    }
#undef VSHMEM_RED
#undef VSHMEM_RED_K
}

}  // extern "C"
