// Internal host-side state shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <vector>

#include "hostalloc.hpp"
#include "vshmem.h"
#include "vshmem_device.hpp"

namespace vshmem {

constexpr uint64_t kSliceAlign = 2ull << 20;      // PE slices are 2 MiB aligned

struct Team {
    bool live = false;
    int start = 0, stride = 1, size = 0;
    int slot = 0;
};

struct State {
    bool initialised = false;
    bool owns_heap = false;
    int device = 0;
    uint8_t *base = nullptr;
    uint64_t stride = 0;
    uint64_t user_bytes = 0;
    int npes = 0;
    int debug = 0;
    uint32_t *d_err = nullptr;
    shmemx_dctx_pub_t *d_ctx = nullptr;     // published, GPU-visible copy
    uint64_t wait_timeout_ticks = 0;
    uint64_t wallclock_hz = 100000000ull;
    int num_cus = 256;
    SymAllocator heap;
    std::vector<Team> teams;
    // Host default context (host-initiated operations): its own stream and
    // a pinned page that receives fetched values.
    hipStream_t host_stream = nullptr;
    uint64_t *host_words = nullptr;       // host view
    uint64_t *host_words_dev = nullptr;   // the same page as kernels address it
    // Explicit device contexts: published records and which are live.
    shmemx_dctx_rec_t *d_ctx_recs = nullptr;
    shmemx_dctx_rec_t ctx_recs[SHMEMX_MAX_DEVICE_CTX] = {};
    bool ctx_live[SHMEMX_MAX_DEVICE_CTX] = {};
    // Active tune table (batched forms without a table of their own): host
    // copy, device copy, and where it came from (SHMEMX_TUNE_SRC_*).
    shmemx_tune_t tune = {};
    shmemx_tune_t *d_tune = nullptr;
    int tune_source = 0;
    // Grid-barrier words outside the heap (one block per live plan), cleared
    // with the heap's barrier words after a wait timeout.
    std::vector<std::pair<void *, size_t>> bar_blocks;
};

constexpr int kHostWords = 512;

State &st();
void set_last_error(int code);
// Record a failed HIP runtime call (its code and where it was made) and set
// the last error to SHMEMX_ERR_HIP.
void set_hip_error(hipError_t e, const char *site);
// Set the last error to `code` with a printf-style explanation that
// shmemx_last_hip_error() reports.
void set_error_detail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
inline bool hip_failed(hipError_t e, const char *site)
{
    if (e == hipSuccess) return false;
    set_hip_error(e, site);
    return true;
}
int check_ready();
shmemx_dctx_pub_t pub();
int team_get(shmem_team_t t, shmemx_dteam_t *out);
bool in_user_heap(uint64_t off, uint64_t n);
// Offset of a canonical symmetric address, or UINT64_MAX if outside PE 0's user range.
uint64_t sym_offset(const void *p, uint64_t n);
const shmemx_launch_t &launch_or_default(const shmemx_launch_t *l, shmemx_launch_t &tmp, int def_wgs,
                                         int def_wg, uint64_t def_chunk);
bool valid_wg_size(int wg);
// Work-groups of `wg` threads of `kernel` that can be resident on one CU.
// The occupancy query has answered 0 for kernels that do launch at that
// size on MI355X; a work-group no larger than the kernel's own per-block
// limit (derived from its registers) fits on an idle CU, so count one then.
template <typename K>
int blocks_per_cu(K kernel, int wg, int *per_cu)
{
    if (hip_failed(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kernel, wg, 0),
                   "blocks_per_cu: hipOccupancyMaxActiveBlocksPerMultiprocessor"))
        return SHMEMX_ERR_HIP;
    if (*per_cu <= 0) {
        hipFuncAttributes fa{};
        if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kernel)) == hipSuccess && wg <= fa.maxThreadsPerBlock)
            *per_cu = 1;
        if (st().debug)
            fprintf(stderr, "vshmem: occupancy query gave 0 blocks of %d threads; kernel limit %d threads, %d registers\n",
                    wg, fa.maxThreadsPerBlock, fa.numRegs);
    }
    return SHMEMX_OK;
}

// Register / forget a block of grid-barrier words (cleared after a timeout).
void register_bar_block(void *p, size_t bytes);
void unregister_bar_block(void *p);
// Free the per-stream workspaces of device-table batches (finalisation).
void batch_release_workspaces();
// Take the device address of the no-allocation batch workspace on `device`
// (current), once per device.
int batch_noalloc_setup(int device);
// Validate a tune table (work-group size, scopes); SHMEMX_OK or SHMEMX_ERR_ARG.
int check_tune(const shmemx_tune_t &t);

bool progress_running();
void progress_release();
// CUs the running persistent progress kernel holds (0 when it is not
// running).  Its work-groups never leave until it stops, so a CU that holds
// one is counted as full.
int progress_reserved_cus();

// Work-groups of `kernel` at `wg` threads that can be resident at once on
// the CUs the progress kernel leaves free.
template <typename K>
int coresident_capacity(K kernel, int wg, int64_t *cap)
{
    int per_cu = 0;
    if (int rc = blocks_per_cu(kernel, wg, &per_cu)) return rc;
    const int free_cus = st().num_cus - progress_reserved_cus();
    *cap = (int64_t)per_cu * (free_cus > 0 ? free_cus : 0);
    return SHMEMX_OK;
}

// Check before launching a kernel whose `grid` work-groups wait for each
// other (team and plan barriers, paired signal waits): all of them must be
// resident together, or the waits can only end at the spin limit.  Returns
// SHMEMX_ERR_BUSY when they would fit an idle device but not next to the
// running progress kernel, SHMEMX_ERR_ARG when they never fit.  Only the
// library's own persistent kernel is accounted for; kernels the caller runs
// on other streams at the same time are the caller's to keep apart.
template <typename K>
int check_coresident(K kernel, int64_t grid, int wg, const char *what)
{
    int per_cu = 0;
    if (int rc = blocks_per_cu(kernel, wg, &per_cu)) return rc;
    const int reserved = progress_reserved_cus();
    const int64_t idle_cap = (int64_t)per_cu * st().num_cus;
    const int64_t cap = (int64_t)per_cu * (st().num_cus > reserved ? st().num_cus - reserved : 0);
    if (grid <= cap) return SHMEMX_OK;
    if (grid <= idle_cap) {
        set_error_detail(SHMEMX_ERR_BUSY,
                         "%s: %lld work-groups of %d threads cannot be co-resident next to the progress kernel "
                         "(%d per CU x %d free CUs of %d)",
                         what, (long long)grid, wg, per_cu, st().num_cus - reserved, st().num_cus);
        return SHMEMX_ERR_BUSY;
    }
    set_error_detail(SHMEMX_ERR_ARG, "%s: %lld work-groups of %d threads cannot be co-resident (%d per CU x %d CUs)",
                     what, (long long)grid, wg, per_cu, st().num_cus);
    if (st().debug) fprintf(stderr, "vshmem: %s: work-groups cannot be co-resident\n", what);
    return SHMEMX_ERR_ARG;
}

}  // namespace vshmem

#define VSHMEM_STR2(x) #x
#define VSHMEM_STR(x) VSHMEM_STR2(x)
// True when the call failed; the failure is recorded as by VSHMEM_HIP.
#define VSHMEM_HIP_FAILED(call) \
    vshmem::hip_failed((call), __FILE__ ":" VSHMEM_STR(__LINE__) ": " #call)
#define VSHMEM_HIP(call)                                                                                  \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) {                                                                           \
            vshmem::set_hip_error(e_, __FILE__ ":" VSHMEM_STR(__LINE__) ": " #call);                      \
            return SHMEMX_ERR_HIP;                                                                        \
        }                                                                                                 \
    } while (0)
