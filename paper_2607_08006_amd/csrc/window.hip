// Windowed batches for serving: the host gathers the requests that arrived
// during a window into a pinned slot; one kernel stages the slot into device
// memory and a second executes every (request, chunk) item of it with a
// fixed grid.  The fused form launches the pair directly; the graph form
// captures the pair once per slot and replays it.
#include <cstring>
#include <vector>

#include "serving.hpp"

using namespace vshmem;

namespace {

// Slot layout: header, then nreq descriptors, then nreq item offsets
// (exclusive prefix of each request's item count).
struct alignas(64) BatchHeader {
    uint64_t nreq;
    uint64_t nitems;
    uint64_t chunk;
    uint64_t bytes;   // bytes of the whole slot to stage, a multiple of 16
    uint64_t pad[4];
};
static_assert(sizeof(BatchHeader) == 64, "header layout");

constexpr size_t kSlotBytes = sizeof(BatchHeader) + kWindowBatchMax * (sizeof(shmemx_desc_t) + 8);

__device__ __forceinline__ uint64_t uniform64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Copy the slot's used bytes from pinned host memory into device memory.
__global__ void __launch_bounds__(256) k_batch_stage(const vshmem_detail::v4u *__restrict__ host,
                                                     vshmem_detail::v4u *__restrict__ dev)
{
    const uint64_t nv = uniform64(((const BatchHeader *)host)->bytes) / 16;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (uint64_t)gridDim.x * blockDim.x)
        dev[i] = host[i];
}

// Work-group w executes items w, w + grid, ...; item j belongs to the last
// request whose first item is <= j.
__global__ void __launch_bounds__(1024) k_batch_exec(shmemx_dctx_pub_t c, const uint8_t *__restrict__ slot)
{
    const BatchHeader *h = (const BatchHeader *)slot;
    const uint64_t nreq = uniform64(h->nreq), nitems = uniform64(h->nitems), chunk = uniform64(h->chunk);
    const shmemx_desc_t *D = (const shmemx_desc_t *)(slot + sizeof(BatchHeader));
    const uint64_t *first = (const uint64_t *)(slot + sizeof(BatchHeader) + nreq * sizeof(shmemx_desc_t));
    for (uint64_t j = blockIdx.x; j < nitems; j += gridDim.x) {
        uint64_t lo = 0, hi = nreq - 1;
        while (lo < hi) {
            const uint64_t mid = (lo + hi + 1) / 2;
            if (uniform64(first[mid]) <= j) lo = mid;
            else hi = mid - 1;
        }
        shmemx_desc_t d;
        const uint32_t *q = (const uint32_t *)(D + lo);
        uint32_t *w = (uint32_t *)&d;
        for (int i = 0; i < (int)(sizeof(d) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(q[i]);
        const uint64_t k = j - uniform64(first[lo]);
        const uint64_t b0 = k * chunk;
        const uint64_t b1 = min(d.nbytes, b0 + chunk);
        exec_request_range(c, d, b0, b1, threadIdx.x, blockDim.x);
    }
    vshmem_detail::release_wg_at_exit();   // quiet
}

}  // namespace

namespace vshmem {

struct WindowBatcher {
    bool graph = false;
    uint64_t chunk = 0;
    int nwg = 0, wg = 0;
    hipStream_t stream = nullptr;
    uint8_t *host[kWindowSlots] = {};     // pinned, written by the host
    uint8_t *host_dev[kWindowSlots] = {}; // the same memory as the device sees it
    uint8_t *dev[kWindowSlots] = {};
    hipGraphExec_t exec[kWindowSlots] = {};
};

namespace {

void launch_pair(const WindowBatcher &b, int s, hipStream_t stream)
{
    hipLaunchKernelGGL(k_batch_stage, dim3(64), dim3(256), 0, stream, (const vshmem_detail::v4u *)b.host_dev[s],
                       (vshmem_detail::v4u *)b.dev[s]);
    hipLaunchKernelGGL(k_batch_exec, dim3(b.nwg), dim3(b.wg), 0, stream, pub(), (const uint8_t *)b.dev[s]);
}

}  // namespace

WindowBatcher *window_batcher_create(bool graph, uint64_t chunk_bytes, int nwg, int wg_size, hipStream_t stream,
                                     int *rc)
{
    auto *b = new WindowBatcher();
    b->graph = graph;
    b->chunk = chunk_bytes;
    b->nwg = nwg;
    b->wg = wg_size;
    b->stream = stream;
    *rc = SHMEMX_OK;
    for (int s = 0; s < kWindowSlots && !*rc; ++s) {
        if (VSHMEM_HIP_FAILED(hipHostMalloc((void **)&b->host[s], kSlotBytes, hipHostMallocMapped)) ||
            VSHMEM_HIP_FAILED(hipHostGetDevicePointer((void **)&b->host_dev[s], b->host[s], 0)) ||
            VSHMEM_HIP_FAILED(hipMalloc((void **)&b->dev[s], kSlotBytes)))
            *rc = SHMEMX_ERR_HIP;
        else
            memset(b->host[s], 0, sizeof(BatchHeader));
    }
    for (int s = 0; s < kWindowSlots && graph && !*rc; ++s) {
        // One graph per slot: the stage and execute kernels with that slot's
        // buffers; what a batch holds is read from the slot at run time.
        hipStream_t cap = nullptr;
        hipGraph_t g = nullptr;
        if (VSHMEM_HIP_FAILED(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking))) {
            *rc = SHMEMX_ERR_HIP;
            break;
        }
        if (VSHMEM_HIP_FAILED(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal))) *rc = SHMEMX_ERR_HIP;
        if (!*rc) launch_pair(*b, s, cap);
        if (VSHMEM_HIP_FAILED(hipStreamEndCapture(cap, &g)) && !*rc) *rc = SHMEMX_ERR_HIP;
        if (!*rc && VSHMEM_HIP_FAILED(hipGraphInstantiate(&b->exec[s], g, nullptr, nullptr, 0))) *rc = SHMEMX_ERR_HIP;
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cap);
    }
    if (*rc) {
        window_batcher_destroy(b);
        return nullptr;
    }
    return b;
}

int window_batcher_launch(WindowBatcher *b, int slot, const shmemx_desc_t *d, size_t n, hipEvent_t done)
{
    if (!b || slot < 0 || slot >= kWindowSlots || n == 0 || n > kWindowBatchMax) return SHMEMX_ERR_ARG;
    uint8_t *h = b->host[slot];
    auto *hdr = (BatchHeader *)h;
    auto *descs = (shmemx_desc_t *)(h + sizeof(BatchHeader));
    auto *first = (uint64_t *)(h + sizeof(BatchHeader) + n * sizeof(shmemx_desc_t));
    uint64_t items = 0;
    for (size_t i = 0; i < n; ++i) {
        descs[i] = d[i];
        first[i] = items;
        items += d[i].nbytes == 0 ? 1 : (d[i].nbytes + b->chunk - 1) / b->chunk;
    }
    hdr->nreq = n;
    hdr->nitems = items;
    hdr->chunk = b->chunk;
    hdr->bytes = (sizeof(BatchHeader) + n * (sizeof(shmemx_desc_t) + 8) + 15) / 16 * 16;
    if (b->graph) {
        VSHMEM_HIP(hipGraphLaunch(b->exec[slot], b->stream));
    } else {
        launch_pair(*b, slot, b->stream);
        VSHMEM_HIP(hipGetLastError());
    }
    VSHMEM_HIP(hipEventRecord(done, b->stream));
    return SHMEMX_OK;
}

void window_batcher_destroy(WindowBatcher *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (int s = 0; s < kWindowSlots; ++s) {
        if (b->exec[s]) (void)hipGraphExecDestroy(b->exec[s]);
        if (b->host[s]) (void)hipHostFree(b->host[s]);
        if (b->dev[s]) (void)hipFree(b->dev[s]);
    }
    delete b;
}

}  // namespace vshmem
