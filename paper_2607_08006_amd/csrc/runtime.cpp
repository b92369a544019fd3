// Host runtime: symmetric heap, allocator, published device context, teams,
// capability query and error reporting.
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "runtime.hpp"

#include <cctype>
#include <cstdlib>
#include <cstring>
#include <string>

namespace vshmem {

static State g_state;
static thread_local int g_last_error = SHMEMX_OK;

State &st() { return g_state; }
void clear_error_detail();
void set_last_error(int code)
{
    clear_error_detail();
    g_last_error = code;
}

namespace {
std::mutex g_detail_mu;
int g_hip_code = 0;
char g_detail[384] = "";
}  // namespace

void set_hip_error(hipError_t e, const char *site)
{
    {
        std::lock_guard<std::mutex> lk(g_detail_mu);
        g_hip_code = (int)e;
        snprintf(g_detail, sizeof g_detail, "%s (%d) at %s", hipGetErrorName(e), (int)e, site);
    }
    g_last_error = SHMEMX_ERR_HIP;
}

void clear_error_detail()
{
    std::lock_guard<std::mutex> lk(g_detail_mu);
    g_hip_code = 0;
    g_detail[0] = 0;
}

void set_error_detail(int code, const char *fmt, ...)
{
    {
        std::lock_guard<std::mutex> lk(g_detail_mu);
        g_hip_code = 0;
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(g_detail, sizeof g_detail, fmt, ap);
        va_end(ap);
    }
    g_last_error = code;
}

int check_ready()
{
    if (!g_state.initialised) {
        set_last_error(SHMEMX_ERR_STATE);
        return SHMEMX_ERR_STATE;
    }
    return SHMEMX_OK;
}

shmemx_dctx_pub_t pub()
{
    shmemx_dctx_pub_t c{};
    c.base = g_state.base;
    c.stride = g_state.stride;
    c.user_bytes = g_state.user_bytes;
    c.scratch_off = g_state.user_bytes;
    c.err = g_state.d_err;
    c.wait_timeout_ticks = g_state.wait_timeout_ticks;
    c.npes = g_state.npes;
    c.debug = g_state.debug;
    return c;
}

bool in_user_heap(uint64_t off, uint64_t n)
{
    return off <= g_state.user_bytes && n <= g_state.user_bytes - off;
}

uint64_t sym_offset(const void *p, uint64_t n)
{
    uintptr_t a = (uintptr_t)p, b = (uintptr_t)g_state.base;
    if (a < b) return UINT64_MAX;
    uint64_t off = a - b;
    if (!in_user_heap(off, n)) return UINT64_MAX;
    return off;
}

int team_get(shmem_team_t t, shmemx_dteam_t *out)
{
    if (t < 0 || t >= (int)g_state.teams.size() || !g_state.teams[t].live) return SHMEMX_ERR_ARG;
    const Team &tm = g_state.teams[t];
    out->start = tm.start;
    out->stride = tm.stride;
    out->size = tm.size;
    out->slot = tm.slot;
    return SHMEMX_OK;
}

bool valid_wg_size(int wg) { return wg >= 64 && wg <= 1024 && (wg % 64) == 0; }

const shmemx_launch_t &launch_or_default(const shmemx_launch_t *l, shmemx_launch_t &tmp, int def_wgs, int def_wg,
                                         uint64_t def_chunk)
{
    tmp = l ? *l : shmemx_launch_t{};
    if (tmp.wgs_per_pe <= 0) tmp.wgs_per_pe = def_wgs;
    if (tmp.wg_size <= 0) tmp.wg_size = def_wg;
    if (tmp.chunk_bytes == 0) tmp.chunk_bytes = def_chunk;
    return tmp;
}

// ------------------------------------------------------------- allocator
static void reset_teams()
{
    g_state.teams.assign(4, Team{});
    for (int t = 0; t < 4; ++t) {
        g_state.teams[t].live = true;
        g_state.teams[t].start = 0;
        g_state.teams[t].stride = 1;
        g_state.teams[t].size = g_state.npes;
        g_state.teams[t].slot = t;
    }
}

static uint64_t parse_size(const char *s, uint64_t def)
{
    if (!s || !*s) return def;
    char *end = nullptr;
    double v = strtod(s, &end);
    if (end == s || v < 0) return def;
    uint64_t mul = 1;
    if (end && *end) {
        switch (toupper((unsigned char)*end)) {
        case 'K': mul = 1ull << 10; break;
        case 'M': mul = 1ull << 20; break;
        case 'G': mul = 1ull << 30; break;
        case 'T': mul = 1ull << 40; break;
        default: mul = 1;
        }
    }
    return (uint64_t)(v * (double)mul);
}

static int finish_init(void *heap, size_t heap_bytes, int npes, hipStream_t stream)
{
    State &s = g_state;
    s.base = (uint8_t *)heap;
    s.npes = npes;
    s.stride = heap_bytes / (uint64_t)npes;
    s.user_bytes = s.stride - VSHMEM_SCRATCH_BYTES;
    const char *dbg = getenv("VSHMEM_DEBUG");
    s.debug = dbg ? atoi(dbg) : 0;
    VSHMEM_HIP(hipGetDevice(&s.device));
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s.device) == hipSuccess && khz > 0)
        s.wallclock_hz = (uint64_t)khz * 1000ull;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s.device) == hipSuccess && cus > 0)
        s.num_cus = cus;
    s.wait_timeout_ticks = s.wallclock_hz * 10ull;        // 10 s
    VSHMEM_HIP(hipMalloc((void **)&s.d_err, 256));
    VSHMEM_HIP(hipMemsetAsync(s.d_err, 0, 256, stream));
    for (int p = 0; p < npes; ++p)
        VSHMEM_HIP(hipMemsetAsync(s.base + (uint64_t)p * s.stride + s.user_bytes, 0, VSHMEM_SCRATCH_BYTES, stream));
    VSHMEM_HIP(hipMalloc((void **)&s.d_ctx, sizeof(shmemx_dctx_pub_t)));
    VSHMEM_HIP(hipMalloc((void **)&s.d_ctx_recs, sizeof(shmemx_dctx_rec_t) * SHMEMX_MAX_DEVICE_CTX));
    VSHMEM_HIP(hipStreamCreateWithFlags(&s.host_stream, hipStreamNonBlocking));
    // Coherent: blocking host calls spin on a completion word kernels store here.
    VSHMEM_HIP(hipHostMalloc((void **)&s.host_words, kHostWords * sizeof(uint64_t),
                             hipHostMallocMapped | hipHostMallocCoherent));
    VSHMEM_HIP(hipHostGetDevicePointer((void **)&s.host_words_dev, s.host_words, 0));
    s.heap.reset(s.user_bytes);
    reset_teams();
    // Active tune table: VSHMEM_TUNE_FILE when it names a table saved on
    // this kind of device, else the built-in defaults.
    shmemx_tune_default(&s.tune);
    s.tune_source = SHMEMX_TUNE_SRC_DEFAULT;
    if (const char *tf = getenv("VSHMEM_TUNE_FILE")) {
        shmemx_tune_t t;
        if (*tf && shmemx_tune_load(&t, tf) == SHMEMX_OK) {
            s.tune = t;
            s.tune_source = SHMEMX_TUNE_SRC_FILE;
        } else if (*tf) {
            s.tune_source = SHMEMX_TUNE_SRC_FILE_REFUSED;
            if (s.debug) fprintf(stderr, "vshmem: VSHMEM_TUNE_FILE=%s refused; using the built-in table\n", tf);
        }
    }
    if (int rc = batch_noalloc_setup(s.device)) return rc;
    VSHMEM_HIP(hipMalloc((void **)&s.d_tune, sizeof(shmemx_tune_t)));
    VSHMEM_HIP(hipMemcpyAsync(s.d_tune, &s.tune, sizeof(shmemx_tune_t), hipMemcpyHostToDevice, stream));
    s.initialised = true;
    shmemx_dctx_pub_t c = pub();
    hipError_t e = hipMemcpyAsync(s.d_ctx, &c, sizeof(c), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        s.initialised = false;
        set_hip_error(e, "publishing the device context");
        return SHMEMX_ERR_HIP;
    }
    return SHMEMX_OK;
}

static int republish()
{
    State &s = g_state;
    shmemx_dctx_pub_t c = pub();
    VSHMEM_HIP(hipMemcpy(s.d_ctx, &c, sizeof(c), hipMemcpyHostToDevice));
    for (int i = 0; i < SHMEMX_MAX_DEVICE_CTX; ++i) {
        if (!s.ctx_live[i]) continue;
        s.ctx_recs[i].pub = c;
        VSHMEM_HIP(hipMemcpy(s.d_ctx_recs + i, &s.ctx_recs[i], sizeof(shmemx_dctx_rec_t), hipMemcpyHostToDevice));
    }
    return SHMEMX_OK;
}

void register_bar_block(void *p, size_t bytes) { g_state.bar_blocks.push_back({p, bytes}); }

void unregister_bar_block(void *p)
{
    auto &v = g_state.bar_blocks;
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i].first == p) {
            v.erase(v.begin() + (long)i);
            return;
        }
}

int check_tune(const shmemx_tune_t &t)
{
    if (!valid_wg_size(t.wg_size) || t.grid_wgs < 0) return SHMEMX_ERR_ARG;
    for (int c = 0; c < SHMEMX_TUNE_CLASSES; ++c)
        if (t.scope[c] > SHMEMX_SCOPE_GRID) return SHMEMX_ERR_ARG;
    return SHMEMX_OK;
}

}  // namespace vshmem

using namespace vshmem;

extern "C" {

int shmemx_init_attach(void *heap, size_t heap_bytes, int npes, void *stream)
{
    State &s = st();
    if (s.initialised) {
        set_last_error(SHMEMX_ERR_STATE);
        return SHMEMX_ERR_STATE;
    }
    if (!heap || npes <= 0 || npes > 65536 || heap_bytes == 0 || heap_bytes % (uint64_t)npes != 0 ||
        ((uintptr_t)heap % kSliceAlign) != 0 || (heap_bytes / (uint64_t)npes) % kSliceAlign != 0) {
        set_last_error(SHMEMX_ERR_ARG);
        return SHMEMX_ERR_ARG;
    }
    s.owns_heap = false;
    return finish_init(heap, heap_bytes, npes, (hipStream_t)stream);
}

uint64_t shmemx_heap_stride_for(uint64_t bytes_per_pe, int spread)
{
    constexpr uint64_t kMaxBytes = 1ull << 50;
    if (bytes_per_pe > kMaxBytes) return 0;
    const uint64_t s = (bytes_per_pe + VSHMEM_SCRATCH_BYTES + kSliceAlign - 1) & ~(kSliceAlign - 1);
    if (!spread) return s;
    // The largest power of two 2^k <= s.
    if (s < (64ull << 20)) return s;
    const uint64_t p2 = 1ull << (63 - __builtin_clzll(s));
    const uint64_t spread_stride = p2 + p2 / 2 + kSliceAlign;
    return s < spread_stride ? spread_stride : s;
}

void shmem_init(void)
{
    State &s = st();
    if (s.initialised) {
        set_last_error(SHMEMX_ERR_STATE);
        return;
    }
    const char *np = getenv("VSHMEM_NPES");
    int npes = np ? atoi(np) : 4;
    uint64_t user = parse_size(getenv("VSHMEM_SYMMETRIC_SIZE"), 64ull << 20);
    if (npes <= 0 || user == 0) {
        set_last_error(SHMEMX_ERR_ARG);
        return;
    }
    uint64_t stride = shmemx_heap_stride_for(user, 1);
    void *heap = nullptr;
    if (stride == 0 || VSHMEM_HIP_FAILED(hipMalloc(&heap, stride * (uint64_t)npes))) {
        // The spread stride does not fit: fall back to the smallest.
        (void)hipGetLastError();
        stride = shmemx_heap_stride_for(user, 0);
        if (stride == 0 || VSHMEM_HIP_FAILED(hipMalloc(&heap, stride * (uint64_t)npes))) {
            set_last_error(SHMEMX_ERR_NOMEM);
            return;
        }
    }
    s.owns_heap = true;
    if (finish_init(heap, stride * (uint64_t)npes, npes, nullptr) != SHMEMX_OK) {
        (void)hipFree(heap);
        s.owns_heap = false;
    }
}

void shmem_finalize(void)
{
    State &s = st();
    if (!s.initialised) {
        set_last_error(SHMEMX_ERR_STATE);
        return;
    }
    if (progress_running()) (void)shmemx_progress_stop(10000);
    (void)hipDeviceSynchronize();
    progress_release();
    batch_release_workspaces();
    if (s.d_tune) (void)hipFree(s.d_tune);
    if (s.d_ctx) (void)hipFree(s.d_ctx);
    if (s.d_ctx_recs) (void)hipFree(s.d_ctx_recs);
    if (s.d_err) (void)hipFree(s.d_err);
    if (s.host_stream) (void)hipStreamDestroy(s.host_stream);
    if (s.host_words) (void)hipHostFree(s.host_words);
    if (s.owns_heap && s.base) (void)hipFree(s.base);
    s = State{};
}

int shmem_n_pes(void) { return st().initialised ? st().npes : 0; }
int shmem_my_pe(void) { return st().initialised ? 0 : -1; }

void *shmem_align(size_t alignment, size_t size)
{
    State &s = st();
    if (!s.initialised || size == 0 || alignment == 0 || (alignment & (alignment - 1))) {
        set_last_error(s.initialised ? SHMEMX_ERR_ARG : SHMEMX_ERR_STATE);
        return nullptr;
    }
    if (alignment < kMinAlign) alignment = kMinAlign;
    uint64_t off = s.heap.alloc(size, alignment);
    if (off == UINT64_MAX) {
        set_last_error(SHMEMX_ERR_NOMEM);
        return nullptr;
    }
    return s.base + off;
}

void *shmem_malloc(size_t size) { return shmem_align(kMinAlign, size); }
void *shmemg_malloc(size_t size) { return shmem_align(kMinAlign, size); }

void *shmem_calloc(size_t count, size_t size)
{
    if (count && size > SIZE_MAX / count) {
        set_last_error(SHMEMX_ERR_ARG);
        return nullptr;
    }
    void *p = shmem_malloc(count * size);
    if (!p) return nullptr;
    State &s = st();
    for (int pe = 0; pe < s.npes; ++pe) {
        if (VSHMEM_HIP_FAILED(hipMemsetAsync((uint8_t *)p + (uint64_t)pe * s.stride, 0, count * size, nullptr))) {
            shmem_free(p);
            return nullptr;
        }
    }
    if (VSHMEM_HIP_FAILED(hipStreamSynchronize(nullptr))) {
        shmem_free(p);
        return nullptr;
    }
    return p;
}

void shmem_free(void *ptr)
{
    State &s = st();
    if (!ptr) return;
    if (!s.initialised) {
        set_last_error(SHMEMX_ERR_STATE);
        return;
    }
    uintptr_t a = (uintptr_t)ptr, b = (uintptr_t)s.base;
    if (a < b || a - b >= s.user_bytes || !s.heap.free(a - b)) set_last_error(SHMEMX_ERR_ARG);
}

void *shmem_team_ptr(shmem_team_t team, const void *dest, int pe)
{
    shmemx_dteam_t t;
    if (!st().initialised || team_get(team, &t) != SHMEMX_OK || pe < 0 || pe >= t.size) return nullptr;
    return shmem_ptr(dest, t.start + pe * t.stride);
}

void *shmem_ptr(const void *sym, int pe)
{
    State &s = st();
    if (!s.initialised || pe < 0 || pe >= s.npes) return nullptr;
    uintptr_t a = (uintptr_t)sym, b = (uintptr_t)s.base;
    if (a < b || a - b >= s.user_bytes) return nullptr;
    return (uint8_t *)sym + (uint64_t)pe * s.stride;
}

int shmem_query_capabilities(shmem_team_t team, shmemx_caps_t *caps)
{
    if (int rc = check_ready()) return rc;
    shmemx_dteam_t t;
    if (!caps || team_get(team, &t) != SHMEMX_OK) {
        set_last_error(SHMEMX_ERR_ARG);
        return SHMEMX_ERR_ARG;
    }
    State &s = st();
    memset(caps, 0, sizeof(*caps));
    caps->gpu_heap = 1;
    caps->default_heap_is_gpu = 1;
    caps->host_initiated = 1;
    caps->device_initiated = 1;
    caps->device_ctx_default = 1;
    caps->explicit_device_ctx = 1;
    caps->max_device_ctx = SHMEMX_MAX_DEVICE_CTX;
    caps->scopes = (1u << SHMEMX_SCOPE_THREAD) | (1u << SHMEMX_SCOPE_WAVE) | (1u << SHMEMX_SCOPE_WG) |
                   (1u << SHMEMX_SCOPE_GRID);
    caps->device_collectives = 1;
    caps->stream_triggered = 1;
    caps->progress = SHMEMX_PROGRESS_KERNEL_LAUNCH | SHMEMX_PROGRESS_PERSISTENT_GPU;
    caps->path = SHMEMX_PATH_SINGLE_GPU_LOADSTORE;
    caps->ptr_domain = SHMEMX_PTR_DOMAIN_DEVICE;
    caps->team_npes = t.size;
    caps->team_start = t.start;
    caps->team_stride = t.stride;
    caps->npes = s.npes;
    caps->heap_user_bytes = s.user_bytes;
    caps->heap_stride = s.stride;
    caps->debug = s.debug;
    return SHMEMX_OK;
}

void *shmemx_heap_base(void) { return st().initialised ? st().base : nullptr; }
uint64_t shmemx_heap_stride(void) { return st().initialised ? st().stride : 0; }
uint64_t shmemx_heap_user_bytes(void) { return st().initialised ? st().user_bytes : 0; }
const void *shmemx_device_ctx(void) { return st().initialised ? st().d_ctx : nullptr; }

int shmemx_device_ctx_create(shmem_team_t team, long options, shmemx_ctx_t *ctx)
{
    if (int rc = check_ready()) return rc;
    State &s = st();
    shmemx_dteam_t t;
    if (!ctx || team_get(team, &t) != SHMEMX_OK) {
        set_last_error(SHMEMX_ERR_ARG);
        return SHMEMX_ERR_ARG;
    }
    int i = 0;
    while (i < SHMEMX_MAX_DEVICE_CTX && s.ctx_live[i]) ++i;
    if (i == SHMEMX_MAX_DEVICE_CTX) {
        set_last_error(SHMEMX_ERR_NOMEM);
        return SHMEMX_ERR_NOMEM;
    }
    s.ctx_recs[i] = shmemx_dctx_rec_t{pub(), t, (int64_t)options};
    VSHMEM_HIP(hipMemcpy(s.d_ctx_recs + i, &s.ctx_recs[i], sizeof(shmemx_dctx_rec_t), hipMemcpyHostToDevice));
    s.ctx_live[i] = true;
    *ctx = i;
    return SHMEMX_OK;
}

const void *shmemx_device_ctx_record(shmemx_ctx_t ctx)
{
    const State &s = st();
    if (!s.initialised || ctx < 0 || ctx >= SHMEMX_MAX_DEVICE_CTX || !s.ctx_live[ctx]) return nullptr;
    return s.d_ctx_recs + ctx;
}

void shmemx_device_ctx_destroy(shmemx_ctx_t ctx)
{
    State &s = st();
    if (!s.initialised || ctx < 0 || ctx >= SHMEMX_MAX_DEVICE_CTX || !s.ctx_live[ctx]) {
        set_last_error(s.initialised ? SHMEMX_ERR_ARG : SHMEMX_ERR_STATE);
        return;
    }
    s.ctx_live[ctx] = false;
}
uint64_t shmemx_wallclock_hz(void) { return st().wallclock_hz; }

int shmem_team_split_strided(shmem_team_t parent, int start, int stride, int size, const void *config,
                             long config_mask, shmem_team_t *new_team)
{
    (void)config;
    (void)config_mask;
    if (int rc = check_ready()) return rc;
    shmemx_dteam_t p;
    if (!new_team || team_get(parent, &p) != SHMEMX_OK || size <= 0 || start < 0 || stride <= 0 ||
        start + (int64_t)(size - 1) * stride >= p.size) {
        if (new_team) *new_team = SHMEM_TEAM_INVALID;
        set_last_error(SHMEMX_ERR_ARG);
        return SHMEMX_ERR_ARG;
    }
    State &s = st();
    int idx = -1;
    for (int i = 4; i < (int)s.teams.size(); ++i)
        if (!s.teams[i].live) {
            idx = i;
            break;
        }
    if (idx < 0) {
        if ((int)s.teams.size() >= VSHMEM_MAX_TEAMS - 8) {
            *new_team = SHMEM_TEAM_INVALID;
            set_last_error(SHMEMX_ERR_NOMEM);
            return SHMEMX_ERR_NOMEM;
        }
        idx = (int)s.teams.size();
        s.teams.push_back(Team{});
    }
    Team &t = s.teams[idx];
    t.live = true;
    t.start = p.start + start * p.stride;
    t.stride = p.stride * stride;
    t.size = size;
    t.slot = idx;
    // Clear the new team's barrier words (count and generation) in its
    // first member's scratch.
    uint8_t *slot = s.base + (uint64_t)t.start * s.stride + s.user_bytes + (uint64_t)t.slot * VSHMEM_SYNC_SLOT_BYTES;
    if (VSHMEM_HIP_FAILED(hipMemset(slot, 0, VSHMEM_SYNC_SLOT_BYTES)) ||
        VSHMEM_HIP_FAILED(hipMemset(slot + VSHMEM_SYNC_GEN_OFF, 0, VSHMEM_SYNC_SLOT_BYTES))) {
        t.live = false;
        return SHMEMX_ERR_HIP;
    }
    *new_team = idx;
    return SHMEMX_OK;
}

int shmem_team_n_pes(shmem_team_t team)
{
    shmemx_dteam_t t;
    if (!st().initialised || team_get(team, &t) != SHMEMX_OK) return -1;
    return t.size;
}

int shmemx_team_device(shmem_team_t team, shmemx_dteam_t *out)
{
    int rc = check_ready();
    if (!rc && (!out || team_get(team, out) != SHMEMX_OK)) rc = SHMEMX_ERR_ARG;
    if (rc) set_last_error(rc);
    return rc;
}

int shmemx_team_pe_index(shmem_team_t team, int pe)
{
    shmemx_dteam_t t;
    if (!st().initialised || team_get(team, &t) != SHMEMX_OK) return -1;
    int d = pe - t.start;
    if (d < 0 || d % t.stride) return -1;
    int k = d / t.stride;
    return k < t.size ? k : -1;
}

void shmem_team_destroy(shmem_team_t team)
{
    State &s = st();
    if (!s.initialised || team < 4 || team >= (int)s.teams.size()) {
        set_last_error(SHMEMX_ERR_ARG);
        return;
    }
    s.teams[team].live = false;
}

const char *shmemx_strerror(int code)
{
    switch (code) {
    case SHMEMX_OK: return "success";
    case SHMEMX_ERR_ARG: return "invalid argument";
    case SHMEMX_ERR_NOMEM: return "out of memory or budget";
    case SHMEMX_ERR_STATE: return "library not in the required state";
    case SHMEMX_ERR_HIP: return "HIP runtime error";
    case SHMEMX_ERR_BUSY: return "resource busy";
    case SHMEMX_ERR_TIMEOUT: return "timed out";
    case SHMEMX_ERR_DEVICE: return "device reported an error";
    case SHMEMX_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown error";
    }
}

int shmemx_last_error(void) { return vshmem::g_last_error; }
void shmemx_clear_last_error(void) { vshmem::set_last_error(SHMEMX_OK); }

int shmemx_device_errors(void)
{
    if (int rc = check_ready()) return rc;
    State &s = st();
    uint32_t v = 0;
    VSHMEM_HIP(hipDeviceSynchronize());
    VSHMEM_HIP(hipMemcpy(&v, s.d_err, 4, hipMemcpyDeviceToHost));
    VSHMEM_HIP(hipMemset(s.d_err, 0, 4));
    if (v & SHMEMX_DEVERR_WAIT_TIMEOUT) {
        // A barrier that timed out keeps the arrivals it got; with the device
        // idle, every barrier word (the scratch tail holds nothing else)
        // restarts at phase 0, count 0.
        for (int p = 0; p < s.npes; ++p)
            VSHMEM_HIP(hipMemsetAsync(s.base + (uint64_t)p * s.stride + s.user_bytes, 0, VSHMEM_SCRATCH_BYTES, nullptr));
        for (const auto &b : s.bar_blocks) VSHMEM_HIP(hipMemsetAsync(b.first, 0, b.second, nullptr));
        VSHMEM_HIP(hipStreamSynchronize(nullptr));
    }
    return (int)(v & 0x7fffffffu);
}

int shmemx_tune_set(const shmemx_tune_t *tune)
{
    if (int rc = check_ready()) return rc;
    if (!tune || check_tune(*tune)) return SHMEMX_ERR_ARG;
    State &s = st();
    // Kernels already queued read the device copy: replace it in stream order
    // after everything issued so far.
    VSHMEM_HIP(hipDeviceSynchronize());
    VSHMEM_HIP(hipMemcpy(s.d_tune, tune, sizeof(*tune), hipMemcpyHostToDevice));
    s.tune = *tune;
    s.tune_source = SHMEMX_TUNE_SRC_SET;
    return SHMEMX_OK;
}

int shmemx_tune_get(shmemx_tune_t *tune)
{
    if (int rc = check_ready()) return rc;
    if (!tune) return SHMEMX_ERR_ARG;
    *tune = st().tune;
    return st().tune_source;
}

int shmemx_set_wait_timeout_ns(uint64_t ns)
{
    if (int rc = check_ready()) return rc;
    State &s = st();
    uint64_t ticks = (uint64_t)((double)ns * (double)s.wallclock_hz / 1e9);
    s.wait_timeout_ticks = ticks ? ticks : 1;
    return republish();
}

const char *shmemx_version(void) { return "vshmem 0.1 (gfx950)"; }

int shmemx_last_hip_error(char *buf, size_t len)
{
    std::lock_guard<std::mutex> lk(g_detail_mu);
    if (buf && len) snprintf(buf, len, "%s", g_detail);
    return g_hip_code;
}

}  // extern "C"
