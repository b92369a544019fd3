// Host-initiated operations (the host default context) and stream-triggered
// operations (ordered in a caller's stream).  Both are host-issued; internal
// kernels and runtime copies execute them: a copy kernel for device-to-
// device moves, one-thread kernels built from the device API for AMOs,
// signal updates and waits, and the collective launchers.
#include <algorithm>
#include <chrono>

#include "runtime.hpp"

using namespace vshmem;

namespace {

enum HostAmo : int {
    HA_FETCH_ADD,
    HA_FETCH_XOR,
    HA_CSWAP,
    HA_FETCH,
    HA_SET,
    HA_SWAP,
    HA_SIGNAL_SET,
    HA_SIGNAL_ADD,
};

// A blocking host call's completion word: after the call's effect and
// result, `seq` is stored to pinned host memory with a system-scope release.
__device__ __forceinline__ void post_done(uint64_t *done, uint64_t seq)
{
    if (done) __hip_atomic_store(done, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// One atomic on PE pe's copy of the canonical word `sym`, issued as PE 0
// through the device API; the previous value goes to *out when out is set,
// then the completion word when done is set.
__global__ void __launch_bounds__(64) k_host_amo(shmemx_dctx_pub_t c, int op, uint64_t *sym, int pe, uint64_t v,
                                                 uint64_t cond, uint64_t *out, uint64_t *done, uint64_t seq)
{
    if (threadIdx.x != 0) return;
    const shmem_dctx_t ctx = shmemx_dctx_bind(c, 0);
    int64_t *d = (int64_t *)sym;
    uint64_t old = 0;
    switch (op) {
    case HA_FETCH_ADD: old = (uint64_t)shmem_int64_atomic_fetch_add(ctx, d, (int64_t)v, pe); break;
    case HA_FETCH_XOR: old = shmem_uint64_atomic_fetch_xor(ctx, sym, v, pe); break;
    case HA_CSWAP: old = (uint64_t)shmem_int64_atomic_compare_swap(ctx, d, (int64_t)cond, (int64_t)v, pe); break;
    case HA_FETCH: old = (uint64_t)shmem_int64_atomic_fetch(ctx, d, pe); break;
    case HA_SET: shmem_int64_atomic_set(ctx, d, (int64_t)v, pe); break;
    case HA_SWAP: old = (uint64_t)shmem_int64_atomic_swap(ctx, d, (int64_t)v, pe); break;
    case HA_SIGNAL_SET: vshmemx_signal_update(ctx, sym, v, SHMEM_SIGNAL_SET, pe); break;
    default: vshmemx_signal_update(ctx, sym, v, SHMEM_SIGNAL_ADD, pe); break;
    }
    if (out) *out = old;
    post_done(done, seq);
}

// Wait on PE 0's copy of `sym`; writes the value seen to *out when set,
// then the completion word when done is set.
__global__ void __launch_bounds__(64) k_host_wait(shmemx_dctx_pub_t c, uint64_t *sym, int cmp, uint64_t v,
                                                  int is_signed, uint64_t *out, uint64_t *done, uint64_t seq)
{
    if (threadIdx.x != 0) return;
    const uint64_t x = is_signed ? vshmem_detail::spin_until<true>(c, sym, cmp, v)
                                 : vshmem_detail::spin_until<false>(c, sym, cmp, v);
    if (out) *out = x;
    post_done(done, seq);
}

// Device-to-device copy striped over the whole grid (lane i moves 16-byte
// vectors i, i + lanes, ...), nontemporal, 8 loads in flight per lane.
__global__ void __launch_bounds__(1024) k_host_copy(uint8_t *d, const uint8_t *s, uint64_t n)
{
    vshmem_detail::copy_bytes<8, true, true>(d, s, n, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x,
                                       (uint64_t)gridDim.x * blockDim.x);
}

int fail(int rc)
{
    set_last_error(rc);
    return rc;
}

// True when [p, p + n) is device memory: inside the heap, or in a device
// allocation of the runtime (the range is assumed to lie in one allocation).
bool is_device_range(const void *p, uint64_t n)
{
    const State &s = st();
    const uint8_t *b = (const uint8_t *)p;
    if (b >= s.base && b + n <= s.base + s.stride * (uint64_t)s.npes) return true;
    hipPointerAttribute_t a{};
    const hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // host memory the runtime never saw is reported as an error
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

// PE pe's copy of a canonical symmetric range, or nullptr when the range is
// not inside PE 0's user heap or pe is out of range.
uint8_t *remote(const void *sym, uint64_t n, int pe)
{
    const State &s = st();
    if (pe < 0 || pe >= s.npes) return nullptr;
    const uint64_t off = sym_offset(sym, n);
    if (off == UINT64_MAX) return nullptr;
    return s.base + (uint64_t)pe * s.stride + off;
}

// A naturally aligned symmetric 8-byte word.
bool sym_word(const void *w) { return w && ((uintptr_t)w & 7) == 0 && sym_offset(w, 8) != UINT64_MAX; }

int enqueue_copy(void *dst, const void *src, uint64_t n, hipStream_t stream)
{
    if (n == 0) return SHMEMX_OK;
    if (is_device_range(dst, n) && is_device_range(src, n)) {
        // 16 vectors per lane per work-group pass: small copies take few
        // work-groups, large ones about one 1024-thread work-group per CU.
        const uint64_t per_wg = 1024ull * 16 * 16;
        const uint64_t nwg = std::min<uint64_t>((uint64_t)st().num_cus, (n + per_wg - 1) / per_wg);
        hipLaunchKernelGGL(k_host_copy, dim3((unsigned)nwg), dim3(1024), 0, stream, (uint8_t *)dst,
                           (const uint8_t *)src, n);
        VSHMEM_HIP(hipGetLastError());
        return SHMEMX_OK;
    }
    VSHMEM_HIP(hipMemcpyAsync(dst, src, n, hipMemcpyDefault, stream));
    return SHMEMX_OK;
}

int rma(bool is_put, void *dest, const void *source, size_t n, int pe, hipStream_t stream)
{
    if (int rc = check_ready()) return rc;
    if (n == 0) return pe >= 0 && pe < st().npes ? SHMEMX_OK : fail(SHMEMX_ERR_ARG);
    const void *sym = is_put ? dest : source;
    uint8_t *r = remote(sym, n, pe);
    const void *local = is_put ? source : dest;
    if (!r || !local) return fail(SHMEMX_ERR_ARG);
    const int rc = is_put ? enqueue_copy(r, source, n, stream) : enqueue_copy(dest, r, n, stream);
    return rc ? fail(rc) : SHMEMX_OK;
}

int amo_enqueue(int op, void *sym, int pe, uint64_t v, uint64_t cond, uint64_t *out, hipStream_t stream,
                uint64_t *done = nullptr, uint64_t seq = 0)
{
    if (int rc = check_ready()) return rc;
    if (!sym_word(sym) || pe < 0 || pe >= st().npes) return fail(SHMEMX_ERR_ARG);
    hipLaunchKernelGGL(k_host_amo, dim3(1), dim3(64), 0, stream, pub(), op, (uint64_t *)sym, pe, v, cond, out, done,
                       seq);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int host_sync()
{
    VSHMEM_HIP(hipStreamSynchronize(st().host_stream));
    return SHMEMX_OK;
}

// Blocking one-kernel calls (AMOs, signal reads, waits) end with a
// completion word instead of a stream synchronisation: the kernel stores the
// call's sequence number to pinned host memory after its result, and the
// host spins on that word.  The spin stops after kDoneSpin (a wait that
// lasts longer then sleeps in the stream synchronisation) or when the
// stream reports an error.  Host words: [0] AMO result, [1] wait result,
// [2] completion.  Calls through the host context are serialised by their
// caller, as the host context's other blocking calls are.
constexpr int kDoneWord = 2;
constexpr auto kDoneSpin = std::chrono::microseconds(200);
uint64_t g_done_seq = 0;

int wait_done(uint64_t seq)
{
    State &s = st();
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t k = 1;; ++k) {
        if (__atomic_load_n(&s.host_words[kDoneWord], __ATOMIC_ACQUIRE) == seq) return SHMEMX_OK;
        if ((k & 255) == 0) {
            const hipError_t e = hipStreamQuery(s.host_stream);
            if (e != hipErrorNotReady || std::chrono::steady_clock::now() - t0 > kDoneSpin) break;
        }
        __builtin_ia32_pause();
    }
    if (int rc = host_sync()) return rc;
    // The kernel ended, so its completion word is in place.
    return __atomic_load_n(&s.host_words[kDoneWord], __ATOMIC_ACQUIRE) == seq ? SHMEMX_OK : fail(SHMEMX_ERR_HIP);
}

// Blocking AMO through the host context; the fetched value lands in the
// pinned page.  Returns 0 (and records the error) on failure.
uint64_t amo_blocking(int op, void *sym, int pe, uint64_t v, uint64_t cond)
{
    State &s = st();
    if (!s.initialised) {
        set_last_error(SHMEMX_ERR_STATE);
        return 0;
    }
    s.host_words[0] = 0;
    const uint64_t seq = ++g_done_seq;
    if (amo_enqueue(op, sym, pe, v, cond, s.host_words_dev, s.host_stream, s.host_words_dev + kDoneWord, seq) ||
        wait_done(seq))
        return 0;
    return __atomic_load_n(&s.host_words[0], __ATOMIC_ACQUIRE);
}

uint64_t wait_blocking(void *sym, int cmp, uint64_t v, int is_signed)
{
    State &s = st();
    if (check_ready()) return 0;
    if (!sym_word(sym) || cmp < SHMEM_CMP_EQ || cmp > SHMEM_CMP_LE) {
        set_last_error(SHMEMX_ERR_ARG);
        return 0;
    }
    s.host_words[1] = 0;
    const uint64_t seq = ++g_done_seq;
    hipLaunchKernelGGL(k_host_wait, dim3(1), dim3(64), 0, s.host_stream, pub(), (uint64_t *)sym, cmp, v, is_signed,
                       s.host_words_dev + 1, s.host_words_dev + kDoneWord, seq);
    if (VSHMEM_HIP_FAILED(hipGetLastError())) {
        set_last_error(SHMEMX_ERR_HIP);
        return 0;
    }
    if (wait_done(seq)) return 0;
    return __atomic_load_n(&s.host_words[1], __ATOMIC_ACQUIRE);
}

int put_signal(void *dest, const void *source, size_t n, uint64_t *sig, uint64_t signal, int sig_op, int pe,
               hipStream_t stream)
{
    if (int rc = check_ready()) return rc;
    if (!sym_word(sig) || (sig_op != SHMEM_SIGNAL_SET && sig_op != SHMEM_SIGNAL_ADD)) return fail(SHMEMX_ERR_ARG);
    if (int rc = rma(true, dest, source, n, pe, stream)) return rc;
    // Stream order completes the data before the signal kernel starts.
    return amo_enqueue(sig_op == SHMEM_SIGNAL_SET ? HA_SIGNAL_SET : HA_SIGNAL_ADD, sig, pe, signal, 0, nullptr, stream);
}

int reduce_typed(shmem_team_t team, int dtype, int op, void *dest, const void *source, size_t n, hipStream_t stream)
{
    return shmemx_reduce_launch(team, dtype, op, dest, source, n, nullptr, stream);
}

void record(int rc)
{
    if (rc) set_last_error(rc);
}

}  // namespace

extern "C" {

// ----------------------------------------------------------- host, blocking
void shmem_putmem(void *dest, const void *source, size_t nelems, int pe)
{
    if (!rma(true, dest, source, nelems, pe, st().host_stream)) record(host_sync());
}

void shmem_getmem(void *dest, const void *source, size_t nelems, int pe)
{
    if (!rma(false, dest, source, nelems, pe, st().host_stream)) record(host_sync());
}

void shmem_putmem_nbi(void *dest, const void *source, size_t nelems, int pe)
{
    (void)rma(true, dest, source, nelems, pe, st().host_stream);
}

void shmem_getmem_nbi(void *dest, const void *source, size_t nelems, int pe)
{
    (void)rma(false, dest, source, nelems, pe, st().host_stream);
}

void shmem_putmem_signal(void *dest, const void *source, size_t nelems, uint64_t *sig_addr, uint64_t signal,
                         int sig_op, int pe)
{
    if (!put_signal(dest, source, nelems, sig_addr, signal, sig_op, pe, st().host_stream)) record(host_sync());
}

void shmem_putmem_signal_nbi(void *dest, const void *source, size_t nelems, uint64_t *sig_addr, uint64_t signal,
                             int sig_op, int pe)
{
    (void)put_signal(dest, source, nelems, sig_addr, signal, sig_op, pe, st().host_stream);
}

uint64_t shmem_signal_fetch(const uint64_t *sig_addr) { return amo_blocking(HA_FETCH, (void *)sig_addr, 0, 0, 0); }

uint64_t shmem_signal_wait_until(uint64_t *sig_addr, int cmp, uint64_t cmp_value)
{
    return wait_blocking(sig_addr, cmp, cmp_value, 0);
}

void shmem_int64_wait_until(int64_t *ivar, int cmp, int64_t cmp_value)
{
    (void)wait_blocking(ivar, cmp, (uint64_t)cmp_value, 1);
}

int shmem_int64_test(int64_t *ivar, int cmp, int64_t cmp_value)
{
    if (cmp < SHMEM_CMP_EQ || cmp > SHMEM_CMP_LE) {
        set_last_error(SHMEMX_ERR_ARG);
        return 0;
    }
    const int64_t x = (int64_t)amo_blocking(HA_FETCH, ivar, 0, 0, 0);
    switch (cmp) {
    case SHMEM_CMP_EQ: return x == cmp_value;
    case SHMEM_CMP_NE: return x != cmp_value;
    case SHMEM_CMP_GT: return x > cmp_value;
    case SHMEM_CMP_GE: return x >= cmp_value;
    case SHMEM_CMP_LT: return x < cmp_value;
    default: return x <= cmp_value;
    }
}

int64_t shmem_int64_atomic_fetch_add(int64_t *dest, int64_t value, int pe)
{
    return (int64_t)amo_blocking(HA_FETCH_ADD, dest, pe, (uint64_t)value, 0);
}
void shmem_int64_atomic_add(int64_t *dest, int64_t value, int pe)
{
    (void)amo_blocking(HA_FETCH_ADD, dest, pe, (uint64_t)value, 0);
}
int64_t shmem_int64_atomic_fetch_xor(int64_t *dest, int64_t value, int pe)
{
    return (int64_t)amo_blocking(HA_FETCH_XOR, dest, pe, (uint64_t)value, 0);
}
void shmem_int64_atomic_xor(int64_t *dest, int64_t value, int pe)
{
    (void)amo_blocking(HA_FETCH_XOR, dest, pe, (uint64_t)value, 0);
}
uint64_t shmem_uint64_atomic_fetch_xor(uint64_t *dest, uint64_t value, int pe)
{
    return amo_blocking(HA_FETCH_XOR, dest, pe, value, 0);
}
void shmem_uint64_atomic_xor(uint64_t *dest, uint64_t value, int pe) { (void)amo_blocking(HA_FETCH_XOR, dest, pe, value, 0); }
int64_t shmem_int64_atomic_compare_swap(int64_t *dest, int64_t cond, int64_t value, int pe)
{
    return (int64_t)amo_blocking(HA_CSWAP, dest, pe, (uint64_t)value, (uint64_t)cond);
}
int64_t shmem_int64_atomic_fetch(const int64_t *source, int pe)
{
    return (int64_t)amo_blocking(HA_FETCH, (void *)source, pe, 0, 0);
}
void shmem_int64_atomic_set(int64_t *dest, int64_t value, int pe)
{
    (void)amo_blocking(HA_SET, dest, pe, (uint64_t)value, 0);
}
int64_t shmem_int64_atomic_swap(int64_t *dest, int64_t value, int pe)
{
    return (int64_t)amo_blocking(HA_SWAP, dest, pe, (uint64_t)value, 0);
}

void shmem_quiet(void)
{
    if (!check_ready()) record(host_sync());
}

void shmem_fence(void) { (void)check_ready(); }

void shmem_barrier_all(void) { shmem_quiet(); }

void shmem_sync_all(void) { shmem_quiet(); }

int shmem_team_sync(shmem_team_t team)
{
    if (int rc = check_ready()) return rc;
    shmemx_dteam_t t;
    if (team_get(team, &t)) return fail(SHMEMX_ERR_ARG);
    if (int rc = host_sync()) return fail(rc);
    return SHMEMX_OK;
}

// Host collectives: the launcher on the context's stream, then completion.
#define VSHMEM_HOST_COLL(CALL)                                     \
    do {                                                           \
        if (int rc_ = check_ready()) return rc_;                   \
        if (int rc_ = (CALL)) return rc_;                          \
        if (int rc_ = host_sync()) return fail(rc_);               \
        return SHMEMX_OK;                                          \
    } while (0)

int shmem_broadcastmem(shmem_team_t team, void *dest, const void *source, size_t nelems, int PE_root)
{
    VSHMEM_HOST_COLL(shmemx_broadcastmem_launch(team, dest, source, nelems, PE_root, nullptr, st().host_stream));
}
int shmem_fcollectmem(shmem_team_t team, void *dest, const void *source, size_t nelems)
{
    VSHMEM_HOST_COLL(shmemx_fcollectmem_launch(team, dest, source, nelems, nullptr, st().host_stream));
}
int shmem_alltoallmem(shmem_team_t team, void *dest, const void *source, size_t nelems)
{
    VSHMEM_HOST_COLL(shmemx_alltoallmem_launch(team, dest, source, nelems, nullptr, st().host_stream));
}
int shmem_int64_sum_reduce(shmem_team_t team, int64_t *dest, const int64_t *source, size_t nreduce)
{
    VSHMEM_HOST_COLL(reduce_typed(team, SHMEMX_DT_INT64, SHMEMX_RED_SUM, dest, source, nreduce, st().host_stream));
}
int shmem_int64_max_reduce(shmem_team_t team, int64_t *dest, const int64_t *source, size_t nreduce)
{
    VSHMEM_HOST_COLL(reduce_typed(team, SHMEMX_DT_INT64, SHMEMX_RED_MAX, dest, source, nreduce, st().host_stream));
}
int shmem_float_sum_reduce(shmem_team_t team, float *dest, const float *source, size_t nreduce)
{
    VSHMEM_HOST_COLL(reduce_typed(team, SHMEMX_DT_FP32, SHMEMX_RED_SUM, dest, source, nreduce, st().host_stream));
}
int shmem_float_max_reduce(shmem_team_t team, float *dest, const float *source, size_t nreduce)
{
    VSHMEM_HOST_COLL(reduce_typed(team, SHMEMX_DT_FP32, SHMEMX_RED_MAX, dest, source, nreduce, st().host_stream));
}
int shmemx_bfloat16_sum_reduce(shmem_team_t team, uint16_t *dest, const uint16_t *source, size_t nreduce)
{
    VSHMEM_HOST_COLL(reduce_typed(team, SHMEMX_DT_BF16, SHMEMX_RED_SUM, dest, source, nreduce, st().host_stream));
}
int shmemx_bfloat16_max_reduce(shmem_team_t team, uint16_t *dest, const uint16_t *source, size_t nreduce)
{
    VSHMEM_HOST_COLL(reduce_typed(team, SHMEMX_DT_BF16, SHMEMX_RED_MAX, dest, source, nreduce, st().host_stream));
}
#undef VSHMEM_HOST_COLL

// ------------------------------------------------------------ stream order
int shmemx_putmem_on_stream(void *dest, const void *source, size_t nelems, int pe, void *stream)
{
    return rma(true, dest, source, nelems, pe, (hipStream_t)stream);
}

int shmemx_getmem_on_stream(void *dest, const void *source, size_t nelems, int pe, void *stream)
{
    return rma(false, dest, source, nelems, pe, (hipStream_t)stream);
}

int shmemx_putmem_signal_on_stream(void *dest, const void *source, size_t nelems, uint64_t *sig_addr,
                                   uint64_t signal, int sig_op, int pe, void *stream)
{
    return put_signal(dest, source, nelems, sig_addr, signal, sig_op, pe, (hipStream_t)stream);
}

int shmemx_signal_wait_until_on_stream(uint64_t *sig_addr, int cmp, uint64_t cmp_value, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!sym_word(sig_addr) || cmp < SHMEM_CMP_EQ || cmp > SHMEM_CMP_LE) return fail(SHMEMX_ERR_ARG);
    hipLaunchKernelGGL(k_host_wait, dim3(1), dim3(64), 0, (hipStream_t)stream, pub(), sig_addr, cmp, cmp_value, 0,
                       nullptr, nullptr, 0ull);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_barrier_all_on_stream(void *stream)
{
    return shmemx_barrier_launch(SHMEM_TEAM_WORLD, 1, UINT64_MAX, nullptr, nullptr, stream);
}

int shmemx_team_sync_on_stream(shmem_team_t team, void *stream)
{
    return shmemx_barrier_launch(team, 1, UINT64_MAX, nullptr, nullptr, stream);
}

int shmemx_quiet_on_stream(void *stream)
{
    (void)stream;
    return check_ready();
}

int shmemx_broadcastmem_on_stream(shmem_team_t team, void *dest, const void *source, size_t nelems, int PE_root,
                                  void *stream)
{
    return shmemx_broadcastmem_launch(team, dest, source, nelems, PE_root, nullptr, stream);
}

int shmemx_fcollectmem_on_stream(shmem_team_t team, void *dest, const void *source, size_t nelems, void *stream)
{
    return shmemx_fcollectmem_launch(team, dest, source, nelems, nullptr, stream);
}

int shmemx_alltoallmem_on_stream(shmem_team_t team, void *dest, const void *source, size_t nelems, void *stream)
{
    return shmemx_alltoallmem_launch(team, dest, source, nelems, nullptr, stream);
}

int shmemx_reduce_on_stream(shmem_team_t team, int dtype, int op, void *dest, const void *source, size_t nreduce,
                            void *stream)
{
    return reduce_typed(team, dtype, op, dest, source, nreduce, (hipStream_t)stream);
}

}  // extern "C"
