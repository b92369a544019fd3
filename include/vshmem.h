/*
 * vshmem: device-initiated OpenSHMEM on virtual PEs, for one MI355X (gfx950).
 *
 * Host C-ABI of libvshmem.so.  Every entry point is `extern "C"` and takes
 * plain pointers and sizes.  "Device pointer" means memory the HIP runtime
 * allocated on the GPU (hipMalloc or a PyTorch CUDA tensor); "host pointer"
 * means ordinary process memory.  A `void *stream` argument is a hipStream_t
 * (NULL = the default stream); every launcher is asynchronous on it.
 *
 * Virtual PEs.  One device allocation of npes * stride bytes is the
 * symmetric heap; PE p owns [base + p*stride, base + (p+1)*stride).  The
 * first `user_bytes` of each slice are allocatable; the tail holds the
 * library's per-PE scratch (barrier words).  A "canonical symmetric
 * address" is PE 0's copy of an object, base + offset; PE p's copy of the
 * object is that address + p*stride (the symmetric heap of the paper's
 * Section 2.1: same size and allocation order on every PE, so remote
 * addresses are computable; no per-operation pointer classification,
 * Section 6.3).
 *
 * Errors.  The paper leaves the error model to a later OpenSHMEM release
 * (Section 6.6).  Here: calls that return int give 0 (SHMEMX_OK) or a
 * negative SHMEMX_ERR_* code; allocators return NULL; OpenSHMEM calls that
 * return void record their failure for shmemx_last_error().  Device-side
 * failures (a wait that timed out, an out-of-heap descriptor) latch bits in
 * a device error word read by shmemx_device_errors().
 *
 * Threading.  Host calls are single-threaded except shmemx_progress_submit
 * and shmemx_progress_poll, which are safe from any number of threads.
 */
#ifndef VSHMEM_H
#define VSHMEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define SHMEMX_OK 0
#define SHMEMX_ERR_ARG (-1)         /* bad argument (range, NULL, alignment) */
#define SHMEMX_ERR_NOMEM (-2)       /* heap, budget or host memory exhausted */
#define SHMEMX_ERR_STATE (-3)       /* not initialised, already initialised, finalised */
#define SHMEMX_ERR_HIP (-4)         /* a HIP runtime call failed */
#define SHMEMX_ERR_BUSY (-5)        /* resource in use (progress kernel running, ring full) */
#define SHMEMX_ERR_TIMEOUT (-6)     /* a bounded wait expired */
#define SHMEMX_ERR_DEVICE (-7)      /* the device latched an error */
#define SHMEMX_ERR_UNSUPPORTED (-8) /* valid request this implementation does not provide */

/* Device error-word bits (shmemx_device_errors). */
#define SHMEMX_DEVERR_WAIT_TIMEOUT 0x1u   /* wait_until / barrier spin limit reached */
#define SHMEMX_DEVERR_BAD_DESC 0x2u       /* descriptor outside the heap or bad op */
#define SHMEMX_DEVERR_PROGRESS_IDLE 0x4u  /* progress kernel stopped by its idle limit */
#define SHMEMX_DEVERR_PROGRESS_STATE 0x8u /* progress kernel saw an inconsistent request record */
/* With VSHMEM_DEBUG set at init the device API checks its arguments; an
 * operation that fails a check latches one of these and does nothing. */
#define SHMEMX_DEVERR_BAD_ADDRESS 0x10u   /* operand outside the symmetric heap, misaligned word, PE out of range */
#define SHMEMX_DEVERR_NONUNIFORM 0x20u    /* participants of a _wave/_wg/_grid call passed different arguments */

/* -------------------------------------------------- operations and scopes
 * Operation codes of a descriptor (Section 2.1 operation list; put with
 * signal and signal wait from Section 4.3; fence/quiet from Section 6.4). */
#define SHMEMX_OP_NOP 0
#define SHMEMX_OP_PUT 1
#define SHMEMX_OP_GET 2
#define SHMEMX_OP_PUT_SIGNAL 3
#define SHMEMX_OP_AMO_FETCH_ADD 4
#define SHMEMX_OP_AMO_FETCH_XOR 5
#define SHMEMX_OP_AMO_COMPARE_SWAP 6
#define SHMEMX_OP_AMO_ADD 7
#define SHMEMX_OP_AMO_XOR 8
#define SHMEMX_OP_AMO_SET 9
#define SHMEMX_OP_AMO_FETCH 10
#define SHMEMX_OP_AMO_SWAP 11
#define SHMEMX_OP_WAIT_UNTIL 12
#define SHMEMX_OP_FENCE 13
#define SHMEMX_OP_QUIET 14
#define SHMEMX_OP_BARRIER_ALL 15

/* Participation scopes (Section 4.1 and Section 6.3: thread, wavefront,
 * work-group, grid; every thread of the scope calls with identical
 * arguments). */
#define SHMEMX_SCOPE_THREAD 0
#define SHMEMX_SCOPE_WAVE 1
#define SHMEMX_SCOPE_WG 2
#define SHMEMX_SCOPE_GRID 3
#define SHMEMX_SCOPE_AUTO 255     /* let the tune table pick per size class */

#define SHMEM_SIGNAL_SET 0
#define SHMEM_SIGNAL_ADD 1

#define SHMEM_CMP_EQ 0
#define SHMEM_CMP_NE 1
#define SHMEM_CMP_GT 2
#define SHMEM_CMP_GE 3
#define SHMEM_CMP_LT 4
#define SHMEM_CMP_LE 5

#define SHMEMX_NO_RESULT 0xFFFFFFFFu

/*
 * One operation, 64 bytes.  Heap locations are byte OFFSETS into the
 * symmetric heap (the same on every PE), not addresses.
 *   PUT:  target's [dst, dst+nbytes) <- issuer's [src, src+nbytes)
 *   GET:  issuer's [dst, dst+nbytes) <- target's [src, src+nbytes)
 *   PUT_SIGNAL: PUT, then the uint64 at target's `cond` is set to (aux =
 *         SHMEM_SIGNAL_SET) or increased by (SHMEM_SIGNAL_ADD) `value`.
 *   AMO_*: on the int64 at target's `src` (8-byte aligned); operand `value`;
 *         COMPARE_SWAP compares with `cond`; fetching AMOs write the old
 *         value to results[result_idx] unless result_idx == SHMEMX_NO_RESULT.
 *   WAIT_UNTIL: issuer waits until its int64 at `src` satisfies `aux`
 *         (SHMEM_CMP_*) against `value`; flags bit 0 = unsigned compare.
 *   FENCE, QUIET, BARRIER_ALL: ordering points of the issuing PE (barrier:
 *         of all PEs; every PE's program has the same number of them).
 */
typedef struct shmemx_desc {
    uint8_t op;
    uint8_t scope;
    uint8_t aux;
    uint8_t flags;
    int32_t issuer_pe;
    int32_t target_pe;
    uint32_t result_idx;
    uint64_t src;
    uint64_t dst;
    uint64_t nbytes;
    uint64_t value;
    uint64_t cond;
    uint64_t reserved;
} shmemx_desc_t;

/* ------------------------------------------------------------------ teams
 * Teams (Section 2.2; device teams of Section 4.1).  On one GPU the world
 * and shared teams have the same members: every virtual PE. */
typedef int32_t shmem_team_t;
#define SHMEM_TEAM_INVALID (-1)
#define SHMEM_TEAM_WORLD 0
#define SHMEM_TEAM_SHARED 1
#define SHMEM_DEVICE_TEAM_WORLD 2
#define SHMEM_DEVICE_TEAM_SHARED 3

/* What a kernel needs to address a team: members are the PEs start +
 * k * stride for k < size; slot selects the team's barrier words in the
 * scratch tail of its first member.  shmemx_team_device fills it on the
 * host; kernels take it by value. */
typedef struct {
    int32_t start;
    int32_t stride;
    int32_t size;
    int32_t slot;
} shmemx_dteam_t;

/* ------------------------------------------------------------ capabilities
 * Capability record (Section 6.5: queries distinguish host GPU-aware
 * support from device-initiated APIs, report stream variants separately,
 * report the active mode and the communication path).  Shape is ours. */
#define SHMEMX_PROGRESS_KERNEL_LAUNCH 0x1
#define SHMEMX_PROGRESS_PERSISTENT_GPU 0x2
#define SHMEMX_PATH_SINGLE_GPU_LOADSTORE 1
#define SHMEMX_PTR_DOMAIN_DEVICE 2

typedef struct shmemx_caps {
    int32_t gpu_heap;              /* 1: a GPU-attached symmetric heap exists */
    int32_t default_heap_is_gpu;   /* 1: GPU-first; shmem_malloc == shmemg_malloc */
    int32_t host_initiated;        /* 1: host-issued RMA, AMO, sync, collectives on GPU buffers */
    int32_t device_initiated;      /* 1: device-initiated RMA, AMO, sync */
    int32_t device_ctx_default;    /* 1: SHMEM_DEVICE_CTX_DEFAULT available */
    int32_t explicit_device_ctx;   /* 1: shmemx_device_ctx_create */
    uint32_t scopes;               /* bit (1 << SHMEMX_SCOPE_*) per supported scope */
    int32_t device_collectives;    /* 1 */
    int32_t stream_triggered;      /* 1: shmemx_*_on_stream host APIs */
    uint32_t progress;             /* SHMEMX_PROGRESS_* bits */
    int32_t path;                  /* SHMEMX_PATH_* */
    int32_t ptr_domain;            /* domain of shmem_ptr results */
    int32_t team_npes;             /* members of the queried team */
    int32_t team_start;
    int32_t team_stride;
    int32_t npes;                  /* virtual PEs */
    uint64_t heap_user_bytes;      /* allocatable bytes per PE */
    uint64_t heap_stride;          /* bytes between PE slices */
    int32_t debug;                 /* VSHMEM_DEBUG */
    int32_t max_device_ctx;        /* explicit device contexts that can be live at once */
    int32_t reserved[6];
} shmemx_caps_t;

/* ---------------------------------------------------- init and allocation */

/* Attach an existing device allocation as the symmetric heap (the paper's
 * GPU heap created at initialisation, Section 6.1; context creation and
 * publication of the device-visible default context, Section 6.2).
 * heap: device pointer, 2 MiB aligned, heap_bytes >= npes * 2 MiB and a
 * multiple of npes; stride = heap_bytes / npes must be a multiple of 2 MiB.
 * The caller keeps ownership of the memory and must keep it alive until
 * shmem_finalize.  The library clears its per-PE scratch tail on `stream`
 * and waits for it.  Returns SHMEMX_OK, SHMEMX_ERR_ARG, SHMEMX_ERR_STATE
 * (already initialised) or SHMEMX_ERR_HIP. */
int shmemx_init_attach(void *heap, size_t heap_bytes, int npes, void *stream);

/* Slice stride for PE slices with at least `bytes_per_pe` allocatable bytes
 * (host only; needs no device and no init).  spread = 0: the smallest,
 * bytes_per_pe plus the library's 64 KiB scratch tail, rounded up to 2 MiB.
 * spread = 1: the stride the library uses itself, and recommends for
 * shmemx_init_attach: when the smallest stride s lies in [2^k,
 * 1.5 * 2^k + 2 MiB) for some 2^k >= 64 MiB (a slice at or just above a
 * power of two, as most requested sizes are), it becomes 1.5 * 2^k + 2 MiB.  Members
 * of a team then sit at p * stride offsets that do not pile onto the same
 * HBM channels and banks: on MI355X a 64-member reduction over 1 GiB slices
 * ran at 5.03-5.07 TB/s with 1026 MiB apart and 6.04-6.06 TB/s with
 * 1538 MiB apart on each of four boxes, a broadcast at 5.63-5.66 against
 * 6.31-6.35 TB/s; copies between two slices were not affected.  The cost is
 * up to a third of the heap's memory.  Returns 0 when the stride would
 * overflow 64 bits. */
uint64_t shmemx_heap_stride_for(uint64_t bytes_per_pe, int spread);

/* OpenSHMEM initialisation (Section 6.1, heaps created at init with traits
 * from the environment): VSHMEM_NPES (default 4) virtual PEs with
 * VSHMEM_SYMMETRIC_SIZE allocatable bytes each (default 64 MiB; suffixes
 * K, M, G); the library allocates the heap with hipMalloc and owns it,
 * with slices shmemx_heap_stride_for(size, 1) apart (the smallest stride
 * when that much does not fit).  Failure is recorded for
 * shmemx_last_error(). */
void shmem_init(void);

/* Destroy the device context and release library resources (Section 6.2
 * context lifecycle: teardown at finalisation).  Every symmetric address,
 * plan and team becomes invalid. */
void shmem_finalize(void);

/* Number of virtual PEs; 0 before init. */
int shmem_n_pes(void);

/* On the host the calling thread acts for PE 0: returns 0 after init and
 * -1 before. */
int shmem_my_pe(void);

/* Symmetric allocation (Section 6.1: same size and order on every PE).
 * Returns a canonical symmetric address (device pointer into PE 0's slice),
 * aligned to 256 bytes, or NULL when size is 0 or the heap is exhausted.
 * First-fit over a coalescing free list, so the result depends only on the
 * sequence of calls.  shmemg_malloc is the paper's GPU-heap allocator; the
 * GPU heap is the default heap here, so the two are the same. */
void *shmem_malloc(size_t size);
void *shmemg_malloc(size_t size);
/* Zeroed allocation on every PE (waits for the clear). */
void *shmem_calloc(size_t count, size_t size);
/* Allocation aligned to `alignment` (a power of two >= 256). */
void *shmem_align(size_t alignment, size_t size);
/* Free a canonical symmetric address returned by an allocator; other
 * pointers are ignored and recorded as SHMEMX_ERR_ARG. */
void shmem_free(void *ptr);

/* PE `pe`'s copy of a symmetric object (Section 6.3 pointer queries).  The
 * result is a DEVICE pointer: valid for loads and stores in kernels, not on
 * the host (access domain reported as SHMEMX_PTR_DOMAIN_DEVICE).  NULL if
 * `sym` is not inside the heap or pe is out of range. */
void *shmem_ptr(const void *sym, int pe);
/* The team-scoped form (Section 6.3: a host-callable team pointer query
 * with a stated access domain): member `pe` of `team` (team numbering).
 * Same domain and NULL cases as shmem_ptr, plus NULL for a team that does
 * not exist. */
void *shmem_team_ptr(shmem_team_t team, const void *dest, int pe);

/* Capability query for a team (Section 6.5).  Returns SHMEMX_OK or an
 * error for an unknown team / NULL out. */
int shmem_query_capabilities(shmem_team_t team, shmemx_caps_t *caps);

/* Heap geometry: device base address, bytes per PE slice, allocatable bytes
 * per PE.  0 before init. */
void *shmemx_heap_base(void);
uint64_t shmemx_heap_stride(void);
uint64_t shmemx_heap_user_bytes(void);

/* Device pointer to the published device context (the GPU-visible
 * SHMEM_DEVICE_CTX_DEFAULT of Section 6.2), for user kernels that include
 * vshmem_device.hpp.  NULL before init. */
const void *shmemx_device_ctx(void);

/* Explicit device contexts (Section 6.2: created on the host, cached in
 * GPU-accessible memory, passed to kernels as device-visible handles;
 * Tier 1 of Section 7).  A context is created from a team: kernels bind it
 * with shmemx_dctx_bind_explicit (vshmem_device.hpp) and then number PEs in
 * that team, shmem_my_pe and shmem_n_pes answering for the team (the team
 * contexts of OpenSHMEM).  The published record is read-only, so one
 * context may be used by any number of threads, wavefronts and work-groups
 * at every scope at once.  Lifetime: from create to destroy or finalise;
 * destroy a context before its team, and not while kernels use it.
 * Ordering: fence and quiet of a caller order and complete its operations
 * through every context, not only the one named (on this part they are a
 * release of the caller's stores), which is stronger than the independent
 * ordering a context may have.  options: SHMEM_CTX_* bits, recorded for
 * kernels to read; they change nothing here.  At most SHMEMX_MAX_DEVICE_CTX
 * contexts are live at once (also reported by shmem_query_capabilities).
 * create returns SHMEMX_OK, SHMEMX_ERR_STATE, SHMEMX_ERR_ARG (bad team or
 * NULL out), SHMEMX_ERR_NOMEM (all in use) or SHMEMX_ERR_HIP.  record
 * returns the device address of the context's record, or NULL when the
 * handle is not live. */
typedef int32_t shmemx_ctx_t;
#define SHMEMX_CTX_INVALID (-1)
#define SHMEM_CTX_SERIALIZED 1L
#define SHMEM_CTX_PRIVATE 2L
#define SHMEM_CTX_NOSTORE 4L
#define SHMEMX_MAX_DEVICE_CTX 64
int shmemx_device_ctx_create(shmem_team_t team, long options, shmemx_ctx_t *ctx);
const void *shmemx_device_ctx_record(shmemx_ctx_t ctx);
void shmemx_device_ctx_destroy(shmemx_ctx_t ctx);

/* Strided team split (OpenSHMEM teams, Section 2.2): members are parent
 * members start, start+stride, ... (size of them).  config/config_mask are
 * accepted for OpenSHMEM signature compatibility and ignored.  On success
 * *new_team is a device team usable by the collective launchers. */
int shmem_team_split_strided(shmem_team_t parent, int start, int stride, int size,
                             const void *config, long config_mask, shmem_team_t *new_team);
int shmem_team_n_pes(shmem_team_t team);
/* Device descriptor of a live team, for user kernels that call the device
 * collectives and team barriers of vshmem_device.hpp.  Returns SHMEMX_OK,
 * SHMEMX_ERR_STATE before init, SHMEMX_ERR_ARG for a NULL out or a team
 * that does not exist.  The descriptor stays valid until the team is
 * destroyed or the library finalised. */
int shmemx_team_device(shmem_team_t team, shmemx_dteam_t *out);
/* Team index of PE `pe` in `team`, or -1 if it is not a member. */
int shmemx_team_pe_index(shmem_team_t team, int pe);
void shmem_team_destroy(shmem_team_t team);

/* Error reporting. */
const char *shmemx_strerror(int code);
/* Code of the most recent failure recorded on this thread (SHMEMX_OK if
 * none since the last clear); successful calls leave it unchanged. */
int shmemx_last_error(void);
/* Reset the recorded failure and its detail to SHMEMX_OK; for checking a
 * call that returns void. */
void shmemx_clear_last_error(void);
/* Detail of the most recent SHMEMX_ERR_HIP: returns the hipError_t code of
 * the HIP runtime call that failed (0 when the library itself refused, e.g.
 * a kernel that cannot be resident) and, when buf is not NULL, writes a
 * description into buf (truncated to len): "<name> (<code>) at
 * <source>:<line>: <call>" for a failed call. */
int shmemx_last_hip_error(char *buf, size_t len);
/* Read and clear the device error word (SHMEMX_DEVERR_* bits); waits for
 * the device.  Returns the bits, or a negative code if not initialised.
 * When SHMEMX_DEVERR_WAIT_TIMEOUT was latched, a barrier may have been left
 * with arrivals that never completed its phase, which would let the next
 * barrier on those words release one arrival early.  So, with the device
 * idle, the call then also clears every PE's scratch tail: every team's and
 * plan's barrier words restart at phase 0.  Calls waiting in other
 * processes' streams are not affected (one process owns the heap). */
int shmemx_device_errors(void);
/* Spin limit of device-side waits in nanoseconds (default 10 s).  A wait
 * that exceeds it gives up, latches SHMEMX_DEVERR_WAIT_TIMEOUT and returns,
 * so every kernel terminates. */
int shmemx_set_wait_timeout_ns(uint64_t ns);

/* ---------------------------------------------- device-initiated launches
 * Per-launch geometry.  NULL selects defaults.  wgs_per_pe: work-groups
 * that act for each virtual PE (a virtual PE is a heap slice plus the
 * work-groups the launcher maps to it: pe = blockIdx.x / wgs_per_pe).
 * wg_size: threads per work-group (multiple of 64, <= 1024).  chunk_bytes:
 * unit of work handed to one work-group when a message or collective is
 * split across work-groups (multiple of 16).  Zero fields take defaults;
 * for the team collectives wgs_per_pe = 0 means one work-group per member
 * per 512 KiB the member writes, at most one per CU over the team and never
 * more than stay co-resident. */
typedef struct shmemx_launch {
    int32_t wgs_per_pe;
    int32_t wg_size;
    uint64_t chunk_bytes;
    int32_t flags;                 /* SHMEMX_LAUNCH_* */
    int32_t reserved;
} shmemx_launch_t;
#define SHMEMX_LAUNCH_NONTEMPORAL 0x1  /* streaming loads/stores in copies */
#define SHMEMX_LAUNCH_DEEP 0x2         /* copies: 8 vectors in flight per lane instead of 4;
                                          reductions of teams below 128: two vectors per lane */

/*
 * Pattern put/get (device-initiated RMA, Section 6.3): every PE p with
 * targets[p] >= 0 issues nmsg messages of msg_bytes at the given scope:
 * message j moves [src_off + j*src_step, +msg_bytes) to
 * [dst_off + j*dst_step, +msg_bytes); for SHMEMX_OP_PUT the source is on p
 * and the destination on targets[p]; for SHMEMX_OP_GET the source is on
 * targets[p] and the destination on p.  Each PE ends with quiet.
 * Scope THREAD: each lane issues whole messages; WAVE: each wavefront; WG:
 * each work-group; GRID: all work-groups of the PE share each message.
 * targets: DEVICE pointer to npes int32.  Ranges must lie in the user part
 * of the heap and destinations must not overlap (the result would be
 * undefined); SHMEMX_ERR_ARG otherwise.
 */
int shmemx_rma_pattern(int op, int scope, const int32_t *targets, uint64_t src_off, uint64_t dst_off,
                       uint64_t msg_bytes, uint64_t nmsg, uint64_t src_step, uint64_t dst_step,
                       const shmemx_launch_t *launch, void *stream);

/*
 * Random-access atomics (GUPS-style; remote atomic updates of Section 4.4
 * case study 2, atomics of Section 2.1).  The table is 2^log2_table int64
 * words spread evenly over the PEs: global index g lives on PE
 * g >> (log2_table - log2(npes)) at heap offset table_off + 8*(g mod
 * per-PE entries); npes must be a power of two.  Update u (0 <= u <
 * nupdates) draws x_{3u}, x_{3u+1}, x_{3u+2} from the SplitMix64 stream
 * `seed`: index x_{3u} mod 2^log2_table, value x_{3u+1}, and it is
 * fetch_add when x_{3u+2} mod add_every == 0, else fetch_xor.  Update u is
 * issued by PE u / (nupdates / npes).  fetched: DEVICE array of nupdates
 * uint64 receiving each fetched value, or NULL; acc: DEVICE uint64 that
 * receives the XOR of all fetched values (so fetches are not elided), or
 * NULL.  Atomics are relaxed, agent scope (atomicity without ordering).
 */
int shmemx_gups(uint64_t table_off, int log2_table, uint64_t nupdates, uint64_t seed, int add_every,
                uint64_t *fetched, uint64_t *acc, const shmemx_launch_t *launch, void *stream);

/*
 * Signal ping-pong (put with signal and signal wait, Section 4.3 and the
 * wait/test operations of Section 2.1).  For pair k, PEs a = pairs[2k] and
 * b = pairs[2k+1]: in round r (1..rounds) a puts payload_bytes from its
 * [data_off] to b's [data_off] with signal SET r on b's uint64 at sig_off,
 * waits until its own signal equals r; b waits for r and answers the same
 * way.  rtt_cycles: DEVICE array of npairs*rounds uint64 receiving each
 * round trip in wall-clock ticks (see shmemx_wallclock_hz), or NULL.
 * same_xcd != 0 places both work-groups of a pair on one XCD, else on
 * different XCDs.  pairs: DEVICE int32 array.
 */
int shmemx_pingpong(uint64_t data_off, uint64_t sig_off, const int32_t *pairs, int npairs, int rounds,
                    uint64_t payload_bytes, int same_xcd, uint64_t *rtt_cycles, void *stream);

/* Device-side wait launched from the host (wait_until of Section 2.1): one
 * work-group acting for PE `pe` waits until its int64 at heap offset ivar_off
 * satisfies cmp (SHMEM_CMP_*) against value (unsigned compare when
 * is_unsigned), then writes the value it observed to *out (DEVICE pointer,
 * may be NULL).  The wait is bounded by the spin limit
 * (shmemx_set_wait_timeout_ns); on expiry it latches
 * SHMEMX_DEVERR_WAIT_TIMEOUT and the kernel ends. */
int shmemx_wait_until_launch(int pe, uint64_t ivar_off, int cmp, uint64_t value, int is_unsigned, uint64_t *out,
                             void *stream);

/* Frequency of the device wall clock used by timing outputs, in Hz. */
uint64_t shmemx_wallclock_hz(void);

/*
 * Team barrier (barrier_all / team_sync, Section 6.3; barrier implies
 * quiet): one work-group per member, `iters` consecutive barriers; with
 * tokens_off != UINT64_MAX each member writes a token (iteration, pe) to
 * every member's [tokens_off + 8*member] before each barrier and checks
 * after it that all tokens of that iteration are present, counting
 * failures into *bad (DEVICE uint64, may be NULL).  cycles: DEVICE uint64
 * receiving the total wall-clock ticks of member 0, or NULL.
 */
int shmemx_barrier_launch(shmem_team_t team, int iters, uint64_t tokens_off, uint64_t *bad,
                          uint64_t *cycles, void *stream);

/*
 * Team collectives executed by every member's work-groups (device
 * collectives with uniform participation, Section 6.3; the collectives
 * named in Section 4.3).  dest/src are canonical symmetric addresses; each
 * call starts and ends with a team barrier and implies quiet for its own
 * traffic.  Source and destination ranges must not overlap (except for
 * the reductions, which may run in place).
 *   broadcast: every member's dest[0, n) <- root member's src[0, n), the
 *              root's dest included; root is a team index.
 *   fcollect:  member p's dest[q*n, +n) <- member q's src[0, n).
 *   alltoall:  member p's dest[q*n, +n) <- member q's src[p*n, +n).
 *   reduce:    every member's dest[k] <- TREE(member 0's src[k], ...,
 *              member P-1's src[k]) where TREE pairs adjacent elements
 *              level by level and carries an odd last element; dtype int64
 *              (wrapping), fp32 (round-to-nearest-even adds), bf16 (inputs
 *              widened exactly to fp32, result rounded once to bf16); op
 *              SUM or MAX with max(a, b) = (b > a) ? b : a.
 * Every member's work-groups must be co-resident: the launch fails with
 * SHMEMX_ERR_ARG if team size * wgs_per_pe work-groups cannot be.
 * launch may be NULL; zero fields take the defaults: wgs_per_pe about one
 * work-group per CU in total, work-groups of 1024 threads (256 for the
 * reductions, which accept at most 256), chunk 256 KiB (reductions 16 KiB),
 * nontemporal copies for alltoall (8 deep) and the reductions.
 */
#define SHMEMX_DT_INT64 0
#define SHMEMX_DT_FP32 1
#define SHMEMX_DT_BF16 2
#define SHMEMX_RED_SUM 0
#define SHMEMX_RED_MAX 1
int shmemx_broadcastmem_launch(shmem_team_t team, void *dest, const void *src, size_t n, int root,
                               const shmemx_launch_t *launch, void *stream);
int shmemx_fcollectmem_launch(shmem_team_t team, void *dest, const void *src, size_t n,
                              const shmemx_launch_t *launch, void *stream);
int shmemx_alltoallmem_launch(shmem_team_t team, void *dest, const void *src, size_t n,
                              const shmemx_launch_t *launch, void *stream);
int shmemx_reduce_launch(shmem_team_t team, int dtype, int op, void *dest, const void *src, size_t nreduce,
                         const shmemx_launch_t *launch, void *stream);

/* --------------------------------------------- host-initiated operations
 * Tier 0 of Section 7: OpenSHMEM operations issued by the host on GPU-
 * resident symmetric objects, through the host default context (Section
 * 6.2).  The calling host thread acts for PE 0 (shmem_my_pe() == 0): a
 * canonical symmetric address used as a local operand names PE 0's copy.
 * Internal GPU kernels and copies on the context's own stream execute the
 * operations (Section 6.3 allows an implementation to accelerate host-
 * issued operations with internal kernels); the issuing agent, ordering and
 * progress contract remain those of the host API.
 *
 * Operands: `dest` of a put and `source` of a get are canonical symmetric
 * addresses, resolved on PE `pe`; the other buffer is any memory the HIP
 * runtime can copy (pageable or pinned host memory, device memory,
 * symmetric addresses).  Device-to-device moves run on a copy kernel;
 * moves that touch host memory use the runtime's copies.  AMO targets and
 * signal words are naturally aligned 8-byte symmetric words; a GPU kernel
 * performs each AMO at device (agent) scope, so host AMOs are atomic with
 * respect to device-initiated AMOs on the same word.
 *
 * Completion (Section 6.3 and the quiet table of Section 6.4): blocking
 * calls return at completion of the operation (stronger than the local
 * completion the paper requires; the data are visible device-wide on
 * return).  _nbi calls return after enqueueing; their buffers must stay
 * unchanged until shmem_quiet, which completes every operation the host
 * context issued and makes it visible device-wide.  shmem_fence orders
 * nothing more: the context executes its operations in issue order.
 * Host operations are not ordered with work on other streams: GPU work that
 * writes a local buffer or a symmetric source must have completed (stream
 * synchronised) before the call, a kernel that consumes host-put data must
 * be launched after shmem_quiet returns (or after the blocking call), and
 * host reads of device-written data need the writing kernel to have
 * finished.
 *
 * Collectives and barriers: the host thread acts for every member at once
 * (all virtual PEs live in this process), so a host collective performs
 * the whole collective, on the context's stream, and returns when it is
 * complete on every member.  shmem_barrier_all / shmem_sync_all /
 * shmem_team_sync complete the host context's operations (quiet); no other
 * agent has to arrive.  Host and device collectives on one team share its
 * barrier words: running them concurrently is undefined (Section 6.3).
 *
 * Errors: calls before init, non-symmetric operands, out-of-range PEs or
 * misaligned words set shmemx_last_error() (SHMEMX_ERR_STATE or
 * SHMEMX_ERR_ARG) and do nothing; fetching calls then return 0.  Integer
 * returning calls return 0 on success and the negative code otherwise.
 */
void shmem_putmem(void *dest, const void *source, size_t nelems, int pe);
void shmem_getmem(void *dest, const void *source, size_t nelems, int pe);
void shmem_putmem_nbi(void *dest, const void *source, size_t nelems, int pe);
void shmem_getmem_nbi(void *dest, const void *source, size_t nelems, int pe);
/* Put, then update PE pe's signal word sig_addr (SHMEM_SIGNAL_SET or
 * SHMEM_SIGNAL_ADD) once the data are complete (Section 4.3 put-with-signal). */
void shmem_putmem_signal(void *dest, const void *source, size_t nelems, uint64_t *sig_addr, uint64_t signal,
                         int sig_op, int pe);
void shmem_putmem_signal_nbi(void *dest, const void *source, size_t nelems, uint64_t *sig_addr, uint64_t signal,
                             int sig_op, int pe);
/* The host PE's (PE 0's) signal word. */
uint64_t shmem_signal_fetch(const uint64_t *sig_addr);
/* Wait until PE 0's word satisfies cmp (SHMEM_CMP_*) against cmp_value and
 * return the value seen (unsigned compare for signals, signed for int64).
 * A GPU kernel on the context's stream polls the word; the wait is bounded
 * by shmemx_set_wait_timeout_ns, after which SHMEMX_DEVERR_WAIT_TIMEOUT is
 * latched and the last value seen is returned. */
uint64_t shmem_signal_wait_until(uint64_t *sig_addr, int cmp, uint64_t cmp_value);
void shmem_int64_wait_until(int64_t *ivar, int cmp, int64_t cmp_value);
/* 1 if PE 0's word satisfies cmp now, else 0. */
int shmem_int64_test(int64_t *ivar, int cmp, int64_t cmp_value);
/* Atomics on PE pe's copy of dest (Section 2.1; relaxed, agent scope). */
int64_t shmem_int64_atomic_fetch_add(int64_t *dest, int64_t value, int pe);
void shmem_int64_atomic_add(int64_t *dest, int64_t value, int pe);
int64_t shmem_int64_atomic_fetch_xor(int64_t *dest, int64_t value, int pe);
void shmem_int64_atomic_xor(int64_t *dest, int64_t value, int pe);
uint64_t shmem_uint64_atomic_fetch_xor(uint64_t *dest, uint64_t value, int pe);
void shmem_uint64_atomic_xor(uint64_t *dest, uint64_t value, int pe);
int64_t shmem_int64_atomic_compare_swap(int64_t *dest, int64_t cond, int64_t value, int pe);
int64_t shmem_int64_atomic_fetch(const int64_t *source, int pe);
void shmem_int64_atomic_set(int64_t *dest, int64_t value, int pe);
int64_t shmem_int64_atomic_swap(int64_t *dest, int64_t value, int pe);
void shmem_quiet(void);
void shmem_fence(void);
void shmem_barrier_all(void);
void shmem_sync_all(void);
int shmem_team_sync(shmem_team_t team);
/* Collectives with the meanings of the launchers above (team-relative
 * root; n in bytes for the data-movement routines, in elements for the
 * reductions), run with the launchers' default shapes. */
int shmem_broadcastmem(shmem_team_t team, void *dest, const void *source, size_t nelems, int PE_root);
int shmem_fcollectmem(shmem_team_t team, void *dest, const void *source, size_t nelems);
int shmem_alltoallmem(shmem_team_t team, void *dest, const void *source, size_t nelems);
int shmem_int64_sum_reduce(shmem_team_t team, int64_t *dest, const int64_t *source, size_t nreduce);
int shmem_int64_max_reduce(shmem_team_t team, int64_t *dest, const int64_t *source, size_t nreduce);
int shmem_float_sum_reduce(shmem_team_t team, float *dest, const float *source, size_t nreduce);
int shmem_float_max_reduce(shmem_team_t team, float *dest, const float *source, size_t nreduce);
/* bf16 passed as its 16-bit pattern; fp32 accumulation, one rounding. */
int shmemx_bfloat16_sum_reduce(shmem_team_t team, uint16_t *dest, const uint16_t *source, size_t nreduce);
int shmemx_bfloat16_max_reduce(shmem_team_t team, uint16_t *dest, const uint16_t *source, size_t nreduce);

/* ------------------------------------------- stream-triggered operations
 * Tier 2 of Section 7 (Section 6.4): host-issued operations whose execution
 * is ordered in the caller's HIP stream `stream` (NULL = the null stream).
 * Each call enqueues and returns; the operation runs after everything
 * enqueued on the stream before it and completes before anything enqueued
 * after it starts, so a consumer later on the same stream sees its results
 * without further calls.  The host observes completion by synchronising
 * the stream.  The issuing agent is the host, as for the blocking calls
 * (PE 0 for local operands).  With pageable host memory as an operand the
 * runtime may stage the copy before the call returns.
 *
 * Prohibited patterns (Section 6.4 requires them to be documented):
 *   - a wait on a stream whose condition only work enqueued later on the
 *     same stream satisfies: it can never complete; the spin limit ends it
 *     with SHMEMX_DEVERR_WAIT_TIMEOUT;
 *   - a wait satisfied by work on another stream that is itself ordered
 *     after the waiting stream (through events or the null stream): same;
 *   - collectives or barriers of one team in flight on two streams at once,
 *     or concurrently with device collectives of that team: they share the
 *     team's barrier words (undefined, as in Section 6.3);
 *   - a collective whose members' work-groups cannot be co-resident with
 *     other kernels running at the same time on other streams: its barriers
 *     wait for work-groups that cannot start (bounded by the spin limit).
 * Returns 0 on success or a negative SHMEMX_ERR_* code (nothing enqueued).
 */
int shmemx_putmem_on_stream(void *dest, const void *source, size_t nelems, int pe, void *stream);
int shmemx_getmem_on_stream(void *dest, const void *source, size_t nelems, int pe, void *stream);
int shmemx_putmem_signal_on_stream(void *dest, const void *source, size_t nelems, uint64_t *sig_addr,
                                   uint64_t signal, int sig_op, int pe, void *stream);
/* Blocks the stream until PE 0's signal word satisfies cmp. */
int shmemx_signal_wait_until_on_stream(uint64_t *sig_addr, int cmp, uint64_t cmp_value, void *stream);
/* A team barrier (one work-group per member) ordered in the stream. */
int shmemx_barrier_all_on_stream(void *stream);
int shmemx_team_sync_on_stream(shmem_team_t team, void *stream);
/* Nothing to enqueue: stream order already completes every earlier
 * operation before later ones start.  Validates and returns 0. */
int shmemx_quiet_on_stream(void *stream);
int shmemx_broadcastmem_on_stream(shmem_team_t team, void *dest, const void *source, size_t nelems, int PE_root,
                                  void *stream);
int shmemx_fcollectmem_on_stream(shmem_team_t team, void *dest, const void *source, size_t nelems, void *stream);
int shmemx_alltoallmem_on_stream(shmem_team_t team, void *dest, const void *source, size_t nelems, void *stream);
/* dtype SHMEMX_DT_*, op SHMEMX_RED_*. */
int shmemx_reduce_on_stream(shmem_team_t team, int dtype, int op, void *dest, const void *source, size_t nreduce,
                            void *stream);

/* ---------------------------------------------------- batched execution
 * A plan is a program of descriptors prepared once and launched many times.
 * Each PE's program is the subsequence of descriptors it issues, in order.
 * Operations between two ordering points of their issuer (fence, quiet,
 * barrier_all) may run concurrently; results equal issuing the operations
 * one at a time (operations in one such phase must not conflict).
 * WAIT_UNTIL is not accepted in plans (SHMEMX_ERR_UNSUPPORTED); use the
 * device API or the progress kernel.  Forms: one fused launch, one launch
 * per operation, or either form captured in a hipGraph.
 */
#define SHMEMX_TUNE_CLASSES 40
typedef struct shmemx_tune {
    int32_t wg_size;                          /* threads per work-group of the fused kernel */
    int32_t grid_wgs;                         /* cap on fused work-groups (0 = automatic) */
    uint8_t scope[SHMEMX_TUNE_CLASSES];       /* scope per floor(log2(nbytes)) class */
    uint64_t chunk[SHMEMX_TUNE_CLASSES];      /* bytes per work-group task per class */
} shmemx_tune_t;

typedef struct shmemx_plan shmemx_plan_t;

/* Fill a tune table with the built-in defaults. */
void shmemx_tune_default(shmemx_tune_t *tune);

/* The library's ACTIVE tune table: the work-group size and grid cap of the
 * device-table launchers below, and the per-class scope and chunk they use
 * when the caller passes no table of its own.  At initialisation it is the
 * table that the file named by VSHMEM_TUNE_FILE holds, when that file loads
 * (shmemx_tune_load: saved on this kind of device, valid), else the built-in
 * defaults.  shmemx_tune_set waits for the device to go idle, then replaces
 * it (SHMEMX_ERR_ARG for an invalid table: work-group size not a multiple of
 * 64 in [64, 1024], negative grid cap, unknown scope).  shmemx_tune_get
 * copies it out and returns where it came from (SHMEMX_TUNE_SRC_*), or a
 * negative error. */
#define SHMEMX_TUNE_SRC_DEFAULT 0
#define SHMEMX_TUNE_SRC_FILE 1
#define SHMEMX_TUNE_SRC_FILE_REFUSED 2   /* VSHMEM_TUNE_FILE was set but refused: defaults */
#define SHMEMX_TUNE_SRC_SET 3
int shmemx_tune_set(const shmemx_tune_t *tune);
int shmemx_tune_get(shmemx_tune_t *tune);
/* Build a plan from HOST descriptors (copied).  tune may be NULL.
 * Validates every descriptor (ranges inside the user heap, PEs, op codes,
 * equal barrier counts) and returns SHMEMX_ERR_ARG with no plan otherwise.
 * Returns SHMEMX_ERR_UNSUPPORTED when no work-group of tune->wg_size threads
 * of the fused kernel can be resident on a CU (shmemx_last_hip_error says
 * why). */
int shmemx_plan_create(const shmemx_desc_t *descs, size_t n, const shmemx_tune_t *tune, shmemx_plan_t **plan);
/* One fused launch of the whole plan.  results: DEVICE uint64 array with
 * room for every result index used, or NULL if none.  Each plan has grid
 * barrier words of its own, so fused launches of DIFFERENT plans may run at
 * the same time on different streams, provided their grids fit the device
 * together (cap them with tune->grid_wgs): work-groups of a multi-phase
 * launch wait for each other.  Launches of ONE plan must be ordered (same
 * stream, or synchronised): they share its barrier words.  A multi-phase
 * plan whose grid does not fit the CUs the running progress kernel leaves
 * free is refused with SHMEMX_ERR_BUSY (nothing is launched). */
int shmemx_plan_launch_fused(shmemx_plan_t *plan, uint64_t *results, void *stream);
/* One kernel launch per operation, in program order. */
int shmemx_plan_launch_per_op(shmemx_plan_t *plan, uint64_t *results, void *stream);
/* Capture form 0 (per-op) or 1 (fused) into a hipGraph bound to `results`. */
int shmemx_plan_graph_build(shmemx_plan_t *plan, int form, uint64_t *results, void *stream);
int shmemx_plan_graph_launch(shmemx_plan_t *plan, void *stream);
/* Measurement mode: when stamps (DEVICE uint64 array with one entry per
 * descriptor of the plan, zeroed by the caller) is non-NULL, every later
 * launch of the plan (fused or per-op; graphs capture the setting at build
 * time) records for descriptor i, once its operation has completed, the
 * device wall clock into stamps[i] (the latest of its work-groups).
 * NULL turns it off. */
int shmemx_plan_set_stamps(shmemx_plan_t *plan, uint64_t *stamps);
/* Record the device wall clock into *dst (DEVICE) when the stream reaches
 * this point: the start reference for completion stamps. */
int shmemx_stamp_launch(uint64_t *dst, void *stream);
/* Number of fused work-group tasks / phases / kernel launches per per-op run. */
int shmemx_plan_info(const shmemx_plan_t *plan, uint64_t *ntasks, uint64_t *nphases, uint64_t *nlaunches);
void shmemx_plan_destroy(shmemx_plan_t *plan);

/* Autotuner.  For each work-group size of the fused kernel (64, 128, 256,
 * 512, 1024; sizes that cannot be resident are skipped) it first picks, per
 * size class from min_bytes to max_bytes (powers of two), the fastest
 * (scope, chunk) on `msgs` isolated puts of that class at that work-group
 * size; it then scores complete tables -- that tuned table, the three
 * uniform-scope tables and the built-in default, each at that work-group
 * size -- on a served mix shaped like a mixed program: `msgs` put/get with
 * sizes uniform in [min_bytes, max_bytes] between random PEs in eight
 * epochs separated by barriers, then 10 * msgs contended fetch_add on 64
 * counters.  Each table's score is the median of max(reps, 9) fused
 * launches of the mix; the four best are scored again in five interleaved
 * rounds and the one with the lowest total is returned (the built-in table
 * when no work-group size is resident).  All traffic stays in
 * the user heap range [scratch_off, scratch_off + scratch_bytes) of every PE,
 * whose contents are overwritten; scratch_bytes >= 2 * max_bytes + 1024.
 * Synchronous. */
int shmemx_autotune(uint64_t scratch_off, uint64_t scratch_bytes, uint64_t min_bytes, uint64_t max_bytes,
                    int msgs, int reps, shmemx_tune_t *tune, void *stream);
/* Save / load a tune table as JSON keyed by the device name (the HIP
 * architecture name, e.g. gfx950:sramecc+:xnack-).  Load refuses a file
 * saved on another kind of device, or without a device key, and an invalid
 * table (SHMEMX_ERR_ARG; *tune unchanged). */
int shmemx_tune_save(const shmemx_tune_t *tune, const char *path);
int shmemx_tune_load(shmemx_tune_t *tune, const char *path);

/* ------------------------------------- batches over a DEVICE descriptor table
 * The same program semantics as plans (each PE's program is the subsequence
 * of descriptors it issues; an operation's phase is its issuer's count of
 * barriers and of fences/quiets since the last barrier; phases run in
 * order, operations inside one run concurrently and must not conflict), but
 * the table is in DEVICE memory and is read on the device at every launch:
 * a kernel may write it, and a graph replays whatever it holds when the
 * replay runs.  Long-lived kernels that consume descriptor tables are the
 * paper's Section 3 case for device-side batching; the launches are
 * stream-ordered (Section 4.3).
 *
 *   d_descs   DEVICE array of n descriptors (caller-owned; it must not change
 *             while a launch reading it runs).
 *   d_results DEVICE uint64 array of n entries, or NULL: fetching atomics
 *             write results[result_idx] (result_idx < n, or SHMEMX_NO_RESULT).
 *   d_tune    DEVICE tune table for scope and chunk per size class, or NULL
 *             for the active table (shmemx_tune_set).  Work-group size and
 *             grid cap always come from the active table.
 *
 * Descriptors the device finds invalid (op code, PEs, ranges outside the
 * user heap, misaligned words, WAIT_UNTIL, result index >= n) are skipped
 * and latch SHMEMX_DEVERR_BAD_DESC; unequal barrier counts across the PEs'
 * programs latch it and run nothing.  Host-side errors: SHMEMX_ERR_ARG
 * (NULL table with n > 0, n > 2^26), SHMEMX_ERR_UNSUPPORTED (more than 4096
 * PEs: the ordering state of the index kernel is per PE), SHMEMX_ERR_BUSY
 * (no CU free next to the progress kernel), SHMEMX_ERR_HIP.
 *
 * shmemx_launch_batch: the fused form.  A classify kernel (one thread per
 * descriptor) validates and resolves scopes and chunks; an index kernel (one
 * work-group) derives phases and a counting sort by (phase, kind), both in a
 * workspace the library keeps per stream (grown on demand; growing
 * synchronises that stream); an executor of up to grid-cap work-groups takes
 * each phase's tasks round robin, with a grid barrier between phases.
 * Launches on one stream are ordered; launches on different streams use
 * different workspaces and must fit the device together.
 * shmemx_launch_per_op: one kernel launch per descriptor, in table order
 * (stream order is the ordering; fence/quiet/barrier descriptors launch
 * nothing).
 * shmemx_graph_build: capture form 0 (per-op) or 1 (fused, with a workspace
 * of the graph's own) into a graph; shmemx_graph_launch replays it on any
 * stream (replays of one graph must be ordered); shmemx_graph_destroy frees
 * it. */
typedef struct shmemx_graph shmemx_graph_t;
int shmemx_launch_batch(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results, const shmemx_tune_t *d_tune,
                        void *stream);
int shmemx_launch_per_op(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results, const shmemx_tune_t *d_tune,
                         void *stream);
int shmemx_graph_build(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results, const shmemx_tune_t *d_tune,
                       int form, shmemx_graph_t **graph);
int shmemx_graph_launch(shmemx_graph_t *graph, void *stream);
void shmemx_graph_destroy(shmemx_graph_t *graph);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): shmemx_launch_batch
 * with the same arguments, results and errors, whose workspace is a fixed
 * 4 MiB array in device memory instead of a per-stream allocation.  It calls
 * no hipMalloc or hipFree.  The array is set up at initialisation; each
 * device holds its own until the process ends.  Tables of at most
 * shmemx_launch_batch_noalloc_max() descriptors (SHMEMX_ERR_ARG above).
 * Every call on a device shares the array and keeps what the last call left
 * there (the index kernel clears what it needs): calls that overlap on one
 * device race and must be ordered by the caller (one stream, or
 * synchronised). */
int shmemx_launch_batch_noalloc(const shmemx_desc_t *d_descs, size_t n, uint64_t *d_results,
                                const shmemx_tune_t *d_tune, void *stream);
uint64_t shmemx_launch_batch_noalloc_max(void);

/* ------------------------------------------------------------- serving
 * Persistent progress kernel (long-lived kernels, Section 3; GPU-driven
 * progress, Section 6.4 and Section 7).  Host threads submit descriptors
 * (PUT, GET, AMO_FETCH_ADD with nbytes/8 counters) into a ring in pinned
 * host memory.  Work-group 0's first wavefront is the front-end: it takes
 * published requests in ticket order and splits each into chunks of
 * chunk_bytes times the number of chunks queued per worker (at least 1, at
 * most 8); every other work-group is a worker that claims one chunk at a
 * time and executes it with all its threads.  The worker finishing a
 * request's last chunk quiets and posts the completion record.  The kernel
 * exits when stopped or after idle_timeout_ms without work.
 */
typedef struct shmemx_progress_cfg {
    int32_t nwg;              /* work-groups, >= 2 (0 = one per CU) */
    int32_t wg_size;          /* threads per work-group (0 = 1024) */
    int32_t ring_slots;       /* power of two */
    int32_t verify;           /* 1: completion carries a hash of the output */
    uint64_t chunk_bytes;     /* split unit for large requests, multiple of 16, at most
                                 2^40 (0 = 256 KiB); up to 8x under backlog */
    uint64_t idle_timeout_ms; /* 0 = 30000 */
} shmemx_progress_cfg_t;

typedef struct shmemx_completion {
    uint64_t ticket;
    uint64_t t_start;         /* device wall clock when a worker first claimed it */
    uint64_t t_end;           /* device wall clock at completion */
    uint64_t hash;            /* output hash when verify is on */
    int32_t status;           /* 0 ok */
    int32_t lane;             /* producer lane the request was submitted on */
    uint64_t t_queued;        /* device wall clock when the front-end took it from the ring */
    uint64_t submit_ns;       /* serving runs: host ns from arrival to ring publish; else 0 */
} shmemx_completion_t;

int shmemx_progress_start(const shmemx_progress_cfg_t *cfg, void *stream);
/* Multi-producer: enqueue one request from producer lane `lane` (0 <= lane <
 * SHMEMX_PROGRESS_LANES: the host streams of arrivals); *ticket identifies
 * it and its completion record carries the lane.  Requests are independent
 * (they must not overlap other requests in flight) and may complete in any
 * order, also within one lane.  AMO fetch results go to the issuer's [dst,
 * dst + nbytes).  The descriptor's `reserved` field is ignored.  Returns
 * SHMEMX_ERR_BUSY when the ring is full, SHMEMX_ERR_ARG for a bad lane or
 * NULL pointers, SHMEMX_ERR_STATE when the kernel is not running. */
#define SHMEMX_PROGRESS_LANES 8
int shmemx_progress_submit(int lane, const shmemx_desc_t *desc, uint64_t *ticket);
/* 1 = complete (out filled), 0 = not yet, <0 = error.  The first poll that
 * sees a request complete consumes its completion record and frees its ring
 * slot; later polls of the same ticket return 1 with only `ticket` set.
 * Every submitted ticket must be polled to completion, or the ring fills. */
int shmemx_progress_poll(uint64_t ticket, shmemx_completion_t *out);
/* Stop the kernel after it drains the ring; waits up to timeout_ms. */
int shmemx_progress_stop(int timeout_ms);

/*
 * Trace-driven serving run in native code: `lanes` producer threads replay
 * the requests at their arrival times (seconds from start), admission
 * reserves each request's destination range from a per-PE first-fit list
 * inside [region_off, region_off + region_bytes) under a total budget of
 * budget_bytes (requests wait while it is exceeded), a completion thread
 * frees reservations as requests finish (continuous batching).  Sources
 * are read from [src_off, ...) as given.  Fills latency_ns[i] (arrival to
 * observed completion) and completions[i].  The progress kernel must be
 * running.  Returns SHMEMX_OK or an error.
 */
typedef struct shmemx_request {
    int32_t op;               /* SHMEMX_OP_PUT / GET / AMO_FETCH_ADD */
    int32_t issuer_pe;
    int32_t target_pe;
    int32_t lane;
    uint64_t nbytes;
    uint64_t src_off;         /* source offset (read-only region) */
    double arrival_s;
} shmemx_request_t;

typedef struct shmemx_serve_stats {
    double wall_s;
    uint64_t bytes;
    uint64_t amo_ops;
    uint64_t max_reserved_bytes;
    uint64_t admission_waits;
    uint64_t ring_full_retries;   /* submissions refused because the ring was full */
} shmemx_serve_stats_t;

int shmemx_serve_run(const shmemx_request_t *reqs, size_t n, int lanes, uint64_t region_off,
                     uint64_t region_bytes, uint64_t budget_bytes, uint64_t *dst_off_out,
                     uint64_t *latency_ns, shmemx_completion_t *completions, shmemx_serve_stats_t *stats);

/* The per-op serving form, for comparison on the same trace: the same
 * producers, admission, destinations and latency accounting as
 * shmemx_serve_run, but each request is one kernel launch
 * (shmemx_launch_request with chunk_bytes / wg_size) on a stream of its
 * producer lane's own, complete when an event recorded after it is.  The
 * progress kernel must not be running (SHMEMX_ERR_STATE).  completions[i]
 * carries only ticket = i (status 0, no hash, no device stamps).  A request's
 * destination is reused only after it completed, so the final contents of a
 * destination byte are those of the last request, by completion time
 * (arrival_s + latency), whose range covers it. */
int shmemx_serve_run_per_op(const shmemx_request_t *reqs, size_t n, int lanes, uint64_t region_off,
                            uint64_t region_bytes, uint64_t budget_bytes, uint64_t chunk_bytes, int wg_size,
                            uint64_t *dst_off_out, uint64_t *latency_ns, shmemx_completion_t *completions,
                            shmemx_serve_stats_t *stats);

/* Windowed batch serving forms on the same trace, admission and accounting
 * as shmemx_serve_run: a dispatcher thread gathers the requests submitted
 * while the oldest one waits window_ns (or up to 4096 of them), and launches
 * them as one batch: a kernel stages the batch from pinned host memory to
 * device memory, and a second, with one work-group of wg_size threads per CU,
 * executes every chunk of chunk_bytes of every request.  use_graph = 0
 * launches the two kernels directly (fused form); 1 replays a graph captured
 * once for each of the 4 batch slots (graph form).  Up to 4 batches are in
 * flight; a request completes with its batch.  The progress kernel must not
 * be running.  completions[i] carries only ticket = i. */
int shmemx_serve_run_batched(const shmemx_request_t *reqs, size_t n, int lanes, uint64_t region_off,
                             uint64_t region_bytes, uint64_t budget_bytes, uint64_t window_ns, int use_graph,
                             uint64_t chunk_bytes, int wg_size, uint64_t *dst_off_out, uint64_t *latency_ns,
                             shmemx_completion_t *completions, shmemx_serve_stats_t *stats);

/* One serving request (PUT, GET, or AMO_FETCH_ADD over nbytes/8 counters with
 * results to the issuer's dst) executed by a launch of its own: work-group
 * b moves bytes [b*chunk_bytes, (b+1)*chunk_bytes).  Asynchronous on stream. */
int shmemx_launch_request(const shmemx_desc_t *desc, uint64_t chunk_bytes, int wg_size, void *stream);

/* ------------------------------------------------------------ utilities */
/* Fill device memory with bytes [word_offset*8, ...) of the SplitMix64
 * stream `seed` (little-endian words): the seeded synthetic payload. */
int shmemx_fill_random(void *dst, uint64_t nbytes, uint64_t seed, uint64_t word_offset, void *stream);
/* Fill `count` elements of type dtype (SHMEMX_DT_INT64, SHMEMX_DT_FP32,
 * SHMEMX_DT_BF16) from SplitMix64 outputs index0, index0+1, ... of `seed`:
 * int64 = the raw output; fp32 = ((x >> 40) * 2^-24) * 2 - 1 (uniform in
 * [-1, 1), exact); bf16 = that fp32 rounded to nearest even.  dst must be
 * aligned to the element size. */
int shmemx_fill_typed(void *dst, uint64_t count, int dtype, uint64_t seed, uint64_t index0, void *stream);
/* Plain device-to-device copy kernel of nbytes (16-byte aligned) used as
 * the achievable-bandwidth probe and as the counter-scaling reference:
 * nwg work-groups of wg_size threads stream 16 MiB chunks (dealt round
 * robin) with nontemporal 16-byte loads and stores, 8 in flight per lane
 * (256 x 1024 was the fastest shape measured on MI355X). */
int shmemx_probe_copy(void *dst, const void *src, uint64_t nbytes, int nwg, int wg_size, void *stream);
/* HBM rate probes on DEVICE buffers of nbytes (a multiple of 16, 16-byte
 * aligned): a copy of src to dst in 16 MiB chunks per work-group (the
 * copy probe above), as one grid-stride sweep, or in tiles of 8 vectors per
 * lane dealt round robin; a read-only stream of src (its words folded into
 * the DEVICE word *acc); a write-only stream to dst.  nwg work-groups of
 * wg_size threads.  Timing references for the copy-shaped rows: a copy
 * reads and writes every byte, so its rate is set against the read and
 * write rates.  Asynchronous on stream; SHMEMX_ERR_ARG for a bad kind or
 * buffer. */
#define SHMEMX_PROBE_COPY_CHUNKED 0
#define SHMEMX_PROBE_COPY_GRIDSTRIDE 1
#define SHMEMX_PROBE_COPY_TILES 2
#define SHMEMX_PROBE_READ 3
#define SHMEMX_PROBE_WRITE 4
int shmemx_probe_hbm(int kind, void *dst, const void *src, uint64_t nbytes, int nwg, int wg_size, uint32_t *acc,
                     void *stream);
/* Agent-scope int64 fetch_add to random words of a DEVICE table of nwords
 * (a power of two): atomic-throughput probe. */
int shmemx_probe_atomics(uint64_t *table, uint64_t nwords, uint64_t nupdates, uint64_t seed, uint64_t *acc,
                         void *stream);
/* XCD id (hardware register XCC_ID) of each of nblocks work-groups. */
int shmemx_probe_xcd(int32_t *out, int nblocks, void *stream);
/* Empty kernel: launch-latency probe. */
int shmemx_probe_empty(void *stream);

/* Library version string. */
const char *shmemx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VSHMEM_H */
