// Batched execution of descriptor programs: one fused launch, one launch per
// operation, or either captured in a hipGraph.  A plan splits the program
// into phases at its ordering points; inside a phase, operations are
// independent and become work-group tasks (packs of thread- or
// wavefront-scope operations, or byte ranges of work-group-scope messages).
#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

#include "exec.hpp"
#include "runtime.hpp"

using namespace vshmem;

struct PlanTask {
    uint32_t kind;    // 0 thread pack, 1 wave pack, 2 work-group byte range
    uint32_t count;   // operations in a pack
    uint32_t first;   // first operation (index into the plan's device descriptor array)
    uint32_t pad;
    uint64_t lo, hi;  // byte range of a work-group task
};
static_assert(sizeof(PlanTask) == 32, "task layout");

struct shmemx_plan {
    std::vector<shmemx_desc_t> host;        // program order
    std::vector<int> host_scope;            // resolved scope per op (program order)
    std::vector<uint64_t> host_chunk;       // resolved chunk per op
    shmemx_desc_t *d_descs = nullptr;       // phase-grouped order
    PlanTask *d_tasks = nullptr;
    uint32_t *d_phase = nullptr;            // nphases + 1 task offsets
    uint64_t ntasks = 0, nphases = 0, nlaunch = 0;
    int wg = 256;
    int grid = 1;
    uint64_t *stamps = nullptr;             // optional per-op completion stamps (device)
    uint64_t *d_bar = nullptr;              // the plan's own grid-barrier words (device)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

enum { TK_THREAD = 0, TK_WAVE = 1, TK_WG = 2 };
constexpr size_t kPlanBarBytes = VSHMEM_SYNC_GEN_OFF + VSHMEM_SYNC_SLOT_BYTES;

using namespace vshmem_exec;

// Completion stamp of operation `idx` (measurement mode): the caller's
// stores are completed first, then the device wall clock is recorded; when
// several work-groups share an operation the latest stamp wins.
__device__ __forceinline__ void stamp(uint64_t *stamps, uint64_t idx)
{
    __hip_atomic_fetch_max(stamps + idx, (uint64_t)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void run_task(const shmemx_dctx_pub_t &c, const shmemx_desc_t *D, const PlanTask &t,
                                         uint64_t *results, uint64_t *stamps)
{
    if (t.kind == TK_THREAD) {
        if (threadIdx.x < t.count) {
            const shmemx_desc_t &d = D[t.first + threadIdx.x];
            exec_thread(c, d, results);
            if (stamps) {
                vshmem_detail::release_agent();
                stamp(stamps, d.reserved);
            }
        }
    } else if (t.kind == TK_WAVE) {
        const uint32_t w = threadIdx.x / 64;
        if (w < t.count) {
            const shmemx_desc_t &d = D[t.first + w];
            exec_wave(c, d, results);
            if (stamps) {
                vshmem_detail::release_agent();
                if (__lane_id() == 0) stamp(stamps, d.reserved);
            }
        }
    } else {
        exec_wg(c, D[t.first], t.lo, t.hi, results);
        if (stamps) {
            vshmem_detail::release_agent();
            __syncthreads();
            if (threadIdx.x == 0) stamp(stamps, D[t.first].reserved);
        }
    }
}

__global__ void __launch_bounds__(1024) k_plan_fused(shmemx_dctx_pub_t c, const shmemx_desc_t *__restrict__ D,
                                                     const PlanTask *__restrict__ T, const uint32_t *__restrict__ phase,
                                                     int nphases, uint64_t *results, uint64_t *stamps, uint64_t *bar)
{
    // Loop bounds and task fields go through readfirstlane: the task loop
    // holds work-group barriers, and the compiler must see its exits (and
    // the branches around the barriers) as uniform.
    for (int ph = 0; ph < nphases; ++ph) {
        const uint32_t t1 = __builtin_amdgcn_readfirstlane(phase[ph + 1]);
        const uint32_t t0 = __builtin_amdgcn_readfirstlane(phase[ph]);
        for (uint32_t t = t0 + blockIdx.x; t < t1; t += gridDim.x) {
            PlanTask task;
            const uint32_t *q = (const uint32_t *)(T + t);
            uint32_t *w = (uint32_t *)&task;
#pragma unroll
            for (int i = 0; i < (int)(sizeof(PlanTask) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(q[i]);
            run_task(c, D, task, results, stamps);
        }
        if (ph + 1 < nphases) {
            // Ordering point: every work-group's earlier operations complete
            // before any later operation starts (thread 0's release and
            // acquire in the barrier cover its work-group).
            vshmem_detail::wait_vm_complete();
            __syncthreads();
            if (threadIdx.x == 0) vshmem_detail::counter_barrier(c, bar, gridDim.x);
            __syncthreads();
        }
    }
    vshmem_detail::release_wg_at_exit();   // quiet
}

// Per-operation form: the kernel receives its descriptor by value.
__global__ void __launch_bounds__(1024) k_plan_one(shmemx_dctx_pub_t c, shmemx_desc_t d, int scope, uint64_t chunk,
                                                   uint64_t *results, uint64_t *stamps)
{
    if (scope == SHMEMX_SCOPE_THREAD) {
        if (threadIdx.x == 0) exec_thread(c, d, results);
    } else if (scope == SHMEMX_SCOPE_WAVE) {
        if (threadIdx.x < 64) exec_wave(c, d, results);
    } else {
        const uint64_t lo = (uint64_t)blockIdx.x * chunk;
        const uint64_t hi = lo + chunk < d.nbytes ? lo + chunk : d.nbytes;
        if (lo < hi || (blockIdx.x == 0 && d.nbytes == 0)) exec_wg(c, d, lo, hi, results);
    }
    vshmem_detail::release_wg_at_exit();   // quiet
    if (stamps && threadIdx.x == 0) stamp(stamps, d.reserved);
}

__global__ void k_stamp(uint64_t *dst) { if (threadIdx.x == 0) *dst = wall_clock64(); }


int validate(const shmemx_desc_t &d)
{
    const State &s = st();
    if (d.op > SHMEMX_OP_BARRIER_ALL) return SHMEMX_ERR_ARG;
    if (d.op == SHMEMX_OP_WAIT_UNTIL) return SHMEMX_ERR_UNSUPPORTED;
    if (d.issuer_pe < 0 || d.issuer_pe >= s.npes) return SHMEMX_ERR_ARG;
    if (d.op == SHMEMX_OP_NOP || is_sync_op(d.op)) return SHMEMX_OK;
    if (d.target_pe < 0 || d.target_pe >= s.npes) return SHMEMX_ERR_ARG;
    if (d.scope > SHMEMX_SCOPE_GRID && d.scope != SHMEMX_SCOPE_AUTO) return SHMEMX_ERR_ARG;
    if (is_amo_op(d.op)) return (d.src & 7) == 0 && in_user_heap(d.src, 8) ? SHMEMX_OK : SHMEMX_ERR_ARG;
    if (!in_user_heap(d.src, d.nbytes) || !in_user_heap(d.dst, d.nbytes)) return SHMEMX_ERR_ARG;
    if (d.op == SHMEMX_OP_PUT_SIGNAL && ((d.cond & 7) || !in_user_heap(d.cond, 8))) return SHMEMX_ERR_ARG;
    return SHMEMX_OK;
}

template <typename T>
int upload(T **dptr, const std::vector<T> &v)
{
    if (v.empty()) return SHMEMX_OK;
    VSHMEM_HIP(hipMalloc((void **)dptr, v.size() * sizeof(T)));
    VSHMEM_HIP(hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return SHMEMX_OK;
}

}  // namespace

extern "C" {

void shmemx_tune_default(shmemx_tune_t *t)
{
    if (!t) return;
    memset(t, 0, sizeof(*t));
    t->wg_size = 256;
    t->grid_wgs = 0;
    for (int c = 0; c < SHMEMX_TUNE_CLASSES; ++c) {
        // below 64 B one lane per message; up to 16 KiB a wavefront; above, a
        // work-group, with messages past 1 MiB split into 256 KiB tasks.  (On
        // the 4-PE mixed program of 8 B - 4 KiB messages, wavefront scope
        // finished the burst 6x sooner than one lane per message.)
        t->scope[c] = c < 6 ? SHMEMX_SCOPE_THREAD : (c < 14 ? SHMEMX_SCOPE_WAVE : SHMEMX_SCOPE_WG);
        t->chunk[c] = c >= 20 ? (256ull << 10) : 0;
    }
}

int shmemx_plan_create(const shmemx_desc_t *descs, size_t n, const shmemx_tune_t *tune_in, shmemx_plan_t **out)
{
    if (int rc = check_ready()) return rc;
    if (!out || (!descs && n) || n >= (1ull << 31)) return SHMEMX_ERR_ARG;
    *out = nullptr;
    shmemx_tune_t tune;
    if (tune_in) tune = *tune_in;
    else shmemx_tune_default(&tune);
    if (!valid_wg_size(tune.wg_size)) return SHMEMX_ERR_ARG;
    const State &s = st();
    // Validate and assign phases: key (barriers seen, fences since) of the issuer.
    std::vector<uint32_t> nbar(s.npes, 0), nfen(s.npes, 0);
    std::vector<std::pair<uint64_t, uint32_t>> keyed;   // (phase key, op index)
    auto plan = new shmemx_plan();
    plan->host.assign(descs, descs + n);
    for (size_t i = 0; i < n; ++i) plan->host[i].reserved = i;
    plan->host_scope.assign(n, 0);
    plan->host_chunk.assign(n, 0);
    plan->wg = tune.wg_size;
    for (size_t i = 0; i < n; ++i) {
        const shmemx_desc_t &d = descs[i];
        int rc = validate(d);
        if (rc) {
            delete plan;
            set_last_error(rc);
            return rc;
        }
        if (d.op == SHMEMX_OP_BARRIER_ALL) {
            nbar[d.issuer_pe]++;
            nfen[d.issuer_pe] = 0;
            continue;
        }
        if (d.op == SHMEMX_OP_FENCE || d.op == SHMEMX_OP_QUIET) {
            nfen[d.issuer_pe]++;
            continue;
        }
        if (d.op == SHMEMX_OP_NOP) continue;
        int sc = resolve_scope(d, tune);
        plan->host_scope[i] = sc;
        plan->host_chunk[i] = resolve_chunk(d, sc, tune);
        keyed.push_back({((uint64_t)nbar[d.issuer_pe] << 32) | nfen[d.issuer_pe], (uint32_t)i});
        plan->nlaunch++;
    }
    for (int p = 1; p < s.npes; ++p)
        if (nbar[p] != nbar[0]) {
            delete plan;
            set_last_error(SHMEMX_ERR_ARG);
            return SHMEMX_ERR_ARG;
        }
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const std::pair<uint64_t, uint32_t> &a, const std::pair<uint64_t, uint32_t> &b) {
                         return a.first < b.first;
                     });
    std::vector<shmemx_desc_t> dd;
    std::vector<PlanTask> tasks;
    std::vector<uint32_t> phase{0};
    const uint32_t waves = (uint32_t)tune.wg_size / 64;
    size_t i = 0;
    while (i < keyed.size()) {
        size_t j = i;
        while (j < keyed.size() && keyed[j].first == keyed[i].first) ++j;
        std::vector<uint32_t> th, wv, wg;
        for (size_t k = i; k < j; ++k) {
            uint32_t idx = keyed[k].second;
            int sc = plan->host_scope[idx];
            (sc == SHMEMX_SCOPE_THREAD ? th : sc == SHMEMX_SCOPE_WAVE ? wv : wg).push_back(idx);
        }
        // Largest work-group tasks first, then the packs.
        std::stable_sort(wg.begin(), wg.end(), [&](uint32_t a, uint32_t b) { return descs[a].nbytes > descs[b].nbytes; });
        for (uint32_t idx : wg) {
            const uint64_t nb = descs[idx].nbytes, ch = plan->host_chunk[idx];
            const uint32_t first = (uint32_t)dd.size();
            dd.push_back(descs[idx]);
            dd.back().reserved = idx;
            if (nb == 0 || ch >= nb) {
                tasks.push_back(PlanTask{TK_WG, 1, first, 0, 0, nb});
            } else {
                for (uint64_t lo = 0; lo < nb; lo += ch)
                    tasks.push_back(PlanTask{TK_WG, 1, first, 0, lo, std::min(nb, lo + ch)});
            }
        }
        for (size_t k = 0; k < wv.size(); k += waves) {
            uint32_t cnt = (uint32_t)std::min<size_t>(waves, wv.size() - k);
            tasks.push_back(PlanTask{TK_WAVE, cnt, (uint32_t)dd.size(), 0, 0, 0});
            for (uint32_t u = 0; u < cnt; ++u) {
                dd.push_back(descs[wv[k + u]]);
                dd.back().reserved = wv[k + u];
            }
        }
        for (size_t k = 0; k < th.size(); k += (size_t)tune.wg_size) {
            uint32_t cnt = (uint32_t)std::min<size_t>((size_t)tune.wg_size, th.size() - k);
            tasks.push_back(PlanTask{TK_THREAD, cnt, (uint32_t)dd.size(), 0, 0, 0});
            for (uint32_t u = 0; u < cnt; ++u) {
                dd.push_back(descs[th[k + u]]);
                dd.back().reserved = th[k + u];
            }
        }
        phase.push_back((uint32_t)tasks.size());
        i = j;
    }
    plan->ntasks = tasks.size();
    plan->nphases = phase.size() - 1;
    uint64_t widest = 1;
    for (size_t p = 0; p + 1 < phase.size(); ++p) widest = std::max<uint64_t>(widest, phase[p + 1] - phase[p]);
    int per_cu = 0;
    if (int rc = blocks_per_cu(k_plan_fused, plan->wg, &per_cu)) {
        delete plan;
        return rc;
    }
    if (per_cu <= 0) {
        hipFuncAttributes fa{};
        (void)hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_plan_fused));
        set_error_detail(SHMEMX_ERR_UNSUPPORTED,
                         "k_plan_fused: no work-group of %d threads can be resident (occupancy %d; %d registers, "
                         "at most %d threads per block)", plan->wg, per_cu, fa.numRegs, fa.maxThreadsPerBlock);
        delete plan;
        return SHMEMX_ERR_UNSUPPORTED;
    }
    uint64_t cap = (uint64_t)per_cu * s.num_cus;
    if (tune.grid_wgs > 0) cap = std::min<uint64_t>(cap, (uint64_t)tune.grid_wgs);
    plan->grid = (int)std::max<uint64_t>(1, std::min(widest, cap));
    int rc = upload(&plan->d_descs, dd);
    if (!rc) rc = upload(&plan->d_tasks, tasks);
    if (!rc) rc = upload(&plan->d_phase, phase);
    // Barrier words of the plan's own: launches of different plans never
    // share an arrival count (count at 0, generation VSHMEM_SYNC_GEN_OFF on).
    if (!rc && VSHMEM_HIP_FAILED(hipMalloc((void **)&plan->d_bar, kPlanBarBytes))) rc = SHMEMX_ERR_HIP;
    if (!rc && VSHMEM_HIP_FAILED(hipMemset(plan->d_bar, 0, kPlanBarBytes))) rc = SHMEMX_ERR_HIP;
    if (!rc) register_bar_block(plan->d_bar, kPlanBarBytes);
    if (rc) {
        shmemx_plan_destroy(plan);
        return rc;
    }
    *out = plan;
    return SHMEMX_OK;
}

int shmemx_plan_launch_fused(shmemx_plan_t *plan, uint64_t *results, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!plan) return SHMEMX_ERR_ARG;
    if (plan->nphases == 0) return SHMEMX_OK;
    // Work-groups of a multi-phase plan wait for each other at its barriers.
    if (plan->nphases > 1)
        if (int rc = check_coresident(k_plan_fused, plan->grid, plan->wg, "fused plan")) return rc;
    hipLaunchKernelGGL(k_plan_fused, dim3(plan->grid), dim3(plan->wg), 0, (hipStream_t)stream, pub(), plan->d_descs,
                       plan->d_tasks, plan->d_phase, (int)plan->nphases, results, plan->stamps, plan->d_bar);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_plan_launch_per_op(shmemx_plan_t *plan, uint64_t *results, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!plan) return SHMEMX_ERR_ARG;
    const shmemx_dctx_pub_t c = pub();
    for (size_t i = 0; i < plan->host.size(); ++i) {
        const shmemx_desc_t &d = plan->host[i];
        if (d.op == SHMEMX_OP_NOP || is_sync_op(d.op)) continue;   // stream order provides the ordering
        const int sc = plan->host_scope[i];
        unsigned grid = 1, block = 64;
        uint64_t ch = plan->host_chunk[i];
        if (sc == SHMEMX_SCOPE_WG || sc == SHMEMX_SCOPE_GRID) {
            block = (unsigned)plan->wg;
            grid = (unsigned)std::max<uint64_t>(1, (d.nbytes + ch - 1) / ch);
        }
        hipLaunchKernelGGL(k_plan_one, dim3(grid), dim3(block), 0, (hipStream_t)stream, c, d, sc, ch, results,
                           plan->stamps);
    }
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_plan_graph_build(shmemx_plan_t *plan, int form, uint64_t *results, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!plan || (form != 0 && form != 1)) return SHMEMX_ERR_ARG;
    if (plan->exec) {
        (void)hipGraphExecDestroy(plan->exec);
        plan->exec = nullptr;
    }
    if (plan->graph) {
        (void)hipGraphDestroy(plan->graph);
        plan->graph = nullptr;
    }
    hipStream_t cap;
    VSHMEM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    int rc = SHMEMX_OK;
    if (VSHMEM_HIP_FAILED(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal))) rc = SHMEMX_ERR_HIP;
    if (!rc) rc = form == 0 ? shmemx_plan_launch_per_op(plan, results, cap) : shmemx_plan_launch_fused(plan, results, cap);
    hipGraph_t g = nullptr;
    if (VSHMEM_HIP_FAILED(hipStreamEndCapture(cap, &g)) && !rc) rc = SHMEMX_ERR_HIP;
    if (!rc && VSHMEM_HIP_FAILED(hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0))) rc = SHMEMX_ERR_HIP;
    plan->graph = g;
    (void)hipStreamDestroy(cap);
    (void)stream;
    if (rc) set_last_error(rc);
    return rc;
}

int shmemx_plan_graph_launch(shmemx_plan_t *plan, void *stream)
{
    if (int rc = check_ready()) return rc;
    if (!plan || !plan->exec) return SHMEMX_ERR_STATE;
    VSHMEM_HIP(hipGraphLaunch(plan->exec, (hipStream_t)stream));
    return SHMEMX_OK;
}

int shmemx_plan_set_stamps(shmemx_plan_t *plan, uint64_t *stamps)
{
    if (!plan) return SHMEMX_ERR_ARG;
    plan->stamps = stamps;
    return SHMEMX_OK;
}

int shmemx_stamp_launch(uint64_t *dst, void *stream)
{
    if (!dst) return SHMEMX_ERR_ARG;
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, (hipStream_t)stream, dst);
    VSHMEM_HIP(hipGetLastError());
    return SHMEMX_OK;
}

int shmemx_plan_info(const shmemx_plan_t *plan, uint64_t *ntasks, uint64_t *nphases, uint64_t *nlaunches)
{
    if (!plan) return SHMEMX_ERR_ARG;
    if (ntasks) *ntasks = plan->ntasks;
    if (nphases) *nphases = plan->nphases;
    if (nlaunches) *nlaunches = plan->nlaunch;
    return SHMEMX_OK;
}

void shmemx_plan_destroy(shmemx_plan_t *plan)
{
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->d_descs) (void)hipFree(plan->d_descs);
    if (plan->d_tasks) (void)hipFree(plan->d_tasks);
    if (plan->d_phase) (void)hipFree(plan->d_phase);
    if (plan->d_bar) {
        unregister_bar_block(plan->d_bar);
        (void)hipFree(plan->d_bar);
    }
    delete plan;
}

}  // extern "C"
