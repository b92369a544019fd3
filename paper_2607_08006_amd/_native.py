"""ctypes declarations of libvshmem.so (the C-ABI in include/vshmem.h)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvshmem.so")

TUNE_CLASSES = 40


class Desc(C.Structure):
    _fields_ = [("op", C.c_uint8), ("scope", C.c_uint8), ("aux", C.c_uint8), ("flags", C.c_uint8),
                ("issuer_pe", C.c_int32), ("target_pe", C.c_int32), ("result_idx", C.c_uint32),
                ("src", C.c_uint64), ("dst", C.c_uint64), ("nbytes", C.c_uint64), ("value", C.c_uint64),
                ("cond", C.c_uint64), ("reserved", C.c_uint64)]


class Caps(C.Structure):
    _fields_ = [("gpu_heap", C.c_int32), ("default_heap_is_gpu", C.c_int32), ("host_initiated", C.c_int32),
                ("device_initiated", C.c_int32), ("device_ctx_default", C.c_int32),
                ("explicit_device_ctx", C.c_int32), ("scopes", C.c_uint32), ("device_collectives", C.c_int32),
                ("stream_triggered", C.c_int32), ("progress", C.c_uint32), ("path", C.c_int32),
                ("ptr_domain", C.c_int32), ("team_npes", C.c_int32), ("team_start", C.c_int32),
                ("team_stride", C.c_int32), ("npes", C.c_int32), ("heap_user_bytes", C.c_uint64),
                ("heap_stride", C.c_uint64), ("debug", C.c_int32), ("max_device_ctx", C.c_int32),
                ("reserved", C.c_int32 * 6)]


class Launch(C.Structure):
    _fields_ = [("wgs_per_pe", C.c_int32), ("wg_size", C.c_int32), ("chunk_bytes", C.c_uint64),
                ("flags", C.c_int32), ("reserved", C.c_int32)]


class Tune(C.Structure):
    _fields_ = [("wg_size", C.c_int32), ("grid_wgs", C.c_int32), ("scope", C.c_uint8 * TUNE_CLASSES),
                ("chunk", C.c_uint64 * TUNE_CLASSES)]


class ProgressCfg(C.Structure):
    _fields_ = [("nwg", C.c_int32), ("wg_size", C.c_int32), ("ring_slots", C.c_int32), ("verify", C.c_int32),
                ("chunk_bytes", C.c_uint64), ("idle_timeout_ms", C.c_uint64)]


class Completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("t_start", C.c_uint64), ("t_end", C.c_uint64), ("hash", C.c_uint64),
                ("status", C.c_int32), ("lane", C.c_int32), ("t_queued", C.c_uint64), ("submit_ns", C.c_uint64)]


class DTeam(C.Structure):
    _fields_ = [("start", C.c_int32), ("stride", C.c_int32), ("size", C.c_int32), ("slot", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("op", C.c_int32), ("issuer_pe", C.c_int32), ("target_pe", C.c_int32), ("lane", C.c_int32),
                ("nbytes", C.c_uint64), ("src_off", C.c_uint64), ("arrival_s", C.c_double)]


class ServeStats(C.Structure):
    _fields_ = [("wall_s", C.c_double), ("bytes", C.c_uint64), ("amo_ops", C.c_uint64),
                ("max_reserved_bytes", C.c_uint64), ("admission_waits", C.c_uint64),
                ("ring_full_retries", C.c_uint64)]


vp, i32, u64, sz = C.c_void_p, C.c_int, C.c_uint64, C.c_size_t
P = C.POINTER

# name: (restype, argtypes)
SIGNATURES = {
    "shmemx_init_attach": (i32, [vp, sz, i32, vp]),
    "shmemx_heap_stride_for": (u64, [u64, i32]),
    "shmem_init": (None, []),
    "shmem_finalize": (None, []),
    "shmem_n_pes": (i32, []),
    "shmem_my_pe": (i32, []),
    "shmem_malloc": (vp, [sz]),
    "shmemg_malloc": (vp, [sz]),
    "shmem_calloc": (vp, [sz, sz]),
    "shmem_align": (vp, [sz, sz]),
    "shmem_free": (None, [vp]),
    "shmem_ptr": (vp, [vp, i32]),
    "shmem_team_ptr": (vp, [C.c_int32, vp, i32]),
    "shmem_query_capabilities": (i32, [C.c_int32, P(Caps)]),
    "shmemx_heap_base": (vp, []),
    "shmemx_heap_stride": (u64, []),
    "shmemx_heap_user_bytes": (u64, []),
    "shmemx_device_ctx": (vp, []),
    "shmemx_device_ctx_create": (i32, [C.c_int32, C.c_long, P(C.c_int32)]),
    "shmemx_device_ctx_record": (vp, [C.c_int32]),
    "shmemx_device_ctx_destroy": (None, [C.c_int32]),
    "shmem_team_split_strided": (i32, [C.c_int32, i32, i32, i32, vp, C.c_long, P(C.c_int32)]),
    "shmem_team_n_pes": (i32, [C.c_int32]),
    "shmemx_team_device": (i32, [C.c_int32, P(DTeam)]),
    "shmemx_team_pe_index": (i32, [C.c_int32, i32]),
    "shmem_team_destroy": (None, [C.c_int32]),
    "shmemx_strerror": (C.c_char_p, [i32]),
    "shmemx_last_error": (i32, []),
    "shmemx_clear_last_error": (None, []),
    "shmemx_device_errors": (i32, []),
    "shmemx_set_wait_timeout_ns": (i32, [u64]),
    "shmemx_rma_pattern": (i32, [i32, i32, vp, u64, u64, u64, u64, u64, u64, P(Launch), vp]),
    "shmemx_gups": (i32, [u64, i32, u64, u64, i32, vp, vp, P(Launch), vp]),
    "shmemx_pingpong": (i32, [u64, u64, vp, i32, i32, u64, i32, vp, vp]),
    "shmemx_wallclock_hz": (u64, []),
    "shmemx_wait_until_launch": (i32, [i32, u64, i32, u64, i32, vp, vp]),
    "shmemx_barrier_launch": (i32, [C.c_int32, i32, u64, vp, vp, vp]),
    "shmemx_broadcastmem_launch": (i32, [C.c_int32, vp, vp, sz, i32, P(Launch), vp]),
    "shmemx_fcollectmem_launch": (i32, [C.c_int32, vp, vp, sz, P(Launch), vp]),
    "shmemx_alltoallmem_launch": (i32, [C.c_int32, vp, vp, sz, P(Launch), vp]),
    "shmemx_reduce_launch": (i32, [C.c_int32, i32, i32, vp, vp, sz, P(Launch), vp]),
    "shmemx_tune_default": (None, [P(Tune)]),
    "shmemx_plan_create": (i32, [vp, sz, P(Tune), P(vp)]),
    "shmemx_plan_launch_fused": (i32, [vp, vp, vp]),
    "shmemx_plan_launch_per_op": (i32, [vp, vp, vp]),
    "shmemx_plan_graph_build": (i32, [vp, i32, vp, vp]),
    "shmemx_plan_graph_launch": (i32, [vp, vp]),
    "shmemx_plan_set_stamps": (i32, [vp, vp]),
    "shmemx_stamp_launch": (i32, [vp, vp]),
    "shmemx_plan_info": (i32, [vp, P(u64), P(u64), P(u64)]),
    "shmemx_plan_destroy": (None, [vp]),
    "shmemx_autotune": (i32, [u64, u64, u64, u64, i32, i32, P(Tune), vp]),
    "shmemx_tune_save": (i32, [P(Tune), C.c_char_p]),
    "shmemx_tune_load": (i32, [P(Tune), C.c_char_p]),
    "shmemx_tune_set": (i32, [P(Tune)]),
    "shmemx_tune_get": (i32, [P(Tune)]),
    "shmemx_launch_batch": (i32, [vp, sz, vp, vp, vp]),
    "shmemx_launch_per_op": (i32, [vp, sz, vp, vp, vp]),
    "shmemx_launch_batch_noalloc": (i32, [vp, sz, vp, vp, vp]),
    "shmemx_launch_batch_noalloc_max": (u64, []),
    "shmemx_graph_build": (i32, [vp, sz, vp, vp, i32, P(vp)]),
    "shmemx_graph_launch": (i32, [vp, vp]),
    "shmemx_graph_destroy": (None, [vp]),
    "shmemx_progress_start": (i32, [P(ProgressCfg), vp]),
    "shmemx_progress_submit": (i32, [i32, P(Desc), P(u64)]),
    "shmemx_progress_poll": (i32, [u64, P(Completion)]),
    "shmemx_progress_stop": (i32, [i32]),
    "shmemx_serve_run": (i32, [P(Request), sz, i32, u64, u64, u64, vp, vp, P(Completion), P(ServeStats)]),
    "shmemx_serve_run_per_op": (i32, [P(Request), sz, i32, u64, u64, u64, u64, i32, vp, vp, P(Completion),
                                       P(ServeStats)]),
    "shmemx_launch_request": (i32, [P(Desc), u64, i32, vp]),
    "shmemx_serve_run_batched": (i32, [P(Request), sz, i32, u64, u64, u64, u64, i32, u64, i32, vp, vp,
                                        P(Completion), P(ServeStats)]),
    # host-initiated operations (host default context)
    "shmem_putmem": (None, [vp, vp, sz, i32]),
    "shmem_getmem": (None, [vp, vp, sz, i32]),
    "shmem_putmem_nbi": (None, [vp, vp, sz, i32]),
    "shmem_getmem_nbi": (None, [vp, vp, sz, i32]),
    "shmem_putmem_signal": (None, [vp, vp, sz, vp, u64, i32, i32]),
    "shmem_putmem_signal_nbi": (None, [vp, vp, sz, vp, u64, i32, i32]),
    "shmem_signal_fetch": (u64, [vp]),
    "shmem_signal_wait_until": (u64, [vp, i32, u64]),
    "shmem_int64_wait_until": (None, [vp, i32, C.c_int64]),
    "shmem_int64_test": (i32, [vp, i32, C.c_int64]),
    "shmem_int64_atomic_fetch_add": (C.c_int64, [vp, C.c_int64, i32]),
    "shmem_int64_atomic_add": (None, [vp, C.c_int64, i32]),
    "shmem_int64_atomic_fetch_xor": (C.c_int64, [vp, C.c_int64, i32]),
    "shmem_int64_atomic_xor": (None, [vp, C.c_int64, i32]),
    "shmem_uint64_atomic_fetch_xor": (u64, [vp, u64, i32]),
    "shmem_uint64_atomic_xor": (None, [vp, u64, i32]),
    "shmem_int64_atomic_compare_swap": (C.c_int64, [vp, C.c_int64, C.c_int64, i32]),
    "shmem_int64_atomic_fetch": (C.c_int64, [vp, i32]),
    "shmem_int64_atomic_set": (None, [vp, C.c_int64, i32]),
    "shmem_int64_atomic_swap": (C.c_int64, [vp, C.c_int64, i32]),
    "shmem_quiet": (None, []),
    "shmem_fence": (None, []),
    "shmem_barrier_all": (None, []),
    "shmem_sync_all": (None, []),
    "shmem_team_sync": (i32, [C.c_int32]),
    "shmem_broadcastmem": (i32, [C.c_int32, vp, vp, sz, i32]),
    "shmem_fcollectmem": (i32, [C.c_int32, vp, vp, sz]),
    "shmem_alltoallmem": (i32, [C.c_int32, vp, vp, sz]),
    "shmem_int64_sum_reduce": (i32, [C.c_int32, vp, vp, sz]),
    "shmem_int64_max_reduce": (i32, [C.c_int32, vp, vp, sz]),
    "shmem_float_sum_reduce": (i32, [C.c_int32, vp, vp, sz]),
    "shmem_float_max_reduce": (i32, [C.c_int32, vp, vp, sz]),
    "shmemx_bfloat16_sum_reduce": (i32, [C.c_int32, vp, vp, sz]),
    "shmemx_bfloat16_max_reduce": (i32, [C.c_int32, vp, vp, sz]),
    # stream-triggered operations
    "shmemx_putmem_on_stream": (i32, [vp, vp, sz, i32, vp]),
    "shmemx_getmem_on_stream": (i32, [vp, vp, sz, i32, vp]),
    "shmemx_putmem_signal_on_stream": (i32, [vp, vp, sz, vp, u64, i32, i32, vp]),
    "shmemx_signal_wait_until_on_stream": (i32, [vp, i32, u64, vp]),
    "shmemx_barrier_all_on_stream": (i32, [vp]),
    "shmemx_team_sync_on_stream": (i32, [C.c_int32, vp]),
    "shmemx_quiet_on_stream": (i32, [vp]),
    "shmemx_broadcastmem_on_stream": (i32, [C.c_int32, vp, vp, sz, i32, vp]),
    "shmemx_fcollectmem_on_stream": (i32, [C.c_int32, vp, vp, sz, vp]),
    "shmemx_alltoallmem_on_stream": (i32, [C.c_int32, vp, vp, sz, vp]),
    "shmemx_reduce_on_stream": (i32, [C.c_int32, i32, i32, vp, vp, sz, vp]),
    "shmemx_fill_random": (i32, [vp, u64, u64, u64, vp]),
    "shmemx_fill_typed": (i32, [vp, u64, i32, u64, u64, vp]),
    "shmemx_probe_hbm": (i32, [i32, vp, vp, u64, i32, i32, vp, vp]),
    "shmemx_probe_copy": (i32, [vp, vp, u64, i32, i32, vp]),
    "shmemx_probe_atomics": (i32, [vp, u64, u64, u64, vp, vp]),
    "shmemx_probe_xcd": (i32, [vp, i32, vp]),
    "shmemx_probe_empty": (i32, [vp]),
    "shmemx_version": (C.c_char_p, []),
    "shmemx_last_hip_error": (i32, [C.c_char_p, sz]),
}

_lib = None


def load() -> C.CDLL:
    """Load libvshmem.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libvshmem.so not found at {LIB_PATH}: build it with "
                          "`python -c 'import __graft_entry__; __graft_entry__.build()'`")
    lib = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
