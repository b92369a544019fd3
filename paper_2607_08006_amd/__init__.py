"""Python binding of libvshmem.so: device-initiated OpenSHMEM on virtual PEs
for one MI355X.

Argument marshalling only: every operation runs in the library's HIP kernels.
PyTorch supplies device memory (the symmetric heap, result arrays) and
streams.  Importing this package loads the native library and raises
ImportError if it has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
# torch (which carries its own HIP runtime) is loaded before the native
# library: with another HIP library already in the process, loading the
# native library between torch's import and torch's device initialisation
# made that initialisation fail on MI355X (no device).
import torch  # noqa: F401

from . import _native
from ._native import Caps, Completion, Desc, DTeam, Launch, ProgressCfg, Request, ServeStats, Tune

lib = _native.load()

OK = 0
ERR_ARG, ERR_NOMEM, ERR_STATE, ERR_HIP, ERR_BUSY, ERR_TIMEOUT, ERR_DEVICE, ERR_UNSUPPORTED = range(-1, -9, -1)
DEVERR_WAIT_TIMEOUT, DEVERR_BAD_DESC, DEVERR_PROGRESS_IDLE, DEVERR_PROGRESS_STATE = 0x1, 0x2, 0x4, 0x8
DEVERR_BAD_ADDRESS, DEVERR_NONUNIFORM = 0x10, 0x20

OP_NOP, OP_PUT, OP_GET, OP_PUT_SIGNAL = 0, 1, 2, 3
OP_AMO_FETCH_ADD, OP_AMO_FETCH_XOR, OP_AMO_COMPARE_SWAP, OP_AMO_ADD, OP_AMO_XOR = 4, 5, 6, 7, 8
OP_AMO_SET, OP_AMO_FETCH, OP_AMO_SWAP, OP_WAIT_UNTIL, OP_FENCE, OP_QUIET, OP_BARRIER_ALL = 9, 10, 11, 12, 13, 14, 15
SCOPE_THREAD, SCOPE_WAVE, SCOPE_WG, SCOPE_GRID, SCOPE_AUTO = 0, 1, 2, 3, 255
SIGNAL_SET, SIGNAL_ADD = 0, 1
CMP_EQ, CMP_NE, CMP_GT, CMP_GE, CMP_LT, CMP_LE = range(6)
DT_INT64, DT_FP32, DT_BF16 = 0, 1, 2
RED_SUM, RED_MAX = 0, 1
TEAM_WORLD, TEAM_SHARED, DEVICE_TEAM_WORLD, DEVICE_TEAM_SHARED = 0, 1, 2, 3
LAUNCH_NONTEMPORAL = 0x1
LAUNCH_DEEP = 0x2
NO_RESULT = 0xFFFFFFFF

SLICE_ALIGN = 2 << 20


class VshmemError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib.shmemx_strerror(code).decode()
        buf = C.create_string_buffer(512)
        lib.shmemx_last_hip_error(buf, len(buf))
        if buf.value:
            msg += ": " + buf.value.decode(errors="replace")
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


def _check(rc: int, what: str) -> int:
    if rc != 0:
        raise VshmemError(rc, what)
    return rc


def _torch():
    import torch
    return torch


def _stream(stream) -> int:
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def launch_cfg(wgs_per_pe: int = 0, wg_size: int = 0, chunk_bytes: int = 0, flags: int = 0) -> Launch:
    return Launch(wgs_per_pe, wg_size, chunk_bytes, flags, 0)


# ------------------------------------------------------------------ heap
_heap_tensor = None


def stride_for(bytes_per_pe: int, spread: bool = True) -> int:
    """shmemx_heap_stride_for: the library's slice stride (spread) or the
    smallest one."""
    s = int(lib.shmemx_heap_stride_for(bytes_per_pe, 1 if spread else 0))
    if s == 0:
        raise VshmemError(ERR_ARG, "stride_for (size out of range)")
    return s


def init(npes: int, bytes_per_pe: int, stream=None, spread: bool = True) -> None:
    """Attach a PyTorch-allocated heap of npes slices with at least
    bytes_per_pe allocatable bytes each (shmemx_init_attach), with slices
    stride_for(bytes_per_pe) apart, or the smallest stride when that much
    memory cannot be allocated (or when spread is False)."""
    global _heap_tensor
    torch = _torch()
    stride = stride_for(bytes_per_pe, spread)
    try:
        t = torch.empty(npes * stride + SLICE_ALIGN, dtype=torch.uint8, device="cuda")
    except torch.OutOfMemoryError:
        stride = stride_for(bytes_per_pe, spread=False)
        t = torch.empty(npes * stride + SLICE_ALIGN, dtype=torch.uint8, device="cuda")
    base = (t.data_ptr() + SLICE_ALIGN - 1) // SLICE_ALIGN * SLICE_ALIGN
    _check(lib.shmemx_init_attach(base, npes * stride, npes, _stream(stream)), "shmemx_init_attach")
    _heap_tensor = t


def finalize() -> None:
    global _heap_tensor
    lib.shmem_finalize()
    _heap_tensor = None


def initialized() -> bool:
    return lib.shmem_n_pes() > 0


def n_pes() -> int:
    return lib.shmem_n_pes()


def my_pe() -> int:
    return lib.shmem_my_pe()


def heap_base() -> int:
    return lib.shmemx_heap_base() or 0


def heap_stride() -> int:
    return lib.shmemx_heap_stride()


def heap_user_bytes() -> int:
    return lib.shmemx_heap_user_bytes()


def heap_view():
    """(npes, stride) uint8 CUDA tensor aliasing the symmetric heap."""
    torch = _torch()
    if _heap_tensor is None:
        raise VshmemError(ERR_STATE, "heap_view (heap not attached from Python)")
    off = heap_base() - _heap_tensor.data_ptr()
    npes, stride = n_pes(), heap_stride()
    return _heap_tensor[off:off + npes * stride].view(npes, stride)


def malloc(n: int) -> int:
    p = lib.shmem_malloc(n)
    if not p:
        raise VshmemError(lib.shmemx_last_error() or ERR_NOMEM, "shmem_malloc")
    return p


def shmemg_malloc(n: int) -> int:
    p = lib.shmemg_malloc(n)
    if not p:
        raise VshmemError(lib.shmemx_last_error() or ERR_NOMEM, "shmemg_malloc")
    return p


def calloc(count: int, size: int) -> int:
    p = lib.shmem_calloc(count, size)
    if not p:
        raise VshmemError(lib.shmemx_last_error() or ERR_NOMEM, "shmem_calloc")
    return p


def align(alignment: int, n: int) -> int:
    p = lib.shmem_align(alignment, n)
    if not p:
        raise VshmemError(lib.shmemx_last_error() or ERR_NOMEM, "shmem_align")
    return p


def free(p: int) -> None:
    lib.shmem_free(p)


def offset(addr: int) -> int:
    return addr - heap_base()


def ptr(sym: int, pe: int) -> Optional[int]:
    return lib.shmem_ptr(sym, pe)


def team_ptr(team: int, sym: int, pe: int) -> Optional[int]:
    return lib.shmem_team_ptr(team, sym, pe)


def query_capabilities(team: int = TEAM_WORLD) -> dict:
    c = Caps()
    _check(lib.shmem_query_capabilities(team, C.byref(c)), "shmem_query_capabilities")
    return {f: getattr(c, f) for f, _ in Caps._fields_ if f != "reserved"}


def team_split_strided(parent: int, start: int, stride: int, size: int) -> int:
    t = C.c_int32(-1)
    _check(lib.shmem_team_split_strided(parent, start, stride, size, None, 0, C.byref(t)), "shmem_team_split_strided")
    return t.value


def team_n_pes(team: int) -> int:
    return lib.shmem_team_n_pes(team)


def team_device(team: int) -> DTeam:
    """The device descriptor of `team` (shmemx_dteam_t), passed by value to
    user kernels that call the device collectives."""
    t = DTeam()
    _check(lib.shmemx_team_device(team, C.byref(t)), "shmemx_team_device")
    return t


def device_ctx() -> int:
    """Device address of the published default device context."""
    p = lib.shmemx_device_ctx()
    if not p:
        raise VshmemError(ERR_STATE, "shmemx_device_ctx")
    return p


CTX_SERIALIZED, CTX_PRIVATE, CTX_NOSTORE = 1, 2, 4


def device_ctx_create(team: int = TEAM_WORLD, options: int = 0) -> int:
    """An explicit device context bound to `team`; its handle."""
    h = C.c_int32(-1)
    _check(lib.shmemx_device_ctx_create(team, options, C.byref(h)), "shmemx_device_ctx_create")
    return h.value


def device_ctx_record(ctx: int) -> int:
    """Device address of an explicit context's published record."""
    p = lib.shmemx_device_ctx_record(ctx)
    if not p:
        raise VshmemError(ERR_ARG, "shmemx_device_ctx_record")
    return p


def device_ctx_destroy(ctx: int) -> None:
    lib.shmemx_clear_last_error()
    lib.shmemx_device_ctx_destroy(ctx)
    rc = lib.shmemx_last_error()
    if rc:
        raise VshmemError(rc, "shmemx_device_ctx_destroy")


def team_destroy(team: int) -> None:
    lib.shmem_team_destroy(team)


def device_errors() -> int:
    rc = lib.shmemx_device_errors()
    if rc < 0:
        raise VshmemError(rc, "shmemx_device_errors")
    return rc


def set_wait_timeout_ns(ns: int) -> None:
    _check(lib.shmemx_set_wait_timeout_ns(ns), "shmemx_set_wait_timeout_ns")


def wallclock_hz() -> int:
    return lib.shmemx_wallclock_hz()


# ------------------------------------------------------------- launches
def rma_pattern(op: int, scope: int, targets, src_off: int, dst_off: int, msg_bytes: int, nmsg: int,
                src_step: Optional[int] = None, dst_step: Optional[int] = None, launch: Optional[Launch] = None,
                stream=None) -> None:
    ss = msg_bytes if src_step is None else src_step
    ds = msg_bytes if dst_step is None else dst_step
    _check(lib.shmemx_rma_pattern(op, scope, _ptr(targets), src_off, dst_off, msg_bytes, nmsg, ss, ds,
                                  C.byref(launch) if launch else None, _stream(stream)), "shmemx_rma_pattern")


def gups(table_off: int, log2_table: int, nupdates: int, seed: int, add_every: int = 5, fetched=None, acc=None,
         launch: Optional[Launch] = None, stream=None) -> None:
    _check(lib.shmemx_gups(table_off, log2_table, nupdates, seed, add_every, _ptr(fetched), _ptr(acc),
                           C.byref(launch) if launch else None, _stream(stream)), "shmemx_gups")


def pingpong(data_off: int, sig_off: int, pairs, npairs: int, rounds: int, payload_bytes: int = 8,
             same_xcd: bool = False, rtt=None, stream=None) -> None:
    _check(lib.shmemx_pingpong(data_off, sig_off, _ptr(pairs), npairs, rounds, payload_bytes, 1 if same_xcd else 0,
                               _ptr(rtt), _stream(stream)), "shmemx_pingpong")


def wait_until(pe: int, ivar_off: int, cmp: int, value: int, unsigned: bool = False, out=None, stream=None) -> None:
    _check(lib.shmemx_wait_until_launch(pe, ivar_off, cmp, value & ((1 << 64) - 1), 1 if unsigned else 0, _ptr(out),
                                        _stream(stream)), "shmemx_wait_until_launch")


def barrier(team: int = DEVICE_TEAM_WORLD, iters: int = 1, tokens_off: Optional[int] = None, bad=None, cycles=None,
            stream=None) -> None:
    tk = (1 << 64) - 1 if tokens_off is None else tokens_off
    _check(lib.shmemx_barrier_launch(team, iters, tk, _ptr(bad), _ptr(cycles), _stream(stream)),
           "shmemx_barrier_launch")


def broadcastmem(dest: int, src: int, n: int, root: int, team: int = DEVICE_TEAM_WORLD,
                 launch: Optional[Launch] = None, stream=None) -> None:
    _check(lib.shmemx_broadcastmem_launch(team, dest, src, n, root, C.byref(launch) if launch else None,
                                          _stream(stream)), "shmemx_broadcastmem_launch")


def fcollectmem(dest: int, src: int, n: int, team: int = DEVICE_TEAM_WORLD, launch: Optional[Launch] = None,
                stream=None) -> None:
    _check(lib.shmemx_fcollectmem_launch(team, dest, src, n, C.byref(launch) if launch else None, _stream(stream)),
           "shmemx_fcollectmem_launch")


def alltoallmem(dest: int, src: int, n: int, team: int = DEVICE_TEAM_WORLD, launch: Optional[Launch] = None,
                stream=None) -> None:
    _check(lib.shmemx_alltoallmem_launch(team, dest, src, n, C.byref(launch) if launch else None, _stream(stream)),
           "shmemx_alltoallmem_launch")


def reduce(dtype: int, op: int, dest: int, src: int, nreduce: int, team: int = DEVICE_TEAM_WORLD,
           launch: Optional[Launch] = None, stream=None) -> None:
    _check(lib.shmemx_reduce_launch(team, dtype, op, dest, src, nreduce, C.byref(launch) if launch else None,
                                    _stream(stream)), "shmemx_reduce_launch")


def fill_random(dst, nbytes: int, seed: int, word_offset: int = 0, stream=None) -> None:
    _check(lib.shmemx_fill_random(_ptr(dst), nbytes, seed, word_offset, _stream(stream)), "shmemx_fill_random")


def fill_typed(dst, count: int, dtype: int, seed: int, index0: int = 0, stream=None) -> None:
    _check(lib.shmemx_fill_typed(_ptr(dst), count, dtype, seed, index0, _stream(stream)), "shmemx_fill_typed")


PROBE_COPY_CHUNKED, PROBE_COPY_GRIDSTRIDE, PROBE_COPY_TILES, PROBE_READ, PROBE_WRITE = range(5)


def probe_hbm(kind: int, dst, src, nbytes: int, nwg: int = 256, wg_size: int = 1024, acc=None, stream=None) -> None:
    _check(lib.shmemx_probe_hbm(kind, _ptr(dst), _ptr(src), nbytes, nwg, wg_size, _ptr(acc), _stream(stream)),
           "shmemx_probe_hbm")


def probe_copy(dst, src, nbytes: int, nwg: int = 256, wg_size: int = 1024, stream=None) -> None:
    _check(lib.shmemx_probe_copy(_ptr(dst), _ptr(src), nbytes, nwg, wg_size, _stream(stream)), "shmemx_probe_copy")


def probe_atomics(table, nwords: int, nupdates: int, seed: int, acc=None, stream=None) -> None:
    _check(lib.shmemx_probe_atomics(_ptr(table), nwords, nupdates, seed, _ptr(acc), _stream(stream)),
           "shmemx_probe_atomics")


def probe_xcd(out, nblocks: int, stream=None) -> None:
    _check(lib.shmemx_probe_xcd(_ptr(out), nblocks, _stream(stream)), "shmemx_probe_xcd")


def probe_empty(stream=None) -> None:
    _check(lib.shmemx_probe_empty(_stream(stream)), "shmemx_probe_empty")


# ----------------------------------------------------------------- plans
def default_tune() -> Tune:
    t = Tune()
    lib.shmemx_tune_default(C.byref(t))
    return t


class Plan:
    """A descriptor program prepared once (shmemx_plan_create)."""

    def __init__(self, descs: np.ndarray, tune: Optional[Tune] = None):
        d = np.ascontiguousarray(descs)
        if d.dtype.itemsize != 64:
            raise ValueError("descriptors must be 64-byte records")
        h = C.c_void_p()
        _check(lib.shmemx_plan_create(d.ctypes.data if len(d) else None, len(d), C.byref(tune) if tune else None,
                                      C.byref(h)), "shmemx_plan_create")
        self._h = h

    def launch_fused(self, results=None, stream=None) -> None:
        _check(lib.shmemx_plan_launch_fused(self._h, _ptr(results), _stream(stream)), "shmemx_plan_launch_fused")

    def launch_per_op(self, results=None, stream=None) -> None:
        _check(lib.shmemx_plan_launch_per_op(self._h, _ptr(results), _stream(stream)), "shmemx_plan_launch_per_op")

    def graph_build(self, form: int, results=None, stream=None) -> None:
        _check(lib.shmemx_plan_graph_build(self._h, form, _ptr(results), _stream(stream)), "shmemx_plan_graph_build")

    def graph_launch(self, stream=None) -> None:
        _check(lib.shmemx_plan_graph_launch(self._h, _stream(stream)), "shmemx_plan_graph_launch")

    def set_stamps(self, stamps) -> None:
        _check(lib.shmemx_plan_set_stamps(self._h, _ptr(stamps)), "shmemx_plan_set_stamps")

    def info(self) -> dict:
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(lib.shmemx_plan_info(self._h, C.byref(a), C.byref(b), C.byref(c)), "shmemx_plan_info")
        return {"tasks": a.value, "phases": b.value, "launches": c.value}

    def destroy(self) -> None:
        if self._h:
            lib.shmemx_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def stamp(dst, stream=None) -> None:
    _check(lib.shmemx_stamp_launch(_ptr(dst), _stream(stream)), "shmemx_stamp_launch")


def autotune(scratch_off: int, scratch_bytes: int, min_bytes: int, max_bytes: int, msgs: int = 256,
             reps: int = 5, stream=None) -> Tune:
    t = Tune()
    _check(lib.shmemx_autotune(scratch_off, scratch_bytes, min_bytes, max_bytes, msgs, reps, C.byref(t),
                               _stream(stream)), "shmemx_autotune")
    return t


def tune_save(t: Tune, path: str) -> None:
    _check(lib.shmemx_tune_save(C.byref(t), path.encode()), "shmemx_tune_save")


def tune_load(path: str) -> Tune:
    t = Tune()
    _check(lib.shmemx_tune_load(C.byref(t), path.encode()), "shmemx_tune_load")
    return t


TUNE_SRC_DEFAULT, TUNE_SRC_FILE, TUNE_SRC_FILE_REFUSED, TUNE_SRC_SET = 0, 1, 2, 3


def tune_set(t: Tune) -> None:
    """Make `t` the library's active tune table."""
    _check(lib.shmemx_tune_set(C.byref(t)), "shmemx_tune_set")


def tune_get():
    """(active tune table, where it came from: TUNE_SRC_*)."""
    t = Tune()
    rc = lib.shmemx_tune_get(C.byref(t))
    if rc < 0:
        raise VshmemError(rc, "shmemx_tune_get")
    return t, rc


# ------------------------------------------------- device descriptor tables
def launch_batch(d_descs, n: int, results=None, d_tune=None, stream=None) -> None:
    """Fused launch over a descriptor table in device memory (a uint8 or
    64-byte-record tensor of at least n descriptors)."""
    _check(lib.shmemx_launch_batch(_ptr(d_descs), n, _ptr(results), _ptr(d_tune), _stream(stream)),
           "shmemx_launch_batch")


def launch_batch_noalloc(d_descs, n: int, results=None, d_tune=None, stream=None) -> None:
    """launch_batch over the library's fixed device workspace (no allocation);
    calls that overlap on one device race."""
    _check(lib.shmemx_launch_batch_noalloc(_ptr(d_descs), n, _ptr(results), _ptr(d_tune), _stream(stream)),
           "shmemx_launch_batch_noalloc")


def launch_batch_noalloc_max() -> int:
    return int(lib.shmemx_launch_batch_noalloc_max())


def launch_per_op(d_descs, n: int, results=None, d_tune=None, stream=None) -> None:
    _check(lib.shmemx_launch_per_op(_ptr(d_descs), n, _ptr(results), _ptr(d_tune), _stream(stream)),
           "shmemx_launch_per_op")


class Graph:
    """A captured launch over a device descriptor table (form 0 per-op, 1 fused)."""

    def __init__(self, d_descs, n: int, form: int, results=None, d_tune=None):
        h = C.c_void_p()
        _check(lib.shmemx_graph_build(_ptr(d_descs), n, _ptr(results), _ptr(d_tune), form, C.byref(h)),
               "shmemx_graph_build")
        self._h = h

    def launch(self, stream=None) -> None:
        _check(lib.shmemx_graph_launch(self._h, _stream(stream)), "shmemx_graph_launch")

    def destroy(self) -> None:
        if self._h:
            lib.shmemx_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# --------------------------------------------------------------- serving
def progress_start(nwg: int = 0, wg_size: int = 0, ring_slots: int = 4096, verify: bool = False,
                   chunk_bytes: int = 256 << 10, idle_timeout_ms: int = 30000, stream=None) -> None:
    cfg = ProgressCfg(nwg, wg_size, ring_slots, 1 if verify else 0, chunk_bytes, idle_timeout_ms)
    _check(lib.shmemx_progress_start(C.byref(cfg), _stream(stream)), "shmemx_progress_start")


PROGRESS_LANES = 8


def progress_submit(desc: Desc, lane: int = 0) -> int:
    t = C.c_uint64()
    _check(lib.shmemx_progress_submit(lane, C.byref(desc), C.byref(t)), "shmemx_progress_submit")
    return t.value


def progress_poll(ticket: int) -> Optional[Completion]:
    c = Completion()
    rc = lib.shmemx_progress_poll(ticket, C.byref(c))
    if rc < 0:
        raise VshmemError(rc, "shmemx_progress_poll")
    return c if rc == 1 else None


def progress_stop(timeout_ms: int = 10000) -> None:
    _check(lib.shmemx_progress_stop(timeout_ms), "shmemx_progress_stop")


def serve_run(reqs: Sequence[Request], lanes: int, region_off: int, region_bytes: int, budget_bytes: int):
    n = len(reqs)
    arr = (Request * n)(*reqs)
    dst = np.zeros(n, dtype=np.uint64)
    lat = np.zeros(n, dtype=np.uint64)
    comps = (Completion * n)()
    stats = ServeStats()
    _check(lib.shmemx_serve_run(arr, n, lanes, region_off, region_bytes, budget_bytes, dst.ctypes.data,
                                lat.ctypes.data, comps, C.byref(stats)), "shmemx_serve_run")
    return dst, lat, comps, stats


def serve_run_per_op(reqs: Sequence[Request], lanes: int, region_off: int, region_bytes: int, budget_bytes: int,
                     chunk_bytes: int = 256 << 10, wg_size: int = 256):
    """The same trace and admission as serve_run, one kernel launch per request."""
    n = len(reqs)
    arr = (Request * n)(*reqs)
    dst = np.zeros(n, dtype=np.uint64)
    lat = np.zeros(n, dtype=np.uint64)
    comps = (Completion * n)()
    stats = ServeStats()
    _check(lib.shmemx_serve_run_per_op(arr, n, lanes, region_off, region_bytes, budget_bytes, chunk_bytes, wg_size,
                                       dst.ctypes.data, lat.ctypes.data, comps, C.byref(stats)),
           "shmemx_serve_run_per_op")
    return dst, lat, comps, stats


def serve_run_batched(reqs: Sequence[Request], lanes: int, region_off: int, region_bytes: int, budget_bytes: int,
                      window_us: float = 20.0, use_graph: bool = False, chunk_bytes: int = 256 << 10,
                      wg_size: int = 1024):
    """The same trace and admission as serve_run, in windowed batches (fused
    launches, or graph replays with use_graph)."""
    n = len(reqs)
    arr = (Request * n)(*reqs)
    dst = np.zeros(n, dtype=np.uint64)
    lat = np.zeros(n, dtype=np.uint64)
    comps = (Completion * n)()
    stats = ServeStats()
    _check(lib.shmemx_serve_run_batched(arr, n, lanes, region_off, region_bytes, budget_bytes, int(window_us * 1000),
                                        1 if use_graph else 0, chunk_bytes, wg_size, dst.ctypes.data, lat.ctypes.data,
                                        comps, C.byref(stats)), "shmemx_serve_run_batched")
    return dst, lat, comps, stats


def launch_request(desc: Desc, chunk_bytes: int = 256 << 10, wg_size: int = 256, stream=None) -> None:
    _check(lib.shmemx_launch_request(C.byref(desc), chunk_bytes, wg_size, _stream(stream)), "shmemx_launch_request")


def version() -> str:
    return lib.shmemx_version().decode()
