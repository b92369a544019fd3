"""Host-issued operations of libvshmem.so: the host default context (blocking
and _nbi RMA, AMOs, signals, waits, quiet, barriers and collectives, the
calling thread acting for PE 0) and the stream-triggered _on_stream calls.
Argument marshalling only; the declarations and their semantics are in
include/vshmem.h.  Buffers are ints (addresses), numpy arrays or torch
tensors; symmetric operands are canonical symmetric addresses."""
from __future__ import annotations

from . import DT_BF16, DT_FP32, DT_INT64, RED_MAX, RED_SUM, TEAM_WORLD, VshmemError, _check, _stream, lib


def _addr(x) -> int:
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"not a buffer: {type(x)!r}")


def _void(fn, what: str, *args):
    lib.shmemx_clear_last_error()
    out = fn(*args)
    rc = lib.shmemx_last_error()
    if rc:
        raise VshmemError(rc, what)
    return out


# ----------------------------------------------------------- RMA and signals
def putmem(dest: int, src, n: int, pe: int) -> None:
    _void(lib.shmem_putmem, "shmem_putmem", dest, _addr(src), n, pe)


def getmem(dest, src: int, n: int, pe: int) -> None:
    _void(lib.shmem_getmem, "shmem_getmem", _addr(dest), src, n, pe)


def putmem_nbi(dest: int, src, n: int, pe: int) -> None:
    _void(lib.shmem_putmem_nbi, "shmem_putmem_nbi", dest, _addr(src), n, pe)


def getmem_nbi(dest, src: int, n: int, pe: int) -> None:
    _void(lib.shmem_getmem_nbi, "shmem_getmem_nbi", _addr(dest), src, n, pe)


def putmem_signal(dest: int, src, n: int, sig: int, signal: int, sig_op: int, pe: int) -> None:
    _void(lib.shmem_putmem_signal, "shmem_putmem_signal", dest, _addr(src), n, sig, signal, sig_op, pe)


def putmem_signal_nbi(dest: int, src, n: int, sig: int, signal: int, sig_op: int, pe: int) -> None:
    _void(lib.shmem_putmem_signal_nbi, "shmem_putmem_signal_nbi", dest, _addr(src), n, sig, signal, sig_op, pe)


def signal_fetch(sig: int) -> int:
    return _void(lib.shmem_signal_fetch, "shmem_signal_fetch", sig)


def signal_wait_until(sig: int, cmp: int, value: int) -> int:
    return _void(lib.shmem_signal_wait_until, "shmem_signal_wait_until", sig, cmp, value)


def int64_wait_until(ivar: int, cmp: int, value: int) -> None:
    _void(lib.shmem_int64_wait_until, "shmem_int64_wait_until", ivar, cmp, value)


def int64_test(ivar: int, cmp: int, value: int) -> bool:
    return bool(_void(lib.shmem_int64_test, "shmem_int64_test", ivar, cmp, value))


# -------------------------------------------------------------------- AMOs
def int64_atomic_fetch_add(dest: int, value: int, pe: int) -> int:
    return _void(lib.shmem_int64_atomic_fetch_add, "shmem_int64_atomic_fetch_add", dest, value, pe)


def int64_atomic_add(dest: int, value: int, pe: int) -> None:
    _void(lib.shmem_int64_atomic_add, "shmem_int64_atomic_add", dest, value, pe)


def int64_atomic_fetch_xor(dest: int, value: int, pe: int) -> int:
    return _void(lib.shmem_int64_atomic_fetch_xor, "shmem_int64_atomic_fetch_xor", dest, value, pe)


def int64_atomic_xor(dest: int, value: int, pe: int) -> None:
    _void(lib.shmem_int64_atomic_xor, "shmem_int64_atomic_xor", dest, value, pe)


def uint64_atomic_fetch_xor(dest: int, value: int, pe: int) -> int:
    return _void(lib.shmem_uint64_atomic_fetch_xor, "shmem_uint64_atomic_fetch_xor", dest, value, pe)


def uint64_atomic_xor(dest: int, value: int, pe: int) -> None:
    _void(lib.shmem_uint64_atomic_xor, "shmem_uint64_atomic_xor", dest, value, pe)


def int64_atomic_compare_swap(dest: int, cond: int, value: int, pe: int) -> int:
    return _void(lib.shmem_int64_atomic_compare_swap, "shmem_int64_atomic_compare_swap", dest, cond, value, pe)


def int64_atomic_fetch(source: int, pe: int) -> int:
    return _void(lib.shmem_int64_atomic_fetch, "shmem_int64_atomic_fetch", source, pe)


def int64_atomic_set(dest: int, value: int, pe: int) -> None:
    _void(lib.shmem_int64_atomic_set, "shmem_int64_atomic_set", dest, value, pe)


def int64_atomic_swap(dest: int, value: int, pe: int) -> int:
    return _void(lib.shmem_int64_atomic_swap, "shmem_int64_atomic_swap", dest, value, pe)


# ------------------------------------------------------ ordering and sync
def quiet() -> None:
    _void(lib.shmem_quiet, "shmem_quiet")


def fence() -> None:
    _void(lib.shmem_fence, "shmem_fence")


def barrier_all() -> None:
    _void(lib.shmem_barrier_all, "shmem_barrier_all")


def sync_all() -> None:
    _void(lib.shmem_sync_all, "shmem_sync_all")


def team_sync(team: int = TEAM_WORLD) -> None:
    _check(lib.shmem_team_sync(team), "shmem_team_sync")


# ------------------------------------------------------------- collectives
def broadcastmem(dest: int, src: int, n: int, root: int, team: int = TEAM_WORLD) -> None:
    _check(lib.shmem_broadcastmem(team, dest, src, n, root), "shmem_broadcastmem")


def fcollectmem(dest: int, src: int, n: int, team: int = TEAM_WORLD) -> None:
    _check(lib.shmem_fcollectmem(team, dest, src, n), "shmem_fcollectmem")


def alltoallmem(dest: int, src: int, n: int, team: int = TEAM_WORLD) -> None:
    _check(lib.shmem_alltoallmem(team, dest, src, n), "shmem_alltoallmem")


_REDUCE = {
    (DT_INT64, RED_SUM): "shmem_int64_sum_reduce", (DT_INT64, RED_MAX): "shmem_int64_max_reduce",
    (DT_FP32, RED_SUM): "shmem_float_sum_reduce", (DT_FP32, RED_MAX): "shmem_float_max_reduce",
    (DT_BF16, RED_SUM): "shmemx_bfloat16_sum_reduce", (DT_BF16, RED_MAX): "shmemx_bfloat16_max_reduce",
}


def reduce(dtype: int, op: int, dest: int, src: int, nreduce: int, team: int = TEAM_WORLD) -> None:
    """The typed host reduction for (dtype, op), e.g. shmem_int64_sum_reduce."""
    name = _REDUCE[(dtype, op)]
    _check(getattr(lib, name)(team, dest, src, nreduce), name)


# ------------------------------------------------------- stream-triggered
def putmem_on_stream(dest: int, src, n: int, pe: int, stream=None) -> None:
    _check(lib.shmemx_putmem_on_stream(dest, _addr(src), n, pe, _stream(stream)), "shmemx_putmem_on_stream")


def getmem_on_stream(dest, src: int, n: int, pe: int, stream=None) -> None:
    _check(lib.shmemx_getmem_on_stream(_addr(dest), src, n, pe, _stream(stream)), "shmemx_getmem_on_stream")


def putmem_signal_on_stream(dest: int, src, n: int, sig: int, signal: int, sig_op: int, pe: int,
                            stream=None) -> None:
    _check(lib.shmemx_putmem_signal_on_stream(dest, _addr(src), n, sig, signal, sig_op, pe, _stream(stream)),
           "shmemx_putmem_signal_on_stream")


def signal_wait_until_on_stream(sig: int, cmp: int, value: int, stream=None) -> None:
    _check(lib.shmemx_signal_wait_until_on_stream(sig, cmp, value, _stream(stream)),
           "shmemx_signal_wait_until_on_stream")


def barrier_all_on_stream(stream=None) -> None:
    _check(lib.shmemx_barrier_all_on_stream(_stream(stream)), "shmemx_barrier_all_on_stream")


def team_sync_on_stream(team: int, stream=None) -> None:
    _check(lib.shmemx_team_sync_on_stream(team, _stream(stream)), "shmemx_team_sync_on_stream")


def quiet_on_stream(stream=None) -> None:
    _check(lib.shmemx_quiet_on_stream(_stream(stream)), "shmemx_quiet_on_stream")


def broadcastmem_on_stream(dest: int, src: int, n: int, root: int, team: int = TEAM_WORLD, stream=None) -> None:
    _check(lib.shmemx_broadcastmem_on_stream(team, dest, src, n, root, _stream(stream)),
           "shmemx_broadcastmem_on_stream")


def fcollectmem_on_stream(dest: int, src: int, n: int, team: int = TEAM_WORLD, stream=None) -> None:
    _check(lib.shmemx_fcollectmem_on_stream(team, dest, src, n, _stream(stream)), "shmemx_fcollectmem_on_stream")


def alltoallmem_on_stream(dest: int, src: int, n: int, team: int = TEAM_WORLD, stream=None) -> None:
    _check(lib.shmemx_alltoallmem_on_stream(team, dest, src, n, _stream(stream)), "shmemx_alltoallmem_on_stream")


def reduce_on_stream(dtype: int, op: int, dest: int, src: int, nreduce: int, team: int = TEAM_WORLD,
                     stream=None) -> None:
    _check(lib.shmemx_reduce_on_stream(team, dtype, op, dest, src, nreduce, _stream(stream)),
           "shmemx_reduce_on_stream")

