"""CPU oracle of the virtual-PE OpenSHMEM semantics (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  The product library never imports it.  The arithmetic lives in
``vshmem_oracle.c`` (plain C, gcc); this module only marshals numpy arrays.

Heaps are numpy arrays of shape (npes, stride) and dtype uint8: row p is PE
p's symmetric heap slice.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vshmem_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

ERRORS = {0: "ok", -1: "bad argument", -2: "out of range", -3: "conflict",
          -4: "deadlock", -5: "bad op", -6: "out of memory", -7: "search budget exhausted"}

DT_INT64, DT_FP32, DT_BF16 = 0, 1, 2
RO_SUM, RO_MAX = 0, 1


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"oracle error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liborc.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64 = ctypes.c_uint64
        vp = ctypes.c_void_p
        L.orc_run_program.argtypes = [vp, ctypes.c_int, u64, vp, u64, vp, u64, ctypes.c_int,
                                      ctypes.c_char_p, ctypes.c_int]
        L.orc_run_program.restype = ctypes.c_int
        for name in ("orc_fcollect", "orc_alltoall"):
            f = getattr(L, name)
            f.argtypes = [vp, ctypes.c_int, u64, ctypes.c_int, ctypes.c_int, ctypes.c_int, u64, u64, u64]
            f.restype = ctypes.c_int
        L.orc_broadcast.argtypes = [vp, ctypes.c_int, u64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    u64, u64, u64, ctypes.c_int]
        L.orc_broadcast.restype = ctypes.c_int
        L.orc_reduce.argtypes = [vp, ctypes.c_int, u64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, u64, u64, u64, vp, u64, vp]
        L.orc_reduce.restype = ctypes.c_int
        L.orc_bf16_round.argtypes = [ctypes.c_float]
        L.orc_bf16_round.restype = ctypes.c_uint16
        L.orc_gups.argtypes = [vp, u64, vp, vp, vp, u64, vp]
        L.orc_gups.restype = ctypes.c_int
        L.orc_witness_check.argtypes = [vp, vp, vp, vp, u64, vp, vp, u64, u64]
        L.orc_witness_check.restype = ctypes.c_int64
        for f in (L.orc_host_put, L.orc_host_get):
            f.argtypes = [vp, ctypes.c_int, u64, ctypes.c_int, u64, vp, u64]
            f.restype = ctypes.c_int
        del u8p
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, msg: str = ""):
    if rc != 0:
        raise OracleError(rc, msg)


def _heap_args(heap: np.ndarray):
    assert heap.dtype == np.uint8 and heap.ndim == 2 and heap.flags["C_CONTIGUOUS"]
    return _ptr(heap), heap.shape[0], heap.shape[1]


def run_program(heap: np.ndarray, descs: np.ndarray, nresults: int = 0, check: bool = True) -> np.ndarray:
    """Apply a multi-PE program in place; returns fetched values (uint64)."""
    descs = np.ascontiguousarray(descs)
    assert descs.dtype.itemsize == 64
    res = np.zeros(max(1, nresults), dtype=np.uint64)
    err = ctypes.create_string_buffer(256)
    hp, npes, stride = _heap_args(heap)
    rc = lib().orc_run_program(hp, npes, stride, _ptr(descs), len(descs), _ptr(res), nresults,
                               1 if check else 0, err, 256)
    _check(rc, err.value.decode())
    return res[:nresults]


def host_put(heap, pe: int, dst: int, buf: np.ndarray) -> None:
    """Host-initiated put from a private host buffer into PE pe's copy."""
    hp, npes, stride = _heap_args(heap)
    b = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(lib().orc_host_put(hp, npes, stride, pe, dst, _ptr(b), b.size))


def host_get(heap, pe: int, src: int, n: int) -> np.ndarray:
    """Host-initiated get of PE pe's bytes [src, src + n) into a new buffer."""
    hp, npes, stride = _heap_args(heap)
    out = np.zeros(n, dtype=np.uint8)
    _check(lib().orc_host_get(hp, npes, stride, pe, src, _ptr(out), n))
    return out


def broadcast(heap, dst, src, n, root, team=None):
    hp, npes, stride = _heap_args(heap)
    start, st, size = team or (0, 1, npes)
    _check(lib().orc_broadcast(hp, npes, stride, start, st, size, dst, src, n, root))


def fcollect(heap, dst, src, n, team=None):
    hp, npes, stride = _heap_args(heap)
    start, st, size = team or (0, 1, npes)
    _check(lib().orc_fcollect(hp, npes, stride, start, st, size, dst, src, n))


def alltoall(heap, dst, src, n, team=None):
    hp, npes, stride = _heap_args(heap)
    start, st, size = team or (0, 1, npes)
    _check(lib().orc_alltoall(hp, npes, stride, start, st, size, dst, src, n))


_DT_NP = {DT_INT64: np.int64, DT_FP32: np.float32, DT_BF16: np.uint16}


def reduce(heap, dt, rop, dst, src, nreduce, team=None, only: Optional[Sequence[int]] = None):
    """Reduce-to-all over the team.  With ``only``, returns those elements'
    results instead of writing the heap."""
    hp, npes, stride = _heap_args(heap)
    start, st, size = team or (0, 1, npes)
    if only is None:
        _check(lib().orc_reduce(hp, npes, stride, start, st, size, dt, rop, dst, src, nreduce,
                                None, 0, None))
        return None
    idx = np.ascontiguousarray(np.asarray(only, dtype=np.uint64))
    out = np.zeros(len(idx), dtype=_DT_NP[dt])
    _check(lib().orc_reduce(hp, npes, stride, start, st, size, dt, rop, dst, src, nreduce,
                            _ptr(idx), len(idx), _ptr(out)))
    return out


def reduce_columns(cols: np.ndarray, dt: int, rop: int) -> np.ndarray:
    """TREE-reduce a (P, K) array of per-PE values column by column (sampled
    outputs): each column is one output element."""
    P, K = cols.shape
    es = {DT_INT64: 8, DT_FP32: 4, DT_BF16: 2}[dt]
    heap = np.ascontiguousarray(cols.astype(_DT_NP[dt], copy=False)).view(np.uint8).reshape(P, K * es)
    heap = np.ascontiguousarray(heap)
    return reduce(heap, dt, rop, 0, 0, K, only=np.arange(K))


def bf16_round(f: float) -> int:
    return int(lib().orc_bf16_round(ctypes.c_float(f)))


def gups(table: np.ndarray, idx: np.ndarray, val: np.ndarray, is_add: np.ndarray,
         want_fetched: bool = False) -> Optional[np.ndarray]:
    assert table.dtype == np.int64 and table.flags["C_CONTIGUOUS"]
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    val = np.ascontiguousarray(val, dtype=np.uint64)
    ia = np.ascontiguousarray(is_add, dtype=np.uint8)
    fetched = np.zeros(len(idx), dtype=np.uint64) if want_fetched else None
    _check(lib().orc_gups(_ptr(table), table.size, _ptr(idx), _ptr(val), _ptr(ia), len(idx), _ptr(fetched)))
    return fetched


KIND_FETCH_ADD, KIND_FETCH_XOR, KIND_FETCH = 0, 1, 2


def witness_check(addr, kind, val, fetched, init, final, budget: int = 1 << 26) -> int:
    """Number of words whose fetched values admit no serial order (0 = valid)."""
    addr = np.ascontiguousarray(addr, dtype=np.uint64)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    val = np.ascontiguousarray(val, dtype=np.uint64)
    fetched = np.ascontiguousarray(fetched, dtype=np.uint64)
    init = np.ascontiguousarray(init, dtype=np.uint64)
    final = np.ascontiguousarray(final, dtype=np.uint64)
    rc = lib().orc_witness_check(_ptr(addr), _ptr(kind), _ptr(val), _ptr(fetched), len(addr),
                                 _ptr(init), _ptr(final), len(init), budget)
    if rc < 0:
        raise OracleError(int(rc), "witness replay")
    return int(rc)
