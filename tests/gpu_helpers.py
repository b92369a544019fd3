"""Shared helpers for the GPU parity tests: attach a heap of a given shape,
move whole heaps between host numpy arrays and the device, and run the CPU
oracle on the same inputs."""
from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np

import workload as W

USER_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "devapi", "libvshmem_usertest.so")
_user = None


def vs():
    import paper_2607_08006_amd as v
    return v


def torch():
    import torch as t
    return t


@contextlib.contextmanager
def heap(npes: int, bytes_per_pe: int, spread: bool = True):
    v = vs()
    if v.initialized():
        v.finalize()
    v.init(npes, bytes_per_pe, spread=spread)
    try:
        yield v
    finally:
        torch().cuda.synchronize()
        v.finalize()


def upload(init: np.ndarray) -> None:
    """Write host rows (npes, n) into the first n bytes of every PE slice."""
    t = torch()
    h = vs().heap_view()
    n = init.shape[1]
    h[:, :n].copy_(t.from_numpy(np.ascontiguousarray(init)).to("cuda"))
    t.cuda.synchronize()


def download(n: int) -> np.ndarray:
    t = torch()
    t.cuda.synchronize()
    return vs().heap_view()[:, :n].cpu().numpy().copy()


def device_array(a: np.ndarray):
    return torch().from_numpy(np.ascontiguousarray(a)).to("cuda")


def assert_no_device_errors():
    e = vs().device_errors()
    assert e == 0, f"device error word {e:#x}"


GOLD = 0x9E3779B97F4A7C15


def out_hash(b: np.ndarray) -> int:
    """Output hash of the progress kernel's completion records: XOR over the
    8-byte words w_i (zero padded) of mix(w_i ^ ((i + 1) * golden))."""
    n = len(b)
    pad = np.zeros(((n + 7) // 8) * 8, dtype=np.uint8)
    pad[:n] = b
    w = pad.view("<u8")
    idx = np.arange(1, len(w) + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = w ^ (idx * np.uint64(GOLD))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return int(np.bitwise_xor.reduce(z)) if len(z) else 0



def user_lib():
    """The user-style kernels of tests/devapi (their own library, built by
    __graft_entry__.build()); fails when it is missing."""
    global _user
    if _user is not None:
        return _user
    if not os.path.exists(USER_LIB):
        raise RuntimeError(f"{USER_LIB} is not built; run __graft_entry__.build()")
    vs()   # torch's runtime and libvshmem.so first, as the package arranges for itself
    lib = ctypes.CDLL(USER_LIB)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    sigs = {
        "usertest_collective": [vp, vp, i32, i32, i32, vp, vp, sz, i32, i32, i32, vp, vp],
        "usertest_pipeline": [vp, vp, vp, vp, vp, vp, sz, sz, i32, i32, vp],
        "usertest_barrier": [vp, vp, i32, i32, i32, vp, vp, i32, vp],
        "usertest_ctx": [vp, i32, vp, vp, vp, sz, vp, vp, vp, i32, vp],
        "usertest_gspace": [vp, i32, vp, vp, vp, vp, sz, sz, sz, vp],
        "usertest_fence": [vp, i32, i32, vp, sz, vp, i32, vp, vp],
        "usertest_debug": [vp, vp, vp, i32, vp, vp, vp, i32, vp],
        "usertest_write_table": [vp, sz, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = i32
    _user = lib
    return lib


def _dev(a, dtype):
    return torch().from_numpy(np.ascontiguousarray(a).astype(dtype)).to("cuda")


def write_table(descs: np.ndarray, out=None):
    """Have a kernel write `descs` into a device table (a uint8 tensor of
    64 bytes per record); returns the table."""
    t = torch()
    n = len(descs)
    if out is None:
        out = t.zeros(max(1, n) * 64, dtype=t.uint8, device="cuda")
    code = (descs["op"].astype(np.uint32) | (descs["scope"].astype(np.uint32) << 8) |
            (descs["aux"].astype(np.uint32) << 16) | (descs["flags"].astype(np.uint32) << 24))
    cols = [_dev(code.view(np.int32), np.int32), _dev(descs["issuer"], np.int32), _dev(descs["target"], np.int32),
            _dev(descs["result_idx"].view(np.int32), np.int32)]
    cols += [_dev(descs[f].view(np.int64), np.int64) for f in ("src", "dst", "nbytes", "value", "cond")]
    rc = user_lib().usertest_write_table(out.data_ptr(), n, *[c.data_ptr() for c in cols], None)
    assert rc == 0
    t.cuda.synchronize()
    return out


def program(seed, npes=4, heap_bytes=1 << 20, base_off=0, n_rma=600, n_amo=3000, fences=40):
    """The 4-PE mixed workload (put/get epochs separated by barriers, then
    contended fetch_add) with per-PE fences inserted at seeded positions."""
    wl = W.small_workload(seed=seed, npes=npes, heap_bytes=heap_bytes, n_rma=n_rma, epoch_ops=100, n_amo=n_amo,
                          base_off=base_off)
    d = wl.descs
    x = W.splitmix64(W.subseed(seed, 0xFE), 0, 2 * fences)
    pos = np.sort(W.bounded(x[0::2], 0, len(d) - 1))
    who = W.bounded(x[1::2], 0, npes - 1)
    parts, last = [], 0
    for p, w in zip(pos, who):
        parts.append(d[last:p])
        parts.append(W.descs([(W.OP_FENCE, W.SCOPE_THREAD, 0, int(w), int(w), W.NO_RESULT, 0, 0, 0, 0, 0)]))
        last = p
    parts.append(d[last:])
    return wl, np.concatenate(parts)
