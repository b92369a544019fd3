"""Shared helpers for the GPU parity tests: attach a heap of a given shape,
move whole heaps between host numpy arrays and the device, and run the CPU
oracle on the same inputs."""
from __future__ import annotations

import contextlib

import numpy as np


def vs():
    import paper_2607_08006_amd as v
    return v


def torch():
    import torch as t
    return t


@contextlib.contextmanager
def heap(npes: int, bytes_per_pe: int):
    v = vs()
    if v.initialized():
        v.finalize()
    v.init(npes, bytes_per_pe)
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
    assert vs().device_errors() == 0


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

