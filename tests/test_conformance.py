"""Conformance suite: one test per representative conformance item of the
paper's Section 8 (context visibility, space symmetry, GPU space at init,
ordering and completion, stream ordering, pointer accessibility, progress),
each checking what the capability record reports against observed
behaviour.  The optional work-group-scoped device collectives are covered by
tests/test_gpu_devapi.py (participation by every thread of the stated
scope)."""
import ctypes
import os
import subprocess
import sys
import textwrap
import time

import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, download, heap, torch, upload, user_lib

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_context_visibility():
    """A default device context exists when device-initiated support is
    reported, kernels can use it, explicit contexts work when reported, and
    the device handle is gone after finalisation."""
    lib = user_lib()
    t = torch()
    with heap(6, 2 << 20) as v:
        caps = v.query_capabilities(v.TEAM_WORLD)
        assert caps["device_initiated"] == 1 and caps["device_ctx_default"] == 1
        tok = v.calloc(1, 8)
        bad = t.zeros(1, dtype=t.int64, device="cuda")
        dteam = v.team_device(v.TEAM_WORLD)
        assert lib.usertest_barrier(v.device_ctx(), ctypes.byref(dteam), v.SCOPE_WG, 1, 8, tok, bad.data_ptr(), 64,
                                    None) == 0
        t.cuda.synchronize()
        assert int(bad.item()) == 0
        assert caps["explicit_device_ctx"] == 1
        ctx = v.device_ctx_create(v.TEAM_WORLD)
        n = 256
        src, dst, back, ctr = v.malloc(n), v.malloc(n), v.malloc(n), v.calloc(1, 8)
        ids = t.zeros(12, dtype=t.int32, device="cuda")
        fetched = t.zeros(6, dtype=t.int64, device="cuda")
        assert lib.usertest_ctx(v.device_ctx_record(ctx), 6, src, dst, back, n, ctr, ids.data_ptr(),
                                fetched.data_ptr(), 64, None) == 0
        t.cuda.synchronize()
        assert sorted(fetched.cpu().tolist()) == list(range(6))
        assert_no_device_errors()
    assert not v.lib.shmemx_device_ctx()
    assert not v.lib.shmemx_device_ctx_record(0)


def test_space_symmetry():
    """Collective allocation yields one offset naming the object on every
    PE; the same call sequence yields the same offsets on a new heap; every
    PE's copy is addressable and holds what was written to it."""
    from paper_2607_08006_amd import host
    seqs = []
    for _ in range(2):
        with heap(5, 4 << 20) as v:
            a = v.malloc(1000)
            b = v.align(4096, 333)
            c = v.calloc(10, 8)
            v.free(a)
            d = v.malloc(500)                    # first fit reuses a's space
            seqs.append([v.offset(x) for x in (a, b, c, d)])
            assert v.offset(d) == v.offset(a) and v.offset(b) % 4096 == 0
            for pe in range(5):
                assert v.ptr(b, pe) == v.heap_base() + pe * v.heap_stride() + v.offset(b)
                host.putmem(b, np.full(333, 10 + pe, dtype=np.uint8), 333, pe)
            got = download(v.offset(b) + 333)[:, v.offset(b):]
            assert all((got[pe] == 10 + pe).all() for pe in range(5))
    assert seqs[0] == seqs[1]


def test_gpu_space_at_init():
    """The GPU heap exists at initialisation and is the default heap: both
    allocators return symmetric device addresses inside it without any
    space creation.  The environment-configured shmem_init path is checked
    in a fresh process."""
    with heap(3, 4 << 20) as v:
        caps = v.query_capabilities(v.TEAM_WORLD)
        assert caps["gpu_heap"] == 1 and caps["default_heap_is_gpu"] == 1 and caps["host_initiated"] == 1
        a, g = v.malloc(4096), v.shmemg_malloc(4096)
        base, total = v.heap_base(), 3 * v.heap_stride()
        assert all(base <= x < base + v.heap_user_bytes() for x in (a, g)) and a != g
        assert all(v.ptr(x, 2) < base + total for x in (a, g))
    script = textwrap.dedent(f"""
        import ctypes, sys
        sys.path.insert(0, {ROOT!r})
        import torch
        torch.cuda.init()
        import paper_2607_08006_amd as v
        v.lib.shmem_init()
        assert v.lib.shmemx_last_error() == 0, v.lib.shmemx_last_error()
        assert v.lib.shmem_n_pes() == 3 and v.lib.shmem_my_pe() == 0
        assert v.lib.shmemx_heap_user_bytes() >= (5 << 20)
        p = v.lib.shmem_malloc(1 << 20)
        assert p and v.lib.shmem_ptr(p, 2) == p + 2 * v.lib.shmemx_heap_stride()
        c = v.Caps()
        assert v.lib.shmem_query_capabilities(0, ctypes.byref(c)) == 0 and c.gpu_heap == 1 and c.npes == 3
        v.lib.shmem_finalize()
        assert v.lib.shmem_n_pes() == 0
        print("init ok")
    """)
    env = dict(os.environ, VSHMEM_NPES="3", VSHMEM_SYMMETRIC_SIZE="5M")
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0 and "init ok" in r.stdout, r.stderr[-2000:]


def test_quiet_completes_and_fence_orders():
    """quiet: host-issued non-blocking puts are complete and visible once it
    returns.  fence: a device producer's data, put before a fence, is always
    in place when the consumer observes the flag set after the fence."""
    from paper_2607_08006_amd import host
    lib = user_lib()
    t = torch()
    npes = 4
    with heap(npes, 4 << 20) as v:
        blk = v.malloc(1 << 20)
        flag = v.calloc(1, 8)
        region = v.offset(flag) + 8
        init = np.zeros((npes, region), dtype=np.uint8)
        upload(init)
        ref = init.copy()
        bufs = [t.from_numpy(W.heap_fill(60 + i, 1, 65536)[0].copy()).pin_memory() for i in range(16)]
        for i, b in enumerate(bufs):
            host.putmem_nbi(blk + 65536 * i, b, 65536, i % npes)
            oracle.host_put(ref, i % npes, v.offset(blk) + 65536 * i, b.numpy())
        host.quiet()
        assert np.array_equal(download(region), ref)
        upload(init)
        bad = t.zeros(1, dtype=t.int64, device="cuda")
        for prod, cons in ((0, 3), (2, 1)):
            upload(init)
            assert lib.usertest_fence(v.device_ctx(), prod, cons, blk, (1 << 20) // 8, flag, 200, bad.data_ptr(),
                                      None) == 0
            t.cuda.synchronize()
            assert int(bad.item()) == 0, (prod, cons)
        assert_no_device_errors()


def test_stream_ordering():
    """Stream-triggered operations run in stream order, and an event orders
    work across two streams."""
    from paper_2607_08006_amd import host
    t = torch()
    npes, n = 4, 1 << 18
    with heap(npes, 2 << 20) as v:
        caps = v.query_capabilities(v.TEAM_WORLD)
        assert caps["stream_triggered"] == 1
        a = v.malloc(n)
        region = v.offset(a) + n
        upload(np.zeros((npes, region), dtype=np.uint8))
        s1, s2 = t.cuda.Stream(), t.cuda.Stream()
        payloads = [t.from_numpy(W.heap_fill(90 + k, 1, n)[0].copy()).pin_memory() for k in range(3)]
        out = t.zeros(n, dtype=t.uint8).pin_memory()
        t.cuda.synchronize()
        # the later put of the same bytes wins, and the get sees it
        for p in payloads:
            host.putmem_on_stream(a, p, n, 2, stream=s1)
        ev = t.cuda.Event()
        ev.record(s1)
        s2.wait_event(ev)
        host.getmem_on_stream(out, a, n, 2, stream=s2)
        s2.synchronize()
        assert np.array_equal(out.numpy(), payloads[-1].numpy())
        assert_no_device_errors()


def test_pointer_accessibility():
    """shmem_ptr reports the device domain and returns the PE's copy inside
    the device heap, or nothing for PEs out of range and non-symmetric
    addresses."""
    with heap(4, 2 << 20) as v:
        caps = v.query_capabilities(v.TEAM_WORLD)
        assert caps["ptr_domain"] == 2     # device
        x = v.malloc(64)
        for pe in range(4):
            p = v.ptr(x, pe)
            assert p == v.heap_base() + pe * v.heap_stride() + v.offset(x)
            view = v.heap_view()[pe, v.offset(x):v.offset(x) + 64]
            assert view.data_ptr() == p and view.is_cuda
        assert v.ptr(x, 4) is None and v.ptr(x, -1) is None
        tm = v.team_split_strided(v.TEAM_WORLD, 1, 2, 2)    # PEs 1 and 3
        assert v.team_ptr(tm, x, 1) == v.ptr(x, 3) and v.team_ptr(tm, x, 2) is None
        assert v.team_ptr(999, x, 0) is None
        assert v.ptr(torch().zeros(8, device="cuda").data_ptr(), 0) is None


def test_progress():
    """Progress needs the host only to submit: device-initiated operations
    inside one kernel complete without it (signal ping-pong), and the
    persistent progress kernel completes requests the host queues while it
    runs.  The capability record reports both models."""
    t = torch()
    npes = 4
    with heap(npes, 4 << 20) as v:
        caps = v.query_capabilities(v.TEAM_WORLD)
        assert caps["progress"] == 0x3    # kernel launch and persistent GPU
        data, sig = v.malloc(64), v.calloc(1, 8)
        upload(np.zeros((npes, v.offset(sig) + 8), dtype=np.uint8))
        pairs = t.arange(4, dtype=t.int32, device="cuda")
        rtt = t.zeros(2 * 50, dtype=t.int64, device="cuda")
        v.pingpong(v.offset(data), v.offset(sig), pairs, 2, 50, 8, False, rtt)
        t.cuda.synchronize()
        assert (rtt.cpu().numpy() > 0).all()
        region = 2 << 20
        init = W.heap_fill(404, npes, region)
        upload(init)
        side = t.cuda.Stream()
        v.progress_start(nwg=8, wg_size=256, ring_slots=16, chunk_bytes=64 << 10, stream=side)
        recs = [(W.OP_PUT, 0, 0, 0, 1, W.NO_RESULT, 4096 * k, (1 << 20) + 4096 * k, 4096, 0, 0) for k in range(8)]
        descs = W.descs(recs)
        tickets = [v.progress_submit(v.Desc.from_buffer_copy(descs[k:k + 1].tobytes())) for k in range(8)]
        done, t0 = set(), time.time()
        while len(done) < len(tickets) and time.time() - t0 < 30:
            done |= {tk for tk in tickets if tk not in done and v.progress_poll(tk) is not None}
        v.progress_stop(10000)
        side.synchronize()
        assert len(done) == len(tickets)
        ref = init.copy()
        oracle.run_program(ref, descs)
        assert np.array_equal(download(region), ref)
        assert_no_device_errors()
