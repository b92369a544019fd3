"""GPU parity: host-initiated operations through the host default context
(the host acting for PE 0) and stream-triggered operations, against the CPU
oracle.  Private host buffers follow the oracle's host put/get; heap-to-heap
moves and atomics follow PE 0's program in the oracle."""
import time

import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, download, heap, torch, upload

pytestmark = pytest.mark.gpu


def _desc(op, target, src=0, dst=0, n=0, value=0, cond=0, aux=0, ridx=W.NO_RESULT):
    return W.descs([(op, W.SCOPE_THREAD, aux, 0, target, ridx, src, dst, n, value, cond)])


def _buffers(t, nbytes, seed):
    """The same seeded bytes in pageable numpy memory, pinned host memory and
    device memory."""
    data = W.heap_fill(seed, 1, nbytes)[0]
    pinned = t.from_numpy(data.copy()).pin_memory()
    dev = t.from_numpy(data.copy()).cuda()
    t.cuda.synchronize()   # host operations are not ordered after work on other streams
    return data, {"pageable": data.copy(), "pinned": pinned, "device": dev}


def _as_numpy(b):
    return b if isinstance(b, np.ndarray) else b.cpu().numpy()


@pytest.mark.parametrize("npes", [1, 5])
def test_host_put_get_every_buffer_kind(npes):
    from paper_2607_08006_amd import host
    t = torch()
    with heap(npes, 4 << 20) as v:
        region = v.offset(v.malloc(3 << 20)) + (3 << 20)
        init = W.heap_fill(W.SEED_SMALL + npes, npes, region)
        upload(init)
        ref = init.copy()
        base = v.heap_base()
        k = 0
        for n in (1, 13, 4096 + 7, (1 << 20) + 3):
            data, bufs = _buffers(t, n, 1000 + n)
            for kind, b in bufs.items():
                pe = (k * 3) % npes
                dst = 17 + (k * 104_729) % (region - n - 17)
                host.putmem(base + dst, b, n, pe)
                oracle.host_put(ref, pe, dst, data)
                k += 1
            # heap to heap: a canonical symmetric source is PE 0's copy
            pe, src, dst = npes - 1, 40, region - n - 9
            host.putmem(base + dst, base + src, n, pe)
            oracle.run_program(ref, _desc(W.OP_PUT, pe, src=src, dst=dst, n=n), check=False)
            got = download(region)
            assert np.array_equal(got, ref), n
            # gets into every kind of buffer
            for kind, b in bufs.items():
                pe, src = (k * 5) % npes, (k * 7919) % (region - n)
                if kind == "pageable":
                    b[:] = 0
                else:
                    b.zero_()
                    t.cuda.synchronize()
                host.getmem(b, base + src, n, pe)
                assert np.array_equal(_as_numpy(b), oracle.host_get(ref, pe, src, n)), (kind, n)
                k += 1
        assert_no_device_errors()


def test_host_nbi_completes_at_quiet():
    from paper_2607_08006_amd import host
    t = torch()
    npes, n = 6, 5000
    with heap(npes, 2 << 20) as v:
        region = v.offset(v.malloc(1 << 20)) + (1 << 20)
        init = W.heap_fill(77, npes, region)
        upload(init)
        ref = init.copy()
        base = v.heap_base()
        srcs = [t.from_numpy(W.heap_fill(500 + i, 1, n)[0].copy()).pin_memory() for i in range(40)]
        for i, s in enumerate(srcs):
            pe, dst = i % npes, (i * 24_001) % (region - n)
            host.putmem_nbi(base + dst, s, n, pe)
            oracle.host_put(ref, pe, dst, s.numpy())
        host.quiet()
        assert np.array_equal(download(region), ref)
        outs = [t.zeros(n, dtype=t.uint8).pin_memory() for _ in range(8)]
        t.cuda.synchronize()
        for i, o in enumerate(outs):
            host.getmem_nbi(o, base + 1000 * i, n, (i + 2) % npes)
        host.fence()
        host.quiet()
        for i, o in enumerate(outs):
            assert np.array_equal(o.numpy(), oracle.host_get(ref, (i + 2) % npes, 1000 * i, n))
        assert_no_device_errors()


def test_host_atomics_follow_pe0_program():
    from paper_2607_08006_amd import host
    npes = 4
    with heap(npes, 2 << 20) as v:
        words = v.calloc(64, 8)
        wo = v.offset(words)
        region = wo + 64 * 8
        init = W.heap_fill(5, npes, region)
        upload(init)
        ref = init.copy()
        rs = W.splitmix64(0xA70, 0, 400)
        ops = []
        got = []
        descs = []
        for i in range(100):
            kind = int(rs[4 * i] % 10)
            pe = int(rs[4 * i + 1] % npes)
            w = int(rs[4 * i + 2] % 64)
            val = int(rs[4 * i + 3])
            sval = val - (1 << 64) if val >= 1 << 63 else val
            addr = words + 8 * w
            src = wo + 8 * w
            if kind == 0:
                got.append(host.int64_atomic_fetch_add(addr, sval, pe))
                descs.append(_desc(W.OP_AMO_FETCH_ADD, pe, src=src, value=val, ridx=len(got) - 1))
            elif kind == 1:
                got.append(host.int64_atomic_fetch_xor(addr, sval, pe))
                descs.append(_desc(W.OP_AMO_FETCH_XOR, pe, src=src, value=val, ridx=len(got) - 1))
            elif kind == 2:
                got.append(host.uint64_atomic_fetch_xor(addr, val, pe))
                descs.append(_desc(W.OP_AMO_FETCH_XOR, pe, src=src, value=val, ridx=len(got) - 1))
            elif kind == 3:
                # compare_swap that succeeds: the condition is the current value
                cur = host.int64_atomic_fetch(addr, pe)
                got.append(cur)
                descs.append(_desc(W.OP_AMO_FETCH, pe, src=src, ridx=len(got) - 1))
                got.append(host.int64_atomic_compare_swap(addr, cur, sval, pe))
                descs.append(_desc(W.OP_AMO_COMPARE_SWAP, pe, src=src, value=val, cond=cur % (1 << 64),
                                   ridx=len(got) - 1))
            elif kind == 4:
                got.append(host.int64_atomic_compare_swap(addr, 12345, sval, pe))   # almost surely fails
                descs.append(_desc(W.OP_AMO_COMPARE_SWAP, pe, src=src, value=val, cond=12345, ridx=len(got) - 1))
            elif kind == 5:
                host.int64_atomic_set(addr, sval, pe)
                descs.append(_desc(W.OP_AMO_SET, pe, src=src, value=val))
            elif kind == 6:
                got.append(host.int64_atomic_swap(addr, sval, pe))
                descs.append(_desc(W.OP_AMO_SWAP, pe, src=src, value=val, ridx=len(got) - 1))
            elif kind == 7:
                host.int64_atomic_add(addr, sval, pe)
                descs.append(_desc(W.OP_AMO_ADD, pe, src=src, value=val))
            elif kind == 8:
                host.int64_atomic_xor(addr, sval, pe)
                descs.append(_desc(W.OP_AMO_XOR, pe, src=src, value=val))
            else:
                host.uint64_atomic_xor(addr, val, pe)
                descs.append(_desc(W.OP_AMO_XOR, pe, src=src, value=val))
        res = oracle.run_program(ref, np.concatenate(descs), nresults=len(got))
        assert [g % (1 << 64) for g in got] == [int(r) for r in res]
        assert np.array_equal(download(region), ref)
        assert_no_device_errors()


def test_host_signals_waits_and_tests():
    from paper_2607_08006_amd import host
    t = torch()
    npes = 4
    with heap(npes, 2 << 20) as v:
        sig = v.calloc(4, 8)
        ivar = sig + 8
        data = v.malloc(8192)
        region = v.offset(data) + 8192
        upload(np.zeros((npes, region), dtype=np.uint8))
        ref = np.zeros((npes, region), dtype=np.uint8)
        payload = W.heap_fill(9, 1, 8192)[0]
        host.putmem_signal(data, payload, 8192, sig, 7, v.SIGNAL_SET, 0)
        oracle.host_put(ref, 0, v.offset(data), payload)
        assert host.signal_fetch(sig) == 7
        assert host.signal_wait_until(sig, v.CMP_GE, 7) == 7
        # signal-add on another PE, read back with an atomic fetch
        for k in range(5):
            host.putmem_signal_nbi(data, payload, 100 * (k + 1), sig, 3, v.SIGNAL_ADD, 2)
        host.quiet()
        oracle.host_put(ref, 2, v.offset(data), payload[:500])
        assert host.int64_atomic_fetch(sig, 2) == 15
        host.int64_atomic_set(ivar, -5, 0)
        host.int64_wait_until(ivar, v.CMP_LT, 0)
        assert host.int64_test(ivar, v.CMP_EQ, -5) and not host.int64_test(ivar, v.CMP_GT, 0)
        got = download(region)
        so = v.offset(sig)
        ref[0, so:so + 8] = np.array([7], dtype=np.uint64).view(np.uint8)
        ref[2, so:so + 8] = np.array([15], dtype=np.uint64).view(np.uint8)
        ref[0, so + 8:so + 16] = np.array([-5], dtype=np.int64).view(np.uint8)
        assert np.array_equal(got, ref)
        with pytest.raises(v.VshmemError):
            host.putmem_signal(data, payload, 8, sig + 4, 1, v.SIGNAL_SET, 0)   # misaligned signal word
        with pytest.raises(v.VshmemError):
            host.putmem(data, payload, 8, npes)                              # PE out of range
        with pytest.raises(v.VshmemError):
            host.putmem(t.zeros(8, dtype=t.uint8, device="cuda").data_ptr(), payload, 8, 0)   # not symmetric
        assert_no_device_errors()


def test_host_wait_outlasts_the_spin():
    """A blocking host wait whose signal arrives only after several
    milliseconds of device work on another stream: the host's spin on the
    completion word runs out and it falls back to the stream
    synchronisation, and it still returns the value that ended the wait and
    the data put before the signal."""
    from paper_2607_08006_amd import host
    t = torch()
    npes = 4
    with heap(npes, 2 << 20) as v:
        sig = v.calloc(1, 8)
        data = v.malloc(4096)
        region = v.offset(data) + 4096
        upload(np.zeros((npes, region), dtype=np.uint8))
        payload = t.from_numpy(W.heap_fill(31, 1, 4096)[0].copy()).pin_memory()
        other = t.cuda.Stream()
        t.cuda.synchronize()
        v.barrier(v.DEVICE_TEAM_WORLD, iters=4000, stream=other)          # milliseconds of device work
        host.putmem_signal_on_stream(data, payload, 4096, sig, 9, v.SIGNAL_SET, 0, stream=other)
        t0 = time.perf_counter()
        assert host.signal_wait_until(sig, v.CMP_EQ, 9) == 9
        waited = time.perf_counter() - t0
        other.synchronize()
        assert waited > 0.5e-3, waited        # longer than the spin
        got = download(region)
        assert np.array_equal(got[0, v.offset(data):region], payload.numpy())
        assert_no_device_errors()


def _red_rows(dt, npes, n, seed):
    gen = {oracle.DT_INT64: W.coll_i64, oracle.DT_FP32: W.coll_f32, oracle.DT_BF16: W.coll_bf16}[dt]
    return np.stack([gen(seed, p, n).view(np.uint8) for p in range(npes)])


@pytest.mark.parametrize("team_args", [None, (1, 2, 3)])
def test_host_collectives(team_args):
    from paper_2607_08006_amd import host
    npes = 7
    with heap(npes, 4 << 20) as v:
        team = v.TEAM_WORLD if team_args is None else v.team_split_strided(v.TEAM_WORLD, *team_args)
        tsize = v.team_n_pes(team)
        src = v.malloc(1 << 20)
        dst = v.malloc(2 << 20)
        so, do = v.offset(src), v.offset(dst)
        region = do + (2 << 20)
        init = W.heap_fill(31, npes, region)
        n = 40_001
        for name in ("broadcast", "fcollect", "alltoall"):
            upload(init)
            ref = init.copy()
            if name == "broadcast":
                host.broadcastmem(dst, src, n, tsize - 1, team=team)
                oracle.broadcast(ref, do, so, n, tsize - 1, team=team_args)
            elif name == "fcollect":
                host.fcollectmem(dst, src, n, team=team)
                oracle.fcollect(ref, do, so, n, team=team_args)
            else:
                host.alltoallmem(dst, src, n // tsize, team=team)
                oracle.alltoall(ref, do, so, n // tsize, team=team_args)
            assert np.array_equal(download(region), ref), name
        for dt, es in ((oracle.DT_INT64, 8), (oracle.DT_FP32, 4), (oracle.DT_BF16, 2)):
            nred = 30_011
            img = np.zeros((npes, region), dtype=np.uint8)
            img[:, so:so + nred * es] = _red_rows(dt, npes, nred, 3 + dt)
            for rop in (oracle.RO_SUM, oracle.RO_MAX):
                upload(img)
                host.reduce(dt, rop, dst, src, nred, team=team)
                ref = img.copy()
                oracle.reduce(ref, dt, rop, do, so, nred, team=team_args)
                assert np.array_equal(download(region), ref), (dt, rop)
        host.team_sync(team)
        host.barrier_all()
        host.sync_all()
        assert_no_device_errors()


def test_stream_triggered_sequence_is_ordered_in_the_stream():
    """One stream carries a put from pinned host memory, a broadcast of it, a
    sum reduction, a put-with-signal, a wait on that signal, barriers and a
    get back to pinned memory; the host only synchronises the stream at the
    end.  The oracle applies the same steps in order."""
    from paper_2607_08006_amd import host
    t = torch()
    npes, n = 8, 1 << 16
    with heap(npes, 2 << 20) as v:
        a = v.malloc(n)
        b = v.malloc(n)
        r = v.malloc(n)
        sig = v.calloc(1, 8)
        region = v.offset(sig) + 8
        init = W.heap_fill(123, npes, region)
        init[:, v.offset(sig):region] = 0
        upload(init)
        ref = init.copy()
        payload = t.from_numpy(W.heap_fill(321, 1, n)[0].copy()).pin_memory()
        out = t.zeros(n, dtype=t.uint8).pin_memory()
        team = v.team_split_strided(v.TEAM_WORLD, 0, 2, 4)
        s = t.cuda.Stream()
        t.cuda.synchronize()
        host.putmem_on_stream(a, payload, n, 3, stream=s)
        oracle.host_put(ref, 3, v.offset(a), payload.numpy())
        host.broadcastmem_on_stream(b, a, n, 3, stream=s)
        oracle.broadcast(ref, v.offset(b), v.offset(a), n, 3)
        host.reduce_on_stream(v.DT_INT64, v.RED_SUM, r, b, n // 8, stream=s)
        oracle.reduce(ref, oracle.DT_INT64, oracle.RO_SUM, v.offset(r), v.offset(b), n // 8)
        host.putmem_signal_on_stream(a, r, 4096, sig, 11, v.SIGNAL_ADD, 0, stream=s)
        oracle.run_program(ref, _desc(W.OP_PUT_SIGNAL, 0, src=v.offset(r), dst=v.offset(a), n=4096, value=11,
                                      cond=v.offset(sig), aux=1), check=False)
        host.signal_wait_until_on_stream(sig, v.CMP_EQ, 11, stream=s)
        host.barrier_all_on_stream(stream=s)
        host.team_sync_on_stream(team, stream=s)
        host.quiet_on_stream(stream=s)
        host.fcollectmem_on_stream(b, r, n // npes, stream=s)
        oracle.fcollect(ref, v.offset(b), v.offset(r), n // npes)
        host.alltoallmem_on_stream(r, a, n // npes, team=team, stream=s)
        oracle.alltoall(ref, v.offset(r), v.offset(a), n // npes, team=(0, 2, 4))
        host.getmem_on_stream(out, b, n, 5, stream=s)
        s.synchronize()
        assert np.array_equal(download(region), ref)
        assert np.array_equal(out.numpy(), oracle.host_get(ref, 5, v.offset(b), n))
        assert_no_device_errors()


def test_copy_alignment_matrix():
    """Every pair of source and destination offsets modulo 16, on lengths
    around the funnel-shift threshold and well past it, through the copy
    kernel of host-issued heap-to-heap puts; the oracle applies PE 0's
    puts in the same order."""
    from paper_2607_08006_amd import host
    npes = 3
    sizes = (200, 255, 256, 300, 4099, 70001)
    with heap(npes, 32 << 20) as v:
        a = v.malloc(1 << 20)
        span = sum(s + 32 for s in sizes) * 256
        b = v.malloc(span)
        region = v.offset(b) + span
        init = W.heap_fill(2718, npes, region)
        upload(init)
        ref = init.copy()
        descs = []
        pos = 0
        for dm in range(16):
            for sm in range(16):
                for n in sizes:
                    src = v.offset(a) + 1024 * sm + sm          # 1024 * sm keeps sources apart
                    dst = v.offset(b) + pos + dm
                    host.putmem(v.heap_base() + dst, v.heap_base() + src, n, 2)
                    descs.append(_desc(W.OP_PUT, 2, src=src, dst=dst, n=n))
                    pos += (n + 32) // 16 * 16
        oracle.run_program(ref, np.concatenate(descs), check=False)
        assert np.array_equal(download(region), ref)
        assert_no_device_errors()
