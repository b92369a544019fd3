"""GPU parity: random-access atomics (witness replay against the oracle),
put-with-signal ping-pong, and the team barrier."""
import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, device_array, download, heap, torch, upload

pytestmark = pytest.mark.gpu


def _gups_check(v, npes, log2_table, nupd, base_seed, table_off, init_table, got_table, fetched):
    idx, val, is_add = W.gups_updates(base_seed, 0, nupd, log2_table)
    kind = np.where(is_add, oracle.KIND_FETCH_ADD, oracle.KIND_FETCH_XOR).astype(np.uint8)
    assert oracle.witness_check(idx, kind, val, fetched, init_table.view(np.uint64),
                                got_table.view(np.uint64)) == 0
    # words hit by one kind only must equal the oracle's serial result
    ref = init_table.copy()
    oracle.gups(ref, idx, val, is_add)
    nadd = np.bincount(idx.astype(np.int64), weights=is_add.astype(np.float64), minlength=1 << log2_table)
    nall = np.bincount(idx.astype(np.int64), minlength=1 << log2_table)
    single = (nadd == 0) | (nadd == nall)
    assert np.array_equal(ref[single], got_table[single])


@pytest.mark.parametrize("npes,log2_table,nupd", [(4, 12, 1 << 15), (16, 14, (1 << 16) + 7), (1, 8, 5000)])
def test_gups_witness_replay(npes, log2_table, nupd):
    per_pe = 8 << (log2_table - int(np.log2(npes)))
    with heap(npes, max(per_pe, 1 << 20)) as v:
        t = torch()
        seed = W.subseed(W.SEED_GUPS, W.TAG_OPS)
        init = W.heap_fill(W.SEED_GUPS, npes, per_pe)
        upload(init)
        fetched = t.zeros(nupd, dtype=t.int64, device="cuda")
        acc = t.zeros(1, dtype=t.int64, device="cuda")
        v.gups(0, log2_table, nupd, seed, 5, fetched=fetched, acc=acc)
        got = download(per_pe)
        f = fetched.cpu().numpy().view(np.uint64)
        x = np.bitwise_xor.reduce(f) if len(f) else np.uint64(0)
        assert int(acc.cpu().numpy().view(np.uint64)[0]) == int(x)
        init_table = init.view(np.int64).reshape(-1)      # PE-major = global index order
        got_table = got.view(np.int64).reshape(-1)
        _gups_check(v, npes, log2_table, nupd, W.SEED_GUPS, 0, init_table, got_table, f)
        assert_no_device_errors()


def test_gups_without_fetch_matches_closed_forms():
    npes, log2_table, nupd = 8, 13, 1 << 14
    per_pe = 8 << (log2_table - 3)
    with heap(npes, 1 << 20) as v:
        t = torch()
        base = W.SEED_GUPS + 9
        init = np.zeros((npes, per_pe), dtype=np.uint8)
        upload(init)
        v.gups(0, log2_table, nupd, W.subseed(base, W.TAG_OPS), 1)          # add_every = 1: all fetch_add
        got = download(per_pe).view(np.int64).reshape(-1)
        idx, val, is_add = W.gups_updates(base, 0, nupd, log2_table, add_every=1)
        assert is_add.all()
        ref = np.zeros(1 << log2_table, dtype=np.int64)
        oracle.gups(ref, idx, val, is_add)
        assert np.array_equal(ref, got)


@pytest.mark.parametrize("same_xcd", [True, False])
def test_pingpong_signal_after_data(same_xcd):
    npes, npairs, rounds = 32, 16, 64
    with heap(npes, 1 << 20) as v:
        t = torch()
        init = W.heap_fill(3, npes, 4096)
        upload(init)
        pairs = np.arange(npes, dtype=np.int32)
        rtt = t.zeros(npairs * rounds, dtype=t.int64, device="cuda")
        v.pingpong(0, 2048, device_array(pairs), npairs, rounds, payload_bytes=8, same_xcd=same_xcd, rtt=rtt)
        got = download(4096)
        r = rtt.cpu().numpy()
        assert (r > 0).all()
        for k in range(npairs):
            a, b = 2 * k, 2 * k + 1
            # a's 8 bytes travelled to b and back; nothing else in the data area moved
            assert np.array_equal(got[b, :8], init[a, :8]) and np.array_equal(got[a, :8], init[a, :8])
            assert np.array_equal(got[a, 8:2048], init[a, 8:2048])
            sa = int(got[a, 2048:2056].view(np.uint64)[0])
            sb = int(got[b, 2048:2056].view(np.uint64)[0])
            assert sa & 0xFFFFFFFF == rounds and sb & 0xFFFFFFFF == rounds and sa == sb
        # the oracle's program of the same exchange ends in the same state
        ref = init.copy()
        recs = []
        for rr in range(1, rounds + 1):
            for k in range(npairs):
                a, b = 2 * k, 2 * k + 1
                recs += [(W.OP_PUT_SIGNAL, 0, W.SIGNAL_SET, a, b, W.NO_RESULT, 0, 0, 8, rr, 2048),
                         (W.OP_WAIT_UNTIL, 0, W.CMP_EQ, b, b, W.NO_RESULT, 2048, 0, 0, rr, 0),
                         (W.OP_PUT_SIGNAL, 0, W.SIGNAL_SET, b, a, W.NO_RESULT, 0, 0, 8, rr, 2048),
                         (W.OP_WAIT_UNTIL, 0, W.CMP_EQ, a, a, W.NO_RESULT, 2048, 0, 0, rr, 0)]
        oracle.run_program(ref, W.descs(recs))
        assert np.array_equal(got[:, :2048], ref[:, :2048])
        assert_no_device_errors()


def test_barrier_tokens_world_and_strided_team():
    npes = 24
    with heap(npes, 1 << 20) as v:
        t = torch()
        upload(np.zeros((npes, 8192), dtype=np.uint8))
        bad = t.zeros(1, dtype=t.int64, device="cuda")
        cyc = t.zeros(1, dtype=t.int64, device="cuda")
        v.barrier(v.DEVICE_TEAM_WORLD, iters=200, tokens_off=0, bad=bad, cycles=cyc)
        t.cuda.synchronize()
        assert int(bad.item()) == 0 and int(cyc.item()) > 0
        team = v.team_split_strided(v.DEVICE_TEAM_WORLD, 1, 3, 7)
        v.barrier(team, iters=100, tokens_off=4096, bad=bad)
        t.cuda.synchronize()
        assert int(bad.item()) == 0
        got = download(8192)
        for p in range(npes):
            member = (p - 1) % 3 == 0 and (p - 1) // 3 < 7 and p >= 1
            assert got[p, 4096:4096 + 16 * 7].any() == member
        assert_no_device_errors()


def test_wait_until_satisfied_and_bounded_timeout():
    """The timeout is forced from the host with a 2 ms spin limit on a wait
    whose value is never written: the kernel gives up, latches the error
    bit and ends normally."""
    npes = 3
    with heap(npes, 1 << 20) as v:
        t = torch()
        init = np.zeros((npes, 64), dtype=np.uint8)
        init[2, 8:16] = np.array([5], dtype=np.int64).view(np.uint8)
        upload(init)
        out = t.zeros(1, dtype=t.int64, device="cuda")
        v.wait_until(2, 8, W.CMP_GE, 5, out=out)
        t.cuda.synchronize()
        assert int(out.item()) == 5 and v.device_errors() == 0
        v.set_wait_timeout_ns(2_000_000)
        v.wait_until(1, 8, W.CMP_EQ, 12345, out=out)
        t.cuda.synchronize()
        assert v.device_errors() == v.DEVERR_WAIT_TIMEOUT
        assert v.device_errors() == 0                      # reading clears the word
        v.set_wait_timeout_ns(10_000_000_000)
