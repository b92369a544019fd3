"""Pins of the CPU oracle against facts fixed outside the oracle itself:
published generator outputs, hand-computed worked examples of the reduction
order, closed forms, invariants of the OpenSHMEM operations, exact integer
arithmetic in Python, and library routines for special cases."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                yield ln.split()


# ------------------------------------------------------------- generators
def test_splitmix64_published_vectors():
    for seed, idx, val in _lines("splitmix64_vectors.txt"):
        seed, idx, val = int(seed, 0), int(idx), int(val, 0)
        assert int(W.splitmix64(seed, idx, 1)[0]) == val
        assert W.splitmix64_scalar(seed, idx) == val


def test_splitmix64_window_is_counter_based():
    full = W.splitmix64(99, 0, 1000)
    assert np.array_equal(full[123:456], W.splitmix64(99, 123, 333))
    b = W.payload(7, 0, 4096)
    assert np.array_equal(b[13:13 + 500], W.payload(7, 13, 500))


def test_bounded_range_and_uniformity():
    x = W.splitmix64(5, 0, 200000)
    v = W.bounded(x, 8, 4096)
    assert v.min() >= 8 and v.max() <= 4096
    # Lemire map equals the exact 128-bit product computed with Python ints.
    for xi in x[:200]:
        assert int(W.bounded(np.array([xi]), 3, 17)[0]) == 3 + ((int(xi) * 15) >> 64)
    counts = np.bincount(W.bounded(x, 0, 9), minlength=10)
    assert counts.min() > 19000 and counts.max() < 21000


def test_uniform_f32_exact_and_bf16_rne_matches_torch():
    torch = pytest.importorskip("torch")
    x = W.splitmix64(11, 0, 4096)
    f = W.uniform_f32(x)
    assert f.min() >= -1.0 and f.max() < 1.0
    exact = (x >> np.uint64(40)).astype(np.float64) * 2.0 ** -23 - 1.0
    assert np.array_equal(f.astype(np.float64), exact)
    ours = W.f32_to_bf16_bits(f)
    ref = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_derangement_has_no_fixed_point():
    for n in (2, 3, 64, 256):
        p = W.derangement(W.subseed(W.SEED_SWEEP, 3), n)
        assert sorted(p.tolist()) == list(range(n))
        assert not np.any(p == np.arange(n))


def test_small_workload_deterministic_and_accepted_by_checker():
    a = W.small_workload(n_rma=200, epoch_ops=50, n_amo=500)
    b = W.small_workload(n_rma=200, epoch_ops=50, n_amo=500)
    assert np.array_equal(a.descs, b.descs) and np.array_equal(a.init, b.init)
    heap = a.init.copy()
    oracle.run_program(heap, a.descs, nresults=a.n_amo, check=True)


# --------------------------------------------------------- put / get pins
def _tagged_heap(npes, stride):
    """Each 8-byte word carries its own (pe, word) tag."""
    words = np.zeros((npes, stride // 8), dtype=np.uint64)
    for p in range(npes):
        words[p] = (np.uint64(p + 1) << np.uint64(32)) + np.arange(stride // 8, dtype=np.uint64)
    return words.view(np.uint8).copy()


def _desc(op, issuer, target, src=0, dst=0, n=0, value=0, cond=0, aux=0, ridx=W.NO_RESULT, flags=0):
    d = W.descs([(op, W.SCOPE_THREAD, aux, issuer, target, ridx, src, dst, n, value, cond)])
    d["flags"] = flags
    return d


def test_put_moves_tagged_words_to_target():
    heap = _tagged_heap(3, 256)
    d = _desc(W.OP_PUT, issuer=2, target=0, src=16, dst=200, n=48)
    oracle.run_program(heap, d)
    w = heap.view(np.uint64).reshape(3, 32)
    # destination words now carry the issuer's source tags
    assert [int(v) for v in w[0, 25:31]] == [(3 << 32) + 2 + k for k in range(6)]
    # nothing else changed
    ref = _tagged_heap(3, 256).view(np.uint64).reshape(3, 32)
    mask = np.ones_like(ref, dtype=bool)
    mask[0, 25:31] = False
    assert np.array_equal(w[mask], ref[mask])


def test_get_is_the_mirror_of_put():
    rng_heap = W.heap_fill(17, 4, 512)
    for (i, p, s, d, n) in [(0, 3, 8, 128, 40), (2, 1, 0, 64, 1), (3, 3, 0, 256, 100), (1, 0, 200, 8, 64)]:
        h1 = rng_heap.copy()
        h2 = rng_heap.copy()
        oracle.run_program(h1, _desc(W.OP_GET, issuer=i, target=p, src=s, dst=d, n=n))
        oracle.run_program(h2, _desc(W.OP_PUT, issuer=p, target=i, src=s, dst=d, n=n))
        assert np.array_equal(h1, h2)


def test_put_then_get_round_trip_and_byte_granularity():
    heap = W.heap_fill(3, 2, 256)
    orig = heap.copy()
    prog = np.concatenate([
        _desc(W.OP_PUT, 0, 1, src=8, dst=100, n=13),       # odd length, unaligned dst
        _desc(W.OP_QUIET, 0, 0),
        _desc(W.OP_GET, 0, 1, src=100, dst=160, n=13),
    ])
    oracle.run_program(heap, prog)
    assert np.array_equal(heap[0, 160:173], orig[0, 8:21])
    assert np.array_equal(heap[1, 100:113], orig[0, 8:21])
    assert np.array_equal(heap[1, 113:], orig[1, 113:]) and np.array_equal(heap[1, :100], orig[1, :100])


def test_host_put_get_agree_with_pe0_programs_and_touch_only_their_range():
    """A host put from a private buffer equals PE 0's put from a heap region
    holding the same bytes; a host get returns what PE 0's get would copy
    into its own heap.  Only the named byte range changes."""
    heap = W.heap_fill(41, 3, 512)
    for pe, dst, n, src0 in [(2, 100, 37, 300), (0, 0, 1, 256), (1, 448, 64, 0)]:
        buf = heap[0, src0:src0 + n].copy()
        h1, h2 = heap.copy(), heap.copy()
        oracle.host_put(h1, pe, dst, buf)
        oracle.run_program(h2, _desc(W.OP_PUT, issuer=0, target=pe, src=src0, dst=dst, n=n))
        assert np.array_equal(h1, h2), (pe, dst, n)
        changed = np.argwhere(h1 != heap)
        assert all(r == pe and dst <= c < dst + n for r, c in changed)
        got = oracle.host_get(heap, pe, dst, n)
        h3 = heap.copy()
        oracle.run_program(h3, _desc(W.OP_GET, issuer=0, target=pe, src=dst, dst=src0, n=n))
        assert np.array_equal(got, h3[0, src0:src0 + n])
    # round trip, and arguments outside the heap are refused
    h = heap.copy()
    data = np.arange(200, dtype=np.uint8)
    oracle.host_put(h, 1, 5, data)
    assert np.array_equal(oracle.host_get(h, 1, 5, 200), data)
    for bad in (lambda: oracle.host_put(h, 3, 0, data), lambda: oracle.host_put(h, 0, 400, data),
                lambda: oracle.host_get(h, -1, 0, 8), lambda: oracle.host_get(h, 0, 500, 13)):
        with pytest.raises(oracle.OracleError):
            bad()


def test_random_tiny_programs_match_exhaustive_byte_tracking():
    """Brute force on tiny heaps: track every byte's provenance (pe, offset)
    through a random conflict-free epoch and compare with the oracle."""
    rs = W.splitmix64(0xABC, 0, 60000)
    c = 0
    for npes in range(1, 6):
        for trial in range(20):
            stride = 256
            heap = _tagged_heap(npes, stride)
            prov = np.empty((npes, stride), dtype=object)
            for p in range(npes):
                for o in range(stride):
                    prov[p, o] = (p, o)
            writes = [set() for _ in range(npes)]
            reads = [set() for _ in range(npes)]
            recs = []
            for _ in range(6):
                kind = W.OP_PUT if int(rs[c]) & 1 else W.OP_GET
                i = int(rs[c + 1] % np.uint64(npes)); t = int(rs[c + 2] % np.uint64(npes))
                n = 1 + int(rs[c + 3] % np.uint64(64))
                s = 8 * int(rs[c + 4] % np.uint64(9)); dd = 8 * int(rs[c + 5] % np.uint64(9)) + 64
                c += 6
                wpe, rpe = (t, i) if kind == W.OP_PUT else (i, t)
                wset = set(range(dd, dd + n)); rset = set(range(s, s + n))
                if wset & writes[wpe] or wset & reads[wpe] or rset & writes[rpe]:
                    continue
                if wpe == rpe and wset & rset:
                    continue
                writes[wpe] |= wset; reads[rpe] |= rset
                recs.append((kind, W.SCOPE_THREAD, 0, i, t, W.NO_RESULT, s, dd, n, 0, 0))
                src_prov = [prov[rpe, s + k] for k in range(n)]
                for k in range(n):
                    prov[wpe, dd + k] = src_prov[k]
            if not recs:
                continue
            oracle.run_program(heap, W.descs(recs))
            init = _tagged_heap(npes, stride)
            for p in range(npes):
                for o in range(stride):
                    sp, so = prov[p, o]
                    assert heap[p, o] == init[sp, so]


# ------------------------------------------------------ checker / scheduler
def test_conflict_checker_flags_write_write_and_read_write():
    heap = W.heap_fill(1, 2, 256)
    ww = np.concatenate([_desc(W.OP_PUT, 0, 1, src=0, dst=64, n=16),
                         _desc(W.OP_PUT, 1, 1, src=128, dst=72, n=16)])
    with pytest.raises(oracle.OracleError) as e:
        oracle.run_program(heap.copy(), ww)
    assert e.value.code == -3
    rw = np.concatenate([_desc(W.OP_PUT, 0, 1, src=0, dst=64, n=16),
                         _desc(W.OP_GET, 0, 1, src=70, dst=128, n=8)])
    with pytest.raises(oracle.OracleError):
        oracle.run_program(heap.copy(), rw)
    # the same pair separated by a fence of the same PE is ordered
    ok = np.concatenate([rw[:1], _desc(W.OP_FENCE, 0, 0), rw[1:]])
    oracle.run_program(heap.copy(), ok)
    # ... and a fence of another PE does not order PE 0 with PE 1
    bad = np.concatenate([ww[:1], _desc(W.OP_FENCE, 1, 1), ww[1:]])
    with pytest.raises(oracle.OracleError):
        oracle.run_program(heap.copy(), bad)
    # a barrier orders everything
    bar = np.concatenate([ww[:1], _desc(W.OP_BARRIER_ALL, 0, 0), _desc(W.OP_BARRIER_ALL, 1, 1), ww[1:]])
    oracle.run_program(heap.copy(), bar)


def test_atomics_do_not_conflict_with_each_other_but_do_with_plain_writes():
    heap = np.zeros((2, 64), dtype=np.uint8)
    amo = np.concatenate([_desc(W.OP_AMO_FETCH_ADD, 0, 1, src=8, value=1, ridx=0),
                          _desc(W.OP_AMO_FETCH_XOR, 1, 1, src=8, value=6, ridx=1)])
    oracle.run_program(heap.copy(), amo, nresults=2)
    mixed = np.concatenate([amo[:1], _desc(W.OP_PUT, 1, 1, src=32, dst=8, n=8)])
    with pytest.raises(oracle.OracleError):
        oracle.run_program(heap.copy(), mixed, nresults=2)


def test_deadlock_reported_for_unsatisfiable_wait():
    heap = np.zeros((2, 64), dtype=np.uint8)
    prog = _desc(W.OP_WAIT_UNTIL, 0, 0, src=0, value=1, aux=W.CMP_EQ)
    with pytest.raises(oracle.OracleError) as e:
        oracle.run_program(heap, prog)
    assert e.value.code == -4
    # a PE that finishes while another waits at a barrier never arrives
    prog = np.concatenate([_desc(W.OP_BARRIER_ALL, 0, 0)])
    with pytest.raises(oracle.OracleError):
        oracle.run_program(np.zeros((2, 64), dtype=np.uint8), prog)


def _pingpong_program(npairs, rounds, data_off=0, sig_off=64, tag_off=128):
    """PE 2k sends round r's tag to 2k+1 with put-with-signal (SET r), then
    waits for the echo; PE 2k+1 waits for r, echoes the data back."""
    recs = []
    for r in range(1, rounds + 1):
        for k in range(npairs):
            a, b = 2 * k, 2 * k + 1
            recs.append((W.OP_PUT_SIGNAL, 0, W.SIGNAL_SET, a, b, W.NO_RESULT, tag_off + 8 * r, data_off, 8, r, sig_off))
            recs.append((W.OP_WAIT_UNTIL, 0, W.CMP_EQ, b, b, W.NO_RESULT, sig_off, 0, 0, r, 0))
            recs.append((W.OP_PUT_SIGNAL, 0, W.SIGNAL_SET, b, a, W.NO_RESULT, data_off, data_off, 8, r, sig_off))
            recs.append((W.OP_WAIT_UNTIL, 0, W.CMP_EQ, a, a, W.NO_RESULT, sig_off, 0, 0, r, 0))
    return W.descs(recs)


def test_pingpong_signal_after_data():
    npairs, rounds = 3, 7
    stride = 256
    heap = np.zeros((2 * npairs, stride), dtype=np.uint8)
    tags = heap.view(np.uint64).reshape(2 * npairs, stride // 8)
    for p in range(2 * npairs):
        for r in range(1, rounds + 1):
            tags[p, 16 + r] = 1000 * p + r
    prog = _pingpong_program(npairs, rounds)
    oracle.run_program(heap, prog, check=True)
    w = heap.view(np.uint64).reshape(2 * npairs, stride // 8)
    for k in range(npairs):
        a, b = 2 * k, 2 * k + 1
        assert w[a, 8] == rounds and w[b, 8] == rounds           # signal == R after R round trips
        assert w[b, 0] == 1000 * a + rounds and w[a, 0] == 1000 * a + rounds   # last tag echoed


def test_signal_add_and_unsigned_wait():
    heap = np.zeros((3, 64), dtype=np.uint8)
    recs = [
        (W.OP_PUT_SIGNAL, 0, W.SIGNAL_ADD, 1, 0, W.NO_RESULT, 0, 16, 8, 5, 8),
        (W.OP_PUT_SIGNAL, 0, W.SIGNAL_ADD, 2, 0, W.NO_RESULT, 0, 24, 8, (1 << 64) - 1, 8),
        (W.OP_WAIT_UNTIL, 0, W.CMP_GE, 0, 0, W.NO_RESULT, 8, 0, 0, 4, 0),
    ]
    d = W.descs(recs)
    d["flags"][2] = 1
    oracle.run_program(heap, d)
    assert int(heap.view(np.uint64).reshape(3, 8)[0, 1]) == 4      # 5 + (2^64-1) wraps to 4


# ------------------------------------------------------------ atomics pins
def test_fetch_add_plus_one_sums_and_permutes():
    n, npes = 777, 3
    recs = [(W.OP_AMO_FETCH_ADD, 0, 0, i % npes, 2, i, 16, 0, 8, 1, 0) for i in range(n)]
    heap = np.zeros((npes, 64), dtype=np.uint8)
    res = oracle.run_program(heap, W.descs(recs), nresults=n)
    assert int(heap.view(np.uint64).reshape(npes, 8)[2, 2]) == n
    assert sorted(res.tolist()) == list(range(n))


def test_compare_swap_single_winner():
    T = 50
    recs = [(W.OP_AMO_COMPARE_SWAP, 0, 0, t % 4, 1, t, 8, 0, 8, t + 1, 0) for t in range(T)]
    heap = np.zeros((4, 32), dtype=np.uint8)
    res = oracle.run_program(heap, W.descs(recs), nresults=T)
    word = int(heap.view(np.uint64).reshape(4, 4)[1, 1])
    winners = [t for t in range(T) if res[t] == 0]
    assert len(winners) == 1 and word == winners[0] + 1
    assert all(int(res[t]) == word for t in range(T) if t not in winners)


def test_xor_and_add_closed_forms_with_wraparound():
    vals = [int(v) for v in W.splitmix64(77, 0, 300)]
    init = 0x7FFF_FFFF_FFFF_FFF0
    heap = np.zeros((2, 32), dtype=np.uint8)
    heap.view(np.uint64).reshape(2, 4)[1, 0] = init
    heap.view(np.uint64).reshape(2, 4)[1, 1] = init
    recs = [(W.OP_AMO_ADD, 0, 0, 0, 1, W.NO_RESULT, 0, 0, 8, v, 0) for v in vals]
    recs += [(W.OP_AMO_XOR, 0, 0, 1, 1, W.NO_RESULT, 8, 0, 8, v, 0) for v in vals]
    oracle.run_program(heap, W.descs(recs))
    w = heap.view(np.uint64).reshape(2, 4)
    x = init
    for v in vals:
        x ^= v
    assert int(w[1, 0]) == (init + sum(vals)) % (1 << 64)
    assert int(w[1, 1]) == x


def test_set_fetch_swap():
    heap = np.zeros((1, 16), dtype=np.uint8)
    recs = [(W.OP_AMO_SET, 0, 0, 0, 0, W.NO_RESULT, 0, 0, 8, 42, 0),
            (W.OP_AMO_SWAP, 0, 0, 0, 0, 0, 0, 0, 8, 7, 0),
            (W.OP_AMO_FETCH, 0, 0, 0, 0, 1, 0, 0, 8, 0, 0)]
    res = oracle.run_program(heap, W.descs(recs), nresults=2)
    assert res.tolist() == [42, 7]


# ------------------------------------------------------------- collectives
def test_alltoall_is_block_transpose_and_involution():
    P, n = 5, 24
    stride = 2 * P * n + 64
    heap = np.zeros((P, stride), dtype=np.uint8)
    for q in range(P):
        for p in range(P):
            heap[q, p * n:(p + 1) * n] = 16 * q + p         # block (src q, for dst p)
    oracle.alltoall(heap, P * n, 0, n)
    for p in range(P):
        for q in range(P):
            assert np.all(heap[p, P * n + q * n:P * n + (q + 1) * n] == 16 * q + p)
    before = heap[:, :P * n].copy()
    oracle.alltoall(heap, 0, P * n, n)          # transpose back
    assert np.array_equal(heap[:, :P * n], before)


def test_fcollect_concatenates_and_broadcast_copies_root():
    P, n = 4, 40
    heap = W.heap_fill(9, P, 512)
    orig = heap.copy()
    oracle.fcollect(heap, 256, 0, n)
    cat = np.concatenate([orig[q, :n] for q in range(P)])
    for p in range(P):
        assert np.array_equal(heap[p, 256:256 + P * n], cat)
    heap = orig.copy()
    oracle.broadcast(heap, 300, 8, 100, root=2)
    for p in range(P):
        assert np.array_equal(heap[p, 300:400], orig[2, 8:108])     # root's dest written too
        assert np.array_equal(heap[p, :300], orig[p, :300])


def test_one_pe_collectives_are_local_copies():
    heap = W.heap_fill(2, 1, 256)
    orig = heap.copy()
    oracle.alltoall(heap, 128, 0, 64)
    assert np.array_equal(heap[0, 128:192], orig[0, 0:64])
    heap = orig.copy()
    oracle.reduce(heap, oracle.DT_INT64, oracle.RO_SUM, 128, 0, 8)
    assert np.array_equal(heap[0, 128:192], orig[0, 0:64])


def test_strided_team_only_touches_members():
    P = 6
    heap = W.heap_fill(4, P, 256)
    orig = heap.copy()
    oracle.broadcast(heap, 128, 0, 32, root=1, team=(1, 2, 3))     # PEs 1, 3, 5; root is PE 3
    for p in (1, 3, 5):
        assert np.array_equal(heap[p, 128:160], orig[3, 0:32])
    for p in (0, 2, 4):
        assert np.array_equal(heap[p], orig[p])


# -------------------------------------------------------------- reductions
def _reduce_cols(cols, dt, rop):
    return oracle.reduce_columns(np.ascontiguousarray(cols), dt, rop)


def test_int64_sum_closed_form():
    for P in (1, 2, 3, 7, 64):
        K = 33
        cols = np.array([[p * (1 << 32) + k for k in range(K)] for p in range(P)], dtype=np.int64)
        got = _reduce_cols(cols, oracle.DT_INT64, oracle.RO_SUM)
        for k in range(K):
            assert int(got[k]) == (1 << 32) * P * (P - 1) // 2 + P * k


def test_int64_sum_full_range_wraps_like_exact_integers():
    P, K = 13, 64
    cols = np.stack([W.coll_i64(1, p, K) for p in range(P)])
    got = _reduce_cols(cols, oracle.DT_INT64, oracle.RO_SUM)
    for k in range(K):
        exact = sum(int(cols[p, k]) for p in range(P)) % (1 << 64)
        if exact >= 1 << 63:
            exact -= 1 << 64
        assert int(got[k]) == exact


def test_fp32_tree_worked_examples():
    for fields in _lines("tree_worked_examples.txt"):
        P = int(fields[0])
        xs = np.array([int(h, 16) for h in fields[1:1 + P]], dtype=np.uint32).view(np.float32)
        want = int(fields[1 + P], 16)
        got = _reduce_cols(xs.reshape(P, 1), oracle.DT_FP32, oracle.RO_SUM)
        assert int(got.view(np.uint32)[0]) == want, (P, hex(int(got.view(np.uint32)[0])))


def test_fp32_two_pe_sum_is_one_rne_add_and_error_bound():
    a = W.coll_f32(1, 0, 1000)
    b = W.coll_f32(1, 1, 1000)
    got = _reduce_cols(np.stack([a, b]), oracle.DT_FP32, oracle.RO_SUM)
    assert np.array_equal(got, (a + b).astype(np.float32))
    for P in (3, 8, 64):
        K = 200
        cols = np.stack([W.coll_f32(2, p, K) for p in range(P)])
        got = _reduce_cols(cols, oracle.DT_FP32, oracle.RO_SUM)
        depth = int(np.ceil(np.log2(P)))
        u = 2.0 ** -24
        for k in range(K):
            exact = sum(Fraction(float(v)) for v in cols[:, k])
            bound = depth * u * sum(abs(Fraction(float(v))) for v in cols[:, k]) * Fraction(1 + 1e-6)
            assert abs(Fraction(float(got[k])) - exact) <= bound


def test_fp32_powers_of_two_are_exact():
    P, K = 16, 50
    e = W.bounded(W.splitmix64(3, 0, P * K), -10, 10).reshape(P, K)
    cols = np.ldexp(np.ones((P, K)), e).astype(np.float32)
    got = _reduce_cols(cols, oracle.DT_FP32, oracle.RO_SUM)
    assert np.array_equal(got.astype(np.float64), cols.astype(np.float64).sum(axis=0))


def test_bf16_rounding_matches_torch_and_reduce_rounds_once():
    torch = pytest.importorskip("torch")
    xs = np.concatenate([W.coll_f32(5, 0, 3000) * 100, np.array([0.0, -0.0, 1.0, 3.0e38, 1e-40], dtype=np.float32)])
    xs = xs.astype(np.float32)
    ref = torch.from_numpy(xs).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    ours = np.array([oracle.bf16_round(float(v)) for v in xs], dtype=np.uint16)
    assert np.array_equal(ours, ref)
    P, K = 8, 300
    cols = np.stack([W.coll_bf16(6, p, K) for p in range(P)])
    got = _reduce_cols(cols, oracle.DT_BF16, oracle.RO_SUM)
    widened = (cols.astype(np.uint32) << 16).view(np.float32)
    f32 = _reduce_cols(widened, oracle.DT_FP32, oracle.RO_SUM)
    want = torch.from_numpy(f32).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, want)


def test_max_matches_numpy_and_tie_keeps_left_operand():
    P, K = 9, 500
    cols = np.stack([W.coll_f32(8, p, K) for p in range(P)])
    got = _reduce_cols(cols, oracle.DT_FP32, oracle.RO_MAX)
    assert np.array_equal(got, cols.max(axis=0))
    ci = np.stack([W.coll_i64(8, p, K) for p in range(P)])
    assert np.array_equal(_reduce_cols(ci, oracle.DT_INT64, oracle.RO_MAX), ci.max(axis=0))
    # +0 and -0 compare equal: the left (lower-PE) operand is kept.
    z = np.array([[0.0], [-0.0]], dtype=np.float32)
    assert np.signbit(_reduce_cols(z, oracle.DT_FP32, oracle.RO_MAX)[0]) == False
    z = np.array([[-0.0], [0.0]], dtype=np.float32)
    assert np.signbit(_reduce_cols(z, oracle.DT_FP32, oracle.RO_MAX)[0]) == True


def _f32(bits):
    return np.asarray(bits, dtype=np.uint32).view(np.float32)


def test_signed_zero_sums_and_max_closed_forms():
    """Sums of signed zeros: RNE gives -0 only for (-0) + (-0), so any order
    yields -0 iff every input is -0.  max of equal values keeps the left
    operand at every pairing, so TREE returns PE 0's element."""
    for P in (2, 3, 13, 64, 130):
        K = 300
        signs = (W.splitmix64(900 + P, 0, P * K) >> np.uint64(63)).reshape(P, K)
        signs[:, 0] = 1                                   # a column of -0 only
        signs[:, 1] = 0                                   # and one of +0 only
        cols = _f32((signs.astype(np.uint32) << 31))
        s = _reduce_cols(cols, oracle.DT_FP32, oracle.RO_SUM)
        assert np.array_equal(np.signbit(s), signs.all(axis=0)), P
        assert np.all(s == 0)
        m = _reduce_cols(cols, oracle.DT_FP32, oracle.RO_MAX)
        assert np.array_equal(np.signbit(m), signs[0].astype(bool)), P
        b = (signs.astype(np.uint16) << 15)
        sb = _reduce_cols(b, oracle.DT_BF16, oracle.RO_SUM)
        assert np.array_equal(sb, np.where(signs.all(axis=0), 0x8000, 0).astype(np.uint16))
        mb = _reduce_cols(b, oracle.DT_BF16, oracle.RO_MAX)
        assert np.array_equal(mb, b[0])


def test_subnormal_sums_are_exact():
    """Inputs that are integer multiples of 2^-149 (fp32 subnormals) or of
    2^-133 (bf16 subnormals): every partial sum is an integer multiple of the
    same unit below 2^24 units, so each fp32 add is exact and TREE equals the
    exact sum, which Python integers give."""
    for P in (2, 13, 64, 130):
        K = 200
        x = W.splitmix64(700 + P, 0, P * K).reshape(P, K)
        m = (x & np.uint64(0xFFFF)).astype(np.int64)           # |m| < 2^16: P * 2^16 < 2^24
        neg = (x >> np.uint64(63)).astype(bool)
        bits = (m.astype(np.uint32) | (neg.astype(np.uint32) << 31))
        got = _reduce_cols(_f32(bits), oracle.DT_FP32, oracle.RO_SUM)
        for k in range(K):
            exact = sum((-int(m[p, k]) if neg[p, k] else int(m[p, k])) for p in range(P))
            assert Fraction(float(got[k])) == Fraction(exact, 1 << 149), (P, k)
        # bf16 subnormals: mantissa m < 128, value m * 2^-133; the fp32 sum is
        # exact, and the result is that sum rounded once (torch's RNE).
        torch = pytest.importorskip("torch")
        mb = (x & np.uint64(0x7F)).astype(np.int64)
        bb = (mb.astype(np.uint16) | (neg.astype(np.uint16) << 15))
        gotb = _reduce_cols(bb, oracle.DT_BF16, oracle.RO_SUM)
        exact = np.array([sum((-int(mb[p, k]) if neg[p, k] else int(mb[p, k])) for p in range(P)) for k in range(K)])
        f = np.ldexp(exact.astype(np.float64), -133).astype(np.float32)
        assert np.array_equal(f.astype(np.float64), np.ldexp(exact.astype(np.float64), -133))  # exact in fp32
        want = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
        assert np.array_equal(gotb, want), P


def test_infinities_and_overflow_closed_forms():
    """IEEE-754 facts: x + inf = inf for finite x; inf + (-inf) is NaN (and
    NaN + x stays NaN); FLT_MAX + FLT_MAX overflows to inf under RNE, while
    FLT_MAX + (-FLT_MAX) = +0; max with an infinity is +inf (or the largest
    finite value when only -inf is present)."""
    inf, ninf, fmax = 0x7F800000, 0xFF800000, 0x7F7FFFFF
    u = W.uniform_f32(W.splitmix64(31, 0, 64)).view(np.uint32)
    for P in (2, 5, 13, 64):
        base = np.resize(u, P).astype(np.uint32)
        col = base.copy(); col[P // 2] = inf
        assert _reduce_cols(_f32(col)[:, None], oracle.DT_FP32, oracle.RO_SUM)[0] == np.inf
        assert _reduce_cols(_f32(col)[:, None], oracle.DT_FP32, oracle.RO_MAX)[0] == np.inf
        col = base.copy(); col[0] = ninf
        assert _reduce_cols(_f32(col)[:, None], oracle.DT_FP32, oracle.RO_SUM)[0] == -np.inf
        assert _reduce_cols(_f32(col)[:, None], oracle.DT_FP32, oracle.RO_MAX)[0] == _f32(base[1:]).max()
        col = base.copy(); col[0] = inf; col[P - 1] = ninf
        assert np.isnan(_reduce_cols(_f32(col)[:, None], oracle.DT_FP32, oracle.RO_SUM)[0])
        col = np.full(P, fmax, dtype=np.uint32)
        assert _reduce_cols(_f32(col)[:, None], oracle.DT_FP32, oracle.RO_SUM)[0] == np.inf
        colb = np.full(P, 0x7F7F, dtype=np.uint16)                 # bf16 max finite: overflows in fp32
        assert _reduce_cols(colb[:, None], oracle.DT_BF16, oracle.RO_SUM)[0] == 0x7F80
    pair = np.array([fmax, fmax | 0x80000000], dtype=np.uint32)
    r = _reduce_cols(_f32(pair)[:, None], oracle.DT_FP32, oracle.RO_SUM)[0]
    assert r == 0 and not np.signbit(r)
    # bf16 max finite plus a value that moves the fp32 sum past the midpoint
    # to the next (infinite) bf16 value rounds to inf once at the end.
    half_ulp = np.float32(2.0 ** (127 - 8))
    top = np.uint32(0x7F7F) << 16
    s = np.float32(_f32(top)) + half_ulp
    assert W.f32_to_bf16_bits(np.array([s]))[0] == 0x7F80


def test_int64_extremes_max_and_wrapping_sum():
    ext = np.array([-(1 << 63), (1 << 63) - 1, -1, 0, 1], dtype=np.int64)
    for P in (2, 13, 64, 130):
        K = 100
        cols = ext[W.bounded(W.splitmix64(50 + P, 0, P * K), 0, 4)].reshape(P, K)
        assert np.array_equal(_reduce_cols(cols, oracle.DT_INT64, oracle.RO_MAX), cols.max(axis=0))
        got = _reduce_cols(cols, oracle.DT_INT64, oracle.RO_SUM)
        for k in range(K):
            exact = sum(int(v) for v in cols[:, k]) % (1 << 64)
            assert int(got[k]) % (1 << 64) == exact


# -------------------------------------------------------- GUPS and witness
def test_gups_closed_forms_for_single_kind_words():
    log2 = 10
    idx, val, is_add = W.gups_updates(123, 0, 4096, log2)
    table = W.splitmix64(9, 0, 1 << log2).view(np.int64).copy()
    init = table.copy()
    oracle.gups(table, idx, val, is_add)
    for g in range(1 << log2):
        sel = idx == np.uint64(g)
        kinds = set(is_add[sel].tolist())
        if kinds == {True}:
            assert (int(init[g]) + sum(int(v) for v in val[sel])) % (1 << 64) == int(table[g]) % (1 << 64)
        elif kinds == {False}:
            x = int(init[g]) % (1 << 64)
            for v in val[sel]:
                x ^= int(v)
            assert x == int(table[g]) % (1 << 64)
        elif not kinds:
            assert table[g] == init[g]


def test_witness_replay_accepts_serial_orders_and_rejects_forgeries():
    log2 = 6
    idx, val, is_add = W.gups_updates(321, 0, 2000, log2)
    table = np.zeros(1 << log2, dtype=np.int64)
    fetched = oracle.gups(table, idx, val, is_add, want_fetched=True)
    kind = np.where(is_add, oracle.KIND_FETCH_ADD, oracle.KIND_FETCH_XOR)
    init = np.zeros(1 << log2, dtype=np.uint64)
    final = table.view(np.uint64)
    # any permutation of the update list is the same history
    perm = np.argsort(W.splitmix64(4, 0, 2000))
    assert oracle.witness_check(idx[perm], kind[perm], val[perm], fetched[perm], init, final) == 0
    bad = fetched.copy()
    bad[17] ^= np.uint64(1)
    assert oracle.witness_check(idx, kind, val, bad, init, final) >= 1
    badf = final.copy()
    badf[int(idx[5])] ^= np.uint64(4)
    assert oracle.witness_check(idx, kind, val, fetched, init, badf) >= 1
