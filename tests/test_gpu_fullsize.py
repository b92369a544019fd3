"""GPU parity at the workloads' full sizes, in the launch shapes bench.py
times, checked on sampled outputs that the oracle (or the counter-based
input generator, for pure movement) computes one by one."""
import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, heap, out_hash, torch

pytestmark = pytest.mark.gpu

MiB = 1 << 20


def _seed_a(p):
    return W.subseed(W.SEED_SWEEP, W.TAG_HEAP + p)


def _windows(rng_seed, count, span, width):
    x = W.splitmix64(rng_seed, 0, count)
    return (W.bounded(x, 0, (span - width) // 16) * 16).tolist()


NT, DEEP = 1, 2   # launch flags: nontemporal, 8 deep


# The benchmark's put/get rows, each in the launch shape (work-groups per PE,
# work-group size, flags) the benchmark times it in.
@pytest.mark.parametrize("op,scope,pattern,size,shape", [
    (W.OP_PUT, W.SCOPE_WG, "ring", 16 * MiB, (4, 1024, NT | DEEP)),
    (W.OP_GET, W.SCOPE_WG, "perm", 16 * MiB, (4, 1024, NT | DEEP)),
    (W.OP_PUT, W.SCOPE_GRID, "perm", 64 * MiB, (4, 256, NT | DEEP)),
    (W.OP_PUT, W.SCOPE_WAVE, "perm", 4096, (4, 256, NT)),
    (W.OP_GET, W.SCOPE_THREAD, "ring", 64, (4, 256, 0)),
    (W.OP_PUT, W.SCOPE_THREAD, "perm", 8, (2, 1024, 0)),
    (W.OP_PUT, W.SCOPE_WG, "ring", 4096, (16, 512, 0)),
    (W.OP_GET, W.SCOPE_THREAD, "perm", 16, (16, 256, 0)),
])
def test_sweep_points_64pes_1gib(op, scope, pattern, size, shape):
    npes = 64
    with heap(npes, 1024 * MiB) as v:
        t = torch()
        A = v.offset(v.malloc(256 * MiB))
        B = v.offset(v.malloc(256 * MiB))
        base, stride = v.heap_base(), v.heap_stride()
        for p in range(npes):
            v.fill_random(base + p * stride + A, 256 * MiB, _seed_a(p))
            v.fill_random(base + p * stride + B, 256 * MiB, W.subseed(W.SEED_SWEEP, 0x200 + p))
        k = W.msgs_per_pe(size)
        while k * size > 256 * MiB:
            k //= 2
        tg = W.pattern_targets(pattern, npes)
        assert v.LAUNCH_NONTEMPORAL == NT and v.LAUNCH_DEEP == DEEP
        launch = v.launch_cfg(wgs_per_pe=shape[0], wg_size=shape[1], flags=shape[2])
        v.rma_pattern(op, scope, t.from_numpy(tg.astype(np.int32)).cuda(), A, B, size, k, launch=launch)
        t.cuda.synchronize()
        h = v.heap_view()
        span = k * size
        width = min(4096, span)
        for p in range(0, npes, 7):
            # PE p's destination region holds the source PE's payload
            src_pe = [q for q in range(npes) if tg[q] == p][0] if op == W.OP_PUT else int(tg[p])
            for off in _windows(1000 + p, 6, span, width) + [0, span - width]:
                got = h[p, B + off:B + off + width].cpu().numpy()
                assert np.array_equal(got, W.payload(_seed_a(src_pe), off, width)), (p, off)
            # bytes past the written span are untouched
            if span + 4096 <= 256 * MiB:
                got = h[p, B + span:B + span + 4096].cpu().numpy()
                assert np.array_equal(got, W.payload(W.subseed(W.SEED_SWEEP, 0x200 + p), span, 4096))
        assert_no_device_errors()


def test_gups_256pes_full_size_sampled_witness():
    npes, log2_table, nupd = 256, 27, 1 << 28
    per_pe = 8 << (log2_table - 8)                      # 4 MiB of table per PE
    with heap(npes, 8 * MiB) as v:
        t = torch()
        base, stride = v.heap_base(), v.heap_stride()
        for p in range(npes):
            v.fill_typed(base + p * stride, per_pe // 8, v.DT_INT64, W.subseed(W.SEED_GUPS, W.TAG_HEAP + p))
        fetched = t.zeros(nupd, dtype=t.int64, device="cuda")
        acc = t.zeros(1, dtype=t.int64, device="cuda")
        v.gups(0, log2_table, nupd, W.subseed(W.SEED_GUPS, W.TAG_OPS), 5, fetched=fetched, acc=acc)
        t.cuda.synchronize()
        # sampled words: every update that hits them, in the oracle's stream order
        samples = np.unique((W.splitmix64(77, 0, 256) & np.uint64((1 << log2_table) - 1)))
        sel_u, sel_idx, sel_val, sel_add = [], [], [], []
        chunk = 1 << 24
        for c0 in range(0, nupd, chunk):
            idx, val, is_add = W.gups_updates(W.SEED_GUPS, c0, chunk, log2_table)
            m = np.isin(idx, samples)
            sel_u.append(np.nonzero(m)[0] + c0)
            sel_idx.append(idx[m]); sel_val.append(val[m]); sel_add.append(is_add[m])
        u = np.concatenate(sel_u)
        idx = np.concatenate(sel_idx); val = np.concatenate(sel_val); is_add = np.concatenate(sel_add)
        f = fetched[t.from_numpy(u.astype(np.int64)).cuda()].cpu().numpy().view(np.uint64)
        init = np.array([int(W.splitmix64(W.subseed(W.SEED_GUPS, W.TAG_HEAP + int(g) // (1 << 19)), int(g) % (1 << 19), 1)[0])
                         for g in samples], dtype=np.uint64)
        h = v.heap_view()
        final = np.array([int(h[int(g) // (1 << 19), (int(g) % (1 << 19)) * 8:(int(g) % (1 << 19)) * 8 + 8]
                              .cpu().numpy().view(np.uint64)[0]) for g in samples], dtype=np.uint64)
        word = np.searchsorted(samples, idx).astype(np.uint64)
        kind = np.where(is_add, oracle.KIND_FETCH_ADD, oracle.KIND_FETCH_XOR).astype(np.uint8)
        assert len(u) > 200
        assert oracle.witness_check(word, kind, val, f, init, final) == 0
        # whole-run invariant: the accumulator is the XOR of every fetched value
        x = np.bitwise_xor.reduce(fetched.cpu().numpy().view(np.uint64))
        assert int(acc.cpu().numpy().view(np.uint64)[0]) == int(x)
        assert_no_device_errors()


def test_collectives_64pes_full_size_sampled():
    npes = 64
    with heap(npes, 1024 * MiB) as v:
        t = torch()
        B = v.offset(v.malloc(256 * MiB))
        C = v.offset(v.malloc(256 * MiB))
        D = v.offset(v.malloc(128 * MiB))
        E = v.offset(v.malloc(64 * MiB))
        F = v.offset(v.malloc(32 * MiB))
        base, stride = v.heap_base(), v.heap_stride()
        for p in range(npes):
            v.fill_random(base + p * stride + C, 256 * MiB, W.subseed(W.SEED_COLL, W.TAG_HEAP + p))
            v.fill_typed(base + p * stride + D, 16 * MiB, v.DT_INT64, W.subseed(W.SEED_COLL, 0x300 + p))
            v.fill_typed(base + p * stride + E, 16 * MiB, v.DT_FP32, W.subseed(W.SEED_COLL, 0x400 + p))
            v.fill_typed(base + p * stride + F, 16 * MiB, v.DT_BF16, W.subseed(W.SEED_COLL, 0x500 + p))
        t.cuda.synchronize()
        h = v.heap_view()
        addr = lambda off: base + off  # noqa: E731
        cseed = lambda q: W.subseed(W.SEED_COLL, W.TAG_HEAP + q)  # noqa: E731
        # alltoall, 1 MiB blocks: PE p's block q is PE q's block p
        blk = MiB
        v.alltoallmem(addr(B), addr(C), blk)
        t.cuda.synchronize()
        for p in range(0, npes, 9):
            for q in range(0, npes, 11):
                for off in _windows(p * 64 + q, 2, blk, 256):
                    got = h[p, B + q * blk + off:B + q * blk + off + 256].cpu().numpy()
                    assert np.array_equal(got, W.payload(cseed(q), p * blk + off, 256)), (p, q, off)
        # fcollect, 4 MiB per PE
        fc = 4 * MiB
        v.fcollectmem(addr(B), addr(C), fc)
        t.cuda.synchronize()
        for p in range(0, npes, 13):
            for q in range(0, npes, 5):
                for off in _windows(7 * p + q, 2, fc, 512):
                    got = h[p, B + q * fc + off:B + q * fc + off + 512].cpu().numpy()
                    assert np.array_equal(got, W.payload(cseed(q), off, 512))
        # broadcast, 256 MiB from PE 0, the root's destination included
        bc = 256 * MiB
        v.broadcastmem(addr(B), addr(C), bc, 0)
        t.cuda.synchronize()
        for p in [0, 1, 31, 63]:
            for off in _windows(99 + p, 8, bc, 4096) + [bc - 4096]:
                got = h[p, B + off:B + off + 4096].cpu().numpy()
                assert np.array_equal(got, W.payload(cseed(0), off, 4096))
        # reductions, 2^24 elements: sampled elements recomputed by the oracle's TREE
        nred = 1 << 24
        ks = np.unique(W.bounded(W.splitmix64(5, 0, 300), 0, nred - 1))
        ks = np.concatenate([ks, [0, nred - 1]])
        for dt, src, es, seed_tag, gen in ((oracle.DT_INT64, D, 8, 0x300, W.coll_i64), (oracle.DT_FP32, E, 4, 0x400, None),
                                           (oracle.DT_BF16, F, 2, 0x500, None)):
            for rop in (oracle.RO_SUM, oracle.RO_MAX):
                if dt == oracle.DT_BF16 and rop == oracle.RO_MAX:
                    continue
                v.reduce(dt, rop, addr(B), addr(src), nred)
                t.cuda.synchronize()
                cols = []
                for q in range(npes):
                    x = np.stack([W.splitmix64(W.subseed(W.SEED_COLL, seed_tag + q), int(k), 1)[0] for k in ks])
                    if dt == oracle.DT_INT64:
                        cols.append(x.view(np.int64))
                    elif dt == oracle.DT_FP32:
                        cols.append(W.uniform_f32(x))
                    else:
                        cols.append(W.f32_to_bf16_bits(W.uniform_f32(x)))
                want = oracle.reduce_columns(np.stack(cols), dt, rop)
                for p in (0, 17, 63):
                    row = h[p, B:B + nred * es].cpu().numpy()
                    got = np.array([row[int(k) * es:(int(k) + 1) * es].view(want.dtype)[0] for k in ks])
                    assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), (dt, rop, p)
        assert_no_device_errors()


def test_serving_128pes_full_size_sampled_hashes():
    """Serving at full size: 128 PEs x 512 MiB, 4000 requests log-uniform
    64 B - 16 MiB over put/get/fetch_add, a 64 GiB budget, the progress
    kernel in the launch shape bench.py times.  Every request completes once
    with status 0; the device's output hash of sampled requests equals the
    hash of the bytes the seeded generator put at their sources (or of the
    zero fetched values of fresh counters)."""
    npes = 128
    with heap(npes, 512 * MiB) as v:
        t = torch()
        src = v.offset(v.malloc(128 * MiB))
        region = v.offset(v.malloc(384 * MiB))
        base, stride = v.heap_base(), v.heap_stride()
        seed_of = lambda p: W.subseed(W.SEED_SERVE, W.TAG_HEAP + p)  # noqa: E731
        for p in range(npes):
            v.fill_random(base + p * stride + src, 128 * MiB, seed_of(p))
        v.heap_view()[:, region + 288 * MiB:region + 384 * MiB].zero_()
        t.cuda.synchronize()
        from paper_2607_08006_amd import Request
        n = 4000
        xs = W.splitmix64(W.subseed(W.SEED_SERVE, 0x77), 0, n)
        reqs = []
        for i, r in enumerate(W.serve_requests(W.SEED_SERVE, n, npes, rate_per_s=1e12, lanes=8)):
            nb = r.nbytes
            s0 = 0 if r.kind == W.OP_AMO_FETCH_ADD else int(xs[i] % np.uint64(128 * MiB - nb + 1))
            reqs.append(Request(r.kind, r.issuer, r.target, r.lane, nb, s0, r.arrival_s))
        side = t.cuda.Stream()
        v.progress_start(nwg=0, wg_size=1024, ring_slots=4096, verify=True, chunk_bytes=256 << 10, stream=side)
        try:
            dst, lat, comps, stats = v.serve_run(reqs, 8, region, 384 * MiB, 64 << 30)
        finally:
            v.progress_stop(60000)
            side.synchronize()
        assert stats.max_reserved_bytes <= 64 << 30
        assert all(c.status == 0 for c in comps)
        assert len(set(c.ticket for c in comps)) == n
        small = [i for i, r in enumerate(reqs) if r.nbytes <= 256 << 10]
        large = [i for i, r in enumerate(reqs) if r.nbytes > 8 << 20]
        pick = small[::max(1, len(small) // 300)] + large[:6]
        assert len(pick) > 200
        for i in pick:
            r = reqs[i]
            if r.op == W.OP_AMO_FETCH_ADD:
                want = out_hash(np.zeros(r.nbytes, dtype=np.uint8))
            else:
                spe = r.issuer_pe if r.op == W.OP_PUT else r.target_pe
                want = out_hash(W.payload(seed_of(spe), r.src_off, r.nbytes))
            assert comps[i].hash == want, (i, r.op, r.nbytes)
        # The bytes themselves: read back the destination of every sampled
        # request whose range no request completing after it overlapped
        # (admission hands freed ranges out again), and compare them with the
        # generator's source bytes (or the zero values fresh counters held).
        out_pe = [r.target_pe if r.op == W.OP_PUT else r.issuer_pe for r in reqs]
        on_pe = {}
        for j in range(n):
            on_pe.setdefault(out_pe[j], []).append(j)
        h = v.heap_view()
        checked = 0
        for i in pick:
            r = reqs[i]
            lo, hi = int(dst[i]), int(dst[i]) + r.nbytes
            if any(j != i and int(dst[j]) < hi and lo < int(dst[j]) + reqs[j].nbytes
                   and comps[j].t_end >= comps[i].t_end for j in on_pe[out_pe[i]]):
                continue
            got = h[out_pe[i], lo:hi].cpu().numpy()
            if r.op == W.OP_AMO_FETCH_ADD:
                assert not got.any(), (i, r.nbytes)
            else:
                spe = r.issuer_pe if r.op == W.OP_PUT else r.target_pe
                assert np.array_equal(got, W.payload(seed_of(spe), r.src_off, r.nbytes)), (i, r.op, r.nbytes)
            checked += 1
        assert checked >= 50, checked
        assert_no_device_errors()



def test_host_paths_64pes_1gib_full_size():
    """The host-initiated transfers at the sizes bench.py times them (64 PEs x
    1 GiB): a 256 MiB blocking put from pinned host memory, the 256 MiB
    device-to-device put the copy kernel executes, and 256 MiB gets back to
    pinned memory, compared byte for byte with the seeded source."""
    from paper_2607_08006_amd import host
    t = torch()
    npes, n = 64, 256 * MiB
    with heap(npes, 1024 * MiB) as v:
        a, b = v.malloc(n), v.malloc(n)
        src = W.heap_fill(W.SEED_SWEEP + 11, 1, n)[0]
        pinned = t.from_numpy(src.copy()).pin_memory()
        back = t.zeros(n, dtype=t.uint8).pin_memory()
        t.cuda.synchronize()
        host.putmem(a, pinned, n, 0)                 # host memory -> PE 0
        host.putmem(b, a, n, npes - 1)               # PE 0 -> PE 63 on the copy kernel
        host.getmem(back, b, n, npes - 1)
        assert np.array_equal(back.numpy(), src)
        back.zero_()
        host.getmem(back, a, n, 0)
        assert np.array_equal(back.numpy(), src)
        # an unaligned sub-range through the copy kernel's head and tail paths
        host.putmem(b + 3, a + 5, n - 4096 - 7, 17)
        host.getmem(back, b, n, 17)
        assert np.array_equal(back.numpy()[3:n - 4096 - 4], src[5:n - 4096 - 2])
        assert_no_device_errors()
