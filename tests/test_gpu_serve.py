"""GPU: the persistent progress kernel and trace-driven serving.

Every request's output must equal the oracle's, whether the request runs
alone or among others; admission must never exceed the heap budget; every
request completes exactly once."""
import time

import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, download, heap, out_hash, torch, upload

pytestmark = pytest.mark.gpu

def _desc(op, issuer, target, src, dst, n, value=0):
    d = W.descs([(op, W.SCOPE_AUTO, 0, issuer, target, W.NO_RESULT, src, dst, n, value, 0)])
    from paper_2607_08006_amd import Desc
    return Desc.from_buffer_copy(d.tobytes())


def test_progress_submit_poll_matches_oracle():
    npes = 8
    with heap(npes, 8 << 20) as v:
        t = torch()
        region = 6 << 20
        init = W.heap_fill(0xC0FFEE, npes, region)
        init[:, 5 << 20:] = 0                             # counters start at zero
        upload(init)
        side = t.cuda.Stream()
        v.progress_start(nwg=64, wg_size=256, ring_slots=64, verify=True, chunk_bytes=64 << 10, stream=side)
        reqs = [
            (W.OP_PUT, 0, 3, 0, 2 << 20, 100),
            (W.OP_GET, 5, 1, 4096, (2 << 20) + 4096, 70_000),          # several chunks + ragged tail
            (W.OP_PUT, 7, 7, 8192, (3 << 20), 1 << 20),                # 16 chunks, self target
            (W.OP_AMO_FETCH_ADD, 2, 6, 5 << 20, (4 << 20), 4096),      # 512 counters, results on issuer
            (W.OP_PUT, 1, 2, 13, (2 << 20) + 77, 999),                 # unaligned
        ]
        tickets = [v.progress_submit(_desc(*r, value=1 if r[0] == W.OP_AMO_FETCH_ADD else 0)) for r in reqs]
        comps = {}
        t0 = time.time()
        while len(comps) < len(tickets) and time.time() - t0 < 30:
            for tk in tickets:
                if tk not in comps:
                    c = v.progress_poll(tk)
                    if c is not None:
                        comps[tk] = c
        v.progress_stop(10000)
        side.synchronize()
        assert len(comps) == len(tickets)
        got = download(region)
        ref = init.copy()
        recs = []
        for k, (op, i, tg, s, d, n) in enumerate(reqs):
            if op == W.OP_AMO_FETCH_ADD:
                for w in range(n // 8):
                    recs.append((op, 0, 0, i, tg, W.NO_RESULT, s + 8 * w, 0, 8, 1, 0))
            else:
                recs.append((op, 0, 0, i, tg, W.NO_RESULT, s, d, n, 0, 0))
        oracle.run_program(ref, W.descs(recs))
        # the AMO's fetched values (zeros) land in the issuer's result range
        op, i, tg, s, d, n = reqs[3]
        ref[i, d:d + n] = 0
        assert np.array_equal(got, ref)
        for tk, (op, i, tg, s, d, n) in zip(tickets, reqs):
            c = comps[tk]
            assert c.status == 0 and c.t_end >= c.t_start > 0
            out_pe = tg if op == W.OP_PUT else i
            assert c.hash == out_hash(ref[out_pe, d:d + n])
        assert_no_device_errors()


def test_backlog_split_matches_oracle():
    """One worker and many queued requests: the front-end switches to the
    larger split while the worker is backlogged; every output (ragged
    tails, unaligned, AMO counters) still equals the oracle's."""
    npes = 4
    with heap(npes, 8 << 20) as v:
        t = torch()
        region = 7 << 20
        init = W.heap_fill(0xB4C106, npes, region)
        init[:, 6 << 20:] = 0                             # counters start at zero
        upload(init)
        side = t.cuda.Stream()
        t.cuda.synchronize()
        v.progress_start(nwg=2, wg_size=256, ring_slots=64, verify=True, chunk_bytes=4 << 10, stream=side)
        rng = np.random.default_rng(17)
        reqs, dst = [], 2 << 20
        for k in range(40):
            n = int(rng.integers(1, 100_000))
            op = (W.OP_PUT, W.OP_GET, W.OP_AMO_FETCH_ADD)[k % 3]
            i, tg = int(rng.integers(npes)), int(rng.integers(npes))
            if op == W.OP_AMO_FETCH_ADD:
                n = (n // 8 + 1) * 8
                src = (6 << 20) + 8 * int(rng.integers(0, 1000))
            else:
                src = int(rng.integers(0, 1 << 20))
            reqs.append((op, i, tg, src, dst + (0 if op == W.OP_AMO_FETCH_ADD else k % 5), n))
            dst += ((n + 4096) // 4096 + 1) * 4096
        assert dst + 8 < (6 << 20)
        tickets = [v.progress_submit(_desc(*r, value=3 if r[0] == W.OP_AMO_FETCH_ADD else 0)) for r in reqs]
        comps, t0 = {}, time.time()
        while len(comps) < len(tickets) and time.time() - t0 < 30:
            for tk in tickets:
                if tk not in comps:
                    c = v.progress_poll(tk)
                    if c is not None:
                        comps[tk] = c
        v.progress_stop(10000)
        side.synchronize()
        assert len(comps) == len(tickets)
        got = download(region)
        # AMO results depend on the order of requests on shared counters;
        # the counters' final values and every copy do not.
        ref = init.copy()
        recs = []
        for op, i, tg, s, d, n in reqs:
            if op == W.OP_AMO_FETCH_ADD:
                for w in range(n // 8):
                    recs.append((op, 0, 0, i, tg, W.NO_RESULT, s + 8 * w, 0, 8, 3, 0))
            else:
                recs.append((op, 0, 0, i, tg, W.NO_RESULT, s, d, n, 0, 0))
        oracle.run_program(ref, W.descs(recs))
        amo_out = np.zeros(got.shape, dtype=bool)
        for op, i, tg, s, d, n in reqs:
            if op == W.OP_AMO_FETCH_ADD:
                amo_out[i, d:d + n] = True
        assert np.array_equal(got[~amo_out], ref[~amo_out])
        ctr0, ctr_words = 6 << 20, (1 << 20) // 8          # every counter lies in [6 MiB, 7 MiB)
        words, fetched = [], []
        for tk, (op, i, tg, s, d, n) in zip(tickets, reqs):
            c = comps[tk]
            assert c.status == 0 and c.t_end >= c.t_start > 0
            if op != W.OP_AMO_FETCH_ADD:
                out_pe = tg if op == W.OP_PUT else i
                assert c.hash == out_hash(ref[out_pe, d:d + n])
            else:
                assert ctr0 <= s and s + n <= ctr0 + 8 * ctr_words
                words.append(tg * ctr_words + (s - ctr0) // 8 + np.arange(n // 8, dtype=np.uint64))
                fetched.append(got[i, d:d + n].view(np.uint64))
        # Requests share counters, so the fetched values depend on the order
        # the device applied them in: witness replay must find, for every
        # counter, a serial order of its fetch_add(+3)s that explains each
        # fetched value and the final value (untouched counters stay zero).
        words, fetched = np.concatenate(words), np.concatenate(fetched)
        init_w = init[:, ctr0:ctr0 + 8 * ctr_words].copy().view(np.uint64).ravel()
        final_w = got[:, ctr0:ctr0 + 8 * ctr_words].copy().view(np.uint64).ravel()
        assert oracle.witness_check(words, np.full(len(words), oracle.KIND_FETCH_ADD, dtype=np.uint8),
                                    np.full(len(words), 3, dtype=np.uint64), fetched, init_w, final_w) == 0
        assert np.array_equal(final_w, ref[:, ctr0:ctr0 + 8 * ctr_words].copy().view(np.uint64).ravel())
        assert_no_device_errors()


def _trace(npes, n, rate, src_bytes, seed, max_log2=14):
    rs = W.serve_requests(seed, n, npes, rate_per_s=rate, lanes=8, size_log2_span=max_log2)
    from paper_2607_08006_amd import Request
    out = []
    for r in rs:
        nb = min(r.nbytes, src_bytes)
        if r.kind == W.OP_AMO_FETCH_ADD:
            nb = max(8, nb & ~7)
        src = 0 if r.kind == W.OP_AMO_FETCH_ADD else int(W.splitmix64(seed, len(out), 1)[0] % np.uint64(src_bytes - nb + 1))
        out.append(Request(r.kind, r.issuer, r.target, r.lane, nb, src, r.arrival_s))
    return out


def _expected_hashes(reqs, init):
    hs = []
    for r in reqs:
        if r.op == W.OP_AMO_FETCH_ADD:
            hs.append(out_hash(np.zeros(r.nbytes, dtype=np.uint8)))
        else:
            spe = r.issuer_pe if r.op == W.OP_PUT else r.target_pe
            hs.append(out_hash(init[spe, r.src_off:r.src_off + r.nbytes]))
    return hs


def test_serving_alone_equals_mix_and_budget_holds():
    npes, n = 16, 400
    src_bytes = 2 << 20
    with heap(npes, 40 << 20) as v:
        t = torch()
        init = W.heap_fill(0xBEEF, npes, src_bytes)
        upload(init)
        region_off, region_bytes = 4 << 20, 32 << 20
        reqs = _trace(npes, n, rate=2e5, src_bytes=src_bytes, seed=W.SEED_SERVE)
        want = _expected_hashes(reqs, init)
        side = t.cuda.Stream()

        def run(trace, budget):
            h = v.heap_view()
            h[:, region_off:region_off + region_bytes].zero_()
            t.cuda.synchronize()
            v.progress_start(nwg=128, wg_size=256, ring_slots=256, verify=True, chunk_bytes=64 << 10, stream=side)
            try:
                dst, lat, comps, stats = v.serve_run(trace, 8, region_off, region_bytes, budget)
            finally:
                v.progress_stop(20000)
                side.synchronize()
            return dst, lat, comps, stats

        # in the mix: bursty Poisson arrivals, a budget small enough to make requests wait
        budget = 3 << 20
        dst, lat, comps, stats = run(reqs, budget)
        assert stats.max_reserved_bytes <= budget
        assert stats.admission_waits > 0
        tickets = [c.ticket for c in comps]
        assert len(set(tickets)) == n                      # no lost or duplicated completion
        mix = [c.hash for c in comps]
        assert all(c.status == 0 for c in comps)
        assert (lat > 0).all()
        # alone: one request at a time, far apart
        from paper_2607_08006_amd import Request
        alone_trace = [Request(r.op, r.issuer_pe, r.target_pe, 0, r.nbytes, r.src_off, 0.0002 * k)
                       for k, r in enumerate(reqs)]
        _, _, comps_a, stats_a = run(alone_trace, 1 << 30)
        alone = [c.hash for c in comps_a]
        bad = [(i, reqs[i].op, reqs[i].nbytes, mix[i] == want[i], alone[i] == want[i])
               for i in range(n) if not (mix[i] == alone[i] == want[i])]
        assert not bad, bad[:20]
        assert_no_device_errors()


def test_progress_rejects_bad_config_and_busy_ring():
    with heap(4, 4 << 20) as v:
        t = torch()
        with pytest.raises(v.VshmemError):
            v.progress_start(nwg=1, wg_size=64)                 # no worker wavefronts
        with pytest.raises(v.VshmemError):
            v.progress_start(ring_slots=3)                      # not a power of two
        with pytest.raises(v.VshmemError):
            v.progress_start(chunk_bytes=(1 << 40) + 16)        # items up to 16x must not overflow
        side = t.cuda.Stream()
        v.progress_start(nwg=8, wg_size=128, ring_slots=4, stream=side, idle_timeout_ms=5000)
        with pytest.raises(v.VshmemError):
            v.progress_start(nwg=8, stream=side)                # already running
        # invalid request (outside the heap) completes with an error status
        bad = _desc(W.OP_PUT, 0, 1, v.heap_user_bytes() - 8, 0, 64)
        tk = v.progress_submit(bad)
        c = None
        t0 = time.time()
        while c is None and time.time() - t0 < 10:
            c = v.progress_poll(tk)
        assert c is not None and c.status == -1
        v.progress_stop(10000)
        side.synchronize()
        assert v.device_errors() & v.DEVERR_BAD_DESC


def test_launch_request_matches_oracle():
    npes = 8
    with heap(npes, 8 << 20) as v:
        t = torch()
        region = 6 << 20
        init = W.heap_fill(0xFACE, npes, region)
        init[:, 5 << 20:] = 0
        upload(init)
        reqs = [
            (W.OP_PUT, 0, 3, 0, 2 << 20, 100),
            (W.OP_GET, 5, 1, 4096, (2 << 20) + 4096, 70_000),          # 5 chunks of 16 KiB, ragged tail
            (W.OP_PUT, 7, 7, 8192, 3 << 20, 1 << 20),
            (W.OP_AMO_FETCH_ADD, 2, 6, 5 << 20, 4 << 20, 4096),
            (W.OP_PUT, 1, 2, 13, (2 << 20) + 77, 999),                  # unaligned
            (W.OP_GET, 4, 4, 0, (4 << 20) + 8192, 0),                   # empty
        ]
        for r in reqs:
            v.launch_request(_desc(*r, value=1 if r[0] == W.OP_AMO_FETCH_ADD else 0), chunk_bytes=16 << 10, wg_size=128)
        t.cuda.synchronize()
        got = download(region)
        ref = init.copy()
        recs = []
        for op, i, tg, s, d, n in reqs:
            if op == W.OP_AMO_FETCH_ADD:
                recs += [(op, 0, 0, i, tg, W.NO_RESULT, s + 8 * w, 0, 8, 1, 0) for w in range(n // 8)]
            elif n:
                recs.append((op, 0, 0, i, tg, W.NO_RESULT, s, d, n, 0, 0))
        oracle.run_program(ref, W.descs(recs))
        op, i, tg, s, d, n = reqs[3]
        ref[i, d:d + n] = 0                                   # fetched values of fresh counters
        assert np.array_equal(got, ref)
        with pytest.raises(v.VshmemError):
            v.launch_request(_desc(W.OP_PUT, 0, npes, 0, 0, 64))          # target PE out of range
        with pytest.raises(v.VshmemError):
            v.launch_request(_desc(W.OP_PUT, 0, 1, 0, 0, 64), chunk_bytes=24)
        assert_no_device_errors()


@pytest.mark.parametrize("form", ["per_op", "batched_fused", "batched_graph"])
def test_serving_other_forms_final_state_and_budget(form):
    """The per-op and windowed-batch forms on a trace: every request completes
    once, the budget holds, and the final heap equals replaying the requests
    in completion order (a destination is reused only after its request
    completed, so the last writer of each byte is the one that finished
    last)."""
    npes, n = 16, 300
    src_bytes = 2 << 20
    with heap(npes, 40 << 20) as v:
        t = torch()
        init = W.heap_fill(0xD00D, npes, src_bytes)
        upload(init)
        region_off, region_bytes = 4 << 20, 32 << 20
        reqs = _trace(npes, n, rate=2e5, src_bytes=src_bytes, seed=W.SEED_SERVE + 1)
        h = v.heap_view()
        h[:, region_off:region_off + region_bytes].zero_()
        t.cuda.synchronize()
        budget = 3 << 20
        if form == "per_op":
            dst, lat, comps, stats = v.serve_run_per_op(reqs, 8, region_off, region_bytes, budget,
                                                        chunk_bytes=64 << 10, wg_size=256)
        else:
            dst, lat, comps, stats = v.serve_run_batched(reqs, 8, region_off, region_bytes, budget, window_us=30.0,
                                                         use_graph=form == "batched_graph", chunk_bytes=64 << 10,
                                                         wg_size=256)
        t.cuda.synchronize()
        assert stats.max_reserved_bytes <= budget
        assert sorted(c.ticket for c in comps) == list(range(n))
        assert (lat > 0).all()
        got = download(region_off + region_bytes)
        want = np.zeros_like(got)
        written = np.zeros(got.shape, dtype=bool)
        done_at = np.array([r.arrival_s * 1e9 for r in reqs]) + lat.astype(np.float64)
        for k in np.argsort(done_at, kind="stable"):
            r, d = reqs[k], int(dst[k])
            if r.op == W.OP_AMO_FETCH_ADD:
                payload = np.zeros(r.nbytes, dtype=np.uint8)
                pe = r.issuer_pe
            else:
                spe = r.issuer_pe if r.op == W.OP_PUT else r.target_pe
                payload = init[spe, r.src_off:r.src_off + r.nbytes]
                pe = r.target_pe if r.op == W.OP_PUT else r.issuer_pe
            want[pe, d:d + r.nbytes] = payload
            written[pe, d:d + r.nbytes] = True
        assert np.array_equal(got[written], want[written])
        # fetch_add counters are bump allocated: every one was incremented exactly once
        n_ctr = sum(r.nbytes // 8 for r in reqs if r.op == W.OP_AMO_FETCH_ADD)
        ctr_base = region_off + ((region_bytes // 4 * 3) & ~255)
        ctr = got[:, ctr_base:].copy().view("<u8")
        assert int(ctr.sum()) == n_ctr and int(ctr.max()) <= 1
        assert_no_device_errors()


def test_progress_request_larger_than_item_queue():
    """A request split into more items than the device queue holds (2 MiB in
    16-byte items = 131072 items, queue 65536) is published in parts and
    still completes with the right bytes; a small request behind it too."""
    npes = 4
    with heap(npes, 8 << 20) as v:
        t = torch()
        region = 6 << 20
        init = W.heap_fill(0xA11CE, npes, region)
        upload(init)
        side = t.cuda.Stream()
        v.progress_start(nwg=64, wg_size=256, ring_slots=16, verify=True, chunk_bytes=16, stream=side)
        reqs = [(W.OP_PUT, 0, 1, 0, 3 << 20, 2 << 20), (W.OP_GET, 2, 3, 4096, (5 << 20) + 16, 1000)]
        tickets = [v.progress_submit(_desc(*r)) for r in reqs]
        comps = {}
        t0 = time.time()
        while len(comps) < len(tickets) and time.time() - t0 < 60:
            for tk in tickets:
                if tk not in comps:
                    c = v.progress_poll(tk)
                    if c is not None:
                        comps[tk] = c
        v.progress_stop(20000)
        side.synchronize()
        assert len(comps) == len(tickets)
        got = download(region)
        ref = init.copy()
        oracle.run_program(ref, W.descs([(op, 0, 0, i, tg, W.NO_RESULT, s, d, n, 0, 0) for op, i, tg, s, d, n in reqs]))
        assert np.array_equal(got, ref)
        for tk, (op, i, tg, s, d, n) in zip(tickets, reqs):
            out_pe = tg if op == W.OP_PUT else i
            assert comps[tk].status == 0 and comps[tk].hash == out_hash(ref[out_pe, d:d + n])
            assert comps[tk].t_queued > 0 and comps[tk].t_end >= comps[tk].t_start >= comps[tk].t_queued
        assert_no_device_errors()


def test_completed_request_is_visible_while_the_kernel_runs():
    """A request's completion means its bytes are visible device-wide: with
    the progress kernel still running (on few work-groups, so other kernels
    get CUs), each completed put is read back at once by a separate copy and
    equals its source.  Every put rewrites the same destination from another
    source range, so a stale or late write would show.  Items are small
    (16 KiB), so each request is split over several workers, which hold
    finished items for a later release."""
    npes = 6
    with heap(npes, 8 << 20) as v:
        t = torch()
        region = 4 << 20
        init = W.heap_fill(0xD0D0, npes, region)
        upload(init)
        side, reader = t.cuda.Stream(), t.cuda.Stream()
        t.cuda.synchronize()
        v.progress_start(nwg=8, wg_size=256, ring_slots=64, chunk_bytes=16 << 10, idle_timeout_ms=5000,
                         stream=side)
        h = v.heap_view()
        dst = 3 << 20
        try:
            for k in range(40):
                n = 200_000 + 4093 * k
                src_pe, tgt = k % npes, (k + 1) % npes
                src = (k * 24_577) % (dst - n)
                tk = v.progress_submit(_desc(W.OP_PUT, src_pe, tgt, src, dst, n))
                t0 = time.time()
                c = None
                while c is None and time.time() - t0 < 20:
                    c = v.progress_poll(tk)
                assert c is not None and c.status == 0, k
                with t.cuda.stream(reader):                    # a copy on a stream of its own
                    got = h[tgt, dst:dst + n].cpu().numpy()
                assert np.array_equal(got, init[src_pe, src:src + n]), k
        finally:
            v.progress_stop(10000)
            side.synchronize()
        assert_no_device_errors()


def test_progress_lanes_are_checked_and_recorded():
    """Requests carry the producer lane they were submitted on into their
    completion records; a lane outside [0, 8) is refused on the host."""
    npes = 2
    with heap(npes, 4 << 20) as v:
        t = torch()
        region = 2 << 20
        init = W.heap_fill(0x1A7E, npes, region)
        upload(init)
        side = t.cuda.Stream()
        t.cuda.synchronize()
        v.progress_start(nwg=8, wg_size=256, ring_slots=64, stream=side)
        reqs, tickets, comps = [], {}, {}
        try:
            for lane in (-1, v.PROGRESS_LANES):
                with pytest.raises(v.VshmemError) as e:
                    v.progress_submit(_desc(W.OP_PUT, 0, 1, 0, 1 << 20, 64), lane=lane)
                assert e.value.code == v.ERR_ARG
            for lane in range(v.PROGRESS_LANES):
                r = (W.OP_PUT if lane % 2 else W.OP_GET, lane % 2, (lane + 1) % 2, 4096 * lane,
                     (1 << 20) + 8192 * lane, 1000 + 7 * lane)
                reqs.append(r)
                tickets[v.progress_submit(_desc(*r), lane=lane)] = lane
            t0 = time.time()
            while len(comps) < len(tickets) and time.time() - t0 < 30:
                for tk in tickets:
                    if tk not in comps:
                        c = v.progress_poll(tk)
                        if c is not None:
                            comps[tk] = c
        finally:
            v.progress_stop(10000)
            side.synchronize()
        assert len(comps) == len(tickets)
        for tk, lane in tickets.items():
            assert comps[tk].status == 0 and comps[tk].lane == lane
        ref = init.copy()
        oracle.run_program(ref, W.descs([(op, 0, 0, i, tg, W.NO_RESULT, s, d, n, 0, 0) for op, i, tg, s, d, n in reqs]))
        assert np.array_equal(download(region), ref)
        assert_no_device_errors()


def test_waiting_kernels_beside_the_progress_kernel():
    """Kernels whose work-groups wait for each other (team collectives,
    barriers, multi-phase fused plans) count only the CUs the persistent
    progress kernel leaves free: beside a kernel that holds every CU they
    are refused with SHMEMX_ERR_BUSY before anything is launched; beside
    one that holds a quarter of the CUs they launch on the rest and still
    equal the oracle."""
    npes, n = 8, 4096
    with heap(npes, 4 << 20) as v:
        t = torch()
        src, dst = v.malloc(npes * n), v.malloc(npes * n)
        so, do = v.offset(src), v.offset(dst)
        region = do + npes * n
        init = W.heap_fill(0xC0DE5, npes, region)
        wl = W.small_workload(npes=npes, heap_bytes=1 << 20, n_rma=100, epoch_ops=50, n_amo=100,
                              base_off=region, fill=False)
        plan = v.Plan(wl.descs)
        assert plan.info()["phases"] > 1
        side = t.cuda.Stream()
        upload(init)
        v.progress_start(nwg=0, wg_size=1024, stream=side)        # one work-group on every CU
        try:
            for name, call in (("alltoall", lambda: v.alltoallmem(dst, src, n)),
                               ("barrier", lambda: v.barrier(v.DEVICE_TEAM_WORLD, iters=1)),
                               ("fused plan", lambda: plan.launch_fused())):
                with pytest.raises(v.VshmemError) as e:
                    call()
                assert e.value.code == v.ERR_BUSY, name
        finally:
            v.progress_stop(10000)
            side.synchronize()
        assert np.array_equal(download(region), init)              # nothing ran
        quarter = max(2, t.cuda.get_device_properties(0).multi_processor_count // 4)
        v.progress_start(nwg=quarter, wg_size=1024, stream=side)
        try:
            v.alltoallmem(dst, src, n)
            v.barrier(v.DEVICE_TEAM_WORLD, iters=3)
            t.cuda.current_stream().synchronize()
        finally:
            v.progress_stop(10000)
            side.synchronize()
        ref = init.copy()
        oracle.alltoall(ref, do, so, n)
        assert np.array_equal(download(region), ref)
        plan.destroy()
        assert_no_device_errors()
