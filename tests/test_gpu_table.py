"""GPU parity: batches over a descriptor table in DEVICE memory, written by a
kernel (the test's own user kernel assembles it from column arrays), in the
fused form (classify, index and executor kernels), the per-operation form
and graphs of both, against the oracle run on the same program.  Also: graphs
replay what the table holds at replay time, invalid descriptors are skipped
and reported, plans launched together on two streams keep their barriers
apart, the active tune table comes from VSHMEM_TUNE_FILE, and empty,
one-operation, ordering-only and zero-byte tables run cleanly."""
import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, download, heap, program as _program, torch, upload, write_table

pytestmark = pytest.mark.gpu


def _tunes(v):
    """(name, device tune or None): the active table; work-group scope with
    256-byte tasks from 256 B up (many tasks per message); one lane for
    everything."""
    t = torch()
    wg = v.default_tune()
    for c in range(W.log2_class(256), 40):
        wg.scope[c] = v.SCOPE_WG
        wg.chunk[c] = 256
    lane = v.default_tune()
    for c in range(40):
        lane.scope[c] = v.SCOPE_THREAD
    out = [("active", None)]
    for name, tb in (("wg_256B_tasks", wg), ("one_lane", lane)):
        buf = bytes(tb)
        out.append((name, t.frombuffer(bytearray(buf), dtype=t.uint8).to("cuda")))
    return out


def _check(v, got, ref, res, wl, descs):
    assert np.array_equal(got, ref)
    fetched = res.cpu().numpy()[:wl.n_amo]
    amo = descs[descs["op"] == W.OP_AMO_FETCH_ADD]
    for c in np.unique(amo["src"]):
        ids = amo[amo["src"] == c]["result_idx"].astype(np.int64)
        assert np.array_equal(np.sort(fetched[ids]), np.arange(len(ids))), "fetched values are not a permutation"


def test_kernel_written_table_all_forms_match_oracle():
    t = torch()
    with heap(4, 2 << 20) as v:
        wl, descs = _program(W.SEED_SMALL)
        n = len(descs)
        table = write_table(descs)
        ref = wl.init.copy()
        oracle.run_program(ref, descs, nresults=wl.n_amo)
        s = t.cuda.Stream()
        for tname, dtune in _tunes(v):
            res = t.zeros(n, dtype=t.int64, device="cuda")
            for form in ("fused", "per_op"):
                upload(wl.init)
                res.zero_()
                with t.cuda.stream(s):
                    if form == "fused":
                        v.launch_batch(table, n, results=res, d_tune=dtune, stream=s)
                    else:
                        v.launch_per_op(table, n, results=res, d_tune=dtune, stream=s)
                s.synchronize()
                _check(v, download(wl.heap_bytes), ref, res, wl, descs)
            for gform in (0, 1):
                g = v.Graph(table, n, gform, results=res, d_tune=dtune)
                for rep in range(3):   # replays with eager work and synchronisation between them
                    upload(wl.init)
                    res.zero_()
                    t.cuda.synchronize()
                    g.launch(stream=s)
                    s.synchronize()
                    _check(v, download(wl.heap_bytes), ref, res, wl, descs)
                g.destroy()
            assert_no_device_errors(), tname


def test_graph_replays_the_table_as_rewritten():
    """A fused graph captured once replays whatever the table holds: a
    kernel rewrites it with another program between replays."""
    t = torch()
    with heap(4, 2 << 20) as v:
        progs = [_program(W.SEED_SMALL + k, n_rma=300, n_amo=1000, fences=10) for k in range(3)]
        n = max(len(d) for _, d in progs)
        table = t.zeros(n * 64, dtype=t.uint8, device="cuda")
        res = t.zeros(n, dtype=t.int64, device="cuda")
        g = v.Graph(table, n, 1, results=res)
        for wl, descs in progs:
            pad = np.zeros(n - len(descs), dtype=W.DESC_DTYPE)        # NOP records
            full = np.concatenate([descs, pad])
            write_table(full, out=table)
            upload(wl.init)
            res.zero_()
            t.cuda.synchronize()
            g.launch()
            t.cuda.synchronize()
            ref = wl.init.copy()
            oracle.run_program(ref, descs, nresults=wl.n_amo)
            _check(v, download(wl.heap_bytes), ref, res, wl, descs)
        g.destroy()
        assert_no_device_errors()


def test_invalid_descriptors_are_skipped_and_reported():
    t = torch()
    with heap(4, 2 << 20) as v:
        wl, descs = _program(W.SEED_SMALL + 7, n_rma=200, n_amo=500, fences=5)
        n = len(descs) + 5
        ub = v.heap_user_bytes()
        bad = W.descs([
            (W.OP_PUT, W.SCOPE_AUTO, 0, 0, 1, W.NO_RESULT, 0, ub - 4, 8, 0, 0),           # past the user heap
            (W.OP_WAIT_UNTIL, W.SCOPE_THREAD, 0, 1, 1, W.NO_RESULT, 0, 0, 8, 1, 0),       # not in batches
            (200, W.SCOPE_THREAD, 0, 2, 2, W.NO_RESULT, 0, 0, 8, 0, 0),                   # unknown op code
            (W.OP_AMO_FETCH_ADD, W.SCOPE_THREAD, 0, 3, 0, n, wl.counter_off, 0, 8, 1, 0),  # result index >= n
            (W.OP_GET, W.SCOPE_AUTO, 0, 1, 4, W.NO_RESULT, 0, 0, 64, 0, 0),               # target PE 4 of 4
        ])
        mixed = np.concatenate([descs[:50], bad[:2], descs[50:400], bad[2:], descs[400:]])
        assert len(mixed) == n
        table = write_table(mixed)
        res = t.zeros(n, dtype=t.int64, device="cuda")
        ref = wl.init.copy()
        oracle.run_program(ref, descs, nresults=wl.n_amo)
        for form in ("fused", "per_op"):
            upload(wl.init)
            res.zero_()
            (v.launch_batch if form == "fused" else v.launch_per_op)(table, n, results=res)
            t.cuda.synchronize()
            assert np.array_equal(download(wl.heap_bytes), ref), form
            assert v.device_errors() & v.DEVERR_BAD_DESC, form
        # Programs with unequal barrier counts run nothing.
        extra = W.descs([(W.OP_BARRIER_ALL, W.SCOPE_WG, 0, 0, 0, W.NO_RESULT, 0, 0, 0, 0, 0)])
        uneven = np.concatenate([descs, extra])
        table = write_table(uneven)
        upload(wl.init)
        v.launch_batch(table, len(uneven), results=res)
        t.cuda.synchronize()
        assert np.array_equal(download(wl.heap_bytes), wl.init)
        assert v.device_errors() & v.DEVERR_BAD_DESC


def test_two_plans_on_two_streams_keep_their_barriers_apart():
    """Multi-phase fused plans launched together on two streams: each plan
    has its own barrier words, so both equal the oracle.  Each plan's grid is
    capped so that the two fit the device together."""
    t = torch()
    with heap(4, 2 << 20) as v:
        half = 512 << 10
        progs = [_program(W.SEED_SMALL + 20 + k, heap_bytes=half, base_off=k * half, n_rma=400, n_amo=1000)
                 for k in range(2)]
        init = np.concatenate([progs[0][0].init, progs[1][0].init], axis=1)
        ref = init.copy()
        for wl, descs in progs:
            oracle.run_program(ref, descs, nresults=wl.n_amo)
        tune = v.default_tune()
        tune.grid_wgs = 32
        plans = [v.Plan(d, tune) for _, d in progs]
        assert all(p.info()["phases"] > 3 for p in plans)
        streams = [t.cuda.Stream(), t.cuda.Stream()]
        res = [t.zeros(len(d), dtype=t.int64, device="cuda") for _, d in progs]
        for rep in range(4):
            upload(init)
            for r in res:
                r.zero_()
            t.cuda.synchronize()
            for p, s, r in zip(plans, streams, res):
                p.launch_fused(results=r, stream=s)
            t.cuda.synchronize()
            got = download(2 * half)
            for k, (wl, descs) in enumerate(progs):
                lo, hi = k * half, (k + 1) * half
                _check(v, got[:, lo:hi], ref[:, lo:hi], res[k], wl, descs)
        for p in plans:
            p.destroy()
        assert_no_device_errors()


def test_tune_file_at_init_and_tune_set(tmp_path, monkeypatch):
    import json
    path = str(tmp_path / "tune.json")
    with heap(2, 2 << 20) as v:
        t0, src = v.tune_get()
        assert src == v.TUNE_SRC_DEFAULT and t0.wg_size == v.default_tune().wg_size
        t0.wg_size = 512
        t0.scope[10] = v.SCOPE_WG
        v.tune_save(t0, path)
    monkeypatch.setenv("VSHMEM_TUNE_FILE", path)
    with heap(2, 2 << 20) as v:
        t1, src = v.tune_get()
        assert src == v.TUNE_SRC_FILE and t1.wg_size == 512 and t1.scope[10] == v.SCOPE_WG
        v.tune_set(v.default_tune())
        t2, src = v.tune_get()
        assert src == v.TUNE_SRC_SET and t2.wg_size == v.default_tune().wg_size
        bad = v.default_tune()
        bad.wg_size = 96
        with pytest.raises(v.VshmemError):
            v.tune_set(bad)
    d = json.load(open(path))
    d["device"] = "gfx000:not-this-one"
    json.dump(d, open(path, "w"))
    with heap(2, 2 << 20) as v:
        t3, src = v.tune_get()
        assert src == v.TUNE_SRC_FILE_REFUSED and t3.wg_size == v.default_tune().wg_size


def test_signal_puts_and_every_amo_kind_from_a_device_table():
    """Signal-puts at three scopes and every atomic kind, with a fence and a
    quiet splitting the issuer's program, through the fused, per-op and
    graph forms over a kernel-written table: signals after their data, one
    compare-swap winner, and every other word and fetched value as the
    oracle's."""
    t = torch()
    npes = 3
    with heap(npes, 1 << 20) as v:
        init = W.heap_fill(77, npes, 8192)
        init[:, 4096:4096 + 256] = 0
        recs = [
            (W.OP_PUT_SIGNAL, W.SCOPE_WG, W.SIGNAL_SET, 0, 1, W.NO_RESULT, 0, 1024, 500, 7, 4096),
            (W.OP_PUT_SIGNAL, W.SCOPE_WAVE, W.SIGNAL_ADD, 1, 2, W.NO_RESULT, 64, 2048, 300, 5, 4104),
            (W.OP_PUT_SIGNAL, W.SCOPE_THREAD, W.SIGNAL_ADD, 2, 2, W.NO_RESULT, 128, 3000, 100, 11, 4104),
            (W.OP_AMO_COMPARE_SWAP, W.SCOPE_THREAD, 0, 0, 0, 0, 4160, 0, 8, 9, 0),
            (W.OP_AMO_COMPARE_SWAP, W.SCOPE_THREAD, 0, 1, 0, 1, 4160, 0, 8, 10, 0),
            (W.OP_AMO_COMPARE_SWAP, W.SCOPE_THREAD, 0, 2, 0, 2, 4160, 0, 8, 11, 0),
            (W.OP_AMO_SET, W.SCOPE_THREAD, 0, 0, 1, W.NO_RESULT, 4168, 0, 8, 42, 0),
            (W.OP_AMO_XOR, W.SCOPE_THREAD, 0, 1, 2, W.NO_RESULT, 4176, 0, 8, 0xF0F0, 0),
            (W.OP_AMO_ADD, W.SCOPE_THREAD, 0, 2, 2, W.NO_RESULT, 4184, 0, 8, (1 << 64) - 3, 0),
            (W.OP_AMO_FETCH_XOR, W.SCOPE_WAVE, 0, 1, 0, 5, 4192, 0, 8, 0x55, 0),
            (W.OP_FENCE, 0, 0, 0, 0, W.NO_RESULT, 0, 0, 0, 0, 0),
            (W.OP_AMO_SWAP, W.SCOPE_THREAD, 0, 0, 1, 3, 4168, 0, 8, 99, 0),
            (W.OP_QUIET, 0, 0, 0, 0, W.NO_RESULT, 0, 0, 0, 0, 0),
            (W.OP_AMO_FETCH, W.SCOPE_THREAD, 0, 0, 1, 4, 4168, 0, 8, 0, 0),
        ]
        d = W.descs(recs)
        n = len(d)
        table = write_table(d)
        ref = init.copy()
        ref_r = oracle.run_program(ref, d, nresults=6)
        res = t.zeros(n, dtype=t.int64, device="cuda")
        runs = {"fused": lambda: v.launch_batch(table, n, results=res),
                "per_op": lambda: v.launch_per_op(table, n, results=res)}
        graphs = {f"graph{f}": v.Graph(table, n, f, results=res) for f in (0, 1)}
        runs.update({k: g.launch for k, g in graphs.items()})
        for name, run in runs.items():
            upload(init)
            res.zero_()
            t.cuda.synchronize()
            run()
            t.cuda.synchronize()
            got = download(8192)
            r = res.cpu().numpy().view(np.uint64)
            cas = got[0, 4160:4168].view(np.uint64)[0]
            winners = [i for i in range(3) if r[i] == 0]
            assert len(winners) == 1 and cas == 9 + winners[0], name
            assert all(r[i] == cas for i in range(3) if i not in winners), name
            mask = np.ones_like(got, dtype=bool)
            mask[0, 4160:4168] = False
            assert np.array_equal(got[mask], ref[mask]), name
            assert r[3] == ref_r[3] == 42 and r[4] == ref_r[4] == 99 and r[5] == ref_r[5], name
        for g in graphs.values():
            g.destroy()
        assert_no_device_errors()


def _long_program(npes, epochs, fences):
    """`epochs` barrier epochs (puts at three scopes in some of them, each
    rewriting the same destination slots), then one epoch whose issuers
    alternate put, fetch_add and fence `fences` times: every phase rewrites
    the slots and bumps a counter only its issuer touches, so the final bytes
    and every fetched value depend on the phases running in order."""
    heap_bytes = 1 << 19
    init = W.heap_fill(91, npes, heap_bytes)
    recs = []
    for e in range(epochs):
        for p in range(npes):
            recs.append((W.OP_BARRIER_ALL, W.SCOPE_WG, 0, p, p, W.NO_RESULT, 0, 0, 0, 0, 0))
        if e % 97 == 0 or 4090 <= e < 4110:
            for p in range(npes):
                scope = (W.SCOPE_THREAD, W.SCOPE_WAVE, W.SCOPE_WG)[e % 3]
                recs.append((W.OP_PUT, scope, 0, p, (p + 1) % npes, W.NO_RESULT, 4096 + 8 * (e % 500),
                             65536 + 64 * p, 64, 0, 0))
    nres = 0
    for f in range(fences):
        for p in range(npes):
            q = (p + 1) % npes
            scope = (W.SCOPE_WAVE, W.SCOPE_WG, W.SCOPE_THREAD)[(f + p) % 3]
            recs.append((W.OP_PUT, scope, 0, p, q, W.NO_RESULT, 8192 + 8 * (f % 1000), 131072 + 64 * p, 64, 0, 0))
            recs.append((W.OP_AMO_FETCH_ADD, W.SCOPE_THREAD, 0, p, q, nres, 262144 + 8 * p, 0, 8, 1 + f, 0))
            recs.append((W.OP_FENCE, 0, 0, p, 0, W.NO_RESULT, 0, 0, 0, 0, 0))
            nres += 1
    return init, W.descs(recs), nres


@pytest.mark.parametrize("epochs,fences", [(4200, 3000), (3, 2000), (5000, 10)])
def test_long_programs_past_the_index_kernels_lds_counters(epochs, fences):
    """Tables of 10k-27k descriptors over several index tiles: 4200 epochs
    and 7200 phases put the epoch and bucket counters in memory; 2000 fences
    in one epoch keep them in LDS; 5000 epochs with few operations put the
    counters in memory in a table of two index tiles.  Fused, no-allocation,
    fused-graph and per-op forms against the oracle, bytes and every fetched
    value."""
    t = torch()
    npes = 2
    with heap(npes, 1 << 20) as v:
        init, d, nres = _long_program(npes, epochs, fences)
        n = len(d)
        assert n <= v.launch_batch_noalloc_max()
        table = write_table(d)
        ref = init.copy()
        ref_r = oracle.run_program(ref, d, nresults=nres)
        res = t.zeros(n, dtype=t.int64, device="cuda")
        g = v.Graph(table, n, 0, results=res)
        runs = {"fused": lambda: v.launch_batch(table, n, results=res),
                "noalloc": lambda: v.launch_batch_noalloc(table, n, results=res),
                "graph0": g.launch,
                "per_op": lambda: v.launch_per_op(table, n, results=res)}
        for name, run in runs.items():
            upload(init)
            res.zero_()
            t.cuda.synchronize()
            run()
            t.cuda.synchronize()
            got = download(init.shape[1])
            assert np.array_equal(got, ref), name
            assert np.array_equal(res.cpu().numpy().view(np.uint64)[:nres], ref_r), name
        g.destroy()
        assert_no_device_errors()


def test_many_issuers_from_a_device_table():
    """256 PEs: every epoch ends with 256 barrier descriptors (sub-tiles made
    of ordering points of many issuers), 200 fences at seeded places, and
    3000 fetch_add spread over every issuer; fused form against the oracle,
    bytes and the counters' fetched values."""
    t = torch()
    npes = 256
    with heap(npes, 1 << 20) as v:
        wl, descs = _program(W.SEED_SMALL + 11, npes=npes, n_rma=1200, n_amo=3000, fences=200)
        n = len(descs)
        table = write_table(descs)
        ref = wl.init.copy()
        oracle.run_program(ref, descs, nresults=wl.n_amo)
        res = t.zeros(n, dtype=t.int64, device="cuda")
        for run in (lambda: v.launch_batch(table, n, results=res),
                    lambda: v.launch_batch_noalloc(table, n, results=res)):
            upload(wl.init)
            res.zero_()
            t.cuda.synchronize()
            run()
            t.cuda.synchronize()
            _check(v, download(wl.heap_bytes), ref, res, wl, descs)
        assert_no_device_errors()


def test_degenerate_tables():
    """An empty table, a table of one put, a table of ordering points only,
    and zero-byte operations (one ending exactly at the user heap's end)
    between NOPs: each runs in the fused, no-allocation and per-op forms,
    changes exactly what the oracle changes, and latches no error."""
    t = torch()
    npes, region = 4, 64 << 10
    with heap(npes, 1 << 20) as v:
        ub = v.heap_user_bytes()
        init = W.heap_fill(0xDE6, npes, region)
        res = t.zeros(4, dtype=t.int64, device="cuda")
        one_put = W.descs([(W.OP_PUT, W.SCOPE_AUTO, 0, 2, 1, W.NO_RESULT, 128, 40000, 1000, 0, 0)])
        order_only = W.descs([(W.OP_FENCE, W.SCOPE_THREAD, 0, 0, 0, W.NO_RESULT, 0, 0, 0, 0, 0)] +
                             [(W.OP_BARRIER_ALL, W.SCOPE_WG, 0, p, p, W.NO_RESULT, 0, 0, 0, 0, 0)
                              for p in range(npes)] +
                             [(W.OP_QUIET, W.SCOPE_THREAD, 0, 3, 3, W.NO_RESULT, 0, 0, 0, 0, 0)])
        zero = W.descs([(W.OP_NOP, W.SCOPE_THREAD, 0, 0, 0, W.NO_RESULT, 0, 0, 0, 0, 0),
                        (W.OP_PUT, W.SCOPE_THREAD, 0, 0, 1, W.NO_RESULT, ub, ub, 0, 0, 0),
                        (W.OP_GET, W.SCOPE_WG, 0, 1, 2, W.NO_RESULT, 64, 4096, 0, 0, 0),
                        (W.OP_NOP, W.SCOPE_THREAD, 0, 3, 3, W.NO_RESULT, 0, 0, 0, 0, 0),
                        (W.OP_PUT, W.SCOPE_WAVE, 0, 3, 0, W.NO_RESULT, 8, 50000, 24, 0, 0)])
        cases = {"empty": W.descs([]), "one_put": one_put, "ordering_only": order_only, "zero_bytes": zero}
        for name, d in cases.items():
            n = len(d)
            table = write_table(d)
            ref = init.copy()
            if name != "zero_bytes":
                oracle.run_program(ref, d)
            else:
                # the zero-byte operations change nothing; the last put moves 24 bytes
                oracle.run_program(ref, d[-1:])
            runs = {"fused": lambda: v.launch_batch(table, n, results=res),
                    "noalloc": lambda: v.launch_batch_noalloc(table, n, results=res),
                    "per_op": lambda: v.launch_per_op(table, n, results=res)}
            for form, run in runs.items():
                upload(init)
                run()
                t.cuda.synchronize()
                assert np.array_equal(download(region), ref), (name, form)
                assert_no_device_errors()
