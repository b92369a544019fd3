"""GPU parity: device-initiated put/get at every scope and the batched plan
forms, bit-exact against the CPU oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, device_array, download, heap, upload

pytestmark = pytest.mark.gpu

SCOPES = [W.SCOPE_THREAD, W.SCOPE_WAVE, W.SCOPE_WG, W.SCOPE_GRID]


def _pattern_descs(op, targets, src_off, dst_off, msg, nmsg, ss, ds):
    recs = []
    for p, t in enumerate(targets):
        if t < 0:
            continue
        for j in range(nmsg):
            recs.append((op, W.SCOPE_THREAD, 0, p, int(t), W.NO_RESULT, src_off + j * ss, dst_off + j * ds, msg, 0, 0))
    return W.descs(recs)


@pytest.mark.parametrize("scope", SCOPES)
def test_pattern_put_get_bit_exact(scope):
    npes, user = 6, 1 << 20
    with heap(npes, user) as v:
        region = 600 << 10
        init = W.heap_fill(0x1234 + scope, npes, region)
        cases = [
            # (op, pattern, msg, nmsg, src_off, dst_off, step)
            (W.OP_PUT, "ring", 1, 5, 0, 300 << 10, 8),
            (W.OP_GET, "perm", 8, 33, 8, 300 << 10, 8),
            (W.OP_PUT, "perm", 24, 7, 16, (300 << 10) + 8, 40),
            (W.OP_GET, "ring", 4136, 9, 0, 300 << 10, 4136),            # ragged tail
            (W.OP_PUT, "ring", 65544, 3, 24, (300 << 10) + 16, 65552),  # several tiles + tail
            (W.OP_PUT, "perm", 1000, 4, 3, (300 << 10) + 5, 1001),      # byte-misaligned
            (W.OP_GET, "perm", 777, 4, 4, (300 << 10) + 2, 800),        # 4- and 2-byte phases
        ]
        for op, pat, msg, nmsg, so, do, step in cases:
            targets = W.pattern_targets(pat, npes, seed=W.SEED_SWEEP + scope).astype(np.int32)
            upload(init)
            launch = v.launch_cfg(wgs_per_pe=3, wg_size=128)
            v.rma_pattern(op, scope, device_array(targets), so, do, msg, nmsg, step, step, launch=launch)
            got = download(region)
            ref = init.copy()
            oracle.run_program(ref, _pattern_descs(op, targets, so, do, msg, nmsg, step, step))
            assert np.array_equal(got, ref), (op, pat, msg, nmsg, scope)
        assert_no_device_errors()


def test_thread_scope_message_runs():
    """One lane per message, more messages than lanes: the lane moves its
    messages four at a time (16- and 8-byte elements, one or two per
    message) and the rest one by one; other sizes and alignments take the
    generic copy, whose edges a lone lane moves in wide pieces."""
    npes, user = 5, 1 << 20
    K = 300 << 10
    with heap(npes, user) as v:
        region = 600 << 10
        init = W.heap_fill(0x3A7, npes, region)
        cases = [
            # (op, msg, nmsg, src_off, dst_off, src_step, dst_step)
            (W.OP_PUT, 16, 4 * 64 * 3 + 17, 0, K, 16, 16),
            (W.OP_GET, 64, 4 * 64 + 63, 64, K, 80, 80),
            (W.OP_PUT, 48, 4 * 64 * 2 + 1, 16, K + 32, 48, 48),
            (W.OP_GET, 8, 4 * 64 * 5 + 7, 8, K, 8, 8),
            (W.OP_PUT, 24, 4 * 64 + 5, 8, K + 8, 24, 24),
            (W.OP_PUT, 32, 4 * 64 + 100, 8, K, 40, 40),
            (W.OP_PUT, 16, 4 * 64 * 2 + 9, 32, K, 0, 16),     # every message reads one source
            (W.OP_GET, 72, 300, 0, K, 72, 72),                # above 64 bytes: generic
            (W.OP_PUT, 12, 600, 4, K + 4, 12, 12),            # 4-byte aligned: generic, 2- and 4-byte edges
            (W.OP_PUT, 8, 4 * 64 + 3, 4, K + 4, 8, 8),        # 8 bytes, 4-aligned: generic
            (W.OP_PUT, 7, 500, 1, K + 3, 9, 9),               # byte path
            (W.OP_GET, 15, 700, 1, K + 1, 16, 16),            # 1-, 2-, 4- and 8-byte head pieces
        ]
        shapes = [v.launch_cfg(wgs_per_pe=1, wg_size=64),
                  v.launch_cfg(wgs_per_pe=2, wg_size=128, flags=v.LAUNCH_NONTEMPORAL | v.LAUNCH_DEEP),
                  v.launch_cfg(wgs_per_pe=1, wg_size=1024)]
        for li, launch in enumerate(shapes):
            for ci, (op, msg, nmsg, so, do, ss, ds) in enumerate(cases):
                targets = W.pattern_targets("perm" if ci % 2 else "ring", npes, seed=W.SEED_SWEEP + ci).astype(np.int32)
                upload(init)
                v.rma_pattern(op, W.SCOPE_THREAD, device_array(targets), so, do, msg, nmsg, ss, ds, launch=launch)
                got = download(region)
                ref = init.copy()
                oracle.run_program(ref, _pattern_descs(op, targets, so, do, msg, nmsg, ss, ds))
                assert np.array_equal(got, ref), (li, op, msg, nmsg, so, do, ss, ds)
        assert_no_device_errors()


def test_pattern_idle_pes_and_arg_checks():
    npes = 4
    with heap(npes, 1 << 20) as v:
        init = W.heap_fill(5, npes, 1 << 19)
        upload(init)
        targets = np.array([1, -1, 3, -1], dtype=np.int32)
        v.rma_pattern(W.OP_PUT, W.SCOPE_WG, device_array(targets), 0, 1 << 18, 4096, 4)
        got = download(1 << 19)
        ref = init.copy()
        oracle.run_program(ref, _pattern_descs(W.OP_PUT, targets, 0, 1 << 18, 4096, 4, 4096, 4096))
        assert np.array_equal(got, ref)
        # out-of-heap ranges and overlapping destination steps are refused on the host
        with pytest.raises(v.VshmemError):
            v.rma_pattern(W.OP_PUT, W.SCOPE_WG, device_array(targets), 0, v.heap_user_bytes() - 8, 64, 1)
        with pytest.raises(v.VshmemError):
            v.rma_pattern(W.OP_PUT, W.SCOPE_WG, device_array(targets), 0, 0, 64, 4, 64, 32)


def _small(**kw):
    return W.small_workload(**kw)


def _check_small(wl, got, fetched):
    ref = wl.init.copy()
    ref_res = oracle.run_program(ref, wl.descs, nresults=wl.n_amo, check=True)
    assert np.array_equal(got[:, :wl.data_bytes], ref[:, :wl.data_bytes])
    # counters: the same final values; fetched values are a valid history
    c0, c1 = wl.counter_off, wl.counter_off + 8 * wl.ncounters
    assert np.array_equal(got[:, c0:c1], ref[:, c0:c1])
    amo = wl.descs[wl.descs["op"] == W.OP_AMO_FETCH_ADD]
    word = ((amo["target"].astype(np.int64) * wl.ncounters) + (amo["src"].astype(np.int64) - c0) // 8).astype(np.uint64)
    init_w = np.zeros(wl.npes * wl.ncounters, dtype=np.uint64)
    final_w = got[:, c0:c1].copy().view(np.uint64).reshape(-1)
    kind = np.zeros(len(amo), dtype=np.uint8)
    assert oracle.witness_check(word, kind, amo["value"], fetched, init_w, final_w) == 0
    assert sorted(ref_res.tolist()) == sorted(fetched.tolist())


@pytest.mark.parametrize("form", ["fused", "per_op", "graph_per_op", "graph_fused"])
def test_small_workload_all_forms(form):
    wl = _small()
    with heap(wl.npes, wl.heap_bytes) as v:
        t = __import__("torch")
        res = t.zeros(wl.n_amo, dtype=t.int64, device="cuda")
        plan = v.Plan(wl.descs)
        info = plan.info()
        assert info["phases"] >= 9
        if form.startswith("graph"):
            plan.graph_build(0 if form == "graph_per_op" else 1, results=res)
        reps = 3 if form.startswith("graph") else 1
        for _ in range(reps):
            upload(wl.init)
            res.zero_()
            t.cuda.synchronize()
            if form == "fused":
                plan.launch_fused(results=res)
            elif form == "per_op":
                plan.launch_per_op(results=res)
            else:
                plan.graph_launch()
            got = download(wl.heap_bytes)
            fetched = res.cpu().numpy().view(np.uint64).copy()
            _check_small(wl, got, fetched)
        plan.destroy()
        assert_no_device_errors()


@pytest.mark.parametrize("scope", [W.SCOPE_THREAD, W.SCOPE_WAVE, W.SCOPE_WG, W.SCOPE_GRID])
def test_small_workload_each_scope(scope):
    wl = _small(n_rma=400, epoch_ops=100, n_amo=3000, scope=scope)
    with heap(wl.npes, wl.heap_bytes) as v:
        t = __import__("torch")
        res = t.zeros(wl.n_amo, dtype=t.int64, device="cuda")
        tune = v.default_tune()
        for c in range(40):
            tune.chunk[c] = 1024     # split work-group messages into several tasks
        plan = v.Plan(wl.descs, tune)
        upload(wl.init)
        plan.launch_fused(results=res)
        got = download(wl.heap_bytes)
        _check_small(wl, got, res.cpu().numpy().view(np.uint64).copy())


def test_put_signal_and_amo_kinds_in_plans():
    npes = 3
    with heap(npes, 1 << 20) as v:
        t = __import__("torch")
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
            (W.OP_FENCE, 0, 0, 0, 0, W.NO_RESULT, 0, 0, 0, 0, 0),
            (W.OP_AMO_SWAP, W.SCOPE_THREAD, 0, 0, 1, 3, 4168, 0, 8, 99, 0),
            (W.OP_QUIET, 0, 0, 0, 0, W.NO_RESULT, 0, 0, 0, 0, 0),
            (W.OP_AMO_FETCH, W.SCOPE_THREAD, 0, 0, 1, 4, 4168, 0, 8, 0, 0),
        ]
        d = W.descs(recs)
        upload(init)
        res = t.zeros(8, dtype=t.int64, device="cuda")
        plan = v.Plan(d)
        assert plan.info()["phases"] == 3
        plan.launch_fused(results=res)
        got = download(8192)
        r = res.cpu().numpy().view(np.uint64)
        ref = init.copy()
        ref_r = oracle.run_program(ref, d, nresults=5)
        cas_pe0 = got[0, 4160:4168].view(np.uint64)[0]
        winners = [i for i in range(3) if r[i] == 0]
        assert len(winners) == 1 and cas_pe0 == 9 + winners[0]
        assert all(r[i] == cas_pe0 for i in range(3) if i not in winners)
        mask = np.ones_like(got, dtype=bool)
        mask[0, 4160:4168] = False
        assert np.array_equal(got[mask], ref[mask])
        assert r[3] == ref_r[3] == 42 and r[4] == ref_r[4] == 99
        plan.destroy()


def test_plan_rejects_bad_programs():
    with heap(2, 1 << 20) as v:
        bad_range = W.descs([(W.OP_PUT, 0, 0, 0, 1, W.NO_RESULT, 0, v.heap_user_bytes() - 4, 8, 0, 0)])
        with pytest.raises(v.VshmemError):
            v.Plan(bad_range)
        wait = W.descs([(W.OP_WAIT_UNTIL, 0, 0, 0, 0, W.NO_RESULT, 0, 0, 0, 1, 0)])
        with pytest.raises(v.VshmemError) as e:
            v.Plan(wait)
        assert e.value.code == v.ERR_UNSUPPORTED
        unequal = W.descs([(W.OP_BARRIER_ALL, 0, 0, 0, 0, W.NO_RESULT, 0, 0, 0, 0, 0)])
        with pytest.raises(v.VshmemError):
            v.Plan(unequal)


def test_heap_allocator_symmetry_and_queries():
    with heap(4, 4 << 20) as v:
        a = v.malloc(1000)
        b = v.shmemg_malloc(3 << 20)
        assert v.offset(a) == 0 and v.offset(b) == 1024
        assert v.offset(a) % 256 == 0
        c = v.align(1 << 16, 100)
        assert v.offset(c) % (1 << 16) == 0
        v.free(b)
        d = v.malloc(2048)
        assert v.offset(d) == 1024            # first fit reuses the freed hole
        with pytest.raises(v.VshmemError):
            v.malloc(1 << 40)
        assert v.ptr(a, 3) == a + 3 * v.heap_stride()
        assert v.ptr(a, 4) is None
        z = v.calloc(64, 8)
        h = download(v.offset(z) + 512)
        assert not h[:, v.offset(z):v.offset(z) + 512].any()
        caps = v.query_capabilities(v.DEVICE_TEAM_WORLD)
        assert caps["gpu_heap"] == 1 and caps["device_initiated"] == 1 and caps["stream_triggered"] == 1 and caps["host_initiated"] == 1
        assert caps["npes"] == 4 and caps["team_npes"] == 4 and caps["ptr_domain"] == 2
        tm = v.team_split_strided(v.DEVICE_TEAM_WORLD, 1, 2, 2)
        assert v.query_capabilities(tm)["team_start"] == 1 and v.team_n_pes(tm) == 2
        v.team_destroy(tm)


def test_device_input_generators_match_workload():
    t = torch_mod = __import__("torch")
    import paper_2607_08006_amd as v
    n = 100_003
    buf = t.zeros(n * 8 + 16, dtype=t.uint8, device="cuda")
    v.fill_random(buf, 1001, 0xABCDEF, word_offset=7)
    assert np.array_equal(buf[:1001].cpu().numpy(), W.payload(0xABCDEF, 56, 1001))
    v.fill_typed(buf, n, v.DT_INT64, 42, index0=5)
    assert np.array_equal(buf[:8 * n].cpu().numpy().view(np.uint64), W.splitmix64(42, 5, n))
    v.fill_typed(buf, n, v.DT_FP32, 43)
    assert np.array_equal(buf[:4 * n].cpu().numpy().view(np.float32), W.uniform_f32(W.splitmix64(43, 0, n)))
    v.fill_typed(buf, n, v.DT_BF16, 44)
    assert np.array_equal(buf[:2 * n].cpu().numpy().view(np.uint16),
                          W.f32_to_bf16_bits(W.uniform_f32(W.splitmix64(44, 0, n))))
    torch_mod.cuda.synchronize()


def test_autotune_table_drives_plans_and_stays_exact(tmp_path):
    wl = W.small_workload(n_rma=300, epoch_ops=100, n_amo=2000)
    with heap(wl.npes, 8 << 20) as v:
        t = __import__("torch")
        scratch = v.offset(v.malloc(4 << 20)) + (2 << 20)      # beyond the workload's 1 MiB window
        tune = v.autotune(scratch, 2 << 20, 64, 256 << 10, msgs=64, reps=2)
        assert tune.wg_size in (64, 128, 256, 512, 1024)
        for c in range(6, 19):
            assert tune.scope[c] in (v.SCOPE_THREAD, v.SCOPE_WAVE, v.SCOPE_WG)
        path = str(tmp_path / "tune.json")
        v.tune_save(tune, path)
        tune2 = v.tune_load(path)
        assert list(tune2.scope) == list(tune.scope) and tune2.wg_size == tune.wg_size
        res = t.zeros(wl.n_amo, dtype=t.int64, device="cuda")
        plan = v.Plan(wl.descs, tune2)
        upload(wl.init)
        plan.launch_fused(results=res)
        got = download(wl.heap_bytes)
        _check_small(wl, got, res.cpu().numpy().view(np.uint64).copy())
        plan.destroy()
