"""GPU parity: the header-only device API called from user-style kernels
(tests/devapi/user_kernels.hip, built into its own library that does not link
libvshmem.so).  Collectives at work-group and grid scope, several of them
chained in one kernel, and team barriers at thread, wavefront and work-group
scope, checked against the CPU oracle bit for bit."""
import ctypes

import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, download, heap, torch, upload, user_lib

pytestmark = pytest.mark.gpu

BROADCAST, FCOLLECT, ALLTOALL, REDUCE = 0, 1, 2, 3
ES = {oracle.DT_INT64: 8, oracle.DT_FP32: 4, oracle.DT_BF16: 2}
_lib = user_lib


def _collective(lib, v, team, kind, dest, src, n, root=0, dt=0, rop=0, nwgs=1, wg=256, expect=0):
    t = torch()
    dteam = v.team_device(team)
    status = t.full((dteam.size * nwgs,), 12345, dtype=t.int32, device="cuda")
    rc = lib.usertest_collective(v.device_ctx(), ctypes.byref(dteam), kind, dt, rop, dest, src, n, root, nwgs, wg,
                                 status.data_ptr(), None)
    assert rc == 0
    t.cuda.synchronize()
    assert (status.cpu().numpy() == expect).all(), (kind, status.cpu().numpy()[:8])


def _red_inputs(dt, npes, nreduce, seed):
    gen = {oracle.DT_INT64: W.coll_i64, oracle.DT_FP32: W.coll_f32, oracle.DT_BF16: W.coll_bf16}[dt]
    return np.stack([gen(seed, p, nreduce).view(np.uint8) for p in range(npes)])


@pytest.mark.parametrize("npes,team_args", [(1, None), (3, None), (8, None), (9, (1, 2, 4))])
def test_user_kernel_data_movement(npes, team_args):
    lib = _lib()
    with heap(npes, 4 << 20) as v:
        team = v.TEAM_WORLD if team_args is None else v.team_split_strided(v.TEAM_WORLD, *team_args)
        members = team_args   # the oracle takes a team as (start, stride, size)
        tsize = v.team_n_pes(team)
        src = v.malloc(1 << 20)
        dst = v.malloc(2 << 20)
        so, do = v.offset(src), v.offset(dst)
        region = do + (2 << 20)
        init = W.heap_fill(W.SEED_COLL + 77 * npes, npes, region)
        for nwgs in (1, 3):
            for n in (1, 40, 4096 + 24, 300_007):
                root = (n + nwgs) % tsize
                upload(init)
                _collective(lib, v, team, BROADCAST, dst, src, n, root=root, nwgs=nwgs)
                ref = init.copy()
                oracle.broadcast(ref, do, so, n, root, team=members)
                assert np.array_equal(download(region), ref), ("broadcast", n, nwgs)
                if n * tsize > (1 << 20):
                    continue
                upload(init)
                _collective(lib, v, team, FCOLLECT, dst, src, n, nwgs=nwgs)
                ref = init.copy()
                oracle.fcollect(ref, do, so, n, team=members)
                assert np.array_equal(download(region), ref), ("fcollect", n, nwgs)
                upload(init)
                _collective(lib, v, team, ALLTOALL, dst, src, n, nwgs=nwgs)
                ref = init.copy()
                oracle.alltoall(ref, do, so, n, team=members)
                assert np.array_equal(download(region), ref), ("alltoall", n, nwgs)
        assert_no_device_errors()


@pytest.mark.parametrize("dt", [oracle.DT_INT64, oracle.DT_FP32, oracle.DT_BF16])
def test_user_kernel_reductions(dt):
    lib = _lib()
    es = ES[dt]
    for npes in (1, 5, 13):
        with heap(npes, 2 << 20) as v:
            nmax = 40_003
            src = v.malloc(nmax * es)
            dst = v.malloc(nmax * es)
            so, do = v.offset(src), v.offset(dst)
            region = do + nmax * es
            for nreduce in (1, 1001, nmax):
                init = np.zeros((npes, region), dtype=np.uint8)
                init[:, so:so + nreduce * es] = _red_inputs(dt, npes, nreduce, 31 * npes + nreduce)
                for rop in (oracle.RO_SUM, oracle.RO_MAX):
                    for nwgs, wg in ((1, 64), (2, 256)):
                        upload(init)
                        _collective(lib, v, v.TEAM_WORLD, REDUCE, dst, src, nreduce, dt=dt, rop=rop, nwgs=nwgs, wg=wg)
                        ref = init.copy()
                        oracle.reduce(ref, dt, rop, do, so, nreduce)
                        assert np.array_equal(download(region), ref), (dt, rop, npes, nreduce, nwgs)
            assert_no_device_errors()


def test_user_kernel_reduction_rejects_teams_of_512():
    """The TREE fold keeps 9 levels: a team of 512 members is refused by every
    caller, before any barrier, and nothing is written."""
    lib = _lib()
    npes = 512
    with heap(npes, 2 << 20) as v:
        src = v.malloc(4096)
        dst = v.malloc(4096)
        region = v.offset(dst) + 4096
        init = W.heap_fill(5, npes, region)
        upload(init)
        _collective(lib, v, v.TEAM_WORLD, REDUCE, dst, src, 512, dt=oracle.DT_INT64, rop=oracle.RO_SUM, wg=64,
                    expect=v.ERR_UNSUPPORTED)
        assert np.array_equal(download(region), init)
        assert_no_device_errors()


def test_user_kernel_chains_collectives_with_compute():
    """One launch: scale the local input, sum-reduce it over the team, then
    fcollect a prefix of the sums.  The oracle runs the same three steps."""
    lib = _lib()
    npes, n, m = 6, 10_007, 333
    with heap(npes, 2 << 20) as v:
        src, x, y, z = (v.malloc(n * 8), v.malloc(n * 8), v.malloc(n * 8), v.malloc(npes * m * 8))
        so, xo, yo, zo = (v.offset(a) for a in (src, x, y, z))
        region = zo + npes * m * 8
        init = W.heap_fill(W.SEED_COLL + 5, npes, region)
        init[:, so:so + n * 8] = _red_inputs(oracle.DT_INT64, npes, n, 99)
        for nwgs in (1, 4):
            upload(init)
            dteam = v.team_device(v.TEAM_WORLD)
            assert lib.usertest_pipeline(v.device_ctx(), ctypes.byref(dteam), src, x, y, z, n, m, nwgs, 256, None) == 0
            got = download(region)
            ref = init.copy()
            with np.errstate(over="ignore"):
                for p in range(npes):
                    s = ref[p, so:so + n * 8].view(np.int64)
                    ref[p, xo:xo + n * 8] = (s * np.int64(p + 1)).view(np.uint8)
            oracle.reduce(ref, oracle.DT_INT64, oracle.RO_SUM, yo, xo, n)
            oracle.fcollect(ref, zo, yo, m * 8)
            assert np.array_equal(got, ref), nwgs
        assert_no_device_errors()


@pytest.mark.parametrize("scope", [0, 1, 2])
def test_user_kernel_barriers(scope):
    """Tokens written before a barrier are seen by the next member after it,
    at thread, wavefront and work-group scope, for the world and for a
    strided team."""
    lib = _lib()
    t = torch()
    npes, iters = 12, 64
    with heap(npes, 2 << 20) as v:
        tok = v.calloc(1, 8)
        for team, world in ((v.TEAM_WORLD, 1), (v.team_split_strided(v.TEAM_WORLD, 2, 3, 3), 0)):
            upload(np.zeros((npes, v.offset(tok) + 8), dtype=np.uint8))
            bad = t.zeros(1, dtype=t.int64, device="cuda")
            dteam = v.team_device(team)
            assert lib.usertest_barrier(v.device_ctx(), ctypes.byref(dteam), scope, world, iters, tok,
                                        bad.data_ptr(), 128, None) == 0
            t.cuda.synchronize()
            assert int(bad.item()) == 0, (scope, world)
            words = download(v.offset(tok) + 8)[:, v.offset(tok):].view(np.int64)[:, 0]
            members = range(npes) if world else (2, 5, 8)
            for p in range(npes):
                assert words[p] == (iters if p in members else 0), (scope, world, p)
        assert_no_device_errors()


@pytest.mark.parametrize("team_args", [None, (2, 3, 4), (5, 1, 1)])
def test_explicit_context_numbers_pes_in_its_team(team_args):
    """An explicit device context created from a team: kernels see team
    numbering for shmem_my_pe, shmem_n_pes and every PE argument.  Puts to
    the next member and gets from the previous one follow the oracle's
    programs in world numbering; the contended fetch_add on member 0 hands
    out every old value once."""
    lib = _lib()
    t = torch()
    npes, n = 14, 3000
    with heap(npes, 2 << 20) as v:
        team = v.TEAM_WORLD if team_args is None else v.team_split_strided(v.TEAM_WORLD, *team_args)
        start, stride, size = team_args or (0, 1, npes)
        world = [start + k * stride for k in range(size)]
        ctx = v.device_ctx_create(team, v.CTX_PRIVATE)
        src, dst, back, ctr = v.malloc(n), v.malloc(n), v.malloc(n), v.calloc(1, 8)
        so, do, bo, co = (v.offset(a) for a in (src, dst, back, ctr))
        region = co + 8
        init = W.heap_fill(W.SEED_SMALL + size, npes, region)
        init[:, co:co + 8] = 0
        upload(init)
        ids = t.zeros(2 * size, dtype=t.int32, device="cuda")
        fetched = t.zeros(size, dtype=t.int64, device="cuda")
        assert lib.usertest_ctx(v.device_ctx_record(ctx), size, src, dst, back, n, ctr, ids.data_ptr(),
                                fetched.data_ptr(), 128, None) == 0
        got = download(region)
        ref = init.copy()
        oracle.run_program(ref, np.concatenate([
            W.descs([(W.OP_PUT, W.SCOPE_WG, 0, world[k], world[(k + 1) % size], W.NO_RESULT, so, do, n, 0, 0)])
            for k in range(size)]))
        oracle.run_program(ref, np.concatenate([
            W.descs([(W.OP_GET, W.SCOPE_WG, 0, world[k], world[(k - 1) % size], W.NO_RESULT, do, bo, n, 0, 0)])
            for k in range(size)]))
        ref[world[0], co:co + 8] = np.array([size], dtype=np.int64).view(np.uint8)
        assert np.array_equal(got, ref)
        assert ids.cpu().numpy().tolist() == [x for k in range(size) for x in (k, size)]
        assert sorted(fetched.cpu().numpy().tolist()) == list(range(size))
        v.device_ctx_destroy(ctx)
        with pytest.raises(v.VshmemError):
            v.device_ctx_record(ctx)
        assert_no_device_errors()


def test_explicit_context_pool_and_capabilities():
    with heap(3, 2 << 20) as v:
        caps = v.query_capabilities(v.TEAM_WORLD)
        assert caps["explicit_device_ctx"] == 1 and caps["max_device_ctx"] == 64
        hs = [v.device_ctx_create(v.TEAM_WORLD) for _ in range(64)]
        assert sorted(hs) == list(range(64))
        with pytest.raises(v.VshmemError) as e:
            v.device_ctx_create(v.TEAM_WORLD)
        assert e.value.code == v.ERR_NOMEM
        v.device_ctx_destroy(hs[10])
        assert v.device_ctx_create(v.TEAM_WORLD) == 10
        with pytest.raises(v.VshmemError):
            v.device_ctx_create(999)


def test_debug_checks_refuse_bad_calls(monkeypatch):
    """With VSHMEM_DEBUG set at init, calls with operands outside the heap,
    PEs outside the context's team, or arguments that differ across a
    _wave/_wg call latch a device error and do nothing; a valid call still
    moves its data."""
    lib = _lib()
    t = torch()
    monkeypatch.setenv("VSHMEM_DEBUG", "1")
    npes = 4
    with heap(npes, 2 << 20) as v:
        assert v.query_capabilities(v.TEAM_WORLD)["debug"] == 1
        sym = v.malloc(8192)
        so = v.offset(sym)
        region = so + 8192
        init = W.heap_fill(55, npes, region)
        pair_team = v.team_split_strided(v.TEAM_WORLD, 0, 1, 2)      # PEs 0 and 1
        pair = v.team_device(pair_team)
        ctx = v.device_ctx_create(pair_team)
        outside = t.zeros(64, dtype=t.uint8, device="cuda")
        out = t.zeros(4, dtype=t.int64, device="cuda")
        bad_addr, nonuniform = v.DEVERR_BAD_ADDRESS, v.DEVERR_NONUNIFORM
        for which, grid, bits in ((0, 1, bad_addr), (1, 1, bad_addr), (2, 1, nonuniform), (3, 1, nonuniform),
                                  (5, 1, bad_addr), (6, 2, bad_addr), (4, 1, 0)):
            upload(init)
            outside.zero_()
            out.fill_(7)
            t.cuda.synchronize()
            assert lib.usertest_debug(v.device_ctx(), v.device_ctx_record(ctx), ctypes.byref(pair), which, sym,
                                      outside.data_ptr(), out.data_ptr(), grid, None) == 0
            t.cuda.synchronize()
            assert v.device_errors() == bits, which
            got = download(region)
            ref = init.copy()
            if which == 4:
                ref[1, so + 4096:so + 4160] = init[0, so:so + 64]
            assert np.array_equal(got, ref), which
            assert not outside.cpu().numpy().any(), which
            if which == 1:
                assert int(out[0].item()) == 0
            if which == 6:
                assert out[:2].cpu().tolist() == [v.ERR_ARG, v.ERR_ARG]


def test_gpu_space_put_get_names():
    """The GPU-space usage example on objects from shmemg_malloc: a
    work-group-scope shmemg_putmem to the next PE, fence, quiet, barrier,
    then a wavefront-scope shmemg_getmem of the whole block and a
    thread-scope one of an unaligned piece from the next PE.  The heap
    follows the oracle's put and get programs."""
    lib = _lib()
    npes, n, at, tail = 6, 5000, 13, 777
    with heap(npes, 2 << 20) as v:
        src, dst, back, part = (v.shmemg_malloc(n) for _ in range(4))
        so, do, bo, po = (v.offset(a) for a in (src, dst, back, part))
        region = max(so, do, bo, po) + n
        init = W.heap_fill(W.SEED_SMALL + 606, npes, region)
        upload(init)
        assert lib.usertest_gspace(v.device_ctx(), npes, src, dst, back, part, n, at, tail, None) == 0
        got = download(region)
        ref = init.copy()
        oracle.run_program(ref, np.concatenate([
            W.descs([(W.OP_PUT, W.SCOPE_WG, 0, k, (k + 1) % npes, W.NO_RESULT, so, do, n, 0, 0)]) for k in range(npes)]))
        oracle.run_program(ref, np.concatenate(
            [W.descs([(W.OP_GET, W.SCOPE_WAVE, 0, k, (k + 1) % npes, W.NO_RESULT, do, bo, n, 0, 0)]) for k in range(npes)]
            + [W.descs([(W.OP_GET, W.SCOPE_THREAD, 0, k, (k + 1) % npes, W.NO_RESULT, do + at, po, tail, 0, 0)])
               for k in range(npes)]))
        assert np.array_equal(got, ref)
        for k in range(npes):      # each PE got its own block back
            assert np.array_equal(got[k, bo:bo + n], init[k, so:so + n])
        assert_no_device_errors()
