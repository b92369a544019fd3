"""GPU parity: team collectives (broadcast, fcollect, alltoall, reductions)
against the CPU oracle, bit-exact (including fp32 and bf16, whose order is
the documented TREE on both sides)."""
import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, download, heap, upload

pytestmark = pytest.mark.gpu

LAUNCHES = [dict(wgs_per_pe=2, wg_size=128, chunk_bytes=4096), dict(wgs_per_pe=1, wg_size=256, chunk_bytes=65536),
            dict(wgs_per_pe=3, wg_size=64, chunk_bytes=16, flags=1)]


@pytest.mark.parametrize("npes", [1, 2, 5, 8])
def test_data_movement_collectives(npes):
    with heap(npes, 4 << 20) as v:
        src = v.malloc(1 << 20)
        dst = v.malloc(2 << 20)
        so, do = v.offset(src), v.offset(dst)
        region = do + (2 << 20)
        init = W.heap_fill(W.SEED_COLL + npes, npes, region)
        for li, L in enumerate(LAUNCHES):
            launch = v.launch_cfg(**L)
            for n in (1, 40, 4096 + 24, 100_003):
                # broadcast from every root index
                root = (n + li) % npes
                upload(init)
                v.broadcastmem(dst, src, n, root, launch=launch)
                got = download(region)
                ref = init.copy()
                oracle.broadcast(ref, do, so, n, root)
                assert np.array_equal(got, ref), ("broadcast", n, root, L)
                if n * npes <= (1 << 20):
                    upload(init)
                    v.fcollectmem(dst, src, n, launch=launch)
                    got = download(region)
                    ref = init.copy()
                    oracle.fcollect(ref, do, so, n)
                    assert np.array_equal(got, ref), ("fcollect", n, L)
                    upload(init)
                    v.alltoallmem(dst, src, n, launch=launch)
                    got = download(region)
                    ref = init.copy()
                    oracle.alltoall(ref, do, so, n)
                    assert np.array_equal(got, ref), ("alltoall", n, L)
        assert_no_device_errors()


def test_alltoall_small_blocks_lane_groups():
    """Blocks (or chunks) shorter than half a work-group pass go to groups of
    1 to 64 lanes; sizes between those powers, chunked blocks, work-group
    sizes that are not powers of two and both unroll depths must all give
    the oracle's transpose."""
    npes = 7
    with heap(npes, 4 << 20) as v:
        src = v.malloc(1 << 20)
        dst = v.malloc(1 << 20)
        so, do = v.offset(src), v.offset(dst)
        region = do + (1 << 20)
        init = W.heap_fill(W.SEED_COLL + 4242, npes, region)
        cases = [(dict(wgs_per_pe=2, wg_size=192, flags=0), (17, 129, 300, 1000, 2049, 8191)),
                 (dict(wgs_per_pe=1, wg_size=1024, flags=v.LAUNCH_DEEP), (16, 128, 129, 4096, 8200, 65_537)),
                 (dict(wgs_per_pe=3, wg_size=256, chunk_bytes=256), (1000, 4099)),
                 (dict(wgs_per_pe=1, wg_size=64, chunk_bytes=48, flags=v.LAUNCH_NONTEMPORAL), (200, 1001))]
        for L, sizes in cases:
            launch = v.launch_cfg(**L)
            for n in sizes:
                upload(init)
                v.alltoallmem(dst, src, n, launch=launch)
                got = download(region)
                ref = init.copy()
                oracle.alltoall(ref, do, so, n)
                assert np.array_equal(got, ref), ("alltoall", n, L)
        assert_no_device_errors()


def test_shared_team_spans_every_pe():
    """On one GPU every virtual PE shares the node, so the shared teams (host
    and device) have the world's members: size, capabilities, the device
    descriptor, barriers and an alltoall on them match the world's."""
    npes, n = 5, 3000
    with heap(npes, 2 << 20) as v:
        for tm in (v.TEAM_SHARED, v.DEVICE_TEAM_SHARED):
            assert v.team_n_pes(tm) == npes
            d = v.team_device(tm)
            assert (d.start, d.stride, d.size) == (0, 1, npes)
            caps = v.query_capabilities(tm)
            assert caps["team_npes"] == npes and caps["team_start"] == 0 and caps["team_stride"] == 1
        src, dst = v.malloc(n * npes), v.malloc(n * npes)
        so, do = v.offset(src), v.offset(dst)
        region = do + n * npes
        init = W.heap_fill(W.SEED_COLL + 515, npes, region)
        upload(init)
        v.barrier(v.DEVICE_TEAM_SHARED, iters=20)
        v.alltoallmem(dst, src, n, team=v.DEVICE_TEAM_SHARED)
        ref = init.copy()
        oracle.alltoall(ref, do, so, n)
        assert np.array_equal(download(region), ref)
        assert_no_device_errors()


def test_alltoall_tags_transpose_and_involution():
    npes, n = 6, 1000
    with heap(npes, 1 << 20) as v:
        a = v.malloc(npes * n)
        b = v.malloc(npes * n)
        tags = np.zeros((npes, v.offset(b) + npes * n), dtype=np.uint8)
        for q in range(npes):
            for p in range(npes):
                tags[q, v.offset(a) + p * n: v.offset(a) + (p + 1) * n] = 16 * q + p
        upload(tags)
        v.alltoallmem(b, a, n)
        v.alltoallmem(a, b, n)
        got = download(tags.shape[1])
        for p in range(npes):
            for q in range(npes):
                assert np.all(got[p, v.offset(b) + q * n: v.offset(b) + (q + 1) * n] == 16 * q + p)
        assert np.array_equal(got[:, v.offset(a):v.offset(a) + npes * n], tags[:, v.offset(a):v.offset(a) + npes * n])


def _red_inputs(dt, npes, nreduce, seed):
    if dt == oracle.DT_INT64:
        rows = [W.coll_i64(seed, p, nreduce).view(np.uint8) for p in range(npes)]
    elif dt == oracle.DT_FP32:
        rows = [W.coll_f32(seed, p, nreduce).view(np.uint8) for p in range(npes)]
    else:
        rows = [W.coll_bf16(seed, p, nreduce).view(np.uint8) for p in range(npes)]
    return np.stack(rows)


@pytest.mark.parametrize("dt", [oracle.DT_INT64, oracle.DT_FP32, oracle.DT_BF16])
@pytest.mark.parametrize("rop", [oracle.RO_SUM, oracle.RO_MAX])
def test_reductions_bit_exact(dt, rop):
    es = {oracle.DT_INT64: 8, oracle.DT_FP32: 4, oracle.DT_BF16: 2}[dt]
    for npes in (1, 3, 8, 13):
        with heap(npes, 2 << 20) as v:
            nmax = 70_001
            src = v.malloc(nmax * es)
            dst = v.malloc(nmax * es)
            so, do = v.offset(src), v.offset(dst)
            region = do + nmax * es
            for nreduce in (1, 7, 1000, nmax):
                init = np.zeros((npes, region), dtype=np.uint8)
                init[:, so:so + nreduce * es] = _red_inputs(dt, npes, nreduce, 1000 * npes + nreduce)
                for L in (dict(wgs_per_pe=2, wg_size=256, chunk_bytes=4096), dict(wgs_per_pe=1, wg_size=64),
                          dict(wgs_per_pe=3, wg_size=128, chunk_bytes=16384, flags=v.LAUNCH_NONTEMPORAL),
                          dict(wgs_per_pe=1, wg_size=512, chunk_bytes=2048),            # members over wavefronts
                          dict(wgs_per_pe=2, wg_size=384, chunk_bytes=65536, flags=v.LAUNCH_NONTEMPORAL),
                          dict(wgs_per_pe=2, wg_size=128, chunk_bytes=4096, flags=v.LAUNCH_DEEP),  # two vectors per lane
                          dict(wgs_per_pe=1, wg_size=256, flags=v.LAUNCH_DEEP | v.LAUNCH_NONTEMPORAL)):
                    upload(init)
                    v.reduce(dt, rop, dst, src, nreduce, launch=v.launch_cfg(**L))
                    got = download(region)
                    ref = init.copy()
                    oracle.reduce(ref, dt, rop, do, so, nreduce)
                    assert np.array_equal(got, ref), (dt, rop, npes, nreduce, L)
            # in place
            init = np.zeros((npes, region), dtype=np.uint8)
            init[:, so:so + 999 * es] = _red_inputs(dt, npes, 999, 7)
            upload(init)
            v.reduce(dt, rop, src, src, 999)
            got = download(region)
            ref = init.copy()
            oracle.reduce(ref, dt, rop, so, so, 999)
            assert np.array_equal(got, ref)
            assert_no_device_errors()


@pytest.mark.parametrize("dt", [oracle.DT_INT64, oracle.DT_FP32, oracle.DT_BF16])
def test_reduction_team_of_130(dt):
    """A team of 130 members needs 8 TREE levels; 130 is not a power of
    two, so odd carries occur at several levels."""
    es = {oracle.DT_INT64: 8, oracle.DT_FP32: 4, oracle.DT_BF16: 2}[dt]
    npes, nreduce = 130, 5003
    with heap(npes, 2 << 20) as v:
        src = v.malloc(nreduce * es)
        dst = v.malloc(nreduce * es)
        so, do = v.offset(src), v.offset(dst)
        region = do + nreduce * es
        init = np.zeros((npes, region), dtype=np.uint8)
        init[:, so:so + nreduce * es] = _red_inputs(dt, npes, nreduce, 4242)
        for rop in (oracle.RO_SUM, oracle.RO_MAX):
            upload(init)
            v.reduce(dt, rop, dst, src, nreduce)
            got = download(region)
            ref = init.copy()
            oracle.reduce(ref, dt, rop, do, so, nreduce)
            assert np.array_equal(got, ref), (dt, rop)
        assert_no_device_errors()


def test_strided_team_collectives():
    npes = 10
    with heap(npes, 2 << 20) as v:
        team = v.team_split_strided(v.DEVICE_TEAM_WORLD, 1, 2, 4)       # PEs 1, 3, 5, 7
        tri = (1, 2, 4)
        src = v.malloc(64 << 10)
        dst = v.malloc(256 << 10)
        so, do = v.offset(src), v.offset(dst)
        region = do + (256 << 10)
        init = W.heap_fill(99, npes, region)
        n = 10_000
        upload(init)
        v.alltoallmem(dst, src, n // 4, team=team)
        got = download(region)
        ref = init.copy()
        oracle.alltoall(ref, do, so, n // 4, team=tri)
        assert np.array_equal(got, ref)
        upload(init)
        v.broadcastmem(dst, src, n, 3, team=team)
        got = download(region)
        ref = init.copy()
        oracle.broadcast(ref, do, so, n, 3, team=tri)
        assert np.array_equal(got, ref)
        init2 = np.zeros((npes, region), dtype=np.uint8)
        init2[:, so:so + 4 * 3000] = _red_inputs(oracle.DT_FP32, npes, 3000, 5)
        upload(init2)
        v.reduce(v.DT_FP32, v.RED_SUM, dst, src, 3000, team=team)
        got = download(region)
        ref = init2.copy()
        oracle.reduce(ref, oracle.DT_FP32, oracle.RO_SUM, do, so, 3000, team=tri)
        assert np.array_equal(got, ref)
        with pytest.raises(v.VshmemError):
            v.alltoallmem(dst, dst + 8, 64)                  # overlapping ranges
        assert_no_device_errors()


_ES = {oracle.DT_INT64: 8, oracle.DT_FP32: 4, oracle.DT_BF16: 2}
_BITS = {oracle.DT_INT64: np.int64, oracle.DT_FP32: np.uint32, oracle.DT_BF16: np.uint16}


def _same_results(got, ref, dt):
    """Bit-identical, except that a NaN result only has to be a NaN: IEEE-754
    fixes neither the sign nor the payload of the NaN an invalid operation
    (inf + -inf) produces, and x86 and gfx950 pick different ones."""
    g, r = got.view(_BITS[dt]), ref.view(_BITS[dt])
    if dt == oracle.DT_INT64:
        return np.array_equal(g, r)
    if dt == oracle.DT_FP32:
        rn, gn = np.isnan(r.view(np.float32)), np.isnan(g.view(np.float32))
    else:
        rn = ((r & 0x7F80) == 0x7F80) & ((r & 0x7F) != 0)
        gn = ((g & 0x7F80) == 0x7F80) & ((g & 0x7F) != 0)
    return np.array_equal(rn, gn) and np.array_equal(g[~rn], r[~rn])


@pytest.mark.parametrize("npes", [13, 64, 130])
@pytest.mark.parametrize("dt", [oracle.DT_INT64, oracle.DT_FP32, oracle.DT_BF16])
def test_reduction_edge_values_bit_exact(npes, dt):
    """Edge-case columns against the oracle, sum and max: signed zeros at
    every TREE position (max ties keep the lower PE), fp32/bf16 subnormal
    inputs and sums that stay subnormal or cross into the normal range,
    one infinity, both infinities, values near the largest finite one
    (overflow in fp32, or at the final bf16 rounding), NaN inputs, bf16
    rounding ties, and int64 MIN/MAX.  Aligned bases take the vector path,
    a base one element past a 16-byte boundary the scalar path."""
    es = _ES[dt]
    K = 4099                                   # several tiles and a ragged tail
    cols = W.reduce_edge_columns(dt, npes, K, W.subseed(W.SEED_COLL, 0xED6E + 131 * npes + dt))
    with heap(npes, 1 << 20) as v:
        src = v.malloc(K * es + 64)
        dst = v.malloc(K * es + 64)
        so, do = v.offset(src), v.offset(dst)
        region = do + K * es + 64
        for shift in (0, es):
            init = np.zeros((npes, region), dtype=np.uint8)
            init[:, so + shift:so + shift + K * es] = np.ascontiguousarray(cols).view(np.uint8).reshape(npes, K * es)
            # the default launch (one lane folds every member), for teams of
            # up to 64 the members split over 8 wavefronts, and for teams of
            # up to 127 two vectors per lane
            cases = [(oracle.RO_SUM, None), (oracle.RO_MAX, None)]
            if npes <= 64:
                cases += [(oracle.RO_SUM, v.launch_cfg(wg_size=512, flags=v.LAUNCH_NONTEMPORAL)),
                          (oracle.RO_MAX, v.launch_cfg(wg_size=512, wgs_per_pe=2))]
            if npes < 128:
                cases += [(oracle.RO_SUM, v.launch_cfg(flags=v.LAUNCH_DEEP | v.LAUNCH_NONTEMPORAL)),
                          (oracle.RO_MAX, v.launch_cfg(wg_size=128, flags=v.LAUNCH_DEEP))]
            for rop, launch in cases:
                upload(init)
                v.reduce(dt, rop, dst + shift, src + shift, K, launch=launch)
                got = download(region)
                ref = init.copy()
                oracle.reduce(ref, dt, rop, do + shift, so + shift, K)
                lo, hi = do + shift, do + shift + K * es
                assert np.array_equal(got[:, :lo], ref[:, :lo]) and np.array_equal(got[:, hi:], ref[:, hi:])
                for p in (0, npes // 2, npes - 1):
                    assert np.array_equal(got[p, lo:hi], got[0, lo:hi])
                g, r = got[0, lo:hi].copy(), ref[0, lo:hi].copy()
                assert _same_results(g, r, dt), (npes, dt, rop, shift, launch is None)
        assert_no_device_errors()


@pytest.mark.parametrize("spread", [True, False])
def test_collectives_at_both_slice_strides(spread):
    """The same movement collectives and a reduction over 64 MiB slices with the
    library's spread stride (98 MiB) and with the smallest one (66 MiB):
    byte-exact against the oracle either way, so the layout is only a
    matter of speed."""
    npes, MiB = 8, 1 << 20
    with heap(npes, 64 * MiB, spread=spread) as v:
        assert v.heap_stride() == (98 if spread else 66) * MiB
        n = 300_001
        src, dst, red = v.malloc(4 * MiB), v.malloc(8 * MiB), v.malloc(4 * n)
        so, do, ro = v.offset(src), v.offset(dst), v.offset(red)
        region = ro + 4 * n
        init = W.heap_fill(W.SEED_COLL + 64, npes, region)
        init[:, ro:ro + 4 * n] = _red_inputs(oracle.DT_FP32, npes, n, 64)
        steps = [
            ("broadcast", lambda: v.broadcastmem(dst, src, 3 * MiB + 5, 3),
             lambda ref: oracle.broadcast(ref, do, so, 3 * MiB + 5, 3)),
            ("fcollect", lambda: v.fcollectmem(dst, src, MiB - 3),
             lambda ref: oracle.fcollect(ref, do, so, MiB - 3)),
            ("alltoall", lambda: v.alltoallmem(dst, src, 512 * 1024 - 16),
             lambda ref: oracle.alltoall(ref, do, so, 512 * 1024 - 16)),
            ("reduce", lambda: v.reduce(oracle.DT_FP32, oracle.RO_SUM, red, red, n),
             lambda ref: oracle.reduce(ref, oracle.DT_FP32, oracle.RO_SUM, ro, ro, n)),
        ]
        for name, run, model in steps:
            upload(init)
            run()
            got = download(region)
            ref = init.copy()
            model(ref)
            assert np.array_equal(got, ref), (name, spread)
        assert_no_device_errors()
