"""GPU edge cases: zero-length operations on every path (launchers, host
calls, stream calls), and the largest team the reductions' TREE fold
accepts (511 members, nine levels) next to the first one it refuses."""
import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, download, heap, torch, upload

pytestmark = pytest.mark.gpu


def test_zero_length_operations_change_nothing():
    from paper_2607_08006_amd import host
    t = torch()
    npes = 5
    with heap(npes, 2 << 20) as v:
        a, b = v.malloc(1 << 16), v.malloc(1 << 16)
        region = v.offset(b) + (1 << 16)
        init = W.heap_fill(808, npes, region)
        upload(init)
        for dt in (v.DT_INT64, v.DT_FP32, v.DT_BF16):
            v.reduce(dt, v.RED_SUM, b, a, 0)
            host.reduce(dt, v.RED_MAX, b, a, 0)
        v.broadcastmem(b, a, 0, 2)
        v.fcollectmem(b, a, 0)
        v.alltoallmem(b, a, 0)
        host.broadcastmem(b, a, 0, 1)
        host.fcollectmem(b, a, 0)
        host.alltoallmem(b, a, 0)
        buf = np.zeros(8, dtype=np.uint8)
        host.putmem(a, buf, 0, 3)
        host.getmem(buf, a, 0, 3)
        host.putmem_nbi(a, buf, 0, 4)
        host.quiet()
        s = t.cuda.Stream()
        host.putmem_on_stream(a, buf, 0, 1, stream=s)
        host.broadcastmem_on_stream(b, a, 0, 0, stream=s)
        host.reduce_on_stream(v.DT_FP32, v.RED_SUM, b, a, 0, stream=s)
        s.synchronize()
        t.cuda.synchronize()
        assert np.array_equal(download(region), init)
        assert_no_device_errors()


@pytest.mark.parametrize("dt", [oracle.DT_INT64, oracle.DT_FP32, oracle.DT_BF16])
def test_reduction_at_the_deepest_tree(dt):
    """511 members fill all nine levels of the fold (every carry path); a
    512-member team is refused before anything runs."""
    es = {oracle.DT_INT64: 8, oracle.DT_FP32: 4, oracle.DT_BF16: 2}[dt]
    gen = {oracle.DT_INT64: W.coll_i64, oracle.DT_FP32: W.coll_f32, oracle.DT_BF16: W.coll_bf16}[dt]
    npes, nreduce = 512, 1001
    with heap(npes, 1 << 20) as v:
        src, dst = v.malloc(nreduce * es), v.malloc(nreduce * es)
        so, do = v.offset(src), v.offset(dst)
        region = do + nreduce * es
        init = np.zeros((npes, region), dtype=np.uint8)
        init[:, so:so + nreduce * es] = np.stack([gen(77 + dt, p, nreduce).view(np.uint8) for p in range(npes)])
        team = v.team_split_strided(v.TEAM_WORLD, 1, 1, 511)                # PEs 1 .. 511
        for rop in (oracle.RO_SUM, oracle.RO_MAX):
            upload(init)
            v.reduce(dt, rop, dst, src, nreduce, team=team)
            ref = init.copy()
            oracle.reduce(ref, dt, rop, do, so, nreduce, team=(1, 1, 511))
            assert np.array_equal(download(region), ref), rop
        upload(init)
        with pytest.raises(v.VshmemError) as e:
            v.reduce(dt, oracle.RO_SUM, dst, src, nreduce, team=v.TEAM_WORLD)
        assert e.value.code == v.ERR_UNSUPPORTED
        assert np.array_equal(download(region), init)
        assert_no_device_errors()
