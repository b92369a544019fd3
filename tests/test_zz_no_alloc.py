"""GPU: shmemx_launch_batch_noalloc (the batch launcher over the library's
fixed device workspace, for callers that cannot allocate) against
shmemx_launch_batch on the same kernel-written tables: two calls in a row,
the second with a smaller table, each checked against the oracle too.  The
heap must be identical bit for bit; the fetched values of the contended
fetch_adds depend on the order the device applied them in, so for both
launchers each counter's fetched values must be a permutation of 0..k-1."""
import numpy as np
import pytest

import oracle
import workload as W
from tests.gpu_helpers import assert_no_device_errors, download, heap, program, torch, upload, write_table

pytestmark = pytest.mark.gpu


def _fetched_ok(res, descs):
    amo = descs[descs["op"] == W.OP_AMO_FETCH_ADD]
    for c in np.unique(amo["src"]):
        ids = amo[amo["src"] == c]["result_idx"].astype(np.int64)
        if not np.array_equal(np.sort(res[ids]), np.arange(len(ids))):
            return False
    return True


def test_noalloc_batch_equals_launch_batch():
    t = torch()
    with heap(4, 2 << 20) as v:
        cap = v.launch_batch_noalloc_max()
        assert cap >= 20000
        for k, (n_rma, n_amo) in enumerate([(800, 6000), (200, 400)]):     # the second call is smaller
            wl, descs = program(W.SEED_SMALL + 40 + k, n_rma=n_rma, n_amo=n_amo)
            n = len(descs)
            table = write_table(descs)
            ref = wl.init.copy()
            oracle.run_program(ref, descs, nresults=wl.n_amo)
            outs = []
            for launch in (v.launch_batch, v.launch_batch_noalloc):
                upload(wl.init)
                res = t.zeros(n, dtype=t.int64, device="cuda")
                t.cuda.synchronize()
                launch(table, n, results=res)
                t.cuda.synchronize()
                outs.append((download(wl.heap_bytes), res.cpu().numpy()))
            (h0, r0), (h1, r1) = outs
            assert np.array_equal(h1, h0) and np.array_equal(h1, ref), k
            assert _fetched_ok(r0, descs) and _fetched_ok(r1, descs), k
            assert not r1[wl.n_amo:].any()
        with pytest.raises(v.VshmemError) as e:                           # refused on the host
            v.launch_batch_noalloc(table, cap + 1)
        assert e.value.code == v.ERR_ARG
        assert_no_device_errors()
