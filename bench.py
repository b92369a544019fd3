#!/usr/bin/env python3
"""Benchmark of the device-initiated SHMEM hot path on one MI355X.

One step is one pass of every hot-path row over one batch of synthetic
input on 64 virtual PEs with a 1 GiB symmetric heap each: put/get at
work-group, wavefront and thread scope (ring and derangement patterns, each
ending in quiet), random-access atomics, put-with-signal ping-pong, barrier,
broadcast, fcollect, alltoall, sum/max reductions (int64, fp32, bf16 with fp32
accumulation), a batch of mixed operations in its fused, per-operation and
hipGraph forms, and the persistent progress kernel serving a request burst.

Prints one JSON line.  `value` is the whole step's algorithmic HBM traffic
(bytes read + written by the operations' definitions) divided by the step
time.  Per-row figures, the latency comparison and the roofline of the
dominant kernel ride along in the same line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workload as W  # noqa: E402

MiB = 1 << 20
# Progress kernel launch shape for the serving rows, from measurements on
# MI355X: whole work-groups execute chunks, and 1024-thread work-groups with
# 256 KiB chunks gave the best tail latency under load (1 MiB chunks: about
# 8% more saturated throughput, twice the p99).  The per-op form is fastest
# with 256 KiB per work-group as well.
PROGRESS_WG = 1024
PROGRESS_CHUNK = 256 << 10
PER_OP_CHUNK = 256 << 10
WINDOW_US = 20.0   # arrival window of the batched serving forms
GiB = 1 << 30
HBM_PEAK_GBS = 8000.0
METRIC = "put/get/alltoall GB/s vs HBM peak; AMO Mops/s; p50/p99 op latency batched vs per-op"


def log(msg: str) -> None:
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--npes", type=int, default=64)
    ap.add_argument("--heap-mib", type=int, default=1024)
    ap.add_argument("--rows", default="", help="comma-separated subset of rows (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the ceilings and the configuration sections (profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--probe-copy-mib", type=int, default=0,
                    help="also run one plain copy of this size (counter scaling reference)")
    ap.add_argument("--hbm-probe-mib", type=int, default=0,
                    help="also run each HBM probe kind once on buffers of this size (counter passes)")
    ap.add_argument("--out", default="", help="also write the JSON line to this file")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the step: the full put/get sweep (8 B - 64 MiB, 3 scopes, 2 patterns)")
    ap.add_argument("--serve", action="store_true",
                    help="instead of the step: open-loop Poisson serving on 128 PEs x 512 MiB, 64 GiB budget")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-wg", type=int, default=PROGRESS_WG, help="progress kernel work-group size")
    ap.add_argument("--serve-chunk-kib", type=int, default=PROGRESS_CHUNK >> 10, help="progress kernel chunk size")
    ap.add_argument("--configs-only", action="store_true",
                    help="instead of the step: only the small-program and 256-PE ping-pong sections")
    ap.add_argument("--summarize-profiles", default="", metavar="DIR",
                    help="no GPU work: write profiles/ summaries from rocprofv3 CSV output under DIR")
    return ap.parse_args()


class Layout:
    """Per-PE heap layout (offsets in bytes, identical on every PE)."""

    def __init__(self, v, heap_mib: int):
        scale = heap_mib / 1024.0
        sz = lambda mib: int(mib * scale) * MiB  # noqa: E731
        self.A = v.offset(v.malloc(sz(256)))   # put/get source (uint8 payload)
        self.B = v.offset(v.malloc(sz(256)))   # destinations of put/get and collectives
        self.C = v.offset(v.malloc(sz(256)))   # broadcast / fcollect / alltoall sources
        self.D = v.offset(v.malloc(sz(128)))   # int64 reduction input
        self.E = v.offset(v.malloc(sz(64)))    # fp32 reduction input
        self.F = v.offset(v.malloc(sz(32)))    # bf16 reduction input
        self.G = v.offset(v.malloc(sz(16)))    # GUPS table slice
        self.H = v.offset(v.malloc(sz(16)))    # batch, ping-pong, barrier area
        self.scale = scale
        self.addr = lambda off: v.heap_base() + off  # noqa: E731


def fill_heap(v, L: Layout, npes: int):
    base = v.heap_base()
    stride = v.heap_stride()
    for p in range(npes):
        pe = base + p * stride
        v.fill_random(pe + L.A, L.B - L.A, W.subseed(W.SEED_SWEEP, W.TAG_HEAP + p))
        v.fill_random(pe + L.B, L.C - L.B, W.subseed(W.SEED_SWEEP, 0x200 + p))
        v.fill_typed(pe + L.C, (L.D - L.C) // 4, v.DT_FP32, W.subseed(W.SEED_COLL, W.TAG_HEAP + p))
        v.fill_typed(pe + L.D, (L.E - L.D) // 8, v.DT_INT64, W.subseed(W.SEED_COLL, 0x300 + p))
        v.fill_typed(pe + L.E, (L.F - L.E) // 4, v.DT_FP32, W.subseed(W.SEED_COLL, 0x400 + p))
        v.fill_typed(pe + L.F, (L.G - L.F) // 2, v.DT_BF16, W.subseed(W.SEED_COLL, 0x500 + p))
        v.fill_typed(pe + L.G, (L.H - L.G) // 8, v.DT_INT64, W.subseed(W.SEED_GUPS, W.TAG_HEAP + p))
        v.fill_random(pe + L.H, int(16 * MiB * L.scale), W.subseed(W.SEED_SMALL, W.TAG_HEAP + p))


class Row:
    def __init__(self, name, fn, bytes_=0, ops=0, kernel=""):
        self.name, self.fn, self.bytes, self.ops, self.kernel = name, fn, bytes_, ops, kernel
        self.ms = []


def build_rows(v, torch, L: Layout, npes: int, want):
    rows = []
    scale = L.scale
    ring = torch.from_numpy(W.ring(npes).astype(np.int32)).cuda()
    perm = torch.from_numpy(W.derangement(W.subseed(W.SEED_SWEEP, W.TAG_PERM), npes).astype(np.int32)).cuda()

    def add(name, fn, b=0, ops=0, kernel=""):
        if not want or name in want:
            rows.append(Row(name, fn, b, ops, kernel))

    # ---- put/get (a2, a3): k(s) = min(2^28 / s, 2^14) messages per PE, each PE ends in quiet
    def rma(op, scope, tgts, size, wgs, wg, nmsg=None, flags=0):
        k = nmsg if nmsg is not None else W.msgs_per_pe(size)
        span = L.B - L.A
        while k * size > span:
            k //= 2
        lc = v.launch_cfg(wgs_per_pe=wgs, wg_size=wg, flags=flags)
        return (lambda: v.rma_pattern(op, scope, tgts, L.A, L.B, size, k, launch=lc)), 2 * npes * k * size

    # Launch shapes from the measured sweep: about one work-group per CU,
    # nontemporal 8-deep copies for large messages.
    big = int(16 * MiB * min(1.0, scale))
    deep = v.LAUNCH_NONTEMPORAL | v.LAUNCH_DEEP
    f, b = rma(v.OP_PUT, v.SCOPE_WG, ring, big, 4, 1024, flags=deep)
    add("put_wg_16MiB_ring", f, b, kernel="k_rma_pattern<2,true,true,8,1024>")
    f, b = rma(v.OP_GET, v.SCOPE_WG, perm, big, 4, 1024, flags=deep)
    add("get_wg_16MiB_perm", f, b, kernel="k_rma_pattern<2,false,true,8,1024>")
    huge = int(64 * MiB * min(1.0, scale))
    f, b = rma(v.OP_PUT, v.SCOPE_GRID, perm, huge, 4, 256, flags=deep)
    add("put_grid_64MiB_perm", f, b, kernel="k_rma_pattern<3,true,true,8,256>")
    f, b = rma(v.OP_PUT, v.SCOPE_WAVE, perm, 4096, 4, 256, flags=v.LAUNCH_NONTEMPORAL)
    add("put_wave_4KiB_perm", f, b, kernel="k_rma_pattern<1,true,true,4,256>")
    f, b = rma(v.OP_GET, v.SCOPE_THREAD, ring, 64, 4, 256)
    add("get_thread_64B_ring", f, b)
    f, b = rma(v.OP_PUT, v.SCOPE_THREAD, perm, 8, 2, 1024)
    add("put_thread_8B_perm", f, b)

    # ---- atomics (a4): 2^26 random fetch_xor / fetch_add updates on a 2^27-entry table
    log2_table = 27 if scale >= 1.0 else max(10, 27 - int(np.ceil(np.log2(1 / scale))))
    nupd = 1 << (log2_table - 1)
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    gseed = W.subseed(W.SEED_GUPS, W.TAG_OPS)
    add("gups_fetch_xor_add", lambda: v.gups(L.G, log2_table, nupd, gseed, 5, acc=acc), 16 * nupd, nupd)

    # ---- signal ping-pong (a5): 32 pairs, 200 round trips, 8-byte payload
    npairs, rounds = min(32, npes // 2), 200
    pairs = torch.arange(2 * npairs, dtype=torch.int32, device="cuda")
    rtt = torch.zeros(npairs * rounds, dtype=torch.int64, device="cuda")
    add("pingpong_signal_8B", lambda: v.pingpong(L.H, L.H + 64, pairs, npairs, rounds, 8, False, rtt),
        0, 2 * npairs * rounds)

    # ---- barrier (a6)
    add("barrier_all", lambda: v.barrier(v.DEVICE_TEAM_WORLD, iters=100), 0, 100)

    # ---- collectives (a7-a10)
    blk = int(1 * MiB * min(1.0, scale))
    add("alltoall_1MiB_fp32", lambda: v.alltoallmem(L.addr(L.B), L.addr(L.C), blk), 2 * npes * npes * blk,
        kernel="k_alltoall<true,8>")
    fc = int(4 * MiB * min(1.0, scale))
    add("fcollect_4MiB", lambda: v.fcollectmem(L.addr(L.B), L.addr(L.C), fc), npes * fc + npes * npes * fc,
        kernel="k_fcollect<false>")
    bc = L.D - L.C
    add("broadcast_256MiB", lambda: v.broadcastmem(L.addr(L.B), L.addr(L.C), bc, 0), bc + npes * bc,
        kernel="k_broadcast<false>")
    nred = (L.E - L.D) // 8
    for dt, src, es, tag, codec in ((v.DT_INT64, L.D, 8, "i64", "CodecI64"), (v.DT_FP32, L.E, 4, "f32", "CodecF32"),
                                    (v.DT_BF16, L.F, 2, "bf16", "CodecBF16")):
        n = min(nred, (L.G - src) // es) if dt != v.DT_INT64 else nred
        add(f"reduce_sum_{tag}", (lambda dt=dt, src=src, n=n: v.reduce(dt, v.RED_SUM, L.addr(L.B), L.addr(src), n)),
            2 * npes * n * es, kernel=f"k_reduce<{codec},OpSum,true>")
    add("reduce_max_i64", lambda: v.reduce(v.DT_INT64, v.RED_MAX, L.addr(L.B), L.addr(L.D), nred), 2 * npes * nred * 8,
        kernel="k_reduce<CodecI64,OpMax,true>")
    add("reduce_max_f32", lambda: v.reduce(v.DT_FP32, v.RED_MAX, L.addr(L.B), L.addr(L.E), nred),
        2 * npes * nred * 4, kernel="k_reduce<CodecF32,OpMax,true>")
    return rows


def batch_setup(v, torch, L: Layout, npes: int):
    """A burst of 1000 uneven put/get and 1000 fetch_add over all PEs, with
    completion stamps for the fused, per-op and graph forms."""
    region = int(16 * MiB * L.scale) - 4 * 4096
    wl = W.small_workload(npes=npes, heap_bytes=region, n_rma=1000, epoch_ops=1000, n_amo=1000,
                          base_off=L.H + 4 * 4096, fill=False)
    nd = len(wl.descs)
    res = torch.zeros(wl.n_amo, dtype=torch.int64, device="cuda")
    st = {k: torch.zeros(nd, dtype=torch.int64, device="cuda") for k in ("fused", "per_op", "graph")}
    t0 = {k: torch.zeros(1, dtype=torch.int64, device="cuda") for k in ("fused", "per_op", "graph")}
    plan = v.Plan(wl.descs)
    plan_graph = v.Plan(wl.descs)
    plan_graph.set_stamps(st["graph"])
    plan_graph.graph_build(1, results=res)
    ops = wl.descs["op"]
    is_op = (ops == W.OP_PUT) | (ops == W.OP_GET) | (ops == W.OP_AMO_FETCH_ADD)
    payload = int(wl.descs["nbytes"][(ops == W.OP_PUT) | (ops == W.OP_GET)].sum())
    return dict(wl=wl, plan=plan, graph=plan_graph, res=res, stamps=st, t0=t0, is_op=is_op,
                bytes=2 * payload + 16 * wl.n_amo, nops=int(is_op.sum()))


def batch_step(v, B):
    """One burst in each form; returns nothing (stamps stay on the device)."""
    for k in ("fused", "per_op", "graph"):
        B["stamps"][k].zero_()
    plan = B["plan"]
    v.stamp(B["t0"]["fused"])
    plan.set_stamps(B["stamps"]["fused"])
    plan.launch_fused(results=B["res"])
    v.stamp(B["t0"]["per_op"])
    plan.set_stamps(B["stamps"]["per_op"])
    plan.launch_per_op(results=B["res"])
    v.stamp(B["t0"]["graph"])
    B["graph"].graph_launch()


def batch_latencies(v, B):
    hz = v.wallclock_hz()
    out = {}
    for k in ("fused", "per_op", "graph"):
        st = B["stamps"][k].cpu().numpy()[B["is_op"]]
        t0 = int(B["t0"][k].cpu().numpy()[0])
        out[k] = (st - t0) / hz * 1e6        # microseconds from burst submission to op completion
    return out


def serve_setup(v, torch, L: Layout, npes: int, nreq: int = 1000):
    """A burst of mixed put/get/fetch_add requests (log-uniform 64 B - 16 MiB)
    for the persistent progress kernel; sources in A, destinations and
    counters in B, admission under an 8 GiB budget."""
    reqs = serve_trace(v, npes, nreq, rate=1e12, src_bytes=L.B - L.A, seed=W.SEED_SERVE)
    side = torch.cuda.Stream()
    return dict(reqs=reqs, side=side, region_off=L.B, region_bytes=L.C - L.B, budget=8 << 30,
                bytes=sum(2 * r.nbytes if r.op != W.OP_AMO_FETCH_ADD else 2 * r.nbytes for r in reqs))


def serve_trace(v, npes, n, rate, src_bytes, seed):
    from paper_2607_08006_amd import Request
    out = []
    xs = W.splitmix64(W.subseed(seed, 0x77), 0, n)
    for i, r in enumerate(W.serve_requests(seed, n, npes, rate_per_s=rate, lanes=8)):
        nb = min(r.nbytes, src_bytes)
        src = 0
        if r.kind == W.OP_AMO_FETCH_ADD:
            nb = max(8, nb & ~7)
        else:
            src = int(xs[i] % np.uint64(src_bytes - nb + 1))
        out.append(Request(r.kind, r.issuer, r.target, r.lane, nb, src, r.arrival_s))
    return out


def serve_step(v, S):
    v.progress_start(nwg=0, wg_size=PROGRESS_WG, ring_slots=4096, verify=False, chunk_bytes=PROGRESS_CHUNK,
                     stream=S["side"])
    try:
        dst, lat, comps, stats = v.serve_run(S["reqs"], 8, S["region_off"], S["region_bytes"], S["budget"])
    finally:
        v.progress_stop(30000)
        S["side"].synchronize()
    return lat, comps, stats


def percentile(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q)) if len(a) else None


# Sources each timed kernel is compiled from: a change to any of them makes
# the committed counter figures stale.
KERNEL_SOURCES = {
    "k_rma_pattern": ["paper_2607_08006_amd/csrc/rma.hip"],
    "k_alltoall": ["paper_2607_08006_amd/csrc/coll.hip"],
    "k_broadcast": ["paper_2607_08006_amd/csrc/coll.hip"],
    "k_fcollect": ["paper_2607_08006_amd/csrc/coll.hip"],
    "k_reduce": ["paper_2607_08006_amd/csrc/coll.hip"],
    "k_reduce_waves": ["paper_2607_08006_amd/csrc/coll.hip"],
}
COMMON_SOURCES = ["include/vshmem.h", "include/vshmem_device.hpp", "paper_2607_08006_amd/csrc/runtime.hpp"]
PROFILE_DIR = os.path.join(ROOT, "profiles")
# Rows whose kernels get HBM counter passes (FETCH_SIZE, WRITE_SIZE).
PMC_ROWS = ["put_wg_16MiB_ring", "get_wg_16MiB_perm", "put_grid_64MiB_perm", "put_wave_4KiB_perm",
            "alltoall_1MiB_fp32", "fcollect_4MiB", "broadcast_256MiB", "reduce_sum_i64", "reduce_sum_f32",
            "reduce_sum_bf16"]


def kernel_digest(kernel: str) -> str:
    files = KERNEL_SOURCES.get(kernel.split("<")[0])
    if files is None:
        return ""
    h = hashlib.sha256()
    for fn in files + COMMON_SOURCES:
        with open(os.path.join(ROOT, fn), "rb") as f:
            h.update(fn.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def pmc_traffic(kernel: str, launches_bytes: int):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when there is none or its sources changed since."""
    path = os.path.join(PROFILE_DIR, "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            ent = json.load(f).get("kernels", {}).get(kernel)
        if not ent or not ent.get("source_digest") or ent["source_digest"] != kernel_digest(kernel):
            return None
        return int(ent["fetch_bytes"] + ent["write_bytes"])
    except (OSError, ValueError, KeyError, TypeError):
        return None


def _csv_rows(pattern):
    import csv
    import glob
    out = []
    for fn in glob.glob(pattern, recursive=True):
        with open(fn) as fh:
            out += list(csv.DictReader(fh))
    return out


def _short_kernel(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("vshmem_detail::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0].replace(", ", ",")


def summarize_profiles(prof_dir: str, probe_mib: int) -> None:
    """Turn rocprofv3 CSV output into the committed summaries: a kernel table
    from `<prof_dir>/trace` and per-launch HBM bytes from the FETCH_SIZE and
    WRITE_SIZE passes in `<prof_dir>/pmc_<counter>`, each counter scaled by
    what it reads for the plain copy probe of probe_mib MiB in, probe_mib out."""
    rel = os.path.relpath(prof_dir, ROOT) if os.path.isabs(prof_dir) else prof_dir
    trace_cmd = (f"rocprofv3 --kernel-trace --stats -d {rel}/trace -o bench --output-format csv "
                 "-- python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-extras")
    pmc_cmd = ("rocprofv3 --pmc {ctr} -d " + rel + "/pmc_{ctr} -o pmc --output-format csv -- python3 bench.py "
               "--rows " + ",".join(PMC_ROWS) + " --steps 2 --warmup 1 "
               f"--no-cpu-baseline --probe-copy-mib {probe_mib} --hbm-probe-mib {probe_mib}")
    stats = _csv_rows(os.path.join(prof_dir, "trace", "**", "*kernel_stats.csv"))
    if stats:
        stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
        lines = ["# Kernel statistics: bench.py step, 64 virtual PEs x 1 GiB", "",
                 "Command (from /tmp with TMPDIR=/tmp, then in the repository root):", "",
                 f"`{trace_cmd}`", "",
                 "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
        for r in stats[:40]:
            lines.append("| `%s` | %s | %.3f | %.2f | %.2f | %.2f | %.2f |" % (
                _short_kernel(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                float(r["Percentage"])))
        with open(os.path.join(PROFILE_DIR, "bench_step_64pe_kernel_stats.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
    per = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        for r in _csv_rows(os.path.join(prof_dir, f"pmc_{ctr}", "**", "*counter_collection.csv")):
            if r["Counter_Name"] == ctr:
                per.setdefault((ctr, _short_kernel(r["Kernel_Name"])), []).append(float(r["Counter_Value"]))
    avg = {k: sum(v) / len(v) for k, v in per.items()}
    probe = probe_mib * MiB
    f_scale = probe / (avg[("FETCH_SIZE", "k_probe_copy")] * 1024)
    w_scale = probe / (avg[("WRITE_SIZE", "k_probe_copy")] * 1024)
    kernels = {}
    for (ctr, k), kib in sorted(avg.items()):
        if ctr != "FETCH_SIZE" or k.split("<")[0] not in KERNEL_SOURCES or ("WRITE_SIZE", k) not in avg:
            continue
        kernels[k] = {"fetch_kib_per_launch": round(kib, 1),
                      "write_kib_per_launch": round(avg[("WRITE_SIZE", k)], 1),
                      "fetch_bytes": int(kib * 1024 * f_scale), "write_bytes": int(avg[("WRITE_SIZE", k)] * 1024 * w_scale),
                      "launches": len(per[(ctr, k)]), "source_digest": kernel_digest(k)}
    hbm = {}
    for k, reads, writes in (("k_probe_copy_gridstride", probe, probe), ("k_probe_copy_tiles", probe, probe),
                             ("k_probe_read", probe, 0), ("k_probe_write", 0, probe)):
        if ("FETCH_SIZE", k) in avg and ("WRITE_SIZE", k) in avg:
            hbm[k] = {"algorithmic_read": reads, "algorithmic_write": writes,
                      "fetch_bytes": int(avg[("FETCH_SIZE", k)] * 1024 * f_scale),
                      "write_bytes": int(avg[("WRITE_SIZE", k)] * 1024 * w_scale)}
    out = {"hbm_probes": hbm,
           "probe": {"bytes_read": probe, "bytes_written": probe,
                     "fetch_kib": round(avg[("FETCH_SIZE", "k_probe_copy")], 1),
                     "write_kib": round(avg[("WRITE_SIZE", "k_probe_copy")], 1),
                     "fetch_scale": round(f_scale, 5), "write_scale": round(w_scale, 5)},
           "kernels": kernels,
           "commands": [pmc_cmd.format(ctr=c) for c in ("FETCH_SIZE", "WRITE_SIZE")]}
    with open(os.path.join(PROFILE_DIR, "pmc_traffic.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


def measure_ceilings(v, torch, L: Layout, npes: int):
    """Measured ceilings the rows are compared with (outside the timed
    steps): the achievable copy rate (the copy probe, 4 GiB), agent-scope
    random atomics on a 4 MiB and a 1 GiB table, and signal ping-pong
    one-way latency for one pair and for all pairs, with the two sides of a
    pair on one XCD or on two."""
    stream = torch.cuda.current_stream()

    def timed(fn, reps=5):
        ts = []
        for r in range(reps + 1):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    out = {}
    n = 4 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    ms = timed(lambda: v.probe_copy(b, a, n))
    out["copy_GB_s"] = round(2 * n / (ms * 1e-3) / 1e9, 1)
    out["hbm_probes_GB_s"] = hbm_probe_rates(v, torch, a, b, n, timed)
    del a, b
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    nupd = 1 << 26
    for tag, lg in (("table_4MiB", 19), ("table_1GiB", 27)):
        table = torch.zeros(1 << lg, dtype=torch.int64, device="cuda")
        ms = timed(lambda: v.probe_atomics(table, 1 << lg, nupd, 0x5EED0003, acc))
        out.setdefault("atomics_G_updates_s", {})[tag] = round(nupd / (ms * 1e-3) / 1e9, 2)
        del table
    torch.cuda.empty_cache()
    hz = v.wallclock_hz()
    rounds = 1000
    npairs_all = npes // 2
    pairs = torch.arange(2 * npairs_all, dtype=torch.int32, device="cuda")
    lat = {}
    for tag, np_, same in (("one_pair_cross_xcd", 1, False), ("one_pair_same_xcd", 1, True),
                           (f"{npairs_all}_pairs_cross_xcd", npairs_all, False),
                           (f"{npairs_all}_pairs_same_xcd", npairs_all, True)):
        rtt = torch.zeros(np_ * rounds, dtype=torch.int64, device="cuda")
        v.pingpong(L.H, L.H + 64, pairs, np_, rounds, 8, same, rtt)
        torch.cuda.synchronize()
        ns = rtt.cpu().numpy().astype(np.float64) / hz * 1e9 / 2
        lat[tag] = {"p50": round(percentile(ns, 50), 1), "p99": round(percentile(ns, 99), 1)}
    out["pingpong_one_way_ns"] = lat
    return out


def hbm_probe_rates(v, torch, a, b, n, timed):
    """HBM rates of the probe kernels on n-byte buffers: three copy schedules
    (read + write bytes), a read-only and a write-only stream, and the copy
    rate those two imply when a copy's reads and writes take turns on the
    memory (2 / (1/read + 1/write))."""
    acc = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = {}
    for name, kind, moved in (("copy_chunked", v.PROBE_COPY_CHUNKED, 2 * n),
                              ("copy_gridstride", v.PROBE_COPY_GRIDSTRIDE, 2 * n),
                              ("copy_tiles", v.PROBE_COPY_TILES, 2 * n),
                              ("read_only", v.PROBE_READ, n), ("write_only", v.PROBE_WRITE, n)):
        ms = timed(lambda: v.probe_hbm(kind, b, a, n, acc=acc))
        out[name] = round(moved / (ms * 1e-3) / 1e9, 1)
    out["copy_bound_from_read_and_write"] = round(2 / (1 / out["read_only"] + 1 / out["write_only"]), 1)
    return out


PCIE_GBS = 64.0   # PCIe 5.0 x16, one direction


def measure_host_paths(v, torch, L: Layout, npes: int):
    """Host-initiated operations (the host default context) and stream-
    triggered puts, outside the timed step: blocking puts and gets of
    256 MiB between pinned host memory and a PE, a 64 MiB put from pageable
    memory, a 256 MiB device-to-device put executed by the copy kernel, the
    round trip of a blocking host fetch_add, and the issue rate of 8-byte
    stream-triggered puts."""
    from paper_2607_08006_amd import host

    def wall(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    base = v.heap_base()
    big = int(256 * MiB * min(1.0, L.scale))
    out = {}
    pinned = torch.empty(big, dtype=torch.uint8).pin_memory()
    pinned.fill_(7)
    s = wall(lambda: host.putmem(base + L.B, pinned, big, 5))
    out["put_pinned_256MiB_GB_s"] = round(big / s / 1e9, 2)
    s = wall(lambda: host.getmem(pinned, base + L.B, big, 5))
    out["get_pinned_256MiB_GB_s"] = round(big / s / 1e9, 2)
    out["pcie_frac_put_get"] = [round(out["put_pinned_256MiB_GB_s"] / PCIE_GBS, 3),
                                round(out["get_pinned_256MiB_GB_s"] / PCIE_GBS, 3)]
    page = np.full(64 * MiB, 3, dtype=np.uint8)
    s = wall(lambda: host.putmem(base + L.B, page, page.size, 6))
    out["put_pageable_64MiB_GB_s"] = round(page.size / s / 1e9, 2)
    del pinned, page
    s = wall(lambda: host.putmem(base + L.B, base + L.A, big, npes - 1))
    out["put_device_256MiB_hbm_GB_s"] = round(2 * big / s / 1e9, 1)
    out["put_device_256MiB_hbm_frac"] = round(out["put_device_256MiB_hbm_GB_s"] / HBM_PEAK_GBS, 4)
    word = base + L.H
    host.int64_atomic_fetch_add(word, 1, 1)
    ts = []
    for _ in range(200):
        t0 = time.perf_counter()
        host.int64_atomic_fetch_add(word, 1, 1)
        ts.append(time.perf_counter() - t0)
    out["fetch_add_round_trip_us"] = {"p50": round(percentile(np.array(ts) * 1e6, 50), 1),
                                      "p99": round(percentile(np.array(ts) * 1e6, 99), 1)}
    stream = torch.cuda.Stream()
    nput = 2000

    def burst():
        for i in range(nput):
            host.putmem_on_stream(base + L.B + 8 * i, base + L.A + 8 * i, 8, i % npes, stream=stream)
        stream.synchronize()
    s = wall(burst, reps=2)
    out["put_on_stream_8B_ops_s"] = round(nput / s, 0)
    return out


def run_config_sections(v, torch):
    """Measurements at the small configurations' own shapes, each on a heap
    of its own: the 4-PE x 1 MiB mixed program (1000 put/get of 8 B - 4 KiB
    and 10^4 fetch_add on 64 counters) at each scope and with the autotuned
    table, in per-op, fused and graph forms; and signal ping-pong with 128
    pairs of 256 PEs."""
    out = {}
    hz = v.wallclock_hz()
    # ---- small mixed program
    v.init(4, 4 * MiB)
    wl = W.small_workload(W.SEED_SMALL)
    res = torch.zeros(wl.n_amo, dtype=torch.int64, device="cuda")
    ops = wl.descs["op"]
    is_op = (ops == W.OP_PUT) | (ops == W.OP_GET) | (ops == W.OP_AMO_FETCH_ADD)
    n_amo = int((ops == W.OP_AMO_FETCH_ADD).sum())
    tune_auto = v.autotune(v.offset(v.malloc(3 * MiB)) + MiB, 2 * MiB, 8, 4096, msgs=1024, reps=5)
    stamps = torch.zeros(len(wl.descs), dtype=torch.int64, device="cuda")
    t0 = torch.zeros(1, dtype=torch.int64, device="cuda")
    init_dev = torch.from_numpy(wl.init).cuda()

    def ev_us(fn, reps=10):
        """Median launch-to-completion time on the stream (HIP events), with
        the heap restored before each launch."""
        ts = []
        for r in range(reps + 1):
            v.heap_view()[:, :wl.heap_bytes].copy_(init_dev)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1) * 1e3)
        return round(float(np.median(ts)), 2)

    small = {}
    for label, scope in (("thread", v.SCOPE_THREAD), ("wave", v.SCOPE_WAVE), ("wg", v.SCOPE_WG),
                         ("default_table", "default"), ("autotuned", None)):
        if scope is None:
            tune = tune_auto
        elif scope == "default":
            tune = v.default_tune()
        else:
            tune = v.default_tune()
            for c in range(len(tune.scope)):
                tune.scope[c] = scope
        plan = v.Plan(wl.descs, tune)
        graph = v.Plan(wl.descs, tune)
        graph.set_stamps(stamps)
        graph.graph_build(1, results=res)
        forms = {}
        for form in ("per_op", "fused", "graph"):
            lat_all, bursts = [], []
            for rep in range(6):
                upload = torch.from_numpy(wl.init).cuda()
                v.heap_view()[:, :wl.heap_bytes].copy_(upload)
                stamps.zero_()
                torch.cuda.synchronize()
                v.stamp(t0)
                if form == "graph":
                    graph.graph_launch()
                else:
                    plan.set_stamps(stamps)
                    (plan.launch_fused if form == "fused" else plan.launch_per_op)(results=res)
                torch.cuda.synchronize()
                if rep == 0:
                    continue
                st_ = stamps.cpu().numpy()[is_op]
                lat = (st_ - int(t0.cpu().numpy()[0])) / hz * 1e6
                lat_all.append(lat)
                bursts.append(float(lat.max()))
            lat = np.concatenate(lat_all)
            burst = float(np.median(bursts))
            forms[form] = {"p50_us": round(percentile(lat, 50), 2), "p99_us": round(percentile(lat, 99), 2),
                           "burst_us": round(burst, 2), "ops_s": round(int(is_op.sum()) / (burst * 1e-6), 0),
                           "amo_Mops_s": round(n_amo / (burst * 1e-6) / 1e6, 2)}
        # The same forms without completion stamps, event-timed: a stamp
        # waits for its operation's stores and writes a timestamp, which
        # weighs on small work-groups more than on large ones.
        bare = v.Plan(wl.descs, tune)
        bare_graph = v.Plan(wl.descs, tune)
        bare_graph.graph_build(1, results=res)
        forms["no_stamps_event_us"] = {"fused": ev_us(lambda: bare.launch_fused(results=res)),
                                       "graph": ev_us(lambda: bare_graph.graph_launch())}
        bare.destroy()
        bare_graph.destroy()
        plan.destroy()
        graph.destroy()
        small[label] = forms
    # The same program from a descriptor table in device memory (index kernel
    # and cursor executor), against the host-built plan, both event-timed
    # from launch to completion on the stream.
    nd = len(wl.descs)
    table = torch.from_numpy(np.ascontiguousarray(wl.descs).view(np.uint8).copy()).cuda()
    res_t = torch.zeros(nd, dtype=torch.int64, device="cuda")
    dplan = v.Plan(wl.descs)
    dgraph = v.Graph(table, nd, 1, results=res_t)

    def ev_ms(fn, reps=8):
        ts = []
        for r in range(reps + 1):
            v.heap_view()[:, :wl.heap_bytes].copy_(torch.from_numpy(wl.init).cuda())
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1) * 1e3)
        return round(float(np.median(ts)), 2)

    small_dev = {"plan_fused_us": ev_ms(lambda: dplan.launch_fused(results=res)),
                 "table_fused_us": ev_ms(lambda: v.launch_batch(table, nd, results=res_t)),
                 "table_graph_us": ev_ms(lambda: dgraph.launch()),
                 "table_per_op_us": ev_ms(lambda: v.launch_per_op(table, nd, results=res_t), reps=2)}
    dgraph.destroy()
    dplan.destroy()
    out["small_program_4pe"] = {"ops": int(is_op.sum()), "fetch_add": n_amo, "heap": "4 PEs x 1 MiB",
                                "device_table_event_timed": small_dev,
                                "autotuned_scopes_log2_3_to_12": [int(tune_auto.scope[c]) for c in range(3, 13)],
                                "autotuned_wg_size": int(tune_auto.wg_size), **small}
    v.finalize()
    # ---- ping-pong, 128 pairs of 256 PEs
    v.init(256, 4 * MiB)
    base = v.offset(v.malloc(4096))
    pairs = torch.arange(256, dtype=torch.int32, device="cuda")
    pp = {}
    for tag, np_, same, rounds in (("one_pair_cross_xcd", 1, False, 100000), ("one_pair_same_xcd", 1, True, 100000),
                                   ("128_pairs_cross_xcd", 128, False, 20000), ("128_pairs_same_xcd", 128, True, 20000)):
        rtt = torch.zeros(np_ * rounds, dtype=torch.int64, device="cuda")
        v.pingpong(base, base + 64, pairs, np_, rounds, 8, same, rtt)
        torch.cuda.synchronize()
        ns = rtt.cpu().numpy().astype(np.float64) / hz * 1e9 / 2
        pp[tag] = {"rounds": rounds, "one_way_p50_ns": round(percentile(ns, 50), 1),
                   "one_way_p99_ns": round(percentile(ns, 99), 1)}
    out["pingpong_256pe"] = pp
    out["device_errors"] = v.device_errors()
    v.finalize()
    # ---- GUPS at full shape: a 2^27-entry int64 table spread over 256 PEs
    # (2^19 entries each), 2^28 updates (80% fetch_xor, 20% fetch_add), the
    # fetched values folded into an accumulator
    v.init(256, 8 * MiB)
    tab = v.offset(v.malloc(4 * MiB))
    for p in range(256):
        v.fill_typed(v.heap_base() + p * v.heap_stride() + tab, 1 << 19, v.DT_INT64,
                     W.subseed(W.SEED_GUPS, W.TAG_HEAP + p))
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    nupd = 1 << 28
    ms = timed_ms(torch, lambda: v.gups(tab, 27, nupd, W.subseed(W.SEED_GUPS, W.TAG_OPS), 5, acc=acc), 3)
    out["gups_256pe"] = {"npes": 256, "table_entries": 1 << 27, "updates": nupd, "mix": "80% fetch_xor, 20% fetch_add",
                         "ms": round(ms, 3), "Mops_s": round(nupd / (ms * 1e-3) / 1e6, 1),
                         "GB_s": round(16 * nupd / (ms * 1e-3) / 1e9, 1),
                         "hbm_frac": round(16 * nupd / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out["device_errors_gups"] = v.device_errors()
    v.finalize()
    return out


def _host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(seconds: float):
    """Time the CPU oracle, unchanged, on bounded samples of the step's rows
    and report algorithmic GB/s, twice: one thread in the defined order, and
    all cores (up to 16 threads, the box's share) on disjoint partitions of
    the same work -- put messages split over the threads, broadcast by byte
    range, reductions by element range -- or, where the oracle has no
    partitioned form (alltoall, GUPS), one independent instance per thread.
    The oracle's C calls release the interpreter lock, so the threads run
    the oracle's arithmetic in parallel."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    model, ncpu = _host_cpu()
    T = max(1, min(16, ncpu))

    def split(n, k):
        b = np.linspace(0, n, k + 1).astype(np.int64)
        return [(int(b[i]), int(b[i + 1])) for i in range(k) if b[i + 1] > b[i]]

    samples = []   # (name, bytes of one instance, single-thread fn, parallel parts, parallel bytes)
    # put ring, 16 MiB messages: 4 PEs x 4 messages
    npes, msg, k = 4, 16 * MiB, 4
    heap = np.zeros((npes, 2 * k * msg), dtype=np.uint8)
    heap[:, :k * msg] = np.frombuffer(np.random.default_rng(1).bytes(npes * k * msg), dtype=np.uint8).reshape(npes, -1)
    recs = [(W.OP_PUT, 0, 0, p, (p + 1) % npes, W.NO_RESULT, j * msg, k * msg + j * msg, msg, 0, 0)
            for p in range(npes) for j in range(k)]
    d = W.descs(recs)
    parts = [(lambda dd=d[a:b]: oracle.run_program(heap, dd)) for a, b in split(len(d), T)]
    samples.append(("put_ring_16MiB 4PEx4msg", 2 * npes * k * msg, lambda: oracle.run_program(heap, d), parts,
                    2 * npes * k * msg))
    # alltoall 1 MiB blocks over 8 PEs
    P, blk = 8, 1 * MiB
    h2 = [np.zeros((P, 2 * P * blk), dtype=np.uint8) for _ in range(T)]
    samples.append(("alltoall_1MiB 8PE", 2 * P * P * blk, lambda: oracle.alltoall(h2[0], P * blk, 0, blk),
                     [(lambda h=h: oracle.alltoall(h, P * blk, 0, blk)) for h in h2], T * 2 * P * P * blk))
    # broadcast 32 MiB over 8 PEs
    bc = 32 * MiB
    h3 = np.zeros((P, 2 * bc), dtype=np.uint8)
    samples.append(("broadcast_32MiB 8PE", bc * (P + 1), lambda: oracle.broadcast(h3, bc, 0, bc, 0),
                    [(lambda a=a, b=b: oracle.broadcast(h3, bc + a, a, b - a, 0)) for a, b in split(bc, T)],
                    bc * (P + 1)))
    # reductions 2^18 elements over 8 PEs
    nr = 1 << 18
    for dt, es, gen, tag in ((oracle.DT_INT64, 8, W.coll_i64, "i64"), (oracle.DT_FP32, 4, W.coll_f32, "f32")):
        h = np.zeros((P, 2 * nr * es), dtype=np.uint8)
        for p in range(P):
            h[p, :nr * es] = gen(5, p, nr).view(np.uint8)
        samples.append((f"reduce_sum_{tag} 2^18 8PE", 2 * P * nr * es,
                        (lambda h=h, dt=dt, es=es: oracle.reduce(h, dt, oracle.RO_SUM, nr * es, 0, nr)),
                        [(lambda h=h, dt=dt, es=es, a=a, b=b: oracle.reduce(h, dt, oracle.RO_SUM, nr * es + a * es,
                                                                             a * es, b - a)) for a, b in split(nr, T)],
                        2 * P * nr * es))
    # GUPS 2^22 updates on 2^20 entries
    idx, val, is_add = W.gups_updates(W.SEED_GUPS, 0, 1 << 22, 20)
    tables = [np.zeros(1 << 20, dtype=np.int64) for _ in range(T)]
    samples.append(("gups 2^22 upd", 16 << 22, lambda: oracle.gups(tables[0], idx, val, is_add),
                    [(lambda tb=tb: oracle.gups(tb, idx, val, is_add)) for tb in tables], T * (16 << 22)))

    def leg(par: bool, budget: float):
        tot_b, tot_t, reps = 0, 0.0, 0
        with ThreadPoolExecutor(max_workers=T) as ex:
            for _, b1, fn, parts, bp in samples:     # untimed: first touch of every page
                if par:
                    for f in [ex.submit(p) for p in parts]:
                        f.result()
                else:
                    fn()
            t_end = time.perf_counter() + budget
            while time.perf_counter() < t_end or reps == 0:
                for _, b1, fn, parts, bp in samples:
                    t0 = time.perf_counter()
                    if par:
                        for f in [ex.submit(p) for p in parts]:
                            f.result()
                    else:
                        fn()
                    tot_t += time.perf_counter() - t0
                    tot_b += bp if par else b1
                reps += 1
        return tot_b / tot_t / 1e9, tot_t, reps

    g1, t1, r1 = leg(False, seconds / 2)
    gp, tp, rp = leg(True, seconds / 2)
    names = "; ".join(s[0] for s in samples)
    return {"value": round(gp, 3), "unit": "GB/s", "cores": T, "kind": "oracle",
            "sample": "oracle as written on %d threads, repeated %dx over: %s (algorithmic read+write bytes / time); "
                      "put split by message, broadcast by byte range, reductions by element range, alltoall and "
                      "GUPS one instance per thread" % (T, rp, names),
            "seconds": round(tp, 2), "host_cores": ncpu, "cpu_model": model,
            "single_thread": {"value": round(g1, 3), "unit": "GB/s", "cores": 1, "repeats": r1,
                              "seconds": round(t1, 2)}}


def timed_ms(torch, fn, reps):
    st = torch.cuda.current_stream()
    ts = []
    for r in range(reps + 1):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        if r:
            ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def sweep_launch(v, scope, size):
    """Launch shape per scope from the measured shape sweeps: about one
    work-group per CU (for thread-scope messages up to 32 bytes half as
    many, of 1024 threads, which measured faster); nontemporal copies from 4 KiB (wave) or 64 KiB (work-
    group, grid) up, 8 deep for work-group and grid scope."""
    nt, deep = v.LAUNCH_NONTEMPORAL, v.LAUNCH_DEEP
    if scope == v.SCOPE_THREAD:
        return v.launch_cfg(wgs_per_pe=2, wg_size=1024) if size <= 32 else v.launch_cfg(wgs_per_pe=4, wg_size=256)
    if scope == v.SCOPE_WAVE:
        return v.launch_cfg(wgs_per_pe=4, wg_size=256, flags=nt if size >= 4096 else 0)
    if scope == v.SCOPE_WG:
        return v.launch_cfg(wgs_per_pe=4, wg_size=1024, flags=(nt | deep) if size >= 65536 else 0)
    return v.launch_cfg(wgs_per_pe=4, wg_size=256, flags=nt | deep)


def run_sweep(v, torch, args):
    """The put/get bandwidth sweep: 8 B - 64 MiB, thread/wavefront/work-group
    (and grid for >= 1 MiB) scopes, ring and derangement, put and get; each
    round is min(2^28 / s, 2^14) messages per PE followed by quiet."""
    npes = args.npes
    v.init(npes, args.heap_mib * MiB)
    A = v.offset(v.malloc(256 * MiB))
    B = v.offset(v.malloc(256 * MiB))
    for p in range(npes):
        pe = v.heap_base() + p * v.heap_stride()
        v.fill_random(pe + A, 256 * MiB, W.subseed(W.SEED_SWEEP, W.TAG_HEAP + p))
    torch.cuda.synchronize()
    tg = {pat: torch.from_numpy(W.pattern_targets(pat, npes).astype(np.int32)).cuda() for pat in ("ring", "perm")}
    points = []
    for size in W.sweep_sizes():
        k = W.msgs_per_pe(size)
        scopes = [v.SCOPE_THREAD, v.SCOPE_WAVE, v.SCOPE_WG] + ([v.SCOPE_GRID] if size >= MiB else [])
        for scope in scopes:
            lc = sweep_launch(v, scope, size)
            for pat in ("ring", "perm"):
                for op in (v.OP_PUT, v.OP_GET):
                    ms = timed_ms(torch, lambda: v.rma_pattern(op, scope, tg[pat], A, B, size, k, launch=lc),
                                  1 if (scope == v.SCOPE_THREAD and size >= MiB) else 3)
                    payload = npes * k * size
                    points.append({"size": size, "scope": ["thread", "wave", "wg", "grid"][scope], "pattern": pat,
                                   "op": "put" if op == v.OP_PUT else "get", "msgs_per_pe": k, "ms": round(ms, 4),
                                   "payload_GB_s": round(payload / ms / 1e6, 2),
                                   "hbm_GB_s": round(2 * payload / ms / 1e6, 2),
                                   "hbm_frac": round(2 * payload / ms / 1e6 / HBM_PEAK_GBS, 4),
                                   "Mops_s": round(npes * k / ms / 1e3, 3)})
                    log(json.dumps(points[-1]))
    v.finalize()
    return {"mode": "sweep", "npes": npes, "heap_bytes_per_pe": args.heap_mib * MiB, "points": points}


def run_serve(v, torch, args):
    return serve_compare(v, torch, args.serve_requests, args.serve_wg, args.serve_chunk_kib << 10)


def serve_compare(v, torch, n, serve_wg=PROGRESS_WG, serve_chunk=PROGRESS_CHUNK):
    """Open-loop serving: saturated burst first, then Poisson arrivals at 50%
    and 80% of the persistent kernel's saturated byte rate, on 128 PEs x
    512 MiB with a 64 GiB budget; every trace runs in four forms: the
    persistent progress kernel, windowed batches replayed from a graph or
    launched fused, and one launch per request.  Latency percentiles drop
    the first 5% of requests (warm-up)."""
    npes, heap = 128, 512 * MiB
    v.init(npes, heap)
    src = v.offset(v.malloc(128 * MiB))
    region = v.offset(v.malloc(384 * MiB))
    for p in range(npes):
        v.fill_random(v.heap_base() + p * v.heap_stride() + src, 128 * MiB, W.subseed(W.SEED_SERVE, W.TAG_HEAP + p))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    budget = 64 << 30

    def once(reqs, form="persistent"):
        v.heap_view()[:, region + 288 * MiB:region + 384 * MiB].zero_()
        torch.cuda.synchronize()
        if form == "per_op":
            dst, lat, comps, stats = v.serve_run_per_op(reqs, 8, region, 384 * MiB, budget, chunk_bytes=PER_OP_CHUNK)
            torch.cuda.synchronize()
            return lat, comps, stats
        if form in ("batched_fused", "batched_graph"):
            dst, lat, comps, stats = v.serve_run_batched(reqs, 8, region, 384 * MiB, budget, window_us=WINDOW_US,
                                                         use_graph=form == "batched_graph",
                                                         chunk_bytes=PROGRESS_CHUNK, wg_size=PROGRESS_WG)
            torch.cuda.synchronize()
            return lat, comps, stats
        v.progress_start(nwg=0, wg_size=serve_wg, ring_slots=4096, chunk_bytes=serve_chunk, stream=side)
        try:
            dst, lat, comps, stats = v.serve_run(reqs, 8, region, 384 * MiB, budget)
        finally:
            v.progress_stop(60000)
            side.synchronize()
        return lat, comps, stats

    def summary(reqs, lat, stats, warm=0):
        pay = sum(r.nbytes for r in reqs)
        amo = sum(r.nbytes // 8 for r in reqs if r.op == W.OP_AMO_FETCH_ADD)
        l = lat[warm:] / 1e3
        return {"GB_s": round(pay / stats.wall_s / 1e9, 2), "req_s": round(len(reqs) / stats.wall_s, 1),
                "amo_Mops_s": round(amo / stats.wall_s / 1e6, 1),
                "p50_us": round(percentile(l, 50), 1), "p99_us": round(percentile(l, 99), 1),
                "admission_waits": int(stats.admission_waits), "max_reserved_bytes": int(stats.max_reserved_bytes)}

    burst = serve_trace(v, npes, n, 1e12, 128 * MiB, W.SEED_SERVE)
    payload = sum(r.nbytes for r in burst)
    lat, comps, stats = once(burst)
    b_sat = payload / stats.wall_s
    mean_size = payload / n
    forms = ("persistent", "batched_graph", "batched_fused", "per_op")
    out = {"mode": "serve", "npes": npes, "heap_bytes_per_pe": heap, "budget_bytes": budget, "requests": n,
           "sizes": "log-uniform 64 B - 16 MiB; kinds put/get/fetch_add uniform; 8 producer lanes",
           "warmup_discarded": n // 20, "batch_window_us": WINDOW_US,
           "persistent": {"saturated": summary(burst, lat, stats)}}
    for form in forms[1:]:
        lat, comps, stats = once(burst, form)
        out[form] = {"saturated": summary(burst, lat, stats)}
    log(json.dumps({f: out[f]["saturated"] for f in forms}))
    warm = n // 20
    for rho in (0.5, 0.8):
        lam = rho * b_sat / mean_size
        reqs = serve_trace(v, npes, n, lam, 128 * MiB, W.SEED_SERVE)
        for form in forms:
            lat, comps, stats = once(reqs, form)
            out[form][f"rho_{rho}"] = dict(offered_GB_s=round(rho * b_sat / 1e9, 2), **summary(reqs, lat, stats, warm))
            log(json.dumps({form: {f"rho_{rho}": out[form][f"rho_{rho}"]}}))
    v.finalize()
    return out


def main():
    args = parse()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args.probe_copy_mib or 1024)
        return
    if args.gpus != 1:
        msg = ("virtual PEs are slices of one device's symmetric heap, so the benchmark runs on one GPU; "
               "--gpus must be 1")
        print(msg, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2607_08006_amd as v

    torch.cuda.set_device(0)
    if args.sweep or args.serve or args.configs_only:
        if args.configs_only:
            rec = {"mode": "configs", "configs": run_config_sections(v, torch)}
        else:
            rec = run_sweep(v, torch, args) if args.sweep else run_serve(v, torch, args)
        line = json.dumps(rec)
        print(line, flush=True)
        if args.out:
            with open(args.out, "w") as f:
                f.write(line + "\n")
        return
    npes = args.npes
    want = set(r for r in args.rows.split(",") if r)
    log(f"init {npes} PEs x {args.heap_mib} MiB")
    if v.initialized():
        v.finalize()
    v.init(npes, args.heap_mib * MiB)
    heap_stride = v.heap_stride()
    L = Layout(v, args.heap_mib)
    fill_heap(v, L, npes)
    torch.cuda.synchronize()
    rows = build_rows(v, torch, L, npes, want)
    do_batch = not want or "batch" in want
    if do_batch:
        log("building batch plan")
        B = batch_setup(v, torch, L, npes)
    do_serve = not want or "serve" in want
    if do_serve:
        S = serve_setup(v, torch, L, npes)
    stream = torch.cuda.current_stream()

    def one_step(record):
        for r in rows:
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            r.fn()
            if record:
                e1.record(stream)
                r._ev = (e0, e1)
        lat = None
        if do_batch:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            batch_step(v, B)
            e1.record(stream)
            if record:
                torch.cuda.synchronize()
                lat = (batch_latencies(v, B), (e0, e1))
        if do_serve:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            slat, scomps, sstats = serve_step(v, S)
            if record:
                lat = (lat, (slat, scomps, sstats, time.perf_counter() - t0))
        return lat

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()
    log(f"timed {args.steps} steps")
    lats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    serve_recs = []
    for _ in range(args.steps):
        lat = one_step(True)
        if do_serve:
            lat, srec = lat
            serve_recs.append(srec)
        for r in rows:
            r._evs = getattr(r, "_evs", []) + [r._ev]
        lats.append(lat)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    errs = v.device_errors()
    for r in rows:
        r.ms = [a.elapsed_time(b) for a, b in r._evs]
    ms_per_step = wall * 1e3 / args.steps
    step_bytes = sum(r.bytes for r in rows)
    out_rows = {}
    for r in rows:
        ms = float(np.mean(r.ms))
        d = {"ms": round(ms, 4)}
        if r.bytes:
            d["GB_s"] = round(r.bytes / (ms * 1e-3) / 1e9, 2)
            d["hbm_frac"] = round(d["GB_s"] / HBM_PEAK_GBS, 4)
            tr = pmc_traffic(r.kernel, r.bytes) if r.kernel else None
            if tr:
                # counter-measured HBM bytes per launch against the algorithmic bytes
                d["pmc_traffic_bytes"] = tr
                d["traffic_over_algorithmic"] = round(tr / r.bytes, 4)
        if r.ops:
            d["Mops_s"] = round(r.ops / (ms * 1e-3) / 1e6, 2)
        out_rows[r.name] = d
    latency = None
    if do_batch:
        step_bytes += 3 * B["bytes"]
        forms = {}
        for k in ("fused", "per_op", "graph"):
            allv = np.concatenate([a[0][k] for a in lats])
            last = np.array([a[0][k].max() for a in lats])
            forms[k] = {"p50_us": round(percentile(allv, 50), 2), "p99_us": round(percentile(allv, 99), 2),
                        "burst_us": round(float(np.median(last)), 2),
                        "Mops_s": round(B["nops"] / (float(np.median(last)) * 1e-6) / 1e6, 3)}
        batch_ms = float(np.mean([a[1][0].elapsed_time(a[1][1]) for a in lats]))
        out_rows["batch_all_forms"] = {"ms": round(batch_ms, 4)}
        latency = {
            "burst_ops": B["nops"], "npes": npes,
            "definition": "a burst of mixed put/get (8 B-4 KiB) and fetch_add submitted together; an op's latency "
                          "is device wall-clock time from the burst's start on the stream to the op's completion "
                          "(its stores completed device-wide). per_op = one kernel launch per op; fused = one "
                          "launch; graph = the fused launch replayed from a hipGraph",
            **forms,
        }
    serving = None
    if do_serve:
        hz = v.wallclock_hz()
        lat_all = np.concatenate([r[0] for r in serve_recs]) / 1e3
        svc = np.concatenate([np.array([(c.t_end - c.t_start) for c in r[1]], dtype=np.float64) for r in serve_recs])
        svc = svc / hz * 1e6
        wall = float(np.median([r[3] for r in serve_recs]))
        nbytes = S["bytes"]
        step_bytes += nbytes
        st_ = serve_recs[-1][2]
        out_rows["serve_progress_kernel"] = {"ms": round(wall * 1e3, 3),
                                             "GB_s": round(nbytes / wall / 1e9, 2),
                                             "req_s": round(len(S["reqs"]) / wall, 1)}
        serving = {"requests": len(S["reqs"]), "arrivals": "burst at t=0 over 8 producer lanes",
                   "sizes": "log-uniform 64 B - 16 MiB; kinds put/get/fetch_add",
                   "budget_bytes": S["budget"], "max_reserved_bytes": int(st_.max_reserved_bytes),
                   "admission_waits": int(st_.admission_waits),
                   "latency_us": {"p50": round(percentile(lat_all, 50), 1), "p99": round(percentile(lat_all, 99), 1)},
                   "device_service_us": {"p50": round(percentile(svc, 50), 1), "p99": round(percentile(svc, 99), 1)}}
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    dom = max((r for r in rows if r.bytes), key=lambda r: float(np.sum(r.ms)), default=None)
    roof = None
    if dom is not None:
        avg_ms = float(np.mean(dom.ms))
        achieved = dom.bytes / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": pmc_traffic(dom.kernel or dom.name, dom.bytes),
                "kernel": dom.kernel or dom.name, "row": dom.name, "algorithmic_bytes_per_launch": dom.bytes,
                "avg_launch_ms": round(avg_ms, 4)}
    gups = out_rows.get("gups_fetch_xor_add", {})
    rec = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"{npes} virtual PEs x {args.heap_mib} MiB symmetric heap each (slices "
                               f"{heap_stride // MiB} MiB apart); one pass of every "
                               "hot-path row (put/get at thread (8 B, 64 B), wavefront (4 KiB), work-group "
                               "(16 MiB) and grid (64 MiB) scope on ring and derangement patterns, 2^26 random "
                               "fetch_xor/fetch_add on a 2^27-entry int64 table, signal ping-pong 32 pairs x 200, "
                               "100 barriers, broadcast 256 MiB, fcollect 4 MiB, alltoall 1 MiB blocks, sum/max "
                               "reduce 2^24 elements int64/fp32/bf16, a 2000-op mixed batch in fused, per-op and "
                               "graph forms, and a 1000-request serving burst on the persistent progress kernel)",
                   "npes": npes, "heap_bytes_per_pe": args.heap_mib * MiB, "heap_stride_bytes": heap_stride,
                   "step_algorithmic_bytes": step_bytes},
        "amo_Mops_s": gups.get("Mops_s"),
        "rows": out_rows,
        "latency": latency,
        "serving": serving,
        "roofline": roof,
        "device_errors": errs,
    }
    if not want and not args.no_extras:
        log("ceilings")
        ceil = measure_ceilings(v, torch, L, npes)
        rec["ceilings"] = ceil
        for name, r in out_rows.items():
            if "hbm_frac" in r and r["GB_s"] > 1000:
                r["frac_of_copy_ceiling"] = round(r["GB_s"] / ceil["copy_GB_s"], 4)
        if "gups_fetch_xor_add" in out_rows:
            g = out_rows["gups_fetch_xor_add"]["Mops_s"] / 1e3
            out_rows["gups_fetch_xor_add"]["frac_of_atomic_ceiling_1GiB"] = round(
                g / ceil["atomics_G_updates_s"]["table_1GiB"], 4)
        rec["errors_after_ceilings"] = v.device_errors()
        log("host-initiated paths")
        rec["host_paths"] = measure_host_paths(v, torch, L, npes)
        rec["errors_after_host_paths"] = v.device_errors()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    if args.hbm_probe_mib:
        n = args.hbm_probe_mib * MiB
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        acc = torch.zeros(1, dtype=torch.int32, device="cuda")
        for kind in (v.PROBE_COPY_GRIDSTRIDE, v.PROBE_COPY_TILES, v.PROBE_READ, v.PROBE_WRITE):
            v.probe_hbm(kind, b, a, n, acc=acc)
        torch.cuda.synchronize()
        rec["hbm_probe_bytes"] = n
        del a, b
    if args.probe_copy_mib:
        n = args.probe_copy_mib * MiB
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        v.probe_copy(b, a, n)
        torch.cuda.synchronize()
        rec["probe_copy_bytes"] = n
    v.finalize()
    if not want and not args.no_extras:
        log("configuration sections")
        rec["configs"] = run_config_sections(v, torch)
        g = rec["configs"]["gups_256pe"]
        rec["amo_Mops_s"] = g["Mops_s"]
        rec["amo_workload"] = "GUPS: 2^27 int64 entries over 256 virtual PEs, 2^28 updates (80% fetch_xor, 20% fetch_add)"
        if "ceilings" in rec:
            g["frac_of_atomic_ceiling_1GiB"] = round(g["Mops_s"] / 1e3 / rec["ceilings"]["atomics_G_updates_s"]["table_1GiB"], 4)
        log("serving comparison at offered load")
        rec["serving_offered_load"] = serve_compare(v, torch, args.serve_requests)
    line = json.dumps(rec)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
