"""Host-side logic of bench.py (no GPU): the JSON contract pieces that do not
need a device, and the profile summariser that turns rocprofv3 CSV output
into the committed traffic figures."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_gpus_above_one_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_short_kernel_names():
    assert bench._short_kernel("void (anonymous namespace)::k_rma_pattern<2, true, true, 8>(shmemx_dctx_pub_t, int)") \
        == "k_rma_pattern<2,true,true,8>"
    assert bench._short_kernel("(anonymous namespace)::k_plan_one(shmemx_dctx_pub_t)") == "k_plan_one"


def test_summarize_profiles_scales_counters_by_the_copy_probe(tmp_path, monkeypatch):
    prof = tmp_path / "prof"
    kib = 1024
    # the probe reads and writes 1 GiB; FETCH_SIZE reports half of what was read
    probe_fetch, probe_write = 524288.0, 1048576.0
    kernel = "void (anonymous namespace)::k_rma_pattern<2, true, true, 8>(shmemx_dctx_pub_t)"
    rows = []
    for ctr, probe_v, k_v in (("FETCH_SIZE", probe_fetch, 8388608.0), ("WRITE_SIZE", probe_write, 16777216.0)):
        rows = [{"Kernel_Name": "(anonymous namespace)::k_probe_copy(v4u*)", "Counter_Name": ctr, "Counter_Value": probe_v}]
        rows += [{"Kernel_Name": kernel, "Counter_Name": ctr, "Counter_Value": k_v} for _ in range(3)]
        _write_csv(str(prof / f"pmc_{ctr}" / "pmc_counter_collection.csv"), rows)
    _write_csv(str(prof / "trace" / "bench_kernel_stats.csv"),
               [{"Name": kernel, "Calls": 4, "TotalDurationNs": 24e6, "AverageNs": 6e6, "MinNs": 5.9e6,
                 "MaxNs": 6.1e6, "Percentage": 50.0}])
    out = tmp_path / "profiles"
    out.mkdir()
    monkeypatch.setattr(bench, "PROFILE_DIR", str(out))
    bench.summarize_profiles(str(prof), 1024)
    d = json.load(open(out / "pmc_traffic.json"))
    assert d["probe"]["fetch_scale"] == pytest.approx(2.0)
    assert d["probe"]["write_scale"] == pytest.approx(1.0)
    k = d["kernels"]["k_rma_pattern<2,true,true,8>"]
    assert k["fetch_bytes"] == 16 << 30 and k["write_bytes"] == 16 << 30
    assert k["source_digest"] == bench.kernel_digest("k_rma_pattern<2,true,true,8>")
    assert (out / "bench_step_64pe_kernel_stats.md").read_text().count("k_rma_pattern<2,true,true,8>") == 1
    # the roofline reads it back while the sources are unchanged, and drops it otherwise
    assert bench.pmc_traffic("k_rma_pattern<2,true,true,8>", 0) == 32 << 30
    d["kernels"]["k_rma_pattern<2,true,true,8>"]["source_digest"] = "stale"
    json.dump(d, open(out / "pmc_traffic.json", "w"))
    assert bench.pmc_traffic("k_rma_pattern<2,true,true,8>", 0) is None
    assert bench.pmc_traffic("k_gups<false>", 0) is None


def test_kernel_digest_covers_only_known_kernels():
    assert bench.kernel_digest("k_gups<false>") == ""
    a = bench.kernel_digest("k_rma_pattern<2,true,true,8>")
    assert len(a) == 16 and a == bench.kernel_digest("k_rma_pattern<0,false,false,4>")
    assert a != bench.kernel_digest("k_alltoall<true,8>")
