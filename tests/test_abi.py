"""CPU-side checks of the C-ABI boundary: the library loads, exports every
function include/vshmem.h declares, the binding declares exactly those, and
host-side argument and state errors are reported without touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vshmem.h")
LIB = os.path.join(ROOT, "paper_2607_08006_amd", "libvshmem.so")


def _ensure_built():
    if not os.path.exists(LIB):
        import importlib.util
        spec = importlib.util.spec_from_file_location("vbuild", os.path.join(ROOT, "paper_2607_08006_amd", "build.py"))
        m = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(m)
        m.build()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    src = re.sub(r"#[^\n]*", "", src)
    # drop typedef/struct bodies
    src = re.sub(r"typedef\s+struct\s+\w*\s*\{.*?\}\s*\w+\s*;", "", src, flags=re.S)
    names = re.findall(r"\b([A-Za-z_]\w*)\s*\([^;{}]*\)\s*;", src)
    return sorted(set(n for n in names if n.startswith("shmem")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("shmemx_init_attach", "shmem_init", "shmem_finalize", "shmem_n_pes", "shmem_my_pe",
                 "shmem_malloc", "shmemg_malloc", "shmem_free", "shmem_ptr", "shmem_query_capabilities",
                 "shmemx_rma_pattern", "shmemx_gups", "shmemx_pingpong", "shmemx_barrier_launch",
                 "shmemx_broadcastmem_launch", "shmemx_fcollectmem_launch", "shmemx_alltoallmem_launch",
                 "shmemx_reduce_launch", "shmemx_plan_create", "shmemx_plan_launch_fused",
                 "shmemx_plan_launch_per_op", "shmemx_plan_graph_build", "shmemx_autotune",
                 "shmemx_progress_start", "shmemx_progress_submit", "shmemx_serve_run",
                 "shmemx_launch_batch", "shmemx_launch_per_op", "shmemx_graph_build", "shmemx_graph_launch",
                 "shmemx_graph_destroy", "shmemx_tune_set", "shmemx_tune_get"):
        assert must in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_binding_declares_exactly_the_header():
    _ensure_built()
    from paper_2607_08006_amd import _native
    assert sorted(_native.SIGNATURES) == declared_functions()


STRUCTS = {"Desc": "shmemx_desc_t", "Caps": "shmemx_caps_t", "Launch": "shmemx_launch_t", "Tune": "shmemx_tune_t",
           "ProgressCfg": "shmemx_progress_cfg_t", "Completion": "shmemx_completion_t", "Request": "shmemx_request_t",
           "ServeStats": "shmemx_serve_stats_t", "DTeam": "shmemx_dteam_t"}


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes record has the size and field offsets the C compiler
    gives the header's struct of the same name."""
    from paper_2607_08006_amd import _native
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "vshmem.h"', "int main(void) {"]
    for py, c in STRUCTS.items():
        lines.append(f'  printf("{py} .sizeof %zu\\n", sizeof({c}));')
        for f, _ in getattr(_native, py)._fields_:
            lines.append(f'  printf("{py} {f} %zu\\n", offsetof({c}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(x.split()[:2]): int(x.split()[2]) for x in out if x}
    for py in STRUCTS:
        cls = getattr(_native, py)
        assert got[(py, ".sizeof")] == ctypes.sizeof(cls), py
        for f, _ in cls._fields_:
            assert got[(py, f)] == getattr(cls, f).offset, (py, f)


def test_desc_record_matches_workload_dtype():
    from paper_2607_08006_amd import _native
    assert ctypes.sizeof(_native.Desc) == 64
    import workload
    assert workload.DESC_DTYPE.itemsize == ctypes.sizeof(_native.Desc)
    for f, _ in _native.Desc._fields_:
        name = {"issuer_pe": "issuer", "target_pe": "target"}.get(f, f)
        assert workload.DESC_DTYPE.fields[name][1] == getattr(_native.Desc, f).offset


def test_calls_before_init_fail_cleanly():
    _ensure_built()
    import paper_2607_08006_amd as v
    lib = v.lib
    assert lib.shmem_n_pes() == 0
    assert lib.shmem_my_pe() == -1
    assert not lib.shmem_malloc(64)
    assert lib.shmemx_last_error() == v.ERR_STATE
    assert lib.shmemx_rma_pattern(1, 2, None, 0, 0, 8, 1, 8, 8, None, None) == v.ERR_STATE
    assert lib.shmemx_gups(0, 10, 1, 1, 5, None, None, None, None) == v.ERR_STATE
    caps = v.Caps()
    assert lib.shmem_query_capabilities(0, ctypes.byref(caps)) == v.ERR_STATE
    assert lib.shmemx_device_errors() == v.ERR_STATE
    assert lib.shmemx_team_device(0, ctypes.byref(v.DTeam())) == v.ERR_STATE
    # host-initiated and stream-triggered calls refuse before init without touching a device
    lib.shmemx_clear_last_error()
    assert lib.shmemx_last_error() == v.OK
    lib.shmem_putmem(None, None, 8, 0)
    assert lib.shmemx_last_error() == v.ERR_STATE
    lib.shmemx_clear_last_error()
    assert lib.shmem_int64_atomic_fetch_add(None, 1, 0) == 0 and lib.shmemx_last_error() == v.ERR_STATE
    assert lib.shmem_broadcastmem(0, None, None, 8, 0) == v.ERR_STATE
    assert lib.shmem_team_sync(0) == v.ERR_STATE
    assert lib.shmemx_putmem_on_stream(None, None, 8, 0, None) == v.ERR_STATE
    assert lib.shmemx_barrier_all_on_stream(None) == v.ERR_STATE
    assert lib.shmemx_quiet_on_stream(None) == v.ERR_STATE
    assert lib.shmemx_init_attach(None, 1 << 21, 1, None) == v.ERR_ARG
    assert lib.shmemx_init_attach(ctypes.c_void_p(1 << 21), 3 << 20, 2, None) == v.ERR_ARG   # odd split
    assert lib.shmemx_strerror(v.ERR_TIMEOUT).decode() == "timed out"
    assert v.version().startswith("vshmem")


def test_tune_table_json_round_trip(tmp_path):
    _ensure_built()
    import paper_2607_08006_amd as v
    t = v.default_tune()
    assert t.wg_size == 256 and t.scope[3] == v.SCOPE_THREAD and t.scope[12] == v.SCOPE_WAVE
    assert t.scope[20] == v.SCOPE_WG and t.chunk[21] == 256 << 10
    t.wg_size = 512
    t.scope[17] = v.SCOPE_WAVE
    t.chunk[25] = 1 << 20
    path = str(tmp_path / "tune.json")
    v.tune_save(t, path)
    u = v.tune_load(path)
    assert u.wg_size == 512 and u.scope[17] == v.SCOPE_WAVE and u.chunk[25] == 1 << 20
    assert list(u.scope) == list(t.scope) and list(u.chunk) == list(t.chunk)
    import json
    d = json.load(open(path))
    assert d["wg_size"] == 512 and len(d["classes"]) == 40


def test_tune_load_refuses_other_devices_and_invalid_tables(tmp_path):
    """A saved table names the device it was measured on; loading it where
    another device (or none, or no key) is seen, or loading an invalid
    table, fails with SHMEMX_ERR_ARG."""
    _ensure_built()
    import json
    import paper_2607_08006_amd as v
    path = str(tmp_path / "tune.json")
    v.tune_save(v.default_tune(), path)
    d = json.load(open(path))
    for name, edit in [("other device", lambda x: x.update(device="gfx000:other")),
                       ("no device key", lambda x: x.pop("device")),
                       ("bad work-group size", lambda x: x.update(wg_size=100)),
                       ("bad scope", lambda x: x["classes"][5].update(scope=9))]:
        e = json.loads(json.dumps(d))
        edit(e)
        bad = str(tmp_path / "bad.json")
        json.dump(e, open(bad, "w"))
        with pytest.raises(v.VshmemError) as err:
            v.tune_load(bad)
        assert err.value.code == v.ERR_ARG, name


def test_heap_stride_policy():
    """shmemx_heap_stride_for needs no device: the smallest stride is the
    request plus the 64 KiB scratch tail rounded to 2 MiB; the spread stride
    moves slices at or just above a power of two (from 64 MiB) to 1.5 times
    it plus 2 MiB, and leaves every other size alone."""
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    f = lib.shmemx_heap_stride_for
    f.restype, f.argtypes = ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_int]
    MiB = 1 << 20
    for b in (1, 4 * MiB, 62 * MiB, 64 * MiB, 512 * MiB, 1024 * MiB - 65536, 1024 * MiB, 1536 * MiB, 1600 * MiB,
              3 * 1024 * MiB, 40 * 1024 * MiB):
        lo, sp = f(b, 0), f(b, 1)
        assert lo >= b + 65536 and lo % (2 * MiB) == 0 and lo - (b + 65536) < 2 * MiB
        assert sp >= lo and sp % (2 * MiB) == 0
        p2 = 1 << (lo.bit_length() - 1)
        want = p2 + p2 // 2 + 2 * MiB if lo >= 64 * MiB and lo < p2 + p2 // 2 + 2 * MiB else lo
        assert sp == want, (b, lo, sp)
    assert f(1024 * MiB, 1) == 1538 * MiB and f(512 * MiB, 1) == 770 * MiB and f(4 * MiB, 1) == 6 * MiB
    assert f(1600 * MiB, 1) == 1602 * MiB and f(1 << 51, 1) == 0 and f(1 << 51, 0) == 0
