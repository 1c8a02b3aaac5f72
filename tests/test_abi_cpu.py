"""The C-ABI library loads, exports every declared entry point, matches the
binding's struct layouts and rejects bad arguments before touching a GPU.
No compute call is made here."""

from __future__ import annotations

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1708_04329_amd import grim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grim.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grim_[a-z_]+)\s*\(", src)))


def test_library_loads():
    L = grim.lib()
    assert L.grim_abi_version() == 2


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "grim_filter_scan" in names and "grim_build_index" in names
    out = subprocess.run(["nm", "-D", "--defined-only", grim.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (grim_\w+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(grim.EXPORTS) <= exported


def test_binding_covers_every_declared_function():
    assert set(declared_functions()) == set(grim.EXPORTS)


def test_struct_layouts_match_header():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "grim.h"
int main(void){
 printf("%zu %zu %zu %zu\n", sizeof(grim_index_info_t), sizeof(grim_reads), sizeof(grim_profile_t), sizeof(grim_kernel_time));
 printf("%zu %zu %zu %zu %zu\n", offsetof(grim_reads, err_permille_all), offsetof(grim_reads, flags), offsetof(grim_index_info_t, device), offsetof(grim_index_info_t, bits_bytes), offsetof(grim_index_info_t, ref_bytes));
 return 0; }
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        lines = subprocess.check_output([exe], text=True).split("\n")
    sizes = [int(x) for x in lines[0].split()]
    offs = [int(x) for x in lines[1].split()]
    assert sizes == [ctypes.sizeof(grim.IndexInfo), ctypes.sizeof(grim._Reads), ctypes.sizeof(grim.Profile),
                     ctypes.sizeof(grim.KernelTime)]
    assert offs == [grim._Reads.err_permille_all.offset, grim._Reads.flags.offset, grim.IndexInfo.device.offset,
                    grim.IndexInfo.bits_bytes.offset, grim.IndexInfo.ref_bytes.offset]


def _err(rc):
    return rc, grim.lib().grim_last_error().decode()


def test_build_rejects_bad_arguments_before_device():
    L = grim.lib()
    h = ctypes.c_void_p()
    ref = (ctypes.c_uint8 * 16)(*b"ACGTACGTACGTACGT")
    assert _err(L.grim_build_index(ref, 16, 0, 4, 0, 0, 1, None, ctypes.byref(h)))[0] == grim.GRIM_EINVAL  # q = 0
    assert _err(L.grim_build_index(ref, 16, 0, 4, 0, 8, 1, None, ctypes.byref(h)))[0] == grim.GRIM_EINVAL  # q = 8
    assert _err(L.grim_build_index(ref, 16, 0, 0, 0, 4, 1, None, ctypes.byref(h)))[0] == grim.GRIM_EINVAL  # B = 0
    assert _err(L.grim_build_index(ref, 16, 0, 4, 0, 4, 0, None, ctypes.byref(h)))[0] == grim.GRIM_EINVAL  # layout
    assert _err(L.grim_build_index(ref, 16, 0, 4, 0, 4, 8, None, ctypes.byref(h)))[0] == grim.GRIM_EINVAL
    assert _err(L.grim_build_index(ref, 3, 0, 4, 0, 4, 1, None, ctypes.byref(h)))[0] == grim.GRIM_EINVAL   # G < q
    assert _err(L.grim_build_index(None, 16, 0, 4, 0, 4, 1, None, ctypes.byref(h)))[0] == grim.GRIM_EINVAL
    rc, msg = _err(L.grim_build_index(ref, 16, 0, 4, 0, 4, 1, None, None))
    assert rc == grim.GRIM_EINVAL and "out" in msg


def test_scan_rejects_null_arguments():
    L = grim.lib()
    r = grim._Reads()
    assert L.grim_filter_scan(None, ctypes.byref(r), None, None, 0, None) == grim.GRIM_EINVAL
    assert L.grim_filter_candidates(None, ctypes.byref(r), None, None, 0, None, None, None) == grim.GRIM_EINVAL
    assert L.grim_verify_candidates(None, ctypes.byref(r), None, None, 0, None, None, None, None) == grim.GRIM_EINVAL
    assert L.grim_verify_candidates_bounded(None, ctypes.byref(r), None, None, 0, None, None, None,
                                            None) == grim.GRIM_EINVAL
    n = ctypes.c_uint64()
    assert L.grim_seed_candidates(None, ctypes.byref(r), 2048, 8, None, None, ctypes.byref(n), None) == grim.GRIM_EINVAL
    assert L.grim_seeds_info(None, None) == grim.GRIM_EINVAL
    h = ctypes.c_void_p()
    ref = (ctypes.c_uint8 * 16)(*b"ACGTACGTACGTACGT")
    assert L.grim_seeds_build(ref, 16, 0, 0, None, ctypes.byref(h)) == grim.GRIM_EINVAL    # k = 0
    assert L.grim_seeds_build(ref, 16, 0, 15, None, ctypes.byref(h)) == grim.GRIM_EINVAL   # k = 15
    assert L.grim_seeds_build(None, 16, 0, 12, None, ctypes.byref(h)) == grim.GRIM_EINVAL
    L.grim_seeds_free(None)
    # mask summaries: a NULL or misaligned mask, or a zero row width, fail before any device work
    assert L.grim_mask_summary(None, 1, 4, None, None, None) == grim.GRIM_EINVAL
    buf = ctypes.create_string_buffer(64)
    base = ctypes.addressof(buf)
    assert L.grim_mask_summary(base, 1, 0, None, None, None) == grim.GRIM_EINVAL
    assert L.grim_mask_summary((base + 4) | 1, 1, 4, None, None, None) == grim.GRIM_EINVAL
    assert L.grim_mask_summary(base, 1, 1 << 32, None, None, None) == grim.GRIM_EINVAL
    assert L.grim_mask_summary(None, 0, 4, None, None, None) == grim.GRIM_OK   # nothing to do
    assert L.grim_index_info(None, None) == grim.GRIM_EINVAL
    assert L.grim_index_read(None, 1, 0, 0, None) == grim.GRIM_EINVAL
    L.grim_index_free(None)   # ignored


def test_load_rejects_missing_and_corrupt_files(tmp_path):
    L = grim.lib()
    h = ctypes.c_void_p()
    rc, msg = _err(L.grim_index_load(str(tmp_path / "nope.grim").encode(), None, ctypes.byref(h)))
    assert rc == grim.GRIM_EIO
    bad = tmp_path / "bad.grim"
    bad.write_bytes(b"NOTGRIM!" + b"\0" * 200)
    assert L.grim_index_load(str(bad).encode(), None, ctypes.byref(h)) == grim.GRIM_EIO
    short = tmp_path / "short.grim"
    short.write_bytes(b"GRIMIDX1")
    assert L.grim_index_load(str(short).encode(), None, ctypes.byref(h)) == grim.GRIM_EIO


def test_profile_roundtrip():
    grim.grim_profile_enable(True)
    p = grim.grim_profile_read(reset=True)
    assert p["scan"]["launches"] == 0
    grim.grim_profile_enable(False)


def test_readset_marshalling_checks_dtypes():
    import numpy as np
    rs = grim.ReadSet(bases=np.zeros(10, np.uint8), offsets=np.array([0, 10], np.int32))
    with pytest.raises(TypeError):
        rs._struct()
    rs = grim.ReadSet(bases=np.zeros(10, np.uint8), offsets=np.array([0, 10], np.int64),
                      max_edits=np.array([1], np.uint16), err_permille_all=50)
    s = rs._struct()
    assert s.n_reads == 1 and s.n_bases == 10 and s.on_device == 0 and s.err_permille_all == 50


def test_batching_entry_points_reject_null_arguments():
    L = grim.lib()
    h = ctypes.c_void_p()
    assert L.grim_batcher_create(None, 1, 10, 10, 0, 0, 0, 0, ctypes.byref(h)) == grim.GRIM_EINVAL
    assert L.grim_batcher_submit(None, 0, 1, 1, 0) == grim.GRIM_EINVAL
    assert L.grim_batcher_wait(None, 0) == grim.GRIM_EINVAL
    assert L.grim_batcher_buffers(None, 0, None) == grim.GRIM_EINVAL
    assert L.grim_batcher_stream(None, 0) is None
    L.grim_batcher_free(None)
    r = grim._Reads()
    t = grim.TuneResult()
    assert L.grim_tune(None, ctypes.byref(r), None, None, 0, None, ctypes.byref(t)) == grim.GRIM_EINVAL
    assert L.grim_index_get_config(None, 1, ctypes.byref(t)) == grim.GRIM_EINVAL
    assert L.grim_index_set_config(None, ctypes.byref(t)) == grim.GRIM_EINVAL


def test_serving_entry_points_reject_null_arguments():
    L = grim.lib()
    h = ctypes.c_void_p()
    res = grim.Result()
    st = grim.ServeStats()
    t = ctypes.c_uint64()
    r = grim._Reads()
    assert L.grim_serve_create(None, None, ctypes.byref(h)) == grim.GRIM_EINVAL
    assert L.grim_serve_submit(None, ctypes.byref(r), ctypes.byref(t)) == grim.GRIM_EINVAL
    assert L.grim_serve_poll(None, 1, ctypes.byref(res)) == grim.GRIM_EINVAL
    assert L.grim_serve_wait(None, 1, 0, ctypes.byref(res)) == grim.GRIM_EINVAL
    assert L.grim_serve_release(None, 1) == grim.GRIM_EINVAL
    assert L.grim_serve_cancel(None, 1) == grim.GRIM_EINVAL
    assert L.grim_serve_stats(None, ctypes.byref(st)) == grim.GRIM_EINVAL
    assert L.grim_serve_reset_stats(None) == grim.GRIM_EINVAL
    L.grim_serve_destroy(None)


def test_serving_struct_layouts_match_header():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "grim.h"
int main(void){
 printf("%zu %zu %zu %zu %zu\n", sizeof(grim_serve_config), sizeof(grim_result), sizeof(grim_serve_stats_t), sizeof(grim_tune_result), sizeof(grim_batch_buffers));
 printf("%zu %zu %zu\n", offsetof(grim_serve_config, flags), offsetof(grim_result, latency_ms), offsetof(grim_serve_stats_t, reads_per_s));
 return 0; }
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        lines = subprocess.check_output([exe], text=True).split("\n")
    assert [int(x) for x in lines[0].split()] == [ctypes.sizeof(grim.ServeConfig), ctypes.sizeof(grim.Result),
                                                 ctypes.sizeof(grim.ServeStats), ctypes.sizeof(grim.TuneResult),
                                                 ctypes.sizeof(grim.BatchBuffers)]
    assert [int(x) for x in lines[1].split()] == [grim.ServeConfig.flags.offset, grim.Result.latency_ms.offset,
                                                 grim.ServeStats.reads_per_s.offset]


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on exactly one GPU and says so (before touching any device)."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode == 2 and "exactly one GPU" in p.stderr


def test_probes_build_for_gfx950():
    """The microbenchmarks behind the scan's stated ceilings compile (hipcc cross-compiles here)."""
    import shutil
    if not os.path.exists(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")) and not shutil.which("hipcc"):
        pytest.skip("hipcc is not installed")
    from paper_1708_04329_amd.probes import run
    exe = run.build()
    assert os.path.getsize(exe) > 0
