"""Serving on the GPU: each request's pass masks are the same bits alone and
in the mix (continuous batching across requests, several streams), and the
admission, rejection, failure and cancellation paths behave as declared."""

from __future__ import annotations

import ctypes
import random
import time

import numpy as np
import pytest

import synth
import synth.configs as C
from gpu_util import dev, empty, host, log
from paper_1708_04329_amd import grim

pytestmark = pytest.mark.gpu

_hip = None


def d2h(ptr: int, nbytes: int) -> np.ndarray:
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    out = np.empty(nbytes, np.uint8)
    assert _hip.hipMemcpy(out.ctypes.data, ptr, nbytes, 2) == 0
    return out


@pytest.fixture(scope="module")
def world():
    """The serving recipe (100/150/250 bp, e in 2..5 %, q = 5, O = 263) on a 4 Mbp genome."""
    w = C.workload("c5")
    w = C.shrink(w, genome_len=4_000_000, n_reads=20000)
    ref = synth.genome(w.genome)
    rd = synth.reads(w.reads, ref)
    idx = grim.grim_build_index(dev(ref), w.bin_size, w.overlap, w.q, grim.LAYOUT_TM)
    log("serving world", idx.info()["n_bins"], "bins", rd.n, "reads")
    return w, ref, rd, idx


def make_requests(rd, sizes, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for n in sizes:
        start = int(rng.integers(0, rd.n - n + 1))
        sub = rd.subset(np.arange(start, start + n))
        reqs.append(sub)
    return reqs


def rs_host(sub):
    return grim.ReadSet(np.ascontiguousarray(sub.bases), np.ascontiguousarray(sub.offsets),
                        err_permille=np.ascontiguousarray(sub.err_pm.astype(np.uint16)))


def alone(idx, sub):
    import torch
    W = idx.info()["mask_words"]
    m = empty((sub.n, W), torch.uint32)
    grim.grim_filter_scan(idx, grim.ReadSet(dev(sub.bases), dev(sub.offsets),
                                            err_permille=dev(sub.err_pm.astype(np.uint16))), m)
    return host(m)


@pytest.mark.parametrize("policy", [grim.SERVE_CONTINUOUS, grim.SERVE_PLAIN])
def test_served_masks_equal_alone(world, policy):
    w, ref, rd, idx = world
    W = idx.info()["mask_words"]
    rng = random.Random(policy)
    sizes = [rng.choice([1, 2, 7, 100, 513, 2000, 4096, 5000]) for _ in range(40)]
    reqs = make_requests(rd, sizes, seed=11 + policy)
    srv = grim.Server(idx, policy, max_batch_reads=3000, slice_reads=700, n_streams=3, max_inflight=16,
                      arena_bytes=2 << 30)
    tickets = [srv.submit(rs_host(s)) for s in reqs]
    for t, sub in zip(tickets, reqs):
        res = srv.wait(t, 60000)
        assert res["status"] == grim.GRIM_OK, res
        got = d2h(res["mask"], sub.n * W * 4).view(np.uint32).reshape(sub.n, W)
        assert np.array_equal(got, alone(idx, sub)), (t, sub.n)
        srv.release(t)
    st = srv.stats()
    log("policy", policy, {k: st[k] for k in ("completed", "launches", "shared_launches", "max_requests_per_launch",
                                              "p50_ms", "p99_ms", "peak_device_bytes")})
    assert st["completed"] == len(reqs) and st["failed"] == 0
    if policy == grim.SERVE_CONTINUOUS:
        assert st["shared_launches"] > 0 and st["max_requests_per_launch"] > 1   # requests shared launches
    else:
        assert st["launches"] == len(reqs) and st["shared_launches"] == 0       # one launch per request
    srv.destroy()


def test_admission_by_device_memory(world):
    w, ref, rd, idx = world
    W = idx.info()["mask_words"]
    reqs = make_requests(rd, [3000] * 8, seed=5)

    def up(v):
        return (v + 255) // 256 * 256

    # device footprint of one request: inputs, tokens, thresholds, descriptors, status, masks
    n, nb = 3000, max(len(r.bases) for r in reqs)
    per_req = (up(nb) + up((n + 1) * 8) + up(n * 2) + up((nb + 64 * (n + 1) + 64) * 4) + up((n + 1) * 4) +
               up(n * 24) + 256 + up(n * W * 4))
    arena = int(per_req * 2.6)        # room for two requests at a time
    srv = grim.Server(idx, grim.SERVE_CONTINUOUS, arena_bytes=arena, max_inflight=8)
    tickets = [srv.submit(rs_host(s)) for s in reqs]
    for t, sub in zip(tickets, reqs):
        res = srv.wait(t, 60000)
        assert res["status"] == grim.GRIM_OK
        got = d2h(res["mask"], sub.n * W * 4).view(np.uint32).reshape(sub.n, W)
        assert np.array_equal(got, alone(idx, sub))
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == 8 and st["peak_device_bytes"] <= arena
    srv.destroy()


def test_never_fitting_request_is_rejected_others_run(world):
    w, ref, rd, idx = world
    W = idx.info()["mask_words"]
    small, big, small2 = make_requests(rd, [10, 6000, 10], seed=9)
    srv = grim.Server(idx, grim.SERVE_CONTINUOUS, arena_bytes=6000 * W * 4 // 2)
    t1 = srv.submit(rs_host(small))
    with pytest.raises(grim.GrimError) as e:
        srv.submit(rs_host(big))
    assert e.value.code == grim.GRIM_ENOMEM
    t3 = srv.submit(rs_host(small2))
    assert srv.wait(t1, 60000)["status"] == grim.GRIM_OK
    assert srv.wait(t3, 60000)["status"] == grim.GRIM_OK
    assert srv.stats()["rejected"] == 1
    srv.destroy()


def test_invalid_request_fails_others_run(world):
    w, ref, rd, idx = world
    good = make_requests(rd, [50], seed=1)[0]
    bad = synth.reads_from_strings([b"ACG", ref[:120].tobytes()])
    srv = grim.Server(idx, grim.SERVE_CONTINUOUS)
    tb = srv.submit(grim.ReadSet(bad.bases, bad.offsets, err_permille_all=40))
    tg = srv.submit(rs_host(good))
    assert srv.wait(tb, 60000)["status"] == grim.GRIM_EINVAL
    assert srv.wait(tg, 60000)["status"] == grim.GRIM_OK
    # a read the overlap cannot cover (L + E - q > O) fails that request only
    long = synth.reads_from_strings([ref[:400].tobytes()])
    tl = srv.submit(grim.ReadSet(long.bases, long.offsets, err_permille_all=50))
    assert srv.wait(tl, 60000)["status"] == grim.GRIM_EOVERLAP
    with pytest.raises(grim.GrimError):
        srv.submit(grim.ReadSet(good.bases, good.offsets[:1] * 0, err_permille_all=40))   # empty request
    srv.destroy()


def test_cancel_and_shutdown_with_work_queued(world):
    w, ref, rd, idx = world
    reqs = make_requests(rd, [5000, 5000, 5000, 20], seed=3)
    srv = grim.Server(idx, grim.SERVE_CONTINUOUS, max_inflight=1)
    ts = [srv.submit(rs_host(s)) for s in reqs]
    srv.cancel(ts[3])
    res = srv.wait(ts[3], 60000)
    assert res["status"] in (grim.GRIM_ECANCELED, grim.GRIM_OK)
    assert srv.wait(ts[0], 60000)["status"] == grim.GRIM_OK
    # destroy with requests still queued or running: queued ones are cancelled, no hang
    srv.destroy()


def test_poll_and_timeout_paths(world):
    w, ref, rd, idx = world
    sub = make_requests(rd, [200], seed=4)[0]
    srv = grim.Server(idx, grim.SERVE_CONTINUOUS)
    t = srv.submit(rs_host(sub))
    deadline = time.time() + 60
    res = None
    while res is None and time.time() < deadline:
        res = srv.poll(t)
        time.sleep(0.001)
    assert res is not None and res["status"] == grim.GRIM_OK and res["latency_ms"] > 0
    with pytest.raises(grim.GrimError):
        srv.poll(t + 999)
    srv.release(t)
    srv.destroy()


def test_device_reads_equal_host_reads(world):
    """A request whose reads are in device memory is copied at submit and served
    to the same masks as the same reads given in host memory."""
    import torch
    w, ref, rd, idx = world
    W = idx.info()["mask_words"]
    reqs = make_requests(rd, [1, 300, 2500], seed=21)
    srv = grim.Server(idx, grim.SERVE_CONTINUOUS, arena_bytes=1 << 30)
    for sub in reqs:
        d_bases, d_offs, d_e = dev(sub.bases), dev(sub.offsets), dev(sub.err_pm.astype(np.uint16))
        torch.cuda.synchronize()
        t = srv.submit(grim.ReadSet(d_bases, d_offs, err_permille=d_e))
        d_bases.fill_(ord("N"))    # the server holds its own copy after submit
        torch.cuda.synchronize()
        res = srv.wait(t, 60000)
        assert res["status"] == grim.GRIM_OK
        got = d2h(res["mask"], sub.n * W * 4).view(np.uint32).reshape(sub.n, W)
        assert np.array_equal(got, alone(idx, sub)), sub.n
        srv.release(t)
    # device offsets that do not run from 0 to n_bases are rejected at submit
    sub = reqs[1]
    bad = sub.offsets.copy()
    bad[-1] += 1
    with pytest.raises(grim.GrimError) as e:
        srv.submit(grim.ReadSet(dev(sub.bases), dev(bad), err_permille=dev(sub.err_pm.astype(np.uint16))))
    assert e.value.code == grim.GRIM_EINVAL
    srv.destroy()


def test_launch_failure_ends_every_request(world, monkeypatch):
    """After a launch fails (forced from the host: the third launch reports a
    failure without launching), every request ends: those whose launches ran
    keep their masks, the rest fail with GRIM_EDEVICE; later submits are refused
    and the server shuts down without hanging."""
    w, ref, rd, idx = world
    W = idx.info()["mask_words"]
    monkeypatch.setenv("GRIM_SERVE_TEST_FAIL_LAUNCH", "3")
    srv = grim.Server(idx, grim.SERVE_CONTINUOUS, max_batch_reads=1000, slice_reads=500, n_streams=1,
                      max_inflight=4, arena_bytes=1 << 30)
    monkeypatch.delenv("GRIM_SERVE_TEST_FAIL_LAUNCH")
    reqs = make_requests(rd, [400, 900, 2000, 3000, 50, 700, 10, 2500], seed=31)
    tickets = []
    for s in reqs:
        try:
            tickets.append(srv.submit(rs_host(s)))
        except grim.GrimError as e:     # refused once the server has stopped
            assert e.code == grim.GRIM_EDEVICE
            tickets.append(None)
    statuses = []
    for t, sub in zip(tickets, reqs):
        if t is None:
            statuses.append(grim.GRIM_EDEVICE)
            continue
        res = srv.wait(t, 60000)
        statuses.append(res["status"])
        assert res["status"] in (grim.GRIM_OK, grim.GRIM_EDEVICE), res
        if res["status"] == grim.GRIM_OK:
            got = d2h(res["mask"], sub.n * W * 4).view(np.uint32).reshape(sub.n, W)
            assert np.array_equal(got, alone(idx, sub))
    log("statuses after the forced failure", statuses)
    assert statuses[0] == grim.GRIM_OK and statuses.count(grim.GRIM_EDEVICE) >= 1
    with pytest.raises(grim.GrimError) as e:
        srv.submit(rs_host(reqs[0]))
    assert e.value.code == grim.GRIM_EDEVICE
    st = srv.stats()
    assert st["completed"] + st["failed"] == sum(t is not None for t in tickets)
    srv.destroy()
