"""Batching layer on the GPU: tuned and persistent launch shapes change no
output bit, and the graph-captured batcher matches the eager calls and the
oracle on every replay (with eager work in between), for both slots and
varying batch sizes."""

from __future__ import annotations

import ctypes
import random

import numpy as np
import pytest

import synth
import synth.configs as C
from gpu_util import dev, empty, host, log, unpack_mask
from paper_1708_04329_amd import grim

pytestmark = pytest.mark.gpu

_hip = None


def d2h(ptr: int, nbytes: int) -> np.ndarray:
    """Copy device memory the library owns into a numpy array."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    out = np.empty(nbytes, np.uint8)
    assert _hip.hipMemcpy(out.ctypes.data, ptr, nbytes, 2) == 0
    return out


@pytest.fixture(scope="module")
def uneven():
    """The uneven-read candidate recipe (100/150/250 bp, e in 2..5 %, q = 6) on a 6 Mbp genome."""
    w = C.shrink(C.workload("c4"), genome_len=6_000_000, n_reads=6000)
    w.genome.repeat_frac = 0.45
    ref = synth.genome(w.genome)
    rd = synth.reads(w.reads, ref)
    co, cb = synth.candidates(ref, rd, w.bin_size, w.cand_cap, w.cand_k)
    idx = grim.grim_build_index(dev(ref), w.bin_size, w.overlap, w.q, grim.LAYOUT_BM | grim.LAYOUT_TM)
    log("uneven workload pairs", len(cb), "reads", rd.n)
    return w, ref, rd, co, cb, idx


def run_cand(idx, rd, co, cb, ep):
    import torch
    cnt = empty((max(1, len(cb)),), torch.uint16)
    pas = empty((max(1, len(cb)),), torch.uint8)
    grim.grim_filter_candidates(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets), err_permille=dev(ep)),
                                dev(co), dev(cb), cnt, pas)
    return host(cnt)[:len(cb)], host(pas)[:len(cb)]


def test_candidate_launch_shapes_agree(oracle, uneven):
    w, ref, rd, co, cb, idx = uneven
    ep = rd.err_pm.astype(np.uint16)
    want = oracle.scan_candidates(oracle.bits(ref, w.bin_size, w.overlap, w.q), w.q, rd.bases, rd.offsets, co, cb,
                                  err_pm_per_read=ep)
    for coop in (0, 1):
        for waves in (1, 2, 4):
            for pers, gpc in ((0, 2), (1, 1), (1, 4), (1, 16)):
                grim.grim_index_set_config(idx, {"mode": grim.MODE_CANDIDATES, "cand_waves": waves,
                                                 "cand_persistent": pers, "cand_groups_per_cu": gpc,
                                                 "cand_coop": coop})
                got = run_cand(idx, rd, co, cb, ep)
                assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (coop, waves, pers, gpc)


def test_tune_candidates(oracle, uneven, tmp_path, monkeypatch):
    w, ref, rd, co, cb, idx = uneven
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("GRIM_TUNE_CACHE", str(cache))
    ep = rd.err_pm.astype(np.uint16)
    res = grim.grim_tune(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets), err_permille=dev(ep)), dev(co), dev(cb))
    log("tuned candidates", res)
    assert res["mode"] == grim.MODE_CANDIDATES and res["n_tried"] >= 8 and res["best_ms"] > 0
    assert res["best_ms"] <= res["default_ms"] + 1e-9
    cfg = grim.grim_index_get_config(idx, grim.MODE_CANDIDATES)
    assert (cfg["cand_waves"], cfg["cand_persistent"]) == (res["cand_waves"], res["cand_persistent"])
    assert "gfx950/cand/q6" in cache.read_text()
    got = run_cand(idx, rd, co, cb, ep)
    want = oracle.scan_candidates(oracle.bits(ref, w.bin_size, w.overlap, w.q), w.q, rd.bases, rd.offsets, co, cb,
                                  err_pm_per_read=ep)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_tune_scan(oracle, tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("GRIM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w = C.shrink(C.workload("c3"), genome_len=8_000_000, n_reads=4096)
    ref = synth.genome(w.genome)
    rd = synth.reads(w.reads, ref)
    idx = grim.grim_build_index(dev(ref), w.bin_size, w.overlap, w.q, grim.LAYOUT_TM)
    nb, W = idx.info()["n_bins"], idx.info()["mask_words"]
    E = np.full(rd.n, w.max_edits, np.uint16)
    rs = grim.ReadSet(dev(rd.bases), dev(rd.offsets), max_edits=dev(E))
    m0 = empty((rd.n, W), torch.uint32)
    grim.grim_filter_scan(idx, rs, m0)
    res = grim.grim_tune(idx, rs)
    log("tuned scan", res)
    assert res["mode"] == grim.MODE_SCAN and res["n_tried"] >= 8
    m1 = empty((rd.n, W), torch.uint32)
    grim.grim_filter_scan(idx, rs, m1)
    assert torch.equal(m0, m1)
    sub = np.arange(0, rd.n, 64)
    s = rd.subset(sub)
    _, wp = oracle.scan_all(oracle.bits(ref, w.bin_size, w.overlap, w.q), w.q, s.bases, s.offsets,
                            max_edits=E[sub])
    assert np.array_equal(unpack_mask(host(m1)[sub], nb), wp)
    # a fresh index of the same size class adopts the cached shape
    idx2 = grim.grim_build_index(dev(ref), w.bin_size, w.overlap, w.q, grim.LAYOUT_TM)
    grim.grim_filter_scan(idx2, rs, m1)
    cfg = grim.grim_index_get_config(idx2, grim.MODE_SCAN)
    assert (cfg["threads"], cfg["reads_per_chunk"], cfg["lane_words"]) == \
        (res["threads"], res["reads_per_chunk"], res["lane_words"])


def test_set_config_rejects_bad_shapes(uneven):
    idx = uneven[5]
    with pytest.raises(grim.GrimError):
        grim.grim_index_set_config(idx, {"mode": grim.MODE_SCAN, "threads": 300, "reads_per_chunk": 4096,
                                         "lane_words": 4})
    with pytest.raises(grim.GrimError):
        grim.grim_index_set_config(idx, {"mode": 7})


def _fill_batch(buf, rd, ids, co=None, cb=None, edits=None):
    sub = rd.subset(ids)
    nb = len(sub.bases)
    buf["bases"][:nb] = sub.bases
    buf["offsets"][:len(ids) + 1] = sub.offsets
    if edits is not None:
        buf["edits"][:len(ids)] = edits[ids]
    npair = 0
    if co is not None:
        lens = co[ids + 1] - co[ids]
        buf["cand_off"][0] = 0
        buf["cand_off"][1:len(ids) + 1] = np.cumsum(lens)
        npair = int(lens.sum())
        if npair:
            buf["cand_bin"][:npair] = np.concatenate([cb[co[i]:co[i + 1]] for i in ids])
    return sub, nb, npair


def test_batcher_candidates_every_replay_matches_eager(uneven, oracle):
    w, ref, rd, co, cb, idx = uneven
    ep = rd.err_pm.astype(np.uint16)
    bits = oracle.bits(ref, w.bin_size, w.overlap, w.q)
    grim.grim_index_set_config(idx, {"mode": grim.MODE_CANDIDATES, "cand_waves": 4, "cand_persistent": 1,
                                     "cand_groups_per_cu": 4, "cand_coop": 1})
    b = grim.Batcher(idx, grim.MODE_CANDIDATES, max_reads=2000, max_bases=2000 * 250, max_cand=2000 * 1024,
                     edits_kind=grim.BATCH_EDITS_ERR)
    rng = random.Random(3)
    pending = {}
    for it in range(8):
        slot = it % 2
        if slot in pending:
            b.wait(slot)
            ids, sub, npair = pending.pop(slot)
            buf = b.buffers(slot)
            got_c, got_p = buf["count_out"][:npair].copy(), buf["pass_out"][:npair].copy()
            # eager call on the same batch, between graph replays
            sco = np.zeros(len(ids) + 1, np.int64)
            sco[1:] = np.cumsum(co[ids + 1] - co[ids])
            scb = np.concatenate([cb[co[i]:co[i + 1]] for i in ids]).astype(np.int32)
            want = run_cand(idx, sub, sco, scb, ep[ids])
            assert np.array_equal(got_c, want[0]) and np.array_equal(got_p, want[1]), it
            # and the oracle on the same batch
            oc, op = oracle.scan_candidates(bits, w.q, sub.bases, sub.offsets, sco, scb, err_pm_per_read=ep[ids])
            assert np.array_equal(got_c, oc) and np.array_equal(got_p, op), it
        n = rng.choice([1, 17, 640, 2000])
        ids = np.sort(np.random.default_rng(it).choice(rd.n, size=n, replace=False))
        buf = b.buffers(slot)
        sub, nbases, npair = _fill_batch(buf, rd, ids, co, cb, edits=ep)
        log("batch", it, "slot", slot, "reads", n, "pairs", npair)
        b.submit(slot, n, nbases, npair)
        pending[slot] = (ids, sub, npair)
    for slot in list(pending):
        b.wait(slot)
    b.free()


def test_batcher_scan_every_replay_matches_eager(oracle):
    import torch
    w = C.shrink(C.workload("c3"), genome_len=3_000_000, n_reads=3000)
    ref = synth.genome(w.genome)
    rd = synth.reads(w.reads, ref)
    idx = grim.grim_build_index(dev(ref), w.bin_size, w.overlap, w.q, grim.LAYOUT_TM)
    W = idx.info()["mask_words"]
    nb = idx.info()["n_bins"]
    bits = oracle.bits(ref, w.bin_size, w.overlap, w.q)
    b = grim.Batcher(idx, grim.MODE_SCAN, max_reads=1000, max_bases=1000 * 150, edits_kind=grim.BATCH_EDITS_NONE,
                     err_permille_all=45)
    for it in range(6):
        slot = it % 2
        n = [1000, 3, 999, 64, 1000, 500][it]
        ids = np.arange(it * 400, it * 400 + n) % rd.n
        buf = b.buffers(slot)
        sub, nbases, _ = _fill_batch(buf, rd, ids)
        b.submit(slot, n, nbases)
        b.wait(slot)
        got = d2h(buf["mask_out_device"], n * W * 4).view(np.uint32).reshape(n, W)
        m = empty((n, W), torch.uint32)
        grim.grim_filter_scan(idx, grim.ReadSet(dev(sub.bases), dev(sub.offsets), err_permille_all=45), m)
        assert np.array_equal(got, host(m)), it
        # every 7th row of the replay against the oracle
        rows = np.arange(0, n, 7)
        s7 = sub.subset(rows)
        _, wp = oracle.scan_all(bits, w.q, s7.bases, s7.offsets, err_permille=45, want_counts=False)
        assert np.array_equal(unpack_mask(got[rows], nb), wp), it
    b.free()


def test_batcher_scan_many_chunks_smaller_replays(oracle):
    """A capture for 40000 reads cuts them into 16 read chunks (two per XCD). Replays of fewer
    reads deal their workgroup iterations over the same chunks, some of which then stay empty;
    every replay must equal the eager call, and sampled rows the oracle."""
    import torch
    w = C.shrink(C.workload("c3"), genome_len=3_000_000, n_reads=40000)
    ref = synth.genome(w.genome)
    rd = synth.reads(w.reads, ref)
    idx = grim.grim_build_index(dev(ref), w.bin_size, w.overlap, w.q, grim.LAYOUT_TM)
    W = idx.info()["mask_words"]
    nb = idx.info()["n_bins"]
    bits = oracle.bits(ref, w.bin_size, w.overlap, w.q)
    b = grim.Batcher(idx, grim.MODE_SCAN, max_reads=40000, max_bases=40000 * 150, edits_kind=grim.BATCH_EDITS_NONE,
                     err_permille_all=45)
    for it, n in enumerate([40000, 12345, 129, 40000, 2047]):
        slot = it % 2
        ids = np.arange(n)
        buf = b.buffers(slot)
        sub, nbases, _ = _fill_batch(buf, rd, ids)
        log("many-chunk replay", it, "reads", n)
        b.submit(slot, n, nbases)
        b.wait(slot)
        got = d2h(buf["mask_out_device"], n * W * 4).view(np.uint32).reshape(n, W)
        m = empty((n, W), torch.uint32)
        grim.grim_filter_scan(idx, grim.ReadSet(dev(sub.bases), dev(sub.offsets), err_permille_all=45), m)
        assert np.array_equal(got, host(m)), it
        rows = np.unique(np.concatenate([np.arange(0, n, max(1, n // 40)), [n - 1]]))
        sr = sub.subset(rows)
        _, wp = oracle.scan_all(bits, w.q, sr.bases, sr.offsets, err_permille=45, want_counts=False)
        assert np.array_equal(unpack_mask(got[rows], nb), wp), it
    b.free()


def test_batcher_errors(uneven):
    w, ref, rd, co, cb, idx = uneven
    b = grim.Batcher(idx, grim.MODE_CANDIDATES, max_reads=10, max_bases=3000, max_cand=100)
    with pytest.raises(grim.GrimError):
        b.submit(0, 11, 100, 0)
    buf = b.buffers(0)
    # a read shorter than q is reported when the batch completes
    buf["bases"][:3] = np.frombuffer(b"ACG", np.uint8)
    buf["offsets"][:2] = [0, 3]
    buf["cand_off"][:2] = [0, 1]
    buf["cand_bin"][0] = 0
    b.submit(0, 1, 3, 1)
    with pytest.raises(grim.GrimError) as e:
        b.wait(0)
    assert e.value.code == grim.GRIM_EINVAL
    # the slot works again afterwards
    seq = ref[:150]
    buf["bases"][:150] = seq
    buf["offsets"][:2] = [0, 150]
    b.submit(0, 1, 150, 1)
    b.wait(0)
    b.free()
