"""GPU path (through the C ABI) against the CPU oracle, element by element.

Integer results, so the bar is bit-exact: index bits, per-bin counts, pass
masks, candidate counts and pass flags. Sizes span several LDS tiles of the
token-major index and several read chunks, with ragged tails."""

from __future__ import annotations

import os
import random

import numpy as np
import pytest

import synth
import synth.configs as C
from gpu_util import bm_to_bits, dev, empty, host, log, tm_to_bits, unpack_mask
from paper_1708_04329_amd import grim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    log("device", torch.cuda.get_device_name(0))
    yield


def rand_ref(rng: random.Random, G: int, n_runs: int = 4) -> np.ndarray:
    ref = bytearray(rng.choice(b"ACGT") for _ in range(G))
    for _ in range(n_runs):
        p = rng.randrange(G)
        ref[p:p + 3] = b"NNN"[:len(ref[p:p + 3])]
    for _ in range(n_runs):
        p = rng.randrange(G)
        ref[p:p + 50] = bytes(ref[p:p + 50]).lower()
    return np.frombuffer(bytes(ref[:G]), np.uint8).copy()


def rand_reads(rng: random.Random, ref: np.ndarray, n: int, lmin: int, lmax: int):
    seqs = []
    G = len(ref)
    for _ in range(n):
        L = rng.randrange(lmin, lmax + 1)
        if rng.random() < 0.8 and G > L:
            p = rng.randrange(0, G - L)
            s = bytearray(ref[p:p + L].tobytes())
            for _ in range(rng.randrange(0, 8)):
                s[rng.randrange(L)] = rng.choice(b"ACGTNacgt")
        else:
            s = bytearray(rng.choice(b"ACGT") for _ in range(L))
        seqs.append(bytes(s))
    return synth.reads_from_strings(seqs)


def build(ref, B, O, q, layout=grim.LAYOUT_TM | grim.LAYOUT_BM):
    return grim.grim_build_index(dev(ref), B, O, q, layout)


def gpu_scan(idx, rd, counts_dtype=None, on_device=True, **kw):
    import torch
    info = idx.info()
    n = rd.n
    mask = empty((max(n, 1), info["mask_words"]), torch.uint32)
    counts = empty((max(n, 1), info["n_bins"]), counts_dtype) if counts_dtype is not None else None
    conv = dev if on_device else (lambda a: np.ascontiguousarray(a))
    me = kw.pop("max_edits", None)
    ep = kw.pop("err_permille", None)
    rs = grim.ReadSet(conv(rd.bases) if len(rd.bases) else conv(np.zeros(1, np.uint8))[:0],
                      conv(rd.offsets), None if me is None else conv(me),
                      None if ep is None else conv(ep), **kw)
    grim.grim_filter_scan(idx, rs, mask, counts)
    torch.cuda.synchronize()
    m = host(mask)[:n]
    c = host(counts)[:n] if counts is not None else None
    return m, c


# ---------------------------------------------------------------------------
# index bits
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6, 7])
def test_index_bits_match_oracle(oracle, q):
    rng = random.Random(100 + q)
    G = {1: 3000, 2: 5000, 3: 40000, 4: 60000, 5: 100000, 6: 60000, 7: 20000}[q]
    B, O = 37, rng.randrange(0, 80)
    ref = rand_ref(rng, G)
    log("index bits q", q, "G", G, "B", B, "O", O)
    idx = build(ref, B, O, q)
    inf = idx.info()
    want = oracle.bits(ref, B, O, q)
    nb, R4 = want.shape
    assert inf["n_bins"] == nb and inf["bits_bytes"] == oracle.index_bytes(nb, q)
    tm = tm_to_bits(idx.read(grim.LAYOUT_TM), R4, inf["tm_row_words"], nb)
    assert np.array_equal(tm, want)
    bm = bm_to_bits(idx.read(grim.LAYOUT_BM), R4, inf["bm_vec_words"], nb)
    assert np.array_equal(bm, want)
    # padding of the token-major rows beyond the last bin is zero
    rows = idx.read(grim.LAYOUT_TM).view("<u4").reshape(R4, inf["tm_row_words"])
    tail = np.unpackbits(rows.view(np.uint8).reshape(R4, -1), axis=1, bitorder="little")[:, nb:]
    assert not tail.any()


# ---------------------------------------------------------------------------
# all-bins scan
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(10))
def test_scan_matches_oracle_random(oracle, seed, monkeypatch):
    rng = random.Random(seed)
    q = [3, 4, 5, 5, 6, 7, 5, 4, 6, 5][seed]
    B = rng.choice([24, 32, 41, 64])
    nb_target = {3: 1500, 4: 2100, 5: 2500, 6: 700, 7: 200}[q]
    G = B * nb_target + rng.randrange(0, B)
    O = rng.randrange(0, 120)
    ref = rand_ref(rng, G)
    n = rng.choice([1, 7, 130, 300])
    lmax = 300 if seed % 3 == 0 else 120          # some reads above 255 tokens
    rd = rand_reads(rng, ref, n, q, lmax)
    mode = seed % 3
    kw = {"allow_short_overlap": True}
    if mode == 0:
        kw["max_edits"] = np.array([rng.randrange(0, 12) for _ in range(n)], np.uint16)
    elif mode == 1:
        kw["err_permille"] = np.array([rng.choice([0, 20, 35, 50, 80]) for _ in range(n)], np.uint16)
    else:
        kw["err_permille_all"] = rng.choice([0, 25, 50])
    monkeypatch.setenv("GRIM_SCAN_CHUNK", str(rng.choice([64, 128, 4096])))
    monkeypatch.setenv("GRIM_SCAN_THREADS", str(rng.choice([256, 512, 1024])))
    monkeypatch.setenv("GRIM_SCAN_SORT", str(1 - seed % 4 // 3))          # length order off for seeds 3 and 7
    monkeypatch.setenv("GRIM_SCAN_LANE_WORDS", str(8 if seed in (2, 5) else 4))
    log("scan seed", seed, "q", q, "B", B, "G", G, "O", O, "n", n, "mode", mode,
        os.environ["GRIM_SCAN_CHUNK"], os.environ["GRIM_SCAN_THREADS"])
    idx = build(ref, B, O, q, grim.LAYOUT_TM)
    bits = oracle.bits(ref, B, O, q)
    nb = bits.shape[0]
    want_c, want_p = oracle.scan_all(bits, q, rd.bases, rd.offsets, max_edits=kw.get("max_edits"),
                                     err_pm_per_read=kw.get("err_permille"),
                                     err_permille=kw.get("err_permille_all", 0))
    m, c = gpu_scan(idx, rd, counts_dtype=__import__("torch").uint16, **kw)
    assert np.array_equal(c.astype(np.uint16), want_c)
    assert np.array_equal(unpack_mask(m, nb), want_p)
    # the mask-only kernel (no count output compiled in) writes the same bits
    m2, _ = gpu_scan(idx, rd, **kw)
    assert np.array_equal(m2, m)
    # mask bits beyond the last bin are zero
    if nb % 32:
        assert not (m[:, -1] >> (nb % 32)).any()


@pytest.mark.parametrize("q,threads,lw", [(5, 1024, 4), (5, 512, 8), (4, 256, 8), (3, 1024, 4), (5, 256, 4)])
def test_scan_every_remainder(oracle, monkeypatch, q, threads, lw):
    """Read lengths give every remainder (0..31 tokens) with 0..9 full blocks in
    one launch, so lanes of one wavefront fold different parts and run
    different loop counts; a few reads above 255 tokens take the 16-plane path
    in the same launch. Reads are not length-ordered."""
    rng = random.Random(1000 * q + threads)
    B = 32
    G = B * 2300 + 17
    ref = rand_ref(rng, G)
    lens = [q - 1 + 32 * nb + r for nb in range(10) for r in range(32)]  # 32 nb + r tokens
    lens = [L for L in lens if L >= q] + [300, 290, 260 + q]
    rng.shuffle(lens)
    seqs = []
    for L in lens:
        p0 = rng.randrange(0, G - L)
        s = bytearray(ref[p0:p0 + L].tobytes())
        for _ in range(rng.randrange(0, 4)):
            if L:
                s[rng.randrange(L)] = rng.choice(b"ACGTN")
        seqs.append(bytes(s))
    rd = synth.reads_from_strings(seqs)
    me = np.array([rng.randrange(0, 6) for _ in range(rd.n)], np.uint16)
    monkeypatch.setenv("GRIM_SCAN_THREADS", str(threads))
    monkeypatch.setenv("GRIM_SCAN_LANE_WORDS", str(lw))
    monkeypatch.setenv("GRIM_SCAN_CHUNK", str(rng.choice([64, 256])))
    monkeypatch.setenv("GRIM_SCAN_SORT", "0")
    idx = build(ref, B, 60, q, grim.LAYOUT_TM)
    bits = oracle.bits(ref, B, 60, q)
    nb = bits.shape[0]
    want_c, want_p = oracle.scan_all(bits, q, rd.bases, rd.offsets, max_edits=me)
    m, c = gpu_scan(idx, rd, counts_dtype=__import__("torch").uint16, max_edits=me, allow_short_overlap=True)
    assert np.array_equal(c.astype(np.uint16), want_c)
    assert np.array_equal(unpack_mask(m, nb), want_p)
    m2, _ = gpu_scan(idx, rd, max_edits=me, allow_short_overlap=True)
    assert np.array_equal(m2, m)
    log("every remainder q", q, "threads", threads, "lane words", lw, "reads", rd.n, "bins", nb)


def test_scan_c1_full_size(oracle):
    """The 1 Mbp all-bins workload at its stated size: uint8 counts and pass bits."""
    import torch
    w = C.workload("c1")
    ref = synth.genome(w.genome)
    rd = synth.reads(w.reads, ref)
    log("c1 full", len(ref), rd.n)
    idx = build(ref, w.bin_size, w.overlap, w.q, grim.LAYOUT_TM)
    E = np.full(rd.n, w.max_edits, np.uint16)
    m, c = gpu_scan(idx, rd, counts_dtype=torch.uint8, max_edits=E)
    bits = oracle.bits(ref, w.bin_size, w.overlap, w.q)
    want_c, want_p = oracle.scan_all(bits, w.q, rd.bases, rd.offsets, max_edits=E)
    assert np.array_equal(c, want_c.astype(np.uint8))
    assert np.array_equal(unpack_mask(m, bits.shape[0]), want_p)
    # every read (5 edits <= E) passes the bin of its true start
    truth_bins = (rd.truth_pos // w.bin_size).astype(np.int64)
    assert want_p[np.arange(rd.n), truth_bins].all()


def test_host_inputs_equal_device_inputs(oracle):
    import torch
    rng = random.Random(42)
    ref = rand_ref(rng, 70000)
    rd = rand_reads(rng, ref, 200, 5, 150)
    idx = build(ref, 50, 150, 5, grim.LAYOUT_TM)
    E = np.array([rng.randrange(0, 6) for _ in range(rd.n)], np.uint16)
    a = gpu_scan(idx, rd, counts_dtype=torch.uint16, max_edits=E, on_device=True)
    b = gpu_scan(idx, rd, counts_dtype=torch.uint16, max_edits=E, on_device=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_threshold_not_positive_passes_all_bins(oracle):
    rng = random.Random(9)
    ref = rand_ref(rng, 40000)
    rd = rand_reads(rng, ref, 50, 20, 60)
    idx = build(ref, 64, 60, 5, grim.LAYOUT_TM)
    nb = idx.info()["n_bins"]
    m, _ = gpu_scan(idx, rd, max_edits=np.full(rd.n, 20, np.uint16), allow_short_overlap=True)
    assert unpack_mask(m, nb).all()
    if nb % 32:
        assert not (m[:, -1] >> (nb % 32)).any()


# ---------------------------------------------------------------------------
# candidate mode
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("coop", [0, 1, 2])
@pytest.mark.parametrize("q", [2, 3, 4, 5, 6, 7])
def test_candidates_match_oracle_random(oracle, q, coop, monkeypatch):
    if coop == 2 and q != 5:
        pytest.skip("four reads per wavefront is the q = 5 layout")
    import torch
    monkeypatch.setenv("GRIM_CAND_COOP", str(coop))
    rng = random.Random(500 + q)
    B = 61
    G = 150000 if q <= 6 else 40000
    ref = rand_ref(rng, G)
    O = 200
    idx = build(ref, B, O, q, grim.LAYOUT_BM)
    nb = idx.info()["n_bins"]
    rd = rand_reads(rng, ref, 257, q, 300)
    # candidate lists: 0..200 bins per read, some reads with every bin
    co, cb = [0], []
    for r in range(rd.n):
        k = rng.choice([0, 1, 3, 64, 65, 200])
        if r % 50 == 7:
            sel = list(range(nb))
        else:
            sel = sorted(rng.sample(range(nb), min(k, nb)))
        cb += sel
        co.append(len(cb))
    co = np.array(co, np.int64)
    cb = np.array(cb, np.int32)
    err = np.array([rng.choice([20, 30, 40, 50]) for _ in range(rd.n)], np.uint16)
    log("cand q", q, "pairs", len(cb))
    cnt = empty((max(1, len(cb)),), torch.uint16)
    pas = empty((max(1, len(cb)),), torch.uint8)
    rs = grim.ReadSet(dev(rd.bases), dev(rd.offsets), err_permille=dev(err), allow_short_overlap=True)
    grim.grim_filter_candidates(idx, rs, dev(co), dev(cb), cnt, pas)
    bits = oracle.bits(ref, B, O, q)
    wc, wp = oracle.scan_candidates(bits, q, rd.bases, rd.offsets, co, cb, err_pm_per_read=err)
    assert np.array_equal(host(cnt)[:len(cb)], wc)
    assert np.array_equal(host(pas)[:len(cb)], wp)


@pytest.mark.parametrize("planes", [8, 16])
@pytest.mark.parametrize("persistent", [0, 1])
def test_candidates_quad_layout_planes(oracle, monkeypatch, planes, persistent):
    """Four reads per wavefront at q = 5 with 8 or 16 LDS planes per read. Reads
    above 255 tokens (which the 8-plane form leaves to a second pass over the
    reads) sit between short ones; homopolymer reads reach counts of 255 (all 8
    planes) and more; some reads have no pairs."""
    import torch
    monkeypatch.setenv("GRIM_CAND_COOP", "2")
    monkeypatch.setenv("GRIM_CAND_PLANES", str(planes))
    monkeypatch.setenv("GRIM_CAND_PERSISTENT", str(persistent))
    rng = random.Random(5150 + planes + persistent)
    B, O, q = 61, 400, 5
    ref = rand_ref(rng, 120000)
    ref[3000:3400] = ord("A")
    idx = build(ref, B, O, q, grim.LAYOUT_BM)
    nb = idx.info()["n_bins"]
    rd = rand_reads(rng, ref, 230, q, 120)
    extra = [b"A" * 259, b"A" * 260, b"A" * 300, b"C" * 140, ref[3000:3300].tobytes(),
             rand_reads(rng, ref, 1, 256, 256).bases.tobytes(), rand_reads(rng, ref, 1, 380, 380).bases.tobytes()]
    strs = [rd.bases[rd.offsets[r]:rd.offsets[r + 1]].tobytes() for r in range(rd.n)]
    for i, e in enumerate(extra):
        strs.insert(17 * i + 3, e)
    rd = synth.reads_from_strings(strs)
    co, cb = [0], []
    for r in range(rd.n):
        k = rng.choice([0, 1, 7, 16, 17, 49, 200])
        sel = sorted(set(rng.sample(range(nb), min(k, nb))) | ({40, 41, 49} if k else set()))
        cb += sel
        co.append(len(cb))
    co = np.array(co, np.int64)
    cb = np.array(cb, np.int32)
    E = np.array([rng.randrange(0, 9) for _ in range(rd.n)], np.uint16)
    cnt = empty((len(cb),), torch.uint16)
    pas = empty((len(cb),), torch.uint8)
    rs = grim.ReadSet(dev(rd.bases), dev(rd.offsets), max_edits=dev(E), allow_short_overlap=True)
    grim.grim_filter_candidates(idx, rs, dev(co), dev(cb), cnt, pas)
    bits = oracle.bits(ref, B, O, q)
    wc, wp = oracle.scan_candidates(bits, q, rd.bases, rd.offsets, co, cb, max_edits=E)
    assert np.array_equal(host(cnt), wc)
    assert np.array_equal(host(pas), wp)
    assert wc.max() >= 255
    log("quad planes", planes, "persistent", persistent, "reads", rd.n, "pairs", len(cb))


def test_candidates_seed_hits_c2_recipe(oracle):
    """The 100 Mbp candidate workload's recipe on a 4 Mbp genome with 20k reads."""
    import torch
    w = C.shrink(C.workload("c2"), genome_len=4_000_000, n_reads=20000)
    ref = synth.genome(w.genome)
    rd = synth.reads(w.reads, ref)
    co, cb = synth.candidates(ref, rd, w.bin_size, w.cand_cap, w.cand_k)
    log("c2-recipe pairs", len(cb))
    idx = build(ref, w.bin_size, w.overlap, w.q, grim.LAYOUT_BM)
    E = np.full(rd.n, w.max_edits, np.uint16)
    cnt = empty((len(cb),), torch.uint16)
    pas = empty((len(cb),), torch.uint8)
    grim.grim_filter_candidates(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets), max_edits=dev(E)),
                                dev(co), dev(cb), cnt, pas)
    bits = oracle.bits(ref, w.bin_size, w.overlap, w.q)
    wc, wp = oracle.scan_candidates(bits, w.q, rd.bases, rd.offsets, co, cb, max_edits=E)
    assert np.array_equal(host(cnt), wc) and np.array_equal(host(pas), wp)


def test_candidates_agree_with_scan():
    import torch
    rng = random.Random(77)
    ref = rand_ref(rng, 90000)
    B, O, q = 45, 120, 5
    idx = build(ref, B, O, q)
    nb = idx.info()["n_bins"]
    rd = rand_reads(rng, ref, 100, 30, 100)
    E = np.array([rng.randrange(0, 5) for _ in range(rd.n)], np.uint16)
    m, c = gpu_scan(idx, rd, counts_dtype=torch.uint16, max_edits=E)
    co = np.arange(rd.n + 1, dtype=np.int64) * nb
    cb = np.tile(np.arange(nb, dtype=np.int32), rd.n)
    cnt = empty((len(cb),), torch.uint16)
    pas = empty((len(cb),), torch.uint8)
    grim.grim_filter_candidates(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets), max_edits=dev(E)),
                                dev(co), dev(cb), cnt, pas)
    assert np.array_equal(host(cnt).reshape(rd.n, nb), c)
    assert np.array_equal(host(pas).reshape(rd.n, nb), unpack_mask(m, nb))


# ---------------------------------------------------------------------------
# errors, empty inputs, persistence
# ---------------------------------------------------------------------------

def test_error_paths_leave_library_usable(oracle):
    import torch
    rng = random.Random(5)
    ref = rand_ref(rng, 20000)
    idx = build(ref, 100, 30, 5)
    nb = idx.info()["n_bins"]
    W = idx.info()["mask_words"]
    mask = empty((4, W), torch.uint32)
    # read shorter than q
    rd = synth.reads_from_strings([b"ACG"])
    with pytest.raises(grim.GrimError) as e:
        grim.grim_filter_scan(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets)), mask)
    assert e.value.code == grim.GRIM_EINVAL
    # overlap too small for a 100 bp read at E = 5 (O = 30 < 100 + 5 - 5)
    rd = synth.reads_from_strings([ref[:100].tobytes()])
    with pytest.raises(grim.GrimError) as e:
        grim.grim_filter_scan(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets), max_edits=dev(np.array([5], np.uint16))), mask)
    assert e.value.code == grim.GRIM_EOVERLAP
    # uint8 counts with more than 255 tokens
    rd = synth.reads_from_strings([ref[:400].tobytes()])
    cnt8 = empty((1, nb), torch.uint8)
    with pytest.raises(grim.GrimError) as e:
        grim.grim_filter_scan(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets), allow_short_overlap=True), mask, cnt8)
    assert e.value.code == grim.GRIM_EINVAL
    # candidate bin out of range
    rd = synth.reads_from_strings([ref[:30].tobytes()])
    with pytest.raises(grim.GrimError) as e:
        grim.grim_filter_candidates(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets)), dev(np.array([0, 2], np.int64)),
                                    dev(np.array([0, nb], np.int32)), empty((2,), torch.uint16), empty((2,), torch.uint8))
    assert e.value.code == grim.GRIM_EINVAL
    # empty read set is a no-op
    grim.grim_filter_scan(idx, grim.ReadSet(dev(np.zeros(1, np.uint8)), dev(np.zeros(1, np.int64))), mask)
    # and a good call still works afterwards
    rd = synth.reads_from_strings([ref[1000:1030].tobytes()])
    m, _ = gpu_scan(idx, rd, max_edits=np.array([0], np.uint16))
    bits = oracle.bits(ref, 100, 30, 5)
    _, wp = oracle.scan_all(bits, 5, rd.bases, rd.offsets, max_edits=np.array([0], np.uint16))
    assert np.array_equal(unpack_mask(m, nb), wp)


def test_maximum_read_length(oracle):
    """Reads of exactly 65535 tokens (the most a count can hold): a homopolymer, whose single
    token reaches count 65535 (all 16 counter planes), and a random read; both in the all-bins
    scan with uint16 counts and in candidate mode. One token more is rejected."""
    import torch
    rng = random.Random(65535)
    q = 5
    G, B, O = 30000, 64, 40
    ref = bytearray(rand_ref(rng, G).tobytes())
    ref[5000:5100] = b"A" * 100                   # an A run: bins around it hold token AAAAA
    ref = np.frombuffer(bytes(ref), np.uint8).copy()
    L = 65535 + q - 1
    seqs = [b"A" * L, bytes(rng.choice(b"ACGT") for _ in range(L))]
    rd = synth.reads_from_strings(seqs)
    idx = build(ref, B, O, q)
    nb = idx.info()["n_bins"]
    E = np.array([0, 9000], np.uint16)
    log("maximum read length: tokens", L - q + 1, "bins", nb)
    m, c = gpu_scan(idx, rd, counts_dtype=torch.uint16, max_edits=E, allow_short_overlap=True)
    bits = oracle.bits(ref, B, O, q)
    want_c, want_p = oracle.scan_all(bits, q, rd.bases, rd.offsets, max_edits=E)
    assert np.array_equal(c.astype(np.uint16), want_c) and np.array_equal(unpack_mask(m, nb), want_p)
    assert want_c[0].max() == 65535 and want_p[0].any() and not want_p[0].all()
    # candidate mode: every bin of both reads
    co = np.array([0, nb, 2 * nb], np.int64)
    cb = np.concatenate([np.arange(nb, dtype=np.int32)] * 2)
    cnt = empty((2 * nb,), torch.uint16)
    pas = empty((2 * nb,), torch.uint8)
    rs = grim.ReadSet(dev(rd.bases), dev(rd.offsets), max_edits=dev(E), allow_short_overlap=True)
    grim.grim_filter_candidates(idx, rs, dev(co), dev(cb), cnt, pas)
    torch.cuda.synchronize()
    assert np.array_equal(host(cnt.view(torch.int16)).view(np.uint16), want_c.reshape(-1))
    assert np.array_equal(host(pas), want_p.reshape(-1))
    # 65536 tokens: rejected, and the index stays usable
    rd2 = synth.reads_from_strings([b"A" * (L + 1)])
    mask = empty((1, idx.info()["mask_words"]), torch.uint32)
    with pytest.raises(grim.GrimError) as e:
        grim.grim_filter_scan(idx, grim.ReadSet(dev(rd2.bases), dev(rd2.offsets), allow_short_overlap=True), mask)
    assert e.value.code == grim.GRIM_EINVAL
    m2, _ = gpu_scan(idx, rd, max_edits=E, allow_short_overlap=True)
    assert np.array_equal(unpack_mask(m2, nb), want_p)


def test_save_load_roundtrip(tmp_path):
    import torch
    rng = random.Random(6)
    ref = rand_ref(rng, 50000)
    idx = build(ref, 80, 100, 5, grim.LAYOUT_TM | grim.LAYOUT_BM | grim.LAYOUT_REF)
    p = str(tmp_path / "i.grim")
    idx.save(p)
    idx2 = grim.grim_index_load(p)
    assert idx2.info() == idx.info() and idx.info()["ref_bytes"] == len(ref)
    assert np.array_equal(idx2.read(grim.LAYOUT_TM), idx.read(grim.LAYOUT_TM))
    assert np.array_equal(idx2.read(grim.LAYOUT_BM), idx.read(grim.LAYOUT_BM))
    assert np.array_equal(idx2.read(grim.LAYOUT_REF), idx.read(grim.LAYOUT_REF))
    raw = bytearray(open(p, "rb").read())
    raw[-5] ^= 0xFF
    bad = str(tmp_path / "bad.grim")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(grim.GrimError) as e:
        grim.grim_index_load(bad)
    assert e.value.code == grim.GRIM_EIO


@pytest.mark.parametrize("shift", [0, 3])
def test_every_byte_value_in_the_reference(oracle, shift):
    """A reference holding every byte value: the index bits follow the oracle (only
    A, C, G, T in either case start a valid window) and the verification copy
    holds codes 0..3 for those and 4 for every other byte. The length is not a
    multiple of 16, and shift 3 hands the build a device pointer that is not
    16-byte aligned."""
    import torch
    rng = random.Random(4242 + shift)
    G = 100_003
    ref = rand_ref(rng, G)
    pos = rng.sample(range(G), 6000)
    ref[pos] = np.arange(6000) % 256                    # every byte value, 23 times or more
    codes = {ord(c): i for i, c in enumerate("ACGT")}
    codes.update({ord(c): i for i, c in enumerate("acgt")})
    want_codes = np.array([codes.get(int(b), 4) for b in ref], np.uint8)
    B, O, q = 211, 40, 4
    buf = torch.zeros(G + shift, dtype=torch.uint8, device="cuda")
    buf[shift:] = dev(ref)
    idx = grim.grim_build_index(buf[shift:], B, O, q, grim.LAYOUT_TM | grim.LAYOUT_BM | grim.LAYOUT_REF)
    inf = idx.info()
    assert np.array_equal(idx.read(grim.LAYOUT_REF), want_codes)
    want = oracle.bits(ref, B, O, q)
    nb, R4 = want.shape
    assert np.array_equal(tm_to_bits(idx.read(grim.LAYOUT_TM), R4, inf["tm_row_words"], nb), want)
    assert np.array_equal(bm_to_bits(idx.read(grim.LAYOUT_BM), R4, inf["bm_vec_words"], nb), want)


# ---------------------------------------------------------------------------
# q = 8: the largest token length the boundary takes (4^8-bit, 8 KB vectors)
# ---------------------------------------------------------------------------

def test_q8_bin_major_bits_and_token_major_rejected(oracle):
    rng = random.Random(808)
    G, B, O, q = 30000, 97, 150, 8
    ref = rand_ref(rng, G)
    idx = build(ref, B, O, q, grim.LAYOUT_BM | grim.LAYOUT_REF)
    inf = idx.info()
    want = oracle.bits(ref, B, O, q)
    nb, R4 = want.shape
    assert R4 == 65536 and inf["bm_vec_words"] == 2048 and inf["bits_bytes"] == oracle.index_bytes(nb, q)
    assert np.array_equal(bm_to_bits(idx.read(grim.LAYOUT_BM), R4, inf["bm_vec_words"], nb), want)
    for layout in (grim.LAYOUT_TM, grim.LAYOUT_TM | grim.LAYOUT_BM):
        with pytest.raises(grim.GrimError) as e:
            build(ref, B, O, q, layout)
        assert e.value.code == grim.GRIM_EINVAL
    with pytest.raises(grim.GrimError) as e:
        build(ref, B, O, 9, grim.LAYOUT_BM)
    assert e.value.code == grim.GRIM_EINVAL


@pytest.mark.parametrize("persistent", [0, 1])
def test_q8_candidates_match_oracle(oracle, persistent, monkeypatch):
    """Candidate counts at q = 8, including reads whose tokens repeat 16 times or
    more (homopolymers and short periods: more than four multiplicity planes)."""
    import torch
    monkeypatch.setenv("GRIM_CAND_PERSISTENT", str(persistent))
    rng = random.Random(880 + persistent)
    G, B, O, q = 40000, 113, 300, 8
    ref = rand_ref(rng, G)
    ref[5000:5400] = ord("A")
    ref[9000:9400] = np.frombuffer(b"ACGTTG" * 66 + b"ACGT", np.uint8)
    idx = build(ref, B, O, q, grim.LAYOUT_BM)
    nb = idx.info()["n_bins"]
    rd = rand_reads(rng, ref, 150, q, 300)
    extra = [b"A" * 300, b"ACGTTG" * 50, b"A" * 8, ref[5100:5350].tobytes(), ref[9010:9290].tobytes()]
    strs = [rd.bases[rd.offsets[r]:rd.offsets[r + 1]].tobytes() for r in range(rd.n)] + extra
    rd = synth.reads_from_strings(strs)
    co, cb = [0], []
    for r in range(rd.n):
        if r >= rd.n - len(extra):
            sel = sorted(set(rng.sample(range(nb), 40)) | set(range(40, 50)) | set(range(77, 85)))
        else:
            sel = sorted(rng.sample(range(nb), rng.choice([0, 1, 5, 64, 130])))
        cb += sel
        co.append(len(cb))
    co = np.array(co, np.int64)
    cb = np.array(cb, np.int32)
    err = np.array([rng.choice([0, 20, 50]) for _ in range(rd.n)], np.uint16)
    log("cand q 8 persistent", persistent, "pairs", len(cb))
    cnt = empty((len(cb),), torch.uint16)
    pas = empty((len(cb),), torch.uint8)
    rs = grim.ReadSet(dev(rd.bases), dev(rd.offsets), err_permille=dev(err), allow_short_overlap=True)
    grim.grim_filter_candidates(idx, rs, dev(co), dev(cb), cnt, pas)
    torch.cuda.synchronize()
    bits = oracle.bits(ref, B, O, q)
    wc, wp = oracle.scan_candidates(bits, q, rd.bases, rd.offsets, co, cb, err_pm_per_read=err)
    got = host(cnt)
    assert np.array_equal(got, wc)
    assert np.array_equal(host(pas), wp)
    # the homopolymer read meets 293 copies of its one token in the A run's bins
    assert got.max() == 293
