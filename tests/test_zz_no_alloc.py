"""grim_filter_candidates_static (no device allocation, fixed per-GPU scratch)
against grim_filter_candidates through the C ABI: bit-exact counts and pass
flags on two calls in a row, the second smaller (the scratch keeps the first
call's contents), in both launch shapes, plus the oracle on the same inputs,
the size limit and the argument checks."""

from __future__ import annotations

import random

import numpy as np
import pytest

import synth
from gpu_util import dev, empty, host, log
from paper_1708_04329_amd import grim

pytestmark = pytest.mark.gpu


def _ref(rng, G):
    ref = bytearray(rng.choice(b"ACGT") for _ in range(G))
    for _ in range(4):
        p = rng.randrange(G - 5)
        ref[p:p + 3] = b"NNN"
    return np.frombuffer(bytes(ref), np.uint8).copy()


def _reads(rng, ref, n, lmin, lmax):
    seqs = []
    for _ in range(n):
        L = rng.randrange(lmin, lmax + 1)
        p = rng.randrange(0, len(ref) - L)
        s = bytearray(ref[p:p + L].tobytes())
        for _ in range(rng.randrange(0, 6)):
            s[rng.randrange(L)] = rng.choice(b"ACGTN")
        seqs.append(bytes(s))
    return synth.reads_from_strings(seqs)


def _cands(rng, n, nb, kmax):
    co, cb = [0], []
    for _ in range(n):
        sel = sorted(rng.sample(range(nb), rng.randrange(0, kmax + 1)))
        cb += sel
        co.append(len(cb))
    return np.array(co, np.int64), np.array(cb, np.int32)


def _run(fn, idx, rd, err, co, cb):
    import torch
    cnt = empty((max(1, len(cb)),), torch.uint16)
    pas = empty((max(1, len(cb)),), torch.uint8)
    cnt.fill_(0xAB)
    pas.fill_(7)
    fn(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets), err_permille=dev(err)), dev(co), dev(cb), cnt, pas)
    torch.cuda.synchronize()
    return host(cnt)[:len(cb)], host(pas)[:len(cb)]


@pytest.mark.parametrize("q,persistent", [(5, 0), (5, 1), (6, 0)])
def test_static_equals_allocating_entry_point(oracle, q, persistent):
    rng = random.Random(70 + q + persistent)
    G, B, O = 300_000, 1024, 300
    ref = _ref(rng, G)
    idx = grim.grim_build_index(dev(ref), B, O, q, grim.LAYOUT_BM)
    nb = idx.info()["n_bins"]
    if persistent:
        cfg = grim.grim_index_get_config(idx, grim.MODE_CANDIDATES)
        cfg.update(cand_persistent=1, cand_groups_per_cu=2)
        grim.grim_index_set_config(idx, cfg)
    # first call large, second smaller: the second must not see the first's scratch
    for call, (n, kmax) in enumerate([(3000, 40), (257, 70)]):
        rd = _reads(rng, ref, n, q, 250)
        err = np.array([rng.choice([20, 30, 40, 50]) for _ in range(rd.n)], np.uint16)
        co, cb = _cands(rng, rd.n, nb, kmax)
        log("static q", q, "persistent", persistent, "call", call, "reads", rd.n, "pairs", len(cb))
        got_c, got_p = _run(grim.grim_filter_candidates_static, idx, rd, err, co, cb)
        want_c, want_p = _run(grim.grim_filter_candidates, idx, rd, err, co, cb)
        assert np.array_equal(got_c, want_c) and np.array_equal(got_p, want_p)
        if call == 1:
            bits = oracle.bits(ref, B, O, q)
            oc, op = oracle.scan_candidates(bits, q, rd.bases, rd.offsets, co, cb, err_pm_per_read=err)
            assert np.array_equal(got_c, oc) and np.array_equal(got_p, op)


def test_static_limits_and_errors():
    import torch
    rng = random.Random(9)
    ref = _ref(rng, 100_000)
    idx = grim.grim_build_index(dev(ref), 1000, 300, 5, grim.LAYOUT_BM)
    nb = idx.info()["n_bins"]
    rd = _reads(rng, ref, 50, 100, 150)
    err = np.full(rd.n, 30, np.uint16)
    co, cb = _cands(rng, rd.n, nb, 20)
    cnt = empty((len(cb),), torch.uint16)
    pas = empty((len(cb),), torch.uint8)
    # host reads are refused (they would need a device staging copy)
    with pytest.raises(grim.GrimError) as e:
        grim.grim_filter_candidates_static(idx, grim.ReadSet(rd.bases, rd.offsets, err_permille=err), dev(co), dev(cb),
                                           cnt, pas)
    assert e.value.code == grim.GRIM_EINVAL
    # a call whose scratch would exceed the fixed size is refused before any work
    n_big = grim.STATIC_SCRATCH_BYTES // (4 * 64) + 1
    big_offs = torch.zeros(n_big + 1, dtype=torch.int64, device="cuda")
    big_co = torch.zeros(n_big + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(grim.GrimError) as e:
        grim.grim_filter_candidates_static(idx, grim.ReadSet(dev(rd.bases), big_offs, err_permille_all=30), big_co,
                                           dev(cb[:0]), cnt, pas)
    assert e.value.code == grim.GRIM_EINVAL and "scratch" in str(e.value)
    # a bad bin fails that call only; the next call starts from cleared status words
    bad = cb.copy()
    bad[len(bad) // 2] = nb + 5
    with pytest.raises(grim.GrimError) as e:
        grim.grim_filter_candidates_static(idx, grim.ReadSet(dev(rd.bases), dev(rd.offsets), err_permille=dev(err)),
                                           dev(co), dev(bad), cnt, pas)
    assert e.value.code == grim.GRIM_EINVAL
    got_c, got_p = _run(grim.grim_filter_candidates_static, idx, rd, err, co, cb)
    want_c, want_p = _run(grim.grim_filter_candidates, idx, rd, err, co, cb)
    assert np.array_equal(got_c, want_c) and np.array_equal(got_p, want_p)
