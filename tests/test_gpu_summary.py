"""Per-read mask summaries on the GPU (through the C ABI) against the oracle,
bit-exact: pass counts and 64-bit digests of masks from the all-bins scan, and
of random words at row widths that put the rows' 16-byte boundaries at every
offset, with more rows than the kernel's grid so its row loop wraps."""

from __future__ import annotations

import random

import numpy as np
import pytest

import synth
from gpu_util import dev, empty, host, log, unpack_mask
from paper_1708_04329_amd import grim

pytestmark = pytest.mark.gpu


def summary(mask_t):
    import torch
    n = mask_t.shape[0]
    pc = empty((max(n, 1),), torch.uint32)
    dg = empty((max(n, 1),), torch.uint64)
    grim.grim_mask_summary(mask_t, pc, dg)
    torch.cuda.synchronize()
    return host(pc.view(torch.int32)).view(np.uint32)[:n], host(dg.view(torch.int64)).view(np.uint64)[:n]


def test_summary_of_scan_masks(oracle):
    import torch
    rng = random.Random(77)
    G, B, O, q = 90_000, 37, 120, 4
    ref = np.frombuffer(bytes(rng.choice(b"ACGT") for _ in range(G)), np.uint8).copy()
    seqs = []
    for _ in range(300):
        L = rng.randrange(30, 110)
        p = rng.randrange(G - L)
        s = bytearray(ref[p:p + L].tobytes())
        for _ in range(rng.randrange(0, 5)):
            s[rng.randrange(L)] = rng.choice(b"ACGT")
        seqs.append(bytes(s))
    rd = synth.reads_from_strings(seqs)
    idx = grim.grim_build_index(dev(ref), B, O, q, grim.LAYOUT_TM)
    nb, W = idx.info()["n_bins"], idx.info()["mask_words"]
    log("summary of scan masks: reads", rd.n, "bins", nb, "words", W)
    mask = empty((rd.n, W), torch.uint32)
    rs = grim.ReadSet(dev(rd.bases), dev(rd.offsets), err_permille_all=40, allow_short_overlap=True)
    grim.grim_filter_scan(idx, rs, mask)
    torch.cuda.synchronize()
    got_c, got_d = summary(mask)
    _, want_pass = oracle.scan_all(oracle.bits(ref, B, O, q), q, rd.bases, rd.offsets, err_permille=40,
                                   want_counts=False)
    assert np.array_equal(unpack_mask(host(mask), nb), want_pass)
    want_c, want_d = oracle.mask_summary(want_pass)
    assert np.array_equal(got_c, want_c) and np.array_equal(got_d, want_d)
    assert 0 < want_c.min() < want_c.max() < nb


@pytest.mark.parametrize("n,W", [(1, 1), (5, 3), (4000, 5), (700, 1027), (1_100_000, 1)])
def test_summary_of_random_words(oracle, n, W):
    import torch
    g = np.random.default_rng(n * 31 + W)
    words = g.integers(0, 1 << 32, size=(n, W), dtype=np.uint64).astype(np.uint32)
    words[g.random((n, W)) < 0.2] = 0
    words[g.random((n, W)) < 0.1] = 0xFFFFFFFF
    log("summary of random words", n, "x", W)
    got_c, got_d = summary(dev(words.view(np.int32)).view(torch.uint32))
    bits = np.unpackbits(words.view(np.uint8), axis=1, bitorder="little")
    want_c = bits.sum(axis=1).astype(np.uint32)
    idx = np.arange(W, dtype=np.uint64) << np.uint64(32)
    with np.errstate(over="ignore"):
        want_d = oracle.mix64(words.astype(np.uint64) | idx[None, :]).sum(axis=1, dtype=np.uint64)
    assert np.array_equal(got_c, want_c) and np.array_equal(got_d, want_d)


def test_summary_optional_outputs_and_errors():
    import torch
    words = dev(np.arange(12, dtype=np.int32).reshape(3, 4)).view(torch.uint32)
    pc = empty((3,), torch.uint32)
    grim.grim_mask_summary(words, pass_count=pc)
    torch.cuda.synchronize()
    assert list(host(pc.view(torch.int32))) == [0 + 1 + 1 + 2, 1 + 2 + 2 + 3, 1 + 2 + 2 + 3]
    with pytest.raises(ValueError):
        grim.grim_mask_summary(words, pass_count=empty((2,), torch.uint32))
