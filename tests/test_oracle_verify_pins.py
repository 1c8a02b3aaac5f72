"""Pins of the oracle's verification step (no GPU).

Verification aligns a read against the bases of a bin that passed the filter:
the smallest Levenshtein distance between the whole read and any substring of
the bin's bases (the paper verifies passing locations by dynamic-programming
alignment, Section 1 step 5, and counts a passing location that yields no
mapping against the filter, Section 5). The pins check the oracle against a
brute force over every substring with an independent edit-distance routine,
against closed forms, against the synthetic reads' own edit scripts, and
against the window definition at its edges."""

from __future__ import annotations

import random

import numpy as np
import pytest

import synth
import synth.configs as C
from brute import edit_distance


def _rand(rng, n, alphabet=b"ACGT"):
    return bytes(rng.choice(alphabet) for _ in range(n))


@pytest.mark.parametrize("seed", range(4))
def test_verify_distance_bruteforce(oracle, seed):
    """min over every substring text[a:b] (empty included) of the plain global distance."""
    rng = random.Random(100 + seed)
    for _ in range(40):
        read = _rand(rng, rng.randrange(1, 11), b"ACGT" if seed % 2 else b"AC")
        text = _rand(rng, rng.randrange(0, 26), b"ACGT" if seed % 2 else b"AC")
        want = min(edit_distance(read, text[a:b]) for a in range(len(text) + 1) for b in range(a, len(text) + 1))
        assert oracle.semiglobal_distance(read, text) == want, (read, text)


def test_verify_nonacgt_matches_nothing(oracle):
    assert oracle.semiglobal_distance(b"ACNGT", b"TTACNGTTT") == 1
    assert oracle.semiglobal_distance(b"ACGT", b"ttacgttt") == 0
    assert oracle.semiglobal_distance(b"acgt", b"TTACGTTT") == 0
    assert oracle.semiglobal_distance(b"NNNN", b"NNNNNNNN") == 4


def test_verify_closed_forms(oracle):
    rng = random.Random(7)
    text = _rand(rng, 300)
    for L in (1, 17, 64, 100):
        a = rng.randrange(0, len(text) - L)
        read = text[a:a + L]
        assert oracle.semiglobal_distance(read, text) == 0           # an exact substring
        assert oracle.semiglobal_distance(read, b"") == L            # nothing to align to
        assert oracle.semiglobal_distance(b"A" * L, b"C" * 50) == L  # no base can match
        # relabelling the bases in both strings changes nothing
        perm = bytes.maketrans(b"ACGT", b"GTCA")
        mut = bytearray(read)
        for _ in range(3):
            mut[rng.randrange(L)] = rng.choice(b"ACGT")
        d = oracle.semiglobal_distance(bytes(mut), text)
        assert oracle.semiglobal_distance(bytes(mut).translate(perm), text.translate(perm)) == d
        assert d <= 3


def test_verify_window_edges(oracle):
    """A read ending at the last base a bin's tokens cover matches that bin exactly;
    one base further it does not (random reference)."""
    rng = random.Random(11)
    G, B, O, q = 1000, 100, 10, 5
    ref = np.frombuffer(_rand(rng, G), np.uint8).copy()
    for x in (0, 3, 9):
        lo, hi = oracle.bin_bases(x, G, B, O, q)
        assert lo == x * B
        inside = [ref[lo:lo + 24].tobytes(), ref[hi - 24:hi].tobytes()]
        outside = [ref[hi - 23:hi + 1].tobytes()] if hi < G else []
        rd = synth.reads_from_strings(inside + outside)
        co = np.arange(rd.n + 1, dtype=np.int64)
        cb = np.full(rd.n, x, np.int32)
        dist, match = oracle.verify(ref, B, O, q, rd.bases, rd.offsets, co, cb, max_edits=np.zeros(rd.n, np.uint16))
        assert list(dist[:2]) == [0, 0] and list(match[:2]) == [1, 1]
        if outside:
            assert dist[2] >= 1 and match[2] == 0
    # the last bin's bases end with the reference
    lo, hi = oracle.bin_bases(9, G, B, O, q)
    assert hi == G


def test_verify_truth_locations(oracle):
    """Each synthetic read is within its applied edits of its true location, and the
    bin holding that location is verified as a mapping (edits <= E)."""
    w = C.shrink(C.workload("c1"), genome_len=200_000, n_reads=300)
    ref = synth.genome(w.genome)
    rd = synth.reads(w.reads, ref)
    truth = (rd.truth_pos // w.bin_size).astype(np.int32)
    nb = -(-len(ref) // w.bin_size)
    far = ((truth + nb // 2) % nb).astype(np.int32)   # a bin far from the truth
    co = np.arange(0, 2 * rd.n + 1, 2, dtype=np.int64)
    cb = np.stack([truth, far], axis=1).reshape(-1)
    E = np.full(rd.n, w.max_edits, np.uint16)
    dist, match = oracle.verify(ref, w.bin_size, w.overlap, w.q, rd.bases, rd.offsets, co, cb, max_edits=E)
    d_truth, d_far = dist[0::2], dist[1::2]
    assert (d_truth <= rd.n_edits).all()
    assert match[0::2].all()
    assert (d_truth == w.max_edits).any()   # the budget is reached, not only approached
    assert (d_far > w.max_edits).mean() > 0.95
    assert rd.n_edits.max() == w.max_edits


def test_verify_mask_skips_pairs(oracle):
    rng = random.Random(5)
    ref = np.frombuffer(_rand(rng, 5000), np.uint8).copy()
    rd = synth.reads_from_strings([ref[100:160].tobytes(), ref[2100:2160].tobytes()])
    co = np.array([0, 2, 4], np.int64)
    cb = np.array([0, 1, 0, 1], np.int32)
    mask = np.array([1, 0, 0, 1], np.uint8)
    dist, match = oracle.verify(ref, 2048, 105, 5, rd.bases, rd.offsets, co, cb, verify_mask=mask,
                                max_edits=np.array([0, 0], np.uint16))
    assert dist[0] == 0 and match[0] == 1
    assert dist[1] == 0xFFFF and match[1] == 0 and dist[2] == 0xFFFF and match[2] == 0
    assert dist[3] == 0 and match[3] == 1
