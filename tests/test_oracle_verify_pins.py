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


# -- bounded verification ----------------------------------------------------
# A mapper's verification only decides whether a location maps within the
# read's budget E_r (Section 1, seed-and-extend step 5), so the bounded form
# reports a distance above E_r as E_r + 1. The cases below use a reference of
# A only, where a read's distance is known by construction: every base other
# than A costs exactly one edit (a substitution) and nothing cheaper exists,
# since such a base can never match.

def _bounded_case(oracle, reads, G=1000, B=200, O=60, q=4, **budget):
    ref = np.full(G, ord("A"), np.uint8)
    rd = synth.reads_from_strings(reads)
    co = np.arange(rd.n + 1, dtype=np.int64)
    cb = np.ones(rd.n, np.int32)
    return oracle.verify_bounded(ref, B, O, q, rd.bases, rd.offsets, co, cb, **budget)


def _read_with(m, L=20, other=b"C"):
    """A read of L bases holding m non-A bases (its distance to an A-only bin is m)."""
    return b"A" * 7 + other * m + b"A" * (L - 7 - m)


def test_verify_bounded_explicit_budget(oracle):
    # (bases that cost an edit, E) -> reported distance, match
    cases = [(0, 3, 0, 1), (2, 3, 2, 1), (3, 3, 3, 1), (4, 3, 4, 0), (5, 3, 4, 0), (9, 3, 4, 0),
             (1, 0, 1, 0), (7, 0, 1, 0), (6, 6, 6, 1), (12, 5, 6, 0)]
    reads = [_read_with(m) for m, _, _, _ in cases]
    E = np.array([e for _, e, _, _ in cases], np.uint16)
    dist, match = _bounded_case(oracle, reads, max_edits=E)
    assert dist.tolist() == [d for _, _, d, _ in cases]
    assert match.tolist() == [mm for _, _, _, mm in cases]
    # a base other than A, C, G, T costs an edit in the read too
    dist, match = _bounded_case(oracle, [_read_with(2, other=b"N"), _read_with(5, other=b"N")],
                                max_edits=np.array([2, 2], np.uint16))
    assert dist.tolist() == [2, 3] and match.tolist() == [1, 0]


def test_verify_bounded_ceiling_budget(oracle):
    """E_r = ceil(e * L) from the per-read rate, or from the rate of every read
    (Section 6, read-existence figure caption): L = 20 and e = 110 per mille give
    E = ceil(2.2) = 3 (2 with a floor), e = 149 gives 3, e = 100 gives exactly 2."""
    reads = [_read_with(5), _read_with(5), _read_with(5), _read_with(3), _read_with(3)]
    e = np.array([110, 149, 100, 110, 100], np.uint16)
    dist, match = _bounded_case(oracle, reads, err_pm_per_read=e)
    assert dist.tolist() == [4, 4, 3, 3, 3]
    assert match.tolist() == [0, 0, 0, 1, 0]
    dist, match = _bounded_case(oracle, reads, err_permille=110)
    assert dist.tolist() == [4, 4, 4, 3, 3]
    assert match.tolist() == [0, 0, 0, 1, 1]
    dist, _ = _bounded_case(oracle, reads, err_permille=0)
    assert dist.tolist() == [1, 1, 1, 1, 1]


def test_verify_bounded_keeps_skipped_pairs(oracle):
    ref = np.full(1000, ord("A"), np.uint8)
    rd = synth.reads_from_strings([_read_with(6), _read_with(1)])
    co = np.array([0, 2, 4], np.int64)
    cb = np.array([1, 2, 1, 2], np.int32)
    mask = np.array([0, 1, 1, 0], np.uint8)
    dist, match = oracle.verify_bounded(ref, 200, 60, 4, rd.bases, rd.offsets, co, cb, verify_mask=mask,
                                        max_edits=np.array([2, 2], np.uint16))
    assert dist.tolist() == [0xFFFF, 3, 1, 0xFFFF]
    assert match.tolist() == [0, 0, 1, 0]


def test_verify_bounded_largest_values(oracle):
    """Distances stay below the skipped marker 0xFFFF: a read of 70000 C bases
    against a one-base bin of A is 70000 edits away, reported as 0xFFFE whatever
    the budget; match compares the true distance."""
    reads = [b"C" * 70000, b"C" * 70000, b"C" * 70000]
    E = np.array([0xFFFF, 0xFFFE, 3], np.uint16)
    dist, match = _bounded_case(oracle, reads, G=10, B=1, O=0, q=1, max_edits=E)
    assert dist.tolist() == [0xFFFE, 0xFFFE, 4]
    assert match.tolist() == [0, 0, 0]
    d_full, m_full = oracle.verify(np.full(10, ord("A"), np.uint8), 1, 0, 1, np.frombuffer(b"C" * 70000, np.uint8),
                                   np.array([0, 70000], np.int64), np.array([0, 1], np.int64),
                                   np.array([1], np.int32), max_edits=np.array([0xFFFF], np.uint16))
    assert d_full.tolist() == [0xFFFE] and m_full.tolist() == [0]


@pytest.mark.parametrize("seed", range(2))
def test_verify_bounded_bruteforce(oracle, seed):
    """On random inputs the bounded distance is the brute-force distance while it
    is within the budget and budget + 1 beyond it."""
    rng = random.Random(300 + seed)
    G, B, O, q = 400, 60, 30, 3
    ref = np.frombuffer(_rand(rng, G), np.uint8).copy()
    nb = -(-G // B)
    reads = [_rand(rng, rng.randrange(q, 18)) for _ in range(12)]
    rd = synth.reads_from_strings(reads)
    co = np.arange(0, 3 * rd.n + 1, 3, dtype=np.int64)
    cb = np.array([rng.randrange(nb) for _ in range(3 * rd.n)], np.int32)
    E = np.array([rng.randrange(0, 8) for _ in range(rd.n)], np.uint16)
    dist, _ = oracle.verify_bounded(ref, B, O, q, rd.bases, rd.offsets, co, cb, max_edits=E)
    for r, read in enumerate(reads):
        for k in range(int(co[r]), int(co[r + 1])):
            lo, hi = oracle.bin_bases(int(cb[k]), G, B, O, q)
            text = ref[lo:hi].tobytes()
            d = min(edit_distance(read, text[a:b]) for a in range(len(text) + 1)
                    for b in range(a, min(len(text), a + len(read) + 10) + 1))
            assert dist[k] == (d if d <= E[r] else E[r] + 1), (r, k)
