"""Pins for the CPU oracle: values the paper prints, closed forms, invariants
and brute force on tiny inputs. These run without a GPU."""

from __future__ import annotations

import json
import math
import os
import random

import numpy as np
import pytest

import synth
from brute import bin_token_sets, brute_count, brute_counts, edit_distance, starts_within

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")
FACTS = json.load(open(GOLDEN))


def rand_seq(rng: random.Random, n: int, alphabet=b"ACGT") -> bytes:
    return bytes(rng.choice(alphabet) for _ in range(n))


# --------------------------------------------------------------------------
# Values printed in the paper
# --------------------------------------------------------------------------

def test_vector_length_q5(oracle):
    # Section 6.1: 4^5 = 1024 bits per bin
    assert oracle.vector_bits(5) == FACTS["vector_bits_q5"]["value"]


def test_index_footprint_paper(oracle):
    # Section 6.1: 450x64k bins of 1024 bits, about 3.8 GB
    f = FACTS["index_footprint_450x64k_q5"]
    got = oracle.index_bytes(f["n_bins"], f["q"])
    assert abs(got - f["approx_bytes"]) <= f["tolerance_bytes"]


def test_counter_width_100bp(oracle):
    # Section 4.2: 7-bit counters for 100 bp reads; the largest sum is the
    # number of tokens of the read.
    f = FACTS["counter_bits_100bp"]
    L = f["read_length"]
    assert math.ceil(math.log2(L)) == f["bits"]
    ref = b"A" * 300
    bits = oracle.bits(ref, 300, 0, 5)
    cnt = oracle.count(bits[0], b"A" * L, 5)
    assert cnt == L - 5 + 1 and cnt < 2 ** f["bits"]


def test_exact_match_threshold(oracle):
    # Section 3: with no errors the threshold is the token count L - (q - 1)
    for L, q, want in FACTS["exact_match_threshold"]["cases"]:
        assert oracle.threshold(L, q, 0) == want


def test_ceil_error_budget(oracle):
    # Section 6 read-existence caption: E = ceil(L * e)
    for L, epm, want in FACTS["ceil_error_budget"]["cases"]:
        assert oracle.max_edits(L, epm) == want


def test_error_propagation_q4(oracle):
    # Threshold-equation caption: for q = 4 one substitution in the middle of
    # a read removes 4 tokens. Build a bin and a read copied from it with one
    # substitution whose new tokens are absent from the bin.
    q = FACTS["error_propagation_q4"]["q"]
    lost = FACTS["error_propagation_q4"]["tokens_lost_per_error"]
    rng = random.Random(7)
    seg, read = _tight_case(rng, q=q, L=30, n_sub=1)
    bits = oracle.bits(seg, len(seg), 0, q)
    assert oracle.count(bits[0], read, q) == (30 - q + 1) - lost


# --------------------------------------------------------------------------
# Tightness: the threshold equals the worst case over E errors
# --------------------------------------------------------------------------

def _tight_case(rng, q, L, n_sub, seg_len=None):
    """A segment and a read copied from it with n_sub substitutions spaced
    >= q apart, away from the ends, such that none of the altered tokens
    occurs in the segment: the read keeps exactly (L-q+1) - q*n_sub tokens."""
    seg_len = seg_len or L + 10
    for _ in range(100000):
        seg = rand_seq(rng, seg_len)
        S = {seg[i:i + q] for i in range(seg_len - q + 1)}
        start = rng.randrange(0, seg_len - L + 1)
        read = bytearray(seg[start:start + L])
        span = range(q - 1, L - q + 1)
        pos = sorted(rng.sample(list(span), n_sub)) if n_sub else []
        if any(b - a < q for a, b in zip(pos, pos[1:])):
            continue
        for k in pos:
            read[k] = rng.choice([c for c in b"ACGT" if c != read[k]])
        read = bytes(read)
        bad = False
        for k in pos:
            for i in range(k - q + 1, k + 1):
                if read[i:i + q] in S:
                    bad = True
        if not bad:
            return seg, read
    raise RuntimeError("no tight case found")


@pytest.mark.parametrize("q,L,E", [(3, 30, 2), (4, 40, 3), (5, 60, 4), (5, 100, 5), (6, 100, 3)])
def test_threshold_is_tight(oracle, q, L, E):
    rng = random.Random(q * 1000 + L + E)
    seg, read = _tight_case(rng, q, L, E, seg_len=L + 3 * q)
    bits = oracle.bits(seg, len(seg), 0, q)
    T = oracle.threshold(L, q, E)
    cnt = oracle.count(bits[0], read, q)
    # a read within E substitutions reaches exactly the threshold and passes
    assert cnt == T
    _, pas = oracle.scan_all(bits, q, np.frombuffer(read, np.uint8), np.array([0, L]),
                             max_edits=np.array([E]))
    assert pas[0, 0] == 1
    # one more substitution drops it below and the bin is rejected
    seg2, read2 = _tight_case(rng, q, L, E + 1, seg_len=L + 3 * q)
    bits2 = oracle.bits(seg2, len(seg2), 0, q)
    _, pas2 = oracle.scan_all(bits2, q, np.frombuffer(read2, np.uint8), np.array([0, L]),
                              max_edits=np.array([E]))
    assert pas2[0, 0] == 0


# --------------------------------------------------------------------------
# Brute force on tiny inputs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_counts_match_set_recount(oracle, seed):
    rng = random.Random(seed)
    q = rng.choice([3, 4, 5])
    B = rng.choice([32, 64, 256])
    G = rng.randrange(B, 3000)
    O = rng.randrange(0, 90)
    ref = bytearray(rand_seq(rng, G))
    # a few N runs and lower-case stretches in the reference
    for _ in range(3):
        p = rng.randrange(G)
        ref[p:p + rng.randrange(1, 4)] = b"N" * len(ref[p:p + 3])
    ref = bytes(ref[:G])
    reads = []
    for _ in range(6):
        L = rng.randrange(q, 80)
        p = rng.randrange(0, max(1, G - L))
        rd = bytearray(ref[p:p + L])
        for _ in range(rng.randrange(0, 6)):
            rd[rng.randrange(len(rd))] = rng.choice(b"ACGTN")
        reads.append(bytes(rd))
    reads.append(rand_seq(rng, rng.randrange(q, 60)))
    rd = synth.reads_from_strings(reads)
    bits = oracle.bits(np.frombuffer(ref, np.uint8), B, O, q)
    E = np.array([rng.randrange(0, 9) for _ in reads], dtype=np.uint16)
    counts, pas = oracle.scan_all(bits, q, rd.bases, rd.offsets, max_edits=E)
    want = brute_counts(ref, reads, B, O, q)
    assert counts.shape == want.shape
    assert np.array_equal(counts.astype(np.int64), want)
    for r, L in enumerate(rd.lengths):
        T = (L - q + 1) - q * int(E[r])
        assert np.array_equal(pas[r], (want[r] >= T).astype(np.uint8))


def test_bits_match_set_definition(oracle):
    rng = random.Random(99)
    ref = rand_seq(rng, 700)
    B, O, q = 64, 20, 4
    bits = oracle.bits(ref, B, O, q)
    sets = bin_token_sets(ref, B, O, q)
    for x, S in enumerate(sets):
        got = {i for i in np.nonzero(bits[x])[0]}
        want = set()
        for tok in S:
            code = 0
            for c in tok:
                code = code * 4 + b"ACGT".index(c)
            want.add(code)
        assert got == want


# --------------------------------------------------------------------------
# Zero false negatives: every start within E edits passes its bin
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_no_false_negatives_bruteforce(oracle, seed):
    rng = random.Random(1000 + seed)
    q = rng.choice([3, 4, 5])
    L = rng.randrange(20, 45)
    E = rng.randrange(1, 5)
    B = rng.choice([32, 48, 64])
    O = L + E - q                      # the smallest overlap the guarantee needs
    G = 2500
    ref = rand_seq(rng, G)
    reads, truths = [], []
    for _ in range(5):
        # copy a reference window and apply up to E random edits (S/I/D)
        p = rng.randrange(0, G - L - E)
        rd = bytearray(ref[p:p + L + E])
        for _ in range(rng.randrange(0, E + 1)):
            k = rng.randrange(0, L)
            t = rng.randrange(3)
            if t == 0:
                rd[k] = rng.choice([c for c in b"ACGT" if c != rd[k]])
            elif t == 1:
                rd.insert(k, rng.choice(b"ACGT"))
            else:
                del rd[k]
        reads.append(bytes(rd[:L]))
        truths.append(p)
    rd = synth.reads_from_strings(reads)
    bits = oracle.bits(ref, B, O, q)
    _, pas = oracle.scan_all(bits, q, rd.bases, rd.offsets, max_edits=np.full(len(reads), E, np.uint16))
    n_checked = 0
    for r, read in enumerate(reads):
        starts = starts_within(read, ref, E)
        assert truths[r] in starts or edit_distance(read, ref[truths[r]:truths[r] + L]) > E
        for p in starts:
            assert pas[r, p // B] == 1, (r, p)
            n_checked += 1
    assert n_checked > 0
    # and the filter is not vacuous here: most bins are rejected
    assert pas.mean() < 0.5


def test_overlap_is_needed(oracle):
    # With no overlap a read whose first base is near the end of a bin loses
    # the tokens that spill into the next bin (Section 3: bins must overlap).
    rng = random.Random(5)
    q, L, B = 4, 30, 64
    ref = rand_seq(rng, 256)
    p = B - 5                               # read starts 5 bases before bin 1
    read = ref[p:p + L]
    T = (L - q + 1)
    bits0 = oracle.bits(ref, B, 0, q)
    bitsO = oracle.bits(ref, B, L - q, q)
    assert oracle.count(bitsO[p // B], read, q) == T
    assert oracle.count(bits0[p // B], read, q) < T


# --------------------------------------------------------------------------
# Closed forms and special cases
# --------------------------------------------------------------------------

def test_exact_substring_counts_all_tokens(oracle):
    rng = random.Random(11)
    ref = rand_seq(rng, 5000)
    B, q = 512, 5
    for L in (5, 37, 100):
        O = L - q
        bits = oracle.bits(ref, B, O, q)
        for p in (0, 511, 1234, 5000 - L):
            assert oracle.count(bits[p // B], ref[p:p + L], q) == L - q + 1


def test_homopolymer(oracle):
    q, L = 5, 50
    with_a = b"CG" * 40 + b"AAAAAA" + b"CG" * 40
    without = b"CG" * 80
    for ref, want in ((with_a, L - q + 1), (without, 0)):
        bits = oracle.bits(ref, len(ref), 0, q)
        assert oracle.count(bits[0], b"A" * L, q) == want


def test_repeated_tokens_count_each_time(oracle):
    q = 3
    ref = b"ACGTTTTGCA"
    bits = oracle.bits(ref, len(ref), 0, q)
    read = b"ACGACGACG"                        # ACG three times, CGA and GAC twice
    want = brute_count(read, bin_token_sets(ref, len(ref), 0, q)[0], q)
    assert oracle.count(bits[0], read, q) == want == 3


def test_nonpositive_threshold_passes_everything(oracle):
    rng = random.Random(3)
    ref = rand_seq(rng, 1000)
    bits = oracle.bits(ref, 100, 10, 5)
    read = rand_seq(rng, 40)
    rd = synth.reads_from_strings([read, read])
    E = np.array([8, 9], dtype=np.uint16)     # T = 36 - 40 <= 0 and 36 - 45
    _, pas = oracle.scan_all(bits, 5, rd.bases, rd.offsets, max_edits=E)
    assert pas.all()


def test_count_bounded_by_tokens(oracle):
    rng = random.Random(21)
    ref = rand_seq(rng, 3000)
    bits = oracle.bits(ref, 64, 40, 3)
    reads = [rand_seq(rng, rng.randrange(3, 70)) for _ in range(20)]
    rd = synth.reads_from_strings(reads)
    counts, _ = oracle.scan_all(bits, 3, rd.bases, rd.offsets, max_edits=np.zeros(20, np.uint16))
    assert (counts <= (rd.lengths - 3 + 1)[:, None]).all()


def test_first_base_rule(oracle):
    # Section 3: a token belongs to the bin holding its first base (extended
    # bins: starts below x*B + B + O), even when it ends past that point.
    B, O, q = 50, 10, 4
    ref = bytearray(b"C" * 200)
    ref[59:63] = b"ACGT"                     # starts at 59 = last start of bin 0
    ref[120:124] = b"TTGA"                   # starts at 120 = first start after bin 1
    bits = oracle.bits(bytes(ref), B, O, q)
    acgt, ttga = oracle.token_code(b"ACGT", q), oracle.token_code(b"TTGA", q)
    assert bits[0, acgt] == 1 and bits[1, acgt] == 1
    assert bits[1, ttga] == 0 and bits[2, ttga] == 1
    assert bits[0, ttga] == 0


def test_last_partial_bin_and_tail_token(oracle):
    B, O, q = 64, 8, 4
    ref = b"C" * 197 + b"GTAC"               # G = 201: bins 0..3, the last holds 9 bases
    bits = oracle.bits(ref, B, O, q)
    assert bits.shape[0] == oracle.num_bins(len(ref), B) == 4
    assert bits[3, oracle.token_code(b"GTAC", q)] == 1   # the very last window
    assert oracle.bin_extent(3, len(ref), B, O, q) == (192, 198)


def test_n_windows(oracle):
    q = 4
    ref = b"ACGTNACGTTGCA"
    bits = oracle.bits(ref, len(ref), 0, q)
    # windows with N set no bit: "CGTN", "GTNA", "TNAC", "NACG" absent
    present = {ref[i:i + q] for i in range(len(ref) - q + 1) if b"N" not in ref[i:i + q]}
    got = {i for i in np.nonzero(bits[0])[0]}
    assert got == {oracle.token_code(t, q) for t in present}
    # a read window holding N adds 0 but the threshold keeps L - q + 1 tokens
    read = b"ACGTNACGT"
    assert oracle.count(bits[0], read, q) == 2
    assert oracle.threshold(len(read), q, 0) == 6


def test_encoding_invariance(oracle):
    # Relabelling the four bases consistently in reference and reads maps
    # tokens one-to-one, so counts cannot change.
    rng = random.Random(8)
    ref = rand_seq(rng, 2000)
    reads = [ref[p:p + 60] for p in (10, 700, 1500)] + [rand_seq(rng, 60)]
    perm = bytes.maketrans(b"ACGT", b"GTAC")
    B, O, q = 128, 60, 5
    a = oracle.scan_all(oracle.bits(ref, B, O, q), q, *_packed(reads), max_edits=np.zeros(4, np.uint16))[0]
    b = oracle.scan_all(oracle.bits(ref.translate(perm), B, O, q), q,
                        *_packed([r.translate(perm) for r in reads]), max_edits=np.zeros(4, np.uint16))[0]
    assert np.array_equal(a, b)


def test_lower_case_is_same_base(oracle):
    rng = random.Random(4)
    ref = rand_seq(rng, 500)
    bits_u = oracle.bits(ref, 100, 20, 4)
    bits_l = oracle.bits(ref.lower(), 100, 20, 4)
    assert np.array_equal(bits_u, bits_l)


def _packed(reads):
    rd = synth.reads_from_strings(reads)
    return rd.bases, rd.offsets


# --------------------------------------------------------------------------
# Candidate mode is the all-bins result restricted to the listed bins
# --------------------------------------------------------------------------

def test_candidates_equal_allbins_subset(oracle):
    rng = random.Random(12)
    ref = rand_seq(rng, 4000)
    B, O, q = 128, 40, 4
    bits = oracle.bits(ref, B, O, q)
    reads = [ref[p:p + 40] for p in (0, 100, 2000)] + [rand_seq(rng, 33)]
    rd = synth.reads_from_strings(reads)
    nb = bits.shape[0]
    co = [0]
    cb = []
    for r in range(len(reads)):
        sel = sorted(rng.sample(range(nb), 7))
        cb += sel
        co.append(len(cb))
    E = np.array([2, 1, 0, 3], np.uint16)
    ca, pa = oracle.scan_all(bits, q, rd.bases, rd.offsets, max_edits=E)
    cc, pc = oracle.scan_candidates(bits, q, rd.bases, rd.offsets, np.array(co), np.array(cb, np.int32),
                                    max_edits=E)
    for r in range(len(reads)):
        for k in range(co[r], co[r + 1]):
            assert cc[k] == ca[r, cb[k]] and pc[k] == pa[r, cb[k]]


def test_per_read_error_rates(oracle):
    offs = np.array([0, 100, 250, 500], np.int64)
    T = oracle.thresholds(offs, 6, err_pm_per_read=np.array([20, 30, 50], np.uint16))
    # E = ceil(2.0) = 2, ceil(4.5) = 5, ceil(12.5) = 13
    assert list(T) == [95 - 12, 145 - 30, 245 - 78]


# --------------------------------------------------------------------------
# The synthetic generators do what they claim (inputs, not the method)
# --------------------------------------------------------------------------

def test_synthetic_reads_have_their_edits():
    g = synth.genome(synth.GenomeSpec(length=20000, seed=5))
    spec = synth.ReadSpec(n_reads=40, seed=6, lens=(60,), len_w=(1,), edit_mode=0, edits=3)
    rd = synth.reads(spec, g)
    for r in range(rd.n):
        p, s = int(rd.truth_pos[r]), int(rd.span[r])
        assert edit_distance(rd.read(r), g[p:p + s].tobytes()) <= 3
        assert rd.n_edits[r] == 3
