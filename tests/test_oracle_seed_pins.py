"""Pins of the oracle's seeding step (no GPU): the candidate bins a read's
seed hits vote for, ranked and capped (the seed-and-extend steps that precede
the filter, paper Section 1). Checked against a brute force that finds every
occurrence of every seed by direct comparison, against the synthetic-input
generator's own table-based implementation, and against constructed cases for
the tie order, the cap, the clamp at the reference start, and invalid seeds."""

from __future__ import annotations

import random
from collections import Counter

import numpy as np
import pytest

import synth
import synth.configs as C


def brute_candidates(ref: bytes, reads, k: int, B: int, cap: int):
    up = ref.upper()
    ok = set(b"ACGT")
    offs = [0]
    bins_all = []
    for s in reads:
        s = s.upper()
        votes = Counter()
        for o in range(0, len(s) - k + 1, k):
            seed = s[o:o + k]
            if not set(seed) <= ok:
                continue
            for p in range(len(up) - k + 1):
                if up[p:p + k] == seed:
                    votes[max(p - o, 0) // B] += 1
        ranked = sorted(votes.items(), key=lambda bv: (-bv[1], bv[0]))[:cap]
        bins = sorted(b for b, _ in ranked)
        bins_all.extend(bins)
        offs.append(offs[-1] + len(bins))
    return np.array(offs, np.int64), np.array(bins_all, np.int32)


def rand_genome(rng: random.Random, G: int) -> bytes:
    g = bytearray(rng.choice(b"ACGT") for _ in range(G))
    for _ in range(12):                      # repeats: copies of a few segments
        a, L = rng.randrange(G - 60), rng.randrange(20, 60)
        b = rng.randrange(G - L)
        g[b:b + L] = g[a:a + L]
    for _ in range(3):
        p = rng.randrange(G - 5)
        g[p:p + 3] = b"NNN"
    p = rng.randrange(G - 40)
    g[p:p + 40] = bytes(g[p:p + 40]).lower()
    return bytes(g)


@pytest.mark.parametrize("seed", range(3))
def test_seed_candidates_bruteforce(oracle, seed):
    rng = random.Random(40 + seed)
    k, B, cap = (6, 100, 5) if seed < 2 else (8, 64, 3)
    ref = rand_genome(rng, 3000)
    reads = []
    for _ in range(25):
        L = rng.randrange(3, 60)
        p = rng.randrange(len(ref) - L)
        s = bytearray(ref[p:p + L])
        for _ in range(rng.randrange(0, 3)):
            s[rng.randrange(L)] = rng.choice(b"ACGTN")
        reads.append(bytes(s))
    rd = synth.reads_from_strings(reads)
    co, cb = oracle.seed_candidates(np.frombuffer(ref, np.uint8), rd.bases, rd.offsets, k, B, cap)
    wo, wb = brute_candidates(ref, reads, k, B, cap)
    assert np.array_equal(co, wo) and np.array_equal(cb, wb)


def test_seed_candidates_equal_input_generator(oracle):
    """The synthetic-input generator's table-based seeding (used for the candidate workloads)
    and the oracle agree on the 100 Mbp recipe at 2 Mbp."""
    w = C.shrink(C.workload("c2"), genome_len=2_000_000, n_reads=3000)
    ref = synth.genome(w.genome)
    rd = synth.reads(w.reads, ref)
    co, cb = synth.candidates(ref, rd, w.bin_size, w.cand_cap, w.cand_k)
    oo, ob = oracle.seed_candidates(ref, rd.bases, rd.offsets, w.cand_k, w.bin_size, w.cand_cap)
    assert np.array_equal(co, oo) and np.array_equal(cb, ob)


def test_seed_ties_cap_and_clamp(oracle):
    k, B = 4, 10
    # a T run with "ACGT" at 5, 25, 45, 65
    ref = bytearray(b"T" * 80)
    for p in (5, 25, 45, 65):
        ref[p:p + 4] = b"ACGT"
    arr = np.frombuffer(bytes(ref), np.uint8)
    rd = synth.reads_from_strings([b"ACGT", b"ACG", b"TTTTACGT", b"ACNT"])
    co, cb = oracle.seed_candidates(arr, rd.bases, rd.offsets, k, B, 2)
    # read 0: bins 0, 2, 4, 6 with one vote each; ties go to the smaller bins
    assert list(cb[co[0]:co[1]]) == [0, 2]
    # read 1 is shorter than k; read 3's only seed holds an N
    assert co[2] - co[1] == 0 and co[4] - co[3] == 0
    # read 2: "TTTT" (offset 0) votes 10 times in bins 1, 3, 5 (no ACGT site inside),
    # fewer elsewhere; "ACGT" (offset 4) adds one vote to bins 0, 2, 4, 6
    assert list(cb[co[2]:co[3]]) == [1, 3]
    # a hit before the seed's offset counts for bin 0: "ACGT" at read offset 20 is
    # found at 5 (location -15, clamped to 0) and at 25, 45, 65 (locations 5, 25,
    # 45: bins 0, 2, 4); the N seeds are skipped
    rd2 = synth.reads_from_strings([b"N" * 20 + b"ACGT"])
    co2, cb2 = oracle.seed_candidates(arr, rd2.bases, rd2.offsets, k, B, 100)
    assert list(cb2) == [0, 2, 4]
