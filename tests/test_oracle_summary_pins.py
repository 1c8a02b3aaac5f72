"""Pins of the oracle's per-read mask summary (no GPU): the pass count and the
digest of a packed pass row. The mixing function is checked against the
published SplitMix64 outputs for seed 0 (Steele, Lea and Flood 2014), the
packing against numpy's own little-endian bit packing, and the digest's
composition through properties any mistake in it would break: it sees every
bit, it sees each word's position, and a change to one word changes it by that
word's term alone."""

from __future__ import annotations

import numpy as np

# SplitMix64 seeded with 0: the state advances by 0x9E3779B97F4A7C15 before the
# output function is applied, and the first three outputs are these
SPLITMIX64_SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
GOLDEN = 0x9E3779B97F4A7C15


def test_mix64_is_splitmix64_output(oracle):
    states = np.array([(GOLDEN * k) % (1 << 64) for k in (1, 2, 3)], dtype=np.uint64)
    got = [int(v) for v in oracle.mix64(states)]
    assert got == SPLITMIX64_SEED0
    assert int(oracle.mix64(np.array([0], np.uint64))[0]) == 0


def test_pack_rows_matches_numpy_bit_packing(oracle):
    rng = np.random.default_rng(5)
    for nb in (1, 31, 32, 33, 95, 200):
        passed = rng.random((7, nb)) < 0.4
        words = oracle.pack_rows(passed)
        W = (nb + 31) // 32
        padded = np.zeros((7, W * 32), bool)
        padded[:, :nb] = passed
        want = np.packbits(padded, axis=1, bitorder="little").view("<u4").reshape(7, W)
        assert np.array_equal(words, want), nb


def test_summary_counts_and_digest_properties(oracle):
    rng = np.random.default_rng(11)
    nb = 100
    passed = rng.random((6, nb)) < 0.5
    counts, digests = oracle.mask_summary(passed)
    assert np.array_equal(counts, passed.sum(axis=1))
    # an empty row: every word is 0, so the digest is the sum of mix64(i << 32)
    zero_c, zero_d = oracle.mask_summary(np.zeros((1, nb), bool))
    assert zero_c[0] == 0
    terms = oracle.mix64(np.arange(4, dtype=np.uint64) << np.uint64(32))
    with np.errstate(over="ignore"):
        assert zero_d[0] == terms.sum(dtype=np.uint64)
    # one bit flipped: the digest moves by that word's term only
    row = passed[0].copy()
    flipped = row.copy()
    flipped[37] = not flipped[37]
    (_, (d0, d1)) = oracle.mask_summary(np.stack([row, flipped]))
    w0 = oracle.pack_rows(row[None])[0].astype(np.uint64)
    w1 = oracle.pack_rows(flipped[None])[0].astype(np.uint64)
    t0 = oracle.mix64(np.uint64(1 << 32) | w0[1])
    t1 = oracle.mix64(np.uint64(1 << 32) | w1[1])
    with np.errstate(over="ignore"):
        assert d1 - d0 == t1 - t0
    assert d0 != d1
    # the same words in another order give another digest (positions count)
    a = np.zeros((1, 64), bool)
    a[0, 3] = True                       # word 0 = 8, word 1 = 0
    b = np.zeros((1, 64), bool)
    b[0, 35] = True                      # word 0 = 0, word 1 = 8
    assert oracle.mask_summary(a)[1][0] != oracle.mask_summary(b)[1][0]
