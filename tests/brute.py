"""Brute-force checkers for tiny inputs, independent of the C oracle.

* ``bin_token_sets`` / ``brute_counts`` recount with Python sets of
  substrings: no token codes, no bit vectors, so an encoding or indexing slip
  in the oracle cannot be mirrored here.
* ``starts_within`` finds, by dynamic programming over the whole reference,
  every start p from which the read aligns with at most E edits (Levenshtein
  distance to some reference substring beginning at p). GRIM-Filter must pass
  the bin holding p for each of them (Section 3: a location is checked against
  the bin of its first base; the threshold is the worst case over E errors).
"""

from __future__ import annotations

from typing import List, Sequence, Set

import numpy as np

ACGT = set(b"ACGT")


def bin_token_sets(ref: bytes, B: int, O: int, q: int) -> List[Set[bytes]]:
    G = len(ref)
    nb = -(-G // B)
    sets = []
    for x in range(nb):
        lo, hi = x * B, min(x * B + B + O, G - q + 1)
        sets.append({ref[s:s + q] for s in range(lo, hi) if set(ref[s:s + q]) <= ACGT})
    return sets


def brute_count(read: bytes, S: Set[bytes], q: int) -> int:
    return sum(1 for i in range(len(read) - q + 1) if read[i:i + q] in S)


def brute_counts(ref: bytes, reads: Sequence[bytes], B: int, O: int, q: int) -> np.ndarray:
    sets = bin_token_sets(ref, B, O, q)
    out = np.zeros((len(reads), len(sets)), dtype=np.int64)
    for r, rd in enumerate(reads):
        for x, S in enumerate(sets):
            out[r, x] = brute_count(rd, S, q)
    return out


def starts_within(read: bytes, ref: bytes, E: int) -> List[int]:
    """Every p such that min_j ED(read, ref[p:j]) <= E.

    Sellers' approximate-matching recurrence run on the reversed strings: an
    occurrence ending at reversed-text position j starts at p = G - j forward.
    """
    P = np.frombuffer(read[::-1], dtype=np.uint8)
    T = np.frombuffer(ref[::-1], dtype=np.uint8)
    m, G = len(P), len(T)
    idx = np.arange(m + 1, dtype=np.int64)
    prev = idx.copy()                     # column j = 0: D[i][0] = i
    out = []
    cand = np.empty(m + 1, dtype=np.int64)
    for j in range(1, G + 1):
        c = T[j - 1]
        cand[0] = 0                       # free start in the text
        cand[1:] = np.minimum(prev[:-1] + (P != c), prev[1:] + 1)
        cur = np.minimum.accumulate(cand - idx) + idx   # vertical moves (read base unaligned)
        if cur[m] <= E:
            out.append(G - j)
        prev = cur
    return sorted(out)


def edit_distance(a: bytes, b: bytes) -> int:
    """Plain Levenshtein distance (for checking the synthetic edit scripts)."""
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j - 1] + (a[i - 1] != b[j - 1]), prev[j] + 1, cur[j - 1] + 1)
        prev = cur
    return prev[-1]
