"""ctypes front end of the GRIM-Filter CPU oracle (``grim_oracle.c``).

TEST INFRASTRUCTURE ONLY: the library and its binding never import this
module. Only the tests, the smoke check and the benchmark's CPU-baseline leg
use it, to check the GPU path and to time a CPU baseline.

Every function mirrors one C function and cites the paper passage it
follows (arXiv 1708.04329):
  * bits               Section 3, bit vector generation; Section 6.1 (4^q bits)
  * threshold          Section 3, threshold paragraph (L-(q-1) tokens, q per error)
  * max_edits          Section 6, read-existence figure caption (ceil of L*e)
  * scan_all           Section 3, steps 1-3 over every bin
  * scan_candidates    Section 3, steps 4-5 (bin of the location's first base)
  * seed_candidates    Section 1, seed-and-extend steps 2-4 (seeds of a read,
                       looked up in the reference, give candidate locations)
  * semiglobal_distance, verify, verify_bounded
                       Section 1, seed-and-extend step 5 (dynamic-programming
                       alignment of the read at a location) and Section 5,
                       evaluation metrics (a passing location either yields a
                       mapping or counts against the filter)
  * mask_summary       per read, the number of bins that pass (Section 3, step 3
                       outcome) and a digest of the packed row: a library
                       convention, not the paper's; mix64 is the SplitMix64
                       output function (Steele, Lea and Flood 2014)
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grim_oracle.c")
_LIB = os.path.join(_HERE, "libgrimoracle.so")

BUILD_CMD = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", "-Wextra"]


def build(src: str = _SRC, out: str = _LIB) -> str:
    subprocess.check_call(BUILD_CMD + [src, "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


_cache = {}


def load(path: str = _LIB):
    """Load (building if absent) the oracle library at ``path``."""
    if path in _cache:
        return _cache[path]
    if not os.path.exists(path):
        if path != _LIB:
            raise FileNotFoundError(path)
        build()
    lib = ctypes.CDLL(path)
    P, U64, U32, I64, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int
    lib.oracle_token_code.argtypes = [P, U32]
    lib.oracle_token_code.restype = I64
    lib.oracle_vector_bits.argtypes = [U32]
    lib.oracle_vector_bits.restype = U64
    lib.oracle_num_bins.argtypes = [U64, U32]
    lib.oracle_num_bins.restype = U64
    lib.oracle_index_bytes.argtypes = [U64, U32]
    lib.oracle_index_bytes.restype = U64
    lib.oracle_bin_extent.argtypes = [U64, U64, U32, U32, U32, P, P]
    lib.oracle_bin_extent.restype = None
    lib.oracle_build_bits.argtypes = [P, U64, U32, U32, U32, P, I]
    lib.oracle_build_bits.restype = I
    lib.oracle_max_edits.argtypes = [U32, U32]
    lib.oracle_max_edits.restype = U32
    lib.oracle_threshold.argtypes = [U32, U32, U32]
    lib.oracle_threshold.restype = I64
    lib.oracle_count.argtypes = [P, P, U32, U32]
    lib.oracle_count.restype = U32
    lib.oracle_thresholds.argtypes = [P, U64, U32, P, P, U32, P]
    lib.oracle_thresholds.restype = None
    lib.oracle_scan_all.argtypes = [P, U64, U32, P, P, U64, P, P, U32, P, P, I]
    lib.oracle_scan_all.restype = I
    lib.oracle_scan_candidates.argtypes = [P, U64, U32, P, P, U64, P, P, U32, P, P, P, P, I]
    lib.oracle_scan_candidates.restype = I
    lib.oracle_semiglobal_distance.argtypes = [P, U32, P, U64]
    lib.oracle_semiglobal_distance.restype = U32
    lib.oracle_bin_bases.argtypes = [U64, U64, U32, U32, U32, P, P]
    lib.oracle_bin_bases.restype = None
    lib.oracle_verify.argtypes = [P, U64, U32, U32, U32, P, P, U64, P, P, U32, P, P, P, P, P, I]
    lib.oracle_verify.restype = I
    lib.oracle_verify_bounded.argtypes = [P, U64, U32, U32, U32, P, P, U64, P, P, U32, P, P, P, P, P, I]
    lib.oracle_verify_bounded.restype = I
    lib.oracle_seed_candidates.argtypes = [P, U64, P, P, U64, U32, U32, U32, P, P]
    lib.oracle_seed_candidates.restype = I64
    lib.oracle_threads.argtypes = [I]
    lib.oracle_threads.restype = I
    _cache[path] = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8)


class Oracle:
    """Plain-loop GRIM-Filter on the CPU (one byte per existence bit)."""

    def __init__(self, path: str = _LIB, threads: int = 0):
        self.lib = load(path)
        self.threads = threads

    # -- small helpers, one per paper formula ---------------------------------
    def token_code(self, s: bytes, q: int) -> int:
        return int(self.lib.oracle_token_code(_p(_u8(s)), q))

    def vector_bits(self, q: int) -> int:
        return int(self.lib.oracle_vector_bits(q))

    def num_bins(self, G: int, B: int) -> int:
        return int(self.lib.oracle_num_bins(G, B))

    def index_bytes(self, n_bins: int, q: int) -> int:
        return int(self.lib.oracle_index_bytes(n_bins, q))

    def bin_extent(self, x: int, G: int, B: int, O: int, q: int):
        lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
        self.lib.oracle_bin_extent(x, G, B, O, q, ctypes.byref(lo), ctypes.byref(hi))
        return lo.value, hi.value

    def max_edits(self, L: int, e_permille: int) -> int:
        return int(self.lib.oracle_max_edits(L, e_permille))

    def threshold(self, L: int, q: int, E: int) -> int:
        return int(self.lib.oracle_threshold(L, q, E))

    # -- bit vectors and scans -----------------------------------------------
    def bits(self, ref, B: int, O: int, q: int) -> np.ndarray:
        """uint8 [n_bins, 4^q]: 1 where the token starts inside the bin's extent."""
        ref = _u8(ref)
        nb = self.num_bins(len(ref), B)
        out = np.empty((nb, self.vector_bits(q)), dtype=np.uint8)
        if self.lib.oracle_build_bits(_p(ref), len(ref), B, O, q, _p(out), self.threads) != 0:
            raise ValueError("oracle_build_bits: bad parameters")
        return out

    def count(self, bits_of_bin: np.ndarray, read: bytes, q: int) -> int:
        rd = _u8(read)
        return int(self.lib.oracle_count(_p(np.ascontiguousarray(bits_of_bin, np.uint8)), _p(rd), len(rd), q))

    @staticmethod
    def _edits(n, max_edits, err_pm_per_read):
        me = None if max_edits is None else np.ascontiguousarray(max_edits, np.uint16)
        ep = None if err_pm_per_read is None else np.ascontiguousarray(err_pm_per_read, np.uint16)
        for a in (me, ep):
            if a is not None and len(a) != n:
                raise ValueError("per-read array length")
        return me, ep

    def thresholds(self, offsets, q, max_edits=None, err_pm_per_read=None, err_permille=0):
        offs = np.ascontiguousarray(offsets, np.int64)
        n = len(offs) - 1
        me, ep = self._edits(n, max_edits, err_pm_per_read)
        out = np.empty(n, dtype=np.int64)
        self.lib.oracle_thresholds(_p(offs), n, q, _p(me), _p(ep), err_permille, _p(out))
        return out

    def scan_all(self, bits: np.ndarray, q: int, bases, offsets, max_edits=None,
                 err_pm_per_read=None, err_permille: int = 0, want_counts: bool = True):
        """(counts uint16 [n, nb] or None, pass uint8 [n, nb])."""
        bases = _u8(bases)
        offs = np.ascontiguousarray(offsets, np.int64)
        n, nb = len(offs) - 1, bits.shape[0]
        me, ep = self._edits(n, max_edits, err_pm_per_read)
        counts = np.empty((n, nb), dtype=np.uint16) if want_counts else None
        pas = np.empty((n, nb), dtype=np.uint8)
        self.lib.oracle_scan_all(_p(bits), nb, q, _p(bases), _p(offs), n, _p(me), _p(ep),
                                 err_permille, _p(counts), _p(pas), self.threads)
        return counts, pas

    @staticmethod
    def mix64(z):
        """SplitMix64's output function on uint64 values (wrapping arithmetic)."""
        z = np.asarray(z, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            return z ^ (z >> np.uint64(31))

    @staticmethod
    def pack_rows(passed: np.ndarray) -> np.ndarray:
        """Pass matrix [n, nb] -> uint32 words [n, ceil(nb/32)], bit x % 32 of word x // 32."""
        n, nb = passed.shape
        W = (nb + 31) // 32
        weights = np.uint64(1) << np.arange(32, dtype=np.uint64)      # bit b has weight 2^b
        words = np.zeros((n, W), dtype=np.uint32)
        step = max(1, (1 << 24) // max(1, W * 32))                     # rows per chunk
        for r0 in range(0, n, step):
            chunk = np.zeros((min(step, n - r0), W * 32), dtype=np.uint64)
            chunk[:, :nb] = passed[r0:r0 + step]
            words[r0:r0 + step] = (chunk.reshape(-1, W, 32) * weights).sum(axis=2).astype(np.uint32)
        return words

    def mask_summary(self, passed: np.ndarray):
        """(pass count uint32 [n], digest uint64 [n]) of a pass matrix [n, nb]:
        the count of passing bins, and the sum over the packed row's words i of
        mix64((i << 32) | word_i), modulo 2^64."""
        passed = np.asarray(passed) != 0
        counts = passed.sum(axis=1).astype(np.uint32)
        words = self.pack_rows(passed)
        idx = np.arange(words.shape[1], dtype=np.uint64) << np.uint64(32)
        digests = np.zeros(len(words), dtype=np.uint64)
        with np.errstate(over="ignore"):
            for r in range(len(words)):
                digests[r] = self.mix64(words[r].astype(np.uint64) | idx).sum(dtype=np.uint64)
        return counts, digests

    def scan_candidates(self, bits: np.ndarray, q: int, bases, offsets, cand_off, cand_bin,
                        max_edits=None, err_pm_per_read=None, err_permille: int = 0):
        """(counts uint16 [P], pass uint8 [P]) in candidate (CSR) order."""
        bases = _u8(bases)
        offs = np.ascontiguousarray(offsets, np.int64)
        co = np.ascontiguousarray(cand_off, np.int64)
        cb = np.ascontiguousarray(cand_bin, np.int32)
        n, nb = len(offs) - 1, bits.shape[0]
        me, ep = self._edits(n, max_edits, err_pm_per_read)
        P = len(cb)
        counts = np.empty(P, dtype=np.uint16)
        pas = np.empty(P, dtype=np.uint8)
        rc = self.lib.oracle_scan_candidates(_p(bits), nb, q, _p(bases), _p(offs), n, _p(me), _p(ep),
                                             err_permille, _p(co), _p(cb), _p(counts), _p(pas),
                                             self.threads)
        if rc != 0:
            raise ValueError("candidate bin out of range")
        return counts, pas

    def semiglobal_distance(self, read: bytes, text: bytes) -> int:
        """Smallest edit distance of the whole read to any substring of text."""
        r = _u8(np.frombuffer(bytes(read), np.uint8))
        t = _u8(np.frombuffer(bytes(text), np.uint8))
        return int(self.lib.oracle_semiglobal_distance(_p(r), len(r), _p(t), len(t)))

    def bin_bases(self, x: int, G: int, B: int, O: int, q: int):
        """Bases [lo, hi) covered by the tokens of bin x."""
        lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
        self.lib.oracle_bin_bases(x, G, B, O, q, ctypes.byref(lo), ctypes.byref(hi))
        return lo.value, hi.value

    def verify(self, ref, B: int, O: int, q: int, bases, offsets, cand_off, cand_bin, verify_mask=None,
               max_edits=None, err_pm_per_read=None, err_permille: int = 0, bounded: bool = False):
        """(dist uint16 [P], match uint8 [P]) in candidate (CSR) order; pairs whose
        verify_mask entry is 0 get dist 0xFFFF and match 0. With ``bounded``, a
        distance above the read's budget E_r reads E_r + 1 (at most 0xFFFE)."""
        ref = _u8(ref)
        bases = _u8(bases)
        offs = np.ascontiguousarray(offsets, np.int64)
        co = np.ascontiguousarray(cand_off, np.int64)
        cb = np.ascontiguousarray(cand_bin, np.int32)
        vm = None if verify_mask is None else np.ascontiguousarray(verify_mask, np.uint8)
        n = len(offs) - 1
        me, ep = self._edits(n, max_edits, err_pm_per_read)
        P = len(cb)
        dist = np.empty(P, dtype=np.uint16)
        match = np.empty(P, dtype=np.uint8)
        fn = self.lib.oracle_verify_bounded if bounded else self.lib.oracle_verify
        rc = fn(_p(ref), len(ref), B, O, q, _p(bases), _p(offs), n, _p(me), _p(ep), err_permille, _p(co), _p(cb),
                _p(vm), _p(dist), _p(match), self.threads)
        if rc != 0:
            raise ValueError("candidate bin out of range")
        return dist, match

    def verify_bounded(self, ref, B: int, O: int, q: int, bases, offsets, cand_off, cand_bin, verify_mask=None,
                       max_edits=None, err_pm_per_read=None, err_permille: int = 0):
        """verify() with each distance above the read's budget E_r reported as E_r + 1
        (capped at 0xFFFE); match flags and skipped pairs (0xFFFF) unchanged."""
        return self.verify(ref, B, O, q, bases, offsets, cand_off, cand_bin, verify_mask, max_edits,
                           err_pm_per_read, err_permille, bounded=True)

    def seed_candidates(self, ref, bases, offsets, k: int, B: int, cap: int):
        """(cand_off int64 [n+1], cand_bin int32 [n_cand]) of the seed-hit candidates."""
        ref = _u8(ref)
        bases = _u8(bases)
        offs = np.ascontiguousarray(offsets, np.int64)
        n = len(offs) - 1
        co = np.empty(n + 1, np.int64)
        cb = np.empty(max(1, n * cap), np.int32)
        total = self.lib.oracle_seed_candidates(_p(ref), len(ref), _p(bases), _p(offs), n, k, B, cap, _p(co),
                                                _p(cb))
        if total < 0:
            raise ValueError("bad seeding arguments")
        return co, cb[:total].copy()

    def threads_used(self) -> int:
        return int(self.lib.oracle_threads(self.threads))
