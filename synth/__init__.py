"""Seeded synthetic inputs for the GRIM-Filter hot path.

The genomes, reads (with their edit scripts and true start positions) and
k-mer seed-hit candidate lists made here feed both the CPU oracle and the GPU
path. Nothing in this module computes any part of the filter itself: no bins,
no q-gram presence bits, no counts and no thresholds.

The C++ core (``synth.cpp``) draws every random number from SplitMix64
(Steele, Lea and Flood, OOPSLA 2014), one independent stream per read and per
genome block, so results do not depend on the thread count.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.cpp")
_LIB = os.path.join(_HERE, "libgrimsynth.so")

MASTER_SEED = 0x170804329


def build(force: bool = True) -> str:
    """Compile ``libgrimsynth.so`` next to its source (g++, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c++17", "-Wall",
               _SRC, "-o", _LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _GenomeParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("length", ctypes.c_uint64),
                ("repeat_frac", ctypes.c_double), ("n_families", ctypes.c_uint32),
                ("fam_len_lo", ctypes.c_uint32), ("fam_len_hi", ctypes.c_uint32),
                ("fam_len_mode", ctypes.c_uint32), ("div_lo", ctypes.c_double),
                ("div_hi", ctypes.c_double), ("indel_share", ctypes.c_double)]


class _ReadParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_reads", ctypes.c_uint64),
                ("n_len", ctypes.c_uint32), ("lens", ctypes.c_uint32 * 4),
                ("len_w", ctypes.c_uint32 * 4), ("n_err", ctypes.c_uint32),
                ("err_pm", ctypes.c_uint32 * 8), ("err_w", ctypes.c_uint32 * 8),
                ("edit_mode", ctypes.c_uint32), ("edits", ctypes.c_uint32),
                ("w_sub", ctypes.c_uint32), ("w_ins", ctypes.c_uint32),
                ("w_del", ctypes.c_uint32), ("n_sub", ctypes.c_uint32),
                ("n_indel", ctypes.c_uint32)]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.synth_genome.argtypes = [ctypes.POINTER(_GenomeParams), P]
        lib.synth_genome.restype = ctypes.c_int64
        lib.synth_read_lengths.argtypes = [ctypes.POINTER(_ReadParams), P]
        lib.synth_read_lengths.restype = ctypes.c_int
        lib.synth_reads.argtypes = [ctypes.POINTER(_ReadParams), P, ctypes.c_uint64, P, P, P, P, P, P]
        lib.synth_reads.restype = ctypes.c_int
        lib.synth_candidates.argtypes = [P, ctypes.c_uint64, P, P, ctypes.c_uint64, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint32, P, P]
        lib.synth_candidates.restype = ctypes.c_int64
        _lib_handle = lib
    return _lib_handle


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class GenomeSpec:
    """Reference genome recipe: uniform ACGT plus interspersed repeat copies."""
    length: int
    seed: int = MASTER_SEED
    repeat_frac: float = 0.0
    n_families: int = 0
    fam_len_lo: int = 300
    fam_len_hi: int = 6000
    fam_len_mode: int = 0          # 0: uniform in [lo, hi]; 1: two classes {lo, hi}, half the bases each
    div_lo: float = 0.10
    div_hi: float = 0.20
    indel_share: float = 0.10


def genome(spec: GenomeSpec) -> np.ndarray:
    """ASCII genome (uint8, 'A','C','G','T') of ``spec.length`` bases."""
    out = np.empty(spec.length, dtype=np.uint8)
    p = _GenomeParams(spec.seed, spec.length, spec.repeat_frac, spec.n_families, spec.fam_len_lo,
                      spec.fam_len_hi, spec.fam_len_mode, spec.div_lo, spec.div_hi, spec.indel_share)
    rc = _lib().synth_genome(ctypes.byref(p), _ptr(out))
    if rc < 0:
        raise ValueError(f"synth_genome failed ({rc})")
    return out


@dataclass
class ReadSpec:
    """Read-set recipe: lengths, error rates and an exact edit script per read."""
    n_reads: int
    seed: int = MASTER_SEED
    lens: Sequence[int] = (100,)
    len_w: Sequence[int] = (1,)
    err_pm: Sequence[int] = (50,)    # error rate e in per mille
    err_w: Sequence[int] = (1,)
    edit_mode: int = 0               # 0 fixed count, 1 floor(e*L), 2 n_sub subs + n_indel indels
    edits: int = 5
    w_sub: int = 8
    w_ins: int = 1
    w_del: int = 1
    n_sub: int = 0
    n_indel: int = 0


@dataclass
class Reads:
    bases: np.ndarray        # uint8 ASCII, all reads concatenated
    offsets: np.ndarray      # int64 [n+1]
    truth_pos: np.ndarray    # uint64 [n] reference start of each read
    span: np.ndarray         # uint32 [n] reference bases the read covers
    err_pm: np.ndarray       # uint16 [n] error rate drawn for the read (per mille)
    n_edits: np.ndarray      # uint16 [n] edits applied

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def read(self, r: int) -> bytes:
        return self.bases[self.offsets[r]:self.offsets[r + 1]].tobytes()

    def subset(self, idx: Sequence[int]) -> "Reads":
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.lengths[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        bases = np.empty(int(offs[-1]), dtype=np.uint8)
        for k, r in enumerate(idx):
            bases[offs[k]:offs[k + 1]] = self.bases[self.offsets[r]:self.offsets[r + 1]]
        return Reads(bases, offs, self.truth_pos[idx], self.span[idx], self.err_pm[idx], self.n_edits[idx])


def _read_params(spec: ReadSpec) -> _ReadParams:
    p = _ReadParams()
    p.seed, p.n_reads = spec.seed, spec.n_reads
    if not (1 <= len(spec.lens) <= 4 and len(spec.lens) == len(spec.len_w)):
        raise ValueError("1..4 read lengths with matching weights")
    if not (1 <= len(spec.err_pm) <= 8 and len(spec.err_pm) == len(spec.err_w)):
        raise ValueError("1..8 error rates with matching weights")
    p.n_len = len(spec.lens)
    for i, (l, w) in enumerate(zip(spec.lens, spec.len_w)):
        p.lens[i], p.len_w[i] = l, w
    p.n_err = len(spec.err_pm)
    for i, (e, w) in enumerate(zip(spec.err_pm, spec.err_w)):
        p.err_pm[i], p.err_w[i] = e, w
    p.edit_mode, p.edits = spec.edit_mode, spec.edits
    p.w_sub, p.w_ins, p.w_del = spec.w_sub, spec.w_ins, spec.w_del
    p.n_sub, p.n_indel = spec.n_sub, spec.n_indel
    return p


def reads(spec: ReadSpec, ref: np.ndarray) -> Reads:
    """Sample ``spec.n_reads`` reads from ``ref`` with their edit scripts applied."""
    p = _read_params(spec)
    n = spec.n_reads
    lens = np.empty(n, dtype=np.uint32)
    if _lib().synth_read_lengths(ctypes.byref(p), _ptr(lens)) != 0:
        raise ValueError("synth_read_lengths failed")
    offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    bases = np.empty(int(offs[-1]), dtype=np.uint8)
    truth = np.empty(n, dtype=np.uint64)
    span = np.empty(n, dtype=np.uint32)
    epm = np.empty(n, dtype=np.uint16)
    ned = np.empty(n, dtype=np.uint16)
    rc = _lib().synth_reads(ctypes.byref(p), _ptr(ref), len(ref), _ptr(offs), _ptr(bases),
                            _ptr(truth), _ptr(span), _ptr(epm), _ptr(ned))
    if rc != 0:
        raise ValueError(f"synth_reads failed ({rc})")
    return Reads(bases, offs, truth, span, epm, ned)


def reads_from_strings(seqs: Sequence[bytes]) -> Reads:
    """Pack explicit read strings (for hand-built cases)."""
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    offs = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    bases = np.frombuffer(b"".join(seqs), dtype=np.uint8).copy() if seqs else np.zeros(0, np.uint8)
    n = len(seqs)
    return Reads(bases, offs, np.zeros(n, np.uint64), lens.astype(np.uint32),
                 np.zeros(n, np.uint16), np.zeros(n, np.uint16))


def candidates(ref: np.ndarray, rd: Reads, bin_size: int, cap: int, k: int = 12):
    """Candidate bins from exact k-mer seed hits: (cand_off int64[n+1], cand_bin int32[P]).

    Seeds are the non-overlapping k-mers at read offsets 0, k, 2k, ...; a hit at
    reference position h of the seed at offset o proposes bin max(h-o, 0) // bin_size.
    Bins are deduplicated, ranked by hit count (then bin), capped and stored ascending.
    """
    n = rd.n
    off = np.zeros(n + 1, dtype=np.int64)
    buf = np.empty(max(1, n * cap), dtype=np.int32)
    tot = _lib().synth_candidates(_ptr(ref), len(ref), _ptr(rd.bases), _ptr(rd.offsets), n, k,
                                  bin_size, cap, _ptr(off), _ptr(buf))
    if tot < 0:
        raise ValueError(f"synth_candidates failed ({tot})")
    return off, buf[:tot].copy()


# ----------------------------------------------------------------------------
# SplitMix64 in Python, for the small host-side draws (request arrivals).
# ----------------------------------------------------------------------------
_M64 = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.s = seed & _M64

    def next(self) -> int:
        self.s = (self.s + 0x9E3779B97F4A7C15) & _M64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)
