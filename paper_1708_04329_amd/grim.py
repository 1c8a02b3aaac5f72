"""Python binding of libgrim (include/grim.h): argument marshalling only.

Every step of the filter runs in the HIP library; this module turns torch
tensors (device memory) or numpy arrays (host memory) into the plain pointers
and sizes of the C ABI and raises ``GrimError`` for non-zero return codes.
There is no fallback: if ``libgrim.so`` is missing or the device is not a
gfx950 GPU, calls fail loudly.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgrim.so")

GRIM_OK = 0
GRIM_EINVAL = -1
GRIM_ENOMEM = -2
GRIM_EDEVICE = -3
GRIM_EOVERLAP = -4
GRIM_EAGAIN = -5
GRIM_ETIMEDOUT = -6
GRIM_ECANCELED = -7
GRIM_EIO = -8

LAYOUT_TM = 1
LAYOUT_BM = 2
LAYOUT_REF = 4
READS_ALLOW_SHORT_OVERLAP = 1
MODE_SCAN = 1
MODE_CANDIDATES = 2
BATCH_EDITS_NONE = 0
BATCH_EDITS_MAX = 1
BATCH_EDITS_ERR = 2

_NAMES = {0: "GRIM_OK", -1: "GRIM_EINVAL", -2: "GRIM_ENOMEM", -3: "GRIM_EDEVICE", -4: "GRIM_EOVERLAP",
          -5: "GRIM_EAGAIN", -6: "GRIM_ETIMEDOUT", -7: "GRIM_ECANCELED", -8: "GRIM_EIO"}


class GrimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class IndexInfo(ctypes.Structure):
    _fields_ = [("ref_len", ctypes.c_uint64), ("bin_size", ctypes.c_uint32), ("overlap", ctypes.c_uint32),
                ("q", ctypes.c_uint32), ("layout", ctypes.c_uint32), ("n_bins", ctypes.c_uint64),
                ("mask_words", ctypes.c_uint64), ("tm_row_words", ctypes.c_uint64),
                ("bm_vec_words", ctypes.c_uint32), ("device", ctypes.c_int32), ("tm_bytes", ctypes.c_uint64),
                ("bm_bytes", ctypes.c_uint64), ("bits_bytes", ctypes.c_uint64), ("ref_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SeedsInfo(ctypes.Structure):
    _fields_ = [("ref_len", ctypes.c_uint64), ("k", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("n_positions", ctypes.c_uint64), ("table_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _Reads(ctypes.Structure):
    _fields_ = [("bases", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("n_reads", ctypes.c_uint64),
                ("n_bases", ctypes.c_uint64), ("max_edits", ctypes.c_void_p), ("err_permille", ctypes.c_void_p),
                ("err_permille_all", ctypes.c_uint32), ("on_device", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("threads", ctypes.c_uint32), ("reads_per_chunk", ctypes.c_uint32),
                ("lane_words", ctypes.c_uint32), ("cand_waves", ctypes.c_uint32), ("cand_persistent", ctypes.c_uint32),
                ("cand_groups_per_cu", ctypes.c_uint32), ("cand_coop", ctypes.c_uint32),
                ("n_tried", ctypes.c_uint32), ("best_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchBuffers(ctypes.Structure):
    _fields_ = [("bases", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("edits", ctypes.c_void_p),
                ("cand_off", ctypes.c_void_p), ("cand_bin", ctypes.c_void_p), ("count_out", ctypes.c_void_p),
                ("pass_out", ctypes.c_void_p), ("mask_out", ctypes.c_void_p)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32), ("max_batch_reads", ctypes.c_uint32),
                ("slice_reads", ctypes.c_uint32), ("n_streams", ctypes.c_uint32),
                ("max_request_reads", ctypes.c_uint32), ("arena_bytes", ctypes.c_uint64),
                ("reserve_bytes", ctypes.c_uint64), ("host_arena_bytes", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("reserved", ctypes.c_uint32),
                ("n_reads", ctypes.c_uint64), ("mask_words", ctypes.c_uint64), ("mask", ctypes.c_void_p),
                ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("canceled", ctypes.c_uint64), ("reads_completed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("shared_launches", ctypes.c_uint64),
                ("max_requests_per_launch", ctypes.c_uint64), ("peak_device_bytes", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_uint64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("mean_ms", ctypes.c_double), ("reads_per_s", ctypes.c_double),
                ("queued", ctypes.c_uint32), ("admitted", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTime(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double), ("last_ms", ctypes.c_double)]


class Profile(ctypes.Structure):
    _fields_ = [("tokenize", KernelTime), ("scan", KernelTime), ("candidates", KernelTime), ("build", KernelTime),
                ("verify", KernelTime)]


EXPORTS = ["grim_abi_version", "grim_last_error", "grim_build_index", "grim_index_info", "grim_index_read",
           "grim_index_save", "grim_index_load", "grim_index_free", "grim_filter_scan", "grim_filter_candidates",
           "grim_profile_enable", "grim_profile_read", "grim_tune", "grim_index_get_config",
           "grim_index_set_config", "grim_batcher_create", "grim_batcher_buffers", "grim_batcher_submit",
           "grim_batcher_wait", "grim_batcher_stream", "grim_batcher_free", "grim_serve_create",
           "grim_serve_submit", "grim_serve_poll", "grim_serve_wait", "grim_serve_release", "grim_serve_cancel",
           "grim_serve_stats", "grim_serve_reset_stats", "grim_serve_destroy", "grim_verify_candidates",
           "grim_seeds_build", "grim_seeds_info", "grim_seeds_free", "grim_seed_candidates",
           "grim_reverse_complement", "grim_mask_summary", "grim_verify_candidates_bounded",
           "grim_filter_candidates_static"]

_lib = None


def lib(path: str = LIB_PATH):
    """Load libgrim.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with `python -m paper_1708_04329_amd.build`")
    L = ctypes.CDLL(path)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "grim_abi_version": ([], I),
        "grim_last_error": ([], ctypes.c_char_p),
        "grim_build_index": ([P, U64, U32, U32, U32, U32, U32, P, PP], I),
        "grim_index_info": ([P, ctypes.POINTER(IndexInfo)], I),
        "grim_index_read": ([P, U32, U64, U64, P], I),
        "grim_index_save": ([P, ctypes.c_char_p], I),
        "grim_index_load": ([ctypes.c_char_p, P, PP], I),
        "grim_index_free": ([P], None),
        "grim_filter_scan": ([P, ctypes.POINTER(_Reads), P, P, U32, P], I),
        "grim_filter_candidates": ([P, ctypes.POINTER(_Reads), P, P, U64, P, P, P], I),
        "grim_filter_candidates_static": ([P, ctypes.POINTER(_Reads), P, P, U64, P, P, P], I),
        "grim_verify_candidates": ([P, ctypes.POINTER(_Reads), P, P, U64, P, P, P, P], I),
        "grim_verify_candidates_bounded": ([P, ctypes.POINTER(_Reads), P, P, U64, P, P, P, P], I),
        "grim_seeds_build": ([P, U64, U32, U32, P, PP], I),
        "grim_seeds_info": ([P, ctypes.POINTER(SeedsInfo)], I),
        "grim_seeds_free": ([P], None),
        "grim_seed_candidates": ([P, ctypes.POINTER(_Reads), U32, U32, P, P, ctypes.POINTER(ctypes.c_uint64), P], I),
        "grim_reverse_complement": ([P, U64, P, U64, P, P], I),
        "grim_mask_summary": ([P, U64, U64, P, P, P], I),
        "grim_profile_enable": ([I], I),
        "grim_profile_read": ([ctypes.POINTER(Profile), I], I),
        "grim_tune": ([P, ctypes.POINTER(_Reads), P, P, U64, P, ctypes.POINTER(TuneResult)], I),
        "grim_index_get_config": ([P, U32, ctypes.POINTER(TuneResult)], I),
        "grim_index_set_config": ([P, ctypes.POINTER(TuneResult)], I),
        "grim_batcher_create": ([P, U32, U64, U64, U64, U32, U32, U32, PP], I),
        "grim_batcher_buffers": ([P, U32, ctypes.POINTER(BatchBuffers)], I),
        "grim_batcher_submit": ([P, U32, U64, U64, U64], I),
        "grim_batcher_wait": ([P, U32], I),
        "grim_batcher_stream": ([P, U32], P),
        "grim_batcher_free": ([P], None),
        "grim_serve_create": ([P, ctypes.POINTER(ServeConfig), PP], I),
        "grim_serve_submit": ([P, ctypes.POINTER(_Reads), ctypes.POINTER(ctypes.c_uint64)], I),
        "grim_serve_poll": ([P, U64, ctypes.POINTER(Result)], I),
        "grim_serve_wait": ([P, U64, I, ctypes.POINTER(Result)], I),
        "grim_serve_release": ([P, U64], I),
        "grim_serve_cancel": ([P, U64], I),
        "grim_serve_stats": ([P, ctypes.POINTER(ServeStats)], I),
        "grim_serve_reset_stats": ([P], I),
        "grim_serve_destroy": ([P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != GRIM_OK:
        raise GrimError(rc, lib().grim_last_error().decode(errors="replace"))


# ---------------------------------------------------------------------------
# pointer helpers: torch tensors (device) or numpy arrays (host)
# ---------------------------------------------------------------------------

def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    raise TypeError(f"expected a torch tensor or numpy array, got {type(x)}")


def _on_device(x) -> bool:
    return _is_torch(x) and x.is_cuda


def _check_dtype(x, name, np_dtype):
    if x is None:
        return
    if _is_torch(x):
        import torch
        want = {np.uint8: torch.uint8, np.int64: torch.int64, np.uint16: torch.uint16, np.int32: torch.int32,
                np.uint32: torch.uint32, np.uint64: torch.uint64}[np_dtype]
        if x.dtype != want:
            raise TypeError(f"{name} must be {want}, got {x.dtype}")
    elif x.dtype != np_dtype:
        raise TypeError(f"{name} must be {np.dtype(np_dtype)}, got {x.dtype}")


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


@dataclass
class ReadSet:
    """A read set for the ABI: all arrays on the device (torch) or all on the host (numpy).

    bases uint8 [n_bases]; offsets int64 [n+1]; optional max_edits / err_permille uint16 [n];
    err_permille_all applies when neither per-read array is given.
    """
    bases: object
    offsets: object
    max_edits: object = None
    err_permille: object = None
    err_permille_all: int = 0
    allow_short_overlap: bool = False

    def _struct(self) -> _Reads:
        arrs = [self.bases, self.offsets, self.max_edits, self.err_permille]
        dev = [_on_device(a) for a in arrs if a is not None]
        if any(dev) and not all(dev):
            raise ValueError("read arrays must be all on the device or all on the host")
        _check_dtype(self.bases, "bases", np.uint8)
        _check_dtype(self.offsets, "offsets", np.int64)
        _check_dtype(self.max_edits, "max_edits", np.uint16)
        _check_dtype(self.err_permille, "err_permille", np.uint16)
        n = len(self.offsets) - 1
        r = _Reads()
        r.bases = _ptr(self.bases)
        r.offsets = _ptr(self.offsets)
        r.n_reads = max(n, 0)
        r.n_bases = len(self.bases)
        r.max_edits = _ptr(self.max_edits)
        r.err_permille = _ptr(self.err_permille)
        r.err_permille_all = int(self.err_permille_all)
        r.on_device = 1 if (dev and all(dev)) else 0
        r.flags = READS_ALLOW_SHORT_OVERLAP if self.allow_short_overlap else 0
        return r

    @property
    def n_reads(self) -> int:
        return len(self.offsets) - 1


class Index:
    """A GRIM bit-vector index resident on one GPU (owns its device memory)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        out = IndexInfo()
        _check(lib().grim_index_info(self._h, ctypes.byref(out)))
        return out.as_dict()

    def read(self, layout: int, offset: int = 0, nbytes: Optional[int] = None) -> np.ndarray:
        inf = self.info()
        size = {LAYOUT_TM: inf["tm_bytes"], LAYOUT_BM: inf["bm_bytes"], LAYOUT_REF: inf["ref_bytes"]}.get(layout, 0)
        nbytes = size - offset if nbytes is None else nbytes
        out = np.empty(nbytes, dtype=np.uint8)
        _check(lib().grim_index_read(self._h, layout, offset, nbytes, out.ctypes.data))
        return out

    def save(self, path: str):
        _check(lib().grim_index_save(self._h, path.encode()))

    def free(self):
        if self._h is not None and self._h.value:
            lib().grim_index_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def grim_build_index(ref, bin_size: int, overlap: int, q: int, layout: int = LAYOUT_TM,
                     stream=None) -> Index:
    """Build the per-bin token existence bits of ``ref`` (uint8 ASCII, torch or numpy)."""
    _check_dtype(ref, "ref", np.uint8)
    h = ctypes.c_void_p()
    _check(lib().grim_build_index(_ptr(ref), len(ref), 1 if _on_device(ref) else 0, bin_size, overlap, q,
                                  layout, _stream_handle(stream), ctypes.byref(h)))
    return Index(h.value)


class Seeds:
    """A seed table (k-mer -> reference positions) resident on one GPU."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        out = SeedsInfo()
        _check(lib().grim_seeds_info(self._h, ctypes.byref(out)))
        return out.as_dict()

    def free(self):
        if self._h is not None and self._h.value:
            lib().grim_seeds_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def grim_seeds_build(ref, k: int = 12, stream=None) -> Seeds:
    """Seed table of ``ref`` (uint8 ASCII, torch or numpy): positions of every k-mer."""
    _check_dtype(ref, "ref", np.uint8)
    h = ctypes.c_void_p()
    _check(lib().grim_seeds_build(_ptr(ref), len(ref), 1 if _on_device(ref) else 0, k, _stream_handle(stream),
                                  ctypes.byref(h)))
    return Seeds(h.value)


def grim_seed_candidates(seeds: Seeds, reads: ReadSet, bin_size: int, cap: int, cand_off, cand_bin,
                         stream=None) -> int:
    """Seed-hit candidate bins as CSR: cand_off int64 [n+1], cand_bin int32 (room for n*cap);
    returns the number of candidates."""
    _check_dtype(cand_off, "cand_off", np.int64)
    _check_dtype(cand_bin, "cand_bin", np.int32)
    n = reads._struct().n_reads
    if len(cand_off) < n + 1 or len(cand_bin) < n * cap:
        raise ValueError("cand_off needs n + 1 entries and cand_bin n * cap")
    r = reads._struct()
    total = ctypes.c_uint64()
    _check(lib().grim_seed_candidates(seeds.handle, ctypes.byref(r), bin_size, cap, _ptr(cand_off), _ptr(cand_bin),
                                      ctypes.byref(total), _stream_handle(stream)))
    return int(total.value)


def grim_reverse_complement(bases, offsets, out, stream=None):
    """Reverse complement of every read into ``out`` (device tensors, same offsets)."""
    _check_dtype(bases, "bases", np.uint8)
    _check_dtype(offsets, "offsets", np.int64)
    _check_dtype(out, "out", np.uint8)
    _check(lib().grim_reverse_complement(_ptr(bases), len(bases), _ptr(offsets), len(offsets) - 1, _ptr(out),
                                         _stream_handle(stream)))


def grim_mask_summary(mask, pass_count=None, digest=None, stream=None):
    """Per-read pass counts (uint32) and digests (uint64) of a [n][mask_words]
    uint32 device mask, written into the given device tensors (asynchronous)."""
    if not _is_torch(mask) or not mask.is_cuda:
        raise TypeError("mask must be a device tensor")
    _check_dtype(mask, "mask", np.uint32)
    if mask.dim() != 2:
        raise ValueError("mask must be [n_reads][mask_words]")
    if not mask.is_contiguous():
        raise ValueError("mask must be contiguous")
    n, W = int(mask.shape[0]), int(mask.shape[1])
    if pass_count is not None:
        _check_dtype(pass_count, "pass_count", np.uint32)
        if pass_count.numel() < n:
            raise ValueError("pass_count has fewer entries than mask rows")
    if digest is not None:
        _check_dtype(digest, "digest", np.uint64)
        if digest.numel() < n:
            raise ValueError("digest has fewer entries than mask rows")
    _check(lib().grim_mask_summary(_ptr(mask), n, W, None if pass_count is None else _ptr(pass_count),
                                   None if digest is None else _ptr(digest), _stream_handle(stream)))


def grim_index_load(path: str, stream=None) -> Index:
    h = ctypes.c_void_p()
    _check(lib().grim_index_load(path.encode(), _stream_handle(stream), ctypes.byref(h)))
    return Index(h.value)


def grim_filter_scan(index: Index, reads: ReadSet, mask_out, counts_out=None, stream=None):
    """All-bins filter: pass mask [n][mask_words] uint32 (+ counts [n][n_bins] uint8/uint16)."""
    _check_dtype(mask_out, "mask_out", np.uint32)
    cb = 0
    if counts_out is not None:
        cb = counts_out.element_size() if _is_torch(counts_out) else counts_out.dtype.itemsize
    r = reads._struct()
    _check(lib().grim_filter_scan(index.handle, ctypes.byref(r), _ptr(mask_out), _ptr(counts_out), cb,
                                  _stream_handle(stream)))


def grim_filter_candidates(index: Index, reads: ReadSet, cand_off, cand_bin, count_out=None, pass_out=None,
                           stream=None):
    """Candidate filter: count [P] uint16 and pass [P] uint8 for each listed (read, bin)."""
    _check_dtype(cand_off, "cand_off", np.int64)
    _check_dtype(cand_bin, "cand_bin", np.int32)
    _check_dtype(count_out, "count_out", np.uint16)
    _check_dtype(pass_out, "pass_out", np.uint8)
    r = reads._struct()
    _check(lib().grim_filter_candidates(index.handle, ctypes.byref(r), _ptr(cand_off), _ptr(cand_bin),
                                        len(cand_bin), _ptr(count_out), _ptr(pass_out),
                                        _stream_handle(stream)))


STATIC_SCRATCH_BYTES = 64 << 20


def grim_filter_candidates_static(index: Index, reads: ReadSet, cand_off, cand_bin, count_out=None, pass_out=None,
                                  stream=None):
    """grim_filter_candidates with no device allocation (fixed per-GPU scratch of
    STATIC_SCRATCH_BYTES); the reads must be device tensors."""
    _check_dtype(cand_off, "cand_off", np.int64)
    _check_dtype(cand_bin, "cand_bin", np.int32)
    _check_dtype(count_out, "count_out", np.uint16)
    _check_dtype(pass_out, "pass_out", np.uint8)
    r = reads._struct()
    _check(lib().grim_filter_candidates_static(index.handle, ctypes.byref(r), _ptr(cand_off), _ptr(cand_bin),
                                               len(cand_bin), _ptr(count_out), _ptr(pass_out),
                                               _stream_handle(stream)))


def grim_verify_candidates(index: Index, reads: ReadSet, cand_off, cand_bin, verify_mask=None, dist_out=None,
                           match_out=None, stream=None):
    """Verification: dist [P] uint16 (semi-global edit distance against the bin's bases, 0xFFFF
    where verify_mask is 0) and match [P] uint8 (dist <= E_r) for each listed (read, bin)."""
    _check_dtype(cand_off, "cand_off", np.int64)
    _check_dtype(cand_bin, "cand_bin", np.int32)
    _check_dtype(verify_mask, "verify_mask", np.uint8)
    _check_dtype(dist_out, "dist_out", np.uint16)
    _check_dtype(match_out, "match_out", np.uint8)
    r = reads._struct()
    _check(lib().grim_verify_candidates(index.handle, ctypes.byref(r), _ptr(cand_off), _ptr(cand_bin),
                                        len(cand_bin), _ptr(verify_mask), _ptr(dist_out), _ptr(match_out),
                                        _stream_handle(stream)))


def grim_verify_candidates_bounded(index: Index, reads: ReadSet, cand_off, cand_bin, verify_mask=None,
                                   dist_out=None, match_out=None, stream=None):
    """As grim_verify_candidates, with distances above E_r reported as E_r + 1 (faster)."""
    _check_dtype(cand_off, "cand_off", np.int64)
    _check_dtype(cand_bin, "cand_bin", np.int32)
    _check_dtype(verify_mask, "verify_mask", np.uint8)
    _check_dtype(dist_out, "dist_out", np.uint16)
    _check_dtype(match_out, "match_out", np.uint8)
    r = reads._struct()
    _check(lib().grim_verify_candidates_bounded(index.handle, ctypes.byref(r), _ptr(cand_off), _ptr(cand_bin),
                                                len(cand_bin), _ptr(verify_mask), _ptr(dist_out),
                                                _ptr(match_out), _stream_handle(stream)))


def grim_profile_enable(on: bool = True):
    _check(lib().grim_profile_enable(1 if on else 0))


def grim_profile_read(reset: bool = False) -> dict:
    p = Profile()
    _check(lib().grim_profile_read(ctypes.byref(p), 1 if reset else 0))
    return {k: {"launches": getattr(p, k).launches, "total_ms": getattr(p, k).total_ms,
                "last_ms": getattr(p, k).last_ms} for k, _ in Profile._fields_}


def grim_abi_version() -> int:
    return lib().grim_abi_version()


# ---------------------------------------------------------------------------
# batching layer
# ---------------------------------------------------------------------------

def grim_tune(index: Index, sample: ReadSet, cand_off=None, cand_bin=None, stream=None) -> dict:
    """Time the launch shapes of one mode on ``sample`` and keep the fastest on ``index``."""
    out = TuneResult()
    r = sample._struct()
    n_cand = 0 if cand_bin is None else len(cand_bin)
    _check(lib().grim_tune(index.handle, ctypes.byref(r), _ptr(cand_off), _ptr(cand_bin), n_cand,
                           _stream_handle(stream), ctypes.byref(out)))
    return out.as_dict()


def grim_index_get_config(index: Index, mode: int) -> dict:
    out = TuneResult()
    _check(lib().grim_index_get_config(index.handle, mode, ctypes.byref(out)))
    return out.as_dict()


def grim_index_set_config(index: Index, cfg: dict):
    t = TuneResult()
    for k, v in cfg.items():
        setattr(t, k, v)
    _check(lib().grim_index_set_config(index.handle, ctypes.byref(t)))


class Batcher:
    """Double-buffered, graph-captured batch loop (see grim_batcher_* in grim.h).

    ``buffers(slot)`` returns numpy views of the slot's pinned host buffers
    (and the device address of its all-bins mask buffer)."""

    def __init__(self, index: Index, mode: int, max_reads: int, max_bases: int, max_cand: int = 0,
                 edits_kind: int = BATCH_EDITS_NONE, err_permille_all: int = 0, allow_short_overlap: bool = False):
        self.index = index  # keeps the index alive
        self.mode = mode
        self.max_reads, self.max_bases, self.max_cand = max_reads, max_bases, max_cand
        self.edits_kind = edits_kind
        h = ctypes.c_void_p()
        _check(lib().grim_batcher_create(index.handle, mode, max_reads, max_bases, max_cand, edits_kind,
                                         err_permille_all, READS_ALLOW_SHORT_OVERLAP if allow_short_overlap else 0,
                                         ctypes.byref(h)))
        self._h = h

    def buffers(self, slot: int) -> dict:
        b = BatchBuffers()
        _check(lib().grim_batcher_buffers(self._h, slot, ctypes.byref(b)))

        def view(ptr, ctype, n):
            if not ptr:
                return None
            return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctype)), shape=(n,))

        out = {"bases": view(b.bases, ctypes.c_uint8, self.max_bases),
               "offsets": view(b.offsets, ctypes.c_int64, self.max_reads + 1),
               "edits": view(b.edits, ctypes.c_uint16, self.max_reads),
               "cand_off": view(b.cand_off, ctypes.c_int64, self.max_reads + 1),
               "cand_bin": view(b.cand_bin, ctypes.c_int32, max(self.max_cand, 1)),
               "count_out": view(b.count_out, ctypes.c_uint16, max(self.max_cand, 1)),
               "pass_out": view(b.pass_out, ctypes.c_uint8, max(self.max_cand, 1)),
               "mask_out_device": b.mask_out}
        return out

    def submit(self, slot: int, n_reads: int, n_bases: int, n_cand: int = 0):
        _check(lib().grim_batcher_submit(self._h, slot, n_reads, n_bases, n_cand))

    def wait(self, slot: int):
        _check(lib().grim_batcher_wait(self._h, slot))

    def stream(self, slot: int) -> int:
        return lib().grim_batcher_stream(self._h, slot)

    def free(self):
        if self._h is not None and self._h.value:
            lib().grim_batcher_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
SERVE_CONTINUOUS = 0
SERVE_PLAIN = 1


class Server:
    """Continuous-batching server over a resident index (grim_serve_* in grim.h)."""

    def __init__(self, index: Index, policy: int = SERVE_CONTINUOUS, **cfg):
        self.index = index  # keeps the index alive
        c = ServeConfig()
        c.policy = policy
        for k, v in cfg.items():
            if k == "allow_short_overlap":
                c.flags = READS_ALLOW_SHORT_OVERLAP if v else 0
            else:
                setattr(c, k, v)
        h = ctypes.c_void_p()
        _check(lib().grim_serve_create(index.handle, ctypes.byref(c), ctypes.byref(h)))
        self._h = h

    def submit(self, reads: ReadSet) -> int:
        """Queue a request (host numpy arrays; copied before returning). Returns its ticket."""
        r = reads._struct()
        t = ctypes.c_uint64()
        _check(lib().grim_serve_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> Optional[dict]:
        """None while pending, else the result dict (with its status)."""
        out = Result()
        rc = lib().grim_serve_poll(self._h, ticket, ctypes.byref(out))
        if rc == GRIM_EAGAIN:
            return None
        if rc == GRIM_EINVAL and out.ticket == 0:
            _check(rc)
        return out.as_dict()

    def wait(self, ticket: int, timeout_ms: int = -1) -> dict:
        out = Result()
        rc = lib().grim_serve_wait(self._h, ticket, timeout_ms, ctypes.byref(out))
        if rc == GRIM_ETIMEDOUT:
            raise GrimError(rc, lib().grim_last_error().decode(errors="replace"))
        if rc == GRIM_EINVAL and out.ticket == 0:
            _check(rc)
        return out.as_dict()

    def release(self, ticket: int):
        _check(lib().grim_serve_release(self._h, ticket))

    def cancel(self, ticket: int):
        _check(lib().grim_serve_cancel(self._h, ticket))

    def stats(self) -> dict:
        out = ServeStats()
        _check(lib().grim_serve_stats(self._h, ctypes.byref(out)))
        return out.as_dict()

    def reset_stats(self):
        _check(lib().grim_serve_reset_stats(self._h))

    def destroy(self):
        if self._h is not None and self._h.value:
            lib().grim_serve_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
