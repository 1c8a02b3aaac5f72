"""Helpers for the GPU tests: device copies and mask unpacking (no filter arithmetic)."""

from __future__ import annotations

import sys

import numpy as np


def log(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t) -> np.ndarray:
    return t.cpu().numpy()


def empty(shape, dtype):
    import torch
    return torch.empty(shape, dtype=dtype, device="cuda")


def unpack_mask(mask_words: np.ndarray, nb: int) -> np.ndarray:
    """uint32 [n][W] -> uint8 [n][nb], bit x%32 of word x/32."""
    n = mask_words.shape[0]
    b = np.unpackbits(mask_words.astype("<u4").view(np.uint8).reshape(n, -1), axis=1, bitorder="little")
    return b[:, :nb]


def tm_to_bits(tm_bytes: np.ndarray, R4: int, row_words: int, nb: int) -> np.ndarray:
    """Token-major layout bytes -> uint8 [nb][R4] (bin-major byte-per-bit view)."""
    rows = tm_bytes.view("<u4").reshape(R4, row_words)
    bits = np.unpackbits(rows.view(np.uint8).reshape(R4, -1), axis=1, bitorder="little")[:, :nb]
    return np.ascontiguousarray(bits.T)


def bm_to_bits(bm_bytes: np.ndarray, R4: int, vec_words: int, nb: int) -> np.ndarray:
    vec = bm_bytes.view("<u4").reshape(nb, vec_words)
    return np.unpackbits(vec.view(np.uint8).reshape(nb, -1), axis=1, bitorder="little")[:, :R4]
