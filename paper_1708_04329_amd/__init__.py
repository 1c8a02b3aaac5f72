"""GRIM-Filter hot path on AMD Instinct MI355X (gfx950).

The compute lives in ``libgrim.so`` (HIP kernels behind the C ABI of
``include/grim.h``); ``paper_1708_04329_amd.grim`` is its Python binding.
Importing the package loads nothing; the binding loads the library on first use.
"""

__all__ = ["grim"]
