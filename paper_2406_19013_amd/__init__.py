"""MI355X-native X-engine: per-channel cross-multiply-accumulate of packed
4+4-bit (or 8+8-bit) complex voltages on gfx950.

The compute path is the C-ABI library ``libxcorr.so`` (HIP kernels); the
Python side is argument marshalling only (``paper_2406_19013_amd.xcorr``).
Importing this package loads nothing: the library is opened on first use and
a missing library is an error, never a fallback.
"""
__all__ = ["synth", "xcorr"]
