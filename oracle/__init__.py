"""Plain CPU oracle for the X-engine cross-multiply-accumulate.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
module; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may load it.  It shares no code with the GPU library.

The arithmetic lives in ``xcorr_oracle.c`` (a plain triple loop over channel,
input pair and time, with int64 or double accumulators).  This wrapper only
marshals numpy arrays through ctypes, plus the int32 range check that the
integer result must pass (the GPU path accumulates in int32 and must refuse,
not wrap, past that bound).

Definition followed (paper, Section 2.3 "X-engine" and Eq. 2 of Section 3.2):
for each channel f and each pair j <= i,
    V_ij[f] = sum_t x_i[f,t] * conj(x_j[f,t]),
stored at pair index p = i(i+1)/2 + j as (re, im).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xcorr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

INT32_MIN = -(2 ** 31)
INT32_MAX = 2 ** 31 - 1

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no SIMD intrinsics, no BLAS)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC",
                               "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path: str | None = None):
    """Load (building first if needed) and declare the oracle's entry points."""
    global _lib
    with _lock:
        if path is None and _lib is not None:
            return _lib
        lib = ctypes.CDLL(path or build())
        i64 = ctypes.c_int64
        p = ctypes.c_void_p
        for name in ("oracle_xcorr_i64", "oracle_xcorr_f64"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [p, ctypes.c_int, i64, i64, i64, p, i64, p]
        lib.oracle_xcorr_pair_i64.restype = ctypes.c_int
        lib.oracle_xcorr_pair_i64.argtypes = [p, ctypes.c_int, i64, i64, i64, i64, i64, i64, p]
        if path is None:
            _lib = lib
        return lib


def n_pairs(n_inputs: int) -> int:
    """Number of baselines including autos: N(N+1)/2."""
    return n_inputs * (n_inputs + 1) // 2


def _check_volts(volts: np.ndarray, bits: int, T: int, F: int, N: int) -> np.ndarray:
    v = np.ascontiguousarray(volts)
    if v.dtype not in (np.uint8, np.int8):
        raise TypeError("voltages must be uint8 (4+4-bit) or int8 pairs (8+8-bit)")
    need = T * F * N * (1 if bits == 4 else 2)
    if v.size != need:
        raise ValueError(f"voltage buffer has {v.size} bytes, expected {need}")
    return v


def xcorr(volts, bits: int, T: int, F: int, N: int, chans=None, lib=None) -> np.ndarray:
    """Exact visibilities, int64 array of shape [n_chans_selected][P][2]."""
    lib = lib or load_library()
    v = _check_volts(volts, bits, T, F, N)
    sel = np.arange(F, dtype=np.int64) if chans is None else np.ascontiguousarray(chans, dtype=np.int64)
    out = np.zeros((sel.size, n_pairs(N), 2), dtype=np.int64)
    rc = lib.oracle_xcorr_i64(v.ctypes.data, bits, T, F, N, sel.ctypes.data, sel.size, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_xcorr_i64 failed with {rc}")
    return out


def xcorr_f64(volts, bits: int, T: int, F: int, N: int, chans=None, lib=None) -> np.ndarray:
    """Visibilities accumulated in double, shape [n_chans_selected][P][2]."""
    lib = lib or load_library()
    v = _check_volts(volts, bits, T, F, N)
    sel = np.arange(F, dtype=np.int64) if chans is None else np.ascontiguousarray(chans, dtype=np.int64)
    out = np.zeros((sel.size, n_pairs(N), 2), dtype=np.float64)
    rc = lib.oracle_xcorr_f64(v.ctypes.data, bits, T, F, N, sel.ctypes.data, sel.size, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_xcorr_f64 failed with {rc}")
    return out


def xcorr_pair(volts, bits: int, T: int, F: int, N: int, f: int, i: int, j: int, lib=None):
    """One visibility (re, im) as Python ints; requires j <= i."""
    lib = lib or load_library()
    v = _check_volts(volts, bits, T, F, N)
    out = np.zeros(2, dtype=np.int64)
    rc = lib.oracle_xcorr_pair_i64(v.ctypes.data, bits, T, F, N, f, i, j, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_xcorr_pair_i64 failed with {rc}")
    return int(out[0]), int(out[1])


def to_int32(v64: np.ndarray) -> np.ndarray:
    """Narrow an exact result to int32, refusing (never wrapping) out-of-range values."""
    if v64.size and (v64.min() < INT32_MIN or v64.max() > INT32_MAX):
        raise OverflowError("visibility outside the int32 range")
    return v64.astype(np.int32)


def pair_index(i: int, j: int) -> int:
    """Row-major lower-triangle index of baseline (i, j), j <= i."""
    return i * (i + 1) // 2 + j
