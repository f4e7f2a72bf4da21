"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that
the pins catch every one of them.  The real oracle is left untouched."""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle
import _pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "xcorr_oracle.c")

# (name, exact text in the oracle, replacement)
MUTANTS = [
    ("conjugate_on_wrong_side", "acc_im += ii * rj - ri * ij;", "acc_im += ri * ij - ii * rj;"),
    ("dropped_imag_imag_term", "acc_re += ri * rj + ii * ij;", "acc_re += ri * rj;"),
    ("plus_instead_of_minus", "acc_im += ii * rj - ri * ij;", "acc_im += ii * rj + ri * ij;"),
    ("nibbles_swapped", "re[i * T + t] = sext4(b >> 4);\n                im[i * T + t] = sext4(b);",
     "re[i * T + t] = sext4(b);\n                im[i * T + t] = sext4(b >> 4);"),
    ("no_sign_extension", "return (v & 8u) ? (int)v - 16 : (int)v;", "return (int)v;"),
    ("wrong_pair_index", "int64_t p = i * (i + 1) / 2 + j;\n                out[(s * P + p) * 2 + 0] = acc_re;",
     "int64_t p = i * (i + 1) / 2 + (i - j);\n                out[(s * P + p) * 2 + 0] = acc_re;"),
    ("transposed_operand", "int64_t rj = re[j * T + t], ij = im[j * T + t];",
     "int64_t rj = re[i * T + t], ij = im[j * T + t];"),
    ("dropped_last_sample", "for (int64_t t = 0; t < T; ++t) {\n                    int64_t ri",
     "for (int64_t t = 0; t + 1 < T; ++t) {\n                    int64_t ri"),
    ("channel_stride_swapped", "uint8_t b = v[(t * F + f) * N + i];", "uint8_t b = v[(f * T + t) * N + i];"),
    ("int32_accumulator", "int64_t acc_re = 0, acc_im = 0;\n                for (int64_t t = 0; t < T; ++t) {\n                    int64_t ri",
     "int32_t acc_re = 0, acc_im = 0;\n                for (int64_t t = 0; t < T; ++t) {\n                    int64_t ri"),
    ("float_accumulator_in_double_loop", "double acc_re = 0.0, acc_im = 0.0;", "float acc_re = 0.0f, acc_im = 0.0f;"),
]


def _build_mutant(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    src = src.replace(old, new, 1)
    c = os.path.join(tmp, name + ".c")
    so = os.path.join(tmp, name + ".so")
    with open(c, "w") as fh:
        fh.write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-w", "-o", so, c])
    return oracle.load_library(so)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new):
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(tmp, name, old, new)
        caught = []
        for pin in _pins.ALL_PINS:
            try:
                pin(lib)
            except (AssertionError, OverflowError, RuntimeError, IndexError, ValueError):
                caught.append(pin.__name__)
        assert caught, f"no pin caught the planted mistake '{name}'"
