"""The F-engine oracle against its pins (no GPU needed), and planted mistakes
in copies of it, each of which some pin must catch."""
import os
import types

import pytest

import _fengine_pins
from oracle import fengine as fe

SRC = fe.__file__


@pytest.mark.parametrize("pin", _fengine_pins.ALL_FENGINE_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(fe)


# (name, exact text in the oracle, replacement)
MUTANTS = [
    ("taps_reversed", "y[m] += h[k * P:(k + 1) * P] * x[(m + k) * P:(m + k + 1) * P]",
     "y[m] += h[(taps - 1 - k) * P:(taps - k) * P] * x[(m + k) * P:(m + k + 1) * P]"),
    ("sinc_off_centre", "np.sinc(n / P - taps / 2.0)", "np.sinc(n / P - taps / 2.0 + 0.5)"),
    ("hann_not_hamming", "window = 0.54 - 0.46 * np.cos", "window = 0.5 - 0.5 * np.cos"),
    ("nyquist_kept_dc_dropped", "np.fft.rfft(pfb_fir(x, h, P, taps), axis=1)[:, :P // 2]",
     "np.fft.rfft(pfb_fir(x, h, P, taps), axis=1)[:, 1:P // 2 + 1]"),
    ("conjugated_spectrum", "np.fft.rfft(pfb_fir(x, h, P, taps), axis=1)[:, :P // 2]",
     "np.conj(np.fft.rfft(pfb_fir(x, h, P, taps), axis=1)[:, :P // 2])"),
    ("floor_not_round", "re = np.clip(np.rint(v.real), -8, 7)", "re = np.clip(np.floor(v.real + 0.5), -8, 7)"),
    ("clip_to_plus_minus_7", "im = np.clip(np.rint(v.imag), -8, 7)", "im = np.clip(np.rint(v.imag), -7, 7)"),
    ("nibbles_swapped", "return (((re & 15) << 4) | (im & 15))", "return (((im & 15) << 4) | (re & 15))"),
    ("corner_turn_swapped", "codes.transpose(1, 2, 0)", "codes.transpose(2, 1, 0)"),
    ("one_spectrum_short", "return max(0, n_samples // P - taps + 1)", "return max(0, n_samples // P - taps)"),
]


def _mutant(name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mod = types.ModuleType("fengine_" + name)
    exec(compile(src.replace(old, new, 1), f"<{name}>", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new):
    mod = _mutant(name, old, new)
    caught = []
    for pin in _fengine_pins.ALL_FENGINE_PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError, IndexError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake '{name}'"
