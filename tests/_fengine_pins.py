"""Pins of the F-engine oracle (paper Section 2.2, "F-engine"): facts fixed
independently of its code (closed forms of the prototype and of a
channel-centred tone, a brute-force DFT on a small filter bank, shift and
linearity invariants, round-half-even ties, the nibble packing the X-engine
reads).  Each pin takes the oracle module, so that planted mistakes in a copy
of it can be checked against the same pins."""
import math

import numpy as np
import pytest

def pin_prototype_closed_form(fe):
    """Hamming window times sinc(n / P - taps / 2): zero at every multiple of P
    except the centre L / 2, where it equals the window value; the end
    coefficient is the Hamming end value 0.08 times sinc(-2) = 0."""
    P, taps = 2048, 4
    h = fe.prototype(P, taps)
    L = P * taps
    assert h.shape == (L,)
    for j in range(taps):
        if j != taps // 2:
            assert abs(h[j * P]) < 1e-12
    assert h[L // 2] == pytest.approx(0.54 - 0.46 * math.cos(2 * math.pi * (L // 2) / (L - 1)), abs=1e-15)
    # one point off the sinc zeros: the product of the two closed forms
    n = 1000
    want = (0.54 - 0.46 * math.cos(2 * math.pi * n / (L - 1))) * math.sin(math.pi * (n / P - 2)) / (math.pi * (n / P - 2))
    assert h[n] == pytest.approx(want, rel=1e-12)


def _direct_pfb(x, h, P, taps):
    """Spectra by explicit loops: weighted overlap-add and a plain DFT sum."""
    M = len(x) // P - taps + 1
    out = np.zeros((M, P // 2), complex)
    for m in range(M):
        y = [sum(h[k * P + n] * x[(m + k) * P + n] for k in range(taps)) for n in range(P)]
        for c in range(P // 2):
            out[m, c] = sum(y[n] * complex(math.cos(2 * math.pi * c * n / P), -math.sin(2 * math.pi * c * n / P))
                            for n in range(P))
    return out


def pin_brute_force_small_bank(fe):
    """P = 16, 4 taps, 3 spectra: every channel equals the direct sums (a
    transposed tap order, a wrong sign or a dropped bin fails)."""
    rng = np.random.default_rng(5)
    P, taps = 16, 4
    x = rng.integers(-128, 128, size=(taps + 2) * P)
    h = fe.prototype(P, taps)
    got = fe.channelise(x, h, P, taps)
    want = _direct_pfb(x, h, P, taps)
    assert got.shape == (3, P // 2)
    assert np.allclose(got, want, rtol=0, atol=1e-9)
    # an asymmetric prototype separates the tap order from its reverse
    h2 = rng.normal(size=taps * P)
    assert np.allclose(fe.channelise(x, h2, P, taps), _direct_pfb(x, h2, P, taps), rtol=0, atol=1e-9)


def pin_channel_centred_tone_closed_form(fe):
    """x[s] = A cos(2 pi c0 s / P + phi): every spectrum is the same and
    X[c0] = (A / 2) (e^{i phi} sum_n H_n + e^{-i phi} sum_n H_n e^{-4 pi i c0 n / P}),
    H_n = sum_k h[k P + n] (the filter taps folded onto one block), computed
    here by explicit sums."""
    P, taps, A, phi, c0 = 64, 4, 37.0, 0.7, 5
    h = fe.prototype(P, taps)
    s = np.arange((taps + 3) * P)
    x = A * np.cos(2 * np.pi * c0 * s / P + phi)
    X = fe.channelise(x, h, P, taps)
    H = [sum(h[k * P + n] for k in range(taps)) for n in range(P)]
    S0 = sum(H)
    S2 = sum(H[n] * complex(math.cos(4 * math.pi * c0 * n / P), -math.sin(4 * math.pi * c0 * n / P)) for n in range(P))
    want = A / 2 * (complex(math.cos(phi), math.sin(phi)) * S0 + complex(math.cos(phi), -math.sin(phi)) * S2)
    for m in range(X.shape[0]):
        assert abs(X[m, c0] - want) < 1e-9 * abs(want)
    # leakage of a 4-tap Hamming bank: about -50 dB into the adjacent
    # channels, below -65 dB two or more channels away
    mag = np.abs(X[0]) / abs(want)
    assert max(mag[c0 - 1], mag[c0 + 1]) < 4e-3
    assert np.delete(mag, [c0 - 1, c0, c0 + 1]).max() < 5e-4


def pin_full_size_dc_and_centre_bin(fe):
    """P = 2048: a constant input lands in channel 0 as A sum(h) (the sum of
    the folded taps), with the bank's leakage into the other channels."""
    P, taps = 2048, 4
    h = fe.prototype(P, taps)
    x = np.full((taps + 1) * P, 3.0)
    X = fe.channelise(x, h, P, taps)
    assert X[0, 0] == pytest.approx(3.0 * h.sum(), rel=1e-12)
    mag = np.abs(X[0]) / abs(X[0, 0])
    assert mag[1] < 4e-3 and mag[2:].max() < 5e-4


def pin_shift_by_one_block_and_linearity(fe):
    rng = np.random.default_rng(9)
    P, taps = 128, 4
    h = fe.prototype(P, taps)
    x1 = rng.normal(size=(taps + 5) * P)
    x2 = rng.normal(size=(taps + 5) * P)
    X1 = fe.channelise(x1, h, P, taps)
    assert np.allclose(fe.channelise(x1[P:], h, P, taps), X1[1:], atol=1e-9)
    assert np.allclose(fe.channelise(2.5 * x1 - 0.5 * x2, h, P, taps),
                       2.5 * X1 - 0.5 * fe.channelise(x2, h, P, taps), atol=1e-9)


def pin_requantise_ties_and_clip(fe):
    v = np.array([2.5, 3.5, -2.5, -0.5, 0.5, 7.5, -8.5, 100.0, -100.0, 6.49, -7.51]) * (1 + 1j)
    re, im = fe.requantise(v)
    assert re.tolist() == [2, 4, -2, 0, 0, 7, -8, 7, -8, 6, -8]
    assert im.tolist() == re.tolist()


def pin_pack_nibbles(fe):
    re = np.array([-8, 7, -1, 0, 3])
    im = np.array([7, -8, -1, 0, -3])
    assert fe.pack4(re, im).tolist() == [0x87, 0x78, 0xFF, 0x00, 0x3D]


def pin_corner_turn_order(fe):
    """codes[m][c][i] is input i's code of channel c in spectrum m."""
    rng = np.random.default_rng(2)
    P, taps, N = 16, 4, 3
    adc = rng.integers(-128, 128, size=(N, (taps + 1) * P))
    gains = rng.uniform(0.02, 0.05, size=(N, P // 2))
    codes = fe.fengine(adc, gains, P, taps)
    h = fe.prototype(P, taps)
    assert codes.shape == (2, P // 2, N)
    for i in range(N):
        X = fe.channelise(adc[i], h, P, taps) * gains[i]
        re, im = fe.requantise(X)
        assert np.array_equal(codes[:, :, i], fe.pack4(re, im))


def pin_n_spectra(fe):
    assert fe.n_spectra(4 * 2048) == 1
    assert fe.n_spectra(7 * 2048 + 5) == 4
    assert fe.n_spectra(100) == 0


ALL_FENGINE_PINS = [pin_prototype_closed_form, pin_brute_force_small_bank, pin_channel_centred_tone_closed_form, pin_full_size_dc_and_centre_bin, pin_shift_by_one_block_and_linearity, pin_requantise_ties_and_clip, pin_pack_nibbles, pin_corner_turn_order, pin_n_spectra]
