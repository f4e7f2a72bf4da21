"""Plain CPU F-engine (channeliser), the reference for the GPU front end.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
module; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may load it.  It shares no code with the GPU library.

What it computes (paper, Section 2.2 "F-engine"): 8-bit ADC samples of each
input go through a polyphase filter bank of size 2^11 with a four-tap
Hamming-windowed prototype and a real FFT of 2^11 points, giving 1024
channels per spectrum; each (input, channel) value is scaled by its EQ gain
and requantised to a 4-bit real and a 4-bit imaginary part; a corner turn
then orders the codes by time, channel and input for the X-engine.

Readings where the paper is silent (each stated again where it is used):
  * prototype: h[n] = w[n] sinc(n / P - taps / 2), n = 0 .. taps P - 1, with
    w the symmetric Hamming window 0.54 - 0.46 cos(2 pi n / (taps P - 1))
    (the window-times-sinc design of the CASPER pfb_fir block the paper
    names, one sinc lobe per channel width);
  * filter: spectrum m is the FFT of y_m[n] = sum_k h[k P + n] x[(m + k) P + n],
    the weighted overlap-add form of a critically sampled PFB, so spectrum m
    covers samples [m P, (m + taps) P);
  * channels: the first P / 2 bins of the real FFT (the Nyquist bin dropped);
  * ADC samples are the integer codes of the Fix_8_7 words (the 1/128 scale
    is left in the EQ gain), and the gain is one real factor per (input,
    channel);
  * requantisation: round half to even, then clip to [-8, 7]; the packed byte
    holds the real part in the high nibble and the imaginary part in the low
    nibble, two's complement (the X-engine's format);
  * corner turn: codes[m][c][i] for spectrum m, channel c, input i.
Arithmetic in float64 throughout; numpy's rfft is the DFT step.
"""
from __future__ import annotations

import numpy as np


def prototype(P: int = 2048, taps: int = 4) -> np.ndarray:
    """Hamming-windowed sinc of taps * P coefficients (float64)."""
    L = taps * P
    n = np.arange(L, dtype=np.float64)
    window = 0.54 - 0.46 * np.cos(2.0 * np.pi * n / (L - 1))
    return window * np.sinc(n / P - taps / 2.0)


def n_spectra(n_samples: int, P: int = 2048, taps: int = 4) -> int:
    """Complete spectra in n_samples ADC samples."""
    return max(0, n_samples // P - taps + 1)


def pfb_fir(x: np.ndarray, h: np.ndarray, P: int, taps: int) -> np.ndarray:
    """Filter one input's samples: y[m][n] = sum_k h[k P + n] x[(m + k) P + n]."""
    x = np.asarray(x, dtype=np.float64)
    M = n_spectra(x.size, P, taps)
    y = np.zeros((M, P))
    for m in range(M):
        for k in range(taps):
            y[m] += h[k * P:(k + 1) * P] * x[(m + k) * P:(m + k + 1) * P]
    return y


def channelise(x: np.ndarray, h: np.ndarray, P: int, taps: int) -> np.ndarray:
    """Complex spectra [M][P / 2] of one input: the real FFT of each filtered
    block, first P / 2 bins."""
    return np.fft.rfft(pfb_fir(x, h, P, taps), axis=1)[:, :P // 2]


def requantise(v: np.ndarray):
    """Round half to even and clip to [-8, 7], real and imaginary parts."""
    re = np.clip(np.rint(v.real), -8, 7).astype(np.int64)
    im = np.clip(np.rint(v.imag), -8, 7).astype(np.int64)
    return re, im


def pack4(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Real part in the high nibble, imaginary part in the low nibble."""
    return (((re & 15) << 4) | (im & 15)).astype(np.uint8)


def spectra(adc: np.ndarray, P: int = 2048, taps: int = 4, h: np.ndarray | None = None) -> np.ndarray:
    """Spectra of every input: adc [N][S] integer codes -> complex [N][M][P / 2]."""
    h = prototype(P, taps) if h is None else h
    return np.stack([channelise(adc[i], h, P, taps) for i in range(adc.shape[0])])


def fengine(adc: np.ndarray, gains: np.ndarray, P: int = 2048, taps: int = 4,
            h: np.ndarray | None = None) -> np.ndarray:
    """Packed 4+4-bit codes [M][P / 2][N] (time, channel, input) from ADC
    codes adc [N][S] and EQ gains [N][P / 2]."""
    X = spectra(adc, P, taps, h)                          # [N][M][F]
    re, im = requantise(X * np.asarray(gains, dtype=np.float64)[:, None, :])
    codes = pack4(re, im)                                 # [N][M][F]
    return np.ascontiguousarray(codes.transpose(1, 2, 0))
