"""Seeded synthetic channelised voltages.

This module only makes inputs: it draws Gaussian noise, adds tones, rounds,
clips and packs them into the two sample formats the X-engine accepts.  It
holds none of the correlation arithmetic, so both the GPU library's tests and
the CPU oracle can be fed from it.

Formats (paper Section 2.1 "F-engine": channel data are truncated to a 4-bit
real and a 4-bit imaginary part; Section 2.3: the fluff step widens them to
8-bit + 8-bit):

* 4+4-bit: one uint8 per (t, f, input), high nibble = real, low nibble =
  imaginary, each two's complement in [-8, 7].
* 8+8-bit: two int8 per (t, f, input), real then imaginary.

Layout is time-major ``[T][F][N]`` (Section 2.1, the transpose / corner-turn
stage orders the data for the X-engine; the order within a block is not given
in the paper, time-major is the order in which blocks arrive).

Every generator is seeded by a tuple; the tuple is hashed into a 63-bit torch
seed so that any (config, array, block) can be regenerated on its own.
Generation runs on whatever device is asked for; the same seed gives the same
bytes on the same device type.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import torch

BASE_SEED = 240619013  # arXiv id of the paper, used as the seed root
_PHASE_TAG = 0x7068  # seed suffix for the per-channel / per-input tone phases

# Channel plan (Section 2.2 "Network"): 250 Msps sampling gives 1024 channels
# of 125/1024 MHz.
BANDWIDTH_HZ = 125e6
C_LIGHT = 299_792_458.0


def seed_of(*parts: int) -> int:
    """Hash an integer tuple into a 63-bit seed."""
    h = hashlib.blake2b(repr(tuple(int(p) for p in parts)).encode(), digest_size=8)
    return int.from_bytes(h.digest(), "little") & ((1 << 63) - 1)


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def pack4(re: torch.Tensor, im: torch.Tensor) -> torch.Tensor:
    """Pack integer tensors in [-8, 7] into 4+4-bit bytes (high nibble = real)."""
    r = re.to(torch.int32) & 0xF
    i = im.to(torch.int32) & 0xF
    return ((r << 4) | i).to(torch.uint8)


def unpack4(b: torch.Tensor):
    """Inverse of pack4 (used by input-format tests only)."""
    x = b.to(torch.int32)
    r = x >> 4
    i = x & 0xF
    r = torch.where(r >= 8, r - 16, r)
    i = torch.where(i >= 8, i - 16, i)
    return r, i


def pack8(re: torch.Tensor, im: torch.Tensor) -> torch.Tensor:
    """Interleave int8 real/imaginary parts: [..., 2] int8."""
    return torch.stack([re.to(torch.int8), im.to(torch.int8)], dim=-1)


def quantise(x: torch.Tensor, lo: int, hi: int) -> torch.Tensor:
    """Round half to even, then clip."""
    return torch.clamp(torch.round(x), lo, hi)


@dataclass
class Tone:
    """A common complex tone A*exp(i(2*pi*delta*t + psi_f + phi_k)).

    ``psi_f`` is drawn per channel, ``phi_k`` per input; ``drift`` adds
    2*pi*k*drift*block to input k's phase (a slow per-block phase drift).
    """
    amp: float = 2.5
    delta: float = 0.01
    drift: float = 0.0


def gaussian_volts(N: int, F: int, T: int, *, sigma: float, bits: int, seed: tuple,
                   tone: Tone | None = None, block: int = 0, t0: int = 0,
                   device="cpu", chunk_t: int = 256) -> torch.Tensor:
    """Gaussian noise (per component sigma) plus an optional common tone.

    Returns ``[T][F][N]`` uint8 for bits=4 or ``[T][F][N][2]`` int8 for bits=8.
    ``t0`` offsets the tone's time axis (for consecutive blocks).
    """
    if bits not in (4, 8):
        raise ValueError("bits must be 4 or 8")
    lo, hi = (-8, 7) if bits == 4 else (-127, 127)
    g = _gen(seed_of(*seed, block), device)
    shape = (T, F, N) if bits == 4 else (T, F, N, 2)
    out = torch.empty(shape, dtype=torch.uint8 if bits == 4 else torch.int8, device=device)
    if tone is not None:
        gp = _gen(seed_of(*seed, _PHASE_TAG), device)
        psi = torch.rand(F, generator=gp, device=device, dtype=torch.float64) * 2 * math.pi
        phi = torch.rand(N, generator=gp, device=device, dtype=torch.float64) * 2 * math.pi
        k = torch.arange(N, device=device, dtype=torch.float64)
        phi = phi + 2 * math.pi * k * tone.drift * block
    for ts in range(0, T, chunk_t):
        tc = min(chunk_t, T - ts)
        re = torch.randn((tc, F, N), generator=g, device=device, dtype=torch.float32) * sigma
        im = torch.randn((tc, F, N), generator=g, device=device, dtype=torch.float32) * sigma
        if tone is not None:
            t = torch.arange(t0 + ts, t0 + ts + tc, device=device, dtype=torch.float64)
            ph = (2 * math.pi * tone.delta * t)[:, None, None] + psi[None, :, None] + phi[None, None, :]
            re += (tone.amp * torch.cos(ph)).to(torch.float32)
            im += (tone.amp * torch.sin(ph)).to(torch.float32)
        re = quantise(re, lo, hi)
        im = quantise(im, lo, hi)
        if bits == 4:
            out[ts:ts + tc] = pack4(re, im)
        else:
            out[ts:ts + tc] = pack8(re, im)
    return out


def uniform_volts4(N: int, F: int, T: int, *, seed: tuple, device="cpu") -> torch.Tensor:
    """Real and imaginary parts iid uniform on {-8..7}, packed 4+4-bit."""
    g = _gen(seed_of(*seed), device)
    re = torch.randint(-8, 8, (T, F, N), generator=g, device=device, dtype=torch.int32)
    im = torch.randint(-8, 8, (T, F, N), generator=g, device=device, dtype=torch.int32)
    return pack4(re, im)


def uniform_volts8(N: int, F: int, T: int, *, seed: tuple, lo: int = -127, hi: int = 127,
                   device="cpu") -> torch.Tensor:
    """Real and imaginary parts iid uniform on {lo..hi}, interleaved int8."""
    g = _gen(seed_of(*seed), device)
    re = torch.randint(lo, hi + 1, (T, F, N), generator=g, device=device, dtype=torch.int32)
    im = torch.randint(lo, hi + 1, (T, F, N), generator=g, device=device, dtype=torch.int32)
    return pack8(re, im)


def delayed_copies(N: int, F: int, T: int, *, taus_s, sigma_common: float, sigma_noise: float,
                   seed: tuple, bits: int = 4, f0_hz: float = 0.0,
                   chan_width_hz: float = BANDWIDTH_HZ / 1024, device="cpu") -> torch.Tensor:
    """A common noise signal seen by every input through its own delay.

    Per channel f the common signal s_f[t] is complex Gaussian noise; input k
    receives s_f[t] * exp(i*2*pi*nu_f*tau_k) plus its own receiver noise, with
    nu_f = f0 + f * chan_width the channel's centre frequency (Section 3.2
    "Phase testing": two copies of one noise signal through cables of
    different length).
    """
    lo, hi = (-8, 7) if bits == 4 else (-127, 127)
    g = _gen(seed_of(*seed), device)
    taus = torch.as_tensor(taus_s, dtype=torch.float64, device=device)
    nu = f0_hz + torch.arange(F, dtype=torch.float64, device=device) * chan_width_hz
    ph = 2 * math.pi * nu[:, None] * taus[None, :]              # [F][N]
    rot_re = torch.cos(ph).to(torch.float32)
    rot_im = torch.sin(ph).to(torch.float32)
    sr = torch.randn((T, F, 1), generator=g, device=device) * sigma_common
    si = torch.randn((T, F, 1), generator=g, device=device) * sigma_common
    re = sr * rot_re - si * rot_im + torch.randn((T, F, N), generator=g, device=device) * sigma_noise
    im = sr * rot_im + si * rot_re + torch.randn((T, F, N), generator=g, device=device) * sigma_noise
    re = quantise(re, lo, hi)
    im = quantise(im, lo, hi)
    return pack4(re, im) if bits == 4 else pack8(re, im)


# --- the benchmark workloads --------------------------------------------------

def tiny(device="cpu") -> torch.Tensor:
    """16 inputs (8 dual-pol feeds), 8 channels, 256 samples, uniform 4+4-bit."""
    return uniform_volts4(16, 8, 256, seed=(BASE_SEED, 1), device=device)


def tianlai(device="cpu", N: int = 192, F: int = 1024, T: int = 4096) -> torch.Tensor:
    """192 inputs, 1024 channels, 4096 samples: 4+4-bit noise (sigma 2.5) plus a
    common tone with a seeded phase per input and per channel."""
    return gaussian_volts(N, F, T, sigma=2.5, bits=4, seed=(BASE_SEED, 2),
                          tone=Tone(amp=2.5, delta=0.01), device=device)


def precision8(device="cpu", N: int = 192, F: int = 512, T: int = 8192) -> torch.Tensor:
    """192 inputs, 512 channels, 8192 samples of 8+8-bit noise, sigma 20, clip +-127."""
    return gaussian_volts(N, F, T, sigma=20.0, bits=8, seed=(BASE_SEED, 3), device=device)


BATCH_ARRAYS = ((64, 256), (192, 1024), (256, 512), (512, 128))  # (inputs, channels)


def batched(device="cpu", T: int = 2048, arrays=BATCH_ARRAYS):
    """Four arrays of uneven input and channel counts, 4+4-bit noise sigma 2.5."""
    return [gaussian_volts(N, F, T, sigma=2.5, bits=4, seed=(BASE_SEED, 4, a), device=device)
            for a, (N, F) in enumerate(arrays)]


def stream_block(N: int, F: int, block: int, *, array_id: int, T: int = 1024,
                 device="cpu") -> torch.Tensor:
    """One 1024-sample block of a streaming array: noise plus a drifting tone."""
    return gaussian_volts(N, F, T, sigma=2.5, bits=4, seed=(BASE_SEED, 5, array_id),
                          tone=Tone(amp=2.5, delta=0.01, drift=1e-5), block=block,
                          t0=block * T, device=device)


# ---- raw ADC samples for the F-engine front end -------------------------------
# Paper Section 2.2 "F-engine": 8-bit samples at 250 Msps (Fix_8_7 words, here
# their integer codes -128 .. 127), one real time series per input.

@dataclass(frozen=True)
class AdcTone:
    freq: float        # cycles per ADC sample
    amp: float         # amplitude in ADC codes


def adc_samples(N: int, S: int, *, sigma: float, seed: tuple, tones=(), device="cpu",
                chunk: int = 1 << 20) -> torch.Tensor:
    """ADC codes ``[N][S]`` int8: Gaussian noise (sigma in codes) plus real
    tones ``amp * cos(2 pi freq s + phase)`` with a seeded phase per (tone,
    input); rounded half to even, clipped to [-128, 127]."""
    g = _gen(seed_of(*seed), device)
    phases = []
    if tones:
        gp = _gen(seed_of(*seed, _PHASE_TAG), device)
        phases = [torch.rand(N, generator=gp, device=device, dtype=torch.float64) * 2 * math.pi for _ in tones]
    out = torch.empty((N, S), dtype=torch.int8, device=device)
    for s0 in range(0, S, chunk):
        sc = min(chunk, S - s0)
        x = torch.randn((N, sc), generator=g, device=device, dtype=torch.float32) * sigma
        if tones:
            s = torch.arange(s0, s0 + sc, device=device, dtype=torch.float64)
            for tone, ph in zip(tones, phases):
                # the phase 2 pi f s reduced modulo 2 pi in float64 before the cosine
                arg = torch.remainder(tone.freq * s, 1.0) * (2 * math.pi)
                x += (tone.amp * torch.cos(arg[None, :] + ph[:, None])).to(torch.float32)
        out[:, s0:s0 + sc] = quantise(x, -128, 127).to(torch.int8)
    return out


def eq_gains(N: int, F: int, *, base: float, seed: tuple, spread: float = 1.25, device="cpu") -> torch.Tensor:
    """EQ gains ``[N][F]`` float32: base times a log-uniform factor in
    [1 / spread, spread] per (input, channel)."""
    g = _gen(seed_of(*seed), device)
    u = torch.rand((N, F), generator=g, device=device, dtype=torch.float64) * 2 - 1
    return (base * torch.exp(u * math.log(spread))).to(torch.float32)


# Per-input ADC noise of the F-engine workloads and the EQ gain that brings a
# channel's components to about 2.5 codes of the 4-bit output (per component
# sigma of a channel = sigma_adc * sqrt(sum h^2 / 2) for the 4 x 2048
# Hamming-sinc prototype, sum h^2 = 1649.6).
FE_ADC_SIGMA = 16.0
FE_EQ_BASE = 0.00544


def fengine_adc(device="cpu", N: int = 192, T: int = 4096, P: int = 2048, taps: int = 4) -> torch.Tensor:
    """ADC codes for T spectra of N inputs: noise (sigma 16 codes) plus two
    tones, one on a channel centre and one between channels."""
    S = (T + taps - 1) * P
    return adc_samples(N, S, sigma=FE_ADC_SIGMA, seed=(BASE_SEED, 6),
                       tones=(AdcTone(freq=300.0 / P, amp=12.0), AdcTone(freq=700.5 / P, amp=8.0)),
                       device=device)


def fengine_gains(device="cpu", N: int = 192, F: int = 1024) -> torch.Tensor:
    return eq_gains(N, F, base=FE_EQ_BASE, seed=(BASE_SEED, 6, 1), device=device)
