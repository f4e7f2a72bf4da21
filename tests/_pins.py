"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, each independent of the oracle's own code.

Every pin takes the oracle library handle so that the same pins can be run
against deliberately broken copies of the oracle (see test_oracle_mutants.py).
Each pin raises AssertionError when violated.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

import oracle
from paper_2406_19013_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str) -> dict:
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _complex_from_packed4(v: np.ndarray) -> np.ndarray:
    """[T][F][N] packed bytes -> complex128 [T][F][N] via the format's own decoder."""
    re, im = synth.unpack4(torch.from_numpy(v))
    return re.numpy().astype(np.float64) + 1j * im.numpy().astype(np.float64)


def _complex_from_int8(v: np.ndarray) -> np.ndarray:
    return v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)


def _numpy_visibilities(X: np.ndarray) -> np.ndarray:
    """ZHERK-style library reference: per channel V = X X^H, lower triangle."""
    T, F, N = X.shape
    ii, jj = np.tril_indices(N)
    out = np.zeros((F, N * (N + 1) // 2, 2), dtype=np.int64)
    for f in range(F):
        Xf = X[:, f, :].T                      # [N][T]
        V = Xf @ Xf.conj().T                   # exact: integers far below 2^53
        out[f, :, 0] = np.rint(V[ii, jj].real).astype(np.int64)
        out[f, :, 1] = np.rint(V[ii, jj].imag).astype(np.int64)
    return out


def pin_library_zherk(lib, cases=((1, 1, 1), (2, 3, 5), (5, 2, 33), (16, 8, 256), (32, 3, 100))):
    """P1: the result is the lower triangle of X X^H (a library matmul)."""
    for k, (N, F, T) in enumerate(cases):
        v = synth.uniform_volts4(N, F, T, seed=(11, k)).numpy()
        ref = _numpy_visibilities(_complex_from_packed4(v))
        got = oracle.xcorr(v, 4, T, F, N, lib=lib)
        assert np.array_equal(ref, got), f"4-bit case {(N, F, T)} differs from X X^H"
        v8 = synth.uniform_volts8(N, F, T, seed=(12, k)).numpy()
        ref8 = _numpy_visibilities(_complex_from_int8(v8))
        got8 = oracle.xcorr(v8, 8, T, F, N, lib=lib)
        assert np.array_equal(ref8, got8), f"8-bit case {(N, F, T)} differs from X X^H"


def pin_reversal_hermitian(lib, N=12, F=3, T=77):
    """P2: reversing the input order k -> N-1-k maps V_ij to conj(V) at the
    mirrored pair: V'_{N-1-j, N-1-i} = conj(V_ij)."""
    v = synth.uniform_volts4(N, F, T, seed=(21,)).numpy()
    vr = np.ascontiguousarray(v[:, :, ::-1])
    a = oracle.xcorr(v, 4, T, F, N, lib=lib)
    b = oracle.xcorr(vr, 4, T, F, N, lib=lib)
    for i in range(N):
        for j in range(i + 1):
            p = oracle.pair_index(i, j)
            q = oracle.pair_index(N - 1 - j, N - 1 - i)
            assert np.array_equal(b[:, q, 0], a[:, p, 0]) and np.array_equal(b[:, q, 1], -a[:, p, 1]), \
                f"pair ({i},{j}) not Hermitian under reversal"


def pin_autos_and_cauchy_schwarz(lib, N=16, F=4, T=200):
    """P3: autos are real and equal sum(re^2+im^2) >= 0; |V_ij|^2 <= V_ii V_jj."""
    v = synth.uniform_volts4(N, F, T, seed=(31,)).numpy()
    X = _complex_from_packed4(v)
    out = oracle.xcorr(v, 4, T, F, N, lib=lib)
    for i in range(N):
        p = oracle.pair_index(i, i)
        assert np.all(out[:, p, 1] == 0), "auto-correlation has an imaginary part"
        power = np.rint((np.abs(X[:, :, i]) ** 2).sum(axis=0)).astype(np.int64)
        assert np.array_equal(out[:, p, 0], power), "auto-correlation is not the total power"
        assert np.all(out[:, p, 0] >= 0)
    for i in range(N):
        for j in range(i):
            p = oracle.pair_index(i, j)
            m2 = out[:, p, 0].astype(object) ** 2 + out[:, p, 1].astype(object) ** 2
            pii = out[:, oracle.pair_index(i, i), 0].astype(object)
            pjj = out[:, oracle.pair_index(j, j), 0].astype(object)
            assert all(m <= a * b for m, a, b in zip(m2, pii, pjj)), "Cauchy-Schwarz violated"


def pin_exact_phase_ramp(lib, N=8, F=2, T=300):
    """P4: x_k = i^{m_k} s  =>  V_ij = i^{(m_i - m_j) mod 4} * sum |s|^2, exactly.
    Multiplying by i maps (a, b) -> (-b, a), exact on integers in [-7, 7]."""
    g = torch.Generator().manual_seed(41)
    sr = torch.randint(-7, 8, (T, F), generator=g)
    si = torch.randint(-7, 8, (T, F), generator=g)
    m = np.array([0, 1, 2, 3, 1, 0, 3, 2])[:N]
    re = torch.empty((T, F, N), dtype=torch.int64)
    im = torch.empty((T, F, N), dtype=torch.int64)
    for k in range(N):
        a, b = sr.clone(), si.clone()
        for _ in range(m[k]):
            a, b = -b, a
        re[:, :, k], im[:, :, k] = a, b
    v = synth.pack4(re, im).numpy()
    out = oracle.xcorr(v, 4, T, F, N, lib=lib)
    power = (sr.long() ** 2 + si.long() ** 2).sum(dim=0).numpy()   # per channel
    unit = {0: (1, 0), 1: (0, 1), 2: (-1, 0), 3: (0, -1)}
    for i in range(N):
        for j in range(i + 1):
            cr, ci = unit[(m[i] - m[j]) % 4]
            p = oracle.pair_index(i, j)
            assert np.array_equal(out[:, p, 0], cr * power) and np.array_equal(out[:, p, 1], ci * power), \
                f"pair ({i},{j}) phase is not (m_i - m_j) * pi/2"


def pin_delay_slope(lib):
    """P5 (the paper's phase test, Section 3.2 / Eq. 2): two inputs see one noise
    signal, the second delayed by 15 m of cable at 0.78 c.  The phase of V_10
    must be linear in frequency with slope 2*pi*tau, giving back 0.78 c."""
    gd = golden("phase_delay.json")
    F, T = gd["n_channels"], 64
    dnu = gd["channel_width_hz"]
    tau = gd["cable_difference_m"] / (gd["velocity_factor"] * synth.C_LIGHT)
    v = synth.delayed_copies(2, F, T, taus_s=[0.0, tau], sigma_common=2.5, sigma_noise=0.7,
                             seed=(51,), chan_width_hz=dnu).numpy()
    out = oracle.xcorr(v, 4, T, F, 2, lib=lib)
    p = oracle.pair_index(1, 0)
    phase = np.unwrap(np.arctan2(out[:, p, 1].astype(float), out[:, p, 0].astype(float)))
    f = np.arange(F)
    slope = np.polyfit(f, phase, 1)[0]                      # rad per channel
    tau_fit = slope / (2 * math.pi * dnu)
    assert tau_fit != 0, "the phase of V_10 does not vary with frequency"
    vf = gd["cable_difference_m"] / tau_fit / synth.C_LIGHT
    assert abs(vf - gd["velocity_factor"]) <= gd["relative_tolerance"] * gd["velocity_factor"], \
        f"phase slope gives {vf:.4f} c, the paper measured {gd['velocity_factor']} c"


def sylvester_hadamard(n: int) -> np.ndarray:
    H = np.array([[1]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


def pin_orthogonal_codes(lib, N=8, T=64):
    """P6: x_k[t] = c * H[k][t] (Hadamard rows, real)  =>  V = c^2 T I exactly."""
    H = sylvester_hadamard(T)[:N]
    for c in (1, 3, 7):
        re = torch.from_numpy((c * H.T)[:, None, :].astype(np.int64))    # [T][1][N]
        im = torch.zeros_like(re)
        v = synth.pack4(re, im).numpy()
        out = oracle.xcorr(v, 4, T, 1, N, lib=lib)[0]
        for i in range(N):
            for j in range(i + 1):
                p = oracle.pair_index(i, j)
                want = c * c * T if i == j else 0
                assert out[p, 0] == want and out[p, 1] == 0, f"Hadamard pair ({i},{j}) c={c}"
        # rotate every input by i: x = i*c*H gives the same V
        v = synth.pack4(torch.zeros_like(re), re).numpy()
        out2 = oracle.xcorr(v, 4, T, 1, N, lib=lib)[0]
        assert np.array_equal(out, out2), "a common phase changed the visibilities"


def pin_additivity_linearity(lib, N=10, F=5, T=90, T1=37):
    """P7: V over [0,T) = V over [0,T1) + V over [T1,T); zero input gives zero;
    permuting channels permutes the output; an empty integration is zero."""
    v = synth.uniform_volts4(N, F, T, seed=(71,)).numpy()
    full = oracle.xcorr(v, 4, T, F, N, lib=lib)
    a = oracle.xcorr(np.ascontiguousarray(v[:T1]), 4, T1, F, N, lib=lib)
    b = oracle.xcorr(np.ascontiguousarray(v[T1:]), 4, T - T1, F, N, lib=lib)
    assert np.array_equal(full, a + b), "integration is not additive over time"
    z = oracle.xcorr(np.zeros_like(v), 4, T, F, N, lib=lib)
    assert not z.any(), "zero voltages gave non-zero visibilities"
    perm = np.array([3, 0, 4, 1, 2])[:F]
    vp = np.ascontiguousarray(v[:, perm, :])
    assert np.array_equal(oracle.xcorr(vp, 4, T, F, N, lib=lib), full[perm]), "channel permutation"
    sel = oracle.xcorr(v, 4, T, F, N, chans=[4, 1], lib=lib)
    assert np.array_equal(sel, full[[4, 1]]), "channel subset"
    e = oracle.xcorr(np.zeros((0, F, N), np.uint8), 4, 0, F, N, lib=lib)
    assert e.shape == full.shape and not e.any()


def pin_overflow_edge(lib, T=16_777_215):
    """P8: all samples -8-8i: every entry is 128*T.  T = floor((2^31-1)/128) is the
    last integration that fits int32; one more sample must be refused."""
    N, F = 2, 1
    v = np.full((T + 1, F, N), 0x88, dtype=np.uint8)
    out = oracle.xcorr(v[:T], 4, T, F, N, lib=lib)
    assert np.all(out[..., 0] == 128 * T) and np.all(out[..., 1] == 0)
    assert np.array_equal(oracle.to_int32(out)[..., 0], np.full((1, 3), 2_147_483_520, dtype=np.int32))
    over = oracle.xcorr(v, 4, T + 1, F, N, lib=lib)
    try:
        oracle.to_int32(over)
    except OverflowError:
        pass
    else:
        raise AssertionError("T_max + 1 samples was not refused")


def pin_distribution(lib, N=16, F=8, T=256):
    """P10: iid uniform components on {-8..7}: E[x]=-1/2, E[x^2]=43/2, so
    E[V_ii] = 43 T and E[V_ij] = (1/4 + 1/4) T = T/2 (real), E[Im] = 0."""
    v = synth.tiny().numpy()
    out = oracle.xcorr(v, 4, T, F, N, lib=lib).astype(np.float64) / T
    autos = [oracle.pair_index(i, i) for i in range(N)]
    cross = [oracle.pair_index(i, j) for i in range(N) for j in range(i)]
    assert abs(out[:, autos, 0].mean() - 43.0) < 0.5
    assert abs(out[:, cross, 0].mean() - 0.5) < 0.3
    assert abs(out[:, cross, 1].mean()) < 0.3


def pin_consistency(lib, N=9, F=3, T=45):
    """The double and single-pair entry points agree with the integer one."""
    for bits in (4, 8):
        v = (synth.uniform_volts4 if bits == 4 else synth.uniform_volts8)(N, F, T, seed=(81, bits)).numpy()
        a = oracle.xcorr(v, bits, T, F, N, lib=lib)
        d = oracle.xcorr_f64(v, bits, T, F, N, lib=lib)
        assert np.array_equal(a, d.astype(np.int64))
        for (f, i, j) in ((0, 0, 0), (2, 8, 3), (1, 5, 5)):
            assert oracle.xcorr_pair(v, bits, T, F, N, f, i, j, lib=lib) == tuple(a[f, oracle.pair_index(i, j)])


def pin_double_beyond_2_pow_24(lib, T=1500):
    """The double oracle is the FP64 reference of the half-precision path,
    whose partial sums pass 2^24 in its stress case: there every integer sum
    must still come out exact (below 2^53).  Closed form: every input carries
    (127, 126) and input 3 carries (-126, 127) = i * (127, 126), so the autos
    are (127^2 + 126^2) T = 32005 T (odd per sample, so a single-precision
    accumulator would round past 2^24), pairs (1, 0) and (2, 0) equal the auto,
    and V_30 = i * 32005 T; random 8-bit inputs then agree with the int64
    oracle at the same magnitude."""
    N, F = 4, 2
    re = torch.full((T, F, N), 127, dtype=torch.int64)
    im = torch.full((T, F, N), 126, dtype=torch.int64)
    re[:, :, 3], im[:, :, 3] = -126, 127
    v = synth.pack8(re, im).numpy()
    d = oracle.xcorr_f64(v, 8, T, F, N, lib=lib)
    big = 32005 * T
    assert big > 2 ** 24
    for i in range(N):
        p = oracle.pair_index(i, i)
        assert np.all(d[:, p, 0] == big) and np.all(d[:, p, 1] == 0), "auto beyond 2^24 is not exact"
    for i in (1, 2):
        assert np.all(d[:, oracle.pair_index(i, 0), 0] == big) and np.all(d[:, oracle.pair_index(i, 0), 1] == 0)
    p30 = oracle.pair_index(3, 0)
    assert np.all(d[:, p30, 0] == 0) and np.all(d[:, p30, 1] == big), "quarter-turn pair beyond 2^24"
    v8 = synth.uniform_volts8(N, F, T, seed=(82,), lo=100, hi=127).numpy()
    a = oracle.xcorr(v8, 8, T, F, N, lib=lib)
    d8 = oracle.xcorr_f64(v8, 8, T, F, N, lib=lib)
    assert np.abs(a).max() > 2 ** 24
    assert np.array_equal(a, d8.astype(np.int64)), "double oracle differs from int64 beyond 2^24"


ALL_PINS = [
    pin_library_zherk,
    pin_reversal_hermitian,
    pin_autos_and_cauchy_schwarz,
    pin_exact_phase_ramp,
    pin_delay_slope,
    pin_orthogonal_codes,
    pin_additivity_linearity,
    pin_overflow_edge,
    pin_distribution,
    pin_consistency,
    pin_double_beyond_2_pow_24,
]
