"""GPU F-engine front end against the F-engine oracle (paper Section 2.2).

The GPU computes in float32, the oracle in float64, each with its own
prototype coefficients (the library's float32 ones and the oracle's float64
ones).  Spectra agree within a float32 error bound; codes agree exactly
except where the oracle's scaled value lies within DELTA of a rounding
boundary (a half-integer, or the clip edge at 7.5 / -8.5), where the two
precisions may round differently and the codes may differ by one.  DELTA
covers the float32 spectrum error (asserted below 2e-6 of the largest
channel value, about 0.03 here; measured 1.7e-3) times the largest EQ gain
used (0.0068, or 0.054 in the clipping test) with a margin of 4x or more."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import fengine as fe  # noqa: E402
from paper_2406_19013_amd import synth  # noqa: E402
from paper_2406_19013_amd import xcorr as X  # noqa: E402

import oracle  # noqa: E402

P, F, TAPS = 2048, 1024, 4
DELTA = 1e-3
DEV = torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)


def _inputs(N, M, seed, extra=0, sigma=synth.FE_ADC_SIGMA, amps=(12.0, 8.0)):
    S = (M + TAPS - 1) * P + extra
    adc = synth.adc_samples(N, S, sigma=sigma, seed=(synth.BASE_SEED, 60, seed),
                            tones=(synth.AdcTone(freq=300.0 / P, amp=amps[0]), synth.AdcTone(freq=700.5 / P, amp=amps[1])))
    gains = synth.eq_gains(N, F, base=synth.FE_EQ_BASE, seed=(synth.BASE_SEED, 61, seed))
    return adc, gains


def _coeffs():
    return torch.from_numpy(X.xcorr_pfb_prototype()).to(DEV)


def _gpu_codes(adc, gains, M=None):
    N, S = adc.shape
    M = X.fe_n_spectra(S) if M is None else M
    out = torch.full((M, F, N), 0x5A, dtype=torch.uint8, device=DEV)
    X.xcorr_fengine(adc.to(DEV), _coeffs(), gains.to(DEV), out, M)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _gpu_codes_dev(adc, gains, M):
    N, S = adc.shape
    out = torch.empty((M, F, N), dtype=torch.uint8, device=DEV)
    X.xcorr_fengine(adc.to(DEV), _coeffs(), gains.to(DEV), out, M)
    return out


def _check_codes(got, adc, gains, M=None):
    """Exact codes away from rounding boundaries; within one code there."""
    a = adc.numpy()
    N, S = a.shape
    M = fe.n_spectra(S) if M is None else M
    want = fe.fengine(a[:, :(M + TAPS - 1) * P], gains.numpy().astype(np.float64))
    assert got.shape == want.shape
    Xs = fe.spectra(a[:, :(M + TAPS - 1) * P]) * gains.numpy().astype(np.float64)[:, None, :]   # [N][M][F]
    v = np.stack([Xs.real, Xs.imag], -1).transpose(1, 2, 0, 3)                                   # [M][F][N][2]
    near = np.abs(np.abs(v - np.floor(v)) - 0.5) < DELTA
    near_any = near[..., 0] | near[..., 1]

    def nib(b, hi):
        x = (b >> 4) if hi else (b & 15)
        return np.where(x >= 8, x.astype(np.int64) - 16, x.astype(np.int64))

    diff = got != want
    bad = diff & ~near_any
    assert not bad.any(), f"{int(bad.sum())} codes differ away from rounding boundaries, first at {np.argwhere(bad)[0]}"
    for hi in (True, False):
        d = np.abs(nib(got, hi) - nib(want, hi))
        assert d.max() <= 1
    _say(f"codes: {got.size} compared, {int(diff.sum())} differ (all within {DELTA} of a rounding boundary, "
         f"{int(near_any.sum())} values that close)")
    return want


@pytest.mark.parametrize("N,M", [(16, 5), (64, 3), (80, 2)])
def test_spectra_match_oracle(N, M):
    adc, _ = _inputs(N, M, seed=N)
    out = torch.empty((N, M, F, 2), dtype=torch.float32, device=DEV)
    X.xcorr_pfb_spectra(adc.to(DEV), _coeffs(), out, M)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    want = fe.spectra(adc.numpy())
    got_c = got[..., 0] + 1j * got[..., 1]
    err = np.abs(got_c - want)
    scale = np.abs(want).max()
    _say(f"spectra N={N} M={M}: max |dX| = {err.max():.3e}, max |X| = {scale:.1f}")
    # float32: FIR sums of 4 products and a 10-level FFT, relative to the
    # largest channel value
    assert err.max() <= 2e-6 * scale + 1e-3


@pytest.mark.parametrize("N,M,extra", [(16, 4, 0), (64, 2, 16), (80, 3, 2048 + 48)])
def test_codes_match_oracle(N, M, extra):
    adc, gains = _inputs(N, M, seed=100 + N, extra=extra)
    got = _gpu_codes(adc, gains, M)
    _check_codes(got, adc, gains, M)


def test_tianlai_shape_sampled_spectra():
    """192 inputs, 24 spectra (the production input count and channelisation,
    fewer spectra so that the oracle finishes in seconds): every code."""
    N, M = 192, 24
    adc, gains = _inputs(N, M, seed=7)
    got = _gpu_codes(adc, gains, M)
    _check_codes(got, adc, gains, M)


def test_requantisation_clips_and_ties():
    """A loud input clips at -8 and 7; gains that make channel values land on
    exact half-integers are avoided by DELTA, so this checks saturation."""
    N, M = 16, 2
    adc, gains = _inputs(N, M, seed=3, sigma=60.0)
    gains = gains * 8
    got = _gpu_codes(adc, gains, M)
    want = _check_codes(got, adc, gains, M)
    hi = want >> 4
    assert (hi == 0x7).any() and (hi == 0x8).any()


def test_fengine_feeds_xengine_end_to_end():
    """ADC samples -> GPU F-engine -> GPU X-engine: the visibilities are the
    X-engine oracle's on the same codes, and at the tone channel (bin 300, a
    1-code tone with a seeded phase per input, about 5.6 codes after EQ
    against 2.5 of noise) the visibility phases are the phase differences
    of the inputs: expected error about 0.03 rad over 1024 spectra."""
    N, M = 32, 1024
    adc, gains = _inputs(N, M, seed=11, amps=(1.0, 1.0))
    codes = _gpu_codes_dev(adc, gains, M)                   # [M][F][N] on the GPU
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA, device=DEV)
    vis, n, _ = c.ingest_dump(codes)
    torch.cuda.synchronize()
    assert n == M
    vis = vis.cpu().numpy()
    c.close()
    chans = np.array([300, 301, 700])
    sub = np.ascontiguousarray(codes.cpu().numpy()[:, chans, :])
    want = oracle.to_int32(oracle.xcorr(sub, 4, M, len(chans), N))
    assert np.array_equal(vis[chans], want)
    # input k carries cos(2 pi 300 s / 2048 + phi_k): phi from the generator's seed
    g = torch.Generator().manual_seed(synth.seed_of(synth.BASE_SEED, 60, 11, 0x7068))
    phi = (torch.rand(N, generator=g, dtype=torch.float64) * 2 * np.pi).numpy()
    V = vis[300, :, 0].astype(np.float64) + 1j * vis[300, :, 1]
    errs = []
    for i in range(N):
        for j in range(i):
            p = i * (i + 1) // 2 + j
            errs.append(abs(np.angle(V[p] * np.exp(-1j * (phi[i] - phi[j])))))
    _say(f"tone channel: max phase error {max(errs):.3f} rad over {len(errs)} baselines")
    assert max(errs) < 0.2


def test_fengine_refusals():
    adc = torch.zeros((16, 4 * P), dtype=torch.int8, device=DEV)
    h = _coeffs()
    g = torch.ones((16, F), dtype=torch.float32, device=DEV)
    out = torch.empty((1, F, 16), dtype=torch.uint8, device=DEV)
    X.xcorr_fengine(adc, h, g, out, 1)
    with pytest.raises(X.XcorrError):
        X.xcorr_fengine(adc, h, g, out, 2)                                     # too few samples
    with pytest.raises(X.XcorrError):
        X.xcorr_fengine(adc[:15], h, g, out, 1)                                # N not a multiple of 16
    with pytest.raises(X.XcorrError):
        X.xcorr_fengine(torch.zeros((16, 3 * P), dtype=torch.int8, device=DEV), h, g, out, 1)
    torch.cuda.synchronize()
