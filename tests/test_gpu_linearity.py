"""Linearity of the whole chain on synthetic data, the paper's correlator
linearity test (Section 3.4: output amplitude against input power, a linear
range of -22 to 0 dBm at the operating ADC gain) with the ADC replaced by
seeded samples: pairs of inputs share a common noise signal (correlation
coefficient 0.5) whose power is stepped over 40 dB; the GPU F-engine (fixed
EQ gains set for 16 ADC codes of noise) and X-engine give the cross power of
each pair.  Ideal response: output proportional to input power.  Checked:
within 1 dB of that line over at least 20 dB around the operating point,
compression above it (4-bit clipping), a floor below it (4-bit codes going to
zero)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2406_19013_amd import synth  # noqa: E402
from paper_2406_19013_amd import xcorr as X  # noqa: E402

DEV = torch.device("cuda:0")
P, F, TAPS = 2048, 1024, 4


def linearity_curve(levels_db, N=16, M=64, seed=0):
    """Mean cross power of the input pairs (2k, 2k+1) over channels 100..900
    for each input power level (dB relative to 16 ADC codes of noise)."""
    S = (M + TAPS - 1) * P
    h = torch.from_numpy(X.xcorr_pfb_prototype()).to(DEV)
    gains = torch.full((N, F), synth.FE_EQ_BASE, dtype=torch.float32, device=DEV)
    codes = torch.empty((M, F, N), dtype=torch.uint8, device=DEV)
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA, device=DEV)
    out = []
    g = torch.Generator(device=DEV).manual_seed(synth.seed_of(synth.BASE_SEED, 80, seed))
    common = torch.randn((N // 2, S), generator=g, device=DEV)
    own = torch.randn((N, S), generator=g, device=DEV)
    for db in levels_db:
        sigma = synth.FE_ADC_SIGMA * 10 ** (db / 20)
        x = (common.repeat_interleave(2, 0) + own) * (sigma / np.sqrt(2))   # rho = 0.5, variance sigma^2
        adc = torch.clamp(torch.round(x), -128, 127).to(torch.int8)
        X.xcorr_fengine(adc, h, gains, codes, M)
        vis, _, _ = c.ingest_dump(codes)
        v = vis.double().cpu().numpy()
        p = np.array([(2 * k + 1) * (2 * k + 2) // 2 + 2 * k for k in range(N // 2)])
        out.append(v[100:900][:, p, 0].mean())
    c.close()
    return np.array(out)


def test_linear_range_around_operating_point():
    levels = np.arange(-30, 12, 2.0)
    y = linearity_curve(levels)
    ydb = 10 * np.log10(np.maximum(y, 1e-12))
    # ideal line through the operating point (0 dB): slope 1 in power
    ref = ydb[levels == 0][0]
    dev = ydb - (ref + levels)
    lin = np.abs(dev) <= 1.0
    # contiguous linear run containing 0 dB
    i0 = int(np.where(levels == 0)[0][0])
    lo = i0
    while lo > 0 and lin[lo - 1]:
        lo -= 1
    hi = i0
    while hi + 1 < len(levels) and lin[hi + 1]:
        hi += 1
    print(f"linear within 1 dB from {levels[lo]:+.0f} to {levels[hi]:+.0f} dB "
          f"(deviations {np.round(dev, 2).tolist()})", flush=True)
    assert levels[hi] - levels[lo] >= 20
    assert dev[-1] < -1.0          # compression at the top (clipping)
    assert dev[0] > 1.0 or dev[0] < -1.0   # the floor departs from the line at the bottom
