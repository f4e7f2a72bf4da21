"""Host side of the GPU F-engine: the library's own prototype filter (float32)
equals the oracle's (float64) to float32 rounding, and the channel count of
the requested shape (paper Section 2.2: 2^11-point filter bank, 4 taps)."""
import numpy as np

from oracle import fengine as fe
from paper_2406_19013_amd import xcorr as X


def test_library_prototype_matches_oracle():
    h = X.xcorr_pfb_prototype(2048, 4).astype(np.float64)
    ho = fe.prototype(2048, 4)
    assert h.shape == ho.shape == (8192,)
    assert np.max(np.abs(h - ho)) <= 2 ** -24 * np.max(np.abs(ho))
    small = X.xcorr_pfb_prototype(16, 4).astype(np.float64)
    assert np.max(np.abs(small - fe.prototype(16, 4))) <= 2 ** -24


def test_spectra_count():
    assert X.fe_n_spectra(4 * 2048) == 1 == fe.n_spectra(4 * 2048)
    assert X.fe_n_spectra(4099 * 2048) == 4096
