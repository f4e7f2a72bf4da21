"""GPU full-Stokes formation against the Stokes oracle, bit for bit (int64)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from oracle import stokes as st  # noqa: E402
from paper_2406_19013_amd import synth  # noqa: E402
from paper_2406_19013_amd import xcorr as X  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("N,F", [(2, 1), (6, 3), (192, 4)])
def test_random_dumps(N, F):
    """Any int32 visibilities, including the extremes: the int64 sums are exact."""
    rng = np.random.default_rng(N * 7 + F)
    P = N * (N + 1) // 2
    v = rng.integers(-2 ** 31, 2 ** 31, size=(F, P, 2), dtype=np.int64).astype(np.int32)
    v[0, 0] = [2 ** 31 - 1, -2 ** 31]
    got = X.xcorr_stokes(torch.from_numpy(v).to(DEV), N).cpu().numpy()
    assert np.array_equal(got, st.stokes(v, N))


def test_polarised_source_end_to_end():
    """4+4-bit voltages: each feed's X carries a common signal s plus noise
    and Y carries s too (linear at 45 degrees), so U dominates Q and V in
    every feed pair; GPU X-engine + GPU Stokes equal the oracles exactly."""
    N, F, T = 32, 4, 512
    g = torch.Generator().manual_seed(synth.seed_of(synth.BASE_SEED, 70))
    s_re = torch.randint(-3, 4, (T, F, 1), generator=g)
    s_im = torch.randint(-3, 4, (T, F, 1), generator=g)
    n_re = torch.randint(-2, 3, (T, F, N), generator=g)
    n_im = torch.randint(-2, 3, (T, F, N), generator=g)
    v = synth.pack4(s_re + n_re, s_im + n_im)
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA, device=DEV)
    vis, _, _ = c.ingest_dump(v.to(DEV))
    c.close()
    got = X.xcorr_stokes(vis, N).cpu().numpy()
    want = st.stokes(oracle.xcorr(v.numpy(), 4, T, F, N), N)
    assert np.array_equal(got, want)
    Q, U, V = (np.abs(want[:, :, k, 0]) for k in (1, 2, 3))
    assert (U > 4 * Q).mean() > 0.9 and (U > 4 * V).mean() > 0.9


def test_refusals():
    v = torch.zeros((1, 6, 2), dtype=torch.int32, device=DEV)
    with pytest.raises(X.XcorrError):
        X.xcorr_stokes(v, 3)
