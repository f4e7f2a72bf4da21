"""GPU parity of the 8+8-bit paths: int8 MFMA (exact, int32) and FP16 MFMA
with FP32 accumulation (against the FP64 oracle)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_19013_amd import synth
from paper_2406_19013_amd import xcorr as X

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def run(v_cpu, N, F, path, tile=0, splits=None):
    v = v_cpu.cuda()
    T = v.shape[0]
    c = X.Correlator(N, F, 8, path, tile)
    t0 = 0
    for n in (splits or [T]):
        c.ingest(v[t0:t0 + n], n)
        t0 += n
    out, n_int, _ = c.dump()
    torch.cuda.synchronize()
    assert n_int == T
    res = out.cpu().numpy()
    c.close()
    return res


RAGGED8 = [(1, 1, 1), (5, 2, 33), (8, 3, 64), (16, 2, 65), (20, 2, 100), (33, 2, 96), (64, 2, 130),
           (96, 2, 64), (100, 2, 70), (192, 3, 129), (200, 2, 64), (256, 2, 66), (300, 2, 40)]


@pytest.mark.parametrize("path", ["int8", "plain"])
@pytest.mark.parametrize("N,F,T", RAGGED8, ids=[f"N{n}F{f}T{t}" for n, f, t in RAGGED8])
def test_8bit_exact(path, N, F, T):
    _say(f"8bit {path} N={N} F={F} T={T}")
    v = synth.uniform_volts8(N, F, T, seed=(2001, N, F, T))
    p = X.PATH_I8_MFMA if path == "int8" else X.PATH_PLAIN
    got = run(v, N, F, p)
    want = oracle.to_int32(oracle.xcorr(v.numpy(), 8, T, F, N))
    assert np.array_equal(got, want)


TILES8 = [(192, 6), (192, 3), (192, 2), (192, 4), (160, 5), (256, 4), (130, 2), (20, 1), (512, 4)]


@pytest.mark.parametrize("N,tile", TILES8, ids=[f"N{n}D{d}" for n, d in TILES8])
def test_8bit_every_tile_shape(N, tile):
    F, T = 2, 192
    _say(f"8bit tile N={N} D={tile}")
    v = synth.gaussian_volts(N, F, T, sigma=20.0, bits=8, seed=(2002, N, tile))
    got = run(v, N, F, X.PATH_I8_MFMA, tile)
    want = oracle.to_int32(oracle.xcorr(v.numpy(), 8, T, F, N))
    assert np.array_equal(got, want)


def test_8bit_splits_and_extremes():
    N, F = 40, 3
    splits = [17, 64, 1, 50]
    T = sum(splits)
    g = torch.Generator().manual_seed(5)
    vals = torch.tensor([-127, 127, -1, 0, 1, 126, -126], dtype=torch.int8)
    v = vals[torch.randint(0, len(vals), (T, F, N, 2), generator=g)]
    got = run(v, N, F, X.PATH_I8_MFMA, splits=splits)
    assert np.array_equal(got, oracle.to_int32(oracle.xcorr(v.numpy(), 8, T, F, N)))


def test_8bit_int32_edge_and_refusal():
    """T_max = 66,572 samples of (-127, -127): every entry is 2*127^2*T =
    2,147,479,576 (closed form); one more sample is refused."""
    N, F, T = 16, 1, X.TMAX_8BIT
    v = torch.full((T, F, N, 2), -127, dtype=torch.int8, device="cuda")
    c = X.Correlator(N, F, 8, X.PATH_I8_MFMA)
    c.ingest(v, T)
    with pytest.raises(X.XcorrError) as ei:
        c.ingest(v[:1], 1)
    assert ei.value.code == X.XCORR_E_OVERFLOW
    out, n, _ = c.dump()
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert n == T and np.all(o[..., 0] == 2 * 127 * 127 * T) and np.all(o[..., 1] == 0)
    c.close()


def fp16_errors(got, want):
    """Max |dV| / sqrt(V_ii V_jj), max |dV| / |V| where |V| >= 1e-3 sqrt(V_ii V_jj),
    and max |dV|, over all channels and pairs."""
    N = int((np.sqrt(8 * got.shape[1] + 1) - 1) / 2)
    autos = np.array([oracle.pair_index(i, i) for i in range(N)])
    ii, jj = np.tril_indices(N)
    d = np.hypot(got[..., 0] - want[..., 0], got[..., 1] - want[..., 1])
    norm = np.sqrt(want[:, autos[ii], 0] * want[:, autos[jj], 0])
    mag = np.hypot(want[..., 0], want[..., 1])
    rel_cc = float(np.max(d / np.maximum(norm, 1e-300)))
    big = mag >= 1e-3 * norm
    rel = float(np.max(d[big] / mag[big])) if big.any() else 0.0
    return rel_cc, rel, float(np.max(d))


def test_fp16_exact_below_2_pow_24():
    """sigma = 20, T = 8192 (the precision workload's statistics): every partial
    sum is an integer below 2^24, so FP32 accumulation of exact FP16 products
    reproduces the FP64 oracle exactly."""
    N, F, T = 96, 4, 8192
    v = synth.gaussian_volts(N, F, T, sigma=20.0, bits=8, seed=(2003,))
    got = run(v, N, F, X.PATH_F16_MFMA)
    want = oracle.xcorr_f64(v.numpy(), 8, T, F, N)
    assert np.abs(want).max() < 2 ** 24
    assert np.array_equal(got.astype(np.float64), want)


def test_fp16_error_bounded_beyond_2_pow_24():
    """sigma = 60 over 65,536 samples: sums pass 2^24 and FP32 rounds; the
    error stays within the worst-case accumulation bound T * 2^-23 in
    correlation-coefficient units."""
    N, F, T = 16, 2, 65536
    v = synth.gaussian_volts(N, F, T, sigma=60.0, bits=8, seed=(2004,))
    got = run(v, N, F, X.PATH_F16_MFMA)
    want = oracle.xcorr_f64(v.numpy(), 8, T, F, N)
    assert np.abs(want).max() > 2 ** 24
    rel_cc, rel, mx = fp16_errors(got.astype(np.float64), want)
    _say(f"fp16 stress: max |dV|/sqrt(ViiVjj) = {rel_cc:.3e}, max |dV|/|V| = {rel:.3e}, max |dV| = {mx:.1f}")
    assert rel_cc <= T * 2.0 ** -23
    assert rel_cc > 0


def test_precision_workload_full_size_sampled():
    """192 inputs x 512 channels x 8192 samples of 8+8-bit noise: int8 path
    bit-exact on sampled channels, FP16 path exact against FP64 there, and the
    int8 and plain paths agree over the whole output."""
    N, F, T = 192, 512, 8192
    _say("precision workload full size")
    v = synth.precision8(device="cuda")
    outs = {}
    for name, p in (("int8", X.PATH_I8_MFMA), ("f16", X.PATH_F16_MFMA), ("plain", X.PATH_PLAIN)):
        c = X.Correlator(N, F, 8, p)
        c.ingest(v, T)
        outs[name], _, _ = c.dump()
        torch.cuda.synchronize()
        c.close()
    chans = [0, 255, 511]
    vc = np.ascontiguousarray(v[:, chans].cpu().numpy())
    want = oracle.xcorr(vc, 8, T, len(chans), N)
    assert np.array_equal(outs["int8"][chans].cpu().numpy(), oracle.to_int32(want))
    assert np.array_equal(outs["f16"][chans].cpu().numpy().astype(np.float64), want.astype(np.float64))
    assert torch.equal(outs["int8"], outs["plain"])


ACC8 = [(192, 6), (512, 4), (160, 5), (192, 3), (130, 2), (20, 1)]


@pytest.mark.parametrize("path", ["int8", "fp16"])
@pytest.mark.parametrize("N,tile", ACC8, ids=[f"N{n}D{d}" for n, d in ACC8])
def test_8bit_accumulating_launches_every_tile_shape(path, N, tile):
    """Several ingests per integration (every launch after the first adds to
    the running sums) on triangles of 1 to 6 blocks and the rectangles
    between segments; the FP16 path is exact here (every partial and total
    sum is an integer below 2^24)."""
    F, splits = 2, [64, 1, 127]
    T = sum(splits)
    _say(f"8bit accumulate {path} N={N} D={tile}")
    v = synth.gaussian_volts(N, F, T, sigma=20.0, bits=8, seed=(2003, N, tile))
    got = run(v, N, F, X.PATH_I8_MFMA if path == "int8" else X.PATH_F16_MFMA, tile, splits=splits)
    want = oracle.xcorr(v.numpy(), 8, T, F, N)
    assert np.abs(want).max() < 2 ** 24
    if path == "int8":
        assert np.array_equal(got, oracle.to_int32(want))
    else:
        assert np.array_equal(got.astype(np.float64), want.astype(np.float64))
