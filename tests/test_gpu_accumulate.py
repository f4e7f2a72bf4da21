"""GPU parity of the accumulating launches (an ingest that adds to running
sums) on every region shape, including the rectangles between diagonal
segments, and of the exact launch the benchmark times at full size."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
from paper_2406_19013_amd import synth
from paper_2406_19013_amd import xcorr as X

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _oracle_channels(v_np, T, N, chans, threads=8):
    """Oracle over whole channels, one thread per channel (each channel is
    independent)."""
    def one(f):
        vc = np.ascontiguousarray(v_np[:, f:f + 1])
        return oracle.to_int32(oracle.xcorr(vc, 4, T, 1, N))[0]
    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, chans))


# (N, F, tile, ingest sizes): several ingests so that every launch after the
# first accumulates; N = 512 with D = 4 has triangles and rectangles, N = 160
# with D = 5 and N = 192 with D = 6 run the batched running-sum loads of the
# large-region epilogue, N = 256 with D = 2 and N = 100 with D = 3 the
# per-element ones.
ACC_CASES = [(512, 6, 4, [128, 64, 192]), (160, 5, 5, [100, 128, 37]), (192, 4, 6, [64, 64, 64, 1]),
             (256, 5, 2, [64, 130]), (100, 3, 3, [77, 64])]


@pytest.mark.parametrize("N,F,tile,splits", ACC_CASES, ids=[f"N{n}D{d}" for n, _, d, _ in ACC_CASES])
def test_accumulating_launches_match_oracle(N, F, tile, splits):
    T = sum(splits)
    _say(f"accumulate N={N} F={F} D={tile} splits={splits}")
    v = synth.gaussian_volts(N, F, T, sigma=2.5, bits=4, seed=(5001, N, tile), tone=synth.Tone())
    vd = v.cuda()
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA, tile=tile)
    t0 = 0
    for n in splits:
        c.ingest(vd[t0:t0 + n], n)
        t0 += n
    out, n_int, _ = c.dump()
    torch.cuda.synchronize()
    assert n_int == T and c.stats()["tile"] == tile
    want = oracle.to_int32(oracle.xcorr(v.numpy(), 4, T, F, N))
    assert np.array_equal(out.cpu().numpy(), want)
    # the same integration with its last ingest fused with the dump
    t0 = 0
    for n in splits[:-1]:
        c.ingest(vd[t0:t0 + n], n)
        t0 += n
    out2, n2, _ = c.ingest_dump(vd[t0:], n_samples=splits[-1])
    torch.cuda.synchronize()
    assert n2 == T and np.array_equal(out2.cpu().numpy(), want)
    c.close()


@pytest.mark.parametrize("N,F,tile", [(512, 4, 4), (256, 3, 4), (96, 3, 3), (64, 5, 2), (192, 6, 6), (160, 3, 5)],
                         ids=["N512D4", "N256D4F3", "N96D3F3", "N64D2F5", "N192D6", "N160D5"])
def test_fused_blocks_accumulate_across_groups(N, F, tile):
    """Ten 128-sample device blocks in groups of at most 8 per launch (the
    second group adds to the first group's sums) against the oracle."""
    B, nb = 128, 10
    _say(f"ingest_blocks N={N} F={F} D={tile}")
    blocks = [synth.uniform_volts4(N, F, B, seed=(5002, N, k)) for k in range(nb)]
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA, tile=tile)
    c.ingest_blocks([b.cuda() for b in blocks])
    out, n, _ = c.dump()
    torch.cuda.synchronize()
    assert n == nb * B and c.stats()["kernel_launches"] == 2 + 1
    v = torch.cat(blocks)
    assert np.array_equal(out.cpu().numpy(), oracle.to_int32(oracle.xcorr(v.numpy(), 4, nb * B, F, N)))
    c.close()


def test_benchmark_launch_full_size_one_channel_per_xcd_range():
    """The call the benchmark times -- xcorr_ingest_dump of 192 inputs x 1024
    channels x 4096 samples, one launch that writes the visibilities straight
    to the caller's buffer -- against the oracle on whole channels: the first
    and last channel and one channel from each eighth of the band (each XCD
    takes a contiguous range of channels)."""
    N, F, T = 192, 1024, 4096
    _say("benchmark launch: generating")
    v = synth.tianlai(device="cuda")
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    out = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
    out.fill_(0x5A5A5A5A)
    for _ in range(2):   # the second call must not depend on the first
        _, n, _ = c.ingest_dump(v, out, T)
        assert n == T
    torch.cuda.synchronize()
    chans = [0, 128, 256, 384, 512, 640, 768, 896, 1023, 77, 1000]
    _say("benchmark launch: oracle on 11 channels")
    vn = v[:, chans, :].cpu().numpy()
    want = _oracle_channels(vn, T, N, range(len(chans)))
    got = out[chans].cpu().numpy()
    for k, f in enumerate(chans):
        assert np.array_equal(got[k], want[k]), f"channel {f}"
    om = out.cpu().numpy()
    autos = [oracle.pair_index(i, i) for i in range(N)]
    assert not om[:, autos, 1].any() and (om[:, autos, 0] > 0).all()
    c.close()


def test_benchmark_integration_full_size_is_n_times_one_ingest():
    """An integration of four identical 4096-sample ingests of the benchmark
    array (192 inputs x 1024 channels; the first stores, the other three add
    to the running sums) dumps exactly four times what one ingest dumps: a
    property of the sum that holds on every pair at full size."""
    N, F, T = 192, 1024, 4096
    _say("integration at full size: generating")
    v = synth.tianlai(device="cuda")
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    one = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
    c.ingest_dump(v, one, T)
    for _ in range(4):
        c.ingest(v, T)
    four = torch.empty_like(one)
    _, n, _ = c.dump(four)
    torch.cuda.synchronize()
    assert n == 4 * T
    assert torch.equal(four, one * 4)
    c.close()
