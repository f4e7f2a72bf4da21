"""The allocation-free entry point (xcorr_correlate_static) against the
context path it varies (xcorr_ingest_dump): two calls in a row on one GPU,
the second with a smaller input, each equal to the context's result bit for
bit (and to the oracle), including integrations whose running sums live in
the library's static array."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_19013_amd import synth
from paper_2406_19013_amd import xcorr as X

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _context_result(cfg, v, n):
    c = X.Correlator(cfg.n_inputs, cfg.n_chans, cfg.sample_bits, cfg.path, cfg.tile)
    out, n_int, _ = c.ingest_dump(v, n_samples=n)
    torch.cuda.synchronize()
    c.close()
    assert n_int == n
    return out.cpu().numpy()


# (inputs, channels, bits, path, [sample counts of the two calls]): one
# 4+4-bit launch (no scratch), integrations across launches (scratch), 8+8-bit
# int8 and FP16 and the plain path (scratch)
CASES = [(64, 8, 4, X.PATH_I8_MFMA, [3000, 700]), (32, 4, 4, X.PATH_I8_MFMA, [140_001, 131_000]),
         (48, 3, 8, X.PATH_I8_MFMA, [2000, 257]), (40, 2, 8, X.PATH_F16_MFMA, [900, 300]),
         (24, 5, 4, X.PATH_PLAIN, [500, 99])]


@pytest.mark.parametrize("N,F,bits,path,ns", CASES, ids=["i8_one_launch", "i8_across_launches", "i8_8bit",
                                                          "f16", "plain"])
def test_static_entry_matches_context_path_twice(N, F, bits, path, ns):
    cfg = X.make_config(N, F, bits, path)
    gen = synth.uniform_volts4 if bits == 4 else synth.uniform_volts8
    for k, n in enumerate(ns):
        _say(f"static N={N} F={F} bits={bits} path={path} call {k} n={n}")
        v = gen(N, F, n, seed=(6001, N, k))
        vd = v.cuda()
        out = torch.full((F, N * (N + 1) // 2, 2), -7, dtype=torch.float32 if path == X.PATH_F16_MFMA
                         else torch.int32, device="cuda")
        n_int = X.xcorr_correlate_static(cfg, vd, n, out)
        torch.cuda.synchronize()
        assert n_int == n
        got = out.cpu().numpy()
        assert np.array_equal(got, _context_result(cfg, vd, n))
        if path == X.PATH_F16_MFMA:
            continue
        if n * N * F < 4_000_000:
            assert np.array_equal(got, oracle.to_int32(oracle.xcorr(v.numpy(), bits, n, F, N)))


def test_static_entry_refuses_sums_beyond_the_scratch():
    """192 inputs x 1024 channels needs 152 MB of running sums: beyond the
    16 MiB array, refused before anything is enqueued (the input pointer is
    never read); a single launch of the same shape needs none and runs."""
    cfg = X.make_config(192, 1024, 4, X.PATH_I8_MFMA)
    dummy = torch.zeros(16, dtype=torch.uint8, device="cuda")
    out = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(X.XcorrError) as ei:
        X.xcorr_correlate_static(cfg, dummy, 140_000, out)
    assert ei.value.code == X.XCORR_E_NOMEM
    with pytest.raises(X.XcorrError) as ei:
        X.xcorr_correlate_static(X.make_config(192, 1024, 8, X.PATH_I8_MFMA), dummy, 10, out)
    assert ei.value.code == X.XCORR_E_NOMEM
    N, F, T = 192, 64, 1024
    v = synth.tianlai(device="cuda", F=F, T=T)
    o = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
    assert X.xcorr_correlate_static(X.make_config(N, F), v, T, o) == T
    torch.cuda.synchronize()
    assert np.array_equal(o.cpu().numpy(), _context_result(X.make_config(N, F), v, T))
