"""GPU tests of the streaming loop: blocks pushed through a pipe (host blocks
over the copy stream into the ring, or device blocks in place) integrate and
dump exactly as the oracle over each integration's samples (additivity over
blocks), with sequence gaps counted and latencies reported."""
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


@pytest.mark.parametrize("host", [True, False], ids=["host_blocks", "device_blocks"])
def test_pipe_dumps_match_oracle(host):
    N, F, B, every, nblk = 64, 8, 256, 4, 10
    blocks = [synth.uniform_volts4(N, F, B, seed=(4001, k)) for k in range(nblk)]
    src = [b.pin_memory() if host else b.cuda() for b in blocks]
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    p = X.Pipe(c, B, every, n_slots=3, host_blocks=host)
    outs = []
    for k, b in enumerate(src):
        o = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
        if p.push(b, out=o):
            outs.append((k, o))
    p.drain()
    torch.cuda.synchronize()
    assert [k for k, _ in outs] == [3, 7]
    for (k, o) in outs:
        v = torch.cat(blocks[k - every + 1:k + 1])
        want = oracle.to_int32(oracle.xcorr(v.numpy(), 4, v.shape[0], F, N))
        assert np.array_equal(o.cpu().numpy(), want), k
    # the two blocks after the last dump are still integrating
    tail, n, _ = c.dump()
    torch.cuda.synchronize()
    v = torch.cat(blocks[8:])
    assert n == 2 * B
    assert np.array_equal(tail.cpu().numpy(), oracle.to_int32(oracle.xcorr(v.numpy(), 4, 2 * B, F, N)))
    st = p.stats()
    assert st["blocks"] == nblk and st["dumps"] == 2 and st["latencies"] == nblk
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    p.close()
    c.close()


def test_pipe_counts_sequence_gaps():
    N, F, B = 32, 2, 64
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    p = X.Pipe(c, B, 100, host_blocks=False)
    blk = synth.uniform_volts4(N, F, B, seed=(4002,)).cuda()
    for seq in (0, 1, 2, 5, 6, 9):
        p.push(blk, seq=seq)
    p.drain()
    st = c.stats()
    assert st["seq_gaps"] == 4 and st["samples_integrated"] == 6 * B
    p.close()
    c.close()


def test_pipe_refuses_integration_past_the_int32_bound():
    c = X.Correlator(16, 1, 4, X.PATH_I8_MFMA, max_samples_per_dump=1000)
    with pytest.raises(X.XcorrError) as ei:
        X.Pipe(c, 100, 11, host_blocks=False)
    assert ei.value.code == X.XCORR_E_OVERFLOW
    c.close()


@pytest.mark.parametrize("fuse", [1, 8])
def test_streaming_workload_first_dump_sampled(fuse):
    """192 inputs x 4096 channels, 1024-sample blocks from a pool of 4
    device-resident blocks in rotation, one dump per 128 blocks (131,072
    samples), one launch per block or 8 blocks per launch (as the benchmark
    runs them): the dump equals the oracle on 8 sampled channels."""
    N, F, B, every, pool_n = 192, 4096, 1024, 128, 4
    _say(f"streaming workload fuse={fuse}: generating the block pool")
    pool = [synth.stream_block(N, F, k, array_id=1, device="cuda") for k in range(pool_n)]
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    p = X.Pipe(c, B, every, host_blocks=False)
    p.set_fuse(fuse)
    out = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
    for k in range(every):
        p.push(pool[k % pool_n], out=out)
    p.drain()
    torch.cuda.synchronize()
    chans = [0, 511, 1024, 2047, 2048, 3000, 4094, 4095]
    sub = [pl[:, chans].cpu().numpy() for pl in pool]
    got = out[chans].cpu().numpy()
    _say("streaming workload: oracle on 8 channels")
    # each channel of the oracle is independent; one thread per channel
    v = np.concatenate([sub[k % pool_n] for k in range(every)])

    def one(ci):
        vc = np.ascontiguousarray(v[:, ci:ci + 1])
        return oracle.xcorr(vc, 4, v.shape[0], 1, N)[0]

    with cf.ThreadPoolExecutor(8) as ex:
        want = list(ex.map(one, range(len(chans))))
    for ci in range(len(chans)):
        assert np.array_equal(got[ci], oracle.to_int32(want[ci])), chans[ci]
    st = p.stats()
    assert st["dumps"] == 1 and st["blocks"] == every
    assert st["latencies"] == every // fuse and st["submit_latencies"] == every
    assert st["submit_p50_ms"] > 0 and st["submit_p99_ms"] <= st["submit_max_ms"]
    p.close()
    c.close()


@pytest.mark.parametrize("N,F,B,bits", [(64, 4, 128, 4), (96, 3, 100, 4), (100, 2, 64, 4), (48, 2, 64, 8)],
                         ids=["one_launch", "ragged_block", "ragged_inputs", "eight_bit"])
def test_ingest_blocks_matches_oracle(N, F, B, bits):
    """Five separate device blocks ingested as one integration: one launch
    when the shape allows it, else one per block; the result is the oracle
    over the concatenated samples either way."""
    nb = 5
    gen = synth.uniform_volts4 if bits == 4 else synth.uniform_volts8
    blocks = [gen(N, F, B, seed=(4010, N, k)) for k in range(nb)]
    c = X.Correlator(N, F, bits, X.PATH_I8_MFMA)
    c.ingest_blocks([b.cuda() for b in blocks])
    out, n, _ = c.dump()
    torch.cuda.synchronize()
    v = torch.cat(blocks)
    assert n == nb * B
    assert np.array_equal(out.cpu().numpy(), oracle.to_int32(oracle.xcorr(v.numpy(), bits, nb * B, F, N)))
    fused = bits == 4 and B % 64 == 0 and N % 16 == 0
    assert c.stats()["kernel_launches"] == (1 if fused else nb) + 1
    c.close()


def test_pipe_fuses_device_blocks():
    """fuse = 3, a dump every 7 blocks, 10 blocks: groups of 3, 3 and 1 (the
    dump), then 3 held until the drain; dumps and the tail match the oracle."""
    N, F, B, every = 64, 4, 128, 7
    blocks = [synth.uniform_volts4(N, F, B, seed=(4011, k)) for k in range(10)]
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    p = X.Pipe(c, B, every, host_blocks=False)
    p.set_fuse(3)
    out = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
    dev = [b.cuda() for b in blocks]
    dumped = [p.push(b, out=out) for b in dev]
    assert dumped == [False] * 6 + [True] + [False] * 3
    p.drain()
    torch.cuda.synchronize()
    first = out.cpu().numpy().copy()
    v = torch.cat(blocks[:7])
    assert np.array_equal(first, oracle.to_int32(oracle.xcorr(v.numpy(), 4, 7 * B, F, N)))
    tail, n, _ = c.dump()
    torch.cuda.synchronize()
    v = torch.cat(blocks[7:])
    assert n == 3 * B
    assert np.array_equal(tail.cpu().numpy(), oracle.to_int32(oracle.xcorr(v.numpy(), 4, 3 * B, F, N)))
    st = p.stats()
    assert st["blocks"] == 10 and st["dumps"] == 1 and st["latencies"] == 4
    # 4 fused launches (3, 3, 1, 3 blocks) and one dump inside the pipe, one dump above
    assert c.stats()["kernel_launches"] == 4 + 2
    p.close()
    c.close()


@pytest.mark.parametrize("host", [False, True], ids=["device_blocks", "host_blocks"])
def test_pipe_keeps_dropped_blocks_alive(host):
    """The caller drops each block right after pushing it and allocates a
    block-sized tensor of junk: with 8 device blocks held per launch (or a
    pinned host block copied by the library) the pipe must keep the block's
    memory until its launch has read it, or the junk would be correlated."""
    N, F, B, nb = 64, 8, 256, 16
    src = [synth.uniform_volts4(N, F, B, seed=(4020, k)) for k in range(nb)]
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    p = X.Pipe(c, B, 0, n_slots=2, host_blocks=host)
    if not host:
        p.set_fuse(8)
    junk = []
    for k in range(nb):
        blk = src[k].pin_memory() if host else src[k].cuda()
        p.push(blk)
        del blk
        j = torch.empty((B, F, N), dtype=torch.uint8).pin_memory() if host else \
            torch.empty((B, F, N), dtype=torch.uint8, device="cuda")
        j.fill_(0x77)
        junk.append(j)
    out = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
    n, _ = p.dump(out)
    p.drain()
    torch.cuda.synchronize()
    assert n == nb * B and p.stats()["held"] == 0
    v = torch.cat(src)
    assert np.array_equal(out.cpu().numpy(), oracle.to_int32(oracle.xcorr(v.numpy(), 4, nb * B, F, N)))
    p.close()
    c.close()
