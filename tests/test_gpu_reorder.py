"""GPU test of sequence-number reassembly in front of the streaming loop:
device blocks arrive shuffled within the reorder window, some are lost and
some duplicated; the reorder stage releases them in order and cuts
integrations at fixed sequence numbers (the nodes' common packet-counter
origin, Sections 2.2 and 2.3), and the pipe dumps on each boundary event.
Every dumped integration must equal the oracle over the blocks of that
integration that arrived, and report their samples and sequence gaps."""
import random

import numpy as np
import pytest
import torch

import oracle
from paper_2406_19013_amd import synth
from paper_2406_19013_amd import xcorr as X

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fuse", [1, 4], ids=["one_launch_per_block", "fused_groups"])
def test_reassembled_stream_matches_oracle(fuse):
    N, F, B, k, w, origin = 48, 4, 128, 6, 3, 1000
    nblk = 30
    print(f"reorder stream N={N} F={F} B={B} k={k} w={w} fuse={fuse}", flush=True)
    rng = random.Random(7)
    lost = {1003, 1010, 1011, 1020}
    blocks = {s: synth.uniform_volts4(N, F, B, seed=(4101, s)) for s in range(origin, origin + nblk)}
    dev = {s: b.cuda() for s, b in blocks.items()}
    arrivals = [s for s in blocks if s not in lost]
    arrivals = sorted(arrivals, key=lambda s: s + rng.uniform(0, w + 1))
    arrivals.insert(9, arrivals[5])                     # a duplicate
    arrivals.insert(0, origin - 2)                      # before the origin
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    p = X.Pipe(c, B, 0, host_blocks=False)              # dumps only on boundary events
    p.set_fuse(fuse)
    r = X.Reorder(k, w, max_missing=1, seq_origin=origin)
    results = []

    def handle(events):
        for e in events:
            if e["kind"] == "block":
                p.push(e["block"], seq=e["seq"])
            elif e["kind"] == "dump":
                o = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
                n, gaps = p.dump(o)
                results.append((e, o, n, gaps))

    for s in arrivals:
        handle(r.push(s, dev.get(s, dev[origin])))
    handle(r.flush(True))
    p.drain()
    torch.cuda.synchronize()
    assert [e["integration"] for e, *_ in results] == [0, 1, 2, 3, 4]
    for e, o, n, gaps in results:
        present = [s for s in range(e["seq"], e["seq"] + k) if s in blocks and s not in lost]
        assert e["n_blocks"] == len(present) and e["n_missing"] == k - len(present)
        assert e["valid"] == (k - len(present) <= 1)
        assert n == len(present) * B
        v = torch.cat([blocks[s] for s in present])
        want = oracle.to_int32(oracle.xcorr(v.numpy(), 4, v.shape[0], F, N))
        assert np.array_equal(o.cpu().numpy(), want), e
    st = r.stats()
    assert st["duplicate"] + st["late"] == 1 and st["before_origin"] == 1
    assert st["missing"] == len(lost) and st["released"] == nblk - len(lost)
    p.close()
    r.close()
    c.close()


def test_explicit_dump_restarts_the_count():
    """An explicit dump ends the integration and restarts the count of
    dump_every: blocks 0-1 (explicit), then 2-4 (automatic after three)."""
    N, F, B = 32, 2, 64
    print(f"explicit dump N={N} F={F} B={B}", flush=True)
    blocks = [synth.uniform_volts4(N, F, B, seed=(4102, k)) for k in range(6)]
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    p = X.Pipe(c, B, 3, host_blocks=False)
    outs = [torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda") for _ in range(2)]
    p.push(blocks[0].cuda(), seq=0)
    p.push(blocks[1].cuda(), seq=1)
    n, gaps = p.dump(outs[0])
    assert (n, gaps) == (2 * B, 0)
    dumped = [p.push(blocks[k].cuda(), out=outs[1], seq=k) for k in (2, 3, 4)]
    assert dumped == [False, False, True]
    p.drain()
    torch.cuda.synchronize()
    for o, ks in ((outs[0], (0, 1)), (outs[1], (2, 3, 4))):
        v = torch.cat([blocks[k] for k in ks])
        want = oracle.to_int32(oracle.xcorr(v.numpy(), 4, v.shape[0], F, N))
        assert np.array_equal(o.cpu().numpy(), want), ks
    p.close()
    c.close()
