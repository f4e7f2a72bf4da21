"""GPU parity of the batched persistent launch (several arrays of uneven N, F
and sample count in one kernel), its HIP-graph replay, and the autotuner.
Integer results must match the oracle bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_19013_amd import synth
from paper_2406_19013_amd import xcorr as X

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def want(v_cpu, N, F):
    return oracle.to_int32(oracle.xcorr(v_cpu.numpy(), 4, v_cpu.shape[0], F, N))


def dump_all(cors):
    outs = []
    for c in cors:
        o, n, _ = c.dump()
        outs.append((o, n))
    torch.cuda.synchronize()
    return [(o.cpu().numpy(), n) for o, n in outs]


# (N, F, T): uneven inputs, channels and sample counts; a batch whose every
# N % 16 == 0 runs the three-product batch kernel (triangles of 2, 4 and 6
# blocks, rectangles of 4 here), any other N the queue-driven one
VEC_SET = [(64, 6, 300), (192, 3, 1000), (256, 2, 77), (32, 5, 2048), (512, 1, 130)]
RAGGED_SET = [(100, 3, 77), (20, 4, 515), (192, 2, 64), (33, 3, 200)]


@pytest.mark.parametrize("arrays", [VEC_SET, RAGGED_SET], ids=["vec", "ragged"])
def test_batch_matches_oracle(arrays):
    _say(f"batch arrays {arrays}")
    vs = [synth.uniform_volts4(N, F, T, seed=(3001, N, F, T)) for N, F, T in arrays]
    cors = [X.Correlator(N, F, 4, X.PATH_I8_MFMA) for N, F, _ in arrays]
    b = X.Batch(cors)
    assert all(t in (2, 3, 4, 6) for t in b.tiles)
    b.ingest([v.cuda() for v in vs])
    for (got, n), v, (N, F, T) in zip(dump_all(cors), vs, arrays):
        assert n == T
        assert np.array_equal(got, want(v, N, F)), (N, F, T)
    b.close()


@pytest.mark.parametrize("arrays", [[(64, 3), (96, 2), (20, 4)], [(64, 3), (96, 2), (160, 4)]],
                         ids=["queue", "three_product"])
def test_batch_uneven_ingests_accumulate_and_skip(arrays):
    """Three batched ingests with per-array counts (some 0) add up to the
    oracle over each array's concatenated samples."""
    _say(f"uneven ingests {arrays}")
    counts = [[100, 0, 33], [1, 50, 0], [129, 7, 64]]
    cors = [X.Correlator(N, F, 4, X.PATH_I8_MFMA) for N, F in arrays]
    b = X.Batch(cors)
    parts = [[] for _ in arrays]
    for k, ns in enumerate(counts):
        vols = []
        for a, ((N, F), n) in enumerate(zip(arrays, ns)):
            if n == 0:
                vols.append(None)
                continue
            v = synth.uniform_volts4(N, F, n, seed=(3002, a, k))
            parts[a].append(v)
            vols.append(v.cuda())
        b.ingest(vols, ns)
    for (got, n), (N, F), p in zip(dump_all(cors), arrays, parts):
        v = torch.cat(p)
        assert n == v.shape[0]
        assert np.array_equal(got, want(v, N, F))
    b.close()


def test_batch_every_region_shape(tmp_path, monkeypatch):
    """Tiles from the batch tune cache put every shape the three-product batch
    kernel carries into one launch: triangles of 2, 3, 4 and 6 blocks and
    rectangles of 2, 3 and 4 (several segments, the last one partial)."""
    cache = tmp_path / "tune.txt"
    cache.write_text("4 320 2 1 2 xc_gauss4_batch_kernel\n"
                     "4 288 3 1 3 xc_gauss4_batch_kernel\n"
                     "4 208 2 1 4 xc_gauss4_batch_kernel\n"
                     "4 128 2 1 4 xc_gauss4_batch_kernel\n"
                     "4 256 3 1 4 xc_gauss4_batch_kernel\n")
    monkeypatch.setenv("XCORR_TUNE_CACHE", str(cache))
    # 2- to 4-block triangles go two channels to an item; 256 x 3, 288 x 3
    # and 48 x 3 leave the last item one channel, 96 x 1, 64 x 1 and 160 x 1
    # run single triangles
    arrays = [(320, 2, 150), (288, 3, 100), (208, 2, 90), (128, 2, 70), (96, 2, 64), (160, 1, 33), (48, 3, 129),
              (256, 3, 77), (96, 1, 50), (64, 1, 40)]
    _say(f"batch region shapes {arrays}")
    assert [X.xcorr_autotune_kernel(X.make_config(N, F, 4, X.PATH_I8_MFMA), batch=True)
            for N, F, _ in arrays] == ["xc_gauss4_batch_kernel"] * len(arrays)
    vs = [synth.uniform_volts4(N, F, T, seed=(3008, N, F, T)) for N, F, T in arrays]
    cors = [X.Correlator(N, F, 4, X.PATH_I8_MFMA) for N, F, _ in arrays]
    b = X.Batch(cors)
    assert b.tiles == [2, 3, 4, 4, 3, 6, 2, 4, 3, 2], b.tiles
    b.ingest([v.cuda() for v in vs])
    for (got, n), v, (N, F, T) in zip(dump_all(cors), vs, arrays):
        assert n == T
        assert np.array_equal(got, want(v, N, F)), (N, F, T)
    b.close()


def test_batch_long_ingest_splits_launches():
    """140,001 samples of -8-8i on one array, 1000 on another: the host splits
    the long one across two launches (131,071 samples per launch)."""
    T1 = 140_001
    v1 = torch.full((T1, 1, 16), 0x88, dtype=torch.uint8)
    v2 = synth.uniform_volts4(48, 2, 1000, seed=(3003,))
    cors = [X.Correlator(16, 1, 4, X.PATH_I8_MFMA), X.Correlator(48, 2, 4, X.PATH_I8_MFMA)]
    b = X.Batch(cors)
    b.ingest([v1.cuda(), v2.cuda()])
    assert cors[0].stats()["kernel_launches"] == 2 and cors[1].stats()["kernel_launches"] == 1
    (g1, n1), (g2, n2) = dump_all(cors)
    assert n1 == T1 and np.all(g1[..., 0] == 128 * T1) and np.all(g1[..., 1] == 0)
    assert np.array_equal(g2, want(v2, 48, 2))
    b.close()


def test_batch_repeated_launches_reset_queue():
    """Five launches in a row: the work queue is back at zero after each, so
    every launch covers every item (the sum is 5x one ingest)."""
    arrays = [(64, 4, 256), (160, 2, 128)]
    vs = [synth.uniform_volts4(N, F, T, seed=(3004, N)) for N, F, T in arrays]
    cors = [X.Correlator(N, F, 4, X.PATH_I8_MFMA) for N, F, _ in arrays]
    b = X.Batch(cors)
    vd = [v.cuda() for v in vs]
    for _ in range(5):
        b.ingest(vd)
    for (got, n), v, (N, F, T) in zip(dump_all(cors), vs, arrays):
        assert n == 5 * T
        assert np.array_equal(got, 5 * want(v, N, F).astype(np.int64))
    b.close()


def test_batched_workload_matches_single_path():
    """The four-array workload (64x256, 192x1024, 256x512, 512x128 inputs x
    channels, 2048 samples): batch equals the single-array path over every
    output, and the oracle on sampled channels."""
    _say("batched workload full size")
    vs = synth.batched(device="cuda")
    cors = [X.Correlator(N, F, 4, X.PATH_I8_MFMA) for N, F in synth.BATCH_ARRAYS]
    b = X.Batch(cors)
    b.ingest(vs)
    outs = [c.dump()[0] for c in cors]
    for v, (N, F), got in zip(vs, synth.BATCH_ARRAYS, outs):
        s = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
        s.ingest(v)
        ref, _, _ = s.dump()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (N, F)
        chans = [0, F // 2, F - 1]
        vc = np.ascontiguousarray(v[:, chans].cpu().numpy())
        assert np.array_equal(got[chans].cpu().numpy(),
                              oracle.to_int32(oracle.xcorr(vc, 4, v.shape[0], len(chans), N)))
        s.close()
    b.close()


@pytest.mark.parametrize("arrays", [[(64, 4, 512), (192, 2, 256), (100, 3, 96)],
                                    [(64, 4, 512), (192, 2, 256), (320, 3, 96)]],
                         ids=["queue", "three_product"])
def test_batch_graph_replay(arrays):
    """Capture [batched ingest, per-array dumps] in a HIP graph; between
    replays refill the inputs and run eager work on the same arrays; every
    replay must equal the oracle for the inputs it saw."""
    _say(f"batch graph {arrays}")
    cors = [X.Correlator(N, F, 4, X.PATH_I8_MFMA) for N, F, _ in arrays]
    b = X.Batch(cors)
    vin = [torch.empty((T, F, N), dtype=torch.uint8, device="cuda") for N, F, T in arrays]
    outs = [torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda") for N, F, _ in arrays]
    sets = [[synth.uniform_volts4(N, F, T, seed=(3005, k, N)) for N, F, T in arrays] for k in range(3)]
    for d, v in zip(vin, sets[0]):
        d.copy_(v)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=side):
        b.ingest(vin)
        for c, o in zip(cors, outs):
            c.dump(o)
    torch.cuda.synchronize()
    for k in range(3):
        for d, v in zip(vin, sets[k]):
            d.copy_(v)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, v, (N, F, T) in zip(outs, sets[k], arrays):
            assert np.array_equal(o.cpu().numpy(), want(v, N, F)), (k, N)
        # eager work in between: a batched ingest and dumps of other data
        b.ingest([x.cuda() for x in sets[(k + 1) % 3]])
        eager = dump_all(cors)
        for (e, n), v, (N, F, T) in zip(eager, sets[(k + 1) % 3], arrays):
            assert n == T and np.array_equal(e, want(v, N, F))
    b.close()


def test_batch_rejects_mixed_paths():
    c4 = X.Correlator(64, 2, 4, X.PATH_I8_MFMA)
    c8 = X.Correlator(64, 2, 8, X.PATH_I8_MFMA)
    with pytest.raises(X.XcorrError) as ei:
        X.Batch([c4, c8])
    assert ei.value.code == X.XCORR_E_INVAL
    b = X.Batch([c4])
    with pytest.raises(X.XcorrError) as ei:
        # refused on the host before anything is enqueued: the buffer is never read
        b.ingest([torch.zeros((1, 2, 64), dtype=torch.uint8, device="cuda")], [X.TMAX_4BIT + 1])
    assert ei.value.code == X.XCORR_E_OVERFLOW
    b.close()


@pytest.mark.parametrize("bits,path,N,F", [(4, X.PATH_I8_MFMA, 192, 64), (8, X.PATH_I8_MFMA, 96, 32),
                                           (8, X.PATH_F16_MFMA, 64, 16)])
def test_autotune_picks_supported_tile_and_caches(tmp_path, monkeypatch, bits, path, N, F):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("XCORR_TUNE_CACHE", str(cache))
    monkeypatch.delenv("XCORR_MFMA4_VARIANT", raising=False)
    best = X.autotune(N, F, bits, path)
    assert 1 <= best <= 6
    lines = cache.read_text().split("\n")
    kernel = X.xcorr_autotune_kernel(X.make_config(N, F, bits, path))
    assert lines[0].split() == [str(bits), str(N), str(F), str(path), str(best), kernel]
    c = X.Correlator(N, F, bits, path)
    assert c.stats()["tile"] == best and c.stats()["tile_from_cache"] == 1
    v = (synth.uniform_volts4(N, F, 70, seed=(3006,)) if bits == 4
         else synth.uniform_volts8(N, F, 70, seed=(3006,)))
    c.ingest(v.cuda())
    got, _, _ = c.dump()
    exp = oracle.xcorr(v.numpy(), bits, 70, F, N)
    if path == X.PATH_F16_MFMA:
        assert np.array_equal(got.cpu().numpy().astype(np.int64), exp)
    else:
        assert np.array_equal(got.cpu().numpy(), oracle.to_int32(exp))
    c.close()


def test_batch_autotune_times_the_batched_kernel_and_batch_uses_it(tmp_path, monkeypatch):
    """The batch tuner times the batched kernel over the tiles it carries
    and writes a line naming it; a batch built afterwards takes that tile for
    the member (the member's own single-array tile is separate) and stays
    exact."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("XCORR_TUNE_CACHE", str(cache))
    monkeypatch.delenv("XCORR_MFMA4_VARIANT", raising=False)
    N, F, T = 256, 32, 130
    best = X.autotune(N, F, 4, X.PATH_I8_MFMA, batch=True)
    assert best in (2, 3, 4)
    assert cache.read_text().split() == ["4", str(N), str(F), "1", str(best), "xc_gauss4_batch_kernel"]
    cfg = X.make_config(N, F, 4, X.PATH_I8_MFMA)
    assert X.xcorr_plan_tile(cfg, batch=True) == (best, True)
    assert X.xcorr_plan_tile(cfg) == (4, False)          # no line for the single-array kernel
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    b = X.Batch([c])
    assert b.tiles == [best]
    v = synth.uniform_volts4(N, F, T, seed=(3007,))
    b.ingest([v.cuda()])
    got, n, _ = c.dump()
    torch.cuda.synchronize()
    assert n == T and np.array_equal(got.cpu().numpy(), want(v, N, F))
    b.close()
    c.close()
