"""GPU parity: the HIP kernels, called through the C ABI, against the CPU
oracle.  Integer paths must match bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_19013_amd import synth
from paper_2406_19013_amd import xcorr as X

pytestmark = pytest.mark.gpu

PATHS = {"plain": X.PATH_PLAIN, "mfma": X.PATH_I8_MFMA}


def _say(msg):
    print(msg, flush=True)


def gpu_correlate(volts_cpu: torch.Tensor, N, F, bits=4, path=X.PATH_I8_MFMA, tile=0, splits=None):
    v = volts_cpu.cuda()
    T = v.shape[0]
    c = X.Correlator(N, F, bits, path, tile)
    if splits is None:
        splits = [T]
    t0 = 0
    for n in splits:
        c.ingest(v[t0:t0 + n], n)
        t0 += n
    assert t0 == T
    out, n_int, gaps = c.dump()
    torch.cuda.synchronize()
    assert n_int == T
    res = out.cpu().numpy()
    c.close()
    return res


def expected(volts_cpu, N, F, bits=4):
    T = volts_cpu.shape[0]
    return oracle.to_int32(oracle.xcorr(volts_cpu.numpy(), bits, T, F, N))


@pytest.mark.parametrize("path", PATHS)
def test_tiny_config_bit_exact(path):
    _say(f"tiny {path}")
    v = synth.tiny()
    got = gpu_correlate(v, 16, 8, 4, PATHS[path])
    assert np.array_equal(got, expected(v, 16, 8))


RAGGED = [(1, 1, 1), (2, 3, 17), (5, 2, 64), (16, 4, 65), (20, 3, 200), (31, 2, 33), (32, 2, 128),
          (33, 2, 96), (63, 2, 70), (64, 3, 129), (65, 2, 64), (96, 2, 150), (100, 2, 77),
          (130, 2, 64), (160, 2, 100), (191, 2, 65), (192, 3, 130), (200, 2, 64), (256, 2, 90),
          (300, 2, 66)]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N,F,T", RAGGED, ids=[f"N{n}F{f}T{t}" for n, f, t in RAGGED])
def test_ragged_shapes_bit_exact(path, N, F, T):
    _say(f"ragged {path} N={N} F={F} T={T}")
    v = synth.uniform_volts4(N, F, T, seed=(1001, N, F, T))
    got = gpu_correlate(v, N, F, 4, PATHS[path])
    assert np.array_equal(got, expected(v, N, F))


TILES = [(192, 2), (192, 3), (192, 4), (192, 6), (160, 5), (96, 3), (64, 2), (256, 4), (256, 2),
         (130, 2), (300, 3), (512, 4), (20, 1),
         # several segments whose last one runs past N (three-product rectangles
         # with partial or empty blocks)
         (208, 4), (400, 3), (336, 2), (272, 4), (112, 2)]


# the default 4+4-bit kernel (fused products) and the per-role one
VARIANTS = ["fused", "roles"]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("N,tile", TILES, ids=[f"N{n}D{d}" for n, d in TILES])
def test_every_tile_shape_bit_exact(N, tile, variant, monkeypatch):
    if variant == "roles":
        monkeypatch.setenv("XCORR_MFMA4_VARIANT", "roles")
    F, T = 2, 200
    _say(f"tile N={N} D={tile} {variant}")
    v = synth.gaussian_volts(N, F, T, sigma=2.5, bits=4, seed=(1002, N, tile), tone=synth.Tone())
    got = gpu_correlate(v, N, F, 4, X.PATH_I8_MFMA, tile)
    assert np.array_equal(got, expected(v, N, F))


# tiles 2 to 4 run their triangles two channels to an item: an odd F
# leaves the last item one channel; F = 1 runs single triangles
PAIRS = [(128, 3, 4), (128, 1, 4), (96, 2, 4), (208, 5, 4), (256, 3, 4), (512, 3, 4),
         (96, 3, 3), (96, 1, 3), (80, 2, 3), (288, 5, 3), (208, 3, 3),
         (64, 3, 2), (64, 1, 2), (48, 2, 2), (320, 3, 2)]


@pytest.mark.parametrize("N,F,tile", PAIRS, ids=[f"N{n}F{f}D{d}" for n, f, d in PAIRS])
def test_channel_pairs_of_small_triangles(N, F, tile):
    T = 150
    _say(f"channel pairs N={N} F={F} D={tile}")
    v = synth.uniform_volts4(N, F, T, seed=(1010, N, F))
    # two ingests: the second launch adds to the first's sums
    got = gpu_correlate(v, N, F, 4, X.PATH_I8_MFMA, tile, splits=[64, 86])
    assert np.array_equal(got, expected(v, N, F))


@pytest.mark.parametrize("path", PATHS)
def test_ingest_splits_accumulate_exactly(path):
    N, F = 48, 3
    splits = [37, 64, 1, 100, 63]
    T = sum(splits)
    _say(f"splits {path}")
    v = synth.uniform_volts4(N, F, T, seed=(1003,))
    got = gpu_correlate(v, N, F, 4, PATHS[path], splits=splits)
    assert np.array_equal(got, expected(v, N, F))


@pytest.mark.parametrize("variant", VARIANTS)
def test_extreme_mix_across_launch_split(variant, monkeypatch):
    """Re and im drawn from {-8, 7} (the largest products of both signs) over
    140,001 samples, more than one launch of either kernel takes."""
    if variant == "roles":
        monkeypatch.setenv("XCORR_MFMA4_VARIANT", "roles")
    N, F, T = 16, 1, 140_001
    _say(f"extreme mix {variant}")
    g = torch.Generator().manual_seed(11)
    pick = torch.tensor([-8, 7], dtype=torch.int32)
    re = pick[torch.randint(0, 2, (T, F, N), generator=g)]
    im = pick[torch.randint(0, 2, (T, F, N), generator=g)]
    v = synth.pack4(re, im)
    got = gpu_correlate(v, N, F, 4, X.PATH_I8_MFMA)
    assert np.array_equal(got, expected(v, N, F))


@pytest.mark.parametrize("path", PATHS)
def test_extreme_values_and_launch_split(path):
    """All samples -8-8i across more samples than one MFMA launch takes:
    every entry is 128*T (closed form)."""
    N, F, T = 16, 1, 140_001
    _say(f"extreme {path}")
    v = torch.full((T, F, N), 0x88, dtype=torch.uint8)
    got = gpu_correlate(v, N, F, 4, PATHS[path])
    assert np.all(got[..., 0] == 128 * T) and np.all(got[..., 1] == 0)


def test_int32_edge_and_refusal():
    """T_max = 16,777,215 samples of -8-8i reach 2,147,483,520; one more sample
    is refused before anything is enqueued."""
    N, F, T = 16, 1, X.TMAX_4BIT
    _say("int32 edge")
    v = torch.full((T, F, N), 0x88, dtype=torch.uint8, device="cuda")
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    c.ingest(v, T)
    with pytest.raises(X.XcorrError) as ei:
        c.ingest(v[:1], 1)
    assert ei.value.code == X.XCORR_E_OVERFLOW
    out, n, _ = c.dump()
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert n == T and np.all(o[..., 0] == 2_147_483_520) and np.all(o[..., 1] == 0)
    c.close()


def test_dump_semantics_and_sequence_gaps():
    N, F, T = 24, 2, 50
    v = synth.uniform_volts4(N, F, T, seed=(1004,)).cuda()
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA, max_samples_per_dump=120)
    c.ingest(v, T, seq=10)
    c.ingest(v, T, seq=11)
    with pytest.raises(X.XcorrError) as ei:
        c.ingest(v, T, seq=12)                       # 150 > 120
    assert ei.value.code == X.XCORR_E_OVERFLOW
    c.ingest(v[:20], 20, seq=14)                     # gap of 2 (12, 13 missing)
    out, n, gaps = c.dump()
    assert n == 120 and gaps == 2
    ref = oracle.xcorr(v.cpu().numpy(), 4, T, F, N) * 2 + oracle.xcorr(v[:20].cpu().numpy(), 4, 20, F, N)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.to_int32(ref))
    out2, n2, gaps2 = c.dump()                        # empty integration
    torch.cuda.synchronize()
    assert n2 == 0 and gaps2 == 0 and not out2.cpu().numpy().any()
    c.ingest(v, T, seq=15)                            # first ingest after a dump overwrites
    out3, n3, _ = c.dump()
    torch.cuda.synchronize()
    assert n3 == T and np.array_equal(out3.cpu().numpy(), expected(v.cpu(), N, F))
    st = c.stats()
    assert st["dumps"] == 3 and st["ingests"] == 4 and st["seq_gaps_total"] == 2
    c.close()


def test_run_to_run_determinism():
    N, F, T = 192, 16, 512
    v = synth.gaussian_volts(N, F, T, sigma=2.5, bits=4, seed=(1005,), tone=synth.Tone()).cuda()
    a = X.Correlator(N, F)
    outs = []
    for _ in range(3):
        a.ingest(v, T)
        o, _, _ = a.dump()
        outs.append(o.clone())
    torch.cuda.synchronize()
    assert all(torch.equal(outs[0], o) for o in outs[1:])
    a.close()


def test_tianlai_full_size_sampled():
    """192 inputs x 1024 channels x 4096 samples (the benchmark workload, same
    launch configuration): 3 whole channels against the oracle, 64 random
    pairs over all channels, and the plain path over the whole output."""
    N, F, T = 192, 1024, 4096
    _say("tianlai full size")
    v = synth.tianlai(device="cuda")
    m = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    m.ingest(v, T)
    out_m, _, _ = m.dump()
    p = X.Correlator(N, F, 4, X.PATH_PLAIN)
    p.ingest(v, T)
    out_p, _, _ = p.dump()
    torch.cuda.synchronize()
    chans = [0, 517, 1023]
    vc = v[:, chans, :].cpu().numpy()
    ref = oracle.to_int32(oracle.xcorr(np.ascontiguousarray(vc), 4, T, len(chans), N))
    got = out_m[chans].cpu().numpy()
    assert np.array_equal(got, ref)
    rng = np.random.default_rng(7)
    vn = None
    om = out_m.cpu().numpy()
    for _ in range(64):
        f = int(rng.integers(F))
        i = int(rng.integers(N))
        j = int(rng.integers(i + 1))
        if vn is None:
            vn = v.cpu().numpy()
        assert tuple(om[f, oracle.pair_index(i, j)]) == oracle.xcorr_pair(vn, 4, T, F, N, f, i, j)
    assert torch.equal(out_m, out_p)
    autos = [oracle.pair_index(i, i) for i in range(N)]
    assert not om[:, autos, 1].any() and (om[:, autos, 0] >= 0).all()
    m.close()
    p.close()


PERSIST = [(256, 300, 4), (96, 700, 3), (64, 1100, 2), (192, 700, 6), (512, 40, 4), (130, 500, 2)]


@pytest.mark.parametrize("N,F,tile", PERSIST, ids=[f"N{n}F{f}D{d}" for n, f, d in PERSIST])
def test_persistent_workgroups_walk_many_regions(N, F, tile):
    """More (channel, region) items than resident work-groups: each work-group
    walks several items, mixing triangles and rectangles; every channel is
    checked on a sample of channels against the oracle."""
    T = 96
    _say(f"persistent N={N} F={F} D={tile}")
    v = synth.uniform_volts4(N, F, T, seed=(1006, N, F))
    got = gpu_correlate(v, N, F, 4, X.PATH_I8_MFMA, tile)
    chans = sorted(set([0, 1, F // 3, F // 2, F - 2, F - 1]))
    ref = oracle.to_int32(oracle.xcorr(v.numpy(), 4, T, F, N, chans=chans))
    assert np.array_equal(got[chans], ref)


SHORT = [(192, 700, 6, 64), (256, 300, 4, 96), (128, 900, 4, 128), (96, 1400, 3, 100), (512, 60, 4, 64)]


@pytest.mark.parametrize("N,F,tile,T", SHORT, ids=[f"N{n}F{f}D{d}T{t}" for n, f, d, t in SHORT])
def test_short_launches_with_many_items_per_workgroup(N, F, tile, T):
    """Launches of at most two 64-sample chunks, several items per
    work-group: consecutive epilogues with no group barrier of the K loop
    between them must not overwrite each other's per-input sums (every
    channel checked, three launches)."""
    _say(f"short launches N={N} F={F} D={tile} T={T}")
    v = synth.uniform_volts4(N, F, T, seed=(1011, N, F, T))
    want = expected(v, N, F)
    for _ in range(3):
        assert np.array_equal(gpu_correlate(v, N, F, 4, X.PATH_I8_MFMA, tile), want)


@pytest.mark.parametrize("N,F,splits", [(192, 4, [300]), (64, 3, [100, 129]), (100, 2, [64, 77]),
                                         (16, 1, [140_001])],
                         ids=["one_ingest", "after_ingest", "ragged_inputs", "launch_split"])
def test_ingest_dump_writes_the_integration(N, F, splits):
    """The last ingest fused with its dump: the output equals the oracle over
    every sample of the integration, and the integration is empty after it."""
    T = sum(splits)
    _say(f"ingest_dump N={N} F={F} splits={splits}")
    v = synth.uniform_volts4(N, F, T, seed=(1010, N, T))
    vd = v.cuda()
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA)
    t0 = 0
    for n in splits[:-1]:
        c.ingest(vd[t0:t0 + n], n)
        t0 += n
    out, n_int, gaps = c.ingest_dump(vd[t0:], n_samples=splits[-1])
    torch.cuda.synchronize()
    assert n_int == T and gaps == 0
    assert np.array_equal(out.cpu().numpy(), expected(v, N, F))
    assert c.stats()["samples_integrated"] == 0 and c.stats()["dumps"] == 1
    empty, n0, _ = c.dump()
    torch.cuda.synchronize()
    assert n0 == 0 and not empty.cpu().numpy().any()
    # the next integration starts from zero
    out2, n2, _ = c.ingest_dump(vd[:50], n_samples=50)
    torch.cuda.synchronize()
    assert n2 == 50 and np.array_equal(out2.cpu().numpy(), expected(v[:50], N, F))
    c.close()


def test_ingest_dump_on_other_paths_matches_two_calls():
    N, F, T = 40, 2, 90
    v = synth.uniform_volts8(N, F, T, seed=(1011,))
    for path in (X.PATH_I8_MFMA, X.PATH_PLAIN):
        c = X.Correlator(N, F, 8, path)
        out, n, _ = c.ingest_dump(v.cuda(), n_samples=T)
        torch.cuda.synchronize()
        assert n == T and np.array_equal(out.cpu().numpy(), oracle.to_int32(oracle.xcorr(v.numpy(), 8, T, F, N)))
        c.close()
