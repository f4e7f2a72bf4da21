"""Benchmark of the X-engine hot path on one MI355X.

A step is one integration of the benchmark workload through the whole hot
path: ingest (HBM read of packed 4+4-bit voltages, unpack/corner turn in LDS,
int8 MFMA contraction, int32 accumulation) followed by dump (accumulators to
the caller's [F][P][2] buffer).

Workload: 192 inputs (96 dual-polarisation feeds), 1024 channels, 4096
samples per channel, 4+4-bit Gaussian noise (sigma 2.5) plus a common tone,
generated on the device from a fixed seed.  The data span of one step is
4096 / (125 MHz / 1024) = 33.55 ms of sky.

Prints one JSON line: complex MAC/s of the int8-MFMA path, the real-time
factor of the MFMA and plain paths, p50/p99 step latency, the roofline of the
dominant kernel from HIP events on its launch stream, and the CPU oracle's
rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_INPUTS, N_CHANS, N_SAMPLES = 192, 1024, 4096
BANDWIDTH_HZ = 125e6
INT8_PEAK_TOPS = 5000.0       # MI355X dense int8 MFMA, 10^12 ops/s
HBM_PEAK_GBS = 8000.0
OPS_PER_CMAC = 8              # one complex multiply-accumulate = 4 real MACs
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_sha() -> str:
    from paper_2406_19013_amd.profsum import kernel_source_sha as sha
    return sha()


def measured_traffic(kernel: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if it was taken on the current
    kernel source; else None."""
    p = os.path.join(PROFILES, f"{kernel}_tianlai_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    if d.get("kernel_src_sha") != kernel_source_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(volts_dev, n_chan_sample: int, n_chan_single: int):
    """The oracle as it stands on the host cores: one thread per channel
    slice over n_chan_sample channels, and one thread over n_chan_single."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    affinity = len(os.sched_getaffinity(0))
    cores = min(16, affinity)
    lib = oracle.load_library()

    def run(n_chan, threads):
        sub = volts_dev[:, :n_chan, :].contiguous().cpu().numpy()
        T, F, N = sub.shape
        chans = np.arange(F)
        slices = [chans[k::threads] for k in range(threads)]
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda c: oracle.xcorr(sub, 4, T, F, N, chans=c, lib=lib), slices))
        dt = time.perf_counter() - t0
        cmacs = F * (N * (N + 1) // 2) * T
        return cmacs / dt, f"{N} inputs x {F} of {N_CHANS} channels x {T} samples ({cmacs:.3e} CMAC) in {dt:.2f} s wall"

    v_all, s_all = run(n_chan_sample, cores)
    v_one, s_one = run(n_chan_single, 1)
    return {"value": v_all, "unit": "CMAC/s", "cores": cores, "kind": "oracle", "sample": s_all,
            "single_thread": {"value": v_one, "unit": "CMAC/s", "cores": 1, "sample": s_one},
            "host": {"cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(), "affinity_cpus": affinity}}


def _progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed(fn, stream, reps: int, warmup: int = 2, after=None):
    """Mean and per-call milliseconds of fn() on `stream`, from HIP events;
    after() (untimed) follows every call."""
    import numpy as np
    import torch
    for _ in range(warmup):
        fn()
        if after:
            after()
    stream.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
        if after:
            after()
    stream.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    return float(ms.mean()), ms


def fp_error_metrics(approx, exact, N: int) -> dict:
    """Error of an FP visibility set against the exact one, three ways:
    max |dV| / sqrt(V_ii V_jj) (correlation-coefficient units), max |dV| / |V|
    over entries with |V| >= 1e-3 sqrt(V_ii V_jj), and max |dV|."""
    import torch
    idx = torch.arange(N, device=exact.device)
    diag = idx * (idx + 1) // 2 + idx
    ii = torch.repeat_interleave(idx, idx + 1)
    jj = torch.cat([torch.arange(i + 1, device=exact.device) for i in range(N)])
    auto = exact[..., diag, 0]                            # [F][N], real and >= 0
    norm = torch.sqrt(auto[:, ii] * auto[:, jj]).clamp_min(1e-300)
    d = torch.linalg.vector_norm(approx - exact, dim=-1)
    mag = torch.linalg.vector_norm(exact, dim=-1)
    big = mag >= 1e-3 * norm
    return {"max_err_over_sqrt_autos": float((d / norm).max()),
            "max_rel_err_large_entries": float((d[big] / mag[big]).max()) if bool(big.any()) else 0.0,
            "max_abs_err": float(d.max()), "max_abs_value": float(mag.max())}


def bench_precision8(dev, stream, reps: int) -> dict:
    """8+8-bit input through the exact int8 path and the FP16-MFMA/FP32 path:
    192 inputs x 512 channels x 8192 samples (sigma 20), and a stress case of
    192 inputs x 16 channels x 65,536 samples (sigma 60) whose sums pass 2^24.
    FP16 errors are stated against the int8 path's exact result (bit-exact to
    the FP64 oracle on these inputs, which the parity tests check)."""
    import torch

    from paper_2406_19013_amd import synth
    from paper_2406_19013_amd import xcorr as X

    res = {}
    for label, (F, T, sigma), timed in (("precision-192in-512ch-8192t-8bit", (512, 8192, 20.0), True),
                                        ("stress-192in-16ch-65536t-8bit-sigma60", (16, 65536, 60.0), False)):
        N = 192
        with torch.cuda.stream(stream):
            v = synth.gaussian_volts(N, F, T, sigma=sigma, bits=8, seed=(synth.BASE_SEED, 3, int(sigma)),
                                     device=dev) if not timed else synth.precision8(device=dev)
        stream.synchronize()
        ops = OPS_PER_CMAC * N * (N + 1) // 2 * F * T
        r, outs = {"workload": label}, {}
        for name, path, peak in (("int8_mfma", X.PATH_I8_MFMA, INT8_PEAK_TOPS), ("f16_mfma", X.PATH_F16_MFMA, 2500.0)):
            c = X.Correlator(N, F, 8, path, device=dev)
            outs[name] = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.float32 if path == X.PATH_F16_MFMA
                                     else torch.int32, device=dev)
            if timed:
                ms, _ = _timed(lambda: c.ingest(v, T, stream=stream), stream, reps,
                               after=lambda: c.dump(outs[name], stream=stream))
                r[name] = {"ingest_ms": ms, "tops": ops / ms / 1e9, "peak": peak, "frac": ops / ms / 1e9 / peak,
                           "tile": c.stats()["tile"]}
            else:
                c.ingest(v, T, stream=stream)
                c.dump(outs[name], stream=stream)
            stream.synchronize()
            c.close()
        exact = outs["int8_mfma"].double()
        r["f16_vs_exact"] = fp_error_metrics(outs["f16_mfma"].double(), exact, N)
        res["config3" if timed else "stress"] = r
        del v, outs, exact
    return res


def bench_batched(dev, stream, reps: int) -> dict:
    """Four arrays (64x256, 192x1024, 256x512, 512x128 inputs x channels,
    2048 samples) in one launch, the same launch replayed from a HIP graph,
    and one launch per array and region shape."""
    import torch

    from paper_2406_19013_amd import synth
    from paper_2406_19013_amd import xcorr as X

    with torch.cuda.stream(stream):
        vs = synth.batched(device=dev)
    stream.synchronize()
    T = vs[0].shape[0]
    # tiles tuned on the batched kernel into a private tune cache
    import tempfile
    cache_dir = tempfile.mkdtemp(prefix="xcorr_tune_")
    prev_cache = os.environ.get("XCORR_TUNE_CACHE")
    os.environ["XCORR_TUNE_CACHE"] = os.path.join(cache_dir, "tune.txt")
    tuned = [X.autotune(N, F, device=dev, stream=stream, batch=True) for N, F in synth.BATCH_ARRAYS]
    cors = [X.Correlator(N, F, 4, X.PATH_I8_MFMA, device=dev) for N, F in synth.BATCH_ARRAYS]
    cmac = sum(N * (N + 1) // 2 * F * T for N, F in synth.BATCH_ARRAYS)
    b = X.Batch(cors, device=dev)
    outs = [torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device=dev) for N, F in synth.BATCH_ARRAYS]

    def dumps():
        for c, o in zip(cors, outs):
            c.dump(o, stream=stream)

    def singles():
        for c, v in zip(cors, vs):
            c.ingest(v, T, stream=stream)

    # the batched launch captured once in a graph and replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            b.ingest(vs, stream=stream)
    stream.synchronize()

    def replay():
        with torch.cuda.stream(stream):
            g.replay()

    # the three ways take turns over several rounds (the part's clock drifts
    # as it warms, which would favour whichever ran first); medians per launch
    import numpy as np
    ways = {"batch": lambda: b.ingest(vs, stream=stream), "separate": singles, "graph": replay}
    samples = {k: [] for k in ways}
    rounds = 5
    for _ in range(rounds):
        for k, fn in ways.items():
            _, ms = _timed(fn, stream, max(2, reps // rounds), after=dumps)
            samples[k].extend(ms.tolist())
    stream.synchronize()
    batch_ms, single_ms, graph_ms = (float(np.median(samples[k])) for k in ("batch", "separate", "graph"))
    if prev_cache is None:
        os.environ.pop("XCORR_TUNE_CACHE", None)
    else:
        os.environ["XCORR_TUNE_CACHE"] = prev_cache
    res = {"workload": "batched-4arrays-2048t-4bit", "arrays": [list(a) for a in synth.BATCH_ARRAYS],
           "tiles": b.tiles, "tuned_tiles": tuned, "batch_ms": batch_ms, "graph_replay_ms": graph_ms,
           "separate_launches_ms": single_ms,
           "cmac_per_s": cmac / (batch_ms / 1e3), "frac_of_int8_peak": OPS_PER_CMAC * cmac / (batch_ms / 1e3) / 1e12
           / INT8_PEAK_TOPS}
    b.close()
    for c in cors:
        c.close()
    return res


def bench_fengine(dev, stream, reps: int) -> dict:
    """F-engine front end on 192 inputs x 4096 spectra (8-bit ADC codes at
    250 Msps: 33.55 ms of sky, 1.61 GB in, 805 MB of 4+4-bit codes out), then
    the end-to-end step ADC -> codes -> one X-engine integration."""
    import torch

    from paper_2406_19013_amd import synth
    from paper_2406_19013_amd import xcorr as X

    N, M, P, F = 192, 4096, X.FE_POINTS, X.FE_CHANS
    with torch.cuda.stream(stream):
        adc = synth.fengine_adc(device=dev, N=N, T=M)
        gains = synth.fengine_gains(device=dev, N=N, F=F)
    h = torch.from_numpy(X.xcorr_pfb_prototype()).to(dev)
    codes = torch.empty((M, F, N), dtype=torch.uint8, device=dev)
    stream.synchronize()
    fe_ms, _ = _timed(lambda: X.xcorr_fengine(adc, h, gains, codes, M, stream=stream), stream, reps)
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA, device=dev)
    vis = torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device=dev)

    def end_to_end():
        X.xcorr_fengine(adc, h, gains, codes, M, stream=stream)
        c.ingest_dump(codes, vis, stream=stream)

    e2e_ms, _ = _timed(end_to_end, stream, reps)
    stream.synchronize()
    c.close()
    span_s = M * P / 250e6
    in_bytes, out_bytes = adc.numel(), codes.numel()
    # float work per (input, spectrum): FIR 2 x 4 x 2048, complex FFT
    # 5 x 1024 x log2(1024), real-spectrum unpack and EQ about 16 x 1024
    flops = N * M * (8 * P + 5 * 1024 * 10 + 16 * 1024)
    return {"workload": "fengine-192in-4096spectra-2048pt-4tap", "ms": fe_ms,
            "hbm_gbs": (in_bytes + out_bytes) / (fe_ms / 1e3) / 1e9,
            "hbm_frac": (in_bytes + out_bytes) / (fe_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "gflops": flops / (fe_ms / 1e3) / 1e9, "fp32_vector_frac": flops / (fe_ms / 1e3) / 157.3e12,
            "rtf": span_s / (fe_ms / 1e3), "data_span_ms": span_s * 1e3,
            "end_to_end_ms": e2e_ms, "end_to_end_rtf": span_s / (e2e_ms / 1e3)}


def bench_linearity(dev) -> dict:
    """Output power against input power through the GPU F- and X-engines on
    synthetic data: 8 pairs of inputs sharing a common noise signal (rho =
    0.5), ADC noise of 16 * 10^(L/20) codes for L = -30 .. +10 dB, fixed EQ
    gains; the response is the pairs' mean cross power over channels
    100 .. 900, and the linear range is where it stays within 1 dB of
    proportionality through the 0 dB point."""
    import numpy as np
    import torch

    from paper_2406_19013_amd import synth
    from paper_2406_19013_amd import xcorr as X

    N, M, P, F = 16, 64, X.FE_POINTS, X.FE_CHANS
    S = (M + X.FE_TAPS - 1) * P
    h = torch.from_numpy(X.xcorr_pfb_prototype()).to(dev)
    gains = torch.full((N, F), synth.FE_EQ_BASE, dtype=torch.float32, device=dev)
    codes = torch.empty((M, F, N), dtype=torch.uint8, device=dev)
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA, device=dev)
    g = torch.Generator(device=dev).manual_seed(synth.seed_of(synth.BASE_SEED, 80, 0))
    common = torch.randn((N // 2, S), generator=g, device=dev)
    own = torch.randn((N, S), generator=g, device=dev)
    pairs = np.array([(2 * k + 1) * (2 * k + 2) // 2 + 2 * k for k in range(N // 2)])
    levels = np.arange(-30, 12, 2.0)
    resp = []
    for db in levels:
        sigma = synth.FE_ADC_SIGMA * 10 ** (db / 20)
        x = (common.repeat_interleave(2, 0) + own) * (sigma / np.sqrt(2))
        adc = torch.clamp(torch.round(x), -128, 127).to(torch.int8)
        X.xcorr_fengine(adc, h, gains, codes, M)
        vis, _, _ = c.ingest_dump(codes)
        resp.append(float(vis.double().cpu().numpy()[100:900][:, pairs, 0].mean()))
    c.close()
    ydb = 10 * np.log10(np.maximum(np.array(resp), 1e-12))
    dev_db = ydb - (ydb[levels == 0][0] + levels)
    i0 = int(np.where(levels == 0)[0][0])
    lo = hi = i0
    while lo > 0 and abs(dev_db[lo - 1]) <= 1.0:
        lo -= 1
    while hi + 1 < len(levels) and abs(dev_db[hi + 1]) <= 1.0:
        hi += 1
    return {"workload": "linearity-16in-64spectra-noise-pairs", "levels_db": levels.tolist(),
            "deviation_db": [round(float(d), 2) for d in dev_db],
            "linear_range_db": [float(levels[lo]), float(levels[hi])], "linear_span_db": float(levels[hi] - levels[lo])}


def bench_streaming(dev, n_blocks: int, paced_blocks: int, concurrent_blocks: int) -> dict:
    """1024-sample blocks of 4096 channels (33.55 ms of data each), a dump
    every 128 blocks: the 192-input stream device-resident (unpaced) and from
    pinned host memory (paced at the data rate), then 96-, 192- and
    512-input arrays concurrently (device-resident, unpaced)."""
    import torch

    from paper_2406_19013_amd import synth
    from paper_2406_19013_amd import xcorr as X

    F, B, every, pool_n, warm = 4096, 1024, 128, 4, 64
    span_s = B * F / BANDWIDTH_HZ
    res = {"workload": "stream-4096ch-1024t-blocks-4bit", "block_span_ms": span_s * 1e3, "dump_every": every}

    def pool_of(N, array_id):
        return [synth.stream_block(N, F, k, array_id=array_id, device=dev) for k in range(pool_n)]

    def out_of(N):
        return torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device=dev)

    # 192 inputs, device-resident, unpaced
    N = 192
    pool = pool_of(N, 1)
    c = X.Correlator(N, F, 4, X.PATH_I8_MFMA, device=dev)
    out = out_of(N)
    p = X.Pipe(c, B, every, host_blocks=False, device=dev)
    for k in range(warm):
        p.push(pool[k % pool_n], out=out)
    p.drain()
    p.reset_latency()
    t0 = time.perf_counter()
    for k in range(n_blocks):
        p.push(pool[k % pool_n], out=out)
    p.drain()
    wall = time.perf_counter() - t0
    st = p.stats()
    res["n192_device_unpaced"] = {"blocks": n_blocks, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                                  "max_ms": st["max_ms"], "rtf": n_blocks * span_s / wall, "dumps": st["dumps"],
                                  "submit_p50_ms": st["submit_p50_ms"], "submit_p99_ms": st["submit_p99_ms"]}
    # the same stream with 8 blocks per launch (the accumulators are read and
    # written once per 8 blocks)
    p.set_fuse(8)
    p.drain()
    p.reset_latency()
    t0 = time.perf_counter()
    for k in range(n_blocks):
        p.push(pool[k % pool_n], out=out)
    p.drain()
    wall = time.perf_counter() - t0
    st = p.stats()
    res["n192_device_unpaced_fuse8"] = {"blocks": n_blocks, "group_p50_ms": st["p50_ms"],
                                        "group_p99_ms": st["p99_ms"], "rtf": n_blocks * span_s / wall,
                                        "submit_p50_ms": st["submit_p50_ms"], "submit_p99_ms": st["submit_p99_ms"]}
    p.close()

    # the same stream arriving out of order (each block up to 8 places late)
    # with 1 % of the blocks lost: sequence-number reassembly in front of the
    # pipe, integrations cut at fixed sequence numbers, 8 blocks per launch
    import random
    rng = random.Random(240619013)
    arrivals = sorted((k for k in range(n_blocks) if rng.random() >= 0.01),
                      key=lambda k: k + rng.uniform(0, 9))
    c.dump(out)
    p = X.Pipe(c, B, 0, host_blocks=False, device=dev)
    p.set_fuse(8)
    r = X.Reorder(every, 8, max_missing=every // 8, seq_origin=0)
    host_s, dumps, invalid = 0.0, 0, 0

    def feed(events):
        nonlocal dumps, invalid
        for e in events:
            if e["kind"] == "block":
                p.push(e["block"], seq=e["seq"])
            elif e["kind"] == "dump":
                p.dump(out)
                dumps += 1
                invalid += not e["valid"]

    t0 = time.perf_counter()
    for k in arrivals:
        h0 = time.perf_counter()
        ev = r.push(k, pool[k % pool_n])
        host_s += time.perf_counter() - h0
        feed(ev)
    feed(r.flush(True))
    p.drain()
    wall = time.perf_counter() - t0
    st, rs = p.stats(), r.stats()
    res["n192_device_reordered_fuse8"] = {
        "blocks": n_blocks, "arrived": len(arrivals), "released": rs["released"], "missing": rs["missing"],
        "dumps": dumps, "invalid_dumps": invalid, "group_p99_ms": st["p99_ms"],
        "rtf": n_blocks * span_s / wall, "reorder_host_us_per_block": host_s / len(arrivals) * 1e6}
    p.close()
    r.close()

    # 192 inputs from pinned host memory through the ring, paced at the data rate
    host_pool = [b.cpu().pin_memory() for b in pool]
    p = X.Pipe(c, B, every, n_slots=4, host_blocks=True, device=dev)
    c.dump(out)
    for k in range(8):
        p.push(host_pool[k % pool_n], out=out)
    p.drain()
    p.reset_latency()
    t0 = time.perf_counter()
    for k in range(paced_blocks):
        due = t0 + k * span_s
        while time.perf_counter() < due:
            time.sleep(min(0.002, max(0.0, due - time.perf_counter())))
        p.push(host_pool[k % pool_n], out=out)
    p.drain()
    st = p.stats()
    res["n192_host_h2d_paced"] = {"blocks": paced_blocks, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                                  "max_ms": st["max_ms"], "submit_p50_ms": st["submit_p50_ms"],
                                  "submit_p99_ms": st["submit_p99_ms"], "submit_max_ms": st["submit_max_ms"],
                                  "clock_anchor_err_ms": st["clock_anchor_err_ms"]}
    # unpaced H2D: the rate the host link sustains
    p.reset_latency()
    t0 = time.perf_counter()
    for k in range(2 * pool_n * 4):
        p.push(host_pool[k % pool_n], out=out)
    p.drain()
    wall = time.perf_counter() - t0
    res["n192_host_h2d_unpaced_rtf"] = 2 * pool_n * 4 * span_s / wall
    p.close()
    c.close()
    del host_pool

    # three arrays at once, each on its own pipe (own streams)
    arrays = (96, 192, 512)
    cfgs = [X.make_config(n, F) for n in arrays]
    free, _ = torch.cuda.mem_get_info()
    admitted, used = X.xcorr_admit(cfgs, [B] * 3, [0] * 3, int(free * 0.8))
    pools = {192: pool}
    for n, a in zip(arrays, admitted):
        if a and n not in pools:
            pools[n] = pool_of(n, arrays.index(n))
    live = [n for n, a in zip(arrays, admitted) if a]
    cs = {n: X.Correlator(n, F, 4, X.PATH_I8_MFMA, device=dev) for n in live}
    outs = {n: out_of(n) for n in live}
    ps = {n: X.Pipe(cs[n], B, every, host_blocks=False, device=dev) for n in live}
    for k in range(16):
        for n in live:
            ps[n].push(pools[n][k % pool_n], out=outs[n])
    for n in live:
        ps[n].drain()
        ps[n].reset_latency()
    t0 = time.perf_counter()
    for k in range(concurrent_blocks):
        for n in live:
            ps[n].push(pools[n][k % pool_n], out=outs[n])
    for n in live:
        ps[n].drain()
    wall = time.perf_counter() - t0
    res["concurrent"] = {"arrays": list(arrays), "admitted": admitted, "admitted_bytes": used,
                         "blocks_per_array": concurrent_blocks, "rtf": concurrent_blocks * span_s / wall,
                         "p99_ms": {str(n): ps[n].stats()["p99_ms"] for n in live}}
    # the same three arrays with 8 blocks per launch
    for n in live:
        ps[n].set_fuse(8)
        ps[n].drain()
        ps[n].reset_latency()
    t0 = time.perf_counter()
    for k in range(concurrent_blocks):
        for n in live:
            ps[n].push(pools[n][k % pool_n], out=outs[n])
    for n in live:
        ps[n].drain()
    wall = time.perf_counter() - t0
    res["concurrent_fuse8"] = {"blocks_per_array": concurrent_blocks, "rtf": concurrent_blocks * span_s / wall,
                               "group_p99_ms": {str(n): ps[n].stats()["p99_ms"] for n in live},
                               "submit_p99_ms": {str(n): ps[n].stats()["submit_p99_ms"] for n in live}}
    for n in live:
        ps[n].close()
        cs[n].close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-channels", type=int, default=256)
    ap.add_argument("--cpu-channels-single", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-path comparison")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the precision, batched and streaming workloads")
    ap.add_argument("--stream-blocks", type=int, default=2048)
    ap.add_argument("--paced-blocks", type=int, default=512)
    ap.add_argument("--concurrent-blocks", type=int, default=128)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the X-engine shards by channel with no cross-GPU "
              "reduction, so --gpus above 1 is not run here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2406_19013_amd import synth
    from paper_2406_19013_amd import xcorr as X

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    N, F, T = N_INPUTS, N_CHANS, N_SAMPLES
    P = N * (N + 1) // 2
    cmac_per_step = P * F * T
    span_s = T / (BANDWIDTH_HZ / F)

    with torch.cuda.stream(stream):
        volts = synth.tianlai(device=dev)
    stream.synchronize()
    mf = X.Correlator(N, F, 4, X.PATH_I8_MFMA, tile=args.tile, device=dev)
    out = torch.empty((F, P, 2), dtype=torch.int32, device=dev)

    def step(c, ev=None):
        """One integration of T samples and its dump, as two calls."""
        if ev:
            ev[0].record(stream)
        c.ingest(volts, T, stream=stream)
        if ev:
            ev[1].record(stream)
        c.dump(out, stream=stream)
        if ev:
            ev[2].record(stream)

    def fused_step(c, ev=None):
        """The same integration with the dump fused into its last ingest."""
        if ev:
            ev[0].record(stream)
        c.ingest_dump(volts, out, T, stream=stream)
        if ev:
            ev[1].record(stream)

    def timed(fn, c, n_ev):
        for _ in range(args.warmup):
            fn(c)
        stream.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(n_ev)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            fn(c, evs[k])
        stream.synchronize()
        torch.cuda.synchronize()
        return evs, time.perf_counter() - t0

    # headline: the fused step (one kernel per integration of T samples)
    evs, wall = timed(fused_step, mf, 2)
    step_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    ms_per_step = wall * 1e3 / args.steps
    kernel_ms = step_ms   # the step is one correlation kernel launch
    # the same work as separate ingest and dump calls
    evs2, wall2 = timed(step, mf, 3)
    ingest_ms = np.array([e[0].elapsed_time(e[1]) for e in evs2])
    dump_ms = np.array([e[1].elapsed_time(e[2]) for e in evs2])
    # an integration over several ingests (Section 2.4: the correlator sums
    # many blocks before it dumps): the first ingest after a dump stores the
    # sums, the later ones read and add to them
    n_acc = 4

    def integration(c, ev=None):
        for k in range(n_acc):
            if ev:
                ev[k].record(stream)
            c.ingest(volts, T, stream=stream)
        if ev:
            ev[n_acc].record(stream)
        c.dump(out, stream=stream)

    single = out.clone()       # the dump of one ingest (left by the step above)
    evs3, _ = timed(integration, mf, n_acc + 1)
    integration_exact = bool(torch.equal(out, single * n_acc))
    del single
    store_ms = np.array([e[0].elapsed_time(e[1]) for e in evs3])
    add_ms = np.array([e[k].elapsed_time(e[k + 1]) for e in evs3 for k in range(1, n_acc)])

    # plain VALU path on the same data, same GPU
    plain_ms = float("nan")
    if not args.no_plain and args.plain_steps > 0:
        pl = X.Correlator(N, F, 4, X.PATH_PLAIN, device=dev)
        step(pl)
        stream.synchronize()
        pev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.plain_steps)]
        for k in range(args.plain_steps):
            step(pl, pev[k])
        stream.synchronize()
        plain_ms = float(np.mean([e[0].elapsed_time(e[2]) for e in pev]))
        pl.close()

    ingest_s = float(kernel_ms.mean()) / 1e3
    algo_ops = OPS_PER_CMAC * cmac_per_step
    achieved_tops = algo_ops / ingest_s / 1e12
    in_bytes = T * F * N
    acc_bytes = F * P * 8
    kernel = X.xcorr_autotune_kernel(mf.cfg)
    traffic = measured_traffic(kernel)
    dump_gbs = 2 * acc_bytes / (float(dump_ms.mean()) / 1e3) / 1e9

    # measured ceilings of this GPU: int8 MFMA issue on voltage bytes, and
    # the input streamed into LDS the way the correlation kernel reads it
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    chk = torch.empty(512 * cus, dtype=torch.int32, device=dev)
    ceil = {}
    for name, kind, iters in (("mfma_int8", X.CEILING_MFMA_I8, 2000), ("stream_read", X.CEILING_STREAM, 1)):
        box = {}

        def launch():
            box["ops"] = X.xcorr_ceiling(kind, volts, T, F, N, iters, chk, stream=stream)

        ms, _ = _timed(launch, stream, max(10, args.steps // 2))
        ceil[name] = box["ops"] / (ms / 1e3)
    mfma_ceiling_tops = ceil["mfma_int8"] / 1e12
    stream_ceiling_gbs = ceil["stream_read"] / 1e9

    result = {
        "metric": "complex MAC/s (int8 MFMA path), real-time factor vs plain path, p99 step latency",
        "value": cmac_per_step / (ms_per_step / 1e3),
        "unit": "CMAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "tianlai-192in-1024ch-4096t-4bit", "n_inputs": N, "n_chans": F,
                   "n_samples": T, "sample_bits": 4, "tile": mf.stats()["tile"],
                   "regions_per_chan": mf.stats()["regions_per_chan"]},
        "rtf": {"int8_mfma": span_s / (ms_per_step / 1e3), "plain": span_s / (plain_ms / 1e3),
                "data_span_ms": span_s * 1e3},
        "plain_path": {"ms_per_step": plain_ms, "cmac_per_s": cmac_per_step / (plain_ms / 1e3)},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "step_mean": float(step_ms.mean())},
        "separate_calls": {"ms_per_step": wall2 * 1e3 / args.steps, "ingest_mean_ms": float(ingest_ms.mean()),
                           "dump_mean_ms": float(dump_ms.mean())},
        "integration": {"ingests_per_dump": n_acc, "store_ingest_ms": float(store_ms.mean()),
                        "accumulate_ingest_ms": float(add_ms.mean()),
                        "accumulate_hbm_gbs": (in_bytes + 2 * acc_bytes) / (float(add_ms.mean()) / 1e3) / 1e9,
                        "dump_equals_n_times_one_ingest": integration_exact,
                        "note": "ingests of 4096 samples each; the later ones also read the running sums"},
        "dump_hbm_gbs": dump_gbs,
        "roofline": {"bound": "mfma", "achieved": achieved_tops, "peak": INT8_PEAK_TOPS,
                     "unit": "TFLOP/s", "frac": achieved_tops / INT8_PEAK_TOPS, "traffic": traffic,
                     "ops": "int8 (2 per multiply-add, 8 per complex MAC), 10^12 per s",
                     "kernel": kernel, "algorithmic_ops_per_launch": algo_ops,
                     "measured_peak": mfma_ceiling_tops, "frac_of_measured_peak": achieved_tops / mfma_ceiling_tops,
                     "hbm_algorithmic_bytes_per_launch": in_bytes + acc_bytes,
                     "hbm_gbs": (in_bytes + acc_bytes) / ingest_s / 1e9,
                     "hbm_frac": (in_bytes + acc_bytes) / ingest_s / 1e9 / HBM_PEAK_GBS,
                     "hbm_frac_of_measured_stream": (in_bytes + acc_bytes) / ingest_s / 1e9 / stream_ceiling_gbs},
        "ceilings": {"mfma_int8_tops": mfma_ceiling_tops, "mfma_int8_frac_of_nominal": mfma_ceiling_tops / INT8_PEAK_TOPS,
                     "stream_read_gbs": stream_ceiling_gbs, "stream_read_frac_of_nominal": stream_ceiling_gbs / HBM_PEAK_GBS,
                     "note": "MFMA: 8 waves per CU issuing independent 32x32x32 int8 MFMAs on voltage bytes; "
                             "stream: the input read into LDS with the correlation kernel's grid and loads"},
        "stages": {"ingest_read_gbs": in_bytes / ingest_s / 1e9, "dump_gbs": dump_gbs},
    }
    mf.close()
    _progress("headline workload done")
    if not args.no_extra:
        del volts
        result["precision8"] = bench_precision8(dev, stream, max(5, args.steps // 2))
        _progress("precision workload done")
        result["batched"] = bench_batched(dev, stream, max(5, args.steps // 2))
        _progress("batched workload done")
        result["streaming"] = bench_streaming(dev, args.stream_blocks, args.paced_blocks, args.concurrent_blocks)
        _progress("streaming workload done")
        result["fengine"] = bench_fengine(dev, stream, max(5, args.steps // 2))
        _progress("F-engine workload done")
        result["linearity"] = bench_linearity(dev)
        _progress("linearity sweep done")
        result["latency_ms"]["p99_block_stream"] = result["streaming"]["n192_device_unpaced"]["p99_ms"]
    if not args.no_cpu:
        with torch.cuda.stream(stream):
            volts = synth.tianlai(device=dev)
        stream.synchronize()
        result["cpu_baseline"] = cpu_baseline(volts, args.cpu_channels, args.cpu_channels_single)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
