"""ctypes binding of libxcorr.so (argument marshalling only).

The functions carry the C names of include/xcorr.h.  Device buffers are torch
tensors (their data_ptr is passed), streams are torch streams (their raw
hipStream_t is passed); every step of the computation runs in the library's
HIP kernels.  A missing library is an error: there is no other code path.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxcorr.so")

XCORR_OK = 0
XCORR_E_INVAL = -1
XCORR_E_NOMEM = -2
XCORR_E_OVERFLOW = -3
XCORR_E_HIP = -4
XCORR_E_DEVICE = -5

PATH_PLAIN = 0
PATH_I8_MFMA = 1
PATH_F16_MFMA = 2
LAYOUT_TFN = 0

TMAX_4BIT = 16_777_215
TMAX_8BIT = 66_572
MAX_BATCH = 16


class XcorrError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        msg = f"{where} failed: {code} ({_strerror(code)})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class Config(ctypes.Structure):
    _fields_ = [
        ("n_inputs", ctypes.c_int32),
        ("n_chans", ctypes.c_int32),
        ("sample_bits", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("max_samples_per_dump", ctypes.c_int64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("samples_integrated", ctypes.c_int64),
        ("samples_total", ctypes.c_int64),
        ("ingests", ctypes.c_int64),
        ("dumps", ctypes.c_int64),
        ("kernel_launches", ctypes.c_int64),
        ("seq_gaps", ctypes.c_uint64),
        ("seq_gaps_total", ctypes.c_uint64),
        ("tile", ctypes.c_int32),
        ("regions_per_chan", ctypes.c_int32),
        ("tile_from_cache", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class PipeStats(ctypes.Structure):
    _fields_ = [
        ("blocks", ctypes.c_int64),
        ("dumps", ctypes.c_int64),
        ("latencies", ctypes.c_int64),
        ("p50_ms", ctypes.c_double),
        ("p99_ms", ctypes.c_double),
        ("max_ms", ctypes.c_double),
        ("mean_ms", ctypes.c_double),
        ("held", ctypes.c_int64),
        ("submit_latencies", ctypes.c_int64),
        ("submit_p50_ms", ctypes.c_double),
        ("submit_p99_ms", ctypes.c_double),
        ("submit_max_ms", ctypes.c_double),
        ("clock_anchor_err_ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


EV_BLOCK, EV_GAP, EV_DUMP = 1, 2, 3


class Event(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("n_blocks", ctypes.c_int32),
        ("n_missing", ctypes.c_int32),
        ("valid", ctypes.c_int32),
        ("seq", ctypes.c_uint64),
        ("integration", ctypes.c_int64),
        ("block", ctypes.c_void_p),
    ]


class ReorderStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("received", "released", "missing", "late", "duplicate",
                                              "before_origin", "held", "integrations",
                                              "invalid_integrations", "empty_integrations")] + [
        ("next_seq", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lock = threading.Lock()
_lib = None


def load(path: str | None = None):
    """Open libxcorr.so and declare its entry points (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise FileNotFoundError(
                f"{p} is not built; run paper_2406_19013_amd.build.build() (hipcc, gfx950)")
        lib = ctypes.CDLL(p)
        vp, i64, u64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
        cfgp = ctypes.POINTER(Config)
        sig = {
            "xcorr_query": [cfgp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(i64)],
            "xcorr_init": [cfgp, vp, sz, ctypes.POINTER(vp)],
            "xcorr_ingest": [vp, vp, i64, u64, vp],
            "xcorr_dump": [vp, vp, ctypes.POINTER(i64), ctypes.POINTER(u64), vp],
            "xcorr_stats": [vp, ctypes.POINTER(Stats)],
            "xcorr_destroy": [vp],
            "xcorr_batch_query": [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(sz)],
            "xcorr_batch_init": [ctypes.POINTER(vp), ctypes.c_int, vp, sz, ctypes.POINTER(vp)],
            "xcorr_batch_ingest": [vp, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(u64), vp],
            "xcorr_batch_tiles": [vp, ctypes.POINTER(ctypes.c_int32)],
            "xcorr_batch_destroy": [vp],
            "xcorr_autotune_query": [cfgp, ctypes.POINTER(sz)],
            "xcorr_autotune": [cfgp, vp, sz, vp, ctypes.POINTER(ctypes.c_int32)],
            "xcorr_autotune_batch": [cfgp, vp, sz, vp, ctypes.POINTER(ctypes.c_int32)],
            "xcorr_autotune_kernel": [cfgp, ctypes.c_int32, ctypes.c_char_p, sz],
            "xcorr_plan_tile": [cfgp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32)],
            "xcorr_correlate_static": [cfgp, vp, i64, vp, ctypes.POINTER(i64), vp],
            "xcorr_cns_plan_make": [u64, u64, u64, i64, i64, i64, vp],
            "xcorr_cns_is_on": [vp, u64],
            "xcorr_cns_integration": [vp, i64],
            "xcorr_stokes": [vp, ctypes.c_int32, ctypes.c_int32, vp, vp],
            "xcorr_pfb_prototype": [ctypes.c_int32, ctypes.c_int32, vp],
            "xcorr_fengine": [vp, i64, ctypes.c_int32, vp, vp, i64, vp, vp],
            "xcorr_pfb_spectra": [vp, i64, ctypes.c_int32, vp, i64, vp, vp],
            "xcorr_ceiling": [ctypes.c_int32, vp, i64, ctypes.c_int32, ctypes.c_int32, i64, vp, i64,
                              ctypes.POINTER(ctypes.c_double), vp],
            "xcorr_pipe_query": [vp, ctypes.c_int, i64, ctypes.POINTER(sz)],
            "xcorr_pipe_init": [vp, ctypes.c_int, i64, i64, vp, sz, vp, vp, ctypes.POINTER(vp)],
            "xcorr_pipe_push": [vp, vp, ctypes.c_int, u64, vp, ctypes.POINTER(ctypes.c_int)],
            "xcorr_pipe_drain": [vp],
            "xcorr_pipe_stats": [vp, ctypes.POINTER(PipeStats)],
            "xcorr_pipe_reset_latency": [vp],
            "xcorr_pipe_set_fuse": [vp, ctypes.c_int],
            "xcorr_ingest_blocks": [vp, ctypes.POINTER(vp), ctypes.c_int, i64, u64, vp],
            "xcorr_ingest_dump": [vp, vp, i64, u64, vp, ctypes.POINTER(i64), ctypes.POINTER(u64), vp],
            "xcorr_pipe_destroy": [vp],
            "xcorr_pipe_dump": [vp, vp, ctypes.POINTER(i64), ctypes.POINTER(u64)],
            "xcorr_reorder_init": [i64, ctypes.c_int32, ctypes.c_int32, u64, ctypes.POINTER(vp)],
            "xcorr_reorder_push": [vp, u64, vp, ctypes.POINTER(Event), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)],
            "xcorr_reorder_flush": [vp, ctypes.c_int32, ctypes.POINTER(Event), ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32)],
            "xcorr_reorder_stats": [vp, ctypes.POINTER(ReorderStats)],
            "xcorr_reorder_destroy": [vp],
            "xcorr_admit": [cfgp, ctypes.c_int, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int32), sz,
                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(sz)],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.xcorr_reorder_max_events.argtypes = [ctypes.c_int32]
        lib.xcorr_reorder_max_events.restype = ctypes.c_int32
        lib.xcorr_strerror.argtypes = [ctypes.c_int]
        lib.xcorr_strerror.restype = ctypes.c_char_p
        lib.xcorr_last_error.argtypes = []
        lib.xcorr_last_error.restype = ctypes.c_char_p
        if path is None:
            _lib = lib
        return lib


def _strerror(code: int) -> str:
    try:
        return load().xcorr_strerror(code).decode()
    except Exception:
        return "?"


def _check(rc: int, where: str):
    if rc != XCORR_OK:
        raise XcorrError(rc, where, load().xcorr_last_error().decode())


def make_config(n_inputs: int, n_chans: int, sample_bits: int = 4, path: int = PATH_I8_MFMA,
                tile: int = 0, max_samples_per_dump: int = 0, layout: int = LAYOUT_TFN) -> Config:
    return Config(n_inputs, n_chans, sample_bits, path, layout, tile, max_samples_per_dump)


def xcorr_query(cfg: Config):
    """(workspace_bytes, out_bytes, t_max) for a config; raises XcorrError."""
    ws, out, tmax = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int64()
    _check(load().xcorr_query(ctypes.byref(cfg), ctypes.byref(ws), ctypes.byref(out), ctypes.byref(tmax)),
           "xcorr_query")
    return ws.value, out.value, tmax.value


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def xcorr_init(cfg: Config, workspace, ws_bytes: int | None = None) -> ctypes.c_void_p:
    """Create a context borrowing `workspace` (a device tensor)."""
    ctx = ctypes.c_void_p()
    nbytes = ws_bytes if ws_bytes is not None else workspace.numel() * workspace.element_size()
    _check(load().xcorr_init(ctypes.byref(cfg), ctypes.c_void_p(workspace.data_ptr()), nbytes,
                             ctypes.byref(ctx)), "xcorr_init")
    return ctx


def xcorr_ingest(ctx, volts, n_samples: int, seq: int = 0, stream=None):
    _check(load().xcorr_ingest(ctx, ctypes.c_void_p(volts.data_ptr()), int(n_samples), int(seq),
                               _stream_handle(stream)), "xcorr_ingest")


def xcorr_ingest_blocks(ctx, blocks, block_samples: int, first_seq: int = 0, stream=None):
    """blocks: device tensors of block_samples samples each."""
    arr = (ctypes.c_void_p * len(blocks))(*[b.data_ptr() for b in blocks])
    _check(load().xcorr_ingest_blocks(ctx, arr, len(blocks), int(block_samples), int(first_seq),
                                      _stream_handle(stream)), "xcorr_ingest_blocks")


def xcorr_ingest_dump(ctx, volts, n_samples: int, seq: int, out, stream=None):
    """Last ingest of an integration plus its dump; returns (n_integrated, n_gaps)."""
    n, g = ctypes.c_int64(), ctypes.c_uint64()
    _check(load().xcorr_ingest_dump(ctx, ctypes.c_void_p(volts.data_ptr()), int(n_samples), int(seq),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.byref(n), ctypes.byref(g),
                                    _stream_handle(stream)), "xcorr_ingest_dump")
    return n.value, g.value


def xcorr_dump(ctx, out, stream=None):
    """Dump into the device tensor `out`; returns (n_integrated, n_gaps)."""
    n, g = ctypes.c_int64(), ctypes.c_uint64()
    _check(load().xcorr_dump(ctx, ctypes.c_void_p(out.data_ptr()), ctypes.byref(n), ctypes.byref(g),
                             _stream_handle(stream)), "xcorr_dump")
    return n.value, g.value


def xcorr_stats(ctx) -> dict:
    st = Stats()
    _check(load().xcorr_stats(ctx, ctypes.byref(st)), "xcorr_stats")
    return st.as_dict()


def xcorr_destroy(ctx):
    _check(load().xcorr_destroy(ctx), "xcorr_destroy")


def _ctx_array(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))()
    for k, c in enumerate(ctxs):
        arr[k] = c.value if isinstance(c, ctypes.c_void_p) else c
    return arr


def xcorr_batch_query(ctxs) -> int:
    ws = ctypes.c_size_t()
    _check(load().xcorr_batch_query(_ctx_array(ctxs), len(ctxs), ctypes.byref(ws)), "xcorr_batch_query")
    return ws.value


def xcorr_batch_init(ctxs, workspace, ws_bytes: int | None = None) -> ctypes.c_void_p:
    b = ctypes.c_void_p()
    nbytes = ws_bytes if ws_bytes is not None else workspace.numel() * workspace.element_size()
    _check(load().xcorr_batch_init(_ctx_array(ctxs), len(ctxs), ctypes.c_void_p(workspace.data_ptr()),
                                   nbytes, ctypes.byref(b)), "xcorr_batch_init")
    return b


def xcorr_batch_ingest(batch, volts, n_samples, seqs=None, stream=None):
    """volts: one device tensor (or None for an array left out) per array."""
    n = len(n_samples)
    vp = (ctypes.c_void_p * n)(*[(v.data_ptr() if v is not None else None) for v in volts])
    ns = (ctypes.c_int64 * n)(*[int(x) for x in n_samples])
    sq = (ctypes.c_uint64 * n)(*[int(x) for x in seqs]) if seqs is not None else None
    _check(load().xcorr_batch_ingest(batch, vp, ns, sq, _stream_handle(stream)), "xcorr_batch_ingest")


def xcorr_batch_tiles(batch, n: int) -> list:
    t = (ctypes.c_int32 * n)()
    _check(load().xcorr_batch_tiles(batch, t), "xcorr_batch_tiles")
    return list(t)


def xcorr_batch_destroy(batch):
    _check(load().xcorr_batch_destroy(batch), "xcorr_batch_destroy")


def xcorr_autotune_query(cfg: Config) -> int:
    sz = ctypes.c_size_t()
    _check(load().xcorr_autotune_query(ctypes.byref(cfg), ctypes.byref(sz)), "xcorr_autotune_query")
    return sz.value


def xcorr_autotune(cfg: Config, scratch, stream=None) -> int:
    best = ctypes.c_int32()
    _check(load().xcorr_autotune(ctypes.byref(cfg), ctypes.c_void_p(scratch.data_ptr()),
                                 scratch.numel() * scratch.element_size(), _stream_handle(stream),
                                 ctypes.byref(best)), "xcorr_autotune")
    return best.value


def xcorr_autotune_batch(cfg: Config, scratch, stream=None) -> int:
    best = ctypes.c_int32()
    _check(load().xcorr_autotune_batch(ctypes.byref(cfg), ctypes.c_void_p(scratch.data_ptr()),
                                       scratch.numel() * scratch.element_size(), _stream_handle(stream),
                                       ctypes.byref(best)), "xcorr_autotune_batch")
    return best.value


def xcorr_autotune_kernel(cfg: Config, batch: bool = False) -> str:
    """Name of the kernel the tuner times for this config (the one it runs)."""
    buf = ctypes.create_string_buffer(96)
    _check(load().xcorr_autotune_kernel(ctypes.byref(cfg), int(batch), buf, len(buf)), "xcorr_autotune_kernel")
    return buf.value.decode()


def xcorr_plan_tile(cfg: Config, batch: bool = False):
    """(tile, from_cache) that xcorr_init (or xcorr_batch_init) would use."""
    t, c = ctypes.c_int32(), ctypes.c_int32()
    _check(load().xcorr_plan_tile(ctypes.byref(cfg), int(batch), ctypes.byref(t), ctypes.byref(c)),
           "xcorr_plan_tile")
    return t.value, bool(c.value)


def autotune(n_inputs: int, n_chans: int, sample_bits: int = 4, path: int = PATH_I8_MFMA, device="cuda",
             stream=None, batch: bool = False) -> int:
    """Run the autotuner (batch: on the batched kernel) with a torch-allocated
    scratch; returns the best tile."""
    import torch
    cfg = make_config(n_inputs, n_chans, sample_bits, path)
    scratch = torch.empty(xcorr_autotune_query(cfg), dtype=torch.uint8, device=device)
    return (xcorr_autotune_batch if batch else xcorr_autotune)(cfg, scratch, stream)


def xcorr_pipe_query(ctx, n_slots: int, block_samples: int) -> int:
    rb = ctypes.c_size_t()
    _check(load().xcorr_pipe_query(ctx, n_slots, block_samples, ctypes.byref(rb)), "xcorr_pipe_query")
    return rb.value


def xcorr_pipe_init(ctx, n_slots, block_samples, dump_every, ring, copy_stream, compute_stream):
    p = ctypes.c_void_p()
    rp = ctypes.c_void_p(ring.data_ptr()) if ring is not None else None
    rb = ring.numel() * ring.element_size() if ring is not None else 0
    _check(load().xcorr_pipe_init(ctx, n_slots, block_samples, dump_every, rp, rb, _stream_handle(copy_stream),
                                  _stream_handle(compute_stream), ctypes.byref(p)), "xcorr_pipe_init")
    return p


def xcorr_pipe_push(pipe, block, on_host: bool, seq: int, out=None) -> bool:
    d = ctypes.c_int()
    _check(load().xcorr_pipe_push(pipe, ctypes.c_void_p(block.data_ptr()), int(on_host), int(seq),
                                  ctypes.c_void_p(out.data_ptr()) if out is not None else None,
                                  ctypes.byref(d)), "xcorr_pipe_push")
    return bool(d.value)


def xcorr_pipe_drain(pipe):
    _check(load().xcorr_pipe_drain(pipe), "xcorr_pipe_drain")


def xcorr_pipe_stats(pipe) -> dict:
    st = PipeStats()
    _check(load().xcorr_pipe_stats(pipe, ctypes.byref(st)), "xcorr_pipe_stats")
    return st.as_dict()


def xcorr_pipe_reset_latency(pipe):
    _check(load().xcorr_pipe_reset_latency(pipe), "xcorr_pipe_reset_latency")


def xcorr_pipe_set_fuse(pipe, fuse: int):
    _check(load().xcorr_pipe_set_fuse(pipe, int(fuse)), "xcorr_pipe_set_fuse")


def xcorr_pipe_destroy(pipe):
    _check(load().xcorr_pipe_destroy(pipe), "xcorr_pipe_destroy")


def xcorr_pipe_dump(pipe, out):
    """End the integration now: (samples integrated, sequence gaps)."""
    n, g = ctypes.c_int64(), ctypes.c_uint64()
    _check(load().xcorr_pipe_dump(pipe, ctypes.c_void_p(out.data_ptr()), ctypes.byref(n), ctypes.byref(g)),
           "xcorr_pipe_dump")
    return n.value, g.value


def xcorr_reorder_max_events(window: int) -> int:
    return int(load().xcorr_reorder_max_events(int(window)))


def xcorr_reorder_init(blocks_per_dump: int, window: int, max_missing: int, seq_origin: int):
    r = ctypes.c_void_p()
    _check(load().xcorr_reorder_init(int(blocks_per_dump), int(window), int(max_missing), int(seq_origin),
                                     ctypes.byref(r)), "xcorr_reorder_init")
    return r


def xcorr_reorder_push(r, seq: int, handle: int, events, max_events: int) -> int:
    n = ctypes.c_int32()
    _check(load().xcorr_reorder_push(r, int(seq), ctypes.c_void_p(handle), events, int(max_events),
                                     ctypes.byref(n)), "xcorr_reorder_push")
    return n.value


def xcorr_reorder_flush(r, to_boundary: bool, events, max_events: int) -> int:
    n = ctypes.c_int32()
    _check(load().xcorr_reorder_flush(r, int(to_boundary), events, int(max_events), ctypes.byref(n)),
           "xcorr_reorder_flush")
    return n.value


def xcorr_reorder_stats(r) -> dict:
    st = ReorderStats()
    _check(load().xcorr_reorder_stats(r, ctypes.byref(st)), "xcorr_reorder_stats")
    return st.as_dict()


def xcorr_reorder_destroy(r):
    _check(load().xcorr_reorder_destroy(r), "xcorr_reorder_destroy")


def xcorr_admit(cfgs, block_samples, n_slots, budget_bytes: int):
    """(admitted flags, bytes used) for configs walked in order against a budget."""
    n = len(cfgs)
    arr = (Config * n)(*cfgs)
    bs = (ctypes.c_int64 * n)(*[int(x) for x in block_samples])
    sl = (ctypes.c_int32 * n)(*[int(x) for x in n_slots])
    adm = (ctypes.c_int32 * n)()
    used = ctypes.c_size_t()
    _check(load().xcorr_admit(arr, n, bs, sl, int(budget_bytes), adm, ctypes.byref(used)), "xcorr_admit")
    return [bool(a) for a in adm], used.value


STATIC_SCRATCH_BYTES = 16 << 20


def xcorr_correlate_static(cfg: Config, volts, n_samples: int, out, stream=None) -> int:
    """One integration into `out` without any allocation (running sums in the
    library's static device array); returns the samples integrated."""
    n = ctypes.c_int64()
    _check(load().xcorr_correlate_static(ctypes.byref(cfg), ctypes.c_void_p(volts.data_ptr()), int(n_samples),
                                         ctypes.c_void_p(out.data_ptr()), ctypes.byref(n), _stream_handle(stream)),
           "xcorr_correlate_static")
    return n.value


def xcorr_stokes(vis, n_inputs: int, out=None, stream=None):
    """Full-Stokes visibilities int64 [F][Nf (Nf + 1) / 2][4][2] from a dump
    vis int32 [F][P][2] of n_inputs = 2 Nf inputs."""
    import torch
    F = vis.shape[0]
    nf = n_inputs // 2
    if out is None:
        out = torch.empty((F, nf * (nf + 1) // 2, 4, 2), dtype=torch.int64, device=vis.device)
    _check(load().xcorr_stokes(ctypes.c_void_p(vis.data_ptr()), int(n_inputs), int(F), ctypes.c_void_p(out.data_ptr()),
                               _stream_handle(stream)), "xcorr_stokes")
    return out


class CnsPlan(ctypes.Structure):
    _fields_ = [
        ("seq_origin", ctypes.c_uint64),
        ("blocks_per_dump", ctypes.c_int64),
        ("period_dumps", ctypes.c_int64),
        ("on_blocks", ctypes.c_int64),
        ("first_on", ctypes.c_uint64),
        ("first_integration", ctypes.c_int64),
        ("period_blocks", ctypes.c_int64),
    ]

    def is_on(self, seq: int) -> bool:
        return bool(load().xcorr_cns_is_on(ctypes.byref(self), int(seq)))

    def integration(self, j: int) -> bool:
        return bool(load().xcorr_cns_integration(ctypes.byref(self), int(j)))


def xcorr_cns_plan_make(now: int, lead: int, seq_origin: int, blocks_per_dump: int, period_dumps: int,
                        on_blocks: int) -> CnsPlan:
    p = CnsPlan()
    _check(load().xcorr_cns_plan_make(int(now), int(lead), int(seq_origin), int(blocks_per_dump),
                                      int(period_dumps), int(on_blocks), ctypes.byref(p)), "xcorr_cns_plan_make")
    return p


FE_POINTS, FE_CHANS, FE_TAPS = 2048, 1024, 4


def xcorr_pfb_prototype(n_points: int = FE_POINTS, taps: int = FE_TAPS):
    """The library's prototype filter (float32 numpy array, host)."""
    import numpy as np
    h = np.empty(n_points * taps, dtype=np.float32)
    _check(load().xcorr_pfb_prototype(int(n_points), int(taps), ctypes.c_void_p(h.ctypes.data)),
           "xcorr_pfb_prototype")
    return h


def fe_n_spectra(n_samples: int) -> int:
    return max(0, n_samples // FE_POINTS - FE_TAPS + 1)


def xcorr_fengine(adc, coeffs, gains, out, n_spectra: int | None = None, stream=None):
    """ADC codes adc [N][S] int8 -> packed 4+4-bit codes out [n_spectra][1024][N]."""
    N, S = adc.shape
    n_spectra = fe_n_spectra(S) if n_spectra is None else n_spectra
    _check(load().xcorr_fengine(ctypes.c_void_p(adc.data_ptr()), int(S), int(N), ctypes.c_void_p(coeffs.data_ptr()),
                                ctypes.c_void_p(gains.data_ptr()), int(n_spectra), ctypes.c_void_p(out.data_ptr()),
                                _stream_handle(stream)), "xcorr_fengine")


def xcorr_pfb_spectra(adc, coeffs, out, n_spectra: int | None = None, stream=None):
    """ADC codes adc [N][S] int8 -> complex spectra out [N][n_spectra][1024][2] float32."""
    N, S = adc.shape
    n_spectra = fe_n_spectra(S) if n_spectra is None else n_spectra
    _check(load().xcorr_pfb_spectra(ctypes.c_void_p(adc.data_ptr()), int(S), int(N),
                                    ctypes.c_void_p(coeffs.data_ptr()), int(n_spectra),
                                    ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), "xcorr_pfb_spectra")


CEILING_MFMA_I8, CEILING_STREAM = 0, 1


def xcorr_ceiling(kind: int, volts, n_samples: int, n_chans: int, n_inputs: int, iters: int, out,
                  stream=None) -> float:
    """Enqueue a hardware-ceiling kernel; returns the ops (MFMA) or bytes
    (stream) it performs."""
    ops = ctypes.c_double()
    _check(load().xcorr_ceiling(int(kind), ctypes.c_void_p(volts.data_ptr()), int(n_samples), int(n_chans),
                                int(n_inputs), int(iters), ctypes.c_void_p(out.data_ptr()), int(out.numel()),
                                ctypes.byref(ops), _stream_handle(stream)), "xcorr_ceiling")
    return ops.value


def xcorr_strerror(code: int) -> str:
    return load().xcorr_strerror(code).decode()


def xcorr_last_error() -> str:
    return load().xcorr_last_error().decode()


class Correlator:
    """One context plus its device workspace (allocated with torch).

    ``ingest(volts)`` takes a device tensor [T][F][N] (uint8, 4+4-bit) or
    [T][F][N][2] (int8, 8+8-bit); ``dump()`` returns a new device tensor
    [F][P][2] (int32, or float32 for the FP16 path).
    """

    def __init__(self, n_inputs: int, n_chans: int, sample_bits: int = 4, path: int = PATH_I8_MFMA,
                 tile: int = 0, max_samples_per_dump: int = 0, device="cuda"):
        import torch
        self.cfg = make_config(n_inputs, n_chans, sample_bits, path, tile, max_samples_per_dump)
        self.ws_bytes, self.out_bytes, self.t_max = xcorr_query(self.cfg)
        self.device = torch.device(device)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.ctx = xcorr_init(self.cfg, self.workspace, self.ws_bytes)
        self.n_inputs, self.n_chans, self.sample_bits, self.path = n_inputs, n_chans, sample_bits, path
        self.n_pairs = n_inputs * (n_inputs + 1) // 2
        self._seq = 0

    def ingest(self, volts, n_samples: int | None = None, seq: int | None = None, stream=None):
        n = volts.shape[0] if n_samples is None else n_samples
        s = self._seq if seq is None else seq
        xcorr_ingest(self.ctx, volts, n, s, stream)
        self._seq = s + 1

    def ingest_dump(self, volts, out=None, n_samples: int | None = None, seq: int | None = None, stream=None):
        """Ingest the last block of an integration and dump it: (out, n, gaps)."""
        import torch
        if out is None:
            dt = torch.float32 if self.path == PATH_F16_MFMA else torch.int32
            out = torch.empty((self.n_chans, self.n_pairs, 2), dtype=dt, device=self.device)
        n = volts.shape[0] if n_samples is None else n_samples
        s = self._seq if seq is None else seq
        n_int, gaps = xcorr_ingest_dump(self.ctx, volts, n, s, out, stream)
        self._seq = s + 1
        return out, n_int, gaps

    def ingest_blocks(self, blocks, seq: int | None = None, stream=None):
        """Several device blocks of equal length as consecutive samples."""
        s = self._seq if seq is None else seq
        xcorr_ingest_blocks(self.ctx, blocks, blocks[0].shape[0], s, stream)
        self._seq = s + len(blocks)

    def dump(self, out=None, stream=None):
        import torch
        if out is None:
            dt = torch.float32 if self.path == PATH_F16_MFMA else torch.int32
            out = torch.empty((self.n_chans, self.n_pairs, 2), dtype=dt, device=self.device)
        n, gaps = xcorr_dump(self.ctx, out, stream)
        return out, n, gaps

    def stats(self) -> dict:
        return xcorr_stats(self.ctx)

    def close(self):
        if self.ctx:
            xcorr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batched persistent launch over several Correlators (4+4-bit int8 MFMA).

    ``ingest([volts_0, volts_1, ...])`` correlates every array in one kernel;
    dumps stay per Correlator.  The Correlators must outlive the Batch.
    """

    def __init__(self, correlators, device="cuda"):
        import torch
        self.members = list(correlators)
        ctxs = [c.ctx for c in self.members]
        self.ws_bytes = xcorr_batch_query(ctxs)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.batch = xcorr_batch_init(ctxs, self.workspace, self.ws_bytes)
        self.tiles = xcorr_batch_tiles(self.batch, len(ctxs))

    def ingest(self, volts, n_samples=None, seqs=None, stream=None):
        ns = [0 if v is None else v.shape[0] for v in volts] if n_samples is None else list(n_samples)
        if seqs is None:
            seqs = [c._seq for c in self.members]
        xcorr_batch_ingest(self.batch, volts, ns, seqs, stream)
        for c, n, s in zip(self.members, ns, seqs):
            if n > 0:
                c._seq = s + 1

    def close(self):
        if self.batch:
            xcorr_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pipe:
    """Streaming loop around one Correlator: a ring of device slots for host
    blocks, a copy stream and a compute stream (torch streams, default
    priority), a dump every ``dump_every`` blocks, per-block latency.

    The pipe keeps a reference to every pushed block (and dump buffer) until
    the compute stream has passed the launch that reads (writes) it, so a
    caller may drop its own reference right after ``push``: a held device
    block's ingest is enqueued only on a later call, and a pinned host block
    is copied by the library outside torch's allocators, so neither torch's
    stream recording nor its host cache would keep that memory alive."""

    def __init__(self, correlator, block_samples: int, dump_every: int, n_slots: int = 4,
                 host_blocks: bool = True, device="cuda"):
        import collections

        import torch
        self.cor = correlator
        self.block_samples = block_samples
        self.copy_stream = torch.cuda.Stream(device=device)
        self.compute_stream = torch.cuda.Stream(device=device)
        self.ring = None
        if host_blocks:
            nbytes = xcorr_pipe_query(correlator.ctx, n_slots, block_samples)
            self.ring = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.pipe = xcorr_pipe_init(correlator.ctx, n_slots, block_samples, dump_every, self.ring,
                                    self.copy_stream, self.compute_stream)
        self.seq = 0
        self._unqueued = collections.deque()   # pushed tensors whose launch is not enqueued yet
        self._inflight = collections.deque()   # (event after their launch, tensors)

    def _settle(self):
        """After a library call: the tensors of every push except the newest
        `held` ones now have their launch on the compute stream; tag them with
        an event there and let go of those whose event has passed."""
        import torch
        held = int(self.stats()["held"]) if self.pipe else 0
        ready = []
        while len(self._unqueued) > held:
            ready.append(self._unqueued.popleft())
        if ready:
            ev = torch.cuda.Event()
            ev.record(self.compute_stream)
            self._inflight.append((ev, ready))
        while self._inflight and self._inflight[0][0].query():
            self._inflight.popleft()

    def push(self, block, out=None, seq: int | None = None) -> bool:
        """Submit one block (pinned host tensor or device tensor).  The pipe's
        streams are ordered after torch's current stream (where the block, the
        output and the ring were produced)."""
        import torch
        cur = torch.cuda.current_stream()
        self.copy_stream.wait_stream(cur)
        self.compute_stream.wait_stream(cur)
        if block.is_cuda:
            block.record_stream(self.compute_stream)
        if out is not None:
            out.record_stream(self.compute_stream)
        s = self.seq if seq is None else seq
        dumped = xcorr_pipe_push(self.pipe, block, not block.is_cuda, s, out)
        self.seq = s + 1
        self._unqueued.append((block, out))
        self._settle()
        return dumped

    def set_fuse(self, fuse: int):
        xcorr_pipe_set_fuse(self.pipe, fuse)
        self._settle()

    def dump(self, out):
        """End the integration now (dump_every = 0 pipes dump only here):
        (samples integrated, sequence gaps)."""
        import torch
        self.compute_stream.wait_stream(torch.cuda.current_stream())
        out.record_stream(self.compute_stream)
        r = xcorr_pipe_dump(self.pipe, out)
        self._unqueued.append((out,))
        self._settle()
        return r

    def drain(self):
        xcorr_pipe_drain(self.pipe)
        self._settle()
        self._inflight.clear()   # the drain waited for every launch

    def stats(self) -> dict:
        return xcorr_pipe_stats(self.pipe)

    def reset_latency(self):
        xcorr_pipe_reset_latency(self.pipe)
        self._settle()
        self._inflight.clear()

    def close(self):
        """Ingest what is held, wait for the streams, destroy the pipe."""
        if self.pipe:
            try:
                xcorr_pipe_drain(self.pipe)
            finally:
                xcorr_pipe_destroy(self.pipe)
                self.pipe = None
                self._unqueued.clear()
                self._inflight.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Reorder:
    """Block reassembly by sequence number (pure host): push arriving blocks
    in any order, get back what each arrival settles, in sequence order, as
    dicts {"kind": "block" | "gap" | "dump", "seq", "integration", ...}; a
    block event carries the object that was pushed."""

    _KIND = {EV_BLOCK: "block", EV_GAP: "gap", EV_DUMP: "dump"}

    def __init__(self, blocks_per_dump: int, window: int, max_missing: int = 0, seq_origin: int = 0):
        self.r = xcorr_reorder_init(blocks_per_dump, window, max_missing, seq_origin)
        self.max_events = xcorr_reorder_max_events(window)
        self._events = (Event * self.max_events)()
        self._held = {}
        self._next_handle = 1
        self._dropped = 0

    def _convert(self, n: int) -> list:
        out = []
        for e in self._events[:n]:
            d = {"kind": self._KIND[e.kind], "seq": e.seq, "integration": e.integration}
            if e.kind == EV_BLOCK:
                d["block"] = self._held.pop(e.block)
            elif e.kind == EV_GAP:
                d["n"] = e.n_blocks
            else:
                d.update(n_blocks=e.n_blocks, n_missing=e.n_missing, valid=bool(e.valid))
            out.append(d)
        return out

    def push(self, seq: int, block=None) -> list:
        h = self._next_handle
        self._next_handle += 1
        self._held[h] = block
        try:
            n = xcorr_reorder_push(self.r, seq, h, self._events, self.max_events)
        except XcorrError:
            self._held.pop(h, None)
            raise
        ev = self._convert(n)
        # a dropped block (late, duplicate, before the origin) is not held
        st = self.stats()
        dropped = st["late"] + st["duplicate"] + st["before_origin"]
        if dropped > self._dropped:
            self._dropped = dropped
            self._held.pop(h, None)
        return ev

    def flush(self, to_boundary: bool = True) -> list:
        return self._convert(xcorr_reorder_flush(self.r, to_boundary, self._events, self.max_events))

    def stats(self) -> dict:
        return xcorr_reorder_stats(self.r)

    def close(self):
        if self.r:
            xcorr_reorder_destroy(self.r)
            self.r = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
