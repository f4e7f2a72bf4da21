"""The C-ABI library on the CPU: it loads, exports what include/xcorr.h
declares, and its pure-host calls validate and size correctly.  No device
call is made here."""
import ctypes
import os
import re

import pytest

from paper_2406_19013_amd import xcorr as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(xcorr_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return X.load()


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/ but not exported"


def test_query_sizes_follow_eq1(lib):
    # Eq. 1 of Section 2.2: N(N+1)/2 * f_ch * 2 * f_b bytes per integration
    for N, F in ((192, 1024), (16, 8), (512, 128), (1, 1), (97, 3)):
        ws, out, tmax = X.xcorr_query(X.make_config(N, F, 4, X.PATH_I8_MFMA))
        assert out == N * (N + 1) // 2 * F * 2 * 4
        assert ws >= out and ws % 256 == 0
        assert tmax == X.TMAX_4BIT
    assert X.xcorr_query(X.make_config(192, 1024))[1] == 151_781_376
    _, _, t8 = X.xcorr_query(X.make_config(192, 512, 8, X.PATH_PLAIN))
    assert t8 == X.TMAX_8BIT


def test_tmax_constants_are_the_int32_bounds():
    # 4-bit: worst sample contributes 2*8*8 = 128; 8-bit: 2*127^2 (-128 excluded)
    assert X.TMAX_4BIT == (2 ** 31 - 1) // 128
    assert X.TMAX_8BIT == (2 ** 31 - 1) // (2 * 127 * 127)


@pytest.mark.parametrize("kw,code", [
    (dict(n_inputs=0, n_chans=4), X.XCORR_E_INVAL),
    (dict(n_inputs=4, n_chans=0), X.XCORR_E_INVAL),
    (dict(n_inputs=4, n_chans=4, sample_bits=5), X.XCORR_E_INVAL),
    (dict(n_inputs=4, n_chans=4, path=7), X.XCORR_E_INVAL),
    (dict(n_inputs=4, n_chans=4, layout=3), X.XCORR_E_INVAL),
    (dict(n_inputs=4, n_chans=4, sample_bits=4, path=X.PATH_F16_MFMA), X.XCORR_E_INVAL),
    (dict(n_inputs=192, n_chans=4, tile=5), X.XCORR_E_INVAL),
    (dict(n_inputs=300, n_chans=4, tile=6), X.XCORR_E_INVAL),
    (dict(n_inputs=4, n_chans=4, max_samples_per_dump=X.TMAX_4BIT + 1), X.XCORR_E_OVERFLOW),
    (dict(n_inputs=4, n_chans=4, max_samples_per_dump=-1), X.XCORR_E_INVAL),
])
def test_query_rejects(kw, code):
    with pytest.raises(X.XcorrError) as ei:
        X.xcorr_query(X.make_config(**kw))
    assert ei.value.code == code


def test_init_rejects_small_or_missing_workspace_before_any_device_call(lib):
    cfg = X.make_config(16, 8)
    ctx = ctypes.c_void_p()
    assert lib.xcorr_init(ctypes.byref(cfg), None, 1 << 20, ctypes.byref(ctx)) == X.XCORR_E_NOMEM
    assert lib.xcorr_init(ctypes.byref(cfg), ctypes.c_void_p(256), 16, ctypes.byref(ctx)) == X.XCORR_E_NOMEM
    assert lib.xcorr_init(ctypes.byref(cfg), ctypes.c_void_p(258), 1 << 20, ctypes.byref(ctx)) == X.XCORR_E_INVAL
    assert not ctx.value


def test_null_context_is_rejected(lib):
    assert lib.xcorr_ingest(None, ctypes.c_void_p(256), 4, 0, None) == X.XCORR_E_INVAL
    assert lib.xcorr_dump(None, ctypes.c_void_p(256), None, None, None) == X.XCORR_E_INVAL
    assert lib.xcorr_destroy(None) == X.XCORR_E_INVAL
    assert lib.xcorr_stats(None, None) == X.XCORR_E_INVAL


def test_batch_calls_reject_bad_arguments_on_the_host(lib):
    ws = ctypes.c_size_t()
    assert lib.xcorr_batch_query(None, 1, ctypes.byref(ws)) == X.XCORR_E_INVAL
    nulls = (ctypes.c_void_p * 17)()
    for n in (0, 17):
        assert lib.xcorr_batch_query(nulls, n, ctypes.byref(ws)) == X.XCORR_E_INVAL
    assert lib.xcorr_batch_query(nulls, 2, ctypes.byref(ws)) == X.XCORR_E_INVAL   # NULL members
    b = ctypes.c_void_p()
    assert lib.xcorr_batch_init(nulls, 1, ctypes.c_void_p(256), 256, ctypes.byref(b)) == X.XCORR_E_INVAL
    assert lib.xcorr_batch_ingest(None, None, None, None, None) == X.XCORR_E_INVAL
    assert lib.xcorr_batch_destroy(None) == X.XCORR_E_INVAL
    assert lib.xcorr_batch_tiles(None, None) == X.XCORR_E_INVAL
    assert not b.value


def test_autotune_query_sizes_and_rejections():
    cfg = X.make_config(192, 1024, 4, X.PATH_I8_MFMA)
    ws, _, _ = X.xcorr_query(cfg)
    # accumulators + input block + the batched kernel's queue counters
    assert X.xcorr_autotune_query(cfg) == ws + 2048 * 1024 * 192 + 256
    cfg8 = X.make_config(96, 16, 8, X.PATH_F16_MFMA)
    ws8, _, _ = X.xcorr_query(cfg8)
    assert X.xcorr_autotune_query(cfg8) == ws8 + 2048 * 16 * 96 * 2 + 256
    with pytest.raises(X.XcorrError) as ei:
        X.xcorr_autotune_query(X.make_config(16, 8, 4, X.PATH_PLAIN))
    assert ei.value.code == X.XCORR_E_INVAL


def test_autotune_rejects_short_scratch_before_any_device_call(lib):
    cfg = X.make_config(64, 8, 4, X.PATH_I8_MFMA)
    best = ctypes.c_int32(-7)
    assert lib.xcorr_autotune(ctypes.byref(cfg), None, 1 << 30, None, ctypes.byref(best)) == X.XCORR_E_NOMEM
    assert lib.xcorr_autotune(ctypes.byref(cfg), ctypes.c_void_p(256), 16, None, ctypes.byref(best)) == X.XCORR_E_NOMEM
    assert lib.xcorr_autotune(ctypes.byref(cfg), ctypes.c_void_p(256), 1 << 30, None, None) == X.XCORR_E_INVAL
    assert best.value == -7


def test_strerror_covers_codes():
    for c in (0, -1, -2, -3, -4, -5):
        assert X.xcorr_strerror(c) and X.xcorr_strerror(c) != "unknown error"
    assert X.xcorr_strerror(-99) == "unknown error"


def test_admission_walks_arrays_in_order_against_the_budget():
    cfgs = [X.make_config(96, 4096), X.make_config(512, 4096), X.make_config(192, 4096)]
    bs, slots = [1024, 1024, 1024], [4, 2, 4]

    def need(cfg, b, k):
        ws, out, _ = X.xcorr_query(cfg)
        r256 = lambda x: (x + 255) // 256 * 256
        return ws + r256(out) + k * r256(b * cfg.n_chans * cfg.n_inputs)

    n = [need(c, b, k) for c, b, k in zip(cfgs, bs, slots)]
    adm, used = X.xcorr_admit(cfgs, bs, slots, sum(n))
    assert adm == [True, True, True] and used == sum(n)
    # the large array does not fit, the one after it still does
    adm, used = X.xcorr_admit(cfgs, bs, slots, n[0] + n[2])
    assert adm == [True, False, True] and used == n[0] + n[2]
    adm, used = X.xcorr_admit(cfgs, bs, slots, n[0] - 1)
    assert adm == [False, False, False] and used == 0
    # device-resident blocks need no ring
    adm, used = X.xcorr_admit(cfgs, bs, [0, 0, 0], 1 << 50)
    assert used == sum(need(c, b, 0) for c, b in zip(cfgs, bs))


def test_pipe_calls_reject_bad_arguments_on_the_host(lib):
    rb = ctypes.c_size_t()
    assert lib.xcorr_pipe_query(None, 4, 1024, ctypes.byref(rb)) == X.XCORR_E_INVAL
    p = ctypes.c_void_p()
    assert lib.xcorr_pipe_init(None, 4, 1024, 8, None, 0, None, None, ctypes.byref(p)) == X.XCORR_E_INVAL
    assert lib.xcorr_pipe_push(None, ctypes.c_void_p(256), 0, 0, None, None) == X.XCORR_E_INVAL
    assert lib.xcorr_pipe_drain(None) == X.XCORR_E_INVAL
    assert lib.xcorr_pipe_stats(None, None) == X.XCORR_E_INVAL
    assert lib.xcorr_pipe_destroy(None) == X.XCORR_E_INVAL
    assert not p.value


def test_tuner_times_the_kernel_the_context_runs(monkeypatch):
    """The tuner labels its cache line with the kernel it timed, which is the
    kernel an ingest of the same config launches."""
    monkeypatch.delenv("XCORR_MFMA4_VARIANT", raising=False)
    c4 = X.make_config(192, 1024, 4, X.PATH_I8_MFMA)
    # one whole-triangle region per channel (tile 6): the three-product kernel;
    # a tile with rectangles between segments: the fused-product kernel
    assert X.xcorr_autotune_kernel(c4) == "xc_gauss4_kernel"
    # several segments (triangles and rectangles) also run the three-product kernel
    assert X.xcorr_autotune_kernel(X.make_config(192, 1024, 4, X.PATH_I8_MFMA, tile=4)) == "xc_gauss4_kernel"
    assert X.xcorr_autotune_kernel(X.make_config(512, 64, 4, X.PATH_I8_MFMA, tile=4)) == "xc_gauss4_kernel"
    assert X.xcorr_autotune_kernel(X.make_config(100, 64, 4, X.PATH_I8_MFMA)) == "xc_mfma4f_kernel"   # N % 16
    # the batched launch: the three-product batch kernel where it carries the
    # plan, else the queue-driven four-product one
    assert X.xcorr_autotune_kernel(c4, batch=True) == "xc_gauss4_batch_kernel"
    assert X.xcorr_autotune_kernel(X.make_config(512, 64, 4, X.PATH_I8_MFMA), batch=True) == "xc_gauss4_batch_kernel"
    assert X.xcorr_autotune_kernel(X.make_config(100, 64, 4, X.PATH_I8_MFMA), batch=True) == "xc_batch4_kernel"
    monkeypatch.setenv("XCORR_MFMA4_VARIANT", "fused")
    assert X.xcorr_autotune_kernel(c4) == "xc_mfma4f_kernel"
    assert X.xcorr_autotune_kernel(c4, batch=True) == "xc_batch4_kernel"
    assert X.xcorr_autotune_kernel(X.make_config(192, 512, 8, X.PATH_I8_MFMA)) == "xc_mfma8_kernel_i8"
    assert X.xcorr_autotune_kernel(X.make_config(192, 512, 8, X.PATH_F16_MFMA)) == "xc_mfma8_kernel_f16"
    monkeypatch.setenv("XCORR_MFMA4_VARIANT", "roles")
    assert X.xcorr_autotune_kernel(c4) == "xc_mfma4_kernel"
    with pytest.raises(X.XcorrError):
        X.xcorr_autotune_kernel(X.make_config(192, 512, 8, X.PATH_I8_MFMA), batch=True)


def test_tune_cache_lines_are_used_only_for_their_kernel(tmp_path, monkeypatch):
    """xcorr_init and xcorr_batch_init take the last cache line of their config
    that names the kernel they will run; lines of other kernels, other configs
    and the old five-field format are ignored."""
    monkeypatch.delenv("XCORR_MFMA4_VARIANT", raising=False)
    cache = tmp_path / "tune.txt"
    cache.write_text("4 192 1024 1 3\n"                          # old format: ignored
                     "4 192 1024 1 2 xc_mfma4_kernel\n"           # per-role kernel: not run
                     "4 192 1024 1 4 xc_gauss4_kernel\n"
                     "4 192 1024 1 4 xc_mfma4f_kernel\n"          # tile 4 runs the three-product kernel
                     "4 192 1024 1 6 xc_mfma4f_kernel\n"          # so does tile 6
                     "4 192 1024 1 5 xc_gauss4_kernel\n"          # tile 5 leaves 5 x 5 rectangles: no kernel
                     "4 192 512 1 3 xc_gauss4_kernel\n"           # another config
                     "4 192 1024 1 3 xc_gauss4_batch_kernel\n"
                     "4 192 1024 1 2 xc_batch4_kernel\n"           # the batch runs the three-product kernel
                     "4 192 1024 1 5 xc_gauss4_batch_kernel\n")    # 5 is not a batch tile: ignored
    monkeypatch.setenv("XCORR_TUNE_CACHE", str(cache))
    cfg = X.make_config(192, 1024, 4, X.PATH_I8_MFMA)
    assert X.xcorr_plan_tile(cfg) == (4, True)
    assert X.xcorr_plan_tile(cfg, batch=True) == (3, True)
    monkeypatch.setenv("XCORR_MFMA4_VARIANT", "roles")
    assert X.xcorr_plan_tile(cfg) == (2, True)
    monkeypatch.delenv("XCORR_MFMA4_VARIANT")
    # an explicit tile wins over the cache; no line: the built-in choice
    assert X.xcorr_plan_tile(X.make_config(192, 1024, 4, X.PATH_I8_MFMA, tile=3)) == (3, False)
    assert X.xcorr_plan_tile(X.make_config(256, 64, 4, X.PATH_I8_MFMA)) == (4, False)
    # a batch member without a batch line keeps its own tile if the batched
    # kernel carries it, else the 2..4 tile that pads least
    assert X.xcorr_plan_tile(X.make_config(192, 512, 4, X.PATH_I8_MFMA), batch=True) == (3, False)
    assert X.xcorr_plan_tile(X.make_config(160, 8, 4, X.PATH_I8_MFMA, tile=5), batch=True)[0] in (2, 3, 4)
    monkeypatch.delenv("XCORR_TUNE_CACHE")
    assert X.xcorr_plan_tile(cfg) == (6, False)
